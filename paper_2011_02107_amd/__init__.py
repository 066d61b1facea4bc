"""DACP central eigenvalues on MI355X: thin Python binding over the HIP C-ABI library."""

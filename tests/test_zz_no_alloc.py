"""The allocation-free entry point dacp_syev_batched_noalloc against dacp_syev_batched (MI355X).

dacp_syev_batched_noalloc runs the same kernels as dacp_syev_batched with every buffer besides the
inputs and outputs in a fixed per-device workspace.  Two calls in a row through the C ABI (the
second with fewer and smaller matrices, so stale workspace contents from the first call sit under
it) must give the same eigenvalues and eigenvectors as the allocating entry point on the same
matrices, and the eigenvalues must match the oracle's dense eigensolver; a request larger than
the workspace is refused with DACP_E_INVALID before any device work.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import _native  # noqa: E402
from paper_2011_02107_amd import binding as B  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _sym(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n))
    return 0.5 * (a + a.T)


def _run(ctx, mats, noalloc):
    As = [torch.as_tensor(m, dtype=torch.float64, device=DEV).contiguous() for m in mats]
    Zs = [torch.empty_like(a) for a in As]
    ws = B.dacp_syev_batched(ctx, As, Zs, noalloc=noalloc)
    torch.cuda.synchronize()
    return ws, [z.cpu().numpy() for z in Zs]


def test_syev_batched_noalloc_matches_the_allocating_entry_point():
    ctx = B.Context(0)
    try:
        for sizes, seed in (([700, 300, 1, 513, 64, 1000], 1), ([120, 7], 2)):
            mats = [_sym(n, seed * 100 + i) for i, n in enumerate(sizes)]
            w1, z1 = _run(ctx, mats, noalloc=False)
            w0, z0 = _run(ctx, mats, noalloc=True)
            for i, m in enumerate(mats):
                norm = np.abs(m).sum(axis=1).max()
                ref = _native.syev(m)
                assert np.abs(w0[i] - ref).max() <= 1e-12 * norm * max(1, sizes[i]) ** 0.5
                # the same kernels on the same matrices: the allocating call's results to rounding
                assert np.abs(w0[i] - w1[i]).max() <= 1e-13 * norm
                assert np.abs(np.abs(z0[i]) - np.abs(z1[i])).max() <= 1e-10
                # rows are orthonormal eigenvectors
                Z = z0[i]
                assert np.abs(Z @ Z.T - np.eye(sizes[i])).max() <= 1e-11 * sizes[i]
                assert np.abs(Z @ m @ Z.T - np.diag(w0[i])).max() <= 1e-11 * norm * sizes[i] ** 0.5
        # beyond the fixed workspace: refused before any device work
        big = [torch.zeros((2048, 2048), dtype=torch.float64, device=DEV) for _ in range(3)]
        with pytest.raises(B.DacpError) as e:
            B.dacp_syev_batched(ctx, big, [torch.empty_like(b) for b in big], noalloc=True)
        assert e.value.status == -1 and "workspace" in e.value.message
    finally:
        torch.cuda.synchronize()
        ctx.close()

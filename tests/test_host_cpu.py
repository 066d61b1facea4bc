"""Host-side behaviour that needs no GPU: the benchmark's one-GPU contract, and the library's
entry points failing cleanly (a status, no crash) where no device exists."""
import ctypes
import os
import subprocess
import sys

import pytest

from paper_2011_02107_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no benchmark line


def _no_gpu():
    import torch

    return not torch.cuda.is_available()


@pytest.mark.skipif(not _no_gpu(), reason="checks the behaviour on a machine without a GPU")
def test_create_without_a_device_returns_invalid():
    lib = binding.load_library()
    h = ctypes.c_void_p()
    st = lib.dacp_create(0, None, ctypes.byref(h))
    assert st == -1  # DACP_E_INVALID: no such device
    assert not h.value


def test_null_arguments_are_rejected_without_a_device():
    lib = binding.load_library()
    assert lib.dacp_create(0, None, None) == -1
    assert lib.dacp_last_error(None).decode() == "null context"
    lib.dacp_destroy(None)  # a no-op


def test_spacing_ratios_through_the_abi_match_the_oracle():
    """Host entry point, no device: ratios equal the oracle's bit for bit, NaN where both spacings
    vanish, and bad input is rejected with a status."""
    import numpy as np

    from oracle import levels

    rng = np.random.default_rng(3)
    E = np.sort(rng.standard_normal(5000))
    E = np.concatenate([E, [E[-1] + 1.0] * 3])  # three equal levels at the end
    r, mean = binding.dacp_spacing_ratios(E)
    r_ref, mean_ref = levels.spacing_ratios(E)
    assert np.array_equal(np.isnan(r), np.isnan(r_ref)) and np.isnan(r[-1])
    fin = ~np.isnan(r_ref)
    assert np.array_equal(r[fin], r_ref[fin])
    assert abs(mean - mean_ref) <= 1e-15
    lib = binding.load_library()
    bad = np.array([0.0, 2.0, 1.0])
    assert lib.dacp_spacing_ratios(bad.ctypes.data_as(binding._dp), 3, None, None) == -1
    assert lib.dacp_spacing_ratios(bad.ctypes.data_as(binding._dp), 2, None, None) == -1
    nan = np.array([0.0, np.nan, 1.0])
    assert lib.dacp_spacing_ratios(nan.ctypes.data_as(binding._dp), 3, None, None) == -1


def test_plan_matches_the_oracle_parameter_rules():
    """The host parameter selection (window, filter order, basis size, sampled orders; Sec. II.A,
    II.B, III) through the C ABI, without a device, against the oracle's window bisection over its
    KPM count, its filter order and its sampled orders."""
    import math

    import numpy as np

    from oracle import chebyshev, hamiltonian, spectral
    from paper_2011_02107_amd import inputs

    L, N = 10, 100
    D = 1 << L
    terms = inputs.ising_chain(L)
    e_b = hamiltonian.sum_abs_coeff(terms)  # a valid bound (>= ||H||)
    R = inputs.gaussian_block(D, 8, 4)
    mu = spectral.kpm_moments(lambda X: hamiltonian.apply_h(L, terms, X), R, e_b, 128)
    for attempt, opts in ((0, binding.default_opts(b=4)), (1, binding.default_opts(b=4)),
                          (0, binding.default_opts(b=0, basis_ratio=1.2, kfac=12.0))):
        p = binding.dacp_plan(D, N, e_b, mu, opts, attempt=attempt)
        wr = 2.2  # the count is decided in FP64 on both sides (2.2 * 100 rounds up to 220.00000000000003)
        for _ in range(attempt):
            wr *= 1.5
        n_w = min(D, math.ceil(wr * N))
        assert p["n_w"] == n_w
        ref = spectral.window_for_count(mu, D, n_w)
        assert abs(p["a_r"] - ref) <= 1e-12
        assert spectral.kpm_count(mu, D, p["a_r"]) >= n_w * (1 - 1e-12)
        assert p["a"] == p["a_r"] * e_b
        assert p["K"] == chebyshev.filter_order(e_b, p["a"], opts.kfac)
        b, n, m = p["b"], p["n"], p["m"]
        assert m == b * (2 * n + 1) and m >= opts.basis_ratio * n_w
        assert n == 1 or b * (2 * n - 1) < opts.basis_ratio * n_w  # the smallest such n
        assert list(p["k_samples"]) == chebyshev.sample_orders(p["a_r"], n)
    # a fixed window skips the moments
    p = binding.dacp_plan(D, N, e_b, None, binding.default_opts(b=4, a=0.5))
    assert p["a_r"] == 0.5 / e_b and p["K"] == chebyshev.filter_order(e_b, p["a"], 18.0)
    with pytest.raises(ValueError):
        binding.dacp_plan(D, N, e_b, None, binding.default_opts(b=4))  # no moments, no window
    with pytest.raises(ValueError):
        binding.dacp_plan(D, D + 1, e_b, mu)
    with pytest.raises(ValueError):
        binding.dacp_plan(D, N, 0.0, mu)


def test_accept_rule_through_the_abi_matches_the_oracle():
    """The library's acceptance rule (host code, no device) against the oracle's plain version on
    random Ritz values and residuals with ghosts, cascades and values beyond the window: the same
    core, the same estimates bit for bit, the same ghost count."""
    import numpy as np

    from oracle import acceptance

    rng = np.random.default_rng(11)
    for trial in range(40):
        r = int(rng.integers(1, 300))
        theta = np.sort(rng.uniform(-1.0, 1.0, r))
        if trial % 5 == 0 and r > 3:
            theta[r // 2] = theta[r // 2 - 1]  # a repeated value
        if trial % 7 == 0 and r > 10:
            theta[r // 3: r // 3 + 4] = theta[r // 3] + 1e-9 * np.arange(4)  # a near-degenerate cluster
        n_sel = int(rng.integers(0, r + 1))
        rn = 10.0 ** rng.uniform(-14, -3, n_sel)
        rn[rng.uniform(size=n_sel) < 0.05] = 50.0  # ghosts
        a, tol = float(rng.uniform(0.2, 0.9)), 10.0 ** rng.uniform(-11, -7)
        pos, est, ng = binding.dacp_accept_rule(theta, rn, a, tol)
        core_ref, est_ref, ng_ref = acceptance.accept(theta, rn, a, tol)
        assert list(pos) == core_ref and ng == ng_ref
        assert np.array_equal(est, np.array(est_ref, dtype=np.float64))
    with pytest.raises(ValueError):
        binding.dacp_accept_rule([0.2, 0.1], [1e-12], 0.5, 1e-10)  # unsorted
    with pytest.raises(ValueError):
        binding.dacp_accept_rule([0.1, 0.2], [1e-12] * 3, 0.5, 1e-10)  # n_sel > r
    with pytest.raises(ValueError):
        binding.dacp_accept_rule([0.1, 0.2], [1e-12], 0.0, 1e-10)  # a <= 0

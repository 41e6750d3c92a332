"""bench.py's command-line contract that holds without a GPU: more than one GPU is refused
with a message and a non-zero status before any device work."""
import os

import pytest
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_host_residual_recheck_matches_the_oracle():
    # bench.py re-checks the first timed solve on the host from the factored form of eq (4.1);
    # on a small indefinite problem it agrees with the oracle's dense residual
    import numpy as np

    sys.path.insert(0, ROOT)
    import bench
    import lyapgen
    from oracle import exact as E
    from oracle import residual as R

    A, L = lyapgen.random_shift(7, 40, 3)
    s = np.array([1.0, -1.0, 0.5])
    X = E.kron_solve(A, E.form_w(L, s))
    w, V = np.linalg.eigh(X)
    keep = np.abs(w) > 1e-12 * np.abs(w).max()
    Z, D = V[:, keep], w[keep]
    Z = Z + 1e-7 * np.random.default_rng(0).standard_normal(Z.shape)
    got = bench._host_relres(A, L, s, Z, D)
    want = R.relres(A, L, s, Z, D)
    assert got == pytest.approx(want, rel=1e-6)

"""Host logic of the library built with g++ and run on the CPU: the persistent-grid admission
(csrc/residency.hpp: a grid's CU-slot charge per XCD, tickets, concurrent holders that never exceed
the pool), the LDS budget of the dense transform passes (csrc/transform_lds.hpp: the boundary N of
each table kind and dimension, static partial sums included) and the Hessenberg eigenvalue solver
behind the Ritz values (csrc/hessenberg.hpp, against LAPACK through numpy)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
INC = os.path.join(ROOT, "paper_2507_02809_amd", "csrc")


def _run(tmp_path, name: str, stdin: str = "") -> str:
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / name
    src = os.path.join(HERE, "native", name + ".cpp")
    subprocess.run([gxx, "-std=c++17", "-O2", "-pthread", "-I", INC, src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], input=stdin, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return r.stdout


def test_residency_admission(tmp_path):
    assert "residency ok" in _run(tmp_path, "residency_check")


def test_transform_pass_lds_boundary(tmp_path):
    out = _run(tmp_path, "transform_lds_check")
    assert "transform lds ok" in out
    # the c3 shape (d = 2, N = 255) fits both table kinds
    assert "d=2 cas: largest N" in out and "d=2 sine: largest N" in out


def _sorted_eigs(ev):
    ev = np.asarray(ev, dtype=complex)
    return ev[np.lexsort((np.round(ev.imag, 8), np.round(ev.real, 8)))]


def test_hessenberg_eigenvalues_match_lapack(tmp_path):
    rng = np.random.default_rng(5)
    mats = []
    for n in [1, 2, 3, 4, 5, 8, 13, 30, 60]:
        H = np.triu(rng.standard_normal((n, n)), -1)
        mats.append(H)
    # an Arnoldi-like matrix with eigenvalues clustered at 1 (identity plus low rank, as P^{-1} A)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    M = np.eye(n) + Q[:, :3] @ np.diag([5.0, -0.5, 20.0]) @ Q[:, :3].T
    from scipy.linalg import hessenberg
    mats.append(hessenberg(M))
    # a matrix with complex pairs and a zero diagonal
    mats.append(np.triu(np.array([[0.0, 2.0, 1.0], [-3.0, 0.0, 4.0], [0.0, 1.0, 0.0]]), -1))
    text = "".join(f"{H.shape[0]}\n" + " ".join(repr(float(v)) for v in H.ravel()) + "\n" for H in mats)
    out = _run(tmp_path, "hessenberg_check", text).split("\n")
    pos = 0
    for H in mats:
        n = H.shape[0]
        assert out[pos] != "fail"
        got = [complex(*map(float, out[pos + i].split())) for i in range(n)]
        assert out[pos + n] == "end"
        pos += n + 1
        ref = np.linalg.eigvals(H)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(_sorted_eigs(got) - _sorted_eigs(ref)).max() <= 1e-10 * scale, n

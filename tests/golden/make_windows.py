"""Write the interval/eigengap fixtures used by the tests and the bench.

Calls only ``oracle`` (and the shared input generators in ``pencils``).  Run
from the repository root:

    python tests/golden/make_windows.py c0          # 10^3 grid, dense LAPACK
    python tests/golden/make_windows.py c1          # 64^3 grid, shift-invert Lanczos
    python tests/golden/make_windows.py small       # the small parity pencils
    python tests/golden/make_windows.py serving     # eigenvalue clusters of the serving pencils
    python tests/golden/make_windows.py c3 32       # complex Hermitian 27-point Peierls pencil, 32^3
    python tests/golden/make_windows.py e1 12 24    # Gaussian-well Hamiltonian, the 88 smallest eigenpairs

Each fixture stores the workload recipe (grid, seeds), the window of
eigenvalues (ascending, the oracle's values) and the eigengaps
(a_-, a_+, b_-, b_+) following the experiments' convention (Sec. 3.1): the
gap endpoints are the true neighbouring eigenvalues and a, b the gap midpoints.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import pencils  # noqa: E402
from oracle.dense import pencil_eigh_lapack  # noqa: E402
from oracle.sparse import count_interval, window_near  # noqa: E402


def _dump(name, obj):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(obj, f, indent=1)
    print("wrote", path)


def dense_window(n, n_lambda, start=None, name=None):
    p = pencils.grid7(n)
    A, B = p.scipy()
    lam, _ = pencil_eigh_lapack(A.toarray(), B.toarray())
    if start is None:
        start = p.n // 2 - n_lambda // 2
    w = pencils.window_from_eigenvalues(lam, start, n_lambda)
    w.update(
        {
            "workload": f"grid7 {n}^3",
            "grid": [n, n, n],
            "seed_v": 0,
            "start_index": int(start),
            "eigenvalues": [float(x) for x in lam[start : start + n_lambda]],
            "source": "oracle.dense.pencil_eigh_lapack (LAPACK generalized Hermitian)",
        }
    )
    _dump(name or f"window_grid7_{n}.json", w)


def c1_window(n=64, n_lambda=64, sigma0=6.0, k=80, verify=True):
    p = pencils.grid7(n)
    A, B = p.scipy()
    t = time.time()
    lam, _ = window_near(A.tocsc(), B.tocsc(), sigma0, k)
    t_eig = time.time() - t
    # central n_lambda of the k nearest, with one neighbour on each side for the gaps
    i0 = (k - n_lambda) // 2
    w = pencils.window_from_eigenvalues(lam, i0, n_lambda)
    cnt = None
    t_cnt = None
    if verify:
        t = time.time()
        cnt = count_interval(A, B, w["a"], w["b"])
        t_cnt = time.time() - t
    w.update(
        {
            "workload": f"grid7 {n}^3 mid-spectrum window near {sigma0}",
            "grid": [n, n, n],
            "seed_v": 0,
            "sigma0": sigma0,
            "eigenvalues": [float(x) for x in lam[i0 : i0 + n_lambda]],
            "neighbours": [float(x) for x in lam],
            "inertia_count": cnt,
            "source": "oracle.sparse.window_near (shift-invert Lanczos, ARPACK) + Sylvester inertia count",
            "seconds": {"eigsh": t_eig, "inertia": t_cnt},
        }
    )
    _dump(f"window_grid7_{n}.json", w)


def c3_window(n=32, n_lambda=64, sigma0=0.0, k=80, verify=True):
    """Complex Hermitian 27-point Peierls pencil: mid-spectrum window of n_lambda
    eigenvalues near sigma0 by shift-invert Lanczos, count checked by inertia."""
    p = pencils.grid27p(n)
    A, B = p.scipy()
    t = time.time()
    lam, _ = window_near(A.tocsc(), B.tocsc(), sigma0, k)
    t_eig = time.time() - t
    i0 = (k - n_lambda) // 2
    w = pencils.window_from_eigenvalues(lam, i0, n_lambda)
    cnt, t_cnt = None, None
    if verify:
        t = time.time()
        cnt = count_interval(A, B, w["a"], w["b"])
        t_cnt = time.time() - t
    w.update(
        {
            "workload": f"grid27p {n}^3 complex Hermitian mid-spectrum window near {sigma0}",
            "grid": [n, n, n],
            "seed_v": 0,
            "seed_theta": 1,
            "sigma0": sigma0,
            "eigenvalues": [float(x) for x in lam[i0 : i0 + n_lambda]],
            "neighbours": [float(x) for x in lam],
            "inertia_count": cnt,
            "source": "oracle.sparse.window_near (shift-invert Lanczos, ARPACK) + Sylvester inertia count",
            "seconds": {"eigsh": t_eig, "inertia": t_cnt},
        }
    )
    _dump(f"window_grid27p_{n}.json", w)


def e1_window(n, k=89, seed_max=64):
    """The paper's first experiment (Sec. 3.1): -(1/2) Laplacian + Gaussian wells,
    B = I, the k - 1 = 88 smallest eigenpairs with a_- = -inf, a_+ = lambda_1,
    b_- = lambda_88, b_+ = lambda_89.  As in the paper, potentials are drawn (seed
    0, 1, ...) until the relative eigengap delta = min(a_+ - a_-, b_+ - b_-) /
    (b_- - a_+) = (lambda_89 - lambda_88) / (lambda_88 - lambda_1) lies in
    [1e-4, 1e-3].  Dense LAPACK up to N = 4096, shift-invert Lanczos below the
    spectrum (sigma0 = 0) above, with the count checked by inertia."""
    for seed in range(seed_max):
        p = pencils.gaussian_wells(n, seed=seed)
        A, B = p.scipy()
        t = time.time()
        if p.n <= 4096:
            lam, _ = pencil_eigh_lapack(A.toarray(), B.toarray())
            lam = lam[:k]
            src = "oracle.dense.pencil_eigh_lapack (LAPACK generalized Hermitian)"
        else:
            lam, _ = window_near(A.tocsc(), B.tocsc(), 0.0, k)
            src = "oracle.sparse.window_near (shift-invert Lanczos below the spectrum, ARPACK)"
        t_eig = time.time() - t
        delta = (lam[k - 1] - lam[k - 2]) / (lam[k - 2] - lam[0])
        print(f"n={n} seed={seed}: delta={delta:.3e} ({t_eig:.1f}s)", flush=True)
        if 1e-4 <= delta <= 1e-3:
            break
    else:
        raise RuntimeError("no potential with a relative eigengap in [1e-4, 1e-3]")
    a, b = float(lam[0] - 1.0), float(0.5 * (lam[k - 2] + lam[k - 1]))
    cnt, t_cnt = None, None
    if p.n <= 40000:
        t = time.time()
        cnt = count_interval(A, B, a, b)
        t_cnt = time.time() - t
    w = {"a": a, "b": b, "a_minus": float("-inf"), "a_plus": float(lam[0]), "b_minus": float(lam[k - 2]),
         "b_plus": float(lam[k - 1]), "n_lambda": k - 1, "delta_lambda": float(delta),
         "workload": f"gaussian_wells {n}^3 (-1/2 Laplacian + 3 Gaussian wells, B = I), the {k - 1} smallest eigenpairs",
         "grid": [n, n, n], "seed": seed, "eigenvalues": [float(x) for x in lam[: k - 1]], "neighbours": [float(lam[k - 1])],
         "inertia_count": cnt, "source": src, "seconds": {"eig": t_eig, "inertia": t_cnt}}
    _dump(f"window_e1_{n}.json", w)


SERVING_GRIDS = [16, 20, 24, 28, 32]
SERVING_CENTERS = [4.0, 5.5, 7.0, 8.5]
SERVING_K = 150


def serving_clusters():
    """Per serving pencil (grid7 n^3, potential seed 0) and per center sigma0,
    the SERVING_K eigenvalues nearest sigma0 (consecutive in the spectrum):
    every run of n_lambda of them with a neighbour on each side is a query
    window with known eigengaps."""
    out = {"grids": SERVING_GRIDS, "centers": SERVING_CENTERS, "k": SERVING_K, "seed_v": 0, "clusters": {},
           "source": "oracle.sparse.window_near (shift-invert Lanczos, ARPACK)"}
    for n in SERVING_GRIDS:
        p = pencils.grid7(n)
        A, B = p.scipy()
        A, B = A.tocsc(), B.tocsc()
        for c in SERVING_CENTERS:
            t = time.time()
            lam, _ = window_near(A, B, c, SERVING_K)
            out["clusters"][f"{n}:{c}"] = [float(x) for x in lam]
            print(f"grid {n} center {c}: {time.time() - t:.1f}s", flush=True)
    _dump("serving_clusters.json", out)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "c0"
    if what == "c0":
        dense_window(10, 16)
    elif what == "small":
        dense_window(6, 8)
        dense_window(8, 12)
        dense_window(12, 16)
    elif what == "c1":
        c1_window()
    elif what == "serving":
        serving_clusters()
    elif what == "e1":
        for n in [int(x) for x in sys.argv[2:]] or [12, 24]:
            e1_window(n)
    elif what == "c3":
        c3_window(n=int(sys.argv[2]) if len(sys.argv) > 2 else 32)
    elif what.startswith("grid"):
        n = int(what[4:])
        c1_window(n=n, verify=True)

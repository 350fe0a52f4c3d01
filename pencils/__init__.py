"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the bench.

This module holds only workload construction: stencil matrices in CSR form,
seeded random potentials and phases, Gaussian start blocks, and the rule that
turns a list of eigenvalues (computed elsewhere) into an interval with its
eigengaps.  It contains none of the eigensolver's arithmetic.

Workloads (stand-ins for the paper's 3-D Hamiltonian and SIESTA pencils,
Sec. 3.1 and 3.2):

* ``grid7``   : A = 7-point integer Laplacian stencil (diagonal 6, face
  neighbours -1, Dirichlet, no 1/h^2 scaling) + diag(v), v ~ U[-1,1];
  B = I + 0.1 * S7 with S7 = (I + face adjacency)/7.  Real symmetric, B SPD.
* ``grid27p`` : complex Hermitian 27-point Peierls pencil: A_ii = v_i ~ N(0,1),
  A_ij = -exp(i theta_ij) for the 26 neighbours j > i, theta ~ U[0, 2 pi),
  A_ji = conj(A_ij); B = I + 0.05 * S27, S27 = (I + 26-neighbour adjacency)/27.

* ``gaussian_wells`` : the 3-D Hamiltonian H = -(1/2) Laplacian + V of the
  paper's first experiment (Sec. 3.1) on [0,1)^3 with Dirichlet boundaries,
  n interior points per dimension, spacing h = 1/(n+1), 7-point stencil:
  A = (1/(2h^2)) (6 I - face adjacency) + diag(V(x_i)), x_i = h (i+1);
  V(x) = -sum_{k=1..3} d_k exp(-|x - c_k|^2 / rho^2), depths d_k ~ U(0,1],
  centres c_k ~ U[0,1)^3, rho = 0.2 (the wells' radius); B = I (stored with
  the stencil's pattern, zero off the diagonal).

Grid index of (x, y, z) on an n^3 grid is x + n*y + n^2*z.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "GridPencil",
    "grid7",
    "grid27p",
    "gaussian_wells",
    "gaussian_block",
    "window_from_eigenvalues",
    "serving_stream",
    "c4_stream",
]


class GridPencil:
    """CSR pencil (A, B) sharing one sparsity pattern (full storage, sorted columns)."""

    def __init__(self, n, rowptr, colind, a_vals, b_vals, grid, stencil):
        self.n = int(n)
        self.rowptr = rowptr
        self.colind = colind
        self.a_vals = a_vals
        self.b_vals = b_vals
        self.grid = tuple(int(g) for g in grid)
        self.stencil = stencil

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    @property
    def is_complex(self) -> bool:
        return np.iscomplexobj(self.a_vals)

    def scipy(self):
        """Return (A, B) as scipy.sparse CSR matrices."""
        import scipy.sparse as sp

        shape = (self.n, self.n)
        A = sp.csr_matrix((self.a_vals, self.colind, self.rowptr), shape=shape)
        B = sp.csr_matrix((self.b_vals, self.colind, self.rowptr), shape=shape)
        return A, B


def _neighbour_offsets(stencil: int):
    if stencil == 7:
        return [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    if stencil == 27:
        return [
            (dx, dy, dz)
            for dz in (-1, 0, 1)
            for dy in (-1, 0, 1)
            for dx in (-1, 0, 1)
            if (dx, dy, dz) != (0, 0, 0)
        ]
    raise ValueError("stencil must be 7 or 27")


def _pattern(nx: int, ny: int, nz: int, stencil: int):
    """Sorted CSR pattern of the stencil graph plus the diagonal.

    Returns rowptr (int64), colind (int32) and, per stored entry, the row index.
    """
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    rows = [idx]
    cols = [idx]
    for dx, dy, dz in _neighbour_offsets(stencil):
        ok = (
            (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) & (z + dz >= 0) & (z + dz < nz)
        )
        r = idx[ok]
        rows.append(r)
        cols.append(r + dx + nx * dy + nx * ny * dz)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr, cols.astype(np.int32), rows


def grid7(n: int, seed_v: int = 0, ny: int | None = None, nz: int | None = None, v_scale: float = 1.0) -> GridPencil:
    """Real 7-point pencil on an n x ny x nz grid (defaults: a cube).

    A = stencil(6, -1) + diag(v_scale v), v ~ U[-1,1] drawn with numpy PCG64(seed_v);
    B = I + 0.1*(I + face adjacency)/7.  v_scale = 0 on a cube gives A and B that
    are polynomials in the same adjacency, so the pencil's eigenvalues are
    degenerate (clusters of 3 and 6 from the permutations of the three directions).
    """
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    N = n * ny * nz
    rowptr, colind, rows = _pattern(n, ny, nz, 7)
    v = np.random.Generator(np.random.PCG64(seed_v)).uniform(-1.0, 1.0, size=N)
    diag = rows == colind
    a_vals = np.where(diag, 6.0 + v_scale * v[rows], -1.0)
    b_vals = np.where(diag, 1.0 + 0.1 / 7.0, 0.1 / 7.0)
    return GridPencil(N, rowptr, colind, a_vals.astype(np.float64), b_vals.astype(np.float64), (n, ny, nz), 7)


def grid27p(n: int, seed_v: int = 0, seed_theta: int = 1, ny: int | None = None, nz: int | None = None) -> GridPencil:
    """Complex Hermitian 27-point Peierls pencil (see module docstring)."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    N = n * ny * nz
    rowptr, colind, rows = _pattern(n, ny, nz, 27)
    v = np.random.Generator(np.random.PCG64(seed_v)).standard_normal(N)
    cols = colind.astype(np.int64)
    upper = cols > rows
    # One phase per undirected edge, drawn in CSR order of the upper triangle.
    n_up = int(upper.sum())
    theta = np.random.Generator(np.random.PCG64(seed_theta)).uniform(0.0, 2.0 * np.pi, size=n_up)
    a_vals = np.zeros(rows.shape[0], dtype=np.complex128)
    a_vals[upper] = -np.exp(1j * theta)
    # Lower entries: conj of the matching upper entry (j, i).
    key_up = rows[upper] * N + cols[upper]
    lower = cols < rows
    key_lo = cols[lower] * N + rows[lower]
    pos = np.searchsorted(key_up, key_lo)
    a_vals[lower] = np.conj(a_vals[upper][pos])
    diag = rows == cols
    a_vals[diag] = v[rows[diag]]
    b_vals = np.where(diag, 1.0 + 0.05 / 27.0, 0.05 / 27.0).astype(np.complex128)
    return GridPencil(N, rowptr, colind, a_vals, b_vals, (n, ny, nz), 27)


def gaussian_wells(n: int, seed: int = 0, wells: int = 3, radius: float = 0.2) -> GridPencil:
    """-(1/2) Laplacian + V with `wells` Gaussian wells (see module docstring);
    depths and centres drawn with numpy PCG64(seed)."""
    N = n * n * n
    rowptr, colind, rows = _pattern(n, n, n, 7)
    g = np.random.Generator(np.random.PCG64(seed))
    depth = 1.0 - g.uniform(0.0, 1.0, size=wells)  # in (0, 1]
    centre = g.uniform(0.0, 1.0, size=(wells, 3))
    h = 1.0 / (n + 1)
    idx = np.arange(N, dtype=np.int64)
    pos = np.stack([idx % n, (idx // n) % n, idx // (n * n)], axis=1).astype(np.float64) * h + h
    V = np.zeros(N)
    for k in range(wells):
        V -= depth[k] * np.exp(-np.sum((pos - centre[k]) ** 2, axis=1) / radius**2)
    diag = rows == colind
    s = 0.5 / (h * h)
    a_vals = np.where(diag, 6.0 * s + V[rows], -s)
    b_vals = np.where(diag, 1.0, 0.0)
    return GridPencil(N, rowptr, colind, a_vals.astype(np.float64), b_vals.astype(np.float64), (n, n, n), 7)


def gaussian_block(n: int, p: int, seed: int = 2, complex_: bool = False) -> np.ndarray:
    """i.i.d. N(0,1) block (N x p, row-major); complex blocks use N(0,1/2) parts."""
    g = np.random.Generator(np.random.PCG64(seed))
    if not complex_:
        return np.ascontiguousarray(g.standard_normal((n, p)))
    s = np.sqrt(0.5)
    re = g.standard_normal((n, p))
    im = g.standard_normal((n, p))
    return np.ascontiguousarray(s * re + 1j * s * im)


def window_from_eigenvalues(lams, start: int, n_lambda: int):
    """Interval and eigengaps for the window lams[start : start+n_lambda].

    Following the experiments' convention (Sec. 3.1), the gap endpoints are the
    true neighbouring eigenvalues: a_+ = lams[start], a_- = lams[start-1],
    b_- = lams[start+n_lambda-1], b_+ = lams[start+n_lambda]; a and b are the
    gap midpoints.  ``start == 0`` gives a_- = -inf (the lowest slice) and a
    window reaching the end gives b_+ = +inf.  ``lams`` must be sorted.
    """
    lams = np.asarray(lams, dtype=np.float64)
    if start < 0 or n_lambda < 1 or start + n_lambda > lams.shape[0]:
        raise ValueError("window outside the eigenvalue list")
    a_plus = float(lams[start])
    b_minus = float(lams[start + n_lambda - 1])
    a_minus = float(lams[start - 1]) if start > 0 else -np.inf
    b_plus = float(lams[start + n_lambda]) if start + n_lambda < lams.shape[0] else np.inf
    a = 0.5 * (a_minus + a_plus) if np.isfinite(a_minus) else a_plus - (b_minus - a_plus) - 1.0
    b = 0.5 * (b_minus + b_plus) if np.isfinite(b_plus) else b_minus + (b_minus - a_plus) + 1.0
    return {
        "a": a,
        "b": b,
        "a_minus": a_minus,
        "a_plus": a_plus,
        "b_minus": b_minus,
        "b_plus": b_plus,
        "n_lambda": int(n_lambda),
    }


def serving_stream(n_queries: int, n_pencils: int, rate: float, seed: int = 3):
    """Poisson arrival stream for the serving workload.

    Returns a list of dicts with arrival time (s), pencil id, n_lambda
    (log-uniform in [8, 128]) and a window-start fraction uniform over the
    middle 80% of the spectrum index range.
    """
    g = np.random.Generator(np.random.PCG64(seed))
    gaps = g.exponential(1.0 / rate, size=n_queries)
    t = np.cumsum(gaps) - gaps[0]
    pencil = g.integers(0, n_pencils, size=n_queries)
    nl = np.rint(np.exp(g.uniform(np.log(8.0), np.log(128.0), size=n_queries))).astype(int)
    frac = g.uniform(0.1, 0.9, size=n_queries)
    return [
        {"t": float(t[i]), "pencil": int(pencil[i]), "n_lambda": int(nl[i]), "start_frac": float(frac[i])}
        for i in range(n_queries)
    ]


def serving_queries(clusters: dict, n_queries: int, rate: float, seed: int = 3, max_lambda: int = 128):
    """Queries of the serving workload drawn from stored eigenvalue clusters.

    ``clusters`` is the fixture written by the window generator (per grid and
    center sigma0, the consecutive eigenvalues nearest sigma0).  Arrival times,
    pencils and n_lambda (log-uniform in [8, max_lambda]) follow
    ``serving_stream``; the start fraction picks the cluster (center) of that
    pencil, and the window is the run of n_lambda eigenvalues in the middle of
    the cluster, with its neighbours as eigengaps.
    """
    grids = clusters["grids"]
    centers = clusters["centers"]
    k = clusters["k"]
    out = []
    for q in serving_stream(n_queries, len(grids), rate, seed):
        n = grids[q["pencil"]]
        c = centers[min(int(q["start_frac"] * len(centers)), len(centers) - 1)]
        lam = np.asarray(clusters["clusters"][f"{n}:{c}"], dtype=np.float64)
        nl = int(min(q["n_lambda"], max_lambda, k - 2))
        start = (k - nl) // 2
        w = window_from_eigenvalues(lam, start, nl)
        w["eigenvalues"] = [float(x) for x in lam[start : start + nl]]
        out.append({"t": q["t"], "grid": n, "center": c, "window": w})
    return out


C4_GRIDS = [32, 39, 46, 53, 59, 66, 73, 80]


def c4_stream(n_queries: int, rate: float, seed: int = 3, windows_per_pencil: int = 3,
              lo: float = 0.0, hi: float = 12.6):
    """The serving workload over eight grid7 pencils 32^3 ... 80^3 (N 32768 - 512000).

    Each pencil gets `windows_per_pencil` intervals (drawn once, PCG64(seed + 1)):
    a centre uniform over the middle 80% of the spectrum's range [lo, hi] (grid7:
    about [0, 12.6]) and a width holding about n_lambda eigenvalues, n_lambda
    log-uniform in [8, 128], from the mean eigenvalue density N / (hi - lo).  The
    queries (Poisson arrivals at `rate`, PCG64(seed)) pick a pencil uniformly and
    one of its intervals uniformly, so intervals repeat.  Only (a, b, n_lambda)
    are given: eigengaps and counts are left to the eigensolver.
    """
    g = np.random.Generator(np.random.PCG64(seed + 1))
    wins = {}
    for n in C4_GRIDS:
        N = n ** 3
        for k in range(windows_per_pencil):
            nl = int(np.rint(np.exp(g.uniform(np.log(8.0), np.log(128.0)))))
            c = lo + (hi - lo) * g.uniform(0.1, 0.9)
            w = nl * (hi - lo) / N
            wins[(n, k)] = {"a": float(c - 0.5 * w), "b": float(c + 0.5 * w), "n_lambda": nl}
    q = np.random.Generator(np.random.PCG64(seed))
    gaps = q.exponential(1.0 / rate, size=n_queries)
    t = np.cumsum(gaps) - gaps[0]
    pen = q.integers(0, len(C4_GRIDS), size=n_queries)
    win = q.integers(0, windows_per_pencil, size=n_queries)
    out = []
    for i in range(n_queries):
        n = C4_GRIDS[int(pen[i])]
        w = wins[(n, int(win[i]))]
        out.append({"t": float(t[i]), "grid": n, "window_id": int(win[i]), **w})
    return out

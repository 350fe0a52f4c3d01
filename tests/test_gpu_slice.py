"""Spectrum slicing (zolo_slice) against LAPACK on dense-sized pencils: every
eigenvalue of (lo, hi) exactly once, in order, eigenvalues to 1e-10, residuals
1e-8.  Within a slice the Rayleigh-Ritz step makes the vectors B-orthonormal to
rounding; across slices the vectors are independently converged eigenvectors
of distinct eigenvalues, B-orthogonal only up to their residuals (1e-8), hence
the 1e-8 bound on the joined block."""
import sys

import numpy as np
import pytest

import pencils
from oracle.dense import pencil_eigh_lapack
from oracle.subspace import b_orthonormality, inf_norm, rel_residuals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
zolo = pytest.importorskip("paper_1701_08935_amd")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return zolo.Context(0)


@pytest.mark.parametrize("gen,shape,i0,i1,slices", [("grid7", (10, 10, 10), 300, 420, 4),
                                                     ("grid7", (10, 10, 10), 0, 40, 3),
                                                     ("grid27p", (7, 8, 6), 100, 180, 2)])
def test_slice_matches_lapack(ctx, gen, shape, i0, i1, slices):
    gp = getattr(pencils, gen)(shape[0], ny=shape[1], nz=shape[2])
    A, B = gp.scipy()
    lam, _ = pencil_eigh_lapack(A.toarray(), B.toarray())
    lo = 0.5 * (lam[i0 - 1] + lam[i0]) if i0 > 0 else lam[0] - 1.0
    hi = 0.5 * (lam[i1 - 1] + lam[i1])
    ref = lam[(lam > lo) & (lam < hi)]
    say(f"slice {gen} {shape}: ({lo:.6g}, {hi:.6g}) holds {len(ref)} eigenvalues, {slices} slices")
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
    o = zolo.zolo_opts_default()
    o.r1 = 0
    o.max_subspace_iter = 6
    eig, vec, st, rc = zolo.zolo_slice(ctx, P, lo, hi, slices, o)
    say(f"  rc={rc} found={len(eig)} count={st['inertia_count']} gmres={st['n_gmres_total']} "
        f"resid={st['max_resid']:.2e} t_gaps={st['t_gaps']:.2f}s")
    assert rc == 0 and st["inertia_count"] == len(ref) == len(eig)
    eig = np.array(eig)
    assert np.all(np.diff(eig) > 0)
    assert np.max(np.abs(eig - ref) / np.abs(ref)) < 1e-10
    X = vec.cpu().numpy()
    assert np.max(rel_residuals(A, B, eig, X, inf_norm(A), inf_norm(B))) < 1e-8
    assert b_orthonormality(B, X) < 1e-8

"""Parity at full size: the 48^3 layered elasticity workload (4 x 4 x 4
substructures of 12^3, adaptive tau = 10) in the configuration bench.py
times.

The oracle's global form of Algorithm 2 does not fit at this size, so the
GPU results are checked on what the oracle can compute one by one and on
properties that hold at any size:
- glob counts and Nc equal the oracle's analysis of the same mesh;
- on sampled faces, the eigenvalues of the face-pair problem (Sec. 3,
  eq. (eig-matrix)) equal the oracle's dense factor-space eigensolve, and
  the selected rows span the same space;
- the PCG solution satisfies the assembled system R^T A R u = R^T f
  (eq. (assembled)), assembled by the oracle: the true residual is at the
  PCG tolerance relative to the initial residual of the reduced problem
  (zero interface, interior Dirichlet solves -- the oracle's own);
- every pair eigenproblem converged, the indicator omega is below tau and
  the Lanczos minimum eigenvalue is at least 1 (Sec. 2);
- two solves give the same bits.
"""
import numpy as np
import pytest

import meshgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TAU = 10.0
SAMPLE_FACES = (0, 71, 143)
_state = {}


def _run():
    if "b" in _state:
        return _state
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0910_5863_amd import BDDC
    p = meshgen.elasticity_layers_48()
    b = BDDC()
    b.setup(p, "ce")
    info0 = b.info()
    ai = b.adapt(TAU)
    b.factor()
    f = torch.from_numpy(p.f).to("cuda:0")
    u, pinfo = b.pcg_solve(f)
    u2, _ = b.pcg_solve(f)
    _state.update(p=p, b=b, info0=info0, ai=ai, u=u.cpu().numpy()[:, 0],
                  u2=u2.cpu().numpy()[:, 0], pinfo=pinfo[0])
    return _state


def _oracle():
    if "S" not in _state:
        from oracle.fem import Substructures
        from oracle.interface import Interface
        from oracle.cov import Constraints
        st = _run()
        S = Substructures(st["p"])
        itf = Interface(S)
        _state.update(S=S, itf=itf, cons=Constraints(itf, "ce"))
    return _state


def test_fullsize_structure():
    st = _oracle()
    c = st["itf"].counts()
    i = st["info0"]
    assert (i.n_corners, i.n_edges, i.n_faces) == (c["corners"], c["edges"], c["faces"]) == (72, 108, 144)
    assert i.nc == st["cons"].Nc()
    assert i.n_glob == st["p"].n_glob == 345744


def test_fullsize_solution_residual_and_spectrum():
    st = _oracle()
    from oracle.bddc import HarmonicExtension
    K = st["S"].assembled()
    f = st["p"].f
    u0 = HarmonicExtension(st["S"], st["itf"]).interior_solve(f)
    r0 = np.linalg.norm(f - K @ u0)
    r = np.linalg.norm(f - K @ st["u"])
    # PCG stops at ||r_k|| <= 1e-8 ||r_0|| on its recursively updated
    # residual of the interface problem, whose operator is the sum of dense
    # Schur complements formed in FP64; with a coefficient contrast of 1e6
    # their rounding puts the true residual a few times above that (2.3e-8
    # relative where the recursive residual reads 7.2e-9), so 5e-8 is asserted
    assert r <= 5e-8 * r0, (r, r0)
    ai, pi = st["ai"], st["pinfo"]
    assert ai.unconverged == 0 and ai.n_pairs == 144
    assert ai.omega < TAU
    assert pi.converged and pi.lmin > 1 - 1e-9
    assert np.array_equal(st["u"], st["u2"])


@pytest.mark.parametrize("f", SAMPLE_FACES)
def test_fullsize_face_eigs_and_rows(f):
    from oracle.adapt import PairProblem, schur_dense
    st = _oracle()
    S, itf, cons, b = st["S"], st["itf"], st["cons"], st["b"]
    gi = itf.face_ids[f]
    subs = sorted(itf.globs[gi]["subs"])
    Sd = {s: schur_dense(S, itf, s) for s in subs}
    pp = PairProblem(S, itf, cons, gi, Sd)
    lam, W = pp.solve()
    lam_ref = lam[::-1]
    lam_gpu = b.face_eigs(f)
    k = int(np.sum(lam_ref >= TAU))
    m = min(len(lam_gpu), k + 1)
    np.testing.assert_allclose(lam_gpu[:m], lam_ref[:m], rtol=1e-6)
    rows, dofs, _ = b.face_rows(f)
    assert np.array_equal(dofs, itf.globs[gi]["dofs"])
    assert rows.shape[0] == k
    if k:
        d = pp.rows(W[:, lam >= TAU])
        ref = pp.face_part(d, itf)
        qa, _ = np.linalg.qr(rows.T)
        qb, _ = np.linalg.qr(ref.T)
        cos = np.linalg.svd(qa.T @ qb)[1]
        assert cos.min() > 1 - 1e-6, (f, cos.min())

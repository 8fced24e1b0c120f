"""GMRES and the exterior Dirichlet solve, with the oracle's direct QBX as
the matvec (no GPU)."""
import numpy as np
import pytest

import oracle
from paper_1602_05301_amd import inputs
from paper_1602_05301_amd.solve import Oversampled, gl_interp, gmres, plane_wave


def test_gmres_matches_dense_solve():
    """A well-conditioned complex system: GMRES (with and without restarts)
    against numpy's LU solve."""
    rng = np.random.default_rng(0)
    n = 120
    A = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = np.linalg.solve(A, b)
    for restart in (200, 15):
        x, info = gmres(lambda v: A @ v, b, tol=1e-12, restart=restart, maxiter=2000)
        assert info["converged"], info["residual"]
        assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-10
        assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-12


def test_gmres_exact_in_few_steps():
    """A matrix with three distinct eigenvalues: GMRES is exact after three
    steps (the Krylov space holds the solution)."""
    rng = np.random.default_rng(1)
    n = 50
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.repeat([1.0, 2.0 + 1j, -3.0], [20, 20, 10])
    A = (Q * lam) @ Q.conj().T
    b = rng.standard_normal(n) + 0j
    x, info = gmres(lambda v: A @ v, b, tol=1e-13, restart=50, maxiter=50)
    assert info["iterations"] <= 4
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) < 1e-12


def _cfie_oracle(g, fine, omega, p):
    src = Oversampled(g, fine)
    tc = np.arange(g.n, dtype=np.int32)

    def apply(s):
        sf = src.upsample(s)
        return oracle.direct_qbx(omega, p, src, g.sx, g.sy, (1j * omega * sf)[None], sf[None], tgt_ctr=tc)[0]
    return apply, src


def test_gl_interp_exact_for_polynomials():
    """Interpolation from 16 to 64 Gauss nodes reproduces degree-15 polynomials."""
    x16 = np.polynomial.legendre.leggauss(16)[0]
    x64 = np.polynomial.legendre.leggauss(64)[0]
    c = np.random.default_rng(2).standard_normal(16)
    P = np.polynomial.Polynomial(c)
    assert np.max(np.abs(gl_interp(16, 64) @ P(x16) - P(x64))) < 1e-12


def test_exterior_dirichlet_point_source():
    """Sec. 1 eq. extdir with u = D[sigma] + i omega S[sigma]: boundary data
    from H0(omega |x - x0|), x0 inside the curve, give back that field
    outside (the exterior problem has one solution).  Sources oversampled
    4x (Table 1); the second-kind equation converges in few iterations."""
    omega, p = 5.0, 12
    g = inputs.ellipse(48, 16, a=1.0, b=0.6)
    fine = inputs.ellipse(48, 64, a=1.0, b=0.6)
    x0 = np.array([0.15, -0.1])
    from scipy.special import hankel1
    hank = lambda x, y: hankel1(0, omega * np.hypot(x - x0[0], y - x0[1]))
    f = hank(g.sx, g.sy)
    A, src = _cfie_oracle(g, fine, omega, p)
    sigma, info = gmres(A, f, tol=1e-12, restart=100, maxiter=200)
    assert info["converged"] and info["iterations"] < 60, info
    th = np.linspace(0, 2 * np.pi, 40, endpoint=False)
    tx, ty = 1.6 * np.cos(th), 1.3 * np.sin(th)
    sf = src.upsample(sigma)
    u = oracle.direct_qbx(omega, p, src, tx, ty, (1j * omega * sf)[None], sf[None])[0]
    err = np.max(np.abs(u - hank(tx, ty))) / np.max(np.abs(hank(tx, ty)))
    print(f"iterations {info['iterations']}, field error {err:.2e}")
    assert err < 1e-9


def test_plane_wave_default_direction():
    """The incident wave of the paper's scattering run: unit direction (-2, 1)/sqrt(5)."""
    u = plane_wave(3.0, np.array([1.0]), np.array([2.0]))
    assert np.allclose(u, np.exp(1j * 3.0 * (-2.0 + 2.0) / np.sqrt(5.0)))


def test_source_nodes_column_choice():
    """Table 1 lookup: the first column whose tolerance is at most eps."""
    from paper_1602_05301_amd.solve import source_nodes
    assert source_nodes(16, 1e-3) == 32 and source_nodes(16, 1e-6) == 48
    assert source_nodes(16, 5e-7) == 64           # between columns: the tighter one
    assert source_nodes(4, 1e-2) == 12 and source_nodes(2, 1e-15) == 32
    with pytest.raises(ValueError):
        source_nodes(6, 1e-6)


def test_source_nodes_meet_tolerance_on_circle():
    """With the tabulated source nodes, on-curve QBX of S and D on the unit
    circle (64 panels of 16 nodes, omega 10, p 12) is within each column's
    tolerance of the closed forms (i pi R/2) J_m H_m and
    (i pi omega R/2) J_m' H_m."""
    from scipy.special import hankel1, jv, jvp
    from paper_1602_05301_amd.solve import source_nodes
    omega, R, p = 10.0, 1.0, 12
    g = inputs.circle(64, 16, radius=R)
    th = np.arctan2(g.sy, g.sx)
    x = omega * R
    tc = np.arange(g.n, dtype=np.int32)
    for eps in (1e-3, 1e-6, 1e-9):
        fine = inputs.circle(64, source_nodes(16, eps), radius=R)
        src = Oversampled(g, fine)
        thf = np.arctan2(fine.sy, fine.sx)
        for m in (0, 5, 12):
            e = np.exp(1j * m * th)
            sig = np.exp(1j * m * thf)[None]
            uS = oracle.direct_qbx(omega, p, src, g.sx, g.sy, sig, None, tgt_ctr=tc)[0]
            uD = oracle.direct_qbx(omega, p, src, g.sx, g.sy, None, sig, tgt_ctr=tc)[0]
            S = (1j * np.pi * R / 2) * jv(m, x) * hankel1(m, x) * e
            D = (1j * np.pi * omega * R / 2) * jvp(m, x) * hankel1(m, x) * e
            assert np.max(np.abs(uS - S)) / np.max(np.abs(S)) < eps
            assert np.max(np.abs(uD - D)) / np.max(np.abs(D)) < eps

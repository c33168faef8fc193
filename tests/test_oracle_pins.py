"""Pins of the oracle against facts that do not come from the oracle itself:
closed-form eigenpairs and manufactured solutions, matrices built here from
Kronecker products, dense solves, triangular solves, exact transfer identities,
and the five-view stencil update of the paper's "Numerical Python" section.

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand, a wrong weight) fails one of them.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import torch

import oracle as O
from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# --- independent constructions -------------------------------------------------

def lap1d(n, h=None):
    h = 1.0 / (n + 1) if h is None else h
    return (np.diag(2.0 * np.ones(n)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)) / h ** 2


def lap_kron(d, n):
    """Discrete Laplacian on n^d nodes, x fastest, as a Kronecker sum."""
    T = lap1d(n)
    Id = np.eye(n)
    if d == 1:
        return T
    if d == 2:
        return np.kron(Id, T) + np.kron(T, Id)
    return np.kron(Id, np.kron(Id, T)) + np.kron(Id, np.kron(T, Id)) + np.kron(T, np.kron(Id, Id))


def eigvec(d, n, k):
    """prod_a sin(j_a k_a pi h) on the interior, shape (n,)*d indexed [z][y][x]."""
    h = 1.0 / (n + 1)
    j = np.arange(1, n + 1)
    v = np.ones((1,) * d)
    for ax in range(d):
        s = np.sin(j * k[ax] * math.pi * h)
        shape = [1] * d
        shape[d - 1 - ax] = n
        v = v * s.reshape(shape)
    return v


def eigval(d, n, k):
    h = 1.0 / (n + 1)
    return 4.0 / h ** 2 * sum(math.sin(k[a] * math.pi * h / 2) ** 2 for a in range(d))


def colour_mask(d, n):
    idx = np.indices((n,) * d) + 1           # 1-based, axes [z][y][x]
    return (idx.sum(axis=0) % 2) == 0        # red


# --- Q1 operator: closed-form eigenpairs --------------------------------------

@pytest.mark.parametrize("d,n,k", [(1, 31, (3,)), (2, 15, (2, 5)), (2, 31, (7, 1)), (3, 7, (1, 2, 3)),
                                   (3, 15, (4, 1, 6))])
def test_q1_eigenpairs(d, n, k):
    v = eigvec(d, n, k)
    Av = O.apply(v)
    lam = eigval(d, n, k)
    assert np.abs(Av - lam * v).max() <= 1e-13 * lam * np.abs(v).max()


@pytest.mark.parametrize("d,n", [(1, 15), (2, 7), (3, 3)])
def test_q1_assembled_matches_kronecker(d, n):
    assert np.abs(O.assemble(d, n) - lap_kron(d, n)).max() <= 1e-12 * (n + 1) ** 2


# --- Q2 whole solver against dense solves ----------------------------------------

@pytest.mark.parametrize("d,n", [(1, 63), (2, 31), (3, 15)])
def test_q2_dense_poisson(d, n):
    f = I.normal_rhs(n, d, 11)
    x = np.linalg.solve(lap_kron(d, n), f.ravel())
    res = O.solve(f, tol=1e-13, opts=O.Opts(ncoarse=1 if d == 1 else 3))
    assert res.status == 0
    assert np.abs(res.u.ravel() - x).max() <= 1e-11 * np.abs(x).max()


def test_q2_dense_varcoef():
    n = 31
    a = I.lognormal_coef_2d(n, 4001)
    f = I.normal_rhs(n, 2, 4501)
    M = O.assemble(2, n, a=a)
    x = np.linalg.solve(M, f.ravel())
    res = O.solve(f, a=a, tol=1e-13)
    assert res.status == 0
    assert np.abs(res.u.ravel() - x).max() <= 1e-11 * np.abs(x).max()


def test_varcoef_operator_structure():
    """Harmonic face means: the matrix is symmetric positive definite, a
    constant coefficient c gives exactly c times the Laplacian, and it has the
    5-point sparsity pattern of the Laplacian."""
    n = 15
    a = I.lognormal_coef_2d(n, 4002)
    M = O.assemble(2, n, a=a)
    L = lap_kron(2, n)
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0
    assert np.array_equal(M != 0, L != 0)
    c = 3.0
    Mc = O.assemble(2, n, a=np.full((n + 2, n + 2), c))
    assert np.abs(Mc - c * L).max() <= 1e-13 * c * np.abs(L).max()


# --- Q3 / Q4 discretisation: manufactured solutions ---------------------------------

@pytest.mark.parametrize("d,n", [(1, 255), (2, 63), (2, 255), (3, 31)])
def test_q3_mms_discrete_exact(d, n):
    h = 1.0 / (n + 1)
    x = I.grid_x(n)
    s = np.sin(math.pi * x)
    u = np.ones((1,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[d - 1 - ax] = n
        u = u * s.reshape(shape)
    f = d * math.pi ** 2 * u
    ch = math.pi ** 2 * h ** 2 / (4 * math.sin(math.pi * h / 2) ** 2)
    res = O.solve(f, tol=1e-12, opts=O.Opts(ncoarse=1 if d == 1 else 3), maxc=60)
    assert np.abs(res.u - ch * u).max() <= 1e-10 * np.abs(u).max()


def test_q3_mms_order():
    errs = []
    for n in (31, 63, 127):
        x = I.grid_x(n)
        u = np.outer(np.sin(math.pi * x), np.sin(math.pi * x))
        res = O.solve(2 * math.pi ** 2 * u, tol=1e-12)
        errs.append(np.abs(res.u - u).max())
    for e0, e1 in zip(errs, errs[1:]):
        assert abs(e0 / e1 - 4.0) < 0.01


def test_q4_mms_varcoef_order():
    """a = 1 + sin(2 pi x) sin(2 pi y)/2, u = sin(pi x) sin(pi y),
    f = -div(a grad u) computed analytically."""
    pi = math.pi
    errs = []
    for n in (31, 63, 127):
        xn = np.arange(0, n + 2) / (n + 1)
        Y, X = np.meshgrid(xn, xn, indexing="ij")
        a = 1.0 + 0.5 * np.sin(2 * pi * X) * np.sin(2 * pi * Y)
        Xi, Yi = X[1:-1, 1:-1], Y[1:-1, 1:-1]
        u = np.sin(pi * Xi) * np.sin(pi * Yi)
        ai = a[1:-1, 1:-1]
        ax = pi * np.cos(2 * pi * Xi) * np.sin(2 * pi * Yi)
        ay = pi * np.sin(2 * pi * Xi) * np.cos(2 * pi * Yi)
        ux = pi * np.cos(pi * Xi) * np.sin(pi * Yi)
        uy = pi * np.sin(pi * Xi) * np.cos(pi * Yi)
        lap = -2 * pi ** 2 * u
        f = -(ax * ux + ay * uy + ai * lap)
        res = O.solve(np.ascontiguousarray(f), a=np.ascontiguousarray(a), tol=1e-12, maxc=80)
        assert res.status == 0
        errs.append(np.abs(res.u - u).max())
    for e0, e1 in zip(errs, errs[1:]):
        assert abs(e0 / e1 - 4.0) < 0.1


# --- Q5 transfers -------------------------------------------------------------------

@pytest.mark.parametrize("d,nc", [(1, 7), (2, 3), (2, 7), (3, 3)])
def test_q5_restriction_is_scaled_prolongation_transpose(d, nc):
    n = 2 * nc + 1
    mc, m = nc ** d, n ** d
    P = np.zeros((m, mc))
    for j in range(mc):
        e = np.zeros(mc)
        e[j] = 1.0
        u = np.zeros(m)
        P[:, j] = O.prolong_add(e.reshape((nc,) * d), u.reshape((n,) * d)).ravel()
    R = np.zeros((mc, m))
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1.0
        R[:, j] = O.restrict(e.reshape((n,) * d)).ravel()
    assert np.array_equal(R, P.T / 2 ** d)
    # prolongation reproduces linear functions away from the boundary
    assert np.array_equal(P.sum(axis=1) > 0, np.ones(m, dtype=bool))


def test_q5_galerkin_1d():
    """In 1D, R A_h P equals the rediscretised A_2h exactly (a textbook
    identity that fixes the scale of R and P against the operator)."""
    nc, n = 15, 31
    P = np.zeros((n, nc))
    for j in range(nc):
        e = np.zeros(nc)
        e[j] = 1.0
        P[:, j] = O.prolong_add(e, np.zeros(n))
    R = P.T / 2
    assert np.abs(R @ lap1d(n) @ P - lap1d(nc)).max() <= 1e-9


def test_q5_prolongation_of_linear_data():
    """Bilinear interpolation of a coarse sample of a bilinear function is exact."""
    nc = 7
    n = 2 * nc + 1
    xc = np.arange(1, nc + 1) / (nc + 1)
    xf = np.arange(1, n + 1) / (n + 1)
    g = lambda X, Y: X * Y + 0.5 * X - 0.25 * Y   # noqa: E731  (bilinear)
    Yc, Xc = np.meshgrid(xc, xc, indexing="ij")
    Yf, Xf = np.meshgrid(xf, xf, indexing="ij")
    uf = O.prolong_add(np.ascontiguousarray(g(Xc, Yc)), np.zeros((n, n)))
    inner = (slice(1, n - 1), slice(1, n - 1))
    assert np.abs(uf[inner] - g(Xf, Yf)[inner]).max() <= 1e-15


# --- Q6 / Q7 / Q11 smoothers ---------------------------------------------------------

@pytest.mark.parametrize("d,n,k", [(1, 31, (5,)), (2, 31, (3, 9)), (3, 15, (2, 7, 5))])
def test_q6_jacobi_eigen_damping(d, n, k):
    v = eigvec(d, n, k)
    om = 2 * d / (2 * d + 1)
    h = 1.0 / (n + 1)
    u = O.sweep(v.copy(), np.zeros_like(v), kind=O.JACOBI, omega=om)
    g = 1 - (2 * om / d) * sum(math.sin(k[a] * math.pi * h / 2) ** 2 for a in range(d))
    assert np.abs(u - g * v).max() <= 1e-14 * np.abs(v).max()


@pytest.mark.parametrize("d,n", [(1, 31), (2, 15), (3, 7)])
def test_q6_rbgs_black_residual_zero(d, n):
    u = I.normal_rhs(n, d, 3)
    f = I.normal_rhs(n, d, 4)
    O.sweep(u, f, kind=O.RBGS)
    r = O.residual(u, f)
    black = ~colour_mask(d, n)
    assert np.abs(r[black]).max() <= 1e-12 * np.abs(f).max()


def test_q7_paper_five_view_jacobi():
    """2D Jacobi with omega = 4/5 and f = 0 equals 0.2*(c+up+down+left+right),
    written with five shifted views of one bordered array as in the paper's
    'Numerical Python' example (coefficient read as applying to all five)."""
    n = 33
    full = np.zeros((n + 2, n + 2))
    full[1:-1, 1:-1] = I.uniform_field((n, n), 8)
    center = full[1:-1, 1:-1]
    up = full[0:-2, 1:-1]
    down = full[2:, 1:-1]
    left = full[1:-1, 0:-2]
    right = full[1:-1, 2:]
    work = 0.2 * (center + up + down + left + right)
    u = np.ascontiguousarray(full[1:-1, 1:-1]).copy()
    O.sweep(u, np.zeros_like(u), kind=O.JACOBI, omega=0.8)
    assert np.abs(u - work).max() <= 1e-15 * 5


@pytest.mark.parametrize("d,n", [(1, 15), (2, 7), (3, 5)])
def test_q11_sweeps_as_triangular_solves(d, n):
    """Lexicographic GS is (D+L) u' = f - U u; red-black GS is the same with the
    red nodes ordered first; Jacobi is u + w D^-1 (f - A u).  Matrices here
    are the Kronecker Laplacian, solves by scipy."""
    A = lap_kron(d, n)
    u0 = I.normal_rhs(n, d, 5)
    f = I.normal_rhs(n, d, 6)
    # lexicographic
    L = np.tril(A)
    Uu = np.triu(A, 1)
    want = sla.solve_triangular(L, f.ravel() - Uu @ u0.ravel(), lower=True)
    got = O.sweep(u0.copy(), f, kind=O.LEX).ravel()
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    # red-black
    red = colour_mask(d, n).ravel()
    perm = np.concatenate([np.nonzero(red)[0], np.nonzero(~red)[0]])
    Ap = A[np.ix_(perm, perm)]
    want_p = sla.solve_triangular(np.tril(Ap), f.ravel()[perm] - np.triu(Ap, 1) @ u0.ravel()[perm], lower=True)
    want = np.empty_like(want_p)
    want[perm] = want_p
    got = O.sweep(u0.copy(), f, kind=O.RBGS).ravel()
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    # weighted Jacobi
    om = 0.7
    want = u0.ravel() + om * (f.ravel() - A @ u0.ravel()) / np.diag(A)
    got = O.sweep(u0.copy(), f, kind=O.JACOBI, omega=om).ravel()
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_q11_varcoef_sweep_as_triangular_solve():
    n = 7
    a = I.lognormal_coef_2d(n, 4003)
    A = O.assemble(2, n, a=a)
    u0 = I.normal_rhs(n, 2, 7)
    f = I.normal_rhs(n, 2, 8)
    red = colour_mask(2, n).ravel()
    perm = np.concatenate([np.nonzero(red)[0], np.nonzero(~red)[0]])
    Ap = A[np.ix_(perm, perm)]
    want_p = sla.solve_triangular(np.tril(Ap), f.ravel()[perm] - np.triu(Ap, 1) @ u0.ravel()[perm], lower=True)
    want = np.empty_like(want_p)
    want[perm] = want_p
    got = O.sweep(u0.copy(), f, a=a, kind=O.RBGS).ravel()
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


# --- Q8 coarsest solves --------------------------------------------------------------

@pytest.mark.parametrize("d", [1, 2, 3])
def test_q8_one_point(d):
    f = np.full((1,) * d, 0.37)
    u = O.vcycle(np.zeros_like(f), f, opts=O.Opts(ncoarse=1))
    h = 0.5
    assert abs(u.ravel()[0] - 0.37 * h * h / (2 * d)) <= 1e-16


@pytest.mark.parametrize("d", [2, 3])
def test_q8_three_per_axis(d):
    f = I.normal_rhs(3, d, 9)
    u = O.vcycle(np.zeros_like(f), f, opts=O.Opts(ncoarse=3))
    x = np.linalg.solve(lap_kron(d, 3), f.ravel())
    assert np.abs(u.ravel() - x).max() <= 1e-15 * 16 * np.abs(x).max()


def test_lu_solve_pivoting():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((20, 20))
    M[0, 0] = 0.0
    b = rng.standard_normal(20)
    assert np.abs(O.lu_solve(M, b) - np.linalg.solve(M, b)).max() <= 1e-10


# --- Q9 convergence -------------------------------------------------------------------

@pytest.mark.parametrize("d,n,smoother", [(2, 127, O.RBGS), (3, 31, O.RBGS), (2, 63, O.JACOBI),
                                          (1, 1023, O.LEX)])
def test_q9_monotone(d, n, smoother):
    f = I.normal_rhs(n, d, 12)
    res = O.solve(f, tol=1e-10, opts=O.Opts(smoother=smoother, ncoarse=1 if d == 1 else 3))
    assert res.status == 0
    assert np.all(np.diff(res.hist) < 0)


@pytest.mark.parametrize("d,n", [(2, 15), (3, 7)])
def test_q9_spectral_radius(d, n):
    """The V-cycle with f = 0 is the linear map I - B A; its spectral radius
    (numpy eigvals of the assembled map) is the asymptotic factor that power
    iteration with the cycle itself must find."""
    m = n ** d
    M = np.zeros((m, m))
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1.0
        M[:, j] = O.vcycle(e.reshape((n,) * d).copy(), np.zeros((n,) * d)).ravel()
    rho = np.abs(np.linalg.eigvals(M)).max()
    assert 0.0 < rho < 0.2
    u = I.normal_rhs(n, d, 13)
    for _ in range(60):
        nrm = np.linalg.norm(u)
        u = O.vcycle(u / nrm, np.zeros_like(u))
    measured = np.linalg.norm(u)
    assert abs(measured - rho) <= 0.05 * rho


# --- Q10 linearity and scaling ----------------------------------------------------------

def test_q10_ir_fp64_reproduces_plain():
    n = 63
    f = I.normal_rhs(n, 2, 14)
    a = I.lognormal_coef_2d(n, 4004)
    p = O.solve(f, a=a, tol=1e-10)
    q = O.solve_ir(f, a=a, prec=O.F64, tol=1e-10)
    assert p.cycles == q.cycles
    assert np.abs(p.hist - q.hist).max() <= 1e-13 * 1
    assert np.abs(p.u - q.u).max() <= 1e-12 * np.abs(p.u).max()


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_q10_power_of_two_scaling(dt):
    n = 31
    f = I.normal_rhs(n, 2, 15).astype(dt)
    u1 = O.vcycle(np.zeros_like(f), f)
    u2 = O.vcycle(np.zeros_like(f), (f * 8).astype(dt))
    assert np.array_equal(u1 * 8, u2)


def test_q10_affine():
    """V(u, f) = u + B (f - A u): the cycle is affine in (u, f)."""
    n = 31
    f = I.normal_rhs(n, 2, 16)
    u0 = I.normal_rhs(n, 2, 17)
    v1 = O.vcycle(u0.copy(), f)
    # same cycle applied to the error equation from zero
    e = O.vcycle(np.zeros_like(f), O.residual(u0, f))
    assert np.abs(v1 - (u0 + e)).max() <= 1e-12 * np.abs(v1).max()


# --- Q12 (oracle side) precision --------------------------------------------------------

@pytest.mark.parametrize("prec", [O.F32, O.BF16])
def test_q12_ir_reaches_fp64_tolerance(prec):
    n = 63
    f = I.normal_rhs(n, 3 - 1, 18)
    ref = O.solve(f, tol=1e-13)
    res = O.solve_ir(f, prec=prec, tol=1e-10)
    assert res.status == 0
    assert res.hist[-1] <= 1e-10
    assert np.abs(res.u - ref.u).max() <= 1e-8 * np.abs(ref.u).max()


def test_bf16_round_matches_torch():
    """The oracle's own bfloat16 rounding against torch's float->bfloat16
    conversion (round to nearest even), ties and specials included."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal(2000).astype(np.float32) * np.float32(1e3)
    bits = np.array([0x3f808000, 0x3f818000, 0x3f80ffff, 0x7f7fffff, 0x00000001, 0x80008000],
                    dtype=np.uint32).view(np.float32)
    x = np.concatenate([x, bits, np.array([np.inf, -np.inf, 0.0, -0.0], dtype=np.float32)])
    got = O.bf16_round(x)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert np.isnan(O.bf16_round(np.array([np.nan], dtype=np.float32))[0])


# --- the C1 configuration on the oracle -------------------------------------------------

def test_c1_lex_gs_1d():
    f = I.sine_plus_noise_1d(1023, 1)
    res = O.solve(f, tol=1e-10, opts=O.Opts(smoother=O.LEX, ncoarse=1))
    assert res.status == 0 and res.cycles <= 20
    assert np.all(np.diff(res.hist) < 0)

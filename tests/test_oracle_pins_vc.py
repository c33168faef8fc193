"""Pins of the oracle's variable-coefficient hierarchy and of its bfloat16
store points, against constructions written here from the definitions:

* the coarse nodal coefficient by injection (coarse node I on fine node 2I,
  boundary nodes included) against numpy strided slicing;
* the diffusion operator against a numpy assembly of the harmonic-mean
  five-point stencil;
* whole V-cycles on the diffusion operator against a second, dense-matrix
  multigrid written here (numpy / scipy: red-black Gauss-Seidel as a
  triangular solve in red-first order, transfers as Kronecker products of the
  1D interpolation matrix, coarse operators rediscretised on the injected
  coefficient, a dense coarsest solve);
* the spectral radius of the diffusion V-cycle's iteration matrix, from that
  dense multigrid, against power iteration with the oracle's cycle;
* the bfloat16 store points of the bf16-state cycle: the correction, the
  coarsest solution, the smoother updates and the first refinement step
  produce bfloat16-representable values, equal to the rounding of the exact
  (float64) result where the float arithmetic is exact.

Each pin is chosen so that a slip in the oracle fails it: injecting from node
2I + 1 instead of 2I changes the coarse operator (and every cycle), and a
dropped bf16 rounding leaves values with more than 8 significant bits.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

import oracle as O
from paper_1210_7774_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# --- independent constructions --------------------------------------------------

def vc_matrix(n, a):
    """-div(a grad) on the n x n interior of [0,1]^2, h = 1/(n+1): face
    weights are harmonic means of the nodal a (array (n+2, n+2) indexed
    [y][x], boundary included); unknowns x fastest."""
    h2 = (1.0 / (n + 1)) ** 2
    m = n * n
    A = np.zeros((m, m))
    for j in range(1, n + 1):
        for i in range(1, n + 1):
            p = (i - 1) + n * (j - 1)
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                w = 2.0 * a[j, i] * a[jj, ii] / (a[j, i] + a[jj, ii])
                A[p, p] += w / h2
                if 1 <= ii <= n and 1 <= jj <= n:
                    A[p, (ii - 1) + n * (jj - 1)] -= w / h2
    return A


def interp_1d(nc):
    """Linear interpolation from nc coarse to 2 nc + 1 fine interior nodes
    (coarse node I sits on fine node 2I; boundary values 0)."""
    n = 2 * nc + 1
    P = np.zeros((n, nc))
    for I_ in range(1, nc + 1):
        P[2 * I_ - 1, I_ - 1] = 1.0          # fine node 2I (0-based 2I-1)
        P[2 * I_ - 2, I_ - 1] += 0.5         # fine node 2I-1
        P[2 * I_, I_ - 1] += 0.5             # fine node 2I+1
    return P


def red_first(n):
    idx = np.indices((n, n)) + 1
    red = ((idx.sum(axis=0) % 2) == 0).ravel()
    return np.concatenate([np.nonzero(red)[0], np.nonzero(~red)[0]])


class DenseMG:
    """A dense-matrix V(nu1, nu2) multigrid for the 2D diffusion operator."""

    def __init__(self, n, a, ncoarse=3, nu1=2, nu2=2):
        self.levels = []
        while True:
            A = vc_matrix(n, a)
            perm = red_first(n)
            Ap = A[np.ix_(perm, perm)]
            self.levels.append(dict(n=n, A=A, perm=perm, L=np.tril(Ap), U=np.triu(Ap, 1)))
            if n <= ncoarse:
                break
            nc = (n - 1) // 2
            P1 = interp_1d(nc)
            self.levels[-1]["P"] = np.kron(P1, P1)          # x fastest: kron(P_y, P_x)
            self.levels[-1]["R"] = np.kron(P1, P1).T / 4.0
            a = a[::2, ::2]
            n = nc
        self.nu1, self.nu2 = nu1, nu2

    def sweep(self, lv, u, f):
        p = lv["perm"]
        x = sla.solve_triangular(lv["L"], f[p] - lv["U"] @ u[p], lower=True)
        out = np.empty_like(x)
        out[p] = x
        return out

    def cycle(self, u, f, l=0, kind="V"):
        """V: one coarse V-cycle; W: two coarse W-cycles (the second from the
        first's result); F: a coarse F-cycle then a coarse V-cycle."""
        lv = self.levels[l]
        if l == len(self.levels) - 1:
            return np.linalg.solve(lv["A"], f)
        for _ in range(self.nu1):
            u = self.sweep(lv, u, f)
        fc = lv["R"] @ (f - lv["A"] @ u)
        uc = np.zeros_like(fc)
        for sub in {"V": "V", "W": "WW", "F": "FV"}[kind]:
            uc = self.cycle(uc, fc, l + 1, sub)
        u = u + lv["P"] @ uc
        for _ in range(self.nu2):
            u = self.sweep(lv, u, f)
        return u

    def vcycle(self, u, f, l=0):
        return self.cycle(u, f, l, "V")

    def fmg(self, f, l=0, kind="V", ncyc=1):
        """Nested iteration: restrict f down, solve the coarsest level,
        interpolate up, ncyc cycles per level."""
        lv = self.levels[l]
        if l == len(self.levels) - 1:
            return np.linalg.solve(lv["A"], f)
        uc = self.fmg(lv["R"] @ f, l + 1, kind, ncyc)
        u = lv["P"] @ uc
        for _ in range(ncyc):
            u = self.cycle(u, f, l, kind)
        return u


def is_bf16(x):
    x = np.asarray(x, dtype=np.float32)
    return np.array_equal(x.view(np.uint32) & np.uint32(0xFFFF), np.zeros(x.shape, dtype=np.uint32))


def torch_bf16(x64):
    """float64 -> float32 -> bfloat16 (round to nearest even) -> float32, by torch."""
    t = torch.from_numpy(np.asarray(x64, dtype=np.float64)).to(torch.float32).to(torch.bfloat16)
    return t.to(torch.float32).numpy()


# --- S12: coarse coefficient by injection ------------------------------------------

@pytest.mark.parametrize("n", [7, 15, 63])
def test_s12_coarsen_coef_2d_is_strided_slice(n):
    a = I.lognormal_coef_2d(n, 4010)
    got = O.coarsen_coef(a, 2)
    assert got.shape == ((n - 1) // 2 + 2,) * 2
    assert np.array_equal(got, a[::2, ::2])


@pytest.mark.parametrize("n", [3, 7, 15])
def test_s12_coarsen_coef_3d_is_strided_slice(n):
    a = I.uniform_field((n + 2,) * 3, 4011) + 0.5
    got = O.coarsen_coef(np.ascontiguousarray(a), 3)
    assert np.array_equal(got, a[::2, ::2, ::2])


def test_s12_coarsen_coef_float_build():
    n = 31
    a = I.lognormal_coef_2d(n, 4012).astype(np.float32)
    assert np.array_equal(O.coarsen_coef(a, 2), a[::2, ::2])


# --- O3 / S11: the diffusion operator --------------------------------------------------

@pytest.mark.parametrize("n", [7, 15])
def test_s11_operator_against_numpy_assembly(n):
    a = I.lognormal_coef_2d(n, 4013)
    want = vc_matrix(n, a)
    assert np.abs(O.assemble(2, n, a=a) - want).max() <= 1e-13 * np.abs(want).max()


# --- O10 / O8: whole diffusion V-cycles against the dense multigrid ---------------------

@pytest.mark.parametrize("n,cycles", [(7, 2), (15, 3), (31, 2)])
def test_vc_vcycle_iterates_against_dense_multigrid(n, cycles):
    a = I.lognormal_coef_2d(n, 4014 + n)
    f = I.normal_rhs(n, 2, 4515 + n)
    mg = DenseMG(n, a)
    u_np = np.zeros(n * n)
    u_or = np.zeros((n, n))
    for _ in range(cycles):
        u_np = mg.vcycle(u_np, f.ravel())
        O.vcycle(u_or, f, a=a)
        assert np.abs(u_or.ravel() - u_np).max() <= 1e-12 * np.abs(u_np).max()


def test_vc_two_grid_coarse_correction_only():
    """V(0,0)-like check of the coarse-grid correction alone (no smoothing):
    u + P A_c^-1 R (f - A u) with A_c from the injected coefficient."""
    n = 15
    a = I.lognormal_coef_2d(n, 4020)
    f = I.normal_rhs(n, 2, 4521)
    u0 = I.normal_rhs(n, 2, 4522)
    nc = 7
    P = np.kron(interp_1d(nc), interp_1d(nc))
    Ac = vc_matrix(nc, a[::2, ::2])
    want = u0.ravel() + P @ np.linalg.solve(Ac, (P.T / 4.0) @ (f.ravel() - vc_matrix(n, a) @ u0.ravel()))
    got = O.vcycle(u0.copy(), f, a=a, opts=O.Opts(nu1=0, nu2=0, ncoarse=7))
    assert np.abs(got.ravel() - want).max() <= 1e-12 * np.abs(want).max()


# --- Q9 for the diffusion operator -----------------------------------------------------

@pytest.mark.parametrize("n", [15, 31])
def test_q9_vc_spectral_radius(n):
    """The iteration matrix of the diffusion V-cycle (f = 0), assembled column
    by column from the dense multigrid, equals the oracle's, and its spectral
    radius is the factor power iteration with the oracle's cycle finds."""
    a = I.lognormal_coef_2d(n, 4030 + n)
    mg = DenseMG(n, a)
    m = n * n
    M = np.zeros((m, m))
    zero = np.zeros(m)
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1.0
        M[:, j] = mg.vcycle(e, zero)
    # the oracle's cycle on a few columns
    for j in (0, m // 3, m - 1):
        e = np.zeros((n, n))
        e.ravel()[j] = 1.0
        col = O.vcycle(e, np.zeros((n, n)), a=a).ravel()
        assert np.abs(col - M[:, j]).max() <= 1e-12
    rho = np.abs(np.linalg.eigvals(M)).max()
    assert 0.0 < rho < 0.5
    # power iteration: the mean log growth over the last 100 of 200 cycles
    u = I.normal_rhs(n, 2, 4040 + n)
    logs = []
    for _ in range(200):
        u = O.vcycle(u, np.zeros_like(u), a=a)
        nrm = np.linalg.norm(u)
        logs.append(np.log(nrm))
        u /= nrm
    measured = np.exp(np.mean(logs[100:]))
    assert abs(measured - rho) <= 0.05 * rho


# --- S19: bfloat16 store points of the bf16-state cycle -----------------------------------

def test_s19_prolong_add_rounds_to_bf16():
    """u + P ec stored as bf16: inputs are small integers, so the float sum is
    exact and the stored value must be the bf16 rounding of the exact value."""
    nc = 15
    n = 2 * nc + 1
    g = I.rng(4050)
    ec = g.integers(-1000, 1000, size=(nc, nc)).astype(np.float32)
    u = g.integers(-3000, 3000, size=(n, n)).astype(np.float32)
    P = np.kron(interp_1d(nc), interp_1d(nc))
    exact = u.astype(np.float64).ravel() + P @ ec.astype(np.float64).ravel()
    got = O.prolong_add(ec, u.copy(), bf16=True)
    assert is_bf16(got)
    assert np.array_equal(got.ravel(), torch_bf16(exact))
    # without the flag the same sum is stored exactly (it is not bf16-representable)
    plain = O.prolong_add(ec, u.copy(), bf16=False)
    assert np.array_equal(plain.ravel().astype(np.float64), exact)
    assert not is_bf16(plain)


@pytest.mark.parametrize("d", [2, 3])
def test_s19_coarsest_solution_rounds_to_bf16(d):
    """On a 3^d grid the cycle is the coarsest FP64 solve; in the bf16 build
    its result is the bf16 rounding of the float of the dense solution."""
    f = (I.normal_rhs(3, d, 4051 + d) * 100).astype(np.float32)
    got = O.vcycle(np.zeros_like(f), f, opts=O.Opts(ncoarse=3, bf16=True))
    T = (np.diag(2.0 * np.ones(3)) - np.diag(np.ones(2), 1) - np.diag(np.ones(2), -1)) * 16.0
    E = np.eye(3)
    A = np.kron(E, T) + np.kron(T, E) if d == 2 else (np.kron(E, np.kron(E, T)) + np.kron(E, np.kron(T, E))
                                                      + np.kron(T, np.kron(E, E)))
    x = np.linalg.solve(A, f.astype(np.float64).ravel())
    assert is_bf16(got)
    assert np.abs(got.ravel() - torch_bf16(x)).max() <= 2.0 ** -7 * np.abs(x).max()


def _poisson_half_update(u, f, h2, mask):
    """Point update (h^2 f + sum of the 4 neighbours) / 4 at the masked nodes,
    every neighbour from u (zero outside), by shifted views."""
    b = np.zeros((u.shape[0] + 2, u.shape[1] + 2))
    b[1:-1, 1:-1] = u
    nb = b[:-2, 1:-1] + b[2:, 1:-1] + b[1:-1, :-2] + b[1:-1, 2:]
    return np.where(mask, (h2 * f + nb) / 4.0, u)


def test_s19_rbgs_sweep_stores_bf16():
    """Red-black sweep in the bf16 build: red values are the bf16 rounding of
    the update from the old black values, black values the rounding of the
    update from the rounded red values (each within one bf16 ulp of this
    float64 construction, which rounds at the same points)."""
    n = 31
    h2 = (1.0 / (n + 1)) ** 2
    u = torch_bf16(I.normal_rhs(n, 2, 4053)).reshape(n, n).astype(np.float64)
    f = (I.normal_rhs(n, 2, 4054) * 1000.0).astype(np.float32)
    idx = np.indices((n, n)) + 1
    red = (idx.sum(axis=0) % 2) == 0
    want = _poisson_half_update(u, f.astype(np.float64), h2, red)
    want = np.where(red, torch_bf16(want).reshape(n, n), want)
    want = _poisson_half_update(want, f.astype(np.float64), h2, ~red)
    want = np.where(~red, torch_bf16(want).reshape(n, n), want)
    got = O.sweep(u.astype(np.float32), f, kind=O.RBGS, bf16=True)
    assert is_bf16(got)
    assert np.all(np.abs(got - want) <= 2.0 ** -8 * np.abs(want))


def test_s19_jacobi_sweep_stores_bf16():
    n = 31
    om = 0.8
    h2 = (1.0 / (n + 1)) ** 2
    u = torch_bf16(I.normal_rhs(n, 2, 4058)).reshape(n, n).astype(np.float64)
    f = (I.normal_rhs(n, 2, 4059) * 1000.0).astype(np.float32)
    full = _poisson_half_update(u, f.astype(np.float64), h2, np.ones((n, n), dtype=bool))
    want = torch_bf16(u + om * (full - u)).reshape(n, n)
    got = O.sweep(u.astype(np.float32), f, kind=O.JACOBI, omega=om, bf16=True)
    assert is_bf16(got)
    assert np.all(np.abs(got - want) <= 2.0 ** -8 * np.abs(want))


@pytest.mark.parametrize("nu2", [0, 2])
def test_s19_first_refinement_step_is_bf16(nu2):
    """The first refinement step from u = 0 sets u = (double) e, e the bf16-state
    inner cycle's iterate, so every entry of u is bf16-representable -- with
    no post-smoothing (nu2 = 0) the last store is the coarse-grid correction."""
    n = 63
    f = I.normal_rhs(n, 2, 4055)
    res = O.solve_ir(f, opts=O.Opts(nu2=nu2), prec=O.BF16, tol=0.0, maxc=1)
    assert res.cycles == 1
    assert is_bf16(res.u.astype(np.float32))
    assert np.array_equal(res.u.astype(np.float32).astype(np.float64), res.u)
    # the FP32-state step gives values that are not all bf16-representable
    r32 = O.solve_ir(f, opts=O.Opts(nu2=nu2), prec=O.F32, tol=0.0, maxc=1)
    assert not is_bf16(r32.u.astype(np.float32))
    # and the bf16 step is the FP32 step up to bf16 resolution
    assert np.abs(res.u - r32.u).max() <= 0.05 * np.abs(r32.u).max()


def test_s19_vc_bf16_cycle_levels():
    """A bf16-state diffusion V(2,0) cycle (coarse levels included) stores only
    bf16 values and stays within bf16 resolution of the FP32 cycle."""
    n = 31
    a = I.lognormal_coef_2d(n, 4056)
    f = I.normal_rhs(n, 2, 4057).astype(np.float32)
    af = a.astype(np.float32)
    got = O.vcycle(np.zeros_like(f), f, a=af, opts=O.Opts(nu2=0, bf16=True))
    ref = O.vcycle(np.zeros_like(f), f, a=af, opts=O.Opts(nu2=0))
    assert is_bf16(got)
    assert np.abs(got - ref).max() <= 0.05 * np.abs(ref).max()


# --- NEXT-2: W- and F-cycles, full multigrid --------------------------------------------

@pytest.mark.parametrize("kind", ["W", "F"])
@pytest.mark.parametrize("n,vc", [(15, True), (31, True), (31, False)])
def test_wf_cycle_iterates_against_dense_multigrid(kind, n, vc):
    a = I.lognormal_coef_2d(n, 4080 + n) if vc else np.ones((n + 2, n + 2))
    f = I.normal_rhs(n, 2, 4580 + n)
    mg = DenseMG(n, a)
    u_np = np.zeros(n * n)
    u_or = np.zeros((n, n))
    for _ in range(2):
        u_np = mg.cycle(u_np, f.ravel(), kind=kind)
        O.cycle(u_or, f, a=a if vc else None, kind=kind)
        assert np.abs(u_or.ravel() - u_np).max() <= 1e-12 * np.abs(u_np).max()


@pytest.mark.parametrize("kind", ["V", "W", "F"])
def test_fmg_against_dense_multigrid(kind):
    n = 31
    a = I.lognormal_coef_2d(n, 4090)
    f = I.normal_rhs(n, 2, 4590)
    want = DenseMG(n, a).fmg(f.ravel(), kind=kind)
    got = O.fmg(f, a=a, kind=kind)
    assert np.abs(got.ravel() - want).max() <= 1e-12 * np.abs(want).max()


def test_w_and_f_cycles_contract_faster_than_v():
    """The iteration matrices' spectral radii (from the dense multigrid):
    rho_W <= rho_F <= rho_V, each < 0.2, and power iteration with the
    oracle's W-cycle finds rho_W."""
    n = 15
    a = I.lognormal_coef_2d(n, 4091)
    mg = DenseMG(n, a)
    m = n * n
    rho = {}
    for kind in "VWF":
        M = np.zeros((m, m))
        for j in range(m):
            e = np.zeros(m)
            e[j] = 1.0
            M[:, j] = mg.cycle(e, np.zeros(m), kind=kind)
        rho[kind] = np.abs(np.linalg.eigvals(M)).max()
    assert rho["W"] <= rho["F"] * (1 + 1e-9) and rho["F"] <= rho["V"] * (1 + 1e-9) and rho["V"] < 0.5
    u = I.normal_rhs(n, 2, 4092)
    logs = []
    for _ in range(120):
        O.cycle(u, np.zeros_like(u), a=a, kind="W")
        nrm = np.linalg.norm(u)
        logs.append(np.log(nrm))
        u /= nrm
    assert abs(np.exp(np.mean(logs[60:])) - rho["W"]) <= 0.05 * rho["W"]


def _sine_problem(n):
    import math
    h = 1.0 / (n + 1)
    x = I.grid_x(n)
    u = np.outer(np.sin(math.pi * x), np.sin(math.pi * x))
    ch = math.pi ** 2 * h ** 2 / (4 * math.sin(math.pi * h / 2) ** 2)
    return u, 2 * math.pi ** 2 * u, ch


@pytest.mark.parametrize("kind", ["W", "F"])
def test_q3_fmg_reaches_discretisation_error(kind):
    """One FMG pass (one W- or F-cycle per level) on the sine problem: the
    error against the continuous solution is the discretisation error
    (c_h - 1) max|u| ~ (pi^2 h^2 / 12) max|u| to within 2 %, the algebraic
    error (against the exact discrete solution c_h u) a small fraction of it."""
    for n in (63, 127, 255):
        u, f, ch = _sine_problem(n)
        disc = (ch - 1) * np.abs(u).max()
        got = O.fmg(f, kind=kind)
        assert abs(np.abs(got - u).max() / disc - 1.0) <= 0.02, n
        assert np.abs(got - ch * u).max() <= 0.02 * disc, n


def test_q3_fmg_v_error_is_second_order():
    """FMG with one V(2,2) per level: the algebraic error stays a bounded
    fraction of the discretisation error as h shrinks, so the total error is
    O(h^2): ratio 4 per halving of h."""
    errs = []
    for n in (63, 127, 255):
        u, f, ch = _sine_problem(n)
        disc = (ch - 1) * np.abs(u).max()
        got = O.fmg(f, kind="V")
        assert np.abs(got - ch * u).max() <= 0.7 * disc
        errs.append(np.abs(got - u).max())
    for e0, e1 in zip(errs, errs[1:]):
        assert abs(e0 / e1 - 4.0) < 0.1


def test_fmg_is_linear():
    f = I.normal_rhs(31, 2, 4093)
    assert np.array_equal(O.fmg(f * 8.0, kind="F") / 8.0, O.fmg(f, kind="F"))


def test_solve_with_fmg_and_cycle_types():
    """Solves to 1e-10 with every cycle type, with and without a leading FMG
    pass: the FMG pass leaves a residual far below one cycle's from zero."""
    f = I.normal_rhs(63, 2, 4094)
    for kind in "VWF":
        plain = O.solve(f, tol=1e-10, kind=kind)
        first = O.solve(f, tol=1e-10, kind=kind, fmg=True)
        assert plain.status == 0 and first.status == 0
        assert first.hist[1] < plain.hist[1]
        assert np.linalg.norm(O.residual(first.u, f)) / np.linalg.norm(f) <= 1e-10


@pytest.mark.parametrize("kind", ["W", "F"])
def test_fp64_refinement_with_wf_cycles_reproduces_plain_solve(kind):
    """Refinement with FP64 inner cycles is the plain cycle written as a
    correction (the cycle is affine in u, so u + C(0; f - A u) = C(u; f)):
    both histories agree step for step away from the rounding floor; the
    float inner cycles of the same type reach the FP64 tolerance too."""
    f = I.normal_rhs(63, 2, 4095)
    plain = O.solve(f, tol=1e-10, kind=kind)
    ir = O.solve_ir(f, prec=O.F64, tol=1e-10, kind=kind)
    assert plain.status == 0 and ir.status == 0 and plain.cycles == ir.cycles
    big = plain.hist >= 1e-8
    assert np.allclose(ir.hist[big], plain.hist[big], rtol=1e-7, atol=0)
    assert np.allclose(ir.hist, plain.hist, rtol=1e-4, atol=0)
    v = O.solve_ir(f, prec=O.F64, tol=0.0, maxc=1, kind="V").hist[1]
    assert ir.hist[1] < v
    for prec in (O.F32, O.BF16):
        r = O.solve_ir(f, prec=prec, tol=1e-10, kind=kind)
        assert r.status == 0
        assert np.linalg.norm(O.residual(r.u, f)) / np.linalg.norm(f) <= 1e-10

"""Pins of the vector-engine oracle (oracle/vector.py), CPU only.

The oracle's exact overlap test is checked against an independent mask
painting; its kernel formation against partitions worked out by hand from
the paper's two blockable properties (the paper's own five-view Jacobi loop
among them); and the rule's purpose -- a kernel may run block by block in any
block order -- against instruction-by-instruction execution, with a
deliberately wrong formation failing the same check.
"""
import numpy as np
import pytest

import oracle.jacobi5 as J
import oracle.vector as V
from paper_1210_7774_amd import inputs as I


def as_oracle(instrs):
    conv = lambda x: V.View(*x) if isinstance(x, tuple) else x
    return [(op, conv(out), tuple(conv(x) for x in ins)) for op, out, ins in instrs]


def fresh(data):
    return {i: np.array(d, dtype=np.float64, copy=True) for i, d in enumerate(data)}


def view2d(base, W, r0, c0, R, C, sr=1, sc=1):
    return V.View(base, r0 * W + c0, (R, C), (sr * W, sc))


def test_share_matches_mask_painting():
    g = np.random.default_rng(5)
    for _ in range(400):
        W = 11
        vs = []
        for _ in range(2):
            sr = int(g.choice([1, 2, -1]))
            sc = int(g.choice([1, 2, -1, 3]))
            R, C = int(g.integers(1, 4)), int(g.integers(1, 4))
            r0 = int(g.integers(0, 10 - 2 * R)) if sr > 0 else int(g.integers(2 * R, 10))
            c0 = int(g.integers(0, 11 - 3 * C)) if sc > 0 else int(g.integers(C, 11))
            vs.append(V.View(0, r0 * W + c0, (R, C), (sr * W, sc)))
        mask = np.zeros(10 * W, dtype=bool)
        V.nd({0: mask}, vs[0])[...] = True
        want = bool(V.nd({0: mask}, vs[1]).any())
        assert V.share(vs[0], vs[1]) == want


def test_same_view_reading():
    a = V.View(0, 0, (8,), (1,))
    assert V.same(a, V.View(0, 0, (8,), (1,)))
    assert not V.same(a, V.View(0, 7, (8,), (-1,)))          # same elements, other order
    assert V.share(a, V.View(0, 7, (8,), (-1,)))
    assert V.same(V.View(0, 3, (1, 4), (99, 1)), V.View(0, 3, (1, 4), (5, 1)))  # unit axis stride is free
    assert not V.share(V.View(0, 0, (4,), (2,)), V.View(0, 1, (4,), (2,)))     # interleaved


def paper_loop(W=10, H=8):
    """The paper's five-view Jacobi loop body (printed form: work = center,
    then work += 0.2 * (up + down + left + right), then center = work) as
    bytecode; bases: 0 = full (H x W), 1 = work, 2..5 temporaries."""
    R, C = H - 2, W - 2
    center, up, down = view2d(0, W, 1, 1, R, C), view2d(0, W, 0, 1, R, C), view2d(0, W, 2, 1, R, C)
    left, right = view2d(0, W, 1, 0, R, C), view2d(0, W, 1, 2, R, C)
    work = V.View(1, 0, (R, C), (C, 1))
    t = [V.View(2 + k, 0, (R, C), (C, 1)) for k in range(4)]
    return [
        ("copy", work, (center,)),
        ("add", t[0], (up, down)),
        ("add", t[1], (t[0], left)),
        ("add", t[2], (t[1], right)),
        ("multiply", t[3], (t[2], 0.2)),
        ("add", work, (work, t[3])),
        ("copy", center, (work,)),
        ("free", t[0], ()), ("free", t[1], ()), ("free", t[2], ()), ("free", t[3], ()),
    ]


def test_paper_loop_forms_two_kernels():
    """By hand: the copy into work, the three additions into fresh
    temporaries, the scaling and the in-place update of work share no data
    with each other's inputs except identical views, so they form one kernel;
    the copy back into center writes data that the kernel reads through the
    shifted views up/down/left/right, so it starts the second; the frees
    belong to none."""
    kernel_of, nk = V.form_kernels(paper_loop())
    assert kernel_of == [0, 0, 0, 0, 0, 0, 1, -1, -1, -1, -1]
    assert nk == 2


def test_small_cases_by_hand():
    a, b = V.View(0, 0, (6,), (1,)), V.View(1, 0, (6,), (1,))
    a1 = V.View(0, 1, (6,), (1,))
    r = V.View(2, 0, (1,), (1,))
    # in-place chain on one view: one kernel
    assert V.form_kernels([("add", a, (a, b)), ("multiply", a, (a, 2.0)), ("sqrt", b, (a,))])[0] == [0, 0, 0]
    # reading a shifted view of a kernel output: new kernel
    assert V.form_kernels([("add", a, (a, b)), ("copy", b, (a1,))])[0] == [0, 1]
    # writing a view the kernel read shifted: new kernel
    assert V.form_kernels([("copy", b, (a1,)), ("negative", a, (b,))])[0] == [0, 1]
    # a reduction of a kernel output joins; reading its result starts a new kernel
    assert V.form_kernels([("multiply", b, (a, a)), ("add_reduce", r, (b,)),
                           ("copy", V.View(2, 0, (1,), (1,)), (r,))])[0] == [0, 0, 1]
    # another index space: new kernel
    assert V.form_kernels([("copy", b, (a,)), ("copy", V.View(3, 0, (3,), (1,)), (V.View(0, 0, (3,), (2,)),))])[0] \
        == [0, 1]
    # interleaved halves of one array are blockable
    ev, od = V.View(0, 0, (3,), (2,)), V.View(0, 1, (3,), (2,))
    assert V.form_kernels([("add", ev, (ev, od)), ("subtract", od, (od, ev))])[0] == [0, 0]  # identical or disjoint
    assert V.form_kernels([("add", ev, (ev, 1.0)), ("add", od, (od, 1.0))])[0] == [0, 0]
    od_next = V.View(0, 3, (3,), (2,))                    # the odd half shifted by one pair
    assert V.form_kernels([("add", ev, (ev, od)), ("copy", od_next, (ev,))])[0] == [0, 1]


def test_paper_loop_matches_jacobi_oracle():
    """The bytecode of the loop with the average read of the update (the
    five views summed centre first, then scaled by 0.2) run instruction by
    instruction equals the jacobi5 oracle bit for bit."""
    H, W = 12, 17
    full = I.uniform_field((H, W), 8)
    R, C = H - 2, W - 2
    center, up, down = view2d(0, W, 1, 1, R, C), view2d(0, W, 0, 1, R, C), view2d(0, W, 2, 1, R, C)
    left, right = view2d(0, W, 1, 0, R, C), view2d(0, W, 1, 2, R, C)
    work = V.View(1, 0, (R, C), (C, 1))
    body = [("add", work, (center, up)), ("add", work, (work, down)), ("add", work, (work, left)),
            ("add", work, (work, right)), ("multiply", work, (work, 0.2)), ("copy", center, (work,))]
    bases = {0: full.reshape(-1).copy(), 1: np.zeros(R * C)}
    for _ in range(4):
        V.execute(body, bases)
    assert np.array_equal(bases[0].reshape(H, W), J.jacobi5(full, 4))
    assert V.form_kernels(body)[0] == [0, 0, 0, 0, 0, 1]


@pytest.mark.parametrize("seed", range(40))
def test_blocked_execution_equals_sequential(seed):
    """Every formed kernel run block by block, blocks in a random order, gives
    what instruction-by-instruction execution gives (bitwise; reductions
    combine per-block partial sums, so sums agree to rounding)."""
    bases, instrs, data = I.vector_program(seed, reductions=(seed % 3 == 0))
    prog = as_oracle(instrs)
    want, got = fresh(data), fresh(data)
    V.execute(prog, want)
    V.execute_blocked(prog, got, blocks=int(1 + seed % 7), rng=np.random.default_rng(seed))
    for k in want:
        if bases[k][0] == 1:
            assert np.allclose(got[k], want[k], rtol=1e-14, atol=0, equal_nan=True)
        else:
            assert np.array_equal(got[k], want[k], equal_nan=True), k


def test_wrong_formation_breaks_blocked_execution():
    """Forcing the paper's loop into a single kernel (the copy back into
    center fused with the kernel that reads center's neighbours) makes the
    blocked result depend on the block order -- the case the rule excludes."""
    H, W = 8, 10
    full = I.uniform_field((H, W), 9).reshape(-1)
    prog = paper_loop(W, H)
    R, C = H - 2, W - 2
    data = [full] + [np.zeros(R * C) for _ in range(5)]
    want = fresh(data)
    V.execute(prog, want)
    bad = ([0, 0, 0, 0, 0, 0, 0, -1, -1, -1, -1], 1)
    diff = False
    for s in range(5):
        got = fresh(data)
        V.execute_blocked(prog, got, blocks=4, rng=np.random.default_rng(s), partition=bad)
        diff = diff or not np.array_equal(got[0], want[0])
    assert diff
    good = fresh(data)
    V.execute_blocked(prog, good, blocks=4, rng=np.random.default_rng(0))
    assert np.array_equal(good[0], want[0])


def test_random_programs_fuse_and_split():
    """The random programs exercise both outcomes of the rule."""
    sizes = []
    for seed in range(40):
        _, instrs, _ = I.vector_program(seed)
        kernel_of, nk = V.form_kernels(as_oracle(instrs))
        sizes += [int(c) for c in np.bincount([k for k in kernel_of if k >= 0]) if c > 0]
    assert min(sizes) == 1 and max(sizes) >= 4


def test_self_overlapping_instruction_is_staged():
    """a[1:] = a[:-1] reads every old value first (whole-array meaning): the
    input is staged through a fresh base, the staged copy forms a kernel and
    the shifted store another; blocked execution equals the shift."""
    a = np.arange(10, dtype=np.float64)
    prog = [("copy", V.View(0, 1, (9,), (1,)), (V.View(0, 0, (9,), (1,)),))]
    kernel_of, nk = V.form_kernels(prog)
    assert kernel_of == [1] and nk == 2
    want = np.concatenate([[0.0], np.arange(9.0)])
    seq, blk = {0: a.copy()}, {0: a.copy()}
    V.execute(prog, seq)
    V.execute_blocked(prog, blk, blocks=3, rng=np.random.default_rng(1))
    assert np.array_equal(seq[0], want) and np.array_equal(blk[0], want)


# ---------------------------------------------------------------- synthetic stencil

@pytest.mark.parametrize("shape,steps", [((3, 3), 2), ((5, 7), 3), ((12, 9), 10), ((3, 20), 1), ((2, 5), 4)])
def test_stencil9_views_match_loops_bitwise(shape, steps):
    import oracle.stencil as S
    full = I.uniform_field(shape, 9)
    assert np.array_equal(S.stencil9(full, steps), S.stencil9_loops(full, steps))


def test_stencil9_invariants():
    """Constants are fixed points; the ring never changes; a single interior
    spike spreads to its 3 x 3 neighbourhood with weight 1/9 after one step
    and the sum over a zero-ring interior is non-increasing."""
    import oracle.stencil as S
    c = np.full((8, 11), 0.75)
    assert np.array_equal(S.stencil9(c, 5), c)
    full = I.uniform_field((9, 13), 10)
    out = S.stencil9(full, 6)
    ring = np.ones_like(full, dtype=bool)
    ring[1:-1, 1:-1] = False
    assert np.array_equal(out[ring], full[ring])
    z = np.zeros((9, 9))
    z[4, 4] = 9.0
    one = S.stencil9(z, 1)
    assert np.array_equal(one[3:6, 3:6], np.ones((3, 3))) and one.sum() == 9.0
    g = np.zeros((20, 20))
    g[1:-1, 1:-1] = I.uniform_field((18, 18), 11)
    sums = [S.stencil9(g, k)[1:-1, 1:-1].sum() for k in range(5)]
    assert all(b <= a + 1e-12 for a, b in zip(sums, sums[1:]))

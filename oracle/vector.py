"""Oracle of the vector-bytecode engine (TEST INFRASTRUCTURE ONLY: the tests,
the smoke check and the benchmark's CPU baseline may use it).

What the paper defines and this module writes out:
  * an array-base is a contiguous allocation; an array-view addresses the
    elements base[offset + sum_d i_d * stride_d], 0 <= i_d < shape_d
    (section "Numerical Python");
  * vector bytecode is an assembly-like list of instructions, one opcode each,
    whose operands are array-views (section "Bytecode"); a batch is executed
    instruction by instruction (the meaning every fused execution must keep);
  * the vector engine forms kernels by scanning the batch in order and adding
    each instruction to the current kernel while it is blockable with it
    (section "Vector Engine"): with A the kernel's instructions and N the
    new one, (1) N's inputs and A's outputs, and (2) N's output and A's
    inputs and outputs, either share no element or are precisely the same
    data; a kernel runs block by block, every instruction on one block before
    the next block.

Readings where the paper is silent (the engine takes the same ones):
  * "precisely the same data" is the same view: equal offset, shape and
    strides (strides of unit-length axes do not matter); views that cover the
    same elements in another order share data without being the same;
  * a kernel is one index space: every instruction in it has the same shape
    (the output's, or the input's for a reduction);
  * a reduction (sum / max of all input elements into a one-element output)
    may join a kernel like any instruction, but its output exists only when
    the kernel is finished: an instruction that reads or writes a reduction
    output of the kernel starts a new kernel;
  * system instructions (sync, discard, free) are not computation: they
    belong to no kernel and do not break one; nor do instructions over an
    empty index space, which do nothing.

Instructions are (op, out, ins): op a name from OPS, out a View, ins a tuple
of Views or Python floats (constants).  Bases are 1-D numpy arrays in a dict
keyed by base id.  Arithmetic is numpy's, in the base's dtype, one
instruction at a time over whole views (no blocking, no reordering).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class View:
    base: int
    offset: int
    shape: tuple
    strides: tuple

    @property
    def size(self) -> int:
        return int(np.prod(self.shape)) if self.shape else 1

    def key(self):
        """Offset, shape and strides with unit-axis strides cleared."""
        st = tuple(0 if n == 1 else s for n, s in zip(self.shape, self.strides))
        return (self.base, self.offset, tuple(self.shape), st)


UNARY = {
    "copy": lambda x: x,
    "negative": np.negative,
    "absolute": np.absolute,
    "sqrt": np.sqrt,
    "exp": np.exp,
    "log": np.log,
    "sin": np.sin,
    "cos": np.cos,
    "tanh": np.tanh,
}
BINARY = {
    "add": np.add,
    "subtract": np.subtract,
    "multiply": np.multiply,
    "divide": np.divide,
    "maximum": np.maximum,
    "minimum": np.minimum,
    "power": np.power,
    "greater": np.greater,
    "greater_equal": np.greater_equal,
    "less": np.less,
    "less_equal": np.less_equal,
    "equal": np.equal,
    "not_equal": np.not_equal,
}
TERNARY = {"where": lambda c, a, b: np.where(c != 0, a, b)}
REDUCE = {"add_reduce": np.sum, "maximum_reduce": np.max}
SYSTEM = ("sync", "discard", "free")
OPS = tuple(UNARY) + tuple(BINARY) + tuple(TERNARY) + tuple(REDUCE) + SYSTEM


def nd(bases, v: View) -> np.ndarray:
    """The numpy view of `v` on its base (writable)."""
    b = bases[v.base]
    it = b.itemsize
    lo = v.offset + sum(min(0, (n - 1) * s) for n, s in zip(v.shape, v.strides))
    hi = v.offset + sum(max(0, (n - 1) * s) for n, s in zip(v.shape, v.strides))
    if lo < 0 or hi >= b.size:
        raise IndexError("view %s outside its base of %d elements" % (v, b.size))
    return np.lib.stride_tricks.as_strided(b[v.offset:], shape=v.shape, strides=tuple(s * it for s in v.strides))


def _operand(bases, x, dtype):
    if isinstance(x, View):
        return nd(bases, x)
    return dtype.type(x)


def execute(batch, bases) -> None:
    """Run a batch instruction by instruction, in place on `bases`."""
    with np.errstate(all="ignore"):
        _execute(batch, bases)


def _execute(batch, bases) -> None:
    for op, out, ins in batch:
        if op in SYSTEM:
            continue
        o = nd(bases, out)
        dt = o.dtype
        if op == "copy":
            x = ins[0]
            o[...] = nd(bases, x).astype(dt) if isinstance(x, View) else dt.type(x)
            continue
        args = [_operand(bases, x, dt) for x in ins]
        if op in UNARY:
            r = UNARY[op](args[0])
        elif op in BINARY:
            r = BINARY[op](args[0], args[1])
        elif op in TERNARY:
            r = TERNARY[op](*args)
        elif op in REDUCE:
            r = REDUCE[op](args[0])
        else:
            raise ValueError("unknown op " + op)
        o[...] = np.asarray(r).astype(dt)


# ---------------------------------------------------------------- the blockable rule

def elements(v: View) -> np.ndarray:
    """Every element offset `v` addresses (small views: tests only)."""
    off = np.full((), v.offset, dtype=np.int64)
    for n, s in zip(v.shape, v.strides):
        off = off[..., None] + np.arange(n, dtype=np.int64) * s
    return off.ravel()


def same(a: View, b: View) -> bool:
    return a.key() == b.key()


def share(a: View, b: View) -> bool:
    """Whether two views address a common element (exact)."""
    if a.base != b.base:
        return False
    return np.intersect1d(elements(a), elements(b)).size > 0


def _separate(a: View, b: View) -> bool:
    """No common element, or precisely the same data."""
    return same(a, b) or not share(a, b)


def _ins(instr):
    return [x for x in instr[2] if isinstance(x, View)]


def _shape(instr):
    op, out, ins = instr
    return tuple(ins[0].shape) if op in REDUCE else tuple(out.shape)


def _size(instr):
    return int(np.prod(_shape(instr)))


def blockable(kernel, new) -> bool:
    """The paper's two properties for instruction `new` against the kernel's
    instructions, plus the one-index-space and reduction readings above."""
    if not kernel:
        return True
    if _shape(new) != _shape(kernel[0]):
        return False
    outs = [k[1] for k in kernel]
    ins = [x for k in kernel for x in _ins(k)]
    red = [k[1] for k in kernel if k[0] in REDUCE]
    for x in _ins(new):                              # property 1
        if any(not _separate(x, o) for o in outs):
            return False
        if any(share(x, r) for r in red):
            return False
    o = new[1]                                       # property 2
    if any(not _separate(o, y) for y in outs + ins):
        return False
    if any(share(o, r) for r in red):
        return False
    return True


def stage(batch):
    """An instruction whose output shares data with one of its own inputs
    without being the same view cannot run block by block at all (a block
    would read what an earlier block of the same instruction wrote); whole-
    array execution reads every input before writing.  Such an input is read
    from a staged copy: a copy into a fresh base ("stage", i, j) placed right
    before instruction i.  Returns [(instr, i or None)] (None: a staging
    copy)."""
    out = []
    for i, (op, o, ins) in enumerate(batch):
        if op in SYSTEM:
            out.append(((op, o, ins), i))
            continue
        new_ins = []
        for j, x in enumerate(ins):
            if isinstance(x, View) and not same(x, o) and share(x, o):
                n = x.size
                strides = tuple(int(np.prod(x.shape[d + 1:])) for d in range(len(x.shape)))
                t = View(("stage", i, j), 0, tuple(x.shape), strides)
                out.append((("copy", t, (x,)), None))
                x = t
            new_ins.append(x)
        out.append(((op, o, tuple(new_ins)), i))
    return out


def plan(batch):
    """Greedy kernel formation over the staged batch: returns (staged,
    kernel ids of the staged instructions, kernel_of for the original
    instructions (-1 for system instructions), number of kernels)."""
    staged = stage(batch)
    sk, kernel_of = [], [None] * len(batch)
    cur, k = [], -1
    for instr, orig in staged:
        if instr[0] in SYSTEM or _size(instr) == 0:
            sk.append(-1)
            kernel_of[orig] = -1
            continue
        if k < 0 or not blockable(cur, instr):
            k += 1
            cur = []
        cur.append(instr)
        sk.append(k)
        if orig is not None:
            kernel_of[orig] = k
    return staged, sk, kernel_of, k + 1


def form_kernels(batch):
    """Greedy kernel formation: kernel_of[i] for every instruction (-1 for
    system instructions) and the number of kernels."""
    _, _, kernel_of, nk = plan(batch)
    return kernel_of, nk


def execute_blocked(batch, bases, blocks, rng=None, partition=None) -> None:
    """Run a batch kernel by kernel, each kernel data block by data block:
    the flat index space of the kernel is cut into `blocks` contiguous blocks
    (visited in a random order when `rng` is given), and every instruction of
    the kernel runs on one block before the next block starts.  Reductions
    combine their per-block partial results when the kernel ends.
    `partition` (kernel_of, count) replaces the greedy formation (tests of
    what a wrong formation does)."""
    with np.errstate(all="ignore"):
        _execute_blocked(batch, bases, blocks, rng, partition)


def _execute_blocked(batch, bases, blocks, rng, partition) -> None:
    staged, sk, _, nk = plan(batch)
    staged = [x for x, _ in staged]
    if partition is not None:
        assert len(staged) == len(batch), "a forced partition needs a batch without staging"
        sk, nk = partition
    bases = dict(bases)
    for op, o, ins in staged:
        if isinstance(o.base, tuple) and o.base not in bases:
            bases[o.base] = np.zeros(o.size, dtype=bases[ins[0].base].dtype)
    for k in range(nk):
        instrs = [staged[i] for i in range(len(staged)) if sk[i] == k]
        shape = _shape(instrs[0])
        size = int(np.prod(shape)) if shape else 1
        cuts = np.linspace(0, size, blocks + 1).astype(np.int64)
        order = list(range(blocks))
        if rng is not None:
            rng.shuffle(order)
        partial = {}
        for b in order:
            lo, hi = cuts[b], cuts[b + 1]
            if lo == hi:
                continue
            for idx, (op, out, ins) in enumerate(instrs):
                if op in REDUCE:
                    x = _flat_view(bases, ins[0])[lo:hi]
                    p = REDUCE[op](x)
                    partial.setdefault(idx, []).append(p)
                    continue
                dt = bases[out.base].dtype
                if op == "copy":
                    x = ins[0]
                    val = _flat_view(bases, x)[lo:hi].astype(dt) if isinstance(x, View) else dt.type(x)
                    _flat_assign(bases, out, lo, hi, val)
                    continue
                args = [(_flat_view(bases, x)[lo:hi] if isinstance(x, View) else dt.type(x)) for x in ins]
                if op in UNARY:
                    r = UNARY[op](args[0])
                elif op in BINARY:
                    r = BINARY[op](args[0], args[1])
                else:
                    r = TERNARY[op](*args)
                _flat_assign(bases, out, lo, hi, np.asarray(r).astype(dt))
        for idx, parts in partial.items():
            op, out, ins = instrs[idx]
            o = nd(bases, out)
            comb = np.sum if op == "add_reduce" else np.max
            o[...] = np.asarray(comb(np.array(parts))).astype(o.dtype)


def _flat_view(bases, v: View) -> np.ndarray:
    """The elements of `v` in index order, as a 1-D array (a copy when the
    view is not contiguous; reads only)."""
    return np.array(nd(bases, v)).reshape(-1)


def _flat_assign(bases, v: View, lo, hi, val) -> None:
    """Store `val` into elements lo..hi-1 (index order) of view `v`."""
    b = bases[v.base]
    offs = elements(v)[lo:hi]
    b[offs] = val

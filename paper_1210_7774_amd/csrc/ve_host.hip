// The vector-bytecode engine (C-ABI in include/ve.h): the paper's vector
// engine manager (array-bases, late allocation, free / discard) and vector
// engine (kernel formation by the blockable rule, data-blocked execution),
// with kernels generated as HIP source and compiled at run time by hipRTC.
//
// Execution of one batch:
//   1. validate and normalise the views;
//   2. stage inputs that overlap their own instruction's output (a copy into
//      a fresh engine base placed right before the instruction);
//   3. form kernels greedily (section "Vector Engine": add the next
//      instruction while it is blockable with the kernel);
//   4. per kernel: the distinct views become memory operands; a view read
//      before it is written is loaded, a view written is stored once (its
//      last value) unless a later free / discard of its base, with no read
//      in between, makes it dead; values between instructions stay in
//      registers;
//   5. generate, compile (all new kernels of the batch in one hipRTC
//      program, cached by source) and launch in batch order.
// A generated kernel covers its index space in tiles of one row segment of
// 1024 elements (4 per thread, 256 threads); each work-group takes a
// contiguous run of tiles, and the runs are dealt so that each of the 8 XCDs
// holds a contiguous part of the space (neighbouring rows, which shifted
// views re-read, stay in one L2).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "ve.h"

namespace {

constexpr int kMaxInstr = 64, kMaxSlots = 48, kMaxConsts = 32;
constexpr int kThreads = 256, kPerThread = 4, kTile = kThreads * kPerThread;
constexpr int kTR = 16;  // rows of a staged tile
constexpr int kMaxBlocks = 2048;
constexpr int kTempBase = 1 << 30;  // ids of staging bases inside one plan

struct View {
    int base = -1;
    int nd = 0;
    long long off = 0;
    long long shape[VE_MAX_NDIM] = {0, 0, 0, 0};
    long long st[VE_MAX_NDIM] = {0, 0, 0, 0};
    long long size() const
    {
        long long s = 1;
        for (int d = 0; d < nd; ++d) s *= shape[d];
        return s;
    }
    long long lo() const
    {
        long long v = off;
        for (int d = 0; d < nd; ++d) v += std::min(0LL, (shape[d] - 1) * st[d]);
        return v;
    }
    long long hi() const
    {
        long long v = off;
        for (int d = 0; d < nd; ++d) v += std::max(0LL, (shape[d] - 1) * st[d]);
        return v;
    }
};

bool same(const View &a, const View &b)
{
    if (a.base != b.base || a.nd != b.nd || a.off != b.off) return false;
    for (int d = 0; d < a.nd; ++d)
        if (a.shape[d] != b.shape[d] || a.st[d] != b.st[d]) return false;
    return true;
}

bool same_shape(const View &a, const View &b)
{
    if (a.nd != b.nd) return false;
    for (int d = 0; d < a.nd; ++d)
        if (a.shape[d] != b.shape[d]) return false;
    return true;
}

// Whether sum_d k_d s_d = D has a solution with k_d in [kmin_d, kmax_d],
// dimensions taken by decreasing |s|; exact when every |s_d| exceeds what the
// smaller dimensions can reach (then at most two candidates per level), else
// *decided = false.
bool lattice_hit(const std::vector<long long> &s, const std::vector<long long> &kmin,
                 const std::vector<long long> &kmax, size_t d, long long D, bool *decided)
{
    if (d == s.size()) return D == 0;
    long long reach = 0;
    for (size_t e = d + 1; e < s.size(); ++e)
        reach += std::llabs(s[e]) * std::max(std::llabs(kmin[e]), std::llabs(kmax[e]));
    const long long a = std::llabs(s[d]);
    if (a <= reach) {
        *decided = false;
        return true;
    }
    // candidates: floor and ceil of D / s[d]
    const long long q = D / s[d];
    for (long long k = q - 1; k <= q + 1; ++k) {
        if (k < kmin[d] || k > kmax[d]) continue;
        const long long rest = D - k * s[d];
        if (std::llabs(rest) > reach) continue;
        if (lattice_hit(s, kmin, kmax, d + 1, rest, decided)) return true;
        if (!*decided) return true;
    }
    return false;
}

void offsets(const View &v, std::vector<long long> &out)
{
    out.clear();
    out.reserve((size_t)v.size());
    long long idx[VE_MAX_NDIM] = {0, 0, 0, 0};
    for (long long n = 0; n < v.size(); ++n) {
        long long o = v.off;
        for (int d = 0; d < v.nd; ++d) o += idx[d] * v.st[d];
        out.push_back(o);
        for (int d = v.nd - 1; d >= 0; --d) {
            if (++idx[d] < v.shape[d]) break;
            idx[d] = 0;
        }
    }
}

// Whether two views address a common element.  Exact for different bases,
// disjoint extents, equal strides (lattice test) and small views (sorted
// offsets); otherwise answers yes (which only splits kernels).
bool share(const View &a, const View &b)
{
    if (a.base != b.base) return false;
    if (a.size() == 0 || b.size() == 0) return false;
    if (a.hi() < b.lo() || b.hi() < a.lo()) return false;
    if (a.nd == b.nd) {
        bool eq = true;
        for (int d = 0; d < a.nd; ++d) eq = eq && a.st[d] == b.st[d];
        if (eq) {
            std::vector<long long> s, kmin, kmax;
            for (int d = 0; d < a.nd; ++d) {
                if (a.st[d] == 0) {
                    if (a.shape[d] > 1 || b.shape[d] > 1) continue;  // broadcast axis: any k works
                    continue;
                }
                s.push_back(a.st[d]);
                kmin.push_back(-(b.shape[d] - 1));
                kmax.push_back(a.shape[d] - 1);
            }
            std::vector<size_t> ord(s.size());
            for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
            std::sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return std::llabs(s[x]) > std::llabs(s[y]); });
            std::vector<long long> s2, k0, k1;
            for (size_t i : ord) {
                s2.push_back(s[i]);
                k0.push_back(kmin[i]);
                k1.push_back(kmax[i]);
            }
            // element of a at index i equals element of b at index j iff
            // sum (i_d - j_d) s_d = b.off - a.off
            bool decided = true;
            const bool hit = lattice_hit(s2, k0, k1, 0, b.off - a.off, &decided);
            if (decided) return hit;
        }
    }
    if (a.size() <= 65536 && b.size() <= 65536) {
        std::vector<long long> x, y;
        offsets(a, x);
        offsets(b, y);
        std::sort(x.begin(), x.end());
        std::sort(y.begin(), y.end());
        size_t i = 0, j = 0;
        while (i < x.size() && j < y.size()) {
            if (x[i] == y[j]) return true;
            if (x[i] < y[j]) ++i;
            else ++j;
        }
        return false;
    }
    return true;
}

bool separate(const View &a, const View &b) { return same(a, b) || !share(a, b); }

bool is_system(int op) { return op == VE_SYNC || op == VE_DISCARD || op == VE_FREE; }
bool is_reduce(int op) { return op == VE_ADD_REDUCE || op == VE_MAXIMUM_REDUCE; }

int builtin_arity(int op)
{
    switch (op) {
    case VE_COPY: case VE_NEGATIVE: case VE_ABSOLUTE: case VE_SQRT: case VE_EXP: case VE_LOG: case VE_SIN:
    case VE_COS: case VE_TANH: case VE_ADD_REDUCE: case VE_MAXIMUM_REDUCE:
        return 1;
    case VE_ADD: case VE_SUBTRACT: case VE_MULTIPLY: case VE_DIVIDE: case VE_MAXIMUM: case VE_MINIMUM: case VE_POWER:
    case VE_GREATER: case VE_GREATER_EQUAL: case VE_LESS: case VE_LESS_EQUAL: case VE_EQUAL: case VE_NOT_EQUAL:
        return 2;
    case VE_WHERE:
        return 3;
    }
    return -1;
}

// One instruction after validation (and staging): inputs are views (in_view)
// or constants.
struct Ins {
    int op = 0;
    View out;
    View in[VE_MAX_IN];
    bool in_view[VE_MAX_IN] = {false, false, false};
    double cst[VE_MAX_IN] = {0, 0, 0};
    int nin = 0;
    int orig = -1;  // index in the caller's batch; -1 for a staging copy
    const View &space() const { return is_reduce(op) ? in[0] : out; }
    long long size() const { return space().size(); }
};

View from_abi(const ve_view &v)
{
    View r;
    r.base = v.base;
    r.nd = v.ndim;
    r.off = v.offset;
    for (int d = 0; d < VE_MAX_NDIM && d < v.ndim; ++d) {
        r.shape[d] = v.shape[d];
        r.st[d] = v.shape[d] == 1 ? 0 : v.stride[d];  // unit axes: the stride does not matter
    }
    return r;
}

// Convert (without base checks: ve_plan has no engine) and stage.
// `arity(op)` gives the number of operand slots in use.
template <class Arity>
int to_internal(const ve_instr *batch, int n, Arity arity, std::vector<Ins> &out, std::string &err)
{
    out.clear();
    int temp = 0;
    for (int i = 0; i < n; ++i) {
        const ve_instr &b = batch[i];
        Ins x;
        x.op = b.opcode;
        x.orig = i;
        if (b.out.ndim < 1 || b.out.ndim > VE_MAX_NDIM) {
            err = "instruction " + std::to_string(i) + ": output ndim out of range";
            return VE_ERR_ARG;
        }
        x.out = from_abi(b.out);
        if (is_system(b.opcode)) {
            out.push_back(x);
            continue;
        }
        const int na = arity(b.opcode);
        if (na < 0) {
            err = "instruction " + std::to_string(i) + ": unknown opcode " + std::to_string(b.opcode);
            return VE_ERR_ARG;
        }
        x.nin = na;
        int nviews = 0;
        for (int k = 0; k < na; ++k) {
            if (b.in[k].base >= 0) {
                if (b.in[k].ndim < 1 || b.in[k].ndim > VE_MAX_NDIM) {
                    err = "instruction " + std::to_string(i) + ": input ndim out of range";
                    return VE_ERR_ARG;
                }
                x.in[k] = from_abi(b.in[k]);
                x.in_view[k] = true;
                ++nviews;
            } else {
                x.cst[k] = b.cst[k];
            }
        }
        if (is_reduce(x.op)) {
            if (!x.in_view[0] || x.out.size() != 1) {
                err = "instruction " + std::to_string(i) + ": a reduction needs a view input and a one-element output";
                return VE_ERR_ARG;
            }
        } else {
            if (nviews == 0 && x.op != VE_COPY) {
                // all-constant operands: allowed (a fill), the index space is the output's
            }
            for (int k = 0; k < na; ++k)
                if (x.in_view[k] && !same_shape(x.in[k], x.out)) {
                    err = "instruction " + std::to_string(i) + ": input " + std::to_string(k) +
                          " has another shape than the output (broadcast with stride-0 views)";
                    return VE_ERR_ARG;
                }
        }
        for (int d = 0; d < x.out.nd; ++d)
            if (x.out.shape[d] < 0) {
                err = "instruction " + std::to_string(i) + ": negative extent";
                return VE_ERR_ARG;
            }
        // staging: an input that shares elements with this instruction's
        // output without being the same view is read from a copy
        for (int k = 0; k < na; ++k) {
            if (!x.in_view[k] || is_reduce(x.op)) continue;
            if (same(x.in[k], x.out) || !share(x.in[k], x.out)) continue;
            Ins c;
            c.op = VE_COPY;
            c.nin = 1;
            c.orig = -1;
            c.in[0] = x.in[k];
            c.in_view[0] = true;
            View t;
            t.base = kTempBase + temp++;
            t.nd = x.in[k].nd;
            long long s = 1;
            for (int d = t.nd - 1; d >= 0; --d) {
                t.shape[d] = x.in[k].shape[d];
                t.st[d] = t.shape[d] == 1 ? 0 : s;
                s *= t.shape[d];
            }
            c.out = t;
            out.push_back(c);
            x.in[k] = t;
        }
        out.push_back(x);
    }
    return VE_OK;
}

struct KernelPlan {
    std::vector<int> members;  // indices into the staged list
};

// Greedy formation (with the launch-argument caps).
void form(const std::vector<Ins> &ins, std::vector<int> &kid, std::vector<KernelPlan> &kernels)
{
    kid.assign(ins.size(), -1);
    kernels.clear();
    std::vector<View> outs, inps, reds, slots;
    int nconst = 0;
    auto slot_count_with = [&](const Ins &x) {
        int extra = 0;
        std::vector<View> add;
        auto consider = [&](const View &v) {
            for (auto &s : slots)
                if (same(s, v)) return;
            for (auto &s : add)
                if (same(s, v)) return;
            add.push_back(v);
            ++extra;
        };
        for (int k = 0; k < x.nin; ++k)
            if (x.in_view[k]) consider(x.in[k]);
        consider(x.out);
        return (int)slots.size() + extra;
    };
    for (size_t i = 0; i < ins.size(); ++i) {
        const Ins &x = ins[i];
        if (is_system(x.op) || x.size() == 0) continue;
        bool ok = !kernels.empty();
        if (ok) {
            const Ins &f = ins[kernels.back().members.front()];
            ok = same_shape(x.space(), f.space());
            for (int k = 0; ok && k < x.nin; ++k) {
                if (!x.in_view[k]) continue;
                for (auto &o : outs) ok = ok && separate(x.in[k], o);
                for (auto &r : reds) ok = ok && !share(x.in[k], r);
            }
            for (auto &o : outs) ok = ok && separate(x.out, o);
            for (auto &y : inps) ok = ok && separate(x.out, y);
            for (auto &r : reds) ok = ok && !share(x.out, r);
            int nc = 0;
            for (int k = 0; k < x.nin; ++k) nc += x.in_view[k] ? 0 : 1;
            ok = ok && (int)kernels.back().members.size() < kMaxInstr && slot_count_with(x) <= kMaxSlots &&
                 nconst + nc <= kMaxConsts;
        }
        if (!ok) {
            kernels.push_back(KernelPlan());
            outs.clear();
            inps.clear();
            reds.clear();
            slots.clear();
            nconst = 0;
        }
        kernels.back().members.push_back((int)i);
        kid[i] = (int)kernels.size() - 1;
        for (int k = 0; k < x.nin; ++k) {
            if (x.in_view[k]) {
                inps.push_back(x.in[k]);
                bool have = false;
                for (auto &s : slots) have = have || same(s, x.in[k]);
                if (!have) slots.push_back(x.in[k]);
            } else {
                ++nconst;
            }
        }
        outs.push_back(x.out);
        if (is_reduce(x.op)) reds.push_back(x.out);
        bool have = false;
        for (auto &s : slots) have = have || same(s, x.out);
        if (!have) slots.push_back(x.out);
    }
}

// ---------------------------------------------------------------- code generation

const char *ctype(int dt) { return dt == VE_F32 ? "float" : "double"; }

std::string fn(int dt, const char *name) { return std::string(name) + (dt == VE_F32 ? "f" : ""); }

// The expression of instruction x on operands a[0..nin), result type T.
std::string expr(int op, int dt, const std::vector<std::string> &a, const std::vector<std::string> &user_exprs)
{
    const std::string T = ctype(dt);
    auto one = "((" + T + ")1)", zero = "((" + T + ")0)";
    switch (op) {
    case VE_COPY: return "(" + T + ")(" + a[0] + ")";
    case VE_NEGATIVE: return "(-" + a[0] + ")";
    case VE_ABSOLUTE: return fn(dt, "fabs") + "(" + a[0] + ")";
    case VE_SQRT: return fn(dt, "sqrt") + "(" + a[0] + ")";
    case VE_EXP: return fn(dt, "exp") + "(" + a[0] + ")";
    case VE_LOG: return fn(dt, "log") + "(" + a[0] + ")";
    case VE_SIN: return fn(dt, "sin") + "(" + a[0] + ")";
    case VE_COS: return fn(dt, "cos") + "(" + a[0] + ")";
    case VE_TANH: return fn(dt, "tanh") + "(" + a[0] + ")";
    case VE_ADD: return "(" + a[0] + " + " + a[1] + ")";
    case VE_SUBTRACT: return "(" + a[0] + " - " + a[1] + ")";
    case VE_MULTIPLY: return "(" + a[0] + " * " + a[1] + ")";
    case VE_DIVIDE: return "(" + a[0] + " / " + a[1] + ")";
    case VE_MAXIMUM: return "((" + a[0] + " >= " + a[1] + " || " + a[0] + " != " + a[0] + ") ? " + a[0] + " : " + a[1] + ")";
    case VE_MINIMUM: return "((" + a[0] + " <= " + a[1] + " || " + a[0] + " != " + a[0] + ") ? " + a[0] + " : " + a[1] + ")";
    case VE_POWER: return fn(dt, "pow") + "(" + a[0] + ", " + a[1] + ")";
    case VE_GREATER: return "((" + a[0] + " > " + a[1] + ") ? " + one + " : " + zero + ")";
    case VE_GREATER_EQUAL: return "((" + a[0] + " >= " + a[1] + ") ? " + one + " : " + zero + ")";
    case VE_LESS: return "((" + a[0] + " < " + a[1] + ") ? " + one + " : " + zero + ")";
    case VE_LESS_EQUAL: return "((" + a[0] + " <= " + a[1] + ") ? " + one + " : " + zero + ")";
    case VE_EQUAL: return "((" + a[0] + " == " + a[1] + ") ? " + one + " : " + zero + ")";
    case VE_NOT_EQUAL: return "((" + a[0] + " != " + a[1] + ") ? " + one + " : " + zero + ")";
    case VE_WHERE: return "((" + a[0] + " != " + zero + ") ? " + a[1] + " : " + a[2] + ")";
    }
    if (op >= VE_USER && op - VE_USER < (int)user_exprs.size()) {
        std::string s = "([&]() -> " + T + " { typedef " + T + " T;";
        for (size_t k = 0; k < a.size(); ++k) s += " const T x" + std::to_string(k) + " = " + a[k] + ";";
        return s + " return (T)(" + user_exprs[op - VE_USER] + "); }())";
    }
    return "0";
}

// Everything needed to generate and launch one kernel.
struct KernelCode {
    std::string src, name;
    std::vector<View> slots;
    std::vector<int> slot_dt;
    std::vector<bool> load, store;
    std::vector<double> consts;
    std::vector<int> red_slot, red_op, red_dt;
    int nd = 1;
    long long shape[VE_MAX_NDIM] = {1, 1, 1, 1};
    double bytes = 0;
    int ninstr = 0;
    bool staged = false;  // 2D tiles of kTR x kThreads with shifted-view groups in LDS
};

// element type and size of real and staging bases (sizes unknown: no bound)
struct DtypeOf {
    const std::vector<int> *real;
    std::map<int, int> temp;
    const std::vector<long long> *real_n = nullptr;
    std::map<int, long long> temp_n;
    int operator()(int b) const
    {
        if (b >= kTempBase) return temp.at(b);
        return (*real)[b];
    }
    long long nelem(int b) const
    {
        if (b >= kTempBase) return temp_n.count(b) ? temp_n.at(b) : LLONG_MAX;
        return real_n ? (*real_n)[b] : LLONG_MAX;
    }
};

// Elements covered by views of one base (for the algorithmic byte count):
// for views with equal strides whose offsets differ by whole index shifts
// (shifted windows, each offset difference split into the nearest multiple of
// the largest stride and so on down), the size of their common bounding box
// in index space; otherwise the sum of the sizes.  Both are capped by the
// extent the views span.
long long union_size(const std::vector<const View *> &vs)
{
    const View &r = *vs.front();
    long long sum = 0, lo = r.lo(), hi = r.hi();
    for (auto *v : vs) {
        sum += v->size();
        lo = std::min(lo, v->lo());
        hi = std::max(hi, v->hi());
    }
    const long long cap = std::min(sum, hi - lo + 1);
    if (vs.size() == 1) return r.size();
    std::vector<int> dims;
    for (int d = 0; d < r.nd; ++d)
        if (r.st[d] != 0) dims.push_back(d);
    std::sort(dims.begin(), dims.end(), [&](int x, int y) { return std::llabs(r.st[x]) > std::llabs(r.st[y]); });
    long long kmin[VE_MAX_NDIM] = {0, 0, 0, 0}, kmax[VE_MAX_NDIM] = {0, 0, 0, 0};
    for (int d = 0; d < r.nd; ++d) kmax[d] = r.shape[d];
    for (auto *v : vs) {
        if (v->nd != r.nd) return cap;
        for (int d = 0; d < r.nd; ++d)
            if (v->st[d] != r.st[d]) return cap;
        long long D = v->off - r.off;
        long long k[VE_MAX_NDIM] = {0, 0, 0, 0};
        for (size_t q = 0; q < dims.size(); ++q) {
            const int d = dims[q];
            const double x = (double)D / (double)r.st[d];
            k[d] = (long long)std::llround(x);
            D -= k[d] * r.st[d];
        }
        if (D != 0) return cap;
        for (int d = 0; d < r.nd; ++d) {
            kmin[d] = std::min(kmin[d], k[d]);
            kmax[d] = std::max(kmax[d], k[d] + v->shape[d]);
        }
    }
    long long box = 1;
    for (int d = 0; d < r.nd; ++d) box *= (r.st[d] == 0 ? 1 : kmax[d] - kmin[d]);
    return std::min(box, cap);
}

uint64_t fnv1a(const std::string &s)
{
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

void generate(const std::vector<Ins> &ins, const KernelPlan &kp, const std::vector<bool> &dead, const DtypeOf &dt,
              const std::vector<std::string> &user_exprs, KernelCode &kc)
{
    kc = KernelCode();
    const View &sp = ins[kp.members.front()].space();
    kc.nd = sp.nd;
    for (int d = 0; d < sp.nd; ++d) kc.shape[d] = sp.shape[d];
    kc.ninstr = (int)kp.members.size();
    auto slot_of = [&](const View &v) {
        for (size_t s = 0; s < kc.slots.size(); ++s)
            if (same(kc.slots[s], v)) return (int)s;
        kc.slots.push_back(v);
        kc.slot_dt.push_back(dt(v.base));
        kc.load.push_back(false);
        kc.store.push_back(false);
        return (int)kc.slots.size() - 1;
    };
    // first pass: operands, which slots are loaded (read before written), stored
    std::vector<bool> written;
    std::vector<int> last_writer;
    struct Op {
        int op, dt;
        std::vector<int> in_slot;   // -1: constant
        std::vector<int> in_const;  // index into consts
        int out_slot;
        bool red;
    };
    std::vector<Op> ops;
    for (int m : kp.members) {
        const Ins &x = ins[m];
        Op o;
        o.op = x.op;
        o.dt = dt(x.out.base);
        o.red = is_reduce(x.op);
        for (int k = 0; k < x.nin; ++k) {
            if (x.in_view[k]) {
                const int s = slot_of(x.in[k]);
                if ((int)written.size() < (int)kc.slots.size()) written.resize(kc.slots.size(), false);
                if (!written[s]) kc.load[s] = true;
                o.in_slot.push_back(s);
                o.in_const.push_back(-1);
            } else {
                o.in_slot.push_back(-1);
                o.in_const.push_back((int)kc.consts.size());
                kc.consts.push_back(x.cst[k]);
            }
        }
        o.out_slot = slot_of(x.out);
        if ((int)written.size() < (int)kc.slots.size()) written.resize(kc.slots.size(), false);
        if (!o.red) {
            written[o.out_slot] = true;
            kc.store[o.out_slot] = !dead[m];
        } else {
            kc.red_slot.push_back(o.out_slot);
            kc.red_op.push_back(x.op);
            kc.red_dt.push_back(o.dt);
        }
        ops.push_back(o);
    }
    const int NS = (int)kc.slots.size(), NC = std::max<int>(1, (int)kc.consts.size()), NR = (int)kc.red_slot.size();
    const int nd = kc.nd;
    // algorithmic bytes: the elements of each base that some load touches
    // (once, however many shifted views read them), plus every store
    std::map<int, std::vector<int>> loads_of;
    for (int s = 0; s < NS; ++s) {
        const double es = kc.slot_dt[s] == VE_F32 ? 4.0 : 8.0;
        bool red_out = false;
        for (int r : kc.red_slot) red_out = red_out || r == s;
        if (kc.load[s]) loads_of[kc.slots[s].base].push_back(s);
        if (kc.store[s] || red_out) kc.bytes += (red_out ? 1.0 : (double)kc.slots[s].size()) * es;
    }
    for (auto &g : loads_of) {
        const double es = kc.slot_dt[g.second.front()] == VE_F32 ? 4.0 : 8.0;
        std::vector<const View *> vs;
        for (int s : g.second) vs.push_back(&kc.slots[s]);
        kc.bytes += (double)union_size(vs) * es;
    }
    // ---- staging: groups of shifted views of one base read through LDS
    // (2D index spaces; views with the stride vector (row stride, 1) whose
    // offsets differ by small row / column shifts): the work-group loads the
    // group's bounding box of a TR x TC tile once, every view reads its
    // shifted window from LDS instead of memory
    struct Group {
        int ref;                    // reference slot (offsets are shifts from it)
        std::vector<int> slots;
        std::vector<long long> kr, kc;
        long long rmin = 0, rmax = 0, cmin = 0, cmax = 0;
    };
    std::vector<Group> groups;
    std::vector<int> group_of(NS, -1), member_of(NS, -1);
    if (nd == 2 && kc.shape[0] >= 2 && kc.shape[1] >= 2) {
        std::map<int, std::vector<int>> by_base;
        for (int s = 0; s < NS; ++s)
            if (kc.load[s] && kc.slots[s].st[1] == 1 && kc.slots[s].st[0] > 8) by_base[kc.slots[s].base].push_back(s);
        size_t lds = 0;
        for (auto &bb : by_base) {
            if (bb.second.size() < 2) continue;
            Group g;
            g.ref = bb.second.front();
            const View &r = kc.slots[g.ref];
            bool ok = true;
            for (int s : bb.second) {
                const View &v = kc.slots[s];
                if (v.st[0] != r.st[0]) {
                    ok = false;
                    break;
                }
                const long long D = v.off - r.off;
                const long long q = (long long)std::llround((double)D / (double)r.st[0]);
                const long long c = D - q * r.st[0];
                if (std::llabs(q) > 4 || std::llabs(c) > 4) {
                    ok = false;
                    break;
                }
                g.slots.push_back(s);
                g.kr.push_back(q);
                g.kc.push_back(c);
                g.rmin = std::min(g.rmin, q);
                g.rmax = std::max(g.rmax, q);
                g.cmin = std::min(g.cmin, c);
                g.cmax = std::max(g.cmax, c);
            }
            if (!ok) continue;
            // the whole box (every tile's box, edges included) must lie in the base
            const long long R = kc.shape[0], Cn = kc.shape[1];
            long long lo = LLONG_MAX, hi = LLONG_MIN;
            for (long long rr : {g.rmin, R - 1 + g.rmax})
                for (long long cc : {g.cmin, Cn - 1 + g.cmax}) {
                    const long long o = r.off + rr * r.st[0] + cc;
                    lo = std::min(lo, o);
                    hi = std::max(hi, o);
                }
            if (lo < 0 || hi >= dt.nelem(r.base)) continue;
            const size_t bytes = (size_t)(kTR + g.rmax - g.rmin) * (kThreads + g.cmax - g.cmin) *
                                 (kc.slot_dt[g.ref] == VE_F32 ? 4 : 8);
            if (lds + bytes > 64 * 1024) continue;
            lds += bytes;
            for (size_t i = 0; i < g.slots.size(); ++i) {
                group_of[g.slots[i]] = (int)groups.size();
                member_of[g.slots[i]] = (int)i;
            }
            groups.push_back(g);
        }
    }
    kc.staged = !groups.empty();
    // ---- source
    std::string b;
    char tmp[4096];
    b += "struct A_@ { long long shape[4]; long long tpr, ntiles, nper; const void *p[" + std::to_string(NS) +
         "]; long long off[" + std::to_string(NS) + "]; long long st[" + std::to_string(NS) + "][4]; double c[" +
         std::to_string(NC) + "]; double *part; };\n";
    b += "extern \"C\" __global__ __launch_bounds__(256) void @(A_@ a) {\n";
    b += "  const int tid = threadIdx.x;\n";
    b += "  const long long blk = blockIdx.x, pos = (blk & 7) * a.nper + (blk >> 3), nb = 8 * a.nper;\n";
    b += "  const long long t0 = pos * a.ntiles / nb, t1 = (pos + 1) * a.ntiles / nb;\n";
    for (int r = 0; r < NR; ++r) {
        const std::string T = ctype(kc.red_dt[r]);
        snprintf(tmp, sizeof tmp, "  %s acc%d = %s;\n", T.c_str(), r,
                 kc.red_op[r] == VE_ADD_REDUCE ? ("(" + T + ")0").c_str() : ("-(" + T + ")INFINITY").c_str());
        b += tmp;
    }
    // the row's first element of every operand, as a typed pointer (64-bit
    // arithmetic once per row); along the row a 32-bit index when the row
    // and every operand's span of it stay below 2^31 elements, and plain
    // indexing for unit-stride operands
    bool idx32 = kc.shape[nd - 1] < (1LL << 31) - kTile;
    for (int s = 0; s < NS; ++s)
        idx32 = idx32 && std::llabs(kc.slots[s].st[nd - 1]) * kc.shape[nd - 1] < (1LL << 31) - kTile;
    const char *IT = idx32 ? "int" : "long long";
    std::vector<std::string> at(NS), rowptr(NS);
    for (int s = 0; s < NS; ++s) {
        bool red_out = false;
        for (int r : kc.red_slot) red_out = red_out || r == s;
        const char *T = ctype(kc.slot_dt[s]);
        const bool wr = kc.store[s] || red_out;
        snprintf(tmp, sizeof tmp, "%s%s *q%d = (%s%s *)a.p[%d] + (", wr ? "" : "const ", T, s, wr ? "" : "const ", T, s);
        rowptr[s] = tmp;
        if (kc.slots[s].st[nd - 1] == 1) {
            at[s] = "q" + std::to_string(s) + "[c]";
        } else {
            snprintf(tmp, sizeof tmp, "q%d[c * (%s)a.st[%d][%d]]", s, IT, s, nd - 1);
            at[s] = tmp;
        }
    }
    // the instructions of one element, given each loaded slot's value
    auto body = [&](const std::vector<std::string> &ld, const std::string &ind) {
        std::string o;
        std::vector<std::string> cur = ld;
        int red_i = 0;
        for (size_t i = 0; i < ops.size(); ++i) {
            const Op &op = ops[i];
            std::vector<std::string> av;
            for (size_t k = 0; k < op.in_slot.size(); ++k) {
                if (op.in_slot[k] >= 0) av.push_back(cur[op.in_slot[k]]);
                else av.push_back("((" + std::string(ctype(op.dt)) + ")a.c[" + std::to_string(op.in_const[k]) + "])");
            }
            if (op.red) {
                if (op.op == VE_ADD_REDUCE) {
                    snprintf(tmp, sizeof tmp, "%sacc%d = acc%d + %s;\n", ind.c_str(), red_i, red_i, av[0].c_str());
                } else {
                    snprintf(tmp, sizeof tmp, "%sacc%d = (acc%d >= %s || acc%d != acc%d) ? acc%d : %s;\n", ind.c_str(),
                             red_i, red_i, av[0].c_str(), red_i, red_i, red_i, av[0].c_str());
                }
                o += tmp;
                ++red_i;
                continue;
            }
            snprintf(tmp, sizeof tmp, "%sconst %s r%zu = ", ind.c_str(), ctype(op.dt), i);
            o += tmp + expr(op.op, op.dt, av, user_exprs) + ";\n";
            cur[op.out_slot] = "r" + std::to_string(i);
        }
        for (int s = 0; s < NS; ++s)
            if (kc.store[s]) o += ind + at[s] + " = " + cur[s] + ";\n";
        return o;
    };
    if (!kc.staged) {
        // tiles: one row segment of kTile elements, kPerThread per thread
        b += "  for (long long t = t0; t < t1; ++t) {\n";
        b += "    const long long row = t / a.tpr, ct = t - row * a.tpr;\n";
        if (nd > 1) {
            b += "    long long rr = row;\n";
            for (int d = nd - 2; d >= 0; --d) {
                snprintf(tmp, sizeof tmp, "    const long long i%d = rr %% a.shape[%d]; rr /= a.shape[%d];\n", d, d, d);
                b += tmp;
            }
        }
        for (int s = 0; s < NS; ++s) {
            std::string e = "a.off[" + std::to_string(s) + "]";
            for (int d = 0; d < nd - 1; ++d)
                e += " + i" + std::to_string(d) + " * a.st[" + std::to_string(s) + "][" + std::to_string(d) + "]";
            b += "    " + rowptr[s] + e + ");\n";
        }
        b += std::string("    const ") + IT + " c0 = (" + IT + ")(ct * " + std::to_string(kTile) + ") + tid;\n";
        // loads of every element first (no store of this kernel can alias them)
        for (int s = 0; s < NS; ++s)
            if (kc.load[s]) {
                snprintf(tmp, sizeof tmp, "    %s l%d[%d];\n", ctype(kc.slot_dt[s]), s, kPerThread);
                b += tmp;
            }
        b += "#pragma unroll\n    for (int v = 0; v < " + std::to_string(kPerThread) + "; ++v) {\n";
        b += std::string("      const ") + IT + " c = c0 + v * " + std::to_string(kThreads) + ";\n";
        b += "      const bool ok = c < a.shape[" + std::to_string(nd - 1) + "];\n";
        for (int s = 0; s < NS; ++s)
            if (kc.load[s]) {
                snprintf(tmp, sizeof tmp, "      l%d[v] = ok ? %s : (%s)0;\n", s, at[s].c_str(), ctype(kc.slot_dt[s]));
                b += tmp;
            }
        b += "    }\n";
        b += "#pragma unroll\n    for (int v = 0; v < " + std::to_string(kPerThread) + "; ++v) {\n";
        b += std::string("      const ") + IT + " c = c0 + v * " + std::to_string(kThreads) + ";\n";
        b += "      if (c < a.shape[" + std::to_string(nd - 1) + "]) {\n";
        std::vector<std::string> ld(NS);
        for (int s = 0; s < NS; ++s)
            if (kc.load[s]) ld[s] = "l" + std::to_string(s) + "[v]";
        b += body(ld, "        ");
        b += "      }\n    }\n  }\n";
    } else {
        // tiles: kTR rows x kThreads columns; one column per thread
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const Group &g = groups[gi];
            const long long BH = kTR + g.rmax - g.rmin, BW = kThreads + g.cmax - g.cmin;
            snprintf(tmp, sizeof tmp, "  __shared__ %s sg%zu[%lld];\n", ctype(kc.slot_dt[g.ref]), gi, BH * BW);
            b += tmp;
        }
        b += "  for (long long t = t0; t < t1; ++t) {\n";
        b += "    const long long tr0 = (t / a.tpr) * " + std::to_string(kTR) + ";\n";
        b += std::string("    const ") + IT + " c0 = (" + IT + ")((t % a.tpr) * " + std::to_string(kThreads) + ");\n";
        b += "    __syncthreads();\n";
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const Group &g = groups[gi];
            const long long BH = kTR + g.rmax - g.rmin, BW = kThreads + g.cmax - g.cmin;
            // box element (i, j) is reference element (r0 + rmin + i, c0 + cmin + j);
            // only the part over the union of the views' index ranges is read
            // (every load of the box issued before the first LDS store)
            const long long NQ = (BH * BW + kThreads - 1) / kThreads;
            snprintf(tmp, sizeof tmp,
                     "    { const %s *qb = (const %s *)a.p[%d] + a.off[%d] + (tr0 + %lld) * a.st[%d][0] + ((long long)c0 + %lld);\n"
                     "      const long long rlast = a.shape[0] - 1 + %lld - (tr0 + %lld), clast = a.shape[1] - 1 + %lld - ((long long)c0 + %lld);\n"
                     "      const long long rs = a.st[%d][0];\n"
                     "      %s v[%lld];\n"
                     "#pragma unroll\n"
                     "      for (int k = 0; k < %lld; ++k) {\n"
                     "        const int q = tid + 256 * k, i = q / %lld, j = q - i * %lld;\n"
                     "        v[k] = (q < %lld && i <= rlast && j <= clast) ? qb[i * rs + j] : (%s)0;\n"
                     "      }\n"
                     "#pragma unroll\n"
                     "      for (int k = 0; k < %lld; ++k) {\n"
                     "        const int q = tid + 256 * k;\n"
                     "        if (q < %lld) sg%zu[q] = v[k];\n"
                     "      } }\n",
                     ctype(kc.slot_dt[g.ref]), ctype(kc.slot_dt[g.ref]), g.ref, g.ref, g.rmin, g.ref, g.cmin, g.rmax,
                     g.rmin, g.cmax, g.cmin, g.ref, ctype(kc.slot_dt[g.ref]), NQ, NQ, BW, BW, BH * BW,
                     ctype(kc.slot_dt[g.ref]), NQ, BH * BW, gi);
            b += tmp;
        }
        b += "    __syncthreads();\n";
        b += std::string("    const ") + IT + " c = c0 + tid;\n";
        b += "    if (c < a.shape[1]) {\n";
        b += "      for (int i = 0; i < " + std::to_string(kTR) + "; ++i) {\n";
        b += "        const long long row = tr0 + i;\n";
        b += "        if (row >= a.shape[0]) break;\n";
        for (int s = 0; s < NS; ++s) {
            if (!kc.store[s] && (group_of[s] >= 0 || !kc.load[s])) continue;  // LDS only, or unused
            b += "        " + rowptr[s] + "a.off[" + std::to_string(s) + "] + row * a.st[" + std::to_string(s) + "][0]);\n";
        }
        std::vector<std::string> ld(NS);
        for (int s = 0; s < NS; ++s) {
            if (!kc.load[s]) continue;
            if (group_of[s] >= 0) {
                const Group &g = groups[group_of[s]];
                const int m = member_of[s];
                const long long BW = kThreads + g.cmax - g.cmin;
                snprintf(tmp, sizeof tmp, "        const %s l%d = sg%d[(i + %lld) * %lld + tid + %lld];\n",
                         ctype(kc.slot_dt[s]), s, group_of[s], g.kr[m] - g.rmin, BW, g.kc[m] - g.cmin);
            } else {
                snprintf(tmp, sizeof tmp, "        const %s l%d = %s;\n", ctype(kc.slot_dt[s]), s, at[s].c_str());
            }
            b += tmp;
            ld[s] = "l" + std::to_string(s);
        }
        b += body(ld, "        ");
        b += "      }\n    }\n  }\n";
    }
    if (NR > 0) {
        // per-work-group partial results, reduced in a fixed order
        b += "  __shared__ double red[" + std::to_string(NR) + "][4];\n";
        for (int r = 0; r < NR; ++r) {
            const bool mx = kc.red_op[r] == VE_MAXIMUM_REDUCE;
            b += "  {\n    double v = (double)acc" + std::to_string(r) + ";\n";
            b += "    for (int o = 32; o > 0; o >>= 1) { const double w = __shfl_down(v, o, 64); ";
            b += mx ? "v = (v >= w || v != v) ? v : w; }\n" : "v = v + w; }\n";
            b += "    if ((tid & 63) == 0) red[" + std::to_string(r) + "][tid >> 6] = v;\n  }\n";
        }
        b += "  __syncthreads();\n  if (tid == 0) {\n";
        for (int r = 0; r < NR; ++r) {
            const bool mx = kc.red_op[r] == VE_MAXIMUM_REDUCE;
            snprintf(tmp, sizeof tmp, "    double s%d = red[%d][0];\n", r, r);
            b += tmp;
            for (int w = 1; w < 4; ++w) {
                if (mx)
                    snprintf(tmp, sizeof tmp, "    s%d = (s%d >= red[%d][%d] || s%d != s%d) ? s%d : red[%d][%d];\n", r, r, r,
                             w, r, r, r, r, w);
                else
                    snprintf(tmp, sizeof tmp, "    s%d = s%d + red[%d][%d];\n", r, r, r, w);
                b += tmp;
            }
            snprintf(tmp, sizeof tmp, "    a.part[blk * %d + %d] = s%d;\n", NR, r, r);
            b += tmp;
        }
        b += "  }\n}\n";
        // finishing kernel: one work-group sums the partial results in order
        b += "extern \"C\" __global__ __launch_bounds__(256) void @_fin(A_@ a, long long nblk) {\n";
        b += "  const int tid = threadIdx.x;\n  __shared__ double red[" + std::to_string(NR) + "][4];\n";
        for (int r = 0; r < NR; ++r) {
            const bool mx = kc.red_op[r] == VE_MAXIMUM_REDUCE;
            const std::string comb = mx ? "v = (v >= w || v != v) ? v : w;" : "v = v + w;";
            b += "  {\n    double v = " + std::string(mx ? "-INFINITY" : "0.0") + ";\n";
            b += "    for (long long q = tid; q < nblk; q += 256) { const double w = a.part[q * " + std::to_string(NR) +
                 " + " + std::to_string(r) + "]; " + comb + " }\n";
            b += "    for (int o = 32; o > 0; o >>= 1) { const double w = __shfl_down(v, o, 64); " + comb + " }\n";
            b += "    if ((tid & 63) == 0) red[" + std::to_string(r) + "][tid >> 6] = v;\n  }\n";
        }
        b += "  __syncthreads();\n  if (tid == 0) {\n";
        for (int r = 0; r < NR; ++r) {
            const bool mx = kc.red_op[r] == VE_MAXIMUM_REDUCE;
            snprintf(tmp, sizeof tmp, "    double v = red[%d][0];\n    for (int w = 1; w < 4; ++w) { const double x = red[%d][w]; %s }\n",
                     r, r, mx ? "v = (v >= x || v != v) ? v : x;" : "v = v + x;");
            b += "    {\n" + std::string(tmp);
            const int s = kc.red_slot[r];
            snprintf(tmp, sizeof tmp, "    ((%s *)a.p[%d])[a.off[%d]] = (%s)v;\n    }\n", ctype(kc.red_dt[r]), s, s,
                     ctype(kc.red_dt[r]));
            b += tmp;
        }
        b += "  }\n}\n";
    } else {
        b += "}\n";
    }
    // name from the structure (the source with a placeholder name)
    char nm[40];
    snprintf(nm, sizeof nm, "vek_%016llx", (unsigned long long)fnv1a(b));
    kc.name = nm;
    std::string out;
    out.reserve(b.size() + 64);
    for (char ch : b) {
        if (ch == '@') out += kc.name;
        else out += ch;
    }
    kc.src = out;
}

// Everything generate() reads for kernel kp, serialized: the members'
// instructions (opcode, views, constants, dead flag), the type and size of
// every base they name, and the expressions of user operations.  Equal keys
// give equal generated kernels, so a batch that repeats an earlier kernel
// reuses its code without building the source again.
std::string kernel_key(const std::vector<Ins> &ins, const KernelPlan &kp, const std::vector<bool> &dead,
                       const DtypeOf &dt, const std::vector<std::string> &user_exprs)
{
    std::string k;
    k.reserve(kp.members.size() * 256);
    auto put = [&](const void *p, size_t n) { k.append((const char *)p, n); };
    auto put_view = [&](const View &v) {
        put(&v.base, sizeof v.base);
        put(&v.nd, sizeof v.nd);
        put(&v.off, sizeof v.off);
        put(v.shape, sizeof v.shape);
        put(v.st, sizeof v.st);
    };
    std::vector<int> bases;
    for (int m : kp.members) {
        const Ins &x = ins[m];
        const char d = dead[m] ? 1 : 0;
        put(&x.op, sizeof x.op);
        put(&x.nin, sizeof x.nin);
        put(&d, 1);
        put_view(x.out);
        bases.push_back(x.out.base);
        for (int q = 0; q < x.nin; ++q) {
            const char iv = x.in_view[q] ? 1 : 0;
            put(&iv, 1);
            if (x.in_view[q]) {
                put_view(x.in[q]);
                bases.push_back(x.in[q].base);
            } else {
                put(&x.cst[q], sizeof x.cst[q]);
            }
        }
        if (x.op >= VE_USER && x.op - VE_USER < (int)user_exprs.size()) k += user_exprs[x.op - VE_USER] + '\0';
    }
    std::sort(bases.begin(), bases.end());
    bases.erase(std::unique(bases.begin(), bases.end()), bases.end());
    for (int b : bases) {
        const int t = dt(b);
        const long long ne = dt.nelem(b);
        put(&b, sizeof b);
        put(&t, sizeof t);
        put(&ne, sizeof ne);
    }
    return k;
}

// Dead outputs: after instruction m, the next reference to m's output base
// outside m's own kernel (whose reads of the same view take the register) is
// a free or a discard (no read, sync or write first).
void dead_outputs(const std::vector<Ins> &ins, const std::vector<int> &kid, std::vector<bool> &dead)
{
    dead.assign(ins.size(), false);
    for (size_t m = 0; m < ins.size(); ++m) {
        if (kid[m] < 0 || is_reduce(ins[m].op)) continue;
        const int b = ins[m].out.base;
        if (b >= kTempBase) continue;
        bool d = false;
        for (size_t j = m + 1; j < ins.size(); ++j) {
            if (kid[j] == kid[m]) continue;
            const Ins &y = ins[j];
            if (is_system(y.op)) {
                if (y.out.base != b) continue;
                d = (y.op == VE_FREE || y.op == VE_DISCARD);
                break;
            }
            bool ref = y.out.base == b;
            for (int k = 0; k < y.nin; ++k) ref = ref || (y.in_view[k] && y.in[k].base == b);
            if (ref) break;
        }
        dead[m] = d;
    }
}

}  // namespace

// ---------------------------------------------------------------- engine

struct ve_engine_s {
    hipStream_t stream = nullptr;
    hipMemPool_t pool = nullptr;  // engine-owned bases and partial sums
    std::string err, arch;
    struct Base {
        int dtype;
        long long nelem;
        void *ptr;
        bool owned, freed;
    };
    std::vector<Base> bases;
    std::vector<std::string> user_exprs;
    std::vector<int> user_nin;
    struct Compiled {
        hipFunction_t fn = nullptr, fin = nullptr;
        int id = 0, ninstr = 0;
    };
    std::unordered_map<std::string, Compiled> cache;  // by kernel name (hash of the source)
    std::unordered_map<std::string, KernelCode> generated;  // by kernel_key (bounded)
    std::vector<hipModule_t> modules;
    double *partials = nullptr;
    size_t partials_cap = 0;
    ve_stats st{};
    bool prof = false;
    // a run of consecutive launches of one kernel between one pair of events
    // (events around every launch would add their own cost to short kernels)
    struct PRec {
        int id;
        hipEvent_t a, b;
        double bytes;
        int count;
    };
    std::vector<PRec> pend;
    bool run_open = false;
    struct PK {
        std::string name;
        int launches = 0;
        double total_ms = 0, bytes = 0;
    };
    std::map<int, PK> pk;
    std::vector<int> pk_order;
};

namespace {

#define VECHK(e, call)                                                   \
    do {                                                                 \
        hipError_t x_ = (call);                                          \
        if (x_ != hipSuccess) {                                          \
            (e)->err = std::string(#call) + ": " + hipGetErrorString(x_); \
            return VE_ERR_HIP;                                           \
        }                                                                \
    } while (0)

ve_status ensure_alloc(ve_engine e, int id)
{
    auto &B = e->bases[id];
    if (B.ptr) return VE_OK;
    const size_t bytes = (size_t)std::max<long long>(B.nelem, 1) * (B.dtype == VE_F32 ? 4 : 8);
    VECHK(e, hipMallocFromPoolAsync(&B.ptr, bytes, e->pool, e->stream));
    B.owned = true;
    return VE_OK;
}

ve_status compile_all(ve_engine e, std::vector<KernelCode *> &todo)
{
    if (todo.empty()) return VE_OK;
    std::string src = "#define INFINITY __builtin_huge_val()\n";
    for (auto *k : todo) src += k->src;
    const auto t0 = std::chrono::steady_clock::now();
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "ve_kernels.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        e->err = "hiprtcCreateProgram failed";
        return VE_ERR_COMPILE;
    }
    const std::string archopt = "--offload-arch=" + e->arch;
    const char *opts[] = {archopt.c_str(), "-O3", "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, 8, opts);
    if (r != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        e->err = "hipRTC compilation failed:\n" + log.substr(0, 4000);
        return VE_ERR_COMPILE;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    std::vector<char> code(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    hipModule_t mod;
    VECHK(e, hipModuleLoadData(&mod, code.data()));
    e->modules.push_back(mod);
    for (auto *k : todo) {
        ve_engine_s::Compiled c;
        VECHK(e, hipModuleGetFunction(&c.fn, mod, k->name.c_str()));
        if (!k->red_slot.empty()) VECHK(e, hipModuleGetFunction(&c.fin, mod, (k->name + "_fin").c_str()));
        c.id = (int)e->cache.size();
        c.ninstr = k->ninstr;
        e->cache[k->name] = c;
        ++e->st.compiled;
    }
    e->st.compile_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return VE_OK;
}

// End the open run of launches (its closing event after its last launch).
hipError_t close_run(ve_engine e)
{
    if (!e->run_open) return hipSuccess;
    e->run_open = false;
    return hipEventRecord(e->pend.back().b, e->stream);
}

void put8(std::vector<char> &buf, const void *p)
{
    const char *c = (const char *)p;
    buf.insert(buf.end(), c, c + 8);
}

ve_status launch(ve_engine e, const KernelCode &kc, const std::vector<void *> &ptrs)
{
    const ve_engine_s::Compiled &c = e->cache.at(kc.name);
    const int NS = (int)kc.slots.size(), NC = std::max<int>(1, (int)kc.consts.size()), NR = (int)kc.red_slot.size();
    long long shape[4] = {1, 1, 1, 1};
    for (int d = 0; d < kc.nd; ++d) shape[d] = kc.shape[d];
    long long rows = 1;
    for (int d = 0; d < kc.nd - 1; ++d) rows *= shape[d];
    const long long cols = shape[kc.nd - 1];
    // row segments of kTile elements, or (staged kernels) tiles of kTR rows
    // x kThreads columns
    const long long tpr = kc.staged ? (cols + kThreads - 1) / kThreads : (cols + kTile - 1) / kTile;
    const long long ntiles = kc.staged ? (rows + kTR - 1) / kTR * tpr : rows * tpr;
    long long nblk = std::min<long long>(std::max<long long>(ntiles, 1), kMaxBlocks);
    const long long nper = (nblk + 7) / 8;
    nblk = 8 * nper;
    if (NR > 0) {
        const size_t need = (size_t)nblk * NR;
        if (need > e->partials_cap) {
            if (e->partials) VECHK(e, hipFreeAsync(e->partials, e->stream));
            VECHK(e, hipMallocFromPoolAsync((void **)&e->partials, need * sizeof(double), e->pool, e->stream));
            e->partials_cap = need;
        }
    }
    std::vector<char> buf;
    for (int d = 0; d < 4; ++d) put8(buf, &shape[d]);
    put8(buf, &tpr);
    put8(buf, &ntiles);
    put8(buf, &nper);
    for (int s = 0; s < NS; ++s) put8(buf, &ptrs[s]);
    for (int s = 0; s < NS; ++s) put8(buf, &kc.slots[s].off);
    for (int s = 0; s < NS; ++s)
        for (int d = 0; d < 4; ++d) {
            const long long v = d < kc.slots[s].nd ? kc.slots[s].st[d] : 0;
            put8(buf, &v);
        }
    for (int q = 0; q < NC; ++q) {
        const double v = q < (int)kc.consts.size() ? kc.consts[q] : 0.0;
        put8(buf, &v);
    }
    put8(buf, &e->partials);
    size_t sz = buf.size();
    void *cfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, buf.data(), HIP_LAUNCH_PARAM_BUFFER_SIZE, &sz, HIP_LAUNCH_PARAM_END};
    hipEvent_t ea = nullptr, eb = nullptr;  // a new run's events
    if (e->prof) {
        if (e->run_open && e->pend.back().id == c.id) {
            e->pend.back().count += 1;
            e->pend.back().bytes += kc.bytes;
        } else {
            VECHK(e, close_run(e));
            VECHK(e, hipEventCreate(&ea));
            VECHK(e, hipEventCreate(&eb));
            VECHK(e, hipEventRecord(ea, e->stream));
            e->pend.push_back({c.id, ea, eb, kc.bytes, 1});
            e->run_open = true;
        }
    }
    VECHK(e, hipModuleLaunchKernel(c.fn, (unsigned)nblk, 1, 1, kThreads, 1, 1, 0, e->stream, nullptr, cfg));
    if (NR > 0) {
        std::vector<char> b2 = buf;
        put8(b2, &nblk);
        size_t sz2 = b2.size();
        void *cfg2[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, b2.data(), HIP_LAUNCH_PARAM_BUFFER_SIZE, &sz2,
                        HIP_LAUNCH_PARAM_END};
        VECHK(e, hipModuleLaunchKernel(c.fin, 1, 1, 1, kThreads, 1, 1, 0, e->stream, nullptr, cfg2));
    }
    if (e->prof) {
        if (!e->pk.count(c.id)) {
            e->pk[c.id].name = "k" + std::to_string(c.id) + ":" + std::to_string(c.ninstr);
            e->pk_order.push_back(c.id);
        }
    }
    ++e->st.kernels;
    return VE_OK;
}

ve_status validate_bases(ve_engine e, const std::vector<Ins> &ins)
{
    auto check = [&](const View &v, bool out, int i) -> ve_status {
        if (v.base >= kTempBase) return VE_OK;
        if (v.base < 0 || v.base >= (int)e->bases.size() || e->bases[v.base].freed) {
            e->err = "instruction " + std::to_string(i) + ": unknown or freed array-base " + std::to_string(v.base);
            return VE_ERR_ARG;
        }
        if (v.size() == 0) return VE_OK;
        if (v.lo() < 0 || v.hi() >= e->bases[v.base].nelem) {
            e->err = "instruction " + std::to_string(i) + ": view outside its array-base";
            return VE_ERR_ARG;
        }
        if (out) {
            for (int d = 0; d < v.nd; ++d)
                if (v.st[d] == 0 && v.shape[d] > 1) {
                    e->err = "instruction " + std::to_string(i) + ": an output view repeats elements (stride 0)";
                    return VE_ERR_UNSUPPORTED;
                }
            // every element once: axes sorted by |stride| must nest
            std::vector<std::pair<long long, long long>> ax;
            for (int d = 0; d < v.nd; ++d)
                if (v.shape[d] > 1) ax.push_back({std::llabs(v.st[d]), v.shape[d]});
            std::sort(ax.begin(), ax.end());
            long long reach = 0;
            for (auto &p : ax) {
                if (p.first <= reach) {
                    e->err = "instruction " + std::to_string(i) + ": an output view addresses some element twice";
                    return VE_ERR_UNSUPPORTED;
                }
                reach += p.first * (p.second - 1);
            }
        }
        return VE_OK;
    };
    for (size_t j = 0; j < ins.size(); ++j) {
        const Ins &x = ins[j];
        const int i = x.orig;
        if (is_system(x.op)) {
            if (x.out.base < 0 || x.out.base >= (int)e->bases.size() || e->bases[x.out.base].freed) {
                e->err = "instruction " + std::to_string(i) + ": unknown or freed array-base";
                return VE_ERR_ARG;
            }
            continue;
        }
        ve_status r = check(x.out, true, i);
        if (r != VE_OK) return r;
        for (int k = 0; k < x.nin; ++k)
            if (x.in_view[k] && (r = check(x.in[k], false, i)) != VE_OK) return r;
        const int odt = x.out.base >= kTempBase ? -1 : e->bases[x.out.base].dtype;
        if (x.op != VE_COPY && odt >= 0)
            for (int k = 0; k < x.nin; ++k)
                if (x.in_view[k] && x.in[k].base < kTempBase && e->bases[x.in[k].base].dtype != odt) {
                    e->err = "instruction " + std::to_string(i) + ": operands of different element types (convert with a copy)";
                    return VE_ERR_ARG;
                }
    }
    // a free ends a base's life in the batch
    std::vector<bool> gone(e->bases.size(), false);
    for (const Ins &x : ins) {
        auto used = [&](const View &v) { return v.base >= 0 && v.base < kTempBase && gone[v.base]; };
        bool bad = used(x.out);
        for (int k = 0; k < x.nin; ++k) bad = bad || (x.in_view[k] && used(x.in[k]));
        if (bad) {
            e->err = "instruction " + std::to_string(x.orig) + ": uses an array-base freed earlier in the batch";
            return VE_ERR_ARG;
        }
        if (x.op == VE_FREE) gone[x.out.base] = true;
    }
    return VE_OK;
}

}  // namespace

// ---------------------------------------------------------------- C-ABI

extern "C" ve_status ve_create(void *stream, ve_engine *out)
{
    if (!out) return VE_ERR_ARG;
    *out = nullptr;
    ve_engine e = new (std::nothrow) ve_engine_s();
    if (!e) return VE_ERR_ARG;
    e->stream = (hipStream_t)stream;
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
        delete e;
        return VE_ERR_HIP;
    }
    e->arch = p.gcnArchName;
    const size_t colon = e->arch.find(':');
    if (colon != std::string::npos) e->arch = e->arch.substr(0, colon);
    // The engine's own stream-ordered pool, which keeps freed memory: a
    // program that loops allocates and frees the same temporaries every
    // iteration, and giving them back to the driver between iterations
    // would map fresh memory each time.
    hipMemPoolProps pp;
    std::memset(&pp, 0, sizeof(pp));
    pp.allocType = hipMemAllocationTypePinned;
    pp.handleTypes = hipMemHandleTypeNone;
    pp.location.type = hipMemLocationTypeDevice;
    pp.location.id = dev;
    uint64_t keep = UINT64_MAX;
    if (hipMemPoolCreate(&e->pool, &pp) != hipSuccess ||
        hipMemPoolSetAttribute(e->pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
        if (e->pool) (void)hipMemPoolDestroy(e->pool);
        delete e;
        return VE_ERR_HIP;
    }
    *out = e;
    return VE_OK;
}

extern "C" ve_status ve_destroy(ve_engine e)
{
    if (!e) return VE_ERR_ARG;
    (void)hipStreamSynchronize(e->stream);
    for (auto &B : e->bases)
        if (B.owned && B.ptr && !B.freed) (void)hipFreeAsync(B.ptr, e->stream);
    if (e->partials) (void)hipFreeAsync(e->partials, e->stream);
    (void)hipStreamSynchronize(e->stream);
    if (e->pool) (void)hipMemPoolDestroy(e->pool);
    for (auto &r : e->pend) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto m : e->modules) (void)hipModuleUnload(m);
    delete e;
    return VE_OK;
}

extern "C" ve_status ve_base_new(ve_engine e, int dtype, long long nelem, void *device_ptr, int *id)
{
    if (!e || !id || nelem < 0 || (dtype != VE_F64 && dtype != VE_F32)) return VE_ERR_ARG;
    if (nelem >= (1LL << 40)) return VE_ERR_ARG;
    ve_engine_s::Base B{dtype, nelem, device_ptr, false, false};
    e->bases.push_back(B);
    *id = (int)e->bases.size() - 1;
    return VE_OK;
}

extern "C" ve_status ve_base_ptr(ve_engine e, int id, void **ptr)
{
    if (!e || !ptr || id < 0 || id >= (int)e->bases.size() || e->bases[id].freed) return VE_ERR_ARG;
    ve_status r = ensure_alloc(e, id);
    if (r != VE_OK) return r;
    *ptr = e->bases[id].ptr;
    return VE_OK;
}

extern "C" ve_status ve_register(ve_engine e, const char *expr_src, int nin, int *opcode)
{
    if (!e || !expr_src || !opcode || nin < 1 || nin > VE_MAX_IN) return VE_ERR_ARG;
    e->user_exprs.push_back(expr_src);
    e->user_nin.push_back(nin);
    *opcode = VE_USER + (int)e->user_exprs.size() - 1;
    return VE_OK;
}

extern "C" ve_status ve_plan(const ve_instr *batch, int n, int *kernel_of, int *nkernels)
{
    if ((!batch && n > 0) || n < 0 || !kernel_of || !nkernels) return VE_ERR_ARG;
    std::vector<Ins> ins;
    std::string err;
    auto arity = [](int op) {
        if (op >= VE_USER) return VE_MAX_IN;  // every view operand of a user operation
        return builtin_arity(op);
    };
    ve_status r = to_internal(batch, n, arity, ins, err);
    if (r != VE_OK) return r;
    std::vector<int> kid;
    std::vector<KernelPlan> ks;
    form(ins, kid, ks);
    for (int i = 0; i < n; ++i) kernel_of[i] = -1;
    for (size_t j = 0; j < ins.size(); ++j)
        if (ins[j].orig >= 0) kernel_of[ins[j].orig] = kid[j];
    *nkernels = (int)ks.size();
    return VE_OK;
}

extern "C" ve_status ve_kernel_source(const ve_instr *batch, int n, const int *base_dtype, int nbases, int k, char *buf,
                                      size_t len, size_t *need)
{
    if ((!batch && n > 0) || n < 0 || !base_dtype || nbases < 0 || !need) return VE_ERR_ARG;
    std::vector<Ins> ins;
    std::string err;
    ve_status r = to_internal(batch, n, [](int op) { return builtin_arity(op); }, ins, err);
    if (r != VE_OK) return r;
    std::vector<int> kid;
    std::vector<KernelPlan> ks;
    form(ins, kid, ks);
    if (k < 0 || k >= (int)ks.size()) return VE_ERR_ARG;
    std::vector<int> real(base_dtype, base_dtype + nbases);
    DtypeOf dt{&real, {}};
    for (auto &x : ins) {
        auto ok = [&](const View &v) { return v.base >= kTempBase || (v.base >= 0 && v.base < nbases); };
        if (!ok(x.out)) return VE_ERR_ARG;
        for (int q = 0; q < x.nin; ++q)
            if (x.in_view[q] && !ok(x.in[q])) return VE_ERR_ARG;
        if (x.orig < 0) dt.temp[x.out.base] = dt(x.in[0].base);
    }
    std::vector<bool> dead;
    dead_outputs(ins, kid, dead);
    KernelCode kc;
    generate(ins, ks[k], dead, dt, {}, kc);
    *need = kc.src.size() + 1;
    if (buf && len >= *need) std::memcpy(buf, kc.src.c_str(), *need);
    return VE_OK;
}

extern "C" ve_status ve_execute(ve_engine e, const ve_instr *batch, int n)
{
    if (!e) return VE_ERR_ARG;
    if ((!batch && n > 0) || n < 0) {
        e->err = "bad batch";
        return VE_ERR_ARG;
    }
    std::vector<Ins> ins;
    auto arity = [e](int op) {
        if (op >= VE_USER) return op - VE_USER < (int)e->user_nin.size() ? e->user_nin[op - VE_USER] : -1;
        return builtin_arity(op);
    };
    ve_status r = to_internal(batch, n, arity, ins, e->err);
    if (r != VE_OK) return r;
    r = validate_bases(e, ins);
    if (r != VE_OK) return r;
    std::vector<int> kid;
    std::vector<KernelPlan> ks;
    form(ins, kid, ks);
    // staging bases: engine bases for this batch only
    std::vector<int> real(e->bases.size());
    std::vector<long long> real_n(e->bases.size());
    for (size_t b = 0; b < e->bases.size(); ++b) {
        real[b] = e->bases[b].dtype;
        real_n[b] = e->bases[b].nelem;
    }
    DtypeOf dt{&real, {}, &real_n, {}};
    std::map<int, int> temp_id;
    for (auto &x : ins)
        if (x.orig < 0) {
            const int d = x.in[0].base >= kTempBase ? dt.temp.at(x.in[0].base) : real[x.in[0].base];
            dt.temp[x.out.base] = d;
            dt.temp_n[x.out.base] = x.out.size();
            int id = 0;
            r = ve_base_new(e, d, x.out.size(), nullptr, &id);
            if (r != VE_OK) return r;
            temp_id[x.out.base] = id;
            ++e->st.staged;
        }
    std::vector<bool> dead;
    dead_outputs(ins, kid, dead);
    std::vector<KernelCode> codes(ks.size());
    std::vector<KernelCode *> todo;
    std::map<std::string, bool> queued;
    for (size_t k = 0; k < ks.size(); ++k) {
        const std::string key = kernel_key(ins, ks[k], dead, dt, e->user_exprs);
        auto g = e->generated.find(key);
        if (g != e->generated.end()) {
            codes[k] = g->second;
        } else {
            generate(ins, ks[k], dead, dt, e->user_exprs, codes[k]);
            if (e->generated.size() >= 1024) e->generated.clear();
            e->generated.emplace(key, codes[k]);
        }
        if (e->cache.count(codes[k].name)) {
            ++e->st.cache_hits;
        } else if (!queued.count(codes[k].name)) {
            queued[codes[k].name] = true;
            todo.push_back(&codes[k]);
        }
        for (size_t s = 0; s < codes[k].slots.size(); ++s)
            if (!codes[k].store[s]) {
                bool red = false;
                for (int q : codes[k].red_slot) red = red || q == (int)s;
                bool written = false;
                for (int m : ks[k].members) written = written || (same(ins[m].out, codes[k].slots[s]) && !red);
                if (written) ++e->st.stores_elided;
            }
    }
    r = compile_all(e, todo);
    if (r != VE_OK) return r;
    for (size_t k = 0; k < ks.size(); ++k) {
        KernelCode &kc = codes[k];
        std::vector<void *> ptrs(kc.slots.size(), nullptr);
        for (size_t s = 0; s < kc.slots.size(); ++s) {
            int b = kc.slots[s].base;
            if (b >= kTempBase) b = temp_id.at(b);
            bool red = false;
            for (int q : kc.red_slot) red = red || q == (int)s;
            if (kc.load[s] || kc.store[s] || red) {
                r = ensure_alloc(e, b);
                if (r != VE_OK) return r;
            }
            ptrs[s] = e->bases[b].ptr;
        }
        r = launch(e, kc, ptrs);
        if (r != VE_OK) return r;
        e->st.instructions += kc.ninstr;
    }
    if (e->prof) VECHK(e, close_run(e));  // a run never spans the host's time between batches
    // releases: staging bases and freed bases, after every launch of the batch
    for (auto &t : temp_id) {
        auto &B = e->bases[t.second];
        if (B.ptr) VECHK(e, hipFreeAsync(B.ptr, e->stream));
        B.ptr = nullptr;
        B.freed = true;
    }
    for (auto &x : ins)
        if (x.op == VE_FREE) {
            auto &B = e->bases[x.out.base];
            if (B.owned && B.ptr) VECHK(e, hipFreeAsync(B.ptr, e->stream));
            B.ptr = nullptr;
            B.freed = true;
        }
    return VE_OK;
}

extern "C" ve_status ve_stats_get(ve_engine e, ve_stats *st)
{
    if (!e || !st) return VE_ERR_ARG;
    *st = e->st;
    return VE_OK;
}

extern "C" ve_status ve_profile(ve_engine e, int on)
{
    if (!e) return VE_ERR_ARG;
    VECHK(e, close_run(e));
    e->prof = on != 0;
    if (!on) {
        e->pk.clear();
        e->pk_order.clear();
    }
    return VE_OK;
}

extern "C" ve_status ve_profile_read(ve_engine e, ve_kernel_timing *out, int max, int *count)
{
    if (!e || !count || (max > 0 && !out)) return VE_ERR_ARG;
    VECHK(e, close_run(e));
    VECHK(e, hipStreamSynchronize(e->stream));
    for (auto &r : e->pend) {
        float ms = 0.f;
        VECHK(e, hipEventElapsedTime(&ms, r.a, r.b));
        auto &p = e->pk[r.id];
        p.launches += r.count;
        p.total_ms += ms;
        p.bytes += r.bytes;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    e->pend.clear();
    int c = 0;
    for (int id : e->pk_order) {
        if (c < max) {
            const auto &p = e->pk[id];
            ve_kernel_timing &t = out[c];
            std::memset(&t, 0, sizeof(t));
            std::snprintf(t.name, sizeof t.name, "%s", p.name.c_str());
            t.launches = p.launches;
            t.total_ms = p.total_ms;
            t.avg_ms = p.launches ? p.total_ms / p.launches : 0.0;
            t.bytes_per_launch = p.launches ? p.bytes / p.launches : 0.0;
        }
        ++c;
    }
    *count = c;
    return VE_OK;
}

extern "C" const char *ve_last_error(ve_engine e) { return e ? e->err.c_str() : ""; }

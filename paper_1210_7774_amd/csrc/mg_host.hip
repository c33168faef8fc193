// Host runtime and C-ABI of libmgx.so: level hierarchy, workspace carve-up,
// the per-cycle launch schedule, the solve loops (plain FP64 and FP64
// iterative refinement around FP32 / bfloat16-state cycles), batches of
// independent systems, and hipGraph replay.
//
// The stop test runs on the device (the norm kernels write the residual
// history and a done flag that every later kernel of the solve checks), so
// the host enqueues cycles in chunks and synchronises once per chunk instead
// of once per cycle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mg.h"
#include "mg_internal.h"
#include "mg_m3.h"

using namespace mgx;

namespace {

constexpr size_t kAlign = 256;
constexpr double kLearnedFallback = 0.9;  // a learned cycle must reduce the residual at least this much
constexpr int kMaxStates = 4096;

struct Lvl {
    int n = 0;
    long long pitch = 0, ppitch = 0;
    double h = 0;
    void *A = nullptr, *B = nullptr, *f = nullptr, *a = nullptr;
    bool march = false;
    int desc = -1;
};

struct Sys {
    int n = 0;
    long long pitch0 = 0, ppitch0 = 0;
    const double *a64 = nullptr;
    std::vector<Lvl> lv;
    int lt = 0;           // first tail level
    int part0 = 0, nparts = 0;
    double *cinv = nullptr;
    double *acoarse64 = nullptr;  // FP64 coefficient of the coarsest level (setup only)
    // iterative refinement buffers (level 0 of the inner cycle)
    float *r32 = nullptr;
    // per call
    double *u = nullptr;
    const double *f = nullptr;
};

struct Group {            // march launches: all non-tail levels of one size
    int n;
    int item0 = 0, nitems = 0;
    int G = 1, Hb = 64, W = 0;
    bool finest = false;      // holds some system's finest level
    bool tiled = false;       // LDS-tiled kernels instead of row marching
    double bytes_pre = 0, bytes_post = 0;  // algorithmic bytes of one launch
};

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// message of the last failed mg_setup / mg_setup_batch of this thread
thread_local std::string g_setup_error;

bool is_pow2m1(int n) { return n >= 1 && ((n + 1) & n) == 0; }

int ipow(int b, int e)
{
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

int env_int(const char *name, int dflt)
{
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

// The bf16-state stall ratio of the history rule: a step that reduces the
// residual by less than this factor "stalls" (0.5: by less than 2x);
// MGX_BF16_STALL overrides it (tests force the fallback with it).
double bf16_stall_ratio()
{
    const char *v = getenv("MGX_BF16_STALL");
    const double r = (v && *v) ? atof(v) : 0.5;
    return (r > 0.0 && r < 1.0) ? r : 0.5;
}

}  // namespace

struct mg_handle_s {
    int dim = 2, nsys = 1;
    bool vc = false, ir = false, batch = false;
    int prec = MG_P_F64;
    int st = ST_F64;       // state type of the cycle
    int cs = 8, fs = 8;    // bytes of compute/coef type, rhs type
    mg_options opt{};
    hipStream_t stream = nullptr, capture = nullptr;
    std::string err;
    std::vector<Sys> sys;
    std::vector<Group> groups;
    int tail_top = 0, tail_nlev = 0, tail_m = 0, tail_threads = 256;
    size_t tail_lds = 0;
    bool tail_faces = false;
    bool tail_all_zero = true;

    // device
    char *ws = nullptr;
    size_t ws_bytes = 0;
    SolveState *d_states = nullptr;
    double *d_partials = nullptr;
    int npartials = 0;
    size_t items_cap = 0;  // MarchItem slots carved in the workspace
    LevelDesc *d_descs = nullptr;
    LevelDesc *d_tail = nullptr;
    MarchItem *d_items = nullptr;
    int *d_part0 = nullptr, *d_nparts = nullptr;     // march norm slots per system
    int *d_npart0 = nullptr, *d_nnparts = nullptr;   // batched outer-norm slots per system
    int *d_flag = nullptr;
    NormSys *d_nsys = nullptr;
    NormItem *d_nitems = nullptr;
    int nnitems = 0;
    int norm_blocks = 0;

    // host mirrors
    std::vector<LevelDesc> descs, tail_descs;
    std::vector<MarchItem> items;
    std::vector<NormSys> nsysv;
    std::vector<NormItem> nitemv;
    std::vector<LevelDesc> up_descs, up_tail;  // last uploaded
    std::vector<NormSys> up_nsys;
    char *pinned = nullptr;
    size_t pinned_bytes = 0;
    SolveState *h_states = nullptr;

    // per-kernel event timing
    struct PRec {
        int cls, step;
        hipEvent_t a, b;
    };
    struct PCls {
        std::string name;
        double bytes = 0;
        int launches = 0;
        double total_ms = 0;
    };
    // learned smoother (finest level of the inner cycle)
    bool learned = false, learned_on = false;
    const float *lw_master = nullptr;
    LearnedW lw{};
    bool learned_unfused = false;  // MGX_LEARNED_UNFUSED=1: one kernel per layer (A/B comparisons)
    float *l_sbuf = nullptr;
    bf16_t *l_x1 = nullptr, *l_x2 = nullptr, *l_x3 = nullptr;

    bool prof = false;
    std::vector<int> level_sizes;  // distinct non-tail level sizes, descending
    // autotuned launch shapes per 2D level size: (block height, LDS tiles)
    std::vector<std::pair<int, std::pair<int, int>>> tune;
    bool prof_finest_only = false;  // mg_profile(h, 2)
    int level_sizes_max = 0;
    bool norm_in_post = false;  // descriptors of the finest level carry norm = 1
    bool m3 = false;            // 3D red-black levels run the fused plane-marching passes
    int skew1 = 0;              // 4: use the skew-1 stage schedule (comparison runs)
    int prof_step = -1;
    std::vector<PRec> pend;
    std::vector<hipEvent_t> pool;
    std::vector<PCls> classes;

    // W- and F-cycles and full multigrid (single systems): descriptors with
    // every level's zero start off (for the later visits of a level within
    // one visit of its parent) and the tail's level-operation schedules
    LevelDesc *d_descs_keep = nullptr;
    std::vector<LevelDesc> descs_keep, up_keep;
    int *d_ops = nullptr;
    std::vector<int> tail_ops;
    int ops_off[3] = {0, 0, 0}, ops_cnt[3] = {0, 0, 0};  // indexed by TailList

    // graph
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    bool graph_ok = false;
    bool first_zero = false;  // enqueueing a zero-start solve's first step (fused 3D path)
};

#define HIPCHK(h, call)                                                   \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) {                                           \
            (h)->err = std::string(#call) + ": " + hipGetErrorString(e_); \
            return MG_ERR_HIP;                                            \
        }                                                                 \
    } while (0)

extern "C" void mg_options_default(mg_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->nu1 = 2;
    o->nu2 = 2;
    o->smoother = MG_SM_RBGS;
    o->precision = MG_P_F64;
    o->ncoarse = 0;
    o->max_cycles = 100;
    o->inner_cycles = 1;
    o->use_graph = 0;
    o->omega = 0.0;
    o->learned = nullptr;
    o->stream = nullptr;
    o->cycle = MG_CYCLE_V;
    o->fmg = 0;
    o->zero_start = 0;
}

namespace {

mg_options normalised(const mg_options *in, int dim)
{
    mg_options o;
    if (in) o = *in;
    else mg_options_default(&o);
    if (o.ncoarse == 0) o.ncoarse = (dim == 1) ? 1 : 3;
    if (o.max_cycles == 0) o.max_cycles = 100;
    if (o.inner_cycles == 0) o.inner_cycles = 1;
    if (o.omega == 0.0) o.omega = 2.0 * dim / (2.0 * dim + 1.0);
    return o;
}

mg_status check_grid(const mg_grid *g, const mg_operator *op, const mg_options &o)
{
    if (!g) return MG_ERR_ARG;
    if (g->dim < 1 || g->dim > 3) return MG_ERR_ARG;
    const int n = g->n[0];
    for (int ax = 0; ax < 3; ++ax) {
        if (ax < g->dim) {
            if (g->n[ax] != n) return MG_ERR_UNSUPPORTED;
        } else if (g->n[ax] != 1 && g->n[ax] != 0) {
            return MG_ERR_ARG;
        }
    }
    if (!is_pow2m1(n)) return MG_ERR_ARG;
    if (o.ncoarse != 1 && o.ncoarse != 3) return MG_ERR_ARG;
    if (n < o.ncoarse) return MG_ERR_ARG;
    if (g->dim > 1 && g->pitch[1] != 0 && g->pitch[1] < n) return MG_ERR_ARG;
    if (g->dim > 2 && g->pitch[2] != 0 && g->pitch[2] < (long long)n * (g->pitch[1] ? g->pitch[1] : n))
        return MG_ERR_ARG;
    if ((long long)n * n * (g->dim > 2 ? n : 1) > (1LL << 31) - 1) return MG_ERR_UNSUPPORTED;
    if (g->dim == 2) {
        // the 2D fused kernels address a level's arrays through buffer
        // descriptors with 32-bit byte counts: the finest FP64 array (with its
        // pitch) and the (n+2)^2 nodal coefficient must stay below 4 GiB
        const long long pitch = g->pitch[1] ? g->pitch[1] : n;
        const long long ext = ((long long)(n - 1) * pitch + n) * 8;
        const long long coef = (long long)(n + 2) * (n + 2) * 8;
        if (ext >= (1LL << 32) - 16 || coef >= (1LL << 32) - 16) return MG_ERR_UNSUPPORTED;
    }
    if (op) {
        if (op->kind != MG_OP_POISSON && op->kind != MG_OP_DIFFUSION) return MG_ERR_ARG;
        if (op->kind == MG_OP_DIFFUSION) {
            if (g->dim != 2) return MG_ERR_UNSUPPORTED;
            if (!op->a) return MG_ERR_ARG;
        }
    }
    if (o.nu1 < 0 || o.nu2 < 0 || o.nu1 > 8 || o.nu2 > 8 || o.nu1 + o.nu2 == 0) return MG_ERR_ARG;
    if (o.smoother != MG_SM_RBGS && o.smoother != MG_SM_JACOBI && o.smoother != MG_SM_LEARNED) return MG_ERR_ARG;
    if (o.smoother == MG_SM_LEARNED) {
        if (g->dim != 2 || o.precision == MG_P_F64) return MG_ERR_UNSUPPORTED;
        if (!op || op->kind != MG_OP_DIFFUSION) return MG_ERR_UNSUPPORTED;
        if (!o.learned) return MG_ERR_ARG;
    }
    if (o.precision < MG_P_F64 || o.precision > MG_P_F32_BF16_IR) return MG_ERR_ARG;
    if (o.max_cycles < 1 || o.max_cycles > MG_MAX_CYCLES) return MG_ERR_ARG;
    if (o.inner_cycles != 1) return MG_ERR_UNSUPPORTED;
    if (!(o.omega > 0.0 && o.omega < 2.0)) return MG_ERR_ARG;
    if (o.cycle < MG_CYCLE_V || o.cycle > MG_CYCLE_F || o.fmg < 0 || o.fmg > 1) return MG_ERR_ARG;
    if (o.zero_start < 0 || o.zero_start > 1) return MG_ERR_ARG;
    if ((o.cycle != MG_CYCLE_V || o.fmg) && o.smoother == MG_SM_LEARNED) return MG_ERR_UNSUPPORTED;
    if (o.fmg && o.precision != MG_P_F64) return MG_ERR_UNSUPPORTED;
    return MG_OK;
}

int tail_top_for(int dim, int st, bool vc)
{
    if (dim == 1) return 1 << 20;
    // the largest level the single-workgroup tail runs: 2D 63 (31 for
    // diffusion when level 63's face tables would not fit in LDS, FP64); 3D 15.
    // MGX_TAIL_TOP overrides (at most 63 in 2D, 15 in 3D)
    int t = 15;
    if (dim == 2) t = vc && tail_lds_bytes(st, 2, 63, false, true) > tail_max_lds() ? 31 : 63;
    return std::min(dim == 2 ? 63 : 15, env_int("MGX_TAIL_TOP", t));
}

// ---- tail schedules for W- and F-cycles and full multigrid ----------------
// Levels are relative to the tail's top level; the tail holds nl levels.
enum TailList { TL_PAIR = 0, TL_SELF = 1, TL_FMG = 2 };

// One visit of tail level r by a cycle of type `kind` (the coarsest level is
// solved directly whatever the type).
void tail_visit(std::vector<int> &ops, int r, int nl, int kind, int nu1, int nu2)
{
    if (r == nl - 1) {
        ops.push_back(TAIL_OP_SOLVE);
        return;
    }
    ops.push_back(TAIL_OP_SMOOTH | r << 4 | nu1 << 12);
    ops.push_back(TAIL_OP_RESTRICT | r << 4);
    if (kind == MG_CYCLE_W) {
        tail_visit(ops, r + 1, nl, MG_CYCLE_W, nu1, nu2);
        tail_visit(ops, r + 1, nl, MG_CYCLE_W, nu1, nu2);
    } else if (kind == MG_CYCLE_F) {
        tail_visit(ops, r + 1, nl, MG_CYCLE_F, nu1, nu2);
        tail_visit(ops, r + 1, nl, MG_CYCLE_V, nu1, nu2);
    } else {
        tail_visit(ops, r + 1, nl, MG_CYCLE_V, nu1, nu2);
    }
    ops.push_back(TAIL_OP_PROLONG | r << 4);
    ops.push_back(TAIL_OP_SMOOTH | r << 4 | nu2 << 12);
}

// The schedules one handle needs, for its cycle type k:
//   TL_PAIR  the visits of the tail's top level made by one visit of its
//            parent (W: two W visits; F: an F then a V visit);
//   TL_SELF  one visit of the top level (the whole hierarchy in the tail);
//   TL_FMG   full multigrid from the top level: f carried down by full
//            weighting, the coarsest solve, then on each finer level
//            u = P u_c and one visit.
void build_tail_ops(mg_handle_s *h)
{
    h->tail_ops.clear();
    if (h->opt.cycle == MG_CYCLE_V && !h->opt.fmg) return;
    const Sys &S = h->sys[0];
    const int nl = (int)S.lv.size() - S.lt, k = h->opt.cycle, nu1 = h->opt.nu1, nu2 = h->opt.nu2;
    std::vector<int> &o = h->tail_ops;
    h->ops_off[TL_PAIR] = (int)o.size();
    if (k == MG_CYCLE_W) {
        tail_visit(o, 0, nl, MG_CYCLE_W, nu1, nu2);
        tail_visit(o, 0, nl, MG_CYCLE_W, nu1, nu2);
    } else if (k == MG_CYCLE_F) {
        tail_visit(o, 0, nl, MG_CYCLE_F, nu1, nu2);
        tail_visit(o, 0, nl, MG_CYCLE_V, nu1, nu2);
    } else {
        tail_visit(o, 0, nl, MG_CYCLE_V, nu1, nu2);
    }
    h->ops_cnt[TL_PAIR] = (int)o.size() - h->ops_off[TL_PAIR];
    h->ops_off[TL_SELF] = (int)o.size();
    tail_visit(o, 0, nl, k, nu1, nu2);
    h->ops_cnt[TL_SELF] = (int)o.size() - h->ops_off[TL_SELF];
    h->ops_off[TL_FMG] = (int)o.size();
    for (int r = 0; r + 1 < nl; ++r) o.push_back(TAIL_OP_RESTRICT_RHS | r << 4);
    o.push_back(TAIL_OP_SOLVE);
    for (int r = nl - 2; r >= 0; --r) {
        o.push_back(TAIL_OP_INTERP | r << 4);
        tail_visit(o, r, nl, k, nu1, nu2);
    }
    h->ops_cnt[TL_FMG] = (int)o.size() - h->ops_off[TL_FMG];
}

// Bytes of workspace needed by `nsys` systems with sizes n[s]; fills offsets
// when `h` is given (carve mode).
struct Carver {
    size_t off = 0;
    char *base = nullptr;
    void *take(size_t bytes)
    {
        off = align_up(off);
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

// Build the hierarchy description (sizes, flags) for system sizes.
void plan(mg_handle_s *h, const std::vector<int> &ns)
{
    h->sys.assign(ns.size(), Sys());
    const int tt = tail_top_for(h->dim, h->st, h->vc);
    for (size_t s = 0; s < ns.size(); ++s) {
        Sys &S = h->sys[s];
        S.n = ns[s];
        for (int n = ns[s];; n = (n - 1) / 2) {
            Lvl L;
            L.n = n;
            L.h = 1.0 / (n + 1);
            S.lv.push_back(L);
            if (n <= h->opt.ncoarse) break;
        }
        S.lt = 0;
        while (S.lt < (int)S.lv.size() && S.lv[S.lt].n > tt) ++S.lt;
        // the learned smoother runs on the finest level outside the tail
        if (h->opt.smoother == MG_SM_LEARNED && S.lt == 0 && S.lv.size() > 1) S.lt = 1;
        // the tail holds at most 12 levels and must fit in LDS; deeper (1D)
        // hierarchies keep more levels outside
        while ((int)S.lv.size() - S.lt > 12) ++S.lt;
        while (S.lt + 1 < (int)S.lv.size() &&
               tail_lds_bytes(h->st, h->dim, S.lv[S.lt].n, h->opt.smoother == MG_SM_JACOBI, false) > tail_max_lds())
            ++S.lt;
        // red-black levels march; with the learned smoother the finest level
        // runs learned steps (generic path) and the coarser ones march
        const bool gs = h->opt.smoother == MG_SM_RBGS || h->opt.smoother == MG_SM_LEARNED;
        const bool march_ok = h->dim == 2 && gs && h->opt.nu1 >= 1 && h->opt.nu1 <= 3 && h->opt.nu2 >= 1 &&
                              h->opt.nu2 <= 3 && h->opt.nu1 == h->opt.nu2;
        for (int l = 0; l < S.lt; ++l)
            S.lv[l].march = march_ok && env_int("MGX_GENERIC", 0) == 0 &&
                            !(l == 0 && h->opt.smoother == MG_SM_LEARNED);
    }
}

size_t state_bytes(int st) { return st == ST_F64 ? 8 : 4; }  // bf16 buffers sized for an FP32 fallback

// Carve the workspace (base == nullptr: only measure).
size_t carve(mg_handle_s *h, char *base)
{
    Carver cv;
    cv.base = base;
    const int nsys = h->nsys;
    h->d_states = (SolveState *)cv.take(sizeof(SolveState) * nsys);
    // partial slots: level-0 march items + generic norm blocks + batched norm items
    size_t nparts = 0;
    for (auto &S : h->sys) {
        const Lvl &L0 = S.lv[0];
        if (L0.march) {
            const int G = env_int("MGX_G", 1);
            const int W = march_strip_width(G, h->opt.nu2);
            const int strips = (L0.n + W - 1) / W;
            nparts += (size_t)strips * (L0.n + 1);  // upper bound (Hb >= 2)
        }
    }
    size_t nni0 = 0;
    for (auto &S : h->sys) nni0 += (S.n + 15) / 16;
    nparts = std::max(nparts, nni0);
    nparts = std::max(nparts, (size_t)8192);
    if (h->dim == 3) {
        nparts = std::max(nparts, (size_t)march3d_blocks(h->sys[0].n, M3_TAIL_NORM, ST_F64));
        nparts = std::max(nparts, (size_t)march3dw_blocks(h->sys[0].n));
    }
    h->npartials = (int)nparts;
    h->d_partials = (double *)cv.take(sizeof(double) * 2 * nparts);
    // descriptors and items (upper bounds)
    size_t nlev = 0, nitems = 0;
    for (auto &S : h->sys) {
        nlev += S.lv.size();
        for (int l = 0; l < S.lt; ++l) {
            const int W = march_strip_width(1, std::max(h->opt.nu1, h->opt.nu2));
            nitems += (size_t)((S.lv[l].n + W - 1) / W + 1) * (S.lv[l].n / 2 + 2);
        }
    }
    h->d_descs = (LevelDesc *)cv.take(sizeof(LevelDesc) * std::max<size_t>(nlev, 1));
    h->d_tail = (LevelDesc *)cv.take(sizeof(LevelDesc) * std::max<size_t>(nlev, 1));
    if (!h->tail_ops.empty()) {
        h->d_descs_keep = (LevelDesc *)cv.take(sizeof(LevelDesc) * std::max<size_t>(nlev, 1));
        h->d_ops = (int *)cv.take(sizeof(int) * h->tail_ops.size());
    }
    h->d_items = (MarchItem *)cv.take(sizeof(MarchItem) * std::max<size_t>(nitems, 1));
    h->items_cap = nitems;
    h->d_part0 = (int *)cv.take(sizeof(int) * nsys);
    h->d_nparts = (int *)cv.take(sizeof(int) * nsys);
    h->d_npart0 = (int *)cv.take(sizeof(int) * nsys);
    h->d_nnparts = (int *)cv.take(sizeof(int) * nsys);
    h->d_nsys = (NormSys *)cv.take(sizeof(NormSys) * nsys);
    size_t nni = 0;
    for (auto &S : h->sys) nni += (S.n + 15) / 16;
    h->d_nitems = (NormItem *)cv.take(sizeof(NormItem) * std::max<size_t>(nni, 1));
    h->d_flag = (int *)cv.take(sizeof(int) * 4);
    {
        const int m = ipow(h->sys[0].lv.back().n, h->dim);
        double *all = (double *)cv.take(sizeof(double) * (size_t)m * m * nsys);
        for (int s = 0; s < nsys; ++s) h->sys[s].cinv = all ? all + (size_t)s * m * m : nullptr;
    }
    for (auto &S : h->sys) {
        if (h->vc) {
            const int nc = S.lv.back().n;
            S.acoarse64 = (double *)cv.take(sizeof(double) * (nc + 2) * (nc + 2));
        }
    }
    const size_t ssz = state_bytes(h->st);
    for (auto &S : h->sys) {
        for (size_t l = 0; l < S.lv.size(); ++l) {
            Lvl &L = S.lv[l];
            const long long m = (long long)L.n * (h->dim > 1 ? L.n : 1) * (h->dim > 2 ? L.n : 1);
            L.pitch = L.n;
            L.ppitch = (long long)L.n * L.n;
            if (l == 0 && !h->ir) {
                L.pitch = S.pitch0;
                L.ppitch = S.ppitch0;
            }
            L.A = cv.take(ssz * m);
            if (l > 0 || h->ir) {
                L.B = cv.take(ssz * m);
                L.f = cv.take((size_t)h->fs * m);
            }
            if (h->vc) {
                const long long ma = (long long)(L.n + 2) * (L.n + 2);
                if (l > 0 || h->ir) L.a = cv.take((size_t)h->cs * ma);
                else L.a = (void *)S.a64;
            }
        }
        if (h->ir) S.r32 = (float *)S.lv[0].f;
    }
    if (h->learned) {
        const long long n0 = h->sys[0].n;
        const long long px = n0 * n0;
        if (h->learned_unfused) {
            h->l_sbuf = (float *)cv.take(sizeof(float) * px);
            h->l_x1 = (bf16_t *)cv.take(sizeof(bf16_t) * 16 * px);
            h->l_x2 = (bf16_t *)cv.take(sizeof(bf16_t) * 16 * px);
            h->l_x3 = (bf16_t *)cv.take(sizeof(bf16_t) * 16 * px);
        }
        h->lw.w1 = (float *)cv.take(sizeof(float) * 144);
        h->lw.w4 = (float *)cv.take(sizeof(float) * 144);
        h->lw.wf2 = (bf16_t *)cv.take(sizeof(bf16_t) * 2304);
        h->lw.wd2 = (bf16_t *)cv.take(sizeof(bf16_t) * 2304);
        h->lw.wf3 = (bf16_t *)cv.take(sizeof(bf16_t) * 2304);
        h->lw.wd3 = (bf16_t *)cv.take(sizeof(bf16_t) * 2304);
        h->lw.w1m = (bf16_t *)cv.take(sizeof(bf16_t) * 256);
        h->lw.w2k = (bf16_t *)cv.take(sizeof(bf16_t) * 2560);
        h->lw.w3k = (bf16_t *)cv.take(sizeof(bf16_t) * 2560);
        h->lw.w4k = (bf16_t *)cv.take(sizeof(bf16_t) * 2560);
    }
    return align_up(cv.off);
}

// Host-side dense inverse by Gauss-Jordan elimination with partial pivoting.
bool invert(int m, std::vector<double> &A, std::vector<double> &inv)
{
    inv.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) inv[(size_t)i * m + i] = 1.0;
    for (int c = 0; c < m; ++c) {
        int p = c;
        for (int r = c + 1; r < m; ++r)
            if (std::fabs(A[(size_t)r * m + c]) > std::fabs(A[(size_t)p * m + c])) p = r;
        if (A[(size_t)p * m + c] == 0.0) return false;
        if (p != c)
            for (int k = 0; k < m; ++k) {
                std::swap(A[(size_t)p * m + k], A[(size_t)c * m + k]);
                std::swap(inv[(size_t)p * m + k], inv[(size_t)c * m + k]);
            }
        const double d = A[(size_t)c * m + c];
        for (int k = 0; k < m; ++k) {
            A[(size_t)c * m + k] /= d;
            inv[(size_t)c * m + k] /= d;
        }
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            const double fct = A[(size_t)r * m + c];
            if (fct == 0.0) continue;
            for (int k = 0; k < m; ++k) {
                A[(size_t)r * m + k] -= fct * A[(size_t)c * m + k];
                inv[(size_t)r * m + k] -= fct * inv[(size_t)c * m + k];
            }
        }
    }
    return true;
}

// The coarsest-level matrix (interior nodes, x fastest) of the Poisson or
// diffusion operator on n^d nodes.
void coarse_matrix(int dim, int n, const double *a, std::vector<double> &M)
{
    const int m = ipow(n, dim);
    M.assign((size_t)m * m, 0.0);
    const double ih2 = (double)(n + 1) * (n + 1);
    auto id = [&](int i, int j, int k) { return (i - 1) + n * ((j - 1) + n * (k - 1)); };
    auto node = [&](int i, int j) { return a[i + (n + 2) * j]; };
    for (int p = 0; p < m; ++p) {
        int t = p;
        const int i = t % n + 1;
        t /= n;
        const int j = dim > 1 ? t % n + 1 : 1;
        t = dim > 1 ? t / n : t;
        const int k = dim > 2 ? t + 1 : 1;
        const int c[3] = {i, j, k};
        double diag = 0.0;
        for (int ax = 0; ax < dim; ++ax)
            for (int dir = -1; dir <= 1; dir += 2) {
                int q[3] = {c[0], c[1], c[2]};
                q[ax] += dir;
                double w = 1.0;
                if (a) {
                    const double ap = node(c[0], c[1]), aq = node(q[0], q[1]);
                    w = 2.0 * ap * aq / (ap + aq);
                }
                diag += w;
                if (q[ax] >= 1 && q[ax] <= n) M[(size_t)p * m + id(q[0], q[1], q[2])] -= w * ih2;
            }
        M[(size_t)p * m + p] += diag * ih2;
    }
}

LevelDesc make_desc(const mg_handle_s *h, const Sys &S, int l, int sysi)
{
    const Lvl &L = S.lv[l];
    LevelDesc d;
    std::memset(&d, 0, sizeof(d));
    d.n = L.n;
    d.dim = h->dim;
    d.sys = sysi;
    d.pitch = L.pitch;
    d.ppitch = L.ppitch;
    d.h2 = L.h * L.h;
    d.inv_h2 = 1.0 / d.h2;
    d.a = L.a;
    d.A = L.A;
    d.B = L.B;
    d.f = L.f;
    if (l + 1 < (int)S.lv.size()) {
        const Lvl &Lc = S.lv[l + 1];
        d.nc = Lc.n;
        d.cpitch = Lc.pitch;
        d.cppitch = Lc.ppitch;
        d.fc = Lc.f;
        d.Bc = Lc.B;
    }
    d.uzero = (l > 0) ? 1 : 0;
    if (l == 0) {
        if (h->ir) {
            d.uzero = 1;
            d.acc = S.u;
            d.acc_pitch = S.pitch0;
            d.acc_ppitch = S.ppitch0;
        } else {
            d.B = S.u;
            d.f = (void *)S.f;
        }
    }
    return d;
}

// Rebuild the per-call descriptors (level-0 pointers) and upload what changed.
mg_status refresh(mg_handle_s *h, bool norm_in_post)
{
    if (h->norm_in_post != norm_in_post) h->graph_ok = false;
    h->norm_in_post = norm_in_post;
    h->descs.clear();
    h->tail_descs.clear();
    for (int s = 0; s < h->nsys; ++s) {
        Sys &S = h->sys[s];
        for (size_t l = 0; l < S.lv.size(); ++l) {
            LevelDesc d = make_desc(h, S, (int)l, s);
            if (l == 0 && !h->ir && S.lv[0].march) d.norm = norm_in_post ? 1 : 0;
            S.lv[l].desc = (int)h->descs.size();
            h->descs.push_back(d);
        }
        for (size_t l = S.lt; l < S.lv.size(); ++l) h->tail_descs.push_back(h->descs[S.lv[l].desc]);
    }
    h->descs_keep.clear();
    if (h->d_descs_keep) {
        h->descs_keep = h->descs;
        for (auto &d : h->descs_keep) d.uzero = 0;
    }
    for (int s = 0; s < h->nsys; ++s) {
        NormSys &ns = h->nsysv[s];
        ns.u = h->sys[s].u;
        ns.f = h->sys[s].f;
    }
    const bool same = h->up_descs.size() == h->descs.size() &&
                      !std::memcmp(h->up_descs.data(), h->descs.data(), sizeof(LevelDesc) * h->descs.size()) &&
                      h->up_tail.size() == h->tail_descs.size() &&
                      !std::memcmp(h->up_tail.data(), h->tail_descs.data(), sizeof(LevelDesc) * h->tail_descs.size()) &&
                      h->up_nsys.size() == h->nsysv.size() &&
                      !std::memcmp(h->up_nsys.data(), h->nsysv.data(), sizeof(NormSys) * h->nsysv.size()) &&
                      h->up_keep.size() == h->descs_keep.size() &&
                      !std::memcmp(h->up_keep.data(), h->descs_keep.data(), sizeof(LevelDesc) * h->descs_keep.size());
    if (same) return MG_OK;
    const size_t b1 = sizeof(LevelDesc) * h->descs.size(), b2 = sizeof(LevelDesc) * h->tail_descs.size(),
                 b3 = sizeof(NormSys) * h->nsysv.size(), b4 = sizeof(LevelDesc) * h->descs_keep.size();
    if (h->pinned_bytes < b1 + b2 + b3 + b4) {
        if (h->pinned) (void)hipHostFree(h->pinned);
        h->pinned = nullptr;
        HIPCHK(h, hipHostMalloc((void **)&h->pinned, b1 + b2 + b3 + b4, hipHostMallocDefault));
        h->pinned_bytes = b1 + b2 + b3 + b4;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    std::memcpy(h->pinned, h->descs.data(), b1);
    std::memcpy(h->pinned + b1, h->tail_descs.data(), b2);
    std::memcpy(h->pinned + b1 + b2, h->nsysv.data(), b3);
    if (b4) std::memcpy(h->pinned + b1 + b2 + b3, h->descs_keep.data(), b4);
    HIPCHK(h, hipMemcpyAsync(h->d_descs, h->pinned, b1, hipMemcpyHostToDevice, h->stream));
    if (b2) HIPCHK(h, hipMemcpyAsync(h->d_tail, h->pinned + b1, b2, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->d_nsys, h->pinned + b1 + b2, b3, hipMemcpyHostToDevice, h->stream));
    if (b4) HIPCHK(h, hipMemcpyAsync(h->d_descs_keep, h->pinned + b1 + b2 + b3, b4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->up_descs = h->descs;
    h->up_tail = h->tail_descs;
    h->up_nsys = h->nsysv;
    h->up_keep = h->descs_keep;
    h->graph_ok = false;
    return MG_OK;
}

// one 64-lane workgroup per item, rounded up to a multiple of the 8 XCDs
int march_grid(int nitems) { return std::min((nitems + 7) / 8 * 8, 65536); }

GenArgs gen_args(const mg_handle_s *h, int s, int l)
{
    GenArgs g;
    std::memset(&g, 0, sizeof(g));
    g.L = h->descs[h->sys[s].lv[l].desc];
    g.state = h->d_states + s;
    g.omega = h->opt.omega;
    g.u_zero = g.L.uzero;
    return g;
}

// Smoothing on one level with the generic kernels (in place on B).
hipError_t gen_smooth(mg_handle_s *h, int s, int l, int nsweeps, hipStream_t st)
{
    GenArgs g = gen_args(h, s, l);
    hipError_t e = hipSuccess;
    if (l == 0 && h->learned && h->learned_on) {
        // learned steps on the inner finest level: e <- e + N(D^-1 (r - A e))
        const Lvl &L = h->sys[s].lv[0];
        if (h->learned_unfused) {
            for (int k = 0; k < nsweeps && e == hipSuccess; ++k)
                e = learned_step(h->st, L.B, (const float *)L.f, (const float *)L.a, L.n, L.h * L.h, h->lw,
                                 h->l_sbuf, h->l_x1, h->l_x2, h->l_x3, st);
            return e;
        }
        // fused steps ping-pong between the level's two state buffers
        void *src = L.B, *dst = L.A;
        for (int k = 0; k < nsweeps && e == hipSuccess; ++k) {
            e = learned_step_fused(h->st, src, dst, (const float *)L.f, (const float *)L.a, L.n, L.h * L.h, h->lw,
                                   st);
            std::swap(src, dst);
        }
        if (e == hipSuccess && (nsweeps & 1)) e = launch_copy_state(h->st, g, g.L.A, g.L.B, st);
        return e;
    }
    if (h->dim == 3 && h->opt.smoother == MG_SM_RBGS && nsweeps % 2 == 0 && env_int("MGX_RB3_HALF", 0) == 0) {
        // fused 3D sweeps, B -> A -> B (A is contiguous)
        const Lvl &L = h->sys[s].lv[l];
        const long long n = L.n;
        for (int k = 0; k < nsweeps && e == hipSuccess; ++k) {
            const bool fwd = (k % 2 == 0);
            e = launch_rb3_sweep(h->st, fwd ? g.L.B : g.L.A, fwd ? g.L.pitch : n, fwd ? g.L.ppitch : n * n,
                                 fwd ? g.L.A : g.L.B, fwd ? n : g.L.pitch, fwd ? n * n : g.L.ppitch, g.L.f, g.L.pitch,
                                 g.L.ppitch, (int)n, g.L.h2, g.state, st);
        }
        return e;
    }
    for (int k = 0; k < nsweeps && e == hipSuccess; ++k) {
        if (h->opt.smoother == MG_SM_JACOBI) {
            g.src = g.L.B;
            g.dst = g.L.A;
            g.u_zero = 0;
            e = launch_jacobi(h->st, h->vc, g, st);
            if (e == hipSuccess) e = launch_copy_state(h->st, g, g.L.A, g.L.B, st);
        } else {
            for (int c = 0; c < 2 && e == hipSuccess; ++c) {
                g.colour = c;
                e = launch_rb_half(h->st, h->vc, g, st);
            }
        }
    }
    return e;
}

long long level_points(int n, int dim) { return (long long)n * (dim > 1 ? n : 1) * (dim > 2 ? n : 1); }

// ---- per-kernel timing -------------------------------------------------------
int prof_class(mg_handle_s *h, const std::string &name, double bytes)
{
    for (size_t i = 0; i < h->classes.size(); ++i)
        if (h->classes[i].name == name) return (int)i;
    mg_handle_s::PCls c;
    c.name = name;
    c.bytes = bytes;
    h->classes.push_back(c);
    return (int)h->classes.size() - 1;
}

hipEvent_t prof_event(mg_handle_s *h)
{
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Bracket one launch with events when profiling (returns the record index or -1).
int prof_begin(mg_handle_s *h, const std::string &name, double bytes, hipStream_t st)
{
    if (!h->prof) return -1;
    // mode 2: only the finest level's launches (the largest level size)
    if (h->prof_finest_only) {
        const std::string tag = " n=" + std::to_string(h->level_sizes_max);
        if (name.size() < tag.size() || name.compare(name.size() - tag.size(), tag.size(), tag) != 0) return -1;
    }
    mg_handle_s::PRec r;
    r.cls = prof_class(h, name, bytes);
    r.step = h->prof_step;
    r.a = prof_event(h);
    r.b = prof_event(h);
    if (!r.a || !r.b) return -1;
    (void)hipEventRecord(r.a, st);
    h->pend.push_back(r);
    return (int)h->pend.size() - 1;
}

void prof_end(mg_handle_s *h, int idx, hipStream_t st)
{
    if (idx >= 0) (void)hipEventRecord(h->pend[idx].b, st);
}

// Fold the pending records into the classes: records of steps < `effective`
// (and of step -1, work outside the cycle loop) count, later ones were no-ops.
void prof_collect(mg_handle_s *h, int effective)
{
    for (auto &r : h->pend) {
        if (r.step < effective) {
            float ms = 0.f;
            if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                h->classes[r.cls].launches += 1;
                h->classes[r.cls].total_ms += ms;
            }
        }
        h->pool.push_back(r.a);
        h->pool.push_back(r.b);
    }
    h->pend.clear();
}

std::string lvname(const char *phase, int n)
{
    return std::string(phase) + " n=" + std::to_string(n);
}

// Timing class and algorithmic bytes per point of one smoothing sweep.  The
// fused learned step reads e, f, a and writes e; the one-kernel-per-layer
// form also moves s and three 16-channel bf16 maps through memory.
std::string smooth_class(mg_handle_s *h, int l, int n)
{
    return lvname((l == 0 && h->learned && h->learned_on) ? "learned_step" : "smooth", n);
}

double smooth_bytes(mg_handle_s *h, int l, double pts)
{
    const double sb = (double)state_bytes(h->st);
    if (l == 0 && h->learned && h->learned_on) {
        const double es = h->st == ST_BF16 ? 2 : 4;
        if (h->learned_unfused) return pts * (16 + 4 + 3 * 64 + 2 * es);
        return pts * (2 * es + 4 + 4);  // fused: e in, f, a, e out
    }
    return pts * (2 * sb + h->fs);
}

// Enqueue one V-cycle of the working precision on every system.  March
// groups and generic levels are interleaved by level size (down: finest
// first; up: coarsest first): with the learned smoother the finest level is
// generic while the coarser ones march.
mg_status enqueue_march(mg_handle_s *h, const Group &g, bool post, hipStream_t st, bool keep = false)
{
    MarchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.levels = keep ? h->d_descs_keep : h->d_descs;
    a.items = h->d_items + g.item0;
    a.nitems = g.nitems;
    a.W = g.W;
    a.Hb = g.Hb;
    a.states = h->d_states;
    a.partials = h->d_partials;
    a.part0 = h->d_part0;
    a.nparts = h->d_nparts;
    if (g.tiled) {
        if (g.nitems > 0 && h->nsys == 1) {
            // one level: tiles from the workgroup index, the level's descriptor alone
            a.levels = (keep ? h->d_descs_keep : h->d_descs) + h->items[g.item0].lvl;
            a.items = nullptr;
        }
        const int pi = prof_begin(h, lvname(post ? "post_tile" : "pre_tile", g.n), post ? g.bytes_post : g.bytes_pre,
                                  st);
        HIPCHK(h, launch_tile2d(post ? 1 : 0, h->st, h->vc, post ? h->opt.nu2 : h->opt.nu1, a, st));
        prof_end(h, pi, st);
        return MG_OK;
    }
    if (!post) {
        const int pi = prof_begin(h, lvname("pre", g.n), g.bytes_pre, st);
        HIPCHK(h, launch_march2d(0 | (g.finest ? 2 : 0) | h->skew1, h->st, h->vc, h->opt.nu1, g.G, a,
                                 march_grid(g.nitems), st));
        prof_end(h, pi, st);
    } else {
        const int pi = prof_begin(h, lvname("post", g.n), g.bytes_post, st);
        HIPCHK(h, launch_march2d(1 | (g.finest ? 2 : 0) | h->skew1 | ((g.finest && h->ir) ? 8 : 0), h->st, h->vc,
                                 h->opt.nu2, g.G, a, march_grid(g.nitems), st));
        prof_end(h, pi, st);
    }
    return MG_OK;
}

// ---- fused 3D passes ------------------------------------------------------
// One red-black sweep per pass, ping-ponging between the level's two state
// buffers: PRE passes start from B (or from zero) and the last one adds the
// residual + restriction into the coarse rhs; POST passes start from where PRE
// left the state with the coarse-grid correction in front of the first sweep
// and end in B (equal sweep counts, or counts of equal parity, make both
// chains meet), the finest one with the residual norm (plain FP64) or added
// into the FP64 iterate (refinement).
bool use_m3(const mg_handle_s *h)
{
    return h->dim == 3 && !h->vc && h->opt.smoother == MG_SM_RBGS && h->opt.nu1 >= 1 && h->opt.nu2 >= 1 &&
           (h->opt.nu1 - h->opt.nu2) % 2 == 0 && env_int("MGX_M3", 1) != 0;
}

// the finest plain-FP64 POST measures the residual norm in its last pass
bool m3_norm_fused(const mg_handle_s *h)
{
    return h->m3 && !h->ir && h->norm_in_post && h->nsys == 1 && h->sys[0].lt > 0;
}

// Levels of at least MGX_M3W points per edge (default 31; 0 = never) run the
// wavefront passes: two sweeps per pass (the last pass of an odd count one),
// so PRE and POST take ceil(nu / 2) passes each, whose parities must agree for
// the two buffer chains to meet.
bool use_m3w(const mg_handle_s *h, int n)
{
    const int mn = env_int("MGX_M3W", 31);
    if (mn <= 0 || n < mn) return false;
    return ((h->opt.nu1 + 1) / 2 - (h->opt.nu2 + 1) / 2) % 2 == 0;
}

mg_status enqueue_m3(mg_handle_s *h, int s, int l, bool post, hipStream_t st, bool keep = false)
{
    Sys &S = h->sys[s];
    const Lvl &L = S.lv[l];
    const LevelDesc &d = h->descs[L.desc];
    const Lvl &Lc = S.lv[l + 1];
    const long long n = L.n;
    const double sb = h->st == ST_F64 ? 8.0 : h->st == ST_F32 ? 4.0 : 2.0;
    const double fb = h->fs, pts = (double)level_points(L.n, 3), cpts = (double)level_points(Lc.n, 3);
    // the two state buffers with their pitches (B may be the caller's array)
    struct Buf {
        void *p;
        long long pitch, ppitch;
    };
    const Buf B{d.B, d.pitch, d.ppitch}, A{d.A, n, n * n};
    M3Args a;
    std::memset(&a, 0, sizeof(a));
    a.n = L.n;
    a.nc = Lc.n;
    a.h2 = d.h2;
    a.ih2 = d.inv_h2;
    a.f = d.f;
    a.fp = d.pitch;
    a.fpp = d.ppitch;
    a.state = h->d_states + s;
    const int nu = post ? h->opt.nu2 : h->opt.nu1;
    // passes and their sweeps: one sweep each, or two (wavefront passes)
    const bool wf = use_m3w(h, L.n);
    const int npass = wf ? (nu + 1) / 2 : nu;
    const int npre = wf ? (h->opt.nu1 + 1) / 2 : h->opt.nu1;
    // PRE starts in B; POST starts where PRE ended (A after an odd count)
    bool inA = post ? (npre % 2 == 1) : false;
    for (int k = 0; k < npass; ++k) {
        const int ns = wf ? std::min(2, nu - 2 * k) : 1;
        const Buf src = inA ? A : B, dst = inA ? B : A;
        int head = M3_HEAD_U, tail = M3_TAIL_NONE;
        a.uin = src.p;
        a.ip = src.pitch;
        a.ipp = src.ppitch;
        a.uout = dst.p;
        a.op = dst.pitch;
        a.opp = dst.ppitch;
        a.acc = nullptr;
        a.fc = nullptr;
        a.uc = nullptr;
        a.partials = nullptr;
        double bytes = pts * (sb + fb + sb);
        std::string cls;
        if (!post) {
            if (k == 0 && (d.uzero || (l == 0 && h->first_zero)) && !keep) {
                head = M3_HEAD_ZERO;
                bytes -= pts * sb;
            }
            if (k == npass - 1) {
                tail = M3_TAIL_RR;
                a.fc = d.fc;
                a.fcp = d.cpitch;
                a.fcpp = d.cppitch;
                bytes += cpts * fb;
            }
            cls = tail == M3_TAIL_RR ? "pre_rr" : "pre_sweep";
            // (the finest level's first pass of a zero-start solve moves
            // fewer bytes: a timing class of its own)
            if (head == M3_HEAD_ZERO && !d.uzero) cls = tail == M3_TAIL_RR ? "pre_zero_rr" : "pre_zero_sweep";
        } else {
            if (k == 0) {
                head = M3_HEAD_CORR;
                a.uc = d.Bc;
                a.ucp = d.cpitch;
                a.ucpp = d.cppitch;
                bytes += cpts * sb;
            }
            if (k == npass - 1 && l == 0) {
                if (h->ir) {
                    a.acc = S.u;
                    a.accp = S.pitch0;
                    a.accpp = S.ppitch0;
                    bytes += pts * (16.0 - sb);
                } else if (m3_norm_fused(h)) {
                    tail = M3_TAIL_NORM;
                    a.partials = h->d_partials;
                }
            }
            cls = k == 0 ? "post_corr" : tail == M3_TAIL_NORM ? "post_norm" : "post_sweep";
            if (wf) cls = tail == M3_TAIL_NORM ? "post_norm" : a.acc ? "post_acc" : k == 0 ? "post_corr" : "post_sweep";
        }
        // wavefront passes: "w<sweeps>" in front of the pass name
        if (wf) cls = "w" + std::to_string(ns) + cls;
        const int pi = prof_begin(h, lvname(cls.c_str(), L.n), bytes, st);
        if (wf) HIPCHK(h, launch_march3dw(h->st, ns, head, tail, a, st));
        else HIPCHK(h, launch_march3d(h->st, head, tail, a, st));
        prof_end(h, pi, st);
        inA = !inA;
    }
    if (post && l == 0 && m3_norm_fused(h)) {
        const int pi = prof_begin(h, "norm_finish", 0.0, st);
        HIPCHK(h, launch_norm_finish(h->d_states, 1, h->d_partials, nullptr, nullptr, 0,
                                     wf ? march3dw_blocks(L.n) : march3d_blocks(L.n, M3_TAIL_NORM, h->st), 0, st));
        prof_end(h, pi, st);
    }
    return MG_OK;
}

mg_status enqueue_generic_down(mg_handle_s *h, int s, int l, hipStream_t st, bool keep = false)
{
    if (h->m3) return enqueue_m3(h, s, l, false, st, keep);
    Sys &S = h->sys[s];
    GenArgs g = gen_args(h, s, l);
    if (g.L.uzero && !keep) {
        const long long m = level_points(S.lv[l].n, h->dim);
        HIPCHK(h, launch_fill_zero(S.lv[l].B, (long long)state_bytes(h->st) * m, st));
    }
    const double pts = (double)level_points(S.lv[l].n, h->dim);
    int pi = prof_begin(h, smooth_class(h, l, S.lv[l].n), smooth_bytes(h, l, pts) * h->opt.nu1, st);
    HIPCHK(h, gen_smooth(h, s, l, h->opt.nu1, st));
    prof_end(h, pi, st);
    pi = prof_begin(h, lvname("resid_restrict", S.lv[l].n),
                    pts * (state_bytes(h->st) + h->fs) + (double)level_points(S.lv[l + 1].n, h->dim) * h->fs, st);
    HIPCHK(h, launch_resid_restrict(h->st, h->vc, g, st));
    prof_end(h, pi, st);
    return MG_OK;
}

mg_status enqueue_generic_up(mg_handle_s *h, int s, int l, hipStream_t st)
{
    if (h->m3) return enqueue_m3(h, s, l, true, st);
    Sys &S = h->sys[s];
    GenArgs g = gen_args(h, s, l);
    const double pts = (double)level_points(S.lv[l].n, h->dim);
    const double sb = (double)state_bytes(h->st);
    int pi = prof_begin(h, lvname("prolong_correct", S.lv[l].n),
                        pts * 2 * sb + (double)level_points(S.lv[l + 1].n, h->dim) * sb, st);
    HIPCHK(h, launch_prolong_correct(h->st, g, st));
    prof_end(h, pi, st);
    pi = prof_begin(h, smooth_class(h, l, S.lv[l].n), smooth_bytes(h, l, pts) * h->opt.nu2, st);
    HIPCHK(h, gen_smooth(h, s, l, h->opt.nu2, st));
    prof_end(h, pi, st);
    return MG_OK;
}

// The single-workgroup tail: a V-cycle from its top level (list < 0) or one
// of the handle's level-operation schedules (TailList).
mg_status enqueue_tail(mg_handle_s *h, hipStream_t st, int list)
{
    TailArgs t;
    std::memset(&t, 0, sizeof(t));
    t.levels = h->d_tail;
    t.nlev = h->tail_nlev;
    t.nsys = h->nsys;
    t.cinv = h->sys[0].cinv;
    t.m = h->tail_m;
    t.nu1 = h->opt.nu1;
    t.nu2 = h->opt.nu2;
    t.smoother = h->opt.smoother == MG_SM_JACOBI ? 1 : 0;
    t.omega = h->opt.omega;
    t.states = h->d_states;
    t.faces = h->tail_faces ? 1 : 0;
    if (list >= 0) {
        if (!h->d_ops) {
            h->err = "tail schedule requested without one";
            return MG_ERR_ARG;
        }
        t.ops = h->d_ops + h->ops_off[list];
        t.nops = h->ops_cnt[list];
    }
    const double tb = (double)h->nsys * level_points(h->tail_top, h->dim) * (h->fs + state_bytes(h->st));
    const int pi = prof_begin(h, "tail", tb, st);
    HIPCHK(h, launch_tail_sized(h->st, h->vc, h->dim, t, h->tail_lds, h->tail_threads, st));
    prof_end(h, pi, st);
    return MG_OK;
}

// plain mode: the finest POST measured the residual; reduce + stop test
mg_status enqueue_post_norm(mg_handle_s *h, hipStream_t st)
{
    if (!h->ir && h->sys[0].lv[0].march && h->norm_in_post) {
        const int pi = prof_begin(h, "norm_finish", 0.0, st);
        HIPCHK(h, launch_norm_finish(h->d_states, h->nsys, h->d_partials, h->d_part0, h->d_nparts, 0, 0, 0, st));
        prof_end(h, pi, st);
    }
    return MG_OK;
}

// One visit of level l of the single system by a cycle of type `kind`
// (standard multigrid cycles): pre-smoothing and the restricted residual,
// then the coarse level visited once (V), twice (W), or by an F- and then a
// V-visit (F), each first visit from a zero correction and later ones from
// the previous result, then the coarse-grid correction and post-smoothing.
// keep: level l starts from its current state instead of zero.  The visits
// of the tail's top level are one tail launch.
mg_status enqueue_visit(mg_handle_s *h, int l, int kind, bool keep, hipStream_t st)
{
    Sys &S = h->sys[0];
    if (l == S.lt) return enqueue_tail(h, st, TL_SELF);  // the whole hierarchy in the tail
    const Group *grp = nullptr;
    if (S.lv[l].march)
        for (auto &g : h->groups)
            if (g.n == S.lv[l].n) grp = &g;
    mg_status rc = grp ? enqueue_march(h, *grp, false, st, keep) : enqueue_generic_down(h, 0, l, st, keep);
    if (rc != MG_OK) return rc;
    if (l + 1 == S.lt) {
        rc = enqueue_tail(h, st, kind == MG_CYCLE_V ? -1 : TL_PAIR);
    } else if (kind == MG_CYCLE_W) {
        if ((rc = enqueue_visit(h, l + 1, MG_CYCLE_W, false, st)) == MG_OK)
            rc = enqueue_visit(h, l + 1, MG_CYCLE_W, true, st);
    } else if (kind == MG_CYCLE_F) {
        if ((rc = enqueue_visit(h, l + 1, MG_CYCLE_F, false, st)) == MG_OK)
            rc = enqueue_visit(h, l + 1, MG_CYCLE_V, true, st);
    } else {
        rc = enqueue_visit(h, l + 1, MG_CYCLE_V, false, st);
    }
    if (rc != MG_OK) return rc;
    return grp ? enqueue_march(h, *grp, true, st) : enqueue_generic_up(h, 0, l, st);
}

// One full-multigrid pass (nested iteration) on the single system: f carried
// down by full weighting, the coarsest level solved, and on every finer level
// u = P u_c followed by one cycle of the handle's type; u is overwritten.
mg_status enqueue_fmg(mg_handle_s *h, hipStream_t st)
{
    Sys &S = h->sys[0];
    for (int l = 0; l < S.lt; ++l) {
        const GenArgs g = gen_args(h, 0, l);
        const int pi = prof_begin(h, lvname("fmg_restrict", S.lv[l].n),
                                  (double)(level_points(S.lv[l].n, h->dim) + level_points(S.lv[l + 1].n, h->dim)) *
                                      h->fs, st);
        HIPCHK(h, launch_restrict_rhs(h->st, g, st));
        prof_end(h, pi, st);
    }
    mg_status rc = enqueue_tail(h, st, TL_FMG);
    if (rc != MG_OK) return rc;
    for (int l = S.lt - 1; l >= 0; --l) {
        const GenArgs g = gen_args(h, 0, l);
        const double sb = (double)state_bytes(h->st);
        const int pi = prof_begin(h, lvname("fmg_interp", S.lv[l].n),
                                  (double)(level_points(S.lv[l].n, h->dim) + level_points(S.lv[l + 1].n, h->dim)) * sb,
                                  st);
        HIPCHK(h, launch_interp(h->st, g, st));
        prof_end(h, pi, st);
        if ((rc = enqueue_visit(h, l, h->opt.cycle, true, st)) != MG_OK) return rc;
    }
    return enqueue_post_norm(h, st);
}

mg_status enqueue_cycle(mg_handle_s *h, hipStream_t st)
{
    if (h->opt.cycle != MG_CYCLE_V) {
        mg_status rc = enqueue_visit(h, 0, h->opt.cycle, false, st);
        if (rc != MG_OK) return rc;
        return enqueue_post_norm(h, st);
    }
    // the distinct level sizes above the tail, finest first (fixed at setup)
    std::vector<int> &sizes = h->level_sizes;
    if (sizes.empty()) {
        for (auto &S : h->sys)
            for (int l = 0; l < S.lt; ++l) sizes.push_back(S.lv[l].n);
        std::sort(sizes.begin(), sizes.end(), [](int x, int y) { return x > y; });
        sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    }
    mg_status rc;
    // ---- down
    for (int n : sizes) {
        for (int s = 0; s < h->nsys; ++s) {
            Sys &S = h->sys[s];
            for (int l = 0; l < S.lt; ++l)
                if (S.lv[l].n == n && !S.lv[l].march && (rc = enqueue_generic_down(h, s, l, st)) != MG_OK) return rc;
        }
        for (auto &g : h->groups)
            if (g.n == n && (rc = enqueue_march(h, g, false, st)) != MG_OK) return rc;
    }
    // ---- tail
    if ((rc = enqueue_tail(h, st, -1)) != MG_OK) return rc;
    // ---- up
    for (auto it = sizes.rbegin(); it != sizes.rend(); ++it) {
        const int n = *it;
        for (auto g = h->groups.rbegin(); g != h->groups.rend(); ++g)
            if (g->n == n && (rc = enqueue_march(h, *g, true, st)) != MG_OK) return rc;
        for (int s = 0; s < h->nsys; ++s) {
            Sys &S = h->sys[s];
            for (int l = S.lt - 1; l >= 0; --l)
                if (S.lv[l].n == n && !S.lv[l].march && (rc = enqueue_generic_up(h, s, l, st)) != MG_OK) return rc;
        }
    }
    return enqueue_post_norm(h, st);
}

// Residual norm of the FP64 problem on every system, with the stop test.
// IR: also writes the FP32 inner rhs.  first: measures ||f|| too.
mg_status enqueue_outer_norm(mg_handle_s *h, int first, bool write_r32, hipStream_t st, bool u_zero = false)
{
    if (h->nsys == 1 && !h->batch) {
        Sys &S = h->sys[0];
        NormArgs a;
        std::memset(&a, 0, sizeof(a));
        a.dim = h->dim;
        a.n = S.n;
        a.pitch = S.pitch0;
        a.ppitch = S.ppitch0;
        a.inv_h2 = (double)(S.n + 1) * (S.n + 1);
        a.u = u_zero ? nullptr : S.u;  // (null: the iterate is zero, only f is read)
        a.f = S.f;
        a.a = h->vc ? S.a64 : nullptr;
        a.r32 = write_r32 ? S.r32 : nullptr;
        a.state = h->d_states;
        a.partials = h->d_partials;
        a.nblocks = h->norm_blocks;
        a.first = first;
        const double pts = (double)level_points(S.n, h->dim);
        const int pi = prof_begin(h, "norm", pts * ((u_zero ? 8 : 16) + (h->vc ? 8 : 0) + (write_r32 ? 4 : 0)), st);
        HIPCHK(h, launch_norm(a, st));
        prof_end(h, pi, st);
        const int pf = prof_begin(h, "norm_finish", 0.0, st);
        HIPCHK(h, launch_norm_finish(h->d_states, 1, h->d_partials, nullptr, nullptr, 0, h->norm_blocks, first, st));
        prof_end(h, pf, st);
        return MG_OK;
    }
    double pts = 0;
    for (auto &S : h->sys) pts += (double)level_points(S.n, h->dim);
    const int pi = prof_begin(h, "norm", pts * (16 + (h->vc ? 8 : 0) + (write_r32 ? 4 : 0)), st);
    HIPCHK(h, launch_norm_batch(h->d_nitems, h->nnitems, h->d_nsys, h->d_states, h->d_partials,
                                first | (write_r32 ? 2 : 0), st));
    prof_end(h, pi, st);
    const int pf = prof_begin(h, "norm_finish", 0.0, st);
    HIPCHK(h, launch_norm_finish(h->d_states, h->nsys, h->d_partials, h->d_npart0, h->d_nnparts, 0, 0, first, st));
    prof_end(h, pf, st);
    return MG_OK;
}

// Plain mode: the cycle's own norm (fused into the finest POST when the
// finest level marches, else a norm kernel).
mg_status enqueue_plain_cycle(mg_handle_s *h, hipStream_t st)
{
    mg_status rc = enqueue_cycle(h, st);
    if (rc != MG_OK) return rc;
    if (!h->sys[0].lv[0].march && !m3_norm_fused(h)) return enqueue_outer_norm(h, 0, false, st);
    return MG_OK;
}

// IR mode: inner cycle (which adds e into u) then the outer residual.
mg_status enqueue_ir_step(mg_handle_s *h, hipStream_t st)
{
    mg_status rc = enqueue_cycle(h, st);
    if (rc != MG_OK) return rc;
    for (int s = 0; s < h->nsys; ++s) {
        Sys &S = h->sys[s];
        if (!S.lv[0].march && !(h->m3 && S.lt > 0)) {
            HIPCHK(h, launch_ir_correct(h->st, S.u, S.pitch0, S.ppitch0, S.lv[0].B, S.n, h->dim, h->d_states + s, st));
        }
    }
    return enqueue_outer_norm(h, 0, true, st);
}

mg_status enqueue_step(mg_handle_s *h, hipStream_t st)
{
    return h->ir ? enqueue_ir_step(h, st) : enqueue_plain_cycle(h, st);
}

// Plain mode: the full-multigrid first step with its residual norm.
mg_status enqueue_fmg_step(mg_handle_s *h, hipStream_t st)
{
    mg_status rc = enqueue_fmg(h, st);
    if (rc != MG_OK) return rc;
    if (!h->sys[0].lv[0].march && !m3_norm_fused(h)) return enqueue_outer_norm(h, 0, false, st);
    return MG_OK;
}

__global__ void k_state_init(SolveState *st, int nsys, double tol, int maxc, double watch, double stall)
{
    for (int s = threadIdx.x + blockIdx.x * blockDim.x; s < nsys; s += blockDim.x * gridDim.x) {
        st[s].done = 0;
        st[s].nres = 0;
        st[s].counter = 0u;
        st[s].maxc = maxc;
        st[s].tol = tol;
        st[s].watch = watch;
        st[s].stall = stall;
        st[s].ff = 0.0;
        st[s].rel = 0.0;
    }
}

// Resume systems stopped by the ratio watch (done == 4) or by a bf16-state
// stall (done == 5), with both rules off.
__global__ void k_state_rearm(SolveState *st, int nsys)
{
    for (int s = threadIdx.x + blockIdx.x * blockDim.x; s < nsys; s += blockDim.x * gridDim.x) {
        if (st[s].done == 4 || st[s].done == 5) st[s].done = 0;
        st[s].watch = 0.0;
        st[s].stall = 0.0;
    }
}

// The learned smoother runs under the ratio watch: the cycle after which the
// residual fell by less than kLearnedFallback stops the chunk on the device.
mg_status state_init(mg_handle_s *h, double tol, int maxc, hipStream_t st)
{
    const double watch = (h->learned && h->learned_on) ? kLearnedFallback : 0.0;
    const double stall = (h->st == ST_BF16 && tol >= 0.0) ? bf16_stall_ratio() : 0.0;
    hipLaunchKernelGGL(k_state_init, dim3((h->nsys + 255) / 256), dim3(256), 0, st, h->d_states, h->nsys, tol, maxc,
                       watch, stall);
    HIPCHK(h, hipGetLastError());
    return MG_OK;
}

mg_status build_graph(mg_handle_s *h)
{
    if (h->gexec) {
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
    if (h->graph) {
        (void)hipGraphDestroy(h->graph);
        h->graph = nullptr;
    }
    HIPCHK(h, hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal));
    mg_status rc = enqueue_step(h, h->capture);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->capture, &g);
    if (rc != MG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) {
        h->err = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
        return MG_ERR_HIP;
    }
    h->graph = g;
    HIPCHK(h, hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0));
    h->graph_ok = true;
    return MG_OK;
}

mg_status enqueue_steps(mg_handle_s *h, int k)
{
    if (h->prof) {
        for (int i = 0; i < k; ++i) {
            mg_status rc = enqueue_step(h, h->stream);
            ++h->prof_step;
            if (rc != MG_OK) return rc;
        }
        return MG_OK;
    }
    if (h->opt.use_graph) {
        if (!h->graph_ok) {
            mg_status rc = build_graph(h);
            if (rc != MG_OK) return rc;
        }
        for (int i = 0; i < k; ++i) HIPCHK(h, hipGraphLaunch(h->gexec, h->stream));
        return MG_OK;
    }
    for (int i = 0; i < k; ++i) {
        mg_status rc = enqueue_step(h, h->stream);
        if (rc != MG_OK) return rc;
    }
    return MG_OK;
}

mg_status read_states(mg_handle_s *h)
{
    HIPCHK(h, hipMemcpyAsync(h->h_states, h->d_states, sizeof(SolveState) * h->nsys, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MG_OK;
}

void fill_stats(const SolveState &s, mg_stats *st, bool fell_back)
{
    if (!st) return;
    std::memset(st, 0, sizeof(*st));
    const int k = std::max(0, s.nres - 1);
    st->cycles = k;
    st->rel_res = s.rel;
    for (int i = 0; i <= k && i <= MG_MAX_CYCLES; ++i) st->hist[i] = s.hist[i];
    st->rho_avg = (k > 0 && s.hist[0] > 0) ? std::pow(s.rel / s.hist[0], 1.0 / k) : 0.0;
    if (k >= 3 && s.hist[k - 3] > 0) st->rho_asym = std::pow(s.hist[k] / s.hist[k - 3], 1.0 / 3.0);
    else st->rho_asym = st->rho_avg;
    st->fell_back = fell_back ? 1 : 0;
}

mg_status status_of(const SolveState &s)
{
    switch (s.done) {
    case 1: return MG_OK;
    case 2: return MG_ERR_NONFINITE;
    case 3: return MG_NOT_CONVERGED;
    case 6: return MG_ERR_DIVERGED;
    }
    return MG_NOT_CONVERGED;
}

// Upload the work lists build_schedule made (items, partial-sum slots, norm items).
mg_status upload_schedule(mg_handle_s *h)
{
    {
        std::vector<int> p0(h->nsys), np(h->nsys);
        for (int s = 0; s < h->nsys; ++s) {
            p0[s] = h->sys[s].part0;
            np[s] = h->sys[s].nparts;
        }
        if (!h->items.empty())
            HIPCHK(h, hipMemcpy(h->d_items, h->items.data(), sizeof(MarchItem) * h->items.size(), hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(h->d_part0, p0.data(), sizeof(int) * h->nsys, hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(h->d_nparts, np.data(), sizeof(int) * h->nsys, hipMemcpyHostToDevice));
        if (!h->nitemv.empty())
            HIPCHK(h, hipMemcpy(h->d_nitems, h->nitemv.data(), sizeof(NormItem) * h->nitemv.size(),
                                hipMemcpyHostToDevice));
        std::vector<int> q0(h->nsys), nq(h->nsys);
        for (int s = 0; s < h->nsys; ++s) {
            q0[s] = h->nsysv[s].part0;
            nq[s] = h->nsysv[s].nparts;
        }
        HIPCHK(h, hipMemcpy(h->d_npart0, q0.data(), sizeof(int) * h->nsys, hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(h->d_nnparts, nq.data(), sizeof(int) * h->nsys, hipMemcpyHostToDevice));
    }
    return MG_OK;
}

// Build items/groups for the march levels and the norm items; returns MG_OK.
mg_status build_schedule(mg_handle_s *h)
{
    h->items.clear();
    h->groups.clear();
    std::vector<int> part0(h->nsys, 0), nparts(h->nsys, 0);
    // distinct march sizes, descending
    std::vector<int> sizes;
    for (auto &S : h->sys)
        for (int l = 0; l < S.lt; ++l)
            if (S.lv[l].march) sizes.push_back(S.lv[l].n);
    std::sort(sizes.begin(), sizes.end(), std::greater<int>());
    sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    int partc = 0;
    const int nsweep = h->opt.nu1;
    for (int n : sizes) {
        Group g;
        g.n = n;
        g.G = env_int("MGX_G", 1);
        if (h->vc) g.G = 1;
        g.W = march_strip_width(g.G, nsweep);
        // small levels that hold no system's finest level: LDS tiles
        bool has_finest = false;
        for (auto &S : h->sys)
            if (S.lt > 0 && S.lv[0].march && S.lv[0].n == n) has_finest = true;
        g.tiled = !has_finest && n <= env_int("MGX_TILE_MAX", 1023);
        if (g.tiled) g.W = 32;
        const int strips = (n + g.W - 1) / g.W;
        // block height: enough work items to fill the device, even, 8..256
        int count = 0;
        for (auto &S : h->sys)
            for (int l = 0; l < S.lt; ++l)
                if (S.lv[l].march && S.lv[l].n == n) ++count;
        bool any_finest = false;
        for (auto &S : h->sys)
            if (S.lt > 0 && S.lv[0].n == n) any_finest = true;
        const int target = any_finest ? env_int("MGX_TARGET_ITEMS", 2048)
                                      : env_int("MGX_TARGET_ITEMS_COARSE", env_int("MGX_TARGET_ITEMS", 2048));
        const int min_hb = env_int("MGX_MIN_HB", 4);
        int hb = 256;
        while (hb > std::max(4, min_hb) && (long long)strips * ((n + hb - 1) / hb) * count < target) hb /= 2;
        hb = env_int("MGX_HB", hb);
        if (hb < 2) hb = 2;
        hb &= ~1;
        if (g.tiled) hb = 32;
        // an autotuned (or caller-set) shape for this size replaces the heuristic
        for (auto &t : h->tune) {
            if (t.first != n) continue;
            const bool can_tile = !has_finest && h->dim == 2;
            g.tiled = t.second.second != 0 && can_tile;
            if (g.tiled) {
                g.W = 32;
                hb = 32;
            } else {
                g.W = march_strip_width(g.G, nsweep);
                hb = std::max(2, std::min(256, t.second.first)) & ~1;
            }
        }
        g.Hb = hb;
        g.item0 = (int)h->items.size();
        for (int s = 0; s < h->nsys; ++s) {
            Sys &S = h->sys[s];
            for (int l = 0; l < S.lt; ++l) {
                if (!S.lv[l].march || S.lv[l].n != n) continue;
                if (l == 0) part0[s] = partc;
                for (int ja = 1; ja <= n; ja += hb)
                    for (int ia = 1; ia <= n; ia += g.W) {
                        MarchItem it;
                        it.lvl = -1;  // patched below (descriptor index)
                        it.ia = ia;
                        it.ja = ja;
                        it.part = (l == 0) ? partc++ : 0;
                        it.lvl = s * 1000 + l;  // temporary key
                        h->items.push_back(it);
                    }
                if (l == 0) nparts[s] = partc - part0[s];
            }
        }
        g.nitems = (int)h->items.size() - g.item0;
        // algorithmic bytes: every array read once, written once
        {
            const double sb = h->st == ST_F64 ? 8 : h->st == ST_F32 ? 4 : 2;
            const double fb = h->fs, ab = h->vc ? h->cs : 0;
            const int nc = (n - 1) / 2;
            for (int s2 = 0; s2 < h->nsys; ++s2) {
                const Sys &S = h->sys[s2];
                for (int l = 0; l < S.lt; ++l) {
                    if (!S.lv[l].march || S.lv[l].n != n) continue;
                    const double pts = (double)n * n, cpts = (double)nc * nc, apts = (double)(n + 2) * (n + 2);
                    const bool uz = l > 0 || h->ir;
                    g.bytes_pre += pts * ((uz ? 0 : sb) + fb + sb) + apts * ab + cpts * fb;
                    const double out = (l == 0 && h->ir) ? 16.0 : sb;
                    g.bytes_post += pts * (sb + fb + out) + apts * ab + cpts * sb;
                    if (l == 0) g.finest = true;
                }
            }
        }
        h->groups.push_back(g);
    }
    if (h->items.size() > h->items_cap) return MG_ERR_WORKSPACE;
    if (partc > h->npartials) return MG_ERR_WORKSPACE;
    // descriptor indices: systems in order, levels in order
    std::vector<int> base(h->nsys, 0);
    int acc = 0;
    for (int s = 0; s < h->nsys; ++s) {
        base[s] = acc;
        acc += (int)h->sys[s].lv.size();
    }
    for (auto &it : h->items) it.lvl = base[it.lvl / 1000] + it.lvl % 1000;
    for (int s = 0; s < h->nsys; ++s) {
        h->sys[s].part0 = part0[s];
        h->sys[s].nparts = nparts[s];
    }
    // batched outer-norm items: rows in chunks of 16
    h->nitemv.clear();
    h->nsysv.assign(h->nsys, NormSys());
    int slot = 0;
    for (int s = 0; s < h->nsys; ++s) {
        Sys &S = h->sys[s];
        NormSys &ns = h->nsysv[s];
        std::memset(&ns, 0, sizeof(ns));
        ns.n = S.n;
        ns.pitch = S.pitch0;
        ns.inv_h2 = (double)(S.n + 1) * (S.n + 1);
        ns.a = h->vc ? S.a64 : nullptr;
        ns.r32 = S.r32;
        ns.part0 = slot;
        for (int j0 = 1; j0 <= S.n; j0 += 16) {
            NormItem it{s, j0, std::min(j0 + 16, S.n + 1), slot++};
            h->nitemv.push_back(it);
        }
        ns.nparts = slot - ns.part0;
    }
    h->nnitems = (int)h->nitemv.size();
    if (slot > h->npartials) return MG_ERR_WORKSPACE;
    return MG_OK;
}

mg_status setup_common(mg_handle_s *h, const std::vector<int> &ns, const mg_grid *g, const mg_operator *op,
                       void *workspace, size_t bytes)
{
    // tail geometry (identical for every system: sizes below the tail top)
    const Sys &S0 = h->sys[0];
    h->tail_nlev = (int)S0.lv.size() - S0.lt;
    for (auto &S : h->sys)
        if ((int)S.lv.size() - S.lt != h->tail_nlev) return MG_ERR_UNSUPPORTED;
    h->tail_top = S0.lv[S0.lt].n;
    h->tail_m = ipow(S0.lv.back().n, h->dim);
    // 2D diffusion: precomputed face tables when they fit in LDS too
    const bool jac = h->opt.smoother == MG_SM_JACOBI;
    h->tail_faces = h->vc && h->dim == 2 && env_int("MGX_TAIL_FACES", 1) != 0 &&
                    tail_lds_bytes(h->st, h->dim, h->tail_top, jac, true) <= tail_max_lds();
    h->tail_lds = tail_lds_bytes(h->st, h->dim, h->tail_top, jac, h->tail_faces);
    if (h->tail_lds > tail_max_lds()) return MG_ERR_UNSUPPORTED;
    const long long top_pts = level_points(h->tail_top, h->dim);
    // the tail maps 64 threads to a 2D row and 16 x 16 threads to a 3D plane
    if (h->dim == 1) h->tail_threads = (int)std::min<long long>(1024, std::max<long long>(64, (top_pts + 63) / 64 * 64));
    else if (h->dim == 2) h->tail_threads = std::max(64, std::min(env_int("MGX_TAIL_THREADS", 1024), 64 * h->tail_top));
    else h->tail_threads = std::max(256, std::min(1024, 256 * h->tail_top));

    const size_t need = carve(h, nullptr);
    if (!workspace || bytes < need || ((uintptr_t)workspace % kAlign)) return MG_ERR_WORKSPACE;
    h->ws = (char *)workspace;
    h->ws_bytes = bytes;
    carve(h, (char *)workspace);
    if (!h->tail_ops.empty())
        HIPCHK(h, hipMemcpy(h->d_ops, h->tail_ops.data(), sizeof(int) * h->tail_ops.size(), hipMemcpyHostToDevice));
    mg_status rc = build_schedule(h);
    if (rc != MG_OK) return rc;

    // norm kernel blocks (single system)
    {
        const long long m = level_points(h->sys[0].n, h->dim);
        h->norm_blocks = (int)std::min<long long>(std::max<long long>((m + 255) / 256, 1), 2048);
        h->norm_blocks = std::min(h->norm_blocks, h->npartials);
    }
    HIPCHK(h, tail_prepare(h->st, h->vc, h->dim));
    if (h->st == ST_BF16) HIPCHK(h, tail_prepare(ST_F32, h->vc, h->dim));
    if (h->learned) HIPCHK(h, learned_prep(h->lw_master, h->lw, h->stream));

    // upload static arrays: items, part0/nparts, norm items
    rc = upload_schedule(h);
    if (rc != MG_OK) return rc;
    // coefficients: check, then inject every level (FP64 -> compute type)
    if (h->vc) {
        int *bad = h->d_flag;
        HIPCHK(h, hipMemsetAsync(bad, 0, sizeof(int), h->stream));
        for (auto &S : h->sys) HIPCHK(h, launch_coef_check(S.a64, (long long)(S.n + 2) * (S.n + 2), bad, h->stream));
        int hb = 0;
        HIPCHK(h, hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        if (hb) return MG_ERR_ARG;
        for (auto &S : h->sys) {
            for (size_t l = 0; l < S.lv.size(); ++l) {
                if (l == 0 && !h->ir) continue;  // FP64 finest: the caller's array
                HIPCHK(h, launch_coef_inject(S.a64, S.n, S.lv[l].a, S.lv[l].n, 1 << l, h->cs == 4, h->stream));
            }
            const int nc = S.lv.back().n;
            HIPCHK(h, launch_coef_inject(S.a64, S.n, S.acoarse64, nc, 1 << (S.lv.size() - 1), 0, h->stream));
        }
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    // coarsest inverse per system
    for (auto &S : h->sys) {
        const int nc = S.lv.back().n;
        std::vector<double> ahost;
        if (h->vc) {
            ahost.resize((size_t)(nc + 2) * (nc + 2));
            HIPCHK(h, hipMemcpy(ahost.data(), S.acoarse64, sizeof(double) * ahost.size(), hipMemcpyDeviceToHost));
        }
        std::vector<double> M, inv;
        coarse_matrix(h->dim, nc, h->vc ? ahost.data() : nullptr, M);
        if (!invert(h->tail_m, M, inv)) return MG_ERR_ARG;
        HIPCHK(h, hipMemcpy(S.cinv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice));
    }
    (void)g;
    (void)op;
    (void)ns;
    HIPCHK(h, hipHostMalloc((void **)&h->h_states, sizeof(SolveState) * h->nsys, hipHostMallocDefault));
    HIPCHK(h, hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking));
    return MG_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

size_t extent_bytes(int dim, int n, long long pitch, long long ppitch)
{
    long long e = n;
    if (dim > 1) e = (long long)(n - 1) * pitch + n;
    if (dim > 2) e = (long long)(n - 1) * ppitch + (long long)(n - 1) * pitch + n;
    return (size_t)e * 8;
}

mg_status bind_call(mg_handle_s *h, int s, double *u, const double *f)
{
    if (!u || !f) return MG_ERR_ARG;
    Sys &S = h->sys[s];
    const size_t ext = extent_bytes(h->dim, S.n, S.pitch0, S.ppitch0);
    if (overlaps(u, ext, f, ext)) return MG_ERR_ARG;
    if (h->vc && overlaps(u, ext, S.a64, sizeof(double) * (S.n + 2) * (S.n + 2))) return MG_ERR_ARG;
    if (h->ws && overlaps(u, ext, h->ws, h->ws_bytes)) return MG_ERR_ARG;
    S.u = u;
    S.f = f;
    return MG_OK;
}

mg_status make_handle(int nsys, const mg_grid *g, const mg_operator *op, const mg_options *o, bool batch,
                      mg_handle_s **out_h, std::vector<int> &ns)
{
    if (nsys < 1 || nsys > kMaxStates || !g) return MG_ERR_ARG;
    const int dim = g[0].dim;
    mg_options opt = normalised(o, dim);
    ns.resize(nsys);
    for (int s = 0; s < nsys; ++s) {
        if (g[s].dim != dim) return MG_ERR_ARG;
        mg_status rc = check_grid(&g[s], op ? &op[s] : nullptr, opt);
        if (rc != MG_OK) return rc;
        if (op && (op[s].kind == MG_OP_DIFFUSION) != (op[0].kind == MG_OP_DIFFUSION)) return MG_ERR_ARG;
        ns[s] = g[s].n[0];
    }
    if (batch && dim != 2) return MG_ERR_UNSUPPORTED;
    if (batch && opt.smoother == MG_SM_LEARNED) return MG_ERR_UNSUPPORTED;  // buffers sized for one system
    if (batch && (opt.cycle != MG_CYCLE_V || opt.fmg || opt.zero_start)) return MG_ERR_UNSUPPORTED;
    mg_handle_s *h = new (std::nothrow) mg_handle_s();
    if (!h) return MG_ERR_ARG;
    h->dim = dim;
    h->nsys = nsys;
    h->batch = batch;
    h->opt = opt;
    h->stream = (hipStream_t)opt.stream;
    h->vc = op && op[0].kind == MG_OP_DIFFUSION;
    h->prec = opt.precision;
    // stage schedule: skew 1 unless MGX_SKEW2 asks for the independent-stage one
    h->skew1 = env_int("MGX_SKEW2", 0) ? 0 : 4;
    h->ir = opt.precision != MG_P_F64;
    h->st = opt.precision == MG_P_F64 ? ST_F64 : opt.precision == MG_P_F32_IR ? ST_F32 : ST_BF16;
    h->cs = h->ir ? 4 : 8;
    h->fs = h->ir ? 4 : 8;
    h->learned = h->learned_on = opt.smoother == MG_SM_LEARNED;
    h->learned_unfused = h->learned && env_int("MGX_LEARNED_UNFUSED", 0) != 0;
    h->lw_master = (const float *)opt.learned;
    h->m3 = use_m3(h);
    plan(h, ns);
    for (int s = 0; s < nsys; ++s) {
        Sys &S = h->sys[s];
        S.pitch0 = (dim > 1 && g[s].pitch[1]) ? g[s].pitch[1] : S.n;
        S.ppitch0 = (dim > 2 && g[s].pitch[2]) ? g[s].pitch[2] : (long long)S.n * S.pitch0;
        S.a64 = h->vc ? op[s].a : nullptr;
        // the fused 3D passes address a plane with 32-bit byte offsets
        const long long plane_bytes = ((long long)(S.n - 1) * std::max(S.pitch0, (long long)S.n) + S.n) * 8;
        if (plane_bytes >= (1LL << 31)) h->m3 = false;
    }
    build_tail_ops(h);
    *out_h = h;
    return MG_OK;
}

void free_handle(mg_handle_s *h)
{
    if (!h) return;
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->capture) (void)hipStreamDestroy(h->capture);
    if (h->pinned) (void)hipHostFree(h->pinned);
    if (h->h_states) (void)hipHostFree(h->h_states);
    for (auto &r : h->pend) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : h->pool) (void)hipEventDestroy(e);
    delete h;
}

// The solve loop shared by single systems and batches.
mg_status solve_loop(mg_handle_s *h, double rtol, std::vector<mg_stats *> stats)
{
    if (!(rtol >= 0.0)) return MG_ERR_ARG;
    mg_status rc = refresh(h, true);
    if (rc != MG_OK) return rc;
    const int maxc = h->opt.max_cycles;
    rc = state_init(h, rtol, maxc, h->stream);
    if (rc != MG_OK) return rc;
    // zero start: the u passed in is not read.  The fused 3D plain path
    // starts its first cycle's finest pre-smoothing from zero (the first
    // post-smoothing then writes every point of u); FMG overwrites u anyway;
    // every other path zeroes u first.
    const bool zs = h->opt.zero_start != 0;
    const bool zs_head = zs && !h->opt.fmg && h->m3 && !h->ir && h->sys[0].lt > 0;
    if (zs && !zs_head && !h->opt.fmg) {
        Sys &S = h->sys[0];
        if (S.pitch0 != S.n || (h->dim == 3 && S.ppitch0 != (long long)S.n * S.n)) return MG_ERR_UNSUPPORTED;
        HIPCHK(h, launch_fill_zero(S.u, (long long)sizeof(double) * level_points(S.n, h->dim), h->stream));
    }
    h->prof_step = -1;
    rc = enqueue_outer_norm(h, 1, h->ir, h->stream, zs);
    if (rc != MG_OK) return rc;
    h->prof_step = 0;
    int enq = 0;
    if (h->opt.fmg) {
        // the first step is one full-multigrid pass (enqueued directly, not
        // part of the captured cycle)
        rc = enqueue_fmg_step(h, h->stream);
        if (rc != MG_OK) return rc;
        enq = 1;
    } else if (zs_head) {
        // the first step from zero (enqueued directly, not part of the
        // captured cycle)
        h->first_zero = true;
        rc = enqueue_step(h, h->stream);
        h->first_zero = false;
        if (rc != MG_OK) return rc;
        enq = 1;
    }
    int chunk = 2;
    bool fell_back = false;
    for (;;) {
        rc = read_states(h);
        if (rc != MG_OK) return rc;
        bool all_done = true;
        double worst_rho = 0.0, worst_rel = 0.0;
        int kmin = 1 << 30;
        for (int s = 0; s < h->nsys; ++s) {
            const SolveState &S = h->h_states[s];
            if (!S.done) {
                all_done = false;
                const int k = S.nres - 1;
                kmin = std::min(kmin, k);
                if (k >= 1 && S.hist[0] > 0) {
                    worst_rho = std::max(worst_rho, std::pow(S.rel / S.hist[0], 1.0 / k));
                    worst_rel = std::max(worst_rel, S.rel);
                }
            }
        }
        // learned smoother fallback: a learned cycle that reduces the residual
        // by less than kLearnedFallback (the device stopped the chunk right
        // after it, done == 4) or a non-finite residual (then u restarts from
        // 0) switches the rest of the solve to red-black Gauss-Seidel
        if (h->learned_on) {
            bool bad = false, restart = false;
            for (int s = 0; s < h->nsys; ++s) {
                const int d = h->h_states[s].done;
                if (d == 2) restart = bad = true;
                if (d == 4) bad = true;
            }
            if (bad) {
                h->learned_on = false;
                h->graph_ok = false;
                fell_back = true;
                if (restart) {
                    for (int s = 0; s < h->nsys; ++s) {
                        Sys &S = h->sys[s];
                        if (S.pitch0 != S.n) return MG_ERR_NONFINITE;
                        HIPCHK(h, launch_fill_zero(S.u, (long long)sizeof(double) * level_points(S.n, h->dim), h->stream));
                    }
                    rc = state_init(h, rtol, maxc, h->stream);
                    if (rc != MG_OK) return rc;
                    rc = enqueue_outer_norm(h, 1, h->ir, h->stream);
                    if (rc != MG_OK) return rc;
                    enq = 0;
                } else {
                    hipLaunchKernelGGL(k_state_rearm, dim3((h->nsys + 255) / 256), dim3(256), 0, h->stream,
                                       h->d_states, h->nsys);
                    HIPCHK(h, hipGetLastError());
                }
                continue;
            }
        }
        // bf16-state fallback: a system whose steps stalled (the device stop
        // test set done = 5 and ended the chunk) continues, with the others,
        // with an FP32-stored iterate (the buffers are sized for it)
        if (h->st == ST_BF16) {
            bool stalled = false;
            for (int s = 0; s < h->nsys; ++s) stalled = stalled || h->h_states[s].done == 5;
            if (stalled) {
                h->st = ST_F32;
                h->graph_ok = false;
                fell_back = true;
                hipLaunchKernelGGL(k_state_rearm, dim3((h->nsys + 255) / 256), dim3(256), 0, h->stream, h->d_states,
                                   h->nsys);
                HIPCHK(h, hipGetLastError());
                continue;
            }
        }
        if (all_done || enq >= maxc) break;
        if (worst_rho > 0.0 && worst_rho < 1.0 && worst_rel > 0.0) {
            const double need = std::log(std::max(rtol, 1e-300) / worst_rel) / std::log(worst_rho);
            chunk = (int)std::ceil(std::max(1.0, need));
        }
        chunk = std::max(1, std::min(chunk, 16));
        chunk = std::min(chunk, maxc - enq);
        rc = enqueue_steps(h, chunk);
        if (rc != MG_OK) return rc;
        enq += chunk;
        (void)kmin;
    }
    mg_status worst = MG_OK;
    for (int s = 0; s < h->nsys; ++s) {
        const SolveState &S = h->h_states[s];
        mg_status r = status_of(S);
        if (r == MG_OK && fell_back) r = MG_FELL_BACK;
        if (!S.done) r = MG_NOT_CONVERGED;
        if (r < 0 && (worst >= 0 || r < worst)) worst = r;
        else if (worst >= 0 && r > worst) worst = r;
        if (s < (int)stats.size() && stats[s]) fill_stats(S, stats[s], fell_back);
    }
    if (h->prof) {
        int eff = 0;
        for (int s = 0; s < h->nsys; ++s) eff = std::max(eff, h->h_states[s].nres - 1);
        prof_collect(h, eff);
        h->prof_step = -1;
    }
    if (h->opt.precision == MG_P_F32_BF16_IR) h->st = ST_BF16;  // next solve starts in bf16 again
    if (h->learned && !h->learned_on) h->graph_ok = false;
    h->learned_on = h->learned;                                   // and with the learned smoother again
    if (fell_back) h->graph_ok = false;
    return worst;
}

}  // namespace

// =============================== C-ABI =====================================

extern "C" mg_status mg_workspace_size(const mg_grid *g, const mg_operator *op, const mg_options *o, size_t *bytes)
{
    if (!bytes) return MG_ERR_ARG;
    mg_handle_s *h = nullptr;
    std::vector<int> ns;
    mg_status rc = make_handle(1, g, op, o, false, &h, ns);
    if (rc != MG_OK) return rc;
    *bytes = carve(h, nullptr);
    free_handle(h);
    return MG_OK;
}

extern "C" mg_status mg_setup(const mg_grid *g, const mg_operator *op, const mg_options *o, void *workspace,
                              size_t bytes, mg_handle *out)
{
    if (!out) return MG_ERR_ARG;
    *out = nullptr;
    mg_handle_s *h = nullptr;
    std::vector<int> ns;
    mg_status rc = make_handle(1, g, op, o, false, &h, ns);
    if (rc != MG_OK) return rc;
    rc = setup_common(h, ns, g, op, workspace, bytes);
    if (rc != MG_OK) {
        g_setup_error = h->err;
        free_handle(h);
        return rc;
    }
    *out = h;
    return MG_OK;
}

extern "C" mg_status mg_vcycle(mg_handle h, double *u, const double *f)
{
    if (!h || h->batch) return MG_ERR_ARG;
    mg_status rc = bind_call(h, 0, u, f);
    if (rc != MG_OK) return rc;
    rc = refresh(h, false);
    if (rc != MG_OK) return rc;
    rc = state_init(h, -1.0, MG_MAX_CYCLES, h->stream);
    if (rc != MG_OK) return rc;
    if (h->ir) {
        // r = f - A u (FP64 -> FP32), inner cycle, u += e
        rc = enqueue_outer_norm(h, 1, true, h->stream);
        if (rc != MG_OK) return rc;
        rc = enqueue_cycle(h, h->stream);
        if (rc != MG_OK) return rc;
        Sys &S = h->sys[0];
        if (!S.lv[0].march && !(h->m3 && S.lt > 0))
            HIPCHK(h, launch_ir_correct(h->st, S.u, S.pitch0, S.ppitch0, S.lv[0].B, S.n, h->dim, h->d_states, h->stream));
        return MG_OK;
    }
    return enqueue_cycle(h, h->stream);
}

extern "C" mg_status mg_residual_norm(mg_handle h, const double *u, const double *f, double *rel)
{
    if (!h || h->batch || !rel) return MG_ERR_ARG;
    mg_status rc = bind_call(h, 0, (double *)u, f);
    if (rc != MG_OK) return rc;
    rc = refresh(h, false);
    if (rc != MG_OK) return rc;
    rc = state_init(h, -1.0, MG_MAX_CYCLES, h->stream);
    if (rc != MG_OK) return rc;
    rc = enqueue_outer_norm(h, 1, false, h->stream);
    if (rc != MG_OK) return rc;
    rc = read_states(h);
    if (rc != MG_OK) return rc;
    *rel = h->h_states[0].rel;
    return MG_OK;
}

extern "C" mg_status mg_solve(mg_handle h, double *u, const double *f, double rtol, mg_stats *st)
{
    if (!h || h->batch) return MG_ERR_ARG;
    mg_status rc = bind_call(h, 0, u, f);
    if (rc != MG_OK) return rc;
    return solve_loop(h, rtol, {st});
}

// ---- level operations on the finest level (FP64 handles) ------------------

extern "C" mg_status mg_smooth_restrict(mg_handle h, const double *u, const double *f, double *u_out, double *fc)
{
    if (!h || h->batch || !u || !f || !u_out || !fc) return MG_ERR_ARG;
    if (h->ir || h->sys[0].lt == 0) return MG_ERR_UNSUPPORTED;
    Sys &S = h->sys[0];
    const size_t ext = extent_bytes(h->dim, S.n, S.pitch0, S.ppitch0);
    if (overlaps(u_out, ext, u, ext) || overlaps(u_out, ext, f, ext)) return MG_ERR_ARG;
    mg_status rc = bind_call(h, 0, (double *)u, f);
    if (rc != MG_OK) return rc;
    rc = refresh(h, false);
    if (rc != MG_OK) return rc;
    rc = state_init(h, -1.0, MG_MAX_CYCLES, h->stream);
    if (rc != MG_OK) return rc;
    LevelDesc d = h->descs[S.lv[0].desc];
    const Lvl &Lc = S.lv[1];
    d.fc = fc;
    d.cpitch = Lc.n;
    d.cppitch = (long long)Lc.n * Lc.n;
    if (S.lv[0].march) {
        d.A = u_out;
        d.B = (void *)u;
        d.uzero = 0;
        LevelDesc *dd = nullptr;
        HIPCHK(h, hipMalloc((void **)&dd, sizeof(LevelDesc)));
        HIPCHK(h, hipMemcpy(dd, &d, sizeof(d), hipMemcpyHostToDevice));
        const Group *grp = nullptr;
        for (auto &g : h->groups)
            if (g.n == S.n) grp = &g;
        MarchArgs a;
        std::memset(&a, 0, sizeof(a));
        std::vector<MarchItem> its(h->items.begin() + grp->item0, h->items.begin() + grp->item0 + grp->nitems);
        for (auto &it : its) it.lvl = 0;
        MarchItem *di = nullptr;
        HIPCHK(h, hipMalloc((void **)&di, sizeof(MarchItem) * its.size()));
        HIPCHK(h, hipMemcpy(di, its.data(), sizeof(MarchItem) * its.size(), hipMemcpyHostToDevice));
        a.levels = dd;
        a.items = di;
        a.nitems = (int)its.size();
        a.W = grp->W;
        a.Hb = grp->Hb;
        a.states = h->d_states;
        a.partials = h->d_partials;
        a.part0 = h->d_part0;
        a.nparts = h->d_nparts;
        HIPCHK(h, launch_march2d(0, h->st, h->vc, h->opt.nu1, grp->G, a, march_grid(a.nitems), h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        (void)hipFree(dd);
        (void)hipFree(di);
        return MG_OK;
    }
    // generic path: copy u to u_out, smooth in place, residual + restriction
    GenArgs g;
    std::memset(&g, 0, sizeof(g));
    g.L = d;
    g.state = h->d_states;
    g.omega = h->opt.omega;
    HIPCHK(h, launch_copy_state(h->st, g, u, u_out, h->stream));
    g.L.B = u_out;
    for (int k = 0; k < h->opt.nu1; ++k) {
        if (h->opt.smoother == MG_SM_JACOBI) {
            // Jacobi needs a second buffer: use level 0's A
            g.src = u_out;
            g.dst = S.lv[0].A;
            HIPCHK(h, launch_jacobi(h->st, h->vc, g, h->stream));
            HIPCHK(h, launch_copy_state(h->st, g, S.lv[0].A, u_out, h->stream));
        } else {
            for (int c = 0; c < 2; ++c) {
                g.colour = c;
                HIPCHK(h, launch_rb_half(h->st, h->vc, g, h->stream));
            }
        }
    }
    HIPCHK(h, launch_resid_restrict(h->st, h->vc, g, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MG_OK;
}

extern "C" mg_status mg_correct_smooth(mg_handle h, const double *u, const double *uc, const double *f, double *u_out)
{
    if (!h || h->batch || !u || !uc || !f || !u_out) return MG_ERR_ARG;
    if (h->ir || h->sys[0].lt == 0) return MG_ERR_UNSUPPORTED;
    Sys &S = h->sys[0];
    const size_t ext = extent_bytes(h->dim, S.n, S.pitch0, S.ppitch0);
    if (overlaps(u_out, ext, u, ext) || overlaps(u_out, ext, f, ext)) return MG_ERR_ARG;
    mg_status rc = bind_call(h, 0, u_out, f);
    if (rc != MG_OK) return rc;
    rc = refresh(h, false);
    if (rc != MG_OK) return rc;
    rc = state_init(h, -1.0, MG_MAX_CYCLES, h->stream);
    if (rc != MG_OK) return rc;
    LevelDesc d = h->descs[S.lv[0].desc];
    const Lvl &Lc = S.lv[1];
    d.Bc = uc;
    d.cpitch = Lc.n;
    d.cppitch = (long long)Lc.n * Lc.n;
    d.norm = 0;
    if (S.lv[0].march) {
        d.A = (void *)u;
        d.B = u_out;
        LevelDesc *dd = nullptr;
        HIPCHK(h, hipMalloc((void **)&dd, sizeof(LevelDesc)));
        HIPCHK(h, hipMemcpy(dd, &d, sizeof(d), hipMemcpyHostToDevice));
        const Group *grp = nullptr;
        for (auto &g : h->groups)
            if (g.n == S.n) grp = &g;
        std::vector<MarchItem> its(h->items.begin() + grp->item0, h->items.begin() + grp->item0 + grp->nitems);
        for (auto &it : its) it.lvl = 0;
        MarchItem *di = nullptr;
        HIPCHK(h, hipMalloc((void **)&di, sizeof(MarchItem) * its.size()));
        HIPCHK(h, hipMemcpy(di, its.data(), sizeof(MarchItem) * its.size(), hipMemcpyHostToDevice));
        MarchArgs a;
        std::memset(&a, 0, sizeof(a));
        a.levels = dd;
        a.items = di;
        a.nitems = (int)its.size();
        a.W = grp->W;
        a.Hb = grp->Hb;
        a.states = h->d_states;
        a.partials = h->d_partials;
        a.part0 = h->d_part0;
        a.nparts = h->d_nparts;
        HIPCHK(h, launch_march2d(1, h->st, h->vc, h->opt.nu2, grp->G, a, march_grid(a.nitems), h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        (void)hipFree(dd);
        (void)hipFree(di);
        return MG_OK;
    }
    GenArgs g;
    std::memset(&g, 0, sizeof(g));
    g.L = d;
    g.L.B = u_out;
    g.state = h->d_states;
    g.omega = h->opt.omega;
    HIPCHK(h, launch_copy_state(h->st, g, u, u_out, h->stream));
    HIPCHK(h, launch_prolong_correct(h->st, g, h->stream));
    for (int k = 0; k < h->opt.nu2; ++k) {
        if (h->opt.smoother == MG_SM_JACOBI) {
            g.src = u_out;
            g.dst = S.lv[0].A;
            HIPCHK(h, launch_jacobi(h->st, h->vc, g, h->stream));
            HIPCHK(h, launch_copy_state(h->st, g, S.lv[0].A, u_out, h->stream));
        } else {
            for (int c = 0; c < 2; ++c) {
                g.colour = c;
                HIPCHK(h, launch_rb_half(h->st, h->vc, g, h->stream));
            }
        }
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MG_OK;
}

extern "C" mg_status mg_residual(mg_handle h, const double *u, const double *f, double *r)
{
    if (!h || h->batch || !u || !f || !r) return MG_ERR_ARG;
    Sys &S = h->sys[0];
    mg_status rc = bind_call(h, 0, (double *)u, f);
    if (rc != MG_OK) return rc;
    rc = state_init(h, -1.0, MG_MAX_CYCLES, h->stream);
    if (rc != MG_OK) return rc;
    NormArgs a;
    std::memset(&a, 0, sizeof(a));
    a.dim = h->dim;
    a.n = S.n;
    a.pitch = S.pitch0;
    a.ppitch = S.ppitch0;
    a.inv_h2 = (double)(S.n + 1) * (S.n + 1);
    a.u = u;
    a.f = f;
    a.a = h->vc ? S.a64 : nullptr;
    a.r64 = r;
    a.state = h->d_states;
    a.partials = h->d_partials;
    a.nblocks = h->norm_blocks;
    a.first = 1;
    HIPCHK(h, launch_norm(a, h->stream));
    HIPCHK(h, launch_norm_finish(h->d_states, 1, h->d_partials, nullptr, nullptr, 0, h->norm_blocks, 1, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MG_OK;
}

extern "C" mg_status mg_profile(mg_handle h, int on)
{
    if (!h) return MG_ERR_ARG;
    if (on) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        prof_collect(h, -1);
        h->classes.clear();
        h->prof = true;
        h->prof_finest_only = (on == 2);
        h->level_sizes_max = 0;
        for (auto &S : h->sys) h->level_sizes_max = std::max(h->level_sizes_max, S.n);
        h->prof_step = -1;
    } else {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        prof_collect(h, 0);
        h->prof = false;
    }
    return MG_OK;
}

extern "C" mg_status mg_profile_read(mg_handle h, mg_kernel_timing *out, int max, int *count)
{
    if (!h || !count || (max > 0 && !out)) return MG_ERR_ARG;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    prof_collect(h, 0);  // records of mg_vcycle (step -1) are pending until here
    int k = 0;
    for (auto &c : h->classes) {
        if (k >= max) break;
        mg_kernel_timing &t = out[k++];
        std::memset(&t, 0, sizeof(t));
        std::strncpy(t.name, c.name.c_str(), sizeof(t.name) - 1);
        t.launches = c.launches;
        t.total_ms = c.total_ms;
        t.avg_ms = c.launches ? c.total_ms / c.launches : 0.0;
        t.bytes_per_launch = c.bytes;
    }
    *count = k;
    return MG_OK;
}

extern "C" mg_status mg_destroy(mg_handle h)
{
    if (!h) return MG_ERR_ARG;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    free_handle(h);
    return MG_OK;
}

extern "C" const char *mg_status_str(mg_status s)
{
    switch (s) {
    case MG_OK: return "ok";
    case MG_NOT_CONVERGED: return "not converged (cycle limit)";
    case MG_FELL_BACK: return "converged after falling back";
    case MG_ERR_ARG: return "invalid argument";
    case MG_ERR_UNSUPPORTED: return "unsupported combination";
    case MG_ERR_HIP: return "HIP runtime error";
    case MG_ERR_NONFINITE: return "non-finite residual";
    case MG_ERR_DIVERGED: return "diverged";
    case MG_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    }
    return "unknown status";
}

extern "C" int mg_monitor(const double *hist, int nres, int precision, double stall_ratio)
{
    const int r = history_rule(hist, nres, precision == MG_P_F32_BF16_IR ? stall_ratio : 0.0);
    return r == 2 ? MG_MONITOR_DIVERGED : r == 1 ? MG_MONITOR_FALLBACK : MG_MONITOR_CONTINUE;
}

extern "C" const char *mg_last_error(mg_handle h) { return h ? h->err.c_str() : g_setup_error.c_str(); }

// ---- batches ----------------------------------------------------------------

extern "C" mg_status mg_workspace_size_batch(int nsys, const mg_grid *g, const mg_operator *op, const mg_options *o,
                                             size_t *bytes)
{
    if (!bytes) return MG_ERR_ARG;
    mg_handle_s *h = nullptr;
    std::vector<int> ns;
    mg_status rc = make_handle(nsys, g, op, o, true, &h, ns);
    if (rc != MG_OK) return rc;
    if (!h->ir) {
        // plain batches keep the caller's arrays on the finest level
    }
    *bytes = carve(h, nullptr);
    free_handle(h);
    return MG_OK;
}

extern "C" mg_status mg_setup_batch(int nsys, const mg_grid *g, const mg_operator *op, const mg_options *o,
                                    void *workspace, size_t bytes, mg_handle *out)
{
    if (!out) return MG_ERR_ARG;
    *out = nullptr;
    mg_handle_s *h = nullptr;
    std::vector<int> ns;
    mg_status rc = make_handle(nsys, g, op, o, true, &h, ns);
    if (rc != MG_OK) return rc;
    for (auto &S : h->sys)
        if (S.lt == 0) {
            free_handle(h);
            return MG_ERR_UNSUPPORTED;
        }
    rc = setup_common(h, ns, g, op, workspace, bytes);
    if (rc != MG_OK) {
        g_setup_error = h->err;
        free_handle(h);
        return rc;
    }
    *out = h;
    return MG_OK;
}

extern "C" mg_status mg_solve_batch(mg_handle h, double *const *u, const double *const *f, double rtol, mg_stats *st)
{
    if (!h || !h->batch || !u || !f) return MG_ERR_ARG;
    for (int s = 0; s < h->nsys; ++s) {
        mg_status rc = bind_call(h, s, u[s], f[s]);
        if (rc != MG_OK) return rc;
    }
    std::vector<mg_stats *> sv(h->nsys, nullptr);
    if (st)
        for (int s = 0; s < h->nsys; ++s) sv[s] = st + s;
    return solve_loop(h, rtol, sv);
}

// ---- autotuner ---------------------------------------------------------------

namespace {

void tune_put(mg_handle_s *h, int n, int hb, int tiled)
{
    for (auto &t : h->tune)
        if (t.first == n) {
            t.second = {hb, tiled};
            return;
        }
    h->tune.push_back({n, {hb, tiled}});
}

// Times the PRE launch of every marching / tiled 2D level size with each
// candidate shape on the bound arrays and keeps the fastest (the paper's
// benchmarks pick the best block size per experiment; here the library
// measures it on the device itself).
mg_status autotune_impl(mg_handle_s *h, int reps)
{
    if (h->dim != 2 || h->groups.empty()) return MG_OK;
    reps = std::max(1, std::min(reps, 50));
    const auto saved = h->tune;  // restored, with its schedule, on any failure
    mg_status rc = refresh(h, false);
    if (rc != MG_OK) return rc;
    rc = state_init(h, -1.0, MG_MAX_CYCLES, h->stream);  // every kernel runs: no stop flag
    if (rc != MG_OK) return rc;
    struct Ev {
        hipEvent_t a = nullptr, b = nullptr;
        ~Ev()
        {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    HIPCHK(h, hipEventCreate(&ev.a));
    HIPCHK(h, hipEventCreate(&ev.b));
    const bool prof = h->prof;
    h->prof = false;
    std::vector<std::pair<int, bool>> sizes;  // (n, holds a finest level)
    for (auto &g : h->groups) sizes.push_back({g.n, g.finest});
    for (auto &sz : sizes) {
        const int n = sz.first;
        std::vector<std::pair<int, int>> cands;
        if (!sz.second && n <= 2047) cands.push_back({32, 1});
        for (int hb = 4; hb <= 256; hb *= 2)
            if (hb <= n + 1) cands.push_back({hb, 0});
        float best = 1e30f;
        std::pair<int, int> pick = cands.front();
        bool any = false;
        for (auto &c : cands) {
            tune_put(h, n, c.first, c.second);
            if (build_schedule(h) != MG_OK) continue;  // a shape the workspace cannot hold
            if ((rc = upload_schedule(h)) != MG_OK) break;
            const Group *g = nullptr;
            for (auto &gg : h->groups)
                if (gg.n == n) g = &gg;
            if (!g) continue;
            if ((rc = enqueue_march(h, *g, false, h->stream)) != MG_OK) break;  // warm-up
            hipError_t he = hipEventRecord(ev.a, h->stream);
            for (int r = 0; r < reps && rc == MG_OK && he == hipSuccess; ++r) rc = enqueue_march(h, *g, false, h->stream);
            if (rc != MG_OK) break;
            float ms = 0.f;
            if (he == hipSuccess) he = hipEventRecord(ev.b, h->stream);
            if (he == hipSuccess) he = hipEventSynchronize(ev.b);
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, ev.a, ev.b);
            if (he != hipSuccess) {
                h->err = std::string("autotune timing: ") + hipGetErrorString(he);
                rc = MG_ERR_HIP;
                break;
            }
            if (ms < best) {
                best = ms;
                pick = c;
                any = true;
            }
        }
        if (rc != MG_OK) break;
        // the fastest candidate; when none fitted, what was there before
        h->tune.erase(std::remove_if(h->tune.begin(), h->tune.end(), [&](const auto &t) { return t.first == n; }),
                      h->tune.end());
        if (any) {
            tune_put(h, n, pick.first, pick.second);
        } else {
            for (auto &t : saved)
                if (t.first == n) tune_put(h, n, t.second.first, t.second.second);
        }
    }
    h->prof = prof;
    h->graph_ok = false;
    if (rc == MG_OK && (rc = build_schedule(h)) == MG_OK) rc = upload_schedule(h);
    if (rc != MG_OK) {
        // back to the shapes the handle had, with their work lists
        h->tune = saved;
        if (build_schedule(h) == MG_OK) (void)upload_schedule(h);
        return rc;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MG_OK;
}

}  // namespace

extern "C" mg_status mg_autotune(mg_handle h, double *const *u, const double *const *f, int reps)
{
    if (!h || !u || !f) return MG_ERR_ARG;
    for (int s = 0; s < h->nsys; ++s) {
        mg_status rc = bind_call(h, s, u[s], f[s]);
        if (rc != MG_OK) return rc;
    }
    return autotune_impl(h, reps);
}

extern "C" mg_status mg_tune_get(mg_handle h, int *n, int *hb, int *tiled, int max, int *count)
{
    if (!h || !count || max < 0 || (max > 0 && (!n || !hb || !tiled))) return MG_ERR_ARG;
    int k = 0;
    for (auto &t : h->tune) {
        if (k >= max) break;
        n[k] = t.first;
        hb[k] = t.second.first;
        tiled[k] = t.second.second;
        ++k;
    }
    *count = (int)h->tune.size();
    return MG_OK;
}

extern "C" mg_status mg_tune_set(mg_handle h, int n, int hb, int tiled)
{
    if (!h || n < 1 || hb < 2 || hb > 256) return MG_ERR_ARG;
    const auto saved = h->tune;
    tune_put(h, n, hb, tiled ? 1 : 0);
    mg_status rc = build_schedule(h);
    if (rc != MG_OK) {
        // keep the handle usable: back to the previous shapes
        h->tune = saved;
        if (build_schedule(h) != MG_OK) return MG_ERR_WORKSPACE;
        return rc;
    }
    rc = upload_schedule(h);
    if (rc != MG_OK) return rc;
    h->graph_ok = false;
    return MG_OK;
}

// ---- learned smoother entry points -------------------------------------------

// Handle-free entry points report HIP failures through mg_last_error(NULL).
#define LCHK(call)                                                               \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            g_setup_error = std::string(#call) + ": " + hipGetErrorString(e_);   \
            return MG_ERR_HIP;                                                   \
        }                                                                        \
    } while (0)

// ---- the paper's fixed-iteration Jacobi benchmark ------------------------------

namespace mgx {
// k_jacobi5.hip: up to jacobi5_max_steps() iterations per launch, in -> out
hipError_t launch_jacobi5(const double *in, double *out, int rows, int cols, int steps, hipStream_t s);
int jacobi5_max_steps();
}  // namespace mgx

namespace {

// iters iterations as ceil(iters / K) launches: pass j writes out when an
// even number of passes follows it, else work, so the last pass lands in out
mg_status jacobi5_passes(const double *in, double *out, double *work, int rows, int cols, int iters, hipStream_t st)
{
    const int K = jacobi5_max_steps();
    const int passes = iters == 0 ? 1 : (iters + K - 1) / K;
    const double *src = in;
    int left = iters;
    for (int j = 0; j < passes; ++j) {
        double *dst = ((passes - 1 - j) % 2 == 0) ? out : work;
        const int steps = std::min(left, K);
        LCHK(launch_jacobi5(src, dst, rows, cols, steps, st));
        left -= steps;
        src = dst;
    }
    return MG_OK;
}

int jacobi5_npasses(int iters)
{
    const int K = jacobi5_max_steps();
    return iters == 0 ? 1 : (iters + K - 1) / K;
}

}  // namespace

extern "C" mg_status mg_jacobi5(const double *in, double *out, double *work, int rows, int cols, int iters,
                                void *stream)
{
    if (!in || !out || rows < 1 || cols < 1 || iters < 0) return MG_ERR_ARG;
    const size_t bytes = sizeof(double) * (size_t)rows * (size_t)cols;
    const int passes = jacobi5_npasses(iters);
    if (overlaps(in, bytes, out, bytes)) return MG_ERR_ARG;
    if (passes > 1 && (!work || overlaps(work, bytes, in, bytes) || overlaps(work, bytes, out, bytes)))
        return MG_ERR_ARG;
    return jacobi5_passes(in, out, work, rows, cols, iters, (hipStream_t)stream);
}

// ---- the same benchmark for callers that cannot allocate ------------------
// The work array of mg_jacobi5_static is this file-scope device array: each
// device the library runs on holds its own copy until the process ends.
// Host code reaches it only through the address hipGetSymbolAddress gives for
// the current device (the array's name is a host-side stand-in).
constexpr long long kJacobiStaticMax = MG_JACOBI5_STATIC_MAX;  // doubles: 32 MiB
static __device__ __align__(256) double scratch[kJacobiStaticMax];

namespace {

std::mutex g_scratch_mu;
std::vector<double *> g_scratch_dev;  // per device id, from hipGetSymbolAddress

// The device address of `scratch` on the current device, looked up once per
// device.
hipError_t scratch_on_current_device(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" mg_status mg_jacobi5_static(const double *in, double *out, int rows, int cols, int iters, void *stream)
{
    if (!in || !out || rows < 1 || cols < 1 || iters < 0) return MG_ERR_ARG;
    const bool need_work = jacobi5_npasses(iters) > 1;
    if (need_work && (long long)rows * (long long)cols > kJacobiStaticMax) {
        g_setup_error = "mg_jacobi5_static: rows * cols = " + std::to_string((long long)rows * cols) +
                        " exceeds the static work array of " + std::to_string(kJacobiStaticMax) + " doubles";
        return MG_ERR_WORKSPACE;
    }
    const size_t bytes = sizeof(double) * (size_t)rows * (size_t)cols;
    if (overlaps(in, bytes, out, bytes)) return MG_ERR_ARG;
    double *work = nullptr;
    if (need_work) LCHK(scratch_on_current_device(&work));
    return jacobi5_passes(in, out, work, rows, cols, iters, (hipStream_t)stream);
}

extern "C" size_t mg_learned_scratch_bytes(int batch, int patch)
{
    if (batch < 1 || patch < 3) return 0;
    return learned_train_scratch(batch, patch);
}

extern "C" mg_status mg_learned_loss_grad(const float *s, const float *e, const float *a, int B, int P, int border,
                                          const float *w, double *loss, float *grad, void *scratch, size_t bytes,
                                          void *stream)
{
    if (!s || !e || !a || !w || !grad || !loss || !scratch || B < 1 || P < 3 || border < 0 || 2 * border >= P)
        return MG_ERR_ARG;
    if (bytes < learned_train_scratch(B, P)) return MG_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    TrainBufs t = learned_carve(scratch, B, P);
    LCHK(learned_prep(w, t.d, st));
    LCHK(learned_loss_grad(s, e, a, nullptr, B, P, border, t, grad, st));
    std::vector<float> lb(B);
    LCHK(hipMemcpyAsync(lb.data(), t.lossb, sizeof(float) * B, hipMemcpyDeviceToHost, st));
    LCHK(hipStreamSynchronize(st));
    double acc = 0.0;
    for (int b = 0; b < B; ++b) acc += lb[b];
    *loss = acc / B;
    return MG_OK;
}

extern "C" mg_status mg_learned_apply(const float *s, int B, int H, int W, const float *w, float *y, void *scratch,
                                      size_t bytes, void *stream)
{
    if (!s || !w || !y || !scratch || B < 1 || H < 1 || W < 1) return MG_ERR_ARG;
    const int P = std::max(H, W);
    if (bytes < learned_train_scratch(B, P)) return MG_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    TrainBufs t = learned_carve(scratch, B, P);
    LCHK(learned_prep(w, t.d, st));
    LCHK(learned_forward(s, nullptr, B, H, W, t.d, t.x1, t.x2, t.x3, y, st));
    LCHK(hipStreamSynchronize(st));
    return MG_OK;
}

extern "C" mg_status mg_learned_train(const float *s, const float *e, const float *a, int npairs, const int *order,
                                      const mg_train_options *o, float *w, double *loss_hist, mg_train_stats *stt,
                                      void *scratch, size_t bytes, void *stream)
{
    if (!s || !e || !a || !order || !o || !w || !scratch || npairs < 1) return MG_ERR_ARG;
    const int B = o->batch, P = o->patch, border = o->border;
    if (B < 1 || P < 3 || border < 0 || 2 * border >= P || o->epochs < 1 || B > npairs) return MG_ERR_ARG;
    if (bytes < learned_train_scratch(B, P)) return MG_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    TrainBufs t = learned_carve(scratch, B, P);
    {
        int bad = -1;
        LCHK(learned_check_order(order, (long long)o->epochs * npairs, npairs, t, st));
        LCHK(hipMemcpyAsync(&bad, (int *)(t.lacc + 1), sizeof(int), hipMemcpyDeviceToHost, st));
        LCHK(hipStreamSynchronize(st));
        if (bad != 0) return MG_ERR_ARG;
    }
    LCHK(hipMemsetAsync(t.m, 0, sizeof(float) * MG_LEARNED_NWEIGHTS, st));
    LCHK(hipMemsetAsync(t.v, 0, sizeof(float) * MG_LEARNED_NWEIGHTS, st));
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events()
        {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    LCHK(hipEventCreate(&ev.a));
    LCHK(hipEventCreate(&ev.b));
    LCHK(hipEventRecord(ev.a, st));
    const int nb = npairs / B;
    int step = 0;
    double first = 0.0, last = 0.0;
    for (int ep = 0; ep < o->epochs; ++ep) {
        for (int bi = 0; bi < nb; ++bi) {
            const int *idx = order + (size_t)ep * npairs + (size_t)bi * B;
            LCHK(learned_prep(w, t.d, st));
            LCHK(learned_loss_grad(s, e, a, idx, B, P, border, t, t.g, st));
            LCHK(learned_loss_accumulate(t, B, bi == 0, st));
            ++step;
            LCHK(learned_adam(w, t.g, t.m, t.v, step, (float)o->lr, (float)o->beta1, (float)o->beta2, (float)o->eps, st));
        }
        double acc = 0.0;
        LCHK(hipMemcpyAsync(&acc, t.lacc, sizeof(double), hipMemcpyDeviceToHost, st));
        LCHK(hipStreamSynchronize(st));
        acc /= (double)nb * B;
        if (loss_hist) loss_hist[ep] = acc;
        if (ep == 0) first = acc;
        last = acc;
    }
    LCHK(hipEventRecord(ev.b, st));
    LCHK(hipEventSynchronize(ev.b));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev.a, ev.b);
    if (stt) {
        stt->steps = step;
        stt->loss_first_epoch = first;
        stt->loss_last_epoch = last;
        stt->ms = ms;
    }
    return MG_OK;
}

extern "C" mg_status mg_learned_step(const void *e, void *e_out, const float *f, const float *a, int n, int precision,
                                     const float *w, void *scratch, size_t bytes, void *stream)
{
    if (!e || !e_out || !f || !a || !w || !scratch || n < 1) return MG_ERR_ARG;
    if (precision != MG_P_F32_IR && precision != MG_P_F32_BF16_IR) return MG_ERR_ARG;
    // the step reads its arrays through buffer descriptors (32-bit byte counts)
    if ((long long)(n + 2) * (n + 2) * 4 >= (1LL << 32) - 16) return MG_ERR_UNSUPPORTED;
    if (bytes < learned_train_scratch(1, 3)) return MG_ERR_WORKSPACE;
    const size_t eb = (size_t)n * n * (precision == MG_P_F32_IR ? 4 : 2);
    // e_out is written while other workgroups still read e, f, a and the
    // weights' copies in the scratch
    if (overlaps(e, eb, e_out, eb) || overlaps(f, (size_t)n * n * 4, e_out, eb) ||
        overlaps(a, (size_t)(n + 2) * (n + 2) * 4, e_out, eb) || overlaps(scratch, bytes, e_out, eb))
        return MG_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    TrainBufs t = learned_carve(scratch, 1, 3);
    const double h = 1.0 / (n + 1);
    LCHK(learned_prep(w, t.d, st));
    LCHK(learned_step_fused(precision == MG_P_F32_IR ? ST_F32 : ST_BF16, e, e_out, f, a, n, h * h, t.d, st));
    LCHK(hipStreamSynchronize(st));
    return MG_OK;
}

extern "C" mg_status mg_learned_crop(const double *s, const double *ustar, const double *uk, const double *a, int n,
                                     const int *y0, const int *x0, int ncrops, int P, float *S, float *E, float *A,
                                     void *stream)
{
    if (!s || !ustar || !uk || !a || !y0 || !x0 || !S || !E || !A || n < 1 || P < 1 || P > n || ncrops < 0)
        return MG_ERR_ARG;
    LCHK(learned_crop(s, ustar, uk, a, n, y0, x0, ncrops, P, S, E, A, (hipStream_t)stream));
    return MG_OK;
}

extern "C" mg_status mg_scaled_residual(mg_handle h, const double *u, const double *f, double *s)
{
    if (!h || h->batch || !u || !f || !s || h->dim != 2) return MG_ERR_ARG;
    Sys &S = h->sys[0];
    HIPCHK(h, launch_scaled_residual64(u, f, h->vc ? S.a64 : nullptr, S.n, S.pitch0, s, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MG_OK;
}

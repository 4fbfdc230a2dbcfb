// rvea_host.hip -- the C ABI of include/rvea.h: argument checks, workspace
// layout inside the caller's device buffer, launch sequencing, state access
// and per-kernel event timing.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "rvea.h"
#include "rvea_dev.h"
#include "rvea_internal.h"

using namespace rvea;

namespace {

constexpr int kKernels = 5;  // timed kernel ids: offspring, assoc, rerank, gamma, rollout
constexpr int kLqFloats = 32 * 32 + 32 * 8 + kPolicyE * 32;  // A, B, x0 of the policy problem

enum Buf {
    B_X, B_SLOT, B_OFF, B_VALID, B_FM, B_MVALID, B_PARENTS, B_VS,
    B_NVALID, B_STAMP, B_V0, B_V, B_V32, B_VN, B_GAMMA, B_ZBITS, B_RBITS, B_PMAX, B_PMASK,
    B_ASSOC, B_APD, B_KEY, B_SURV, B_TDONE, B_COUNTERS, B_VCHANGED, B_BCOUNT, B_FREECNT, B_PEN,
    B_NDONE, B_LQ, B_GPART, B_VEL,
    B_GR, B_GCELL, B_GCNT, B_GSTART, B_GNUM, B_GVEC, B_GVH, B_LCNT, B_LSTART, B_GTOT,
    B_LREC, B_LIDX, B_COUNT
};

struct Layout {
    int ld, stride, KC, CS, osplit;
    int gG;        // index grid side (0: none)
    int64_t gcap;  // index list records
    size_t off[B_COUNT];
    size_t total;
};

int64_t binomial(int64_t n, int64_t k)
{
    if (k < 0 || n < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    int64_t r = 1;
    for (int64_t i = 1; i <= k; ++i) {
        r = r * (n - k + i) / i;
        if (r > ((int64_t)1 << 40)) return -1;
    }
    return r;
}

int find_H(int m, int64_t K)
{
    for (int h = 1; h < (1 << 24); ++h) {
        const int64_t c = binomial((int64_t)h + m - 1, m - 1);
        if (c == K) return h;
        if (c < 0 || c > K) return 0;
    }
    return 0;
}

rvea_status check_args(int problem, int m, int d, int64_t N, int64_t K, const rvea_params &p)
{
    if (problem == kPolicy) {
        if (m != 2 || d != kPolicyD) return RVEA_EINVAL;
    } else if (problem < 1 || problem > 3) {
        return RVEA_EINVAL;
    }
    if (m < 2 || m > kMaxM || d < m || d > (1 << 26)) return RVEA_EINVAL;
    if (K < 1 || K > (int64_t)1 << 27 || N < 1 || N > K) return RVEA_EINVAL;
    if (find_H(m, K) == 0) return RVEA_EINVAL;
    if (!(p.alpha >= 0) || !(p.fr > 0) || p.t_max < 1) return RVEA_EINVAL;
    switch (p.op) {  // the operator's parameters (rvea.h); unused ones must be 0
    case OP_DE:
        if (!(p.op_a >= 0 && p.op_a <= 2) || !(p.op_b >= 0 && p.op_b <= 1)) return RVEA_EINVAL;
        break;
    case OP_PSO:
        if (!(p.op_a >= 0 && p.op_a <= 1) || !(p.op_b >= 0 && p.op_b <= 4)) return RVEA_EINVAL;
        break;
    case OP_GA:
    case OP_CSO:
    case OP_RAND:
        if (p.op_a != 0.0 || p.op_b != 0.0) return RVEA_EINVAL;
        break;
    default: return RVEA_EINVAL;
    }
    if (!(p.eta_c >= 0) || !(p.eta_m >= 0) || !(p.p_c >= 0 && p.p_c <= 1)) return RVEA_EINVAL;
    if (!(p.p_m >= 0 && p.p_m <= 4)) return RVEA_EINVAL;
    if (!(p.lb < p.ub) || !std::isfinite(p.lb) || !std::isfinite(p.ub)) return RVEA_EINVAL;
    return RVEA_OK;
}

bool swarm(int op) { return op == OP_PSO || op == OP_CSO; }

void make_layout(int problem, int m, int d, int64_t N, int64_t K, int op, Layout &L)
{
    const int64_t M = K + N;
    L.ld = (d + 31) / 32 * 32;
    L.stride = m <= 4 ? 4 : 8;
    // association grid: enough (row block x vector chunk) workgroups to fill
    // the 256 CUs several times over, chunks of at most 32 tiles
    const int64_t nbi = (M + assoc_rows_per_block() - 1) / assoc_rows_per_block();
    int64_t kc0 = (2048 + nbi - 1) / nbi;
    if (kc0 < 1) kc0 = 1;
    int64_t cs = (K + kc0 - 1) / kc0;
    cs = (cs + kTile - 1) / kTile * kTile;
    cs = std::min<int64_t>(std::max<int64_t>(cs, kTile), 32 * kTile);
    L.CS = (int)cs;
    L.KC = (int)((K + cs - 1) / cs);
    const int64_t P = (N + 1) / 2;
    L.osplit = op == OP_GA ? offspring_splits(d, N) : 1;
    // index of the vectors: for three objectives G x G cells, G = sqrt(K)
    // (about two vectors per cell inside the simplex), each with a slot of
    // grid_slot() list records (the lists average about eight); for two a
    // line of G = K cells, no lists
    L.gG = grid_side(m, K);
    const size_t cells = (size_t)index_cells(m, L.gG);
    L.gcap = m == 3 ? (int64_t)grid_slot() * (int64_t)cells : 0;
    const size_t sz[] = {
        (size_t)(K + N) * L.ld * 4, (size_t)2 * K * 4, (size_t)N * 4, (size_t)2 * K,
        (size_t)2 * M * m * 4, (size_t)M,
        (size_t)P * 2 * 4, (size_t)K * 8, 4, (size_t)(K + N) * 4, (size_t)K * m * 8,
        (size_t)K * m * 8, (size_t)K * L.stride * 4, (size_t)K * 8, (size_t)K * 8,
        (size_t)2 * m * 4, (size_t)2 * m * 4, (size_t)L.KC * M * 4, (size_t)L.KC * M * 4,
        (size_t)M * 4, (size_t)M * 8, (size_t)K * 8, (size_t)K * 4, 8, 3 * 8, 4,
        (size_t)((K + N + 255) / 256) * 4, 4, 8, 4,
        problem == kPolicy ? (size_t)kLqFloats * 4 : 0,
        L.osplit > 1 ? (size_t)P * L.osplit * 2 * 8 : 8,
        swarm(op) ? (size_t)(K + N) * L.ld * 4 : 8,
        (size_t)m * 8, (size_t)K * 4, cells * 4, cells * 4, cells * 4, (size_t)K * 4,
        (size_t)K * 32, cells * 4, cells * 4, 32, (size_t)L.gcap * 32, (size_t)L.gcap * 4};
    static_assert(sizeof(sz) / sizeof(sz[0]) == B_COUNT, "one size per buffer");
    size_t o = 0;
    for (int b = 0; b < B_COUNT; ++b) {
        L.off[b] = o;
        o += (sz[b] + 255) / 256 * 256;
    }
    L.total = o;
}

}  // namespace

struct rvea_run_s {
    RunView R;
    Layout L;
    hipStream_t stream;
    int device;
    int H;
    int64_t t;  // completed generations (host mirror)
    int phase;  // 0 ready, 1 stepped, 2 selected
    bool has_selection;
    rvea_params params;
    char err[512];
    int timing;  // kernel mask
    struct Ev {
        int id;
        hipEvent_t a, b;
    };
    std::vector<Ev> events;
    std::vector<hipEvent_t> pool;
    // captured runs of consecutive generations, keyed by their length and
    // which of them adapt (bit k: the k-th generation of the run)
    struct Graph {
        int len;
        uint64_t adapt;
        hipGraph_t g;
        hipGraphExec_t x;
    };
    hipStream_t cap_stream = nullptr;
    std::vector<Graph> graphs;
    bool use_graphs = true;
    rvea_batch batch = nullptr;  // non-null while admitted to a batch
};

struct rvea_batch_s {
    int max_runs;
    hipStream_t stream;
    RunView *d_runs;    // max_runs views, device
    RunView *d_gruns;   // the same views with the gamma pass's vector chunks, device
    Span *d_spans;      // BP_COUNT * max_runs spans, device
    std::vector<rvea_run> runs;
    struct Launch {
        int phase, cls;
        int64_t span_off;
        int n;
        int64_t blocks;
    };
    std::vector<Launch> plan;
    bool dirty = true;
    int64_t version = 0, graph_version = -1, last_step_version = -1;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool use_graphs = true;
    char err[512] = "";
};

namespace {

// the index's scaling before any adaptation (and after a host-set V)
const double kUnitScale[3] = {1.0, 1.0, 1.0};

// message of the last failed rvea_create on this thread (no handle exists)
thread_local char g_create_err[512] = "";

}  // namespace

// the thread's message for calls without a handle (rvea_create, indicators)
void rvea::note_thread_error(const char *what, hipError_t e)
{
    std::snprintf(g_create_err, sizeof g_create_err, "%s: %s", what, hipGetErrorString(e));
}

void rvea::note_thread_message(const char *msg)
{
    std::snprintf(g_create_err, sizeof g_create_err, "%s", msg);
}

namespace {

rvea_status fail(rvea_run r, hipError_t e, const char *what)
{
    if (r) std::snprintf(r->err, sizeof r->err, "%s: %s", what, hipGetErrorString(e));
    return RVEA_EDEVICE;
}

#define HIPCHK(r, call)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return fail(r, e_, #call);                                     \
    } while (0)

hipEvent_t take_event(rvea_run r)
{
    if (!r->pool.empty()) {
        hipEvent_t e = r->pool.back();
        r->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// two events from the run's pool, handed back when the holder goes out of
// scope unless keep() passed them on
struct EventPair {
    rvea_run r;
    hipEvent_t a, b;
    explicit EventPair(rvea_run r_) : r(r_), a(take_event(r_)), b(take_event(r_)) {}
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
    ~EventPair()
    {
        if (a) r->pool.push_back(a);
        if (b) r->pool.push_back(b);
    }
    bool ok() const { return a && b; }
    void keep() { a = b = nullptr; }
};

// launches fn; when timing is on, brackets it with events on the run's stream
template <class Fn>
rvea_status timed(rvea_run r, int id, Fn fn, const char *what)
{
    if (!((r->timing >> id) & 1)) {
        hipError_t e = fn();
        return e == hipSuccess ? RVEA_OK : fail(r, e, what);
    }
    EventPair ev(r);
    if (ev.ok()) HIPCHK(r, hipEventRecord(ev.a, r->stream));
    hipError_t e = fn();
    if (e != hipSuccess) return fail(r, e, what);
    if (ev.ok()) {
        HIPCHK(r, hipEventRecord(ev.b, r->stream));
        r->events.push_back({id, ev.a, ev.b});
        ev.keep();
    }
    return RVEA_OK;
}

rvea_status check_counters(rvea_run r)
{
    unsigned long long c[3];
    HIPCHK(r, hipMemcpy(c, r->R.counters, sizeof c, hipMemcpyDeviceToHost));
    if (c[2] != 0) {
        std::snprintf(r->err, sizeof r->err,
                      "a child drew more than %d mutation sites; lower p_m", kMaxSites);
        return RVEA_EUNSUPPORTED;
    }
    return RVEA_OK;
}

}  // namespace

extern "C" {

rvea_status rvea_default_params(rvea_params *out)
{
    if (!out) return RVEA_EINVAL;
    out->alpha = 2.0;
    out->fr = 0.1;
    out->t_max = 100;
    out->op = OP_GA;
    out->eta_c = 20.0;
    out->eta_m = 20.0;
    out->p_c = 1.0;
    out->p_m = 1.0;
    out->lb = 0.0;
    out->ub = 1.0;
    out->op_a = 0.0;
    out->op_b = 0.0;
    return RVEA_OK;
}

rvea_status rvea_operator_params(int op, rvea_params *p)
{
    if (!p) return RVEA_EINVAL;
    switch (op) {
    case OP_GA: case OP_CSO: case OP_RAND: p->op_a = 0.0; p->op_b = 0.0; break;
    case OP_DE: p->op_a = 0.5; p->op_b = 0.9; break;   // F, CR
    case OP_PSO: p->op_a = 0.5; p->op_b = 1.5; break;  // w, c
    default: return RVEA_EINVAL;
    }
    p->op = op;
    return RVEA_OK;
}

rvea_status rvea_lattice_divisions(int m, int64_t K, int *H)
{
    if (!H || m < 1 || K < 1) return RVEA_EINVAL;
    const int h = find_H(m, K);
    if (h == 0) return RVEA_EINVAL;
    *H = h;
    return RVEA_OK;
}

rvea_status rvea_footprint(int problem, int m, int d, int64_t N, int64_t K,
                           const rvea_params *params, size_t *bytes)
{
    rvea_params p;
    if (params) p = *params; else rvea_default_params(&p);
    if (!bytes) return RVEA_EINVAL;
    const rvea_status st = check_args(problem, m, d, N, K, p);
    if (st != RVEA_OK) return st;
    Layout L;
    make_layout(problem, m, d, N, K, p.op, L);
    *bytes = L.total;
    return RVEA_OK;
}

}  // extern "C"

namespace {

rvea_status create_run(int problem, int m, int d, int64_t N, int64_t K, uint64_t seed,
                       const rvea_params *params, const rvea_lq_system *sys, void *workspace,
                       size_t workspace_bytes, void *hip_stream, rvea_run *out)
{
    if (!out) return RVEA_EINVAL;
    *out = nullptr;
    rvea_params p;
    if (params) p = *params; else rvea_default_params(&p);
    rvea_status st = check_args(problem, m, d, N, K, p);
    if (st != RVEA_OK) return st;
    if (!workspace || ((uintptr_t)workspace & 255u)) return RVEA_EINVAL;
    if (problem == kPolicy) {
        if (!sys || !sys->A || !sys->B || !sys->x0 || sys->T < 1 || !(sys->init_sigma > 0) ||
            !std::isfinite(sys->init_sigma))
            return RVEA_EINVAL;
        if (sys->E != kPolicyE) {
            std::snprintf(g_create_err, sizeof g_create_err,
                          "the policy rollouts run %d start states per individual", kPolicyE);
            return RVEA_EUNSUPPORTED;
        }
    }
    Layout L;
    make_layout(problem, m, d, N, K, p.op, L);
    if (workspace_bytes < L.total) return RVEA_ENOMEM;

    rvea_run r = new rvea_run_s();
    r->L = L;
    r->stream = (hipStream_t)hip_stream;
    r->H = find_H(m, K);
    r->t = 0;
    r->phase = 0;
    r->has_selection = false;
    r->params = p;
    r->err[0] = 0;
    r->timing = 0;
    if (hipGetDevice(&r->device) != hipSuccess) r->device = 0;

    RunView &R = r->R;
    std::memset(&R, 0, sizeof R);
    R.m = m;
    R.d = d;
    R.ld = L.ld;
    R.problem = problem;
    R.N = N;
    R.K = K;
    R.M = K + N;
    R.key0 = (uint32_t)seed;
    R.key1 = (uint32_t)(seed >> 32);
    R.t_max = p.t_max;
    {
        const double x = p.fr * (double)p.t_max;
        double c = std::ceil(x - 1e-9 * (x > 1.0 ? x : 1.0));
        R.period = c < 1.0 ? 1 : (int)c;
    }
    R.alpha = p.alpha;
    R.eta_c = p.eta_c;
    R.eta_m = p.eta_m;
    R.p_c = p.p_c;
    R.p_m = p.p_m;
    R.lb = p.lb;
    R.ub = p.ub;
    R.KC = L.KC;
    R.CS = L.CS;
    R.rr = 4;
    R.rk = default_rerank_rows(K + N);
    R.gKC = L.KC;
    R.gCS = L.CS;
    R.grr = 4;
    char *w = (char *)workspace;
    R.X = (float *)(w + L.off[B_X]);
    R.slot_rows = (int32_t *)(w + L.off[B_SLOT]);
    R.off_row = (int32_t *)(w + L.off[B_OFF]);
    R.valids = (uint8_t *)(w + L.off[B_VALID]);
    R.Fms = (float *)(w + L.off[B_FM]);
    R.mvalid = (uint8_t *)(w + L.off[B_MVALID]);
    R.parents = (int32_t *)(w + L.off[B_PARENTS]);
    R.osplit = L.osplit;
    R.gpart = (double *)(w + L.off[B_GPART]);
    R.op = p.op;
    R.op_a = p.op_a;
    R.op_b = p.op_b;
    R.Vel = swarm(p.op) ? (float *)(w + L.off[B_VEL]) : nullptr;
    R.gG = L.gG;
    R.gcap = L.gcap;
    if (L.gG > 0) {
        R.gr = (double *)(w + L.off[B_GR]);
        R.gcell = (int32_t *)(w + L.off[B_GCELL]);
        R.gcnt = (int32_t *)(w + L.off[B_GCNT]);
        R.gstart = (int32_t *)(w + L.off[B_GSTART]);
        R.gnum = (int32_t *)(w + L.off[B_GNUM]);
        R.gvec = (int32_t *)(w + L.off[B_GVEC]);
        R.gvh = (double *)(w + L.off[B_GVH]);
        R.lcnt = (int32_t *)(w + L.off[B_LCNT]);
        R.lstart = (int32_t *)(w + L.off[B_LSTART]);
        R.gtot = (unsigned long long *)(w + L.off[B_GTOT]);
        R.lrec = (double *)(w + L.off[B_LREC]);
        R.lidx = (int32_t *)(w + L.off[B_LIDX]);
    }
    R.vs = (int32_t *)(w + L.off[B_VS]);
    R.nvalid = (int32_t *)(w + L.off[B_NVALID]);
    R.stamp = (int32_t *)(w + L.off[B_STAMP]);
    R.bcount = (int32_t *)(w + L.off[B_BCOUNT]);
    R.freecnt = (int32_t *)(w + L.off[B_FREECNT]);
    R.pen = (double *)(w + L.off[B_PEN]);
    R.V0 = (double *)(w + L.off[B_V0]);
    R.V = (double *)(w + L.off[B_V]);
    R.V32 = (float *)(w + L.off[B_V32]);
    R.vn = (double *)(w + L.off[B_VN]);
    R.gamma = (double *)(w + L.off[B_GAMMA]);
    R.zbits = (uint32_t *)(w + L.off[B_ZBITS]);
    R.rbits = (uint32_t *)(w + L.off[B_RBITS]);
    R.pmax = (float *)(w + L.off[B_PMAX]);
    R.pmask = (uint32_t *)(w + L.off[B_PMASK]);
    R.assoc = (int32_t *)(w + L.off[B_ASSOC]);
    R.apd = (double *)(w + L.off[B_APD]);
    R.key = (unsigned long long *)(w + L.off[B_KEY]);
    R.surv = (int32_t *)(w + L.off[B_SURV]);
    R.kb = 1;
    while (((int64_t)1 << R.kb) <= R.M) ++R.kb;  // row indices below 2^kb
    R.ndone = (uint32_t *)(w + L.off[B_NDONE]);
    R.t_done = (int64_t *)(w + L.off[B_TDONE]);
    R.counters = (unsigned long long *)(w + L.off[B_COUNTERS]);
    R.vchanged = (int32_t *)(w + L.off[B_VCHANGED]);
    hipError_t e = hipMemsetAsync(R.zbits, 0xff, (size_t)2 * m * 4, r->stream);
    if (e == hipSuccess && problem == kPolicy) {
        float *lq = (float *)(w + L.off[B_LQ]);
        R.lq = lq;
        R.lq_E = sys->E;
        R.lq_T = sys->T;
        R.lq_sigma = sys->init_sigma;
        e = hipMemcpyAsync(lq, sys->A, 1024 * 4, hipMemcpyHostToDevice, r->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(lq + 1024, sys->B, 256 * 4, hipMemcpyHostToDevice, r->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(lq + 1280, sys->x0, (size_t)kPolicyE * 32 * 4,
                               hipMemcpyHostToDevice, r->stream);
        // the caller may free the host arrays once this returns
        if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    }

    if (e == hipSuccess)
        e = hipMemsetAsync(R.counters, 0, 3 * sizeof(unsigned long long), r->stream);
    if (e == hipSuccess) e = hipMemsetAsync(R.vchanged, 0, 4, r->stream);
    if (e == hipSuccess && R.Vel)  // every individual starts at rest
        e = hipMemsetAsync(R.Vel, 0, (size_t)(K + N) * L.ld * 4, r->stream);
    if (e == hipSuccess) e = hipMemsetAsync(R.ndone, 0, 4, r->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(R.stamp, 0xff, (size_t)(K + N) * 4, r->stream);
    if (e == hipSuccess && R.gG > 0) {  // the index starts unscaled, with no vectors counted
        e = hipMemcpyAsync(R.gr, kUnitScale, (size_t)m * sizeof(double), hipMemcpyHostToDevice,
                           r->stream);
        if (e == hipSuccess)
            e = hipMemsetAsync(R.gcnt, 0, (size_t)index_cells(m, R.gG) * 4, r->stream);
        if (e == hipSuccess) e = hipMemsetAsync(R.gtot, 0, 32, r->stream);
    }
    if (e == hipSuccess) e = launch_lattice(R, r->stream, r->H);
    if (e == hipSuccess) e = launch_gamma(R, r->stream, 1);
    if (e == hipSuccess) e = launch_grid_build(R, r->stream, 1);
    if (e == hipSuccess) e = launch_init(R, r->stream);
    if (e != hipSuccess) {
        std::snprintf(g_create_err, sizeof g_create_err, "initialization: %s (%d)",
                      hipGetErrorString(e), (int)e);
        delete r;
        return RVEA_EDEVICE;
    }
    g_create_err[0] = 0;
    *out = r;
    return RVEA_OK;
}

}  // namespace

extern "C" {

rvea_status rvea_create(int problem, int m, int d, int64_t N, int64_t K, uint64_t seed,
                        const rvea_params *params, void *workspace, size_t workspace_bytes,
                        void *hip_stream, rvea_run *out)
{
    if (problem == kPolicy) {
        std::snprintf(g_create_err, sizeof g_create_err,
                      "the policy problem is created with rvea_create_policy");
        if (out) *out = nullptr;
        return RVEA_EINVAL;
    }
    return create_run(problem, m, d, N, K, seed, params, nullptr, workspace, workspace_bytes,
                      hip_stream, out);
}

rvea_status rvea_create_policy(int64_t N, int64_t K, uint64_t seed, const rvea_params *params,
                               const rvea_lq_system *system, void *workspace,
                               size_t workspace_bytes, void *hip_stream, rvea_run *out)
{
    return create_run(kPolicy, 2, kPolicyD, N, K, seed, params, system, workspace,
                      workspace_bytes, hip_stream, out);
}

rvea_status rvea_step(rvea_run r)
{
    if (!r) return RVEA_EINVAL;
    if (r->phase != 0 || r->batch) return RVEA_ESTATE;
    HIPCHK(r, launch_prepare(r->R, r->stream));
    rvea_status st = timed(r, 0, [&] { return launch_offspring(r->R, r->stream); }, "offspring");
    if (st != RVEA_OK) return st;
    if (r->R.problem == kPolicy) {
        st = timed(r, 4, [&] { return launch_rollout(r->R, r->stream, true); }, "rollout");
        if (st != RVEA_OK) return st;
    }
    r->phase = 1;
    return RVEA_OK;
}

rvea_status rvea_select(rvea_run r)
{
    if (!r) return RVEA_EINVAL;
    if (r->phase != 1) return RVEA_ESTATE;
    rvea_status st = timed(r, 1, [&] { return launch_assoc(r->R, r->stream); }, "assoc");
    if (st != RVEA_OK) return st;
    st = timed(r, 2, [&] { return launch_rerank(r->R, r->stream); }, "rerank");
    if (st != RVEA_OK) return st;
    HIPCHK(r, launch_select_back(r->R, r->stream));
    r->t += 1;
    r->phase = 2;
    r->has_selection = true;
    return RVEA_OK;
}

rvea_status rvea_adapt(rvea_run r)
{
    if (!r) return RVEA_EINVAL;
    if (r->phase != 2) return RVEA_ESTATE;
    if (r->t % r->R.period == 0) {
        rvea_status st = timed(r, 3, [&] { return launch_adapt(r->R, r->stream); }, "adapt");
        if (st != RVEA_OK) return st;
    }
    r->phase = 0;
    return RVEA_OK;
}

namespace {

// enqueue one generation's kernels on stream s (graph capture or eager)
hipError_t enqueue_generation(const RunView &R, hipStream_t s, bool adapt)
{
    hipError_t e = launch_prepare(R, s);
    if (e == hipSuccess) e = launch_offspring(R, s);
    if (e == hipSuccess && R.problem == kPolicy) e = launch_rollout(R, s, true);
    if (e == hipSuccess) e = launch_assoc(R, s);
    if (e == hipSuccess) e = launch_rerank(R, s);
    if (e == hipSuccess) e = launch_select_back(R, s);
    if (e == hipSuccess && adapt) e = launch_adapt(R, s);
    return e;
}

constexpr int kGraphGens = 16;   // generations per graph launch at most
constexpr size_t kGraphCache = 8;  // captured graphs kept per run

void drop_graphs(rvea_run r)
{
    for (auto &g : r->graphs) {
        if (g.x) (void)hipGraphExecDestroy(g.x);
        if (g.g) (void)hipGraphDestroy(g.g);
    }
    r->graphs.clear();
}

// the graph of len consecutive generations whose adapting ones are the set
// bits of adapt, captured on first use
rvea_status graph_for(rvea_run r, int len, uint64_t adapt, hipGraphExec_t *out)
{
    for (auto &g : r->graphs) {
        if (g.len == len && g.adapt == adapt) {
            *out = g.x;
            return RVEA_OK;
        }
    }
    if (r->graphs.size() >= kGraphCache) {  // none of them may still be running
        HIPCHK(r, hipStreamSynchronize(r->stream));
        drop_graphs(r);
    }
    if (!r->cap_stream)
        HIPCHK(r, hipStreamCreateWithFlags(&r->cap_stream, hipStreamNonBlocking));
    HIPCHK(r, hipStreamBeginCapture(r->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < len && e == hipSuccess; ++k)
        e = enqueue_generation(r->R, r->cap_stream, (adapt >> k) & 1u);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(r->cap_stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(r, e, "graph capture");
    }
    if (e2 != hipSuccess) return fail(r, e2, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(r, e, "hipGraphInstantiate");
    }
    r->graphs.push_back({len, adapt, g, x});
    *out = x;
    return RVEA_OK;
}

// n generations from generation r->t + 1 as launches of up to kGraphGens
// generations; a length that is a multiple of the adaptation period keeps
// the adapting positions, and so the graph, the same from one launch to the
// next.  launch = false only captures the graphs.
rvea_status graph_launches(rvea_run r, int n, bool launch)
{
    const int64_t P = r->R.period;
    const int L = P <= kGraphGens ? (int)(P * (kGraphGens / P)) : kGraphGens;
    int64_t t = r->t;
    for (int i = 0; i < n;) {
        const int len = n - i < L ? n - i : L;
        uint64_t adapt = 0;
        for (int k = 0; k < len; ++k)
            if ((t + 1 + k) % P == 0) adapt |= 1ull << k;
        hipGraphExec_t x = nullptr;
        rvea_status st = graph_for(r, len, adapt, &x);
        if (st != RVEA_OK) return st;
        if (launch) HIPCHK(r, hipGraphLaunch(x, r->stream));
        t += len;
        i += len;
    }
    if (launch) r->t = t;
    return RVEA_OK;
}

}  // namespace

rvea_status rvea_prepare_generations(rvea_run r, int n)
{
    if (!r || n < 0) return RVEA_EINVAL;
    if (n > 0 && (r->phase != 0 || r->batch)) return RVEA_ESTATE;
    if (!r->use_graphs || n == 0) return RVEA_OK;
    return graph_launches(r, n, false);
}

rvea_status rvea_run_generations(rvea_run r, int n)
{
    if (!r || n < 0) return RVEA_EINVAL;
    if (n > 0 && (r->phase != 0 || r->batch)) return RVEA_ESTATE;
    if (r->use_graphs && r->timing == 0 && n > 0) {
        rvea_status st = graph_launches(r, n, true);
        if (st != RVEA_OK) return st;
        r->has_selection = true;
        return RVEA_OK;
    }
    for (int i = 0; i < n; ++i) {
        rvea_status st = rvea_step(r);
        if (st == RVEA_OK) st = rvea_select(r);
        if (st == RVEA_OK) st = rvea_adapt(r);
        if (st != RVEA_OK) return st;
    }
    return RVEA_OK;
}

static hipStream_t active_stream(rvea_run r) { return r->batch ? r->batch->stream : r->stream; }

rvea_status rvea_synchronize(rvea_run r)
{
    if (!r) return RVEA_EINVAL;
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    return check_counters(r);
}

namespace {

// copy the rows rows[0..n) of a (K+N) x ld pool (the genes by default, or
// the velocities) into dst (n x d, host)
rvea_status copy_rows(rvea_run r, const std::vector<int32_t> &rows, float *dst,
                      const float *pool_base = nullptr)
{
    const RunView &R = r->R;
    const float *base = pool_base ? pool_base : R.X;
    const size_t rowb = (size_t)R.d * 4;
    const size_t pool_bytes = (size_t)(R.K + R.N) * R.ld * 4;
    if (pool_bytes <= ((size_t)1 << 28) || rows.size() * 4 > (size_t)(R.K + R.N)) {
        std::vector<float> pool((size_t)(R.K + R.N) * R.ld);
        HIPCHK(r, hipMemcpy(pool.data(), base, pool_bytes, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < rows.size(); ++i)
            std::memcpy(dst + i * R.d, pool.data() + (size_t)rows[i] * R.ld, rowb);
    } else {
        for (size_t i = 0; i < rows.size(); ++i)
            HIPCHK(r, hipMemcpy(dst + i * R.d, base + (size_t)rows[i] * R.ld, rowb,
                                hipMemcpyDeviceToHost));
    }
    return RVEA_OK;
}

}  // namespace

namespace {

// the population buffers of population p (completed generations)
int32_t *slot_rows_at(const RunView &R, int64_t p) { return R.slot_rows + (p & 1) * R.K; }
uint8_t *valids_at(const RunView &R, int64_t p) { return R.valids + (p & 1) * R.K; }
float *fm_at(const RunView &R, int64_t p) { return R.Fms + (p & 1) * R.M * R.m; }

// completed generations as the device counts them (after a synchronize)
rvea_status device_t(rvea_run r, int64_t *t)
{
    HIPCHK(r, hipMemcpy(t, r->R.t_done, 8, hipMemcpyDeviceToHost));
    return RVEA_OK;
}

// the population whose merged buffer holds the offspring: after rvea_step
// the parents' (the generation is not counted yet); after rvea_select, and
// between generations for the last completed one, one less than the count
int64_t offspring_pop(rvea_run r, int64_t td) { return r->phase == 1 ? td : td - 1; }

// offspring are readable after rvea_step and, between generations, for the
// last completed generation until the next step (their rows are only reused
// by the next reproduction); not after set_state or an autotune, which
// drew offspring without completing a generation
bool offspring_readable(rvea_run r) { return r->phase != 0 || r->has_selection; }

}  // namespace

rvea_status rvea_get_state(rvea_run r, float *X, float *F, uint8_t *valid, double *V,
                           double *V0, double *gamma, int64_t *t)
{
    if (!r) return RVEA_EINVAL;
    const RunView &R = r->R;
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    int64_t td = 0;
    rvea_status st0 = device_t(r, &td);
    if (st0 != RVEA_OK) return st0;
    std::vector<uint8_t> vh(R.K);
    HIPCHK(r, hipMemcpy(vh.data(), valids_at(R, td), R.K, hipMemcpyDeviceToHost));
    if (valid) std::memcpy(valid, vh.data(), R.K);
    if (X) {
        std::vector<int32_t> rows(R.K);
        HIPCHK(r, hipMemcpy(rows.data(), slot_rows_at(R, td), R.K * 4, hipMemcpyDeviceToHost));
        rvea_status st = copy_rows(r, rows, X);
        if (st != RVEA_OK) return st;
        for (int64_t j = 0; j < R.K; ++j)
            if (!vh[j]) std::memset(X + j * R.d, 0, (size_t)R.d * 4);
    }
    if (F) HIPCHK(r, hipMemcpy(F, fm_at(R, td), (size_t)R.K * R.m * 4, hipMemcpyDeviceToHost));
    if (V) HIPCHK(r, hipMemcpy(V, R.V, (size_t)R.K * R.m * 8, hipMemcpyDeviceToHost));
    if (V0) HIPCHK(r, hipMemcpy(V0, R.V0, (size_t)R.K * R.m * 8, hipMemcpyDeviceToHost));
    if (gamma) HIPCHK(r, hipMemcpy(gamma, R.gamma, (size_t)R.K * 8, hipMemcpyDeviceToHost));
    if (t) *t = td;
    return check_counters(r);
}

rvea_status rvea_set_state(rvea_run r, const float *X, const float *F, const uint8_t *valid,
                           const double *V, const double *gamma, int64_t t)
{
    if (!r || !X || !F || !valid || t < 0) return RVEA_EINVAL;
    if (r->phase != 0 || r->batch) return RVEA_ESTATE;
    const RunView &R = r->R;
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    HIPCHK(r, hipMemcpy2D(R.X, (size_t)R.ld * 4, X, (size_t)R.d * 4, (size_t)R.d * 4,
                          (size_t)R.K, hipMemcpyHostToDevice));
    std::vector<int32_t> rows(R.K);
    std::vector<uint8_t> vv(R.K);
    for (int64_t j = 0; j < R.K; ++j) {
        rows[j] = (int32_t)j;
        vv[j] = valid[j] ? 1 : 0;
    }
    HIPCHK(r, hipMemcpy(slot_rows_at(R, t), rows.data(), R.K * 4, hipMemcpyHostToDevice));
    HIPCHK(r, hipMemcpy(valids_at(R, t), vv.data(), R.K, hipMemcpyHostToDevice));
    HIPCHK(r, hipMemcpy(fm_at(R, t), F, (size_t)R.K * R.m * 4, hipMemcpyHostToDevice));
    if (V) {
        HIPCHK(r, hipMemcpy(R.V, V, (size_t)R.K * R.m * 8, hipMemcpyHostToDevice));
        HIPCHK(r, launch_vec_aux(R, r->stream));
    }
    if (gamma)
        HIPCHK(r, hipMemcpy(R.gamma, gamma, (size_t)R.K * 8, hipMemcpyHostToDevice));
    else if (V)
        HIPCHK(r, launch_gamma(R, r->stream, 1));
    if (V && r->L.gG > 0) {  // a host-set V: the index unscaled and rebuilt
        HIPCHK(r, hipStreamSynchronize(r->stream));
        HIPCHK(r, hipMemcpy(R.gr, kUnitScale, (size_t)R.m * sizeof(double), hipMemcpyHostToDevice));
        if (R.gG > 0) HIPCHK(r, launch_grid_build(R, r->stream, 1));
    }
    HIPCHK(r, hipMemcpy(R.t_done, &t, 8, hipMemcpyHostToDevice));
    HIPCHK(r, hipMemset(R.stamp, 0xff, (size_t)(R.K + R.N) * 4));
    HIPCHK(r, hipMemset(R.zbits, 0xff, (size_t)2 * R.m * 4));
    if (R.Vel) HIPCHK(r, hipMemset(R.Vel, 0, (size_t)(R.K + R.N) * R.ld * 4));
    HIPCHK(r, hipDeviceSynchronize());
    HIPCHK(r, launch_stamp(R, r->stream));
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    r->t = t;
    r->has_selection = false;
    return RVEA_OK;
}

rvea_status rvea_get_offspring(rvea_run r, float *X, float *F, int32_t *parents)
{
    if (!r) return RVEA_EINVAL;
    if (!offspring_readable(r)) return RVEA_ESTATE;
    const RunView &R = r->R;
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    if (X) {
        std::vector<int32_t> rows(R.N);
        HIPCHK(r, hipMemcpy(rows.data(), R.off_row, R.N * 4, hipMemcpyDeviceToHost));
        rvea_status st = copy_rows(r, rows, X);
        if (st != RVEA_OK) return st;
    }
    if (F) {
        int64_t td = 0;
        rvea_status st = device_t(r, &td);
        if (st != RVEA_OK) return st;
        HIPCHK(r, hipMemcpy(F, fm_at(R, offspring_pop(r, td)) + R.K * R.m,
                            (size_t)R.N * R.m * 4, hipMemcpyDeviceToHost));
    }
    if (parents)
        HIPCHK(r, hipMemcpy(parents, R.parents, (size_t)((R.N + 1) / 2) * 8,
                            hipMemcpyDeviceToHost));
    return check_counters(r);
}

rvea_status rvea_get_selection(rvea_run r, float *zstar, int32_t *assoc, double *apd,
                               int32_t *surv)
{
    if (!r) return RVEA_EINVAL;
    if (!r->has_selection || r->phase == 1) return RVEA_ESTATE;
    const RunView &R = r->R;
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    if (zstar) {
        int64_t td = 0;  // the last selection's generation picks the buffer
        HIPCHK(r, hipMemcpy(&td, R.t_done, 8, hipMemcpyDeviceToHost));
        uint32_t zb[kMaxM];
        HIPCHK(r, hipMemcpy(zb, R.zbits + (td & 1) * R.m, R.m * 4, hipMemcpyDeviceToHost));
        for (int k = 0; k < R.m; ++k) {
            const uint32_t e = zb[k];
            const uint32_t u = (e & 0x80000000u) ? (e & 0x7FFFFFFFu) : ~e;
            std::memcpy(zstar + k, &u, 4);
        }
    }
    if (assoc) HIPCHK(r, hipMemcpy(assoc, R.assoc, R.M * 4, hipMemcpyDeviceToHost));
    if (apd) HIPCHK(r, hipMemcpy(apd, R.apd, R.M * 8, hipMemcpyDeviceToHost));
    if (surv) HIPCHK(r, hipMemcpy(surv, R.surv, R.K * 4, hipMemcpyDeviceToHost));
    return RVEA_OK;
}

rvea_status rvea_get_rows(rvea_run r, int offspring, const int64_t *idx, int64_t n, float *X,
                          float *F)
{
    if (!r || (n > 0 && !idx) || n < 0) return RVEA_EINVAL;
    if (offspring && !offspring_readable(r)) return RVEA_ESTATE;
    const RunView &R = r->R;
    const int64_t lim = offspring ? R.N : R.K;
    for (int64_t q = 0; q < n; ++q)
        if (idx[q] < 0 || idx[q] >= lim) return RVEA_EINVAL;
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    int64_t td = 0;
    rvea_status st0 = device_t(r, &td);
    if (st0 != RVEA_OK) return st0;
    const int64_t pop = offspring ? offspring_pop(r, td) : td;
    std::vector<int32_t> map(lim);
    HIPCHK(r, hipMemcpy(map.data(), offspring ? R.off_row : slot_rows_at(R, td), lim * 4,
                        hipMemcpyDeviceToHost));
    for (int64_t q = 0; q < n; ++q) {
        const int64_t i = idx[q];
        if (X)
            HIPCHK(r, hipMemcpy(X + q * R.d, R.X + (size_t)map[i] * R.ld, (size_t)R.d * 4,
                                hipMemcpyDeviceToHost));
        if (F)
            HIPCHK(r, hipMemcpy(F + q * R.m, fm_at(R, pop) + ((offspring ? R.K : 0) + i) * R.m,
                                (size_t)R.m * 4, hipMemcpyDeviceToHost));
    }
    return check_counters(r);
}

rvea_status rvea_get_velocities(rvea_run r, int offspring, float *Vel)
{
    if (!r || !Vel) return RVEA_EINVAL;
    const RunView &R = r->R;
    if (!R.Vel) return RVEA_EINVAL;
    if (offspring && !offspring_readable(r)) return RVEA_ESTATE;
    if (!offspring && r->phase != 0) return RVEA_ESTATE;
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    int64_t td = 0;
    rvea_status st = device_t(r, &td);
    if (st != RVEA_OK) return st;
    const int64_t n = offspring ? R.N : R.K;
    std::vector<int32_t> rows(n);
    HIPCHK(r, hipMemcpy(rows.data(), offspring ? R.off_row : slot_rows_at(R, td), n * 4,
                        hipMemcpyDeviceToHost));
    st = copy_rows(r, rows, Vel, R.Vel);
    if (st != RVEA_OK) return st;
    if (!offspring) {
        std::vector<uint8_t> vh(R.K);
        HIPCHK(r, hipMemcpy(vh.data(), valids_at(R, td), R.K, hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < R.K; ++j)
            if (!vh[j]) std::memset(Vel + j * R.d, 0, (size_t)R.d * 4);
    }
    return RVEA_OK;
}

rvea_status rvea_set_velocities(rvea_run r, const float *Vel)
{
    if (!r || !Vel) return RVEA_EINVAL;
    const RunView &R = r->R;
    if (!R.Vel) return RVEA_EINVAL;
    if (r->phase != 0 || r->batch) return RVEA_ESTATE;
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    int64_t td = 0;
    rvea_status st = device_t(r, &td);
    if (st != RVEA_OK) return st;
    std::vector<int32_t> rows(R.K);
    HIPCHK(r, hipMemcpy(rows.data(), slot_rows_at(R, td), R.K * 4, hipMemcpyDeviceToHost));
    // the pool through host memory: the slots' rows are scattered over it
    const size_t pool_bytes = (size_t)(R.K + R.N) * R.ld * 4;
    std::vector<float> pool((size_t)(R.K + R.N) * R.ld);
    HIPCHK(r, hipMemcpy(pool.data(), R.Vel, pool_bytes, hipMemcpyDeviceToHost));
    for (int64_t j = 0; j < R.K; ++j)
        std::memcpy(pool.data() + (size_t)rows[j] * R.ld, Vel + j * R.d, (size_t)R.d * 4);
    HIPCHK(r, hipMemcpy(R.Vel, pool.data(), pool_bytes, hipMemcpyHostToDevice));
    return RVEA_OK;
}

rvea_status rvea_get_counters(rvea_run r, rvea_counters *out)
{
    if (!r || !out) return RVEA_EINVAL;
    unsigned long long c[3];
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    HIPCHK(r, hipMemcpy(c, r->R.counters, sizeof c, hipMemcpyDeviceToHost));
    out->nonfinite_rows = (int64_t)c[0];
    out->full_rescans = (int64_t)c[1];
    out->generations = r->t;
    return RVEA_OK;
}

rvea_status rvea_set_graphs(rvea_run r, int enable)
{
    if (!r) return RVEA_EINVAL;
    r->use_graphs = enable != 0;
    return RVEA_OK;
}

rvea_status rvea_set_index(rvea_run r, int enable)
{
    if (!r) return RVEA_EINVAL;
    if (r->phase != 0 || r->batch) return RVEA_ESTATE;
    if (enable && r->L.gG == 0) return RVEA_EUNSUPPORTED;
    const int G = enable ? r->L.gG : 0;
    if (G == r->R.gG) return RVEA_OK;
    HIPCHK(r, hipStreamSynchronize(r->stream));
    r->R.gG = G;
    // V may have changed while the index was off
    if (G > 0) HIPCHK(r, launch_grid_build(r->R, r->stream, 1));
    drop_graphs(r);  // they hold the old launch sequence
    return RVEA_OK;
}

rvea_status rvea_set_timing(rvea_run r, int kernel_mask)
{
    if (!r) return RVEA_EINVAL;
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    for (auto &ev : r->events) {
        r->pool.push_back(ev.a);
        r->pool.push_back(ev.b);
    }
    r->events.clear();
    r->timing = kernel_mask & ((1 << kKernels) - 1);
    return RVEA_OK;
}

rvea_status rvea_kernel_time(rvea_run r, int kernel, double *ms, int64_t *launches)
{
    if (!r || kernel < 0 || kernel >= kKernels || !ms || !launches) return RVEA_EINVAL;
    HIPCHK(r, hipStreamSynchronize(active_stream(r)));
    double tot = 0.0;
    int64_t n = 0;
    for (auto &ev : r->events) {
        if (ev.id != kernel) continue;
        float x = 0.f;
        HIPCHK(r, hipEventElapsedTime(&x, ev.a, ev.b));
        tot += x;
        ++n;
    }
    *ms = tot;
    *launches = n;
    return RVEA_OK;
}

rvea_status rvea_time_kernels(rvea_run r, int reps, double *ms)
{
    if (!r || reps < 1 || !ms) return RVEA_EINVAL;
    if (r->phase != 1 || r->batch || r->timing) return RVEA_ESTATE;
    const RunView &R = r->R;
    HIPCHK(r, hipStreamSynchronize(r->stream));
    unsigned long long saved[3];
    HIPCHK(r, hipMemcpy(saved, R.counters, sizeof saved, hipMemcpyDeviceToHost));
    EventPair ev(r);
    if (!ev.ok()) return fail(r, hipErrorOutOfMemory, "hipEventCreate");
    const hipEvent_t a = ev.a, b = ev.b;
    // each pass rewrites the same outputs from the same inputs: the
    // offspring from the parents, the partials from F and V, and the
    // re-rank's minima (order-free) from the partials
    for (int k = 0; k < 3; ++k) {
        auto launch = [&]() {
            return k == 0 ? launch_offspring(R, r->stream)
                          : (k == 1 ? launch_assoc(R, r->stream) : launch_rerank(R, r->stream));
        };
        HIPCHK(r, launch());  // warm
        HIPCHK(r, hipEventRecord(a, r->stream));
        for (int i = 0; i < reps; ++i) HIPCHK(r, launch());
        HIPCHK(r, hipEventRecord(b, r->stream));
        HIPCHK(r, hipEventSynchronize(b));
        float x = 0.f;
        HIPCHK(r, hipEventElapsedTime(&x, a, b));
        ms[k] = (double)x / reps;
    }
    HIPCHK(r, hipMemcpy(R.counters, saved, sizeof saved, hipMemcpyHostToDevice));
    return RVEA_OK;
}

rvea_status rvea_batch_retire(rvea_batch b, rvea_run r);


}  // extern "C"

namespace {

// Chunk lengths to try for `rows` rows against K vectors at rr rows per
// lane: the default length times powers of two, and the lengths that make
// the workgroup count (row blocks x chunks) just below k times the CU count,
// k = 1..8, so that no CU runs one more workgroup than the others (each the
// shortest multiple of the tile with its chunk count).  At most KC0 chunks;
// the default length comes first.
std::vector<int> chunk_candidates(int64_t rows, int64_t K, int rr, int CS0, int KC0, int cus)
{
    std::vector<int> out;
    auto add = [&](int64_t cs) {
        if (cs < CS0 || cs > 32 * kTile || (K + cs - 1) / cs > KC0) return;
        for (int c : out)
            if (c == cs) return;
        out.push_back((int)cs);
    };
    for (int64_t cs = CS0;; cs *= 2) {
        add(cs);
        if (cs >= K || cs >= 32 * kTile) break;
    }
    const int64_t nbi = (rows + 256 * rr - 1) / (256 * rr);
    for (int k = 1; k <= 8; ++k) {
        const int64_t kc = (int64_t)k * cus / nbi;
        if (kc >= 1) add(((K + kc - 1) / kc + kTile - 1) / kTile * kTile);
    }
    return out;
}

}  // namespace

extern "C" {

rvea_status rvea_autotune(rvea_run r, rvea_tuning *out)
{
    if (!r) return RVEA_EINVAL;
    if (r->phase != 0 || r->batch || r->timing) return RVEA_ESTATE;
    RunView &R = r->R;
    const int KC0 = r->L.KC, CS0 = r->L.CS;
    HIPCHK(r, hipStreamSynchronize(r->stream));
    unsigned long long saved[3];
    HIPCHK(r, hipMemcpy(saved, R.counters, sizeof saved, hipMemcpyDeviceToHost));
    // the next generation's offspring and ideal point give the association
    // its real input; nothing is committed, so the state is unchanged
    HIPCHK(r, launch_prepare(R, r->stream));
    HIPCHK(r, launch_offspring(R, r->stream));
    if (R.problem == kPolicy) HIPCHK(r, launch_rollout(R, r->stream, true));
    EventPair ev(r);
    if (!ev.ok()) return fail(r, hipErrorOutOfMemory, "hipEventCreate");
    const hipEvent_t a = ev.a, b = ev.b;
    // a candidate's time per launch: kTuneReps launches back to back between
    // two events (no per-launch event overhead), best of two rounds, after a
    // warm launch; every timed pass rewrites the same outputs
    constexpr int kTuneReps = 5;
    auto time_launches = [&](auto &&launch, float *out) -> hipError_t {
        hipError_t e = launch();
        if (e != hipSuccess) return e;
        float best = 1e30f;
        for (int round = 0; round < 2; ++round) {
            if ((e = hipEventRecord(a, r->stream)) != hipSuccess) return e;
            for (int i = 0; i < kTuneReps; ++i)
                if ((e = launch()) != hipSuccess) return e;
            if ((e = hipEventRecord(b, r->stream)) != hipSuccess) return e;
            if ((e = hipEventSynchronize(b)) != hipSuccess) return e;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) return e;
            best = std::min(best, ms / kTuneReps);
        }
        *out = best;
        return hipSuccess;
    };
    struct Cand {
        int rr, cs;
        float ms;  // association + re-rank
    };
    int cus = 0;
    HIPCHK(r, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, r->device));
    // the full-scan passes' shapes are tuned with the index off (they serve
    // the gamma pass, batches, and runs without an index)
    const int gG0 = R.gG;
    R.gG = 0;
    std::vector<Cand> cands;
    for (int rr : {4, 2, 1})
        for (int cs : chunk_candidates(R.M, R.K, rr, CS0, KC0, cus)) cands.push_back({rr, cs, 0.f});
    const int saved_rr = R.rr, saved_cs = R.CS, saved_kc = R.KC;
    double def_ms = -1.0;
    for (auto &c : cands) {
        R.rr = c.rr;
        R.CS = c.cs;
        R.KC = (int)((R.K + c.cs - 1) / c.cs);
        if (R.KC > KC0) continue;  // the workspace holds KC0 chunk partials
        // the chunk count also sets the re-rank's work (partials per row),
        // so each candidate is timed with the re-rank that follows it
        float best = 0.f;
        HIPCHK(r, time_launches(
                      [&]() {
                          const hipError_t e = launch_assoc(R, r->stream);
                          return e != hipSuccess ? e : launch_rerank(R, r->stream);
                      },
                      &best));
        c.ms = best;
        if (c.rr == saved_rr && c.cs == saved_cs) def_ms = best;
    }
    const Cand *win = nullptr;
    for (auto &c : cands)
        if (c.ms > 0.f && (!win || c.ms < win->ms)) win = &c;
    if (win) {
        R.rr = win->rr;
        R.CS = win->cs;
        R.KC = (int)((R.K + win->cs - 1) / win->cs);
    } else {
        R.rr = saved_rr;
        R.CS = saved_cs;
        R.KC = saved_kc;
    }
    // re-rank rows per wave, on the chosen association's partials (the pass
    // is idempotent: the same minima and outputs every time)
    HIPCHK(r, launch_assoc(R, r->stream));
    const int rk0 = R.rk;
    double rk_def = -1.0, rk_best = 1e30;
    int rk_win = rk0;
    for (int rk : {4, 8, 16}) {
        R.rk = rk;
        float best = 0.f;
        HIPCHK(r, time_launches([&]() { return launch_rerank(R, r->stream); }, &best));
        if (rk == rk0) rk_def = best;
        if (best < rk_best) {
            rk_best = best;
            rk_win = rk;
        }
    }
    R.rk = rk_win;
    // the gamma pass (rows = vectors, at adaptations): its own chunking and
    // rows per lane, timed on the current vectors (it rewrites the same
    // gamma every time)
    const int grr0 = R.grr, gcs0 = R.gCS;
    double g_def = -1.0, g_best = 1e30;
    int g_rr = grr0, g_cs = gcs0;
    int ncand = (int)cands.size() + 3;
    for (int rr : {4, 2, 1}) {
        for (int cs : chunk_candidates(R.K, R.K, rr, CS0, KC0, cus)) {
            const int kc = (int)((R.K + cs - 1) / cs);
            {  // timed as one launch of both passes
                R.grr = rr;
                R.gCS = cs;
                R.gKC = kc;
                float best = 0.f;
                HIPCHK(r, time_launches([&]() { return launch_gamma(R, r->stream, 1); }, &best));
                ++ncand;
                if (rr == grr0 && cs == gcs0) g_def = best;
                if (best < g_best) {
                    g_best = best;
                    g_rr = rr;
                    g_cs = cs;
                }
            }
        }
    }
    R.grr = g_rr;
    R.gCS = g_cs;
    R.gKC = (int)((R.K + g_cs - 1) / g_cs);
    R.gG = gG0;
    HIPCHK(r, hipMemcpy(R.counters, saved, sizeof saved, hipMemcpyHostToDevice));
    // the trial's preparation handed out free rows: the real one starts over
    HIPCHK(r, hipMemsetAsync(R.freecnt, 0, 4, r->stream));
    HIPCHK(r, hipStreamSynchronize(r->stream));
    drop_graphs(r);            // captured with the old launch shapes
    r->has_selection = false;  // the trial overwrote the last selection's buffers
    if (out) {
        out->rows_per_lane = R.rr;
        out->chunk_vectors = R.CS;
        out->rerank_rows = R.rk;
        out->candidates = ncand;
        out->assoc_us = win ? 1e3 * win->ms : -1.0;
        out->default_us = 1e3 * def_ms;
        out->rerank_us = 1e3 * rk_best;
        out->rerank_default_us = 1e3 * rk_def;
        out->gamma_rows_per_lane = R.grr;
        out->gamma_chunk_vectors = R.gCS;
        out->gamma_us = 1e3 * g_best;
        out->gamma_default_us = 1e3 * g_def;
    }
    return RVEA_OK;
}

rvea_status rvea_destroy(rvea_run r)
{
    if (!r) return RVEA_EINVAL;
    if (r->batch) rvea_batch_retire(r->batch, r);
    (void)hipStreamSynchronize(r->stream);
    for (auto &ev : r->events) {
        (void)hipEventDestroy(ev.a);
        (void)hipEventDestroy(ev.b);
    }
    for (auto e : r->pool) (void)hipEventDestroy(e);
    drop_graphs(r);
    if (r->cap_stream) (void)hipStreamDestroy(r->cap_stream);
    delete r;
    return RVEA_OK;
}

// ------------------------------------------------------------------ batches
namespace {

rvea_status bfail(rvea_batch b, hipError_t e, const char *what)
{
    std::snprintf(b->err, sizeof b->err, "%s: %s", what, hipGetErrorString(e));
    return RVEA_EDEVICE;
}

#define BHIPCHK(b, call)                                                                     \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return bfail(b, e_, #call);                                    \
    } while (0)

// span tables of every (phase, class) over the admitted runs, uploaded once
// per membership change
rvea_status rebuild_plan(rvea_batch b)
{
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    const int n = (int)b->runs.size();
    std::vector<RunView> views(n), gviews(n), wide(n);
    int64_t wide_blocks = 0;
    for (int i = 0; i < n; ++i) {
        views[i] = b->runs[i]->R;
        // the gamma passes (rows = vectors) keep the run's own chunking, as
        // alone: their few rows need the chunks for parallelism
        gviews[i] = views[i];
        gviews[i].KC = gviews[i].gKC;
        gviews[i].CS = gviews[i].gCS;
        // a batch whose runs fill the device by themselves needs no vector
        // chunks for occupancy: chunks of up to 32 tiles (never more chunks
        // than the run's buffers hold) cut the per-chunk maxima written and
        // re-read and the re-rank's walk over them (the exact argmax does not
        // depend on the chunking)
        RunView &v = wide[i];
        v = views[i];
        const int64_t cs = std::min<int64_t>(32 * kTile, (v.K + kTile - 1) / kTile * kTile);
        if (cs > v.CS) {
            v.CS = (int)cs;
            v.KC = (int)((v.K + cs - 1) / cs);
        }
        if (v.gG <= 0) wide_blocks += batch_phase_blocks(BP_ASSOC, v);
    }
    if (wide_blocks >= kFillBlocks) views = wide;
    std::vector<Span> spans;
    b->plan.clear();
    for (int phase = 0; phase < BP_COUNT; ++phase) {
        std::vector<int> classes;
        const std::vector<RunView> &pv = batch_phase_gamma(phase) ? gviews : views;
        for (int i = 0; i < n; ++i) {
            const int c = batch_phase_class(phase, pv[i]);
            if (std::find(classes.begin(), classes.end(), c) == classes.end()) classes.push_back(c);
        }
        std::sort(classes.begin(), classes.end());
        for (int c : classes) {
            rvea_batch_s::Launch L{phase, c, (int64_t)spans.size(), 0, 0};
            for (int i = 0; i < n; ++i) {
                if (batch_phase_class(phase, pv[i]) != c) continue;
                const int64_t nb = batch_phase_blocks(phase, pv[i]);
                if (nb <= 0) continue;
                spans.push_back(Span{L.blocks, i, (int32_t)batch_phase_nbx(phase, pv[i])});
                L.blocks += nb;
                ++L.n;
            }
            if (L.n > 0) b->plan.push_back(L);
        }
    }
    if (n > 0) {
        BHIPCHK(b, hipMemcpy(b->d_runs, views.data(), sizeof(RunView) * n, hipMemcpyHostToDevice));
        BHIPCHK(b, hipMemcpy(b->d_gruns, gviews.data(), sizeof(RunView) * n, hipMemcpyHostToDevice));
        BHIPCHK(b, hipMemcpy(b->d_spans, spans.data(), sizeof(Span) * spans.size(),
                             hipMemcpyHostToDevice));
    }
    b->dirty = false;
    ++b->version;
    return RVEA_OK;
}

hipError_t enqueue_batch_generation(rvea_batch b, hipStream_t s)
{
    for (const auto &L : b->plan) {
        hipError_t e = launch_batch(L.phase, L.cls, batch_phase_gamma(L.phase) ? b->d_gruns : b->d_runs,
                                    b->d_spans + L.span_off, L.n, L.blocks, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

rvea_status rvea_batch_footprint(int max_runs, size_t *bytes)
{
    if (!bytes || max_runs < 1 || max_runs > (1 << 16)) return RVEA_EINVAL;
    const size_t a = ((size_t)max_runs * sizeof(RunView) + 255) / 256 * 256;
    const size_t c = ((size_t)BP_COUNT * max_runs * sizeof(Span) + 255) / 256 * 256;
    *bytes = 2 * a + c;
    return RVEA_OK;
}

rvea_status rvea_batch_create(int max_runs, void *workspace, size_t workspace_bytes,
                              void *hip_stream, rvea_batch *out)
{
    if (!out) return RVEA_EINVAL;
    *out = nullptr;
    size_t need = 0;
    rvea_status st = rvea_batch_footprint(max_runs, &need);
    if (st != RVEA_OK) return st;
    if (!workspace || ((uintptr_t)workspace & 255u)) return RVEA_EINVAL;
    if (workspace_bytes < need) return RVEA_ENOMEM;
    rvea_batch b = new rvea_batch_s();
    b->max_runs = max_runs;
    b->stream = (hipStream_t)hip_stream;
    const size_t a = ((size_t)max_runs * sizeof(RunView) + 255) / 256 * 256;
    b->d_runs = (RunView *)workspace;
    b->d_gruns = (RunView *)((char *)workspace + a);
    b->d_spans = (Span *)((char *)workspace + 2 * a);
    *out = b;
    return RVEA_OK;
}

rvea_status rvea_batch_admit(rvea_batch b, rvea_run r)
{
    if (!b || !r) return RVEA_EINVAL;
    if (r->batch || r->phase != 0 || r->timing) return RVEA_ESTATE;
    if (r->R.problem == kPolicy) return RVEA_EUNSUPPORTED;
    if ((int)b->runs.size() >= b->max_runs) return RVEA_ENOMEM;
    // the run's pending work (creation, earlier generations) precedes the batch
    HIPCHK(r, hipStreamSynchronize(r->stream));
    r->batch = b;
    b->runs.push_back(r);
    b->dirty = true;
    return RVEA_OK;
}

rvea_status rvea_batch_retire(rvea_batch b, rvea_run r)
{
    if (!b || !r || r->batch != b) return RVEA_EINVAL;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    b->runs.erase(std::find(b->runs.begin(), b->runs.end(), r));
    r->batch = nullptr;
    b->dirty = true;
    return RVEA_OK;
}

rvea_status rvea_batch_step(rvea_batch b)
{
    if (!b) return RVEA_EINVAL;
    if (b->dirty) {
        rvea_status st = rebuild_plan(b);
        if (st != RVEA_OK) return st;
    }
    if (b->runs.empty()) return RVEA_OK;
    const bool stable = b->last_step_version == b->version;
    b->last_step_version = b->version;
    if (b->use_graphs && (stable || b->graph_version == b->version)) {
        if (b->graph_version != b->version) {
            if (b->gexec) {
                BHIPCHK(b, hipGraphExecDestroy(b->gexec));
                BHIPCHK(b, hipGraphDestroy(b->graph));
                b->gexec = nullptr;
                b->graph = nullptr;
            }
            if (!b->cap_stream)
                BHIPCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
            BHIPCHK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_batch_generation(b, b->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
            if (e != hipSuccess) return bfail(b, e, "batch capture");
            if (e2 != hipSuccess) return bfail(b, e2, "hipStreamEndCapture");
            b->graph = g;
            BHIPCHK(b, hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
            b->graph_version = b->version;
        }
        BHIPCHK(b, hipGraphLaunch(b->gexec, b->stream));
    } else {
        BHIPCHK(b, enqueue_batch_generation(b, b->stream));
    }
    for (rvea_run r : b->runs) {
        r->t += 1;
        r->has_selection = true;
    }
    return RVEA_OK;
}

rvea_status rvea_batch_set_graphs(rvea_batch b, int enable)
{
    if (!b) return RVEA_EINVAL;
    b->use_graphs = enable != 0;
    return RVEA_OK;
}

rvea_status rvea_batch_size(rvea_batch b, int *n)
{
    if (!b || !n) return RVEA_EINVAL;
    *n = (int)b->runs.size();
    return RVEA_OK;
}

rvea_status rvea_batch_synchronize(rvea_batch b)
{
    if (!b) return RVEA_EINVAL;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    return RVEA_OK;
}

rvea_status rvea_batch_destroy(rvea_batch b)
{
    if (!b) return RVEA_EINVAL;
    (void)hipStreamSynchronize(b->stream);
    for (rvea_run r : b->runs) r->batch = nullptr;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return RVEA_OK;
}

const char *rvea_batch_last_error(rvea_batch b) { return b ? b->err : "no batch"; }

const char *rvea_status_str(rvea_status s)
{
    switch (s) {
    case RVEA_OK: return "ok";
    case RVEA_EINVAL: return "invalid argument";
    case RVEA_ENOMEM: return "workspace too small";
    case RVEA_EDEVICE: return "HIP device error";
    case RVEA_ESTATE: return "call out of order";
    case RVEA_EUNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

const char *rvea_last_error(rvea_run r)
{
    if (r) return r->err;
    return g_create_err[0] ? g_create_err : "no run";
}

}  // extern "C"

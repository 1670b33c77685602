// gkr.hip -- host driver of the GKR prover / verifier and the C ABI (gkr.h).
//
// The prover is a fixed sequence of kernel launches on one stream: load the
// inputs, evaluate the layers (output last), then per layer the p-phase
// rounds (a-variables), the two omega-phases (b- then c-variables) and the
// line step.  Challenges are drawn on the device right after each message
// is reduced, so the host never waits inside a proof; it copies the
// transcript back once at the end.  Device scratch is allocated on the
// first proof of a circuit and kept with it (Sec. 6.1 does not count
// scratch allocation in prover time).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gkr.h"
#include "fp61.hpp"
#include "kernels.hpp"
#include "steps.hpp"
#include "nif2.hpp"

using namespace gkr;

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

static int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? GKR_ERR_NOMEM : GKR_ERR_DEVICE,          \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                  \
    } while (0)

extern "C" const char *gkr_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------- profiling

namespace {

// Profiling classes: one per step kind (the kernel k_step_one<kind, ...>),
// then the verifier's and the F2 sum-check's kernels.
enum ProfClass {
    PC_STEP = 0,  // + StepKind
    PC_WIRING = 21, PC_MLE, PC_TABLES, PC_F2SC, PC_FINAL, PC_MISC, PC_BATCH, PC_NIF2, PC_SERVE, PC_COUNT
};
const char *kProfNames[PC_COUNT] = {
    "step_eval", "step_start", "step_eq", "step_p", "step_w", "step_fold", "step_lt",
    "step_line", "step_sge", "step_end", "step_wagg", "step_wt0", "step_wt", "step_wtail",
    "step_ptail", "step_load", "step_wa0", "step_finish", "step_wsmall", "step_top", "step_lfold", "wiring", "mle", "eq_tables", "f2sc_round",
    "f2sc_final", "misc", "batch_step", "nif2", "serve_step"};
static_assert(ST_LFOLD + 1 == PC_WIRING, "one profiling class per step kind");

struct ProfRec {
    int cls;
    hipEvent_t a, b;
    double bytes, mods;
    int sclass;  // size class of the launch (ceil log2 of its work items), -1 if none
};

// One timed launch, kept while per-launch records are asked for.
struct LaunchRec {
    int cls, sclass;
    float ms;
    double bytes, mods;
};

struct Profiler {
    std::mutex mu;
    bool on = false;
    bool keep = false;  // keep per-launch records (gkr_profile_launches)
    std::vector<ProfRec> recs;
    std::vector<LaunchRec> launches;
    std::vector<hipEvent_t> pool;
    double ms[PC_COUNT] = {0};
    uint64_t n[PC_COUNT] = {0};
    double bytes[PC_COUNT] = {0};
    double mods[PC_COUNT] = {0};

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
} g_prof;

// Events timing one dispatch when profiling is on (NULL otherwise); the
// record is kept for gkr_profile_read.
bool prof_pair(int cls, double bytes, hipEvent_t *a, hipEvent_t *b, double mods = 0, int sclass = -1) {
    *a = *b = nullptr;
    if (!g_prof.on) return false;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    *a = g_prof.get();
    *b = g_prof.get();
    if (!*a || !*b) return false;
    g_prof.recs.push_back({cls, *a, *b, bytes, mods, sclass});
    return true;
}

// Brackets one launch with events when profiling is on.
struct Scope {
    int cls;
    double bytes;
    hipStream_t st;
    hipEvent_t a = nullptr;
    Scope(int c, hipStream_t s, double b) : cls(c), bytes(b), st(s) {
        if (!g_prof.on) return;
        std::lock_guard<std::mutex> lk(g_prof.mu);
        a = g_prof.get();
        if (a) (void)hipEventRecord(a, st);
    }
    ~Scope() {
        if (!a) return;
        std::lock_guard<std::mutex> lk(g_prof.mu);
        hipEvent_t b = g_prof.get();
        if (!b) return;
        (void)hipEventRecord(b, st);
        g_prof.recs.push_back({cls, a, b, bytes, 0.0, -1});
    }
};

}  // namespace

static int prof_collect();

extern "C" int gkr_profile_enable(int flag) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    // launches recorded so far are kept (or not) as the setting they ran under says
    const int rc = prof_collect();
    g_prof.on = flag != 0;
    g_prof.keep = flag == 2;
    return rc;
}

// Timings of the recorded launches into the per-class totals (and the
// per-launch list while it is kept).
static int prof_collect() {
    for (auto &r : g_prof.recs) {
        HIP_TRY(hipEventSynchronize(r.b));
        float t = 0;
        HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        g_prof.ms[r.cls] += t;
        g_prof.n[r.cls] += 1;
        g_prof.bytes[r.cls] += r.bytes;
        g_prof.mods[r.cls] += r.mods;
        if (g_prof.keep) g_prof.launches.push_back({r.cls, r.sclass, t, r.bytes, r.mods});
        g_prof.pool.push_back(r.a);
        g_prof.pool.push_back(r.b);
    }
    g_prof.recs.clear();
    return GKR_OK;
}

extern "C" int gkr_profile_read(uint32_t *n_classes, const char **names, double *ms,
                                uint64_t *launches, double *bytes, double *mods) {
    if (!n_classes) return fail(GKR_ERR_INVALID, "n_classes is NULL");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    const int rc = prof_collect();
    if (rc) return rc;
    uint32_t cap = *n_classes;
    *n_classes = PC_COUNT;
    const bool totals = ms || launches || bytes || mods;  // names alone: nothing is reset
    for (uint32_t k = 0; k < PC_COUNT && k < cap; k++) {
        if (names) names[k] = kProfNames[k];
        if (!totals) continue;
        if (ms) ms[k] = g_prof.ms[k];
        if (launches) launches[k] = g_prof.n[k];
        if (bytes) bytes[k] = g_prof.bytes[k];
        if (mods) mods[k] = g_prof.mods[k];
        g_prof.ms[k] = 0;
        g_prof.n[k] = 0;
        g_prof.bytes[k] = 0;
        g_prof.mods[k] = 0;
    }
    return GKR_OK;
}

extern "C" int gkr_profile_launches(uint64_t *n, int32_t *cls, int32_t *size_class, float *ms,
                                    double *bytes, double *mods) {
    if (!n) return fail(GKR_ERR_INVALID, "n is NULL");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    const int rc = prof_collect();
    if (rc) return rc;
    const uint64_t cap = *n, have = g_prof.launches.size();
    *n = have;
    if (!cls && !size_class && !ms && !bytes && !mods) return GKR_OK;  // count only
    for (uint64_t k = 0; k < have && k < cap; k++) {
        const LaunchRec &r = g_prof.launches[k];
        if (cls) cls[k] = r.cls;
        if (size_class) size_class[k] = r.sclass;
        if (ms) ms[k] = r.ms;
        if (bytes) bytes[k] = r.bytes;
        if (mods) mods[k] = r.mods;
    }
    g_prof.launches.clear();
    return GKR_OK;
}

// ------------------------------------------------------------------ helpers

namespace {

u32 log2ceil(u64 n) {
    u32 s = 0;
    while ((1ull << s) < n) s++;
    return s;
}

// The library's own stream per device, used when the caller passes NULL.
hipStream_t default_stream() {
    static std::mutex mu;
    static std::vector<hipStream_t> streams;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
    if (!streams[dev]) {
        if (hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
            return nullptr;
    }
    return streams[dev];
}

hipStream_t pick_stream(void *s) { return s ? (hipStream_t)s : default_stream(); }

// Bump allocator over one device allocation; every piece 256-byte aligned.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    template <class T>
    T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        if (base == nullptr) {  // sizing pass
            used += bytes;
            return nullptr;
        }
        T *p = reinterpret_cast<T *>(base + used);
        used += bytes;
        return p;
    }
};

constexpr u32 HALF_MAX = 1u << 16;  // eq half tables: at most 2^16 entries
// Up to this many gates an omega round folds its table itself (two extra
// products per gate) instead of a separate fold step.
constexpr u32 INLINE_FOLD_MAX_GATES = 1u << 19;

void split_half(u32 s, u32 *L) { *L = s / 2; }

// Line-step shape for s' variables: lanes 2^L, waves 2^M, steps 2^H.
void line_shape(u32 sp, u32 *L, u32 *M, u32 *H) {
    *L = std::min<u32>(6, sp);
    *M = std::min<u32>(sp - *L, 11);
    *H = sp - *L - *M;
}

}  // namespace

// ------------------------------------------------------------------ circuit

// ------------------------------------------------------------ launch shapes
//
// A grid step over `units` work items launches ceil(units / (SBLOCK q))
// workgroups, at most `cap`, with q (items per thread) and cap chosen per
// step kind and size class (ceil log2 of the units) by gkr_autotune; a class
// above the largest one measured for its kind takes that one's shape, the
// other classes it has not measured keep their defaults.  A shape code packs
// log2 q (bits 0-1) and log2 cap - 8 (bits 2-3): 16 candidates.
constexpr u32 CAP_MAX = 2048;
constexpr int NKIND = ST_WA0 + 1;
constexpr int NCLASS = 48;
constexpr u8 SHAPE_DEFAULT = 0xFF;
constexpr int NSHAPE = 16;
std::mutex g_tune_mu;
u8 g_tune[NKIND][NCLASS];
std::atomic<u32> g_tune_epoch{1};  // bumped when shapes change: plans are rebuilt
int g_force = -1;                  // while tuning: the shape of every tunable step

struct TuneInit {
    TuneInit() { memset(g_tune, SHAPE_DEFAULT, sizeof g_tune); }
} g_tune_init;

bool tunable(u32 kind) {
    switch (kind) {
        case ST_LOAD: case ST_EVAL: case ST_EQ: case ST_P: case ST_W: case ST_FOLD:
        case ST_LT: case ST_WAGG: case ST_WT0: case ST_WT: case ST_WA0:
            return true;
        default:
            return false;
    }
}

u32 size_class(u64 units) {
    u32 b = 0;
    while (b + 1 < NCLASS && (1ull << b) < units) b++;
    return b;
}

u32 grid_for(u32 kind, u64 units, u32 qdef) {
    u32 qlog = 0;
    while ((1u << qlog) < qdef) qlog++;
    u32 caplog = 9;  // 512 workgroups: two per CU
    int code = SHAPE_DEFAULT;
    if (tunable(kind)) code = g_force >= 0 ? g_force : g_tune[kind][size_class(units)];
    if (code == SHAPE_DEFAULT && g_force < 0 && tunable(kind)) {
        // a class above every class tuned for this kind takes the shape of
        // the largest tuned one (the wide launches of circuits larger than
        // the one tuned on)
        const u32 b = size_class(units);
        for (int k = NCLASS - 1; k >= 0; k--)
            if (g_tune[kind][k] != SHAPE_DEFAULT) {
                if ((u32)k < b) code = g_tune[kind][k];
                break;
            }
    }
    if (code != SHAPE_DEFAULT) {
        qlog = code & 3;
        caplog = 8 + ((code >> 2) & 3);
    }
    const u64 t = (units + (1ull << qlog) - 1) >> qlog;
    const u64 b = (t + SBLOCK - 1) / SBLOCK;
    return (u32)std::max<u64>(1, std::min<u64>(b, 1ull << caplog));
}

// Scratch of one proof on a circuit: the layer tables, the per-round tables
// of the sum-checks, the transcript, and the step program (descriptors and
// one-job launch entries) with every pointer bound to this scratch.
struct Workspace {
    void *mem = nullptr;
    std::vector<u64 *> V;  // per layer, 2^{s_i} values
    u64 *pA, *pB, *bA, *bB, *fA, *fB;
    u64 *w, *off;
    u64 *zlo, *zhi, *alo, *ahi, *blo, *bhi;
    u64 *llo, *lhl, *lhh;
    u64 *rowpool;        // every reducing step's rows, each at its own offset
    u64 *frec;           // records of p-phase finishes (C, z_j, z_{j+1})
    FinItem *d_items;    // the finish step's items
    TopLayer *d_top;     // descriptors of the layers ST_TOP runs
    u64 *msgs, *chals, *rngst, *zbuf, *state;
    u32 *flag;
    // omega phases over tables
    u64 *tA0, *tC0, *tA[2], *tC[2], *partA, *partC;
    StepDesc *d_steps;
    JobEntry *d_jobs;
    std::vector<StepDesc> steps;  // host copy of the program
    std::vector<int> pclass;      // profiling class of each step
    std::vector<double> pbytes;   // algorithmic bytes of each step
    std::vector<double> pmods;    // algorithmic modular products of each step
    std::vector<u64> punits;      // work items of each tunable step (0: not tunable)
    u32 epoch = 0;                // launch shapes the program was planned with
    u64 cap_rows = 0, cap_recs = 0, cap_items = 0;  // room carved for them
    hipGraph_t graph = nullptr;   // the proof's launches, captured once per plan
    hipGraphExec_t gexec = nullptr;
    u32 gepoch = 0;
    u64 *instage;  // host inputs land here
    size_t bytes = 0;  // device memory held
    u32 gen = 0;       // the circuit's generation when the workspace was made
    // Out-of-core proofs (Sec. 5.1.2, 5.1.3).  mode GKR_MEM_LAYER: V holds
    // every layer's table in pinned host memory and the steps use three
    // device slots (layer i's table in Vslot[i % 3]) and, for gate arrays in
    // host memory, two gate slots (layer i's block in Gslot[i % 2]); xfers
    // are the copies between them, on the copy stream cs.  GKR_MEM_MESSAGE:
    // the layer and round tables are in pinned host memory, read and written
    // in place by every message's kernels.
    int mode = GKR_MEM_RESIDENT;
    void *hmem = nullptr;  // pinned host part
    size_t hbytes = 0;
    u64 *Vslot[3] = {nullptr, nullptr, nullptr};
    char *Gslot[2] = {nullptr, nullptr};
    size_t gslot = 0;  // bytes of a gate slot
    struct Xfer {
        int after;   // step whose completion lets the copy start (-1: the proof's start)
        int before;  // step that waits for the copy
        void *dst;
        const void *src;
        size_t bytes;
        hipMemcpyKind kind;
    };
    std::vector<Xfer> xfers;  // in order of `after`
    hipStream_t cs = nullptr;
    std::vector<hipEvent_t> xev;  // per transfer: step done (on the proof's stream), copy done (on cs)
    hipEvent_t ev_begin = nullptr, ev_join = nullptr;
    u64 *h_msgs = nullptr, *h_chals = nullptr, *h_setup = nullptr;  // pinned staging
};

struct gkr_circuit {
    int device = 0;
    u32 L = 0;  // layers incl. input
    std::vector<u32> S, s;
    std::vector<int> kind;
    std::vector<int> form;  // GKR_WIRING_* per layer
    std::vector<u8 *> type;
    std::vector<u32 *> in1, in2;
    void *soa = nullptr;
    u64 n_msgs = 0, n_chals = 0, gates = 0, rounds = 0;
    std::vector<u64> mo, co;  // per layer: offset of its round messages / challenges
    u32 smax = 0, spmax = 0;
    u64 gmax = 0;
    u64 line_lo = 1, line_hl = 1, line_hh = 1;  // table sizes (entries)
    u64 nch_max = 1;  // most chunks of a phase grouping
    size_t ws_bytes[3] = {0, 0, 0};  // device bytes of one workspace per memory mode (0: not yet sized)
    std::mutex mu;
    Workspace *ws = nullptr;
    int omega_algo = GKR_OMEGA_TABLES;
    u32 gen = 1;  // bumped when its workspaces go stale (algorithm change)
    std::vector<std::vector<u32>> h_in1, h_in2;  // host copies of the wires (grouping)
    std::vector<std::vector<u8>> h_type;         // host gate types of mixed layers (else empty)
    struct Group {  // gates of a layer grouped by the wire a phase binds
        u32 *perm = nullptr, *cstart = nullptr, *xch = nullptr;
        u32 *rowptr = nullptr;  // wire x's gates: sorted positions [rowptr[x], rowptr[x+1])
        u32 *oths = nullptr;    // other wire of each gate, in sorted order
        u8 *types = nullptr;    // gate types in sorted order (mixed layers)
        u32 *tch = nullptr;     // tiles of whole chunks (at most TILE_POS positions each)
        u32 nch = 0, ntiles = 0;
        bool single = false;    // every wire carries at most one chunk
    };
    std::vector<Group> grp[2];  // [phase - 1][layer], built with the first table workspace
    void *gmem = nullptr;       // memory of the groups (allocated with the first table workspace)
    bool grouped = false;       // grp[][] sized (chunk counts, single flags)
    // Per layer i: entries of its omega phases' tables that can be nonzero,
    // max(S_{i+1}, 1 + the largest wire read); entries above are zero at
    // every level (no gate reads them and V_{i+1} is zero there).
    std::vector<u64> wlive;
    // Where the gate arrays (soa, gmem) live: device memory, or pinned host
    // memory when the circuit's proofs run out of core; and the byte ranges
    // of each layer's block in them (layer i: [off[i], off[i+1])).
    bool gates_host = false;
    std::vector<size_t> soa_off, g_off;
    int mem_mode = GKR_MEM_RESIDENT;  // how gkr_prove places a proof's tables
};

// ---------------------------------------------------------------------------
// Wiring predicates in closed form (the verifier's add~ and mult~ at a point,
// Sec. 3.1).  For the layer shapes below the predicate
//   W(a, b, c) = sum_{g < S} chi_g(a) chi_{in1(g)}(b) chi_{in2(g)}(c)
// is a product over the bits of g, so the verifier evaluates it with
// O(s_i + s_{i+1}) field operations instead of a pass over the gates.

// The shape of a layer's wiring (all gates of one type), from one pass.
static int wiring_form(u32 S, const uint32_t *in1, const uint32_t *in2) {
    bool tree = true, square = true;
    for (u32 g = 0; g < S && (tree || square); g++) {
        tree = tree && in1[g] == 2ull * g && in2[g] == 2ull * g + 1;
        square = square && in1[g] == g && in2[g] == g;
    }
    if (tree) return GKR_WIRING_TREE;
    if (square) return GKR_WIRING_SQUARE;
    const u32 n = log2ceil(S) / 3;  // S = N^3, N = 2^n
    if (S != 1u << (3 * n) || n > 10) return GKR_WIRING_GATES;
    const u64 N = 1ull << n;
    for (u64 g = 0; g < S; g++) {
        const u64 i = g >> (2 * n), j = (g >> n) & (N - 1), k = g & (N - 1);
        if (in1[g] != i * N + k || in2[g] != N * N + k * N + j) return GKR_WIRING_GATES;
    }
    return GKR_WIRING_MATMULT;
}

// sum over g in [0, S) of prod_{k < K} f[k][bit k of g], for S <= 2^K: the
// g below S share S's bits above some bit j where S has a 1 and g a 0, and
// range freely below it.
static u64 bits_sum(const std::vector<std::array<u64, 2>> &f, u64 S) {
    using namespace fp;
    const u32 K = (u32)f.size();
    std::vector<u64> low(K + 1);  // low[j] = prod_{k < j} (f[k][0] + f[k][1])
    low[0] = 1;
    for (u32 k = 0; k < K; k++) low[k + 1] = mul(low[k], add(f[k][0], f[k][1]));
    if (S == 1ull << K) return low[K];
    u64 tot = 0, pre = 1;
    for (int j = (int)K - 1; j >= 0; j--) {
        if ((S >> j) & 1) {
            tot = add(tot, mul(pre, mul(f[j][0], low[j])));
            pre = mul(pre, f[j][1]);
        } else {
            pre = mul(pre, f[j][0]);
        }
    }
    return tot;
}

// W(a, b, c) for a layer of S gates in closed form; a has s coordinates, b
// and c sp each.  Wire bits beyond a point's coordinates are zero.
static u64 wiring_closed(int form, u32 S, u32 s, u32 sp, const u64 *a, const u64 *b, const u64 *c) {
    using namespace fp;
    auto side = [](const u64 *v, u32 m, u32 len, u32 x) -> u64 { return m < len ? eqbit(x, v[m]) : (x ? 0 : 1); };
    auto E3 = [](u64 x, u64 y, u64 w) {  // sum over t in {0,1} of eq(x,t) eq(y,t) eq(w,t)
        return add(mul(mul(x, y), w), mul(mul(sub(1, x), sub(1, y)), sub(1, w)));
    };
    u64 v = 1;
    u32 top = 0;  // b, c coordinates from here on take bit 0
    if (form == GKR_WIRING_TREE || form == GKR_WIRING_SQUARE) {
        const u32 sh = form == GKR_WIRING_TREE ? 1 : 0;  // g's bit k is bit k + sh of both wires
        std::vector<std::array<u64, 2>> f(s);
        for (u32 k = 0; k < s; k++)
            for (u32 x = 0; x < 2; x++)
                f[k][x] = mul(eqbit(x, a[k]), mul(side(b, k + sh, sp, x), side(c, k + sh, sp, x)));
        v = bits_sum(f, S);
        if (sh) v = mul(v, mul(sub(1, b[0]), c[0]));  // in1 even, in2 odd
        top = s + sh;
    } else {  // MatMult: g = (iN + j)N + k, in1 = iN + k, in2 = N^2 + kN + j
        const u32 n = s / 3;
        for (u32 t = 0; t < n; t++) {
            v = mul(v, E3(a[t], b[t], c[n + t]));          // k
            v = mul(v, eq(a[n + t], c[t]));                // j
            v = mul(v, eq(a[2 * n + t], b[n + t]));        // i
        }
        v = mul(v, mul(sub(1, b[2 * n]), c[2 * n]));       // A's half, B's half
        top = 2 * n + 1;
    }
    for (u32 m = top; m < sp; m++) v = mul(v, mul(sub(1, b[m]), sub(1, c[m])));
    return v;
}

static std::atomic<int> g_closed_forms{1};

extern "C" int gkr_circuit_wiring(const gkr_circuit *c, uint32_t layer, int *form) {
    if (!c || !form) return fail(GKR_ERR_INVALID, "NULL argument");
    if (layer + 1 >= c->L) return fail(GKR_ERR_INVALID, "layer out of range");
    *form = c->form[layer];
    return GKR_OK;
}

extern "C" int gkr_verify_closed_forms(int enable) { return g_closed_forms.exchange(enable ? 1 : 0); }

extern "C" int gkr_circuit_create(uint32_t num_layers, const uint32_t *layer_sizes,
                                  const uint8_t *const *gate_type, const uint32_t *const *in1,
                                  const uint32_t *const *in2, gkr_circuit **out) {
    if (!out) return fail(GKR_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (num_layers < 2) return fail(GKR_ERR_INVALID, "need at least 2 layers");
    if (!layer_sizes || !gate_type || !in1 || !in2) return fail(GKR_ERR_INVALID, "NULL array");
    for (u32 i = 0; i < num_layers; i++) {
        if (layer_sizes[i] == 0 || layer_sizes[i] >= (1u << 31))
            return fail(GKR_ERR_INVALID, "layer size must be in [1, 2^31)");
    }
    std::unique_ptr<gkr_circuit> c(new gkr_circuit());
    HIP_TRY(hipGetDevice(&c->device));
    c->L = num_layers;
    c->S.assign(layer_sizes, layer_sizes + num_layers);
    c->s.resize(num_layers);
    for (u32 i = 0; i < num_layers; i++) {
        c->s[i] = log2ceil(c->S[i]);
        c->gates += c->S[i];
        c->smax = std::max(c->smax, c->s[i]);
        c->gmax = std::max<u64>(c->gmax, c->S[i]);
    }
    const u32 d = num_layers - 1;
    c->kind.resize(d);
    c->form.resize(d);
    size_t soa_bytes = 0;
    for (u32 i = 0; i < d; i++) {
        if (!gate_type[i] || !in1[i] || !in2[i]) return fail(GKR_ERR_INVALID, "NULL layer array");
        const u64 lim = 1ull << c->s[i + 1];
        bool any_add = false, any_mul = false;
        for (u32 g = 0; g < c->S[i]; g++) {
            if (gate_type[i][g] > 1) return fail(GKR_ERR_INVALID, "gate type must be 0 or 1");
            if (in1[i][g] >= lim || in2[i][g] >= lim)
                return fail(GKR_ERR_INVALID, "wire beyond the padded next layer");
            (gate_type[i][g] ? any_mul : any_add) = true;
        }
        c->kind[i] = any_add && any_mul ? KIND_MIXED : (any_mul ? KIND_MUL : KIND_ADD);
        c->form[i] = c->kind[i] == KIND_MIXED ? GKR_WIRING_GATES : wiring_form(c->S[i], in1[i], in2[i]);
        size_t n = c->S[i];
        soa_bytes += ((n * 4 + 255) & ~size_t(255)) * 2;
        if (c->kind[i] == KIND_MIXED) soa_bytes += (n + 255) & ~size_t(255);
    }
    // transcript layout
    c->n_msgs = c->S[0];
    c->n_chals = c->s[0];
    c->mo.resize(d);
    c->co.resize(d);
    for (u32 i = 0; i < d; i++) {
        const u64 n = c->s[i] + 2ull * c->s[i + 1];
        const u32 sp = c->s[i + 1];
        c->mo[i] = c->n_msgs;
        c->co[i] = c->n_chals;
        c->n_msgs += 3 * n + 2 + (sp >= 2 ? sp - 1 : 0);
        c->n_chals += n + 1;
        c->rounds += n;
        c->spmax = std::max(c->spmax, sp);
        if (sp >= 2) {
            u32 Ll, M, H;
            line_shape(sp, &Ll, &M, &H);
            c->line_lo = std::max<u64>(c->line_lo, (u64)(sp - 1) << Ll);
            c->line_hl = std::max<u64>(c->line_hl, (u64)(sp - 1) << M);
            c->line_hh = std::max<u64>(c->line_hh, (u64)(sp - 1) << H);
        }
    }
    // struct-of-arrays upload
    HIP_TRY(hipMalloc(&c->soa, std::max<size_t>(soa_bytes, 256)));
    char *p = (char *)c->soa;
    c->type.assign(d, nullptr);
    c->in1.assign(d, nullptr);
    c->in2.assign(d, nullptr);
    c->soa_off.assign(d + 1, 0);
    for (u32 i = 0; i < d; i++) {
        size_t n = c->S[i];
        c->soa_off[i] = (size_t)(p - (char *)c->soa);
        c->in1[i] = (u32 *)p;
        p += (n * 4 + 255) & ~size_t(255);
        c->in2[i] = (u32 *)p;
        p += (n * 4 + 255) & ~size_t(255);
        HIP_TRY(hipMemcpy(c->in1[i], in1[i], n * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->in2[i], in2[i], n * 4, hipMemcpyHostToDevice));
        c->h_in1.emplace_back(in1[i], in1[i] + n);
        c->h_in2.emplace_back(in2[i], in2[i] + n);
        c->h_type.emplace_back();
        if (c->kind[i] == KIND_MIXED) {
            c->h_type.back().assign(gate_type[i], gate_type[i] + n);
            c->type[i] = (u8 *)p;
            p += (n + 255) & ~size_t(255);
            HIP_TRY(hipMemcpy(c->type[i], gate_type[i], n, hipMemcpyHostToDevice));
        }
    }
    c->soa_off[d] = (size_t)(p - (char *)c->soa);
    *out = c.release();
    return GKR_OK;
}

// Gate arrays and out-of-core tables: device memory, or pinned host memory
// that kernels read and write in place through its device mapping.
static hipError_t mem_alloc(bool host, size_t bytes, void **p) {
    *p = nullptr;
    if (!host) return hipMalloc(p, bytes);
    void *h = nullptr;
    hipError_t e = hipHostMalloc(&h, bytes, hipHostMallocMapped);
    if (e != hipSuccess) return e;
    void *d = nullptr;
    e = hipHostGetDevicePointer(&d, h, 0);
    if (e != hipSuccess || d != h) {  // kernels take the host address as is
        (void)hipHostFree(h);
        return e != hipSuccess ? e : hipErrorInvalidValue;
    }
    *p = h;
    return hipSuccess;
}

static void gate_free(bool host, void *p) {
    if (!p) return;
    if (host)
        (void)hipHostFree(p);
    else
        (void)hipFree(p);
}

static void free_workspace(Workspace *ws) {
    if (!ws) return;
    if (ws->gexec) (void)hipGraphExecDestroy(ws->gexec);
    if (ws->graph) (void)hipGraphDestroy(ws->graph);
    if (ws->cs) (void)hipStreamSynchronize(ws->cs);
    for (hipEvent_t e : ws->xev) (void)hipEventDestroy(e);
    if (ws->ev_begin) (void)hipEventDestroy(ws->ev_begin);
    if (ws->ev_join) (void)hipEventDestroy(ws->ev_join);
    if (ws->cs) (void)hipStreamDestroy(ws->cs);
    if (ws->mem) (void)hipFree(ws->mem);
    if (ws->hmem) (void)hipHostFree(ws->hmem);
    if (ws->h_msgs) (void)hipHostFree(ws->h_msgs);
    if (ws->h_chals) (void)hipHostFree(ws->h_chals);
    if (ws->h_setup) (void)hipHostFree(ws->h_setup);
    delete ws;
}

static void drop_batches_of(const gkr_circuit *c);
static void drop_served_scratch_of(const gkr_circuit *c);

extern "C" void gkr_circuit_destroy(gkr_circuit *c) {
    if (!c) return;
    drop_batches_of(c);
    drop_served_scratch_of(c);
    free_workspace(c->ws);
    gate_free(c->gates_host, c->gmem);
    gate_free(c->gates_host, c->soa);
    delete c;
}

extern "C" int gkr_circuit_set_algorithm(gkr_circuit *c, int omega_algo) {
    if (!c) return fail(GKR_ERR_INVALID, "circuit is NULL");
    if (omega_algo != GKR_OMEGA_GATES && omega_algo != GKR_OMEGA_TABLES && omega_algo != GKR_OMEGA_TABLES_STEPWISE)
        return fail(GKR_ERR_INVALID, "unknown omega-phase algorithm");
    bool changed = false;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        if (c->omega_algo != omega_algo) {
            free_workspace(c->ws);  // the step program is rebuilt on the next proof
            c->ws = nullptr;
            c->omega_algo = omega_algo;
            for (size_t &b : c->ws_bytes) b = 0;
            c->gen++;  // pooled server scratch of the old program is discarded
            changed = true;
        }
    }
    if (changed) {  // (a server takes its own lock before the circuit's)
        drop_batches_of(c);
        drop_served_scratch_of(c);
    }
    return GKR_OK;
}

extern "C" int gkr_transcript_size(const gkr_circuit *c, uint64_t *n_msgs, uint64_t *n_chals) {
    if (!c) return fail(GKR_ERR_INVALID, "circuit is NULL");
    if (n_msgs) *n_msgs = c->n_msgs;
    if (n_chals) *n_chals = c->n_chals;
    return GKR_OK;
}

extern "C" int gkr_circuit_info(const gkr_circuit *c, uint64_t *gates, uint64_t *rounds,
                                uint32_t *num_layers) {
    if (!c) return fail(GKR_ERR_INVALID, "circuit is NULL");
    if (gates) *gates = c->gates;
    if (rounds) *rounds = c->rounds;
    if (num_layers) *num_layers = c->L;
    return GKR_OK;
}

// Gates of a layer grouped by the wire x a phase binds: perm lists the
// gates in order of x (counting sort), cut into chunks of at most
// GROUP_CHUNK gates of one wire; chunks of wire x are [xch[x], xch[x+1]).
// A wire of more than HEAVY_WIRE gates (pattern matching's pattern values
// feed 2^18) is cut into chunks of BIG_CHUNK gates instead, each summed by
// a whole wave, so that the chunks of one wire stay few.
constexpr u32 GROUP_CHUNK = 32;
constexpr u32 HEAVY_WIRE = 64 * GROUP_CHUNK;
constexpr u32 BIG_CHUNK = 512;
__host__ __device__ constexpr u32 chunk_of(u64 gates) { return gates > HEAVY_WIRE ? BIG_CHUNK : GROUP_CHUNK; }
struct HostGroup {
    std::vector<u32> perm, cstart, xch, rowptr, oths, tch;
    std::vector<u8> types;
};


// Counting sort of the gates by their wire idx (stable): positions, the
// other wire and the type in that order, chunks of <= GROUP_CHUNK gates of
// one wire.
static void build_group(const std::vector<u32> &idx, const std::vector<u32> &other,
                        const std::vector<u8> &type, u64 N, HostGroup &G) {
    const u64 S = idx.size();
    std::vector<u32> &rowptr = G.rowptr;
    rowptr.assign(N + 1, 0);
    for (u64 g = 0; g < S; g++) rowptr[idx[g] + 1]++;
    for (u64 x = 0; x < N; x++) rowptr[x + 1] += rowptr[x];
    G.perm.assign(S, 0);
    std::vector<u32> fill(rowptr.begin(), rowptr.end() - 1);
    for (u64 g = 0; g < S; g++) G.perm[fill[idx[g]]++] = (u32)g;
    G.oths.resize(S);
    for (u64 p = 0; p < S; p++) G.oths[p] = other[G.perm[p]];
    G.types.clear();
    if (!type.empty()) {
        G.types.resize(S);
        for (u64 p = 0; p < S; p++) G.types[p] = type[G.perm[p]];
    }
    G.xch.assign(N + 1, 0);
    G.cstart.clear();
    for (u64 x = 0; x < N; x++) {
        G.xch[x] = (u32)G.cstart.size();
        const u32 csz = chunk_of(rowptr[x + 1] - rowptr[x]);
        for (u32 p = rowptr[x]; p < rowptr[x + 1]; p += csz) G.cstart.push_back(p);
    }
    G.xch[N] = (u32)G.cstart.size();
    G.cstart.push_back((u32)S);
    // a chunk that would carry the open tile past TILE_POS positions opens a
    // tile of its own (a big chunk always stands alone in its tile)
    G.tch.assign(1, 0);
    const size_t nch = G.cstart.size() - 1;
    for (size_t ch = 0; ch < nch; ch++)
        if (ch > G.tch.back() && G.cstart[ch + 1] - G.cstart[G.tch.back()] > TILE_POS) G.tch.push_back((u32)ch);
    G.tch.push_back((u32)nch);
}

// Lay out (or size, when a.base is NULL) a proof's scratch.
// What a step program needs besides its steps: row storage, p-phase
// records and finish items (the same for every launch shape).
struct PlanSizes {
    size_t nsteps;
    u64 rows, recs, items;
};

// Bytes of the largest per-layer block a gate slot receives: the struct of
// arrays for evaluation, and the groups (tables algorithm) or the struct of
// arrays (per-gate rounds) for the layer's sum-check.
static size_t gate_block_max(const gkr_circuit *c) {
    size_t m = 0;
    for (u32 i = 0; i + 1 < c->L; i++) {
        m = std::max(m, c->soa_off[i + 1] - c->soa_off[i]);
        if (c->omega_algo != GKR_OMEGA_GATES) m = std::max(m, c->g_off[i + 1] - c->g_off[i]);
    }
    return m;
}

// Lay out (or size, when the arenas' bases are NULL) a proof's scratch in
// device memory (a) and pinned host memory (h) as w.mode places it:
// resident, every table on the device; per layer, the layer tables in host
// memory with three device slots for them (and two for the gate arrays
// when those are in host memory); per message, the layer and round tables
// in host memory.  Small state (eq half tables, rows, transcript, step
// program) is always on the device.
static void carve(const gkr_circuit *c, Arena &a, Arena &h, Workspace &w, const PlanSizes &ps) {
    const size_t nsteps = ps.nsteps;
    const int mode = w.mode;
    Arena &vt = mode == GKR_MEM_RESIDENT ? a : h;  // layer value tables
    Arena &rt = mode == GKR_MEM_MESSAGE ? h : a;   // round tables
    w.V.assign(c->L, nullptr);
    for (u32 i = 0; i < c->L; i++) w.V[i] = vt.take<u64>(1ull << c->s[i]);
    if (mode == GKR_MEM_LAYER) {
        for (int k = 0; k < 3; k++) w.Vslot[k] = a.take<u64>(1ull << c->smax);
        w.gslot = c->gates_host ? gate_block_max(c) : 0;
        for (int k = 0; k < 2; k++) w.Gslot[k] = w.gslot ? a.take<char>(w.gslot) : nullptr;
    }
    const u64 half = std::max<u64>(1ull << (c->smax ? c->smax - 1 : 0), 2);
    w.pA = rt.take<u64>(half);
    w.pB = rt.take<u64>(half);
    w.bA = rt.take<u64>(half);
    w.bB = rt.take<u64>(half);
    w.fA = rt.take<u64>(half);
    w.fB = rt.take<u64>(half);
    const bool gates = c->omega_algo == GKR_OMEGA_GATES;
    w.w = rt.take<u64>(gates ? c->gmax : 1);   // per-gate weights: per-gate rounds only
    w.off = rt.take<u64>(gates ? c->gmax : 1);
    w.zlo = a.take<u64>(HALF_MAX);
    w.zhi = a.take<u64>(HALF_MAX);
    w.alo = a.take<u64>(HALF_MAX);
    w.ahi = a.take<u64>(HALF_MAX);
    w.blo = a.take<u64>(HALF_MAX);
    w.bhi = a.take<u64>(HALF_MAX);
    w.llo = a.take<u64>(c->line_lo);
    w.lhl = a.take<u64>(c->line_hl);
    w.lhh = a.take<u64>(c->line_hh);
    w.rowpool = a.take<u64>(std::max<u64>(ps.rows, 1));
    w.frec = a.take<u64>(std::max<u64>(ps.recs, 1));
    w.d_items = a.take<FinItem>(std::max<u64>(ps.items, 1));
    w.d_top = a.take<TopLayer>(c->L);
    w.msgs = a.take<u64>(c->n_msgs);
    w.chals = a.take<u64>(std::max<u64>(c->n_chals, 1));
    w.rngst = a.take<u64>(c->n_chals + 1);
    w.zbuf = a.take<u64>(64);
    w.state = a.take<u64>(8);
    w.flag = a.take<u32>(1);
    w.instage = vt.take<u64>(c->S[c->L - 1]);
    w.d_steps = a.take<StepDesc>(nsteps);
    w.d_jobs = a.take<JobEntry>(2 * nsteps);
    if (c->omega_algo != GKR_OMEGA_GATES) {
        const u64 N = 1ull << c->spmax;
        w.tA0 = rt.take<u64>(N);
        w.tC0 = rt.take<u64>(N);
        w.tA[0] = rt.take<u64>(std::max<u64>(N / 2, 2));
        w.tA[1] = rt.take<u64>(std::max<u64>(N / 2, 2));
        w.tC[0] = rt.take<u64>(std::max<u64>(N / 2, 2));
        w.tC[1] = rt.take<u64>(std::max<u64>(N / 2, 2));
        w.partA = rt.take<u64>(c->nch_max);
        w.partC = rt.take<u64>(c->nch_max);
    }
}


// Builds a proof's step program.  With `ws` NULL it only counts the steps.
// Leading layers ST_TOP runs: layer i < K with 2^s_i and 2^s_{i+1} at most
// TAIL_LIM entries, s_{i+1} >= 1 and one chunk of gates on every wire of
// both omega phases (the tables algorithm; not with the per-layer copies of
// GKR_MEM_LAYER, whose slots hold three value tables).
static u32 top_layers(const gkr_circuit *c) {
    if (c->omega_algo != GKR_OMEGA_TABLES || c->mem_mode == GKR_MEM_LAYER) return 0;
    const u32 d = c->L - 1;
    u32 K = 0;
    while (K < d && (1ull << c->s[K]) <= (u64)TAIL_LIM && c->s[K + 1] >= 1 &&
           (1ull << c->s[K + 1]) <= (u64)TAIL_LIM && c->grp[0][K].single && c->grp[1][K].single)
        K++;
    return K;
}

struct Planner {
    const gkr_circuit *c;
    Workspace *w;

    std::vector<StepDesc> out;
    std::vector<int> cls;
    std::vector<double> bytes;
    std::vector<double> mods;   // algorithmic 64 x 64-bit modular products of each step
    std::vector<u64> units;
    std::vector<FinItem> items;
    std::vector<TopLayer> top;  // the layers ST_TOP runs
    u64 rows_used = 0, recs_used = 0;
    ProofPtrs pp{};
    // step indices: evaluation of layer i, first and last step of its sum-check
    std::vector<int> eval_at, sc_first, sc_last;

    // Layer i's gate arrays as its steps see them: in place, or in gate
    // slot i % 2 when the workspace stages host gate arrays layer by layer.
    template <typename T>
    T *soa_at(u32 i, T *p) const {
        if (!w || !p || !w->gslot) return p;
        return (T *)(w->Gslot[i % 2] + ((const char *)p - ((const char *)c->soa + c->soa_off[i])));
    }
    template <typename T>
    T *grp_at(u32 i, T *p) const {
        if (!w || !p || !w->gslot) return p;
        return (T *)(w->Gslot[i % 2] + ((const char *)p - ((const char *)c->gmem + c->g_off[i])));
    }
    gkr_circuit::Group group(u32 ph, u32 i) const {
        gkr_circuit::Group g = c->grp[ph - 1][i];
        g.perm = grp_at(i, g.perm);
        g.cstart = grp_at(i, g.cstart);
        g.xch = grp_at(i, g.xch);
        g.rowptr = grp_at(i, g.rowptr);
        g.oths = grp_at(i, g.oths);
        g.tch = grp_at(i, g.tch);
        g.types = grp_at(i, g.types);
        return g;
    }

    PlanSizes sizes() const { return PlanSizes{out.size(), rows_used, recs_used, items.size()}; }

    StepDesc &add(u32 kind, u32 nblocks, double nbytes) {
        StepDesc s;
        memset(&s, 0, sizeof s);
        s.kind = kind;
        s.nblocks = nblocks;
        s.fin.kind = FIN_NONE;
        s.fin.draw = -1;
        s.pp = pp;
        out.push_back(s);
        cls.push_back(PC_STEP + (int)kind);
        bytes.push_back(nbytes);
        mods.push_back(0);
        units.push_back(0);
        return out.back();
    }
    // A grid step over n work items, qdef items per thread by default.
    StepDesc &addg(u32 kind, u64 n, u32 qdef, double nbytes) {
        StepDesc &s = add(kind, grid_for(kind, n, qdef), nbytes);
        if (tunable(kind)) units.back() = std::max<u64>(n, 1);
        return s;
    }
    // The step just added writes K-value rows: room for as many workgroups
    // as any launch shape gives it (q = 1, the largest cap), so a re-plan
    // with other shapes keeps every offset.
    void reduces(u32 K) {
        StepDesc &s = out.back();
        s.reduces = 1;
        s.K = K;
        const u64 n = units.back();
        const u64 most = n ? std::min<u64>(CAP_MAX, std::max<u64>(1, (n + SBLOCK - 1) / SBLOCK)) : s.nblocks;
        s.rows = w ? w->rowpool + rows_used : nullptr;
        rows_used += std::max<u64>(most, s.nblocks) * ROW_STRIDE;
    }
    // Finish info for a step that follows a reducing step (p-phase finishes
    // get a record slot).
    Fin fin_of_prev(u32 kind) {
        Fin f;
        memset(&f, 0, sizeof f);
        f.kind = kind;
        f.draw = -1;
        const StepDesc &p = out.back();
        f.rows = p.rows;
        f.nrows = p.nblocks;
        if (kind == FIN_P || kind == FIN_P2) {
            f.rec = w ? w->frec + recs_used : nullptr;
            recs_used += 3;
        }
        return f;
    }
    // The finish step: one item per message (per chunk of line values).
    void add_finish() {
        for (const StepDesc &sd : out) {
            const Fin &f = sd.fin;
            if (f.kind == FIN_NONE) continue;
            if (f.kind == FIN_LINE) {
                for (u32 q = 0; q * f.ch < f.T; q++)
                    items.push_back(FinItem{FIN_LINE, f.chunk_blocks, f.rows ? f.rows + (u64)q * f.chunk_blocks * ROW_STRIDE : nullptr,
                                            f.msg ? f.msg + q * f.ch : nullptr, nullptr, -1,
                                            std::min<u32>(f.ch, f.T - q * f.ch)});
                continue;
            }
            items.push_back(FinItem{f.kind, f.nrows, f.rows, f.msg, f.rec, f.draw + 0, 0});
        }
        if (items.empty()) return;
        double nbytes = 0;
        for (const FinItem &it : items)
            nbytes += it.nrows * 8.0 * (it.kind == FIN_P ? 2 : it.kind == FIN_P2 ? 6 : it.kind == FIN_W ? 4
                                        : it.kind == FIN_T ? 3 : it.kind == FIN_T2 ? 12 : LINE_CHUNK);
        StepDesc &s = add(ST_FINISH, (u32)items.size(), nbytes);
        s.u.finish = FinishArgs{w ? w->d_items : nullptr, w ? w->chals : nullptr};
    }

    void build() {
        const u32 d = c->L - 1;
        if (w) pp = ProofPtrs{w->msgs, w->chals, w->rngst, w->zbuf, w->state};
        // layer i's value table: its own, or slot i % 3 (per-layer staging)
        auto V = [&](u32 i) -> u64 * {
            return w ? (w->mode == GKR_MEM_LAYER ? w->Vslot[i % 3] : w->V[i]) : nullptr;
        };
        eval_at.assign(d, -1);
        sc_first.assign(d, -1);
        sc_last.assign(d, -1);
        auto P_ = [&](u64 *p) -> u64 * { return w ? p : nullptr; };
        {
            const u64 Sd = c->S[d], npad = 1ull << c->s[d];
            StepDesc &s = addg(ST_LOAD, npad, 4, Sd * 8.0 + npad * 8.0);
            s.u.load = LoadArgs{c->S[d], npad, V(d)};
        }
        // circuit evaluation (a3), layer d-1 down to 0; the first K layers
        // (run by ST_TOP, which evaluates them and starts the proof itself)
        // down to K
        const u32 K = top_layers(c);
        for (int i = (int)d - 1; i >= (int)K; i--) {
            const u64 S = c->S[i], npad = 1ull << c->s[i];
            eval_at[i] = (int)out.size();
            StepDesc &s = addg(ST_EVAL, npad, 4,
                              S * (8.0 + 16 + 8 + (c->kind[i] == KIND_MIXED)) + (npad - S) * 8.0);
            mods.back() = c->kind[i] == KIND_ADD ? 0.0 : (double)S;  // one product a MUL gate
            s.u.eval = EvalArgs{(u32)c->kind[i], c->S[i], npad, soa_at(i, c->type[i]), soa_at(i, c->in1[i]),
                                soa_at(i, c->in2[i]), V(i + 1), V(i)};
        }
        if (!K) {
            StepDesc &s = addg(ST_START, c->S[0], 1, c->S[0] * 16.0);
            s.u.start = StartArgs{c->s[0], c->S[0], V(0)};
        }
        Fin layer_end;  // how the previous layer is finished (line values, tau)
        memset(&layer_end, 0, sizeof layer_end);
        layer_end.kind = FIN_NONE;
        layer_end.draw = -1;
        // The first K layers run whole in one workgroup (ST_TOP); the step
        // after it draws the last one's tau.
        if (K) {
            top.clear();
            double nbytes = 0, nmods = 0;
            for (u32 i = 0; i < K; i++) {
                const u32 s = c->s[i], sp = c->s[i + 1];
                const u64 S = c->S[i], N = 1ull << sp;
                TopLayer t;
                memset(&t, 0, sizeof t);
                t.s = s;
                t.sp = sp;
                t.kind = (u32)c->kind[i];
                t.co = (u32)c->co[i];
                t.msg = w ? w->msgs + c->mo[i] : nullptr;
                t.Vn = V(i + 1);
                t.S = (u32)S;
                t.in1 = soa_at(i, c->in1[i]);
                t.in2 = soa_at(i, c->in2[i]);
                t.type = soa_at(i, c->type[i]);
                t.V = V(i);
                for (u32 ph = 1; ph <= 2; ph++) {
                    const gkr_circuit::Group &g = c->grp[ph - 1][i];
                    t.rowptr[ph - 1] = g.rowptr;
                    t.perm[ph - 1] = g.perm;
                    t.oths[ph - 1] = g.oths;
                    t.types[ph - 1] = g.types;
                }
                top.push_back(t);
                sc_first[i] = sc_last[i] = (int)out.size();
                // V_{i+1} 8 per entry; per phase: row pointers 4 per wire, sorted
                // index and other wire 8 per gate (+1 type)
                nbytes += 8.0 * N + 2 * (4.0 * (N + 1) + S * (8.0 + (c->kind[i] == KIND_MIXED)));
                // its evaluation: wires 8 (+1 type) per gate, V_i written
                nbytes += S * (8.0 + (c->kind[i] == KIND_MIXED)) + 8.0 * (1ull << s);
                nmods += c->kind[i] == KIND_ADD ? 0.0 : (double)S;
                // p-phase ~4 per entry of V_i; per gate 4 (phase 1) and 5 (phase 2);
                // per table entry 8 per phase; the line one product per point and entry
                nmods += 4.0 * (1ull << s) + 9.0 * S + 16.0 * N + (sp >= 2 ? 1.5 * (sp - 1) * N : 0.0);
            }
            StepDesc &st = add(ST_TOP, 1, nbytes);
            mods.back() = nmods;
            st.u.top = TopArgs{K, w ? w->d_top : nullptr, V(0)};
            const u32 i = K - 1, s = c->s[i], sp = c->s[i + 1], co = (u32)c->co[i];
            layer_end.kind = FIN_LINE;
            layer_end.draw = (i32)(co + s + 2 * sp);
            layer_end.sp = sp;
            layer_end.T = 0;  // h(2..sp) written by ST_TOP
            layer_end.bstar = w ? w->chals + co + s : nullptr;
            layer_end.cstar = w ? w->chals + co + s + sp : nullptr;
        }
        for (u32 i = K; i < d; i++) {
            if (i > 0) sc_last[i - 1] = (int)out.size() - 1;
            sc_first[i] = (int)out.size();
            const u32 s = c->s[i], sp = c->s[i + 1], S = c->S[i];
            const u32 n = s + 2 * sp;
            const int kind = c->kind[i];
            const u32 co = (u32)c->co[i];
            u64 *msg = w ? w->msgs + c->mo[i] : nullptr;
            u64 *chals = w ? w->chals : nullptr;
            u64 *vslot = w ? msg + 3ull * n : nullptr;  // v1, v2, then h(2..s')
            // A p-phase whose table fits a tail runs whole in one workgroup:
            // the tail starts at round 0 from V_i, forms the suffix weights
            // B_0 from z itself and carries the previous layer's finish.
            const bool ptail_only = s > 0 && (1ull << s) <= (u64)TAIL_LIM;
            if (ptail_only) {
                StepDesc &st = add(ST_PTAIL, 1, 8.0 * (1ull << s));
                st.fin = layer_end;
                PtailArgs pt;
                memset(&pt, 0, sizeof pt);
                pt.j0 = 0;
                pt.s = s;
                pt.pend = 0;
                pt.V = V(i);
                pt.B = nullptr;  // B_0 from z
                pt.live = 1u << s;
                pt.c0 = co;
                pt.msg = msg;
                st.u.ptail = pt;
            }
            // ---- eq tables of z_i[1..s) for the p-phase's first round
            if (!ptail_only) {
                const u32 nz = s ? s - 1 : 0;
                const u64 ne = (1ull << (nz / 2)) + (1ull << (nz - nz / 2));
                StepDesc &e = addg(ST_EQ, ne, 1, 8.0 * ne);
                mods.back() = 0.5 * ne * nz;
                e.fin = layer_end;
                e.u.eq = EqArgs{PT_Z, nz, nz / 2, 1, P_(w ? w->zlo : nullptr), P_(w ? w->zhi : nullptr)};
            }
            // ---- p-phase (a5): grid steps of two rounds while the table is
            // large, then the remaining rounds in one workgroup.  The first
            // step does round 0 (and round 1's coefficients); a step reading
            // V^(j) does rounds j+2, j+3; the tail starts at round j0.
            if (s > 0 && !ptail_only) {
                const bool look = s >= 2;
                u32 j0 = 1;
                if (look) j0 = s > 12 ? ((s - 10 + 1) & ~1u) : 2;  // even, 2^(s - j0) <= TAIL_LIM
                // V_i is zero from S_i on, and so is every V^(j) from S_i >> j:
                // the grid steps take the first NP entries of V_i (S_i rounded
                // up to 2^j0, so every step's range is exact) and the tail
                // zeroes V^(j0) from NP >> j0 on.  The suffix weights B are not
                // zero there; the steps write them below the bound only, so a
                // trimmed tail forms its B_{j0} from z.
                const u64 NP = std::min<u64>(1ull << s, ((u64)c->S[i] + (1ull << j0) - 1) >> j0 << j0);
                u64 *vbuf[2] = {w ? w->pA : nullptr, w ? w->pB : nullptr};
                u64 *bbuf[2] = {w ? w->bA : nullptr, w ? w->bB : nullptr};
                const u32 nz = s - 1;
                int bw = 0;           // B buffer the last step wrote
                const u64 *vlast = V(i);
                {
                    PArgs pa;
                    memset(&pa, 0, sizeof pa);
                    pa.first = 1;
                    pa.look = look;
                    pa.nu = look ? NP >> 2 : 1;
                    pa.Vsrc = V(i);
                    pa.Bout = look ? bbuf[0] : nullptr;  // B_1
                    pa.zlo = w ? w->zlo : nullptr;
                    pa.zhi = w ? w->zhi : nullptr;
                    pa.L = nz / 2;
                    // V 8 per entry, eq halves 16 per pair, B_1 8 per quad
                    StepDesc &st = addg(ST_P, look ? 4 * pa.nu : pa.nu, 1, look ? pa.nu * (32.0 + 32 + 8) : 32.0);
                    // per quad: a suffix weight and two products in each lane; per pair: 3
                    mods.back() = look ? pa.nu * 12.0 : pa.nu * 3.0;
                    st.u.p = pa;
                    reduces(look ? 6 : 2);
                }
                for (u32 j = 0; j + 2 < j0; j += 2) {
                    Fin f = fin_of_prev(FIN_P2);
                    f.j = j;
                    f.draw = (i32)(co + j);
                    f.msg = w ? msg + 3ull * j : nullptr;
                    PArgs pa;
                    memset(&pa, 0, sizeof pa);
                    pa.nu = NP >> (j + 4);  // (j + 4 <= j0)
                    pa.Vsrc = vlast;
                    pa.Vout = vbuf[(j / 2) & 1];
                    pa.Bprev = bbuf[bw];
                    pa.Bout = bbuf[bw ^ 1];
                    // per unit: V^(j) 16 read, V^(j+2) 4 written, B 4 read and 1 written
                    StepDesc &st = addg(ST_P, 4 * pa.nu, 1, pa.nu * 8.0 * (16 + 4 + 4 + 1));
                    mods.back() = pa.nu * 20.0;  // per quad: four two-challenge folds (3 each), 8 products
                    st.fin = f;
                    st.u.p = pa;
                    reduces(6);
                    vlast = pa.Vout;
                    bw ^= 1;
                }
                const u32 pend = look ? 2 : 1;
                Fin f = fin_of_prev(look ? FIN_P2 : FIN_P);
                f.j = j0 - pend;
                f.draw = (i32)(co + j0 - pend);
                f.msg = w ? msg + 3ull * (j0 - pend) : nullptr;
                StepDesc &st = add(ST_PTAIL, 1, 8.0 * (1ull << (s - j0 + pend)));
                mods.back() = 4.0 * (1ull << (s - j0 + pend));
                st.fin = f;
                PtailArgs pt;
                memset(&pt, 0, sizeof pt);
                pt.j0 = j0;
                pt.s = s;
                pt.pend = pend;
                pt.V = vlast;       // V^(j0 - pend)
                pt.B = NP == (1ull << s) ? bbuf[bw] : nullptr;  // B_{j0-1}, or B_{j0} from z
                pt.live = (u32)(NP >> j0);
                pt.c0 = co + j0;
                pt.msg = w ? msg + 3ull * j0 : nullptr;
                st.u.ptail = pt;
            }
            // A small layer whose wires each carry one chunk of gates runs each
            // omega phase in one workgroup (ST_WSMALL), which also forms the
            // eq table of the phase's point.
            const bool wsmall = c->omega_algo != GKR_OMEGA_GATES && sp >= 1 &&
                                (1ull << sp) <= (u64)TAIL_LIM && c->grp[0][i].single && c->grp[1][i].single;
            // ---- eq tables of a* (the p-phase tail recorded every challenge)
            if (!wsmall) {
                const u32 La = s / 2;
                const u64 ne = (1ull << La) + (1ull << (s - La));
                StepDesc &e = addg(ST_EQ, ne, 1, 8.0 * ne);
                e.u.eq = EqArgs{PT_CHAL, s, La, co, w ? w->alo : nullptr, w ? w->ahi : nullptr, 1};
            }
            if (sp == 0) {
                StepDesc &e = add(ST_SGE, 1, 8);
                e.u.sge = SgeArgs{V(i + 1), vslot};
                memset(&layer_end, 0, sizeof layer_end);
                layer_end.kind = FIN_LINE;
                layer_end.draw = (i32)(co + n);
                layer_end.T = 0;
                layer_end.sp = 0;
                layer_end.bstar = chals ? chals + co + s : nullptr;
                layer_end.cstar = chals ? chals + co + s : nullptr;
                continue;
            }
            u32 Ll = 0, M = 0, H = 0;  // shape of the line step (a9)
            if (sp >= 2) line_shape(sp, &Ll, &M, &H);
            // A wide layer's line is V_{i+1} folded along it (ST_LFOLD, a
            // workgroup per 2^(tb+9) entries; ST_FINISH adds its rows into
            // h(2..s')) instead of sums over eq tables of the line points
            // (ST_LT, ST_LINE).
            const bool lfold = sp >= LFOLD_MIN && sp <= LFOLD_MAX;
            const u32 ltb = lfold_tb(sp), lwg = lfold ? lfold_wg_live(sp, c->S[i + 1]) : 0;
            u64 *lrows = nullptr;
            auto lfold_step = [&](const Fin &f) {
                StepDesc &e = add(ST_LFOLD, lwg, 8.0 * (1ull << sp) + 8.0 * (sp - 1) * lwg);
                // ~6 products an entry (two a fold coefficient), then the terms at 2..s'
                mods.back() = 6.0 * (1ull << sp) + 2.0 * sp * (sp - 1) * lwg;
                e.fin = f;
                lrows = w ? w->rowpool + rows_used : nullptr;
                rows_used += (u64)LFOLD_CHUNKS * lwg * ROW_STRIDE;
                e.u.lfold = LfoldArgs{sp, ltb, co + s, co + s + sp, V(i + 1), lrows, chals};
            };
            const u64 ntab = sp >= 2 ? (u64)(sp - 1) * ((1ull << Ll) + (1ull << M) + (1ull << H)) : 1;
            if (c->omega_algo != GKR_OMEGA_GATES) {
                // ---- omega-phases over tables (a6, a7, a8): round 0 (and
                // round 1's coefficients) with the level-0 tables, then grid
                // steps of two rounds while the tables are large, then the
                // remaining rounds in one workgroup from round k0
                // Round 0 with the level-0 tables.  If level 1 fits a tail it
                // starts at round 1; otherwise a step folding once gives round 1
                // and round 2's coefficients, steps folding twice follow, and
                // the tail starts at an odd round k0 >= 3 (2^(s' - k0) <= TAIL_LIM).
                if (wsmall) {
                    for (u32 ph = 1; ph <= 2; ph++) {
                        const u32 rbase = s + (ph == 2 ? sp : 0);
                        const gkr_circuit::Group gd = group(ph, i);
                        const gkr_circuit::Group *dg = &gd;
                        WsmallArgs a;
                        memset(&a, 0, sizeof a);
                        a.w.kind = kind;
                        a.w.ph = ph;
                        a.w.hasC = kind != KIND_MUL;
                        a.w.npairs = (1ull << sp) / 2;
                        a.w.perm = dg->perm;
                        a.w.rowptr = dg->rowptr;
                        a.w.oths = dg->oths;
                        a.w.types = dg->types;
                        a.w.Vn = V(i + 1);
                        a.w.alo = w ? w->alo : nullptr;
                        a.w.ahi = w ? w->ahi : nullptr;
                        a.w.La = s / 2;
                        a.w.blo = w ? w->blo : nullptr;
                        a.w.bhi = w ? w->bhi : nullptr;
                        a.w.Lb = sp / 2;
                        a.eqn = ph == 1 ? s : sp;
                        a.eqL = ph == 1 ? s / 2 : sp / 2;
                        a.eqbase = ph == 1 ? co : co + s;
                        a.eqlo = ph == 1 ? (w ? w->alo : nullptr) : (w ? w->blo : nullptr);
                        a.eqhi = ph == 1 ? (w ? w->ahi : nullptr) : (w ? w->bhi : nullptr);
                        a.sp = sp;
                        a.last = ph;
                        a.c0 = co + rbase;
                        a.msg = w ? msg + 3ull * rbase : nullptr;
                        a.vout = vslot ? vslot + (ph - 1) : nullptr;
                        // eq entries 8, per gate sorted index 4 + other 4 + operand 8, per wire F 8
                        const u64 ne = (1ull << (a.eqn / 2)) + (1ull << (a.eqn - a.eqn / 2));
                        StepDesc &st = add(ST_WSMALL, 1, 8.0 * ne + 16.0 * S + 16.0 * (1ull << sp));
                        mods.back() = (ph == 1 ? 4.0 : 5.0) * S + 8.0 * (1ull << sp);
                        st.u.wsmall = a;
                    }
                } else {
                const u64 N = 1ull << sp;
                u32 k0 = 1;
                if (sp > 11) k0 = std::max<u32>(3, (sp - 10) | 1u);
                // Entries above c->wlive[i] stay zero at every level, so the
                // grid steps take only the first NL entries of level 0 (NL
                // a multiple of 2^k0: every step's range is then exact) and
                // the tail zeroes its level's entries from NL >> k0 on.
                const u64 wl = i < c->wlive.size() ? c->wlive[i] : N;
                const u64 NL = std::min<u64>(N, (wl + (1ull << k0) - 1) >> k0 << k0);
                for (u32 ph = 1; ph <= 2; ph++) {
                    const u32 rbase = s + (ph == 2 ? sp : 0);
                    const u32 Lb = sp / 2;
                    if (ph == 2) {
                        const u64 ne = (1ull << Lb) + (1ull << (sp - Lb));
                        StepDesc &e = addg(ST_EQ, ne, 1, 8.0 * ne);
                        e.u.eq = EqArgs{PT_CHAL, sp, Lb, co + s, w ? w->blo : nullptr, w ? w->bhi : nullptr};
                    }
                    const gkr_circuit::Group gd = group(ph, i);
                        const gkr_circuit::Group *dg = &gd;
                    const u32 nch = dg->nch;
                    const u32 hasC = kind != KIND_MUL;
                    if (dg->single) {
                        // gates summed per wire and round 0 in one pass
                        Wa0Args a;
                        memset(&a, 0, sizeof a);
                        a.kind = kind;
                        a.ph = ph;
                        a.hasC = hasC;
                        a.npairs = NL / 2;
                        a.perm = dg->perm;
                        a.rowptr = dg->rowptr;
                        a.oths = dg->oths;
                        a.types = dg->types;
                        a.Vn = V(i + 1);
                        a.alo = w ? w->alo : nullptr;
                        a.ahi = w ? w->ahi : nullptr;
                        a.La = s / 2;
                        a.blo = w ? w->blo : nullptr;
                        a.bhi = w ? w->bhi : nullptr;
                        a.Lb = Lb;
                        a.A = w ? w->tA0 : nullptr;
                        a.C = w ? w->tC0 : nullptr;
                        // per gate: perm 4, other wire 4, operand gather 8 (ph 1), type 1;
                        // per table entry: chunk index 4, F 8, A 8 (+ C 8)
                        StepDesc &st = addg(ST_WA0, NL / 2, 1,
                                           S * (8.0 + (ph == 1 ? 8 : 0) + (kind == KIND_MIXED)) +
                                               NL * (4.0 + 8 + 8 + (hasC ? 8 : 0)) + 8.0 * nch);
                        // per gate: chi_g(a*) (1), beta (1), the operand or chi_in1(b*) (1 or 2);
                        // per wire (phase 2) v1 twice; per pair three term products
                        mods.back() = S * (ph == 1 ? 3.0 : 4.0) + NL * (ph == 2 ? 2.0 : 0.0) + 1.5 * NL;
                        st.u.wa0 = a;
                        reduces(3);
                    } else {
                        // gate sums per chunk, then level-0 tables and round 0
                        {
                            WaggArgs a;
                            memset(&a, 0, sizeof a);
                            a.kind = kind;
                            a.ph = ph;
                            a.nch = nch;
                            a.perm = dg->perm;
                            a.cstart = dg->cstart;
                            a.oths = dg->oths;
                            a.types = dg->types;
                            a.Vn = V(i + 1);
                            a.alo = w ? w->alo : nullptr;
                            a.ahi = w ? w->ahi : nullptr;
                            a.La = s / 2;
                            a.blo = w ? w->blo : nullptr;
                            a.bhi = w ? w->bhi : nullptr;
                            a.Lb = Lb;
                            a.partA = w ? w->partA : nullptr;
                            a.partC = w ? w->partC : nullptr;
                            a.ntiles = dg->ntiles;
                            a.tch = dg->tch;
                            // per gate: perm 4, other wire 4, operand gather 8 (ph 1), type 1;
                            // per chunk: start 4, sums 16; per tile 4.  A lane per position of a tile.
                            StepDesc &st = addg(ST_WAGG, (u64)dg->ntiles * TILE_POS, 1,
                                               S * (8.0 + (ph == 1 ? 8 : 0) + (kind == KIND_MIXED)) + 20.0 * nch +
                                                   4.0 * dg->ntiles);
                            mods.back() = S * (ph == 1 ? 2.0 : 3.0) + 2.0 * nch;  // beta once per chunk
                            st.u.wagg = a;
                        }
                        {
                            Wt0Args a;
                            memset(&a, 0, sizeof a);
                            a.ph = ph;
                            a.hasC = hasC;
                            a.npairs = NL / 2;
                            a.xch = dg->xch;
                            a.partA = w ? w->partA : nullptr;
                            a.partC = w ? w->partC : nullptr;
                            a.F = V(i + 1);
                            a.A = w ? w->tA0 : nullptr;
                            a.C = w ? w->tC0 : nullptr;
                            StepDesc &st = addg(ST_WT0, NL / 2, 1,
                                               NL * (4.0 + 8 + 8 + (hasC ? 8 : 0)) + 16.0 * nch);
                            mods.back() = NL * (ph == 2 ? 2.0 : 0.0) + 1.5 * NL;
                            st.u.wt0 = a;
                            reduces(3);
                        }
                    }
                    // tables of level k (0, or odd k: two buffers alternate)
                    auto level = [&](u32 k, const u64 **A, const u64 **C, const u64 **F) {
                        if (k == 0) {
                            *A = w ? w->tA0 : nullptr;
                            *C = w ? w->tC0 : nullptr;
                            *F = V(i + 1);
                        } else {
                            const u32 b = ((k - 1) / 2) & 1;
                            *A = w ? w->tA[b] : nullptr;
                            *C = w ? w->tC[b] : nullptr;
                            *F = w ? (b ? w->fB : w->fA) : nullptr;
                        }
                    };
                    // a table step reading level k with pend pending challenges
                    auto table_step = [&](u32 k, u32 pend) {
                        Fin f = fin_of_prev(pend == 1 ? FIN_T : FIN_T2);
                        f.draw = (i32)(co + rbase + k);
                        f.msg = w ? msg + 3ull * (rbase + k) : nullptr;
                        WtArgs a;
                        memset(&a, 0, sizeof a);
                        a.hasC = hasC;
                        a.pend = pend;
                        a.nu = NL >> (k + pend + 2);  // quads of level k + pend (k + pend + 2 <= k0)
                        const u64 *A, *C, *F;
                        level(k, &A, &C, &F);
                        a.A = A;
                        a.C = C;
                        a.F = F;
                        level(k + pend, &A, &C, &F);
                        a.An = const_cast<u64 *>(A);
                        a.Cn = const_cast<u64 *>(C);
                        a.Fn = const_cast<u64 *>(F);
                        // per unit and table: 4 << pend entries read, 4 written
                        const double tabs = hasC ? 3.0 : 2.0;
                        StepDesc &st = addg(ST_WT, 4 * a.nu, 1, a.nu * tabs * 8.0 * ((4u << pend) + 4));
                        // per quad: each table's four entries folded (one product, or three for two
                        // challenges), then six products in each of the three value lanes
                        mods.back() = a.nu * (4.0 * tabs * (pend == 1 ? 1 : 3) + 18.0);
                        st.fin = f;
                        st.u.wt = a;
                        reduces(12);
                    };
                    if (k0 > 1) table_step(0, 1);
                    for (u32 k = 1; k + 4 <= k0; k += 2) table_step(k, 2);
                    {
                        const u32 pend = k0 == 1 ? 1 : 2;
                        Fin f = fin_of_prev(pend == 1 ? FIN_T : FIN_T2);
                        f.draw = (i32)(co + rbase + k0 - pend);
                        f.msg = w ? msg + 3ull * (rbase + k0 - pend) : nullptr;
                        WtailArgs a;
                        memset(&a, 0, sizeof a);
                        a.k0 = k0;
                        a.sp = sp;
                        a.hasC = hasC;
                        a.last = ph;
                        a.pend = pend;
                        a.live = (u32)(NL >> k0);
                        level(k0 - pend, &a.A, &a.C, &a.F);
                        a.c0 = co + rbase + k0;
                        a.msg = w ? msg + 3ull * (rbase + k0) : nullptr;
                        a.vout = vslot ? vslot + (ph - 1) : nullptr;
                        StepDesc &st = add(ST_WTAIL, 1, 24.0 * (1ull << (sp - k0 + pend)));
                        mods.back() = 8.0 * (1ull << (sp - k0 + pend));
                        st.fin = f;
                        st.u.wtail = a;
                    }
                }
                }  // small layer or not
                // ---- line step (a9): every omega challenge is recorded
                if (lfold) {
                    lfold_step(Fin{FIN_NONE, -1});
                } else {
                    StepDesc &e = addg(ST_LT, ntab, 1, 8.0 * ntab);
                    e.u.lt = LtArgs{sp >= 2 ? sp : 0, Ll, M, co + s, co + s + sp, w ? w->llo : nullptr,
                                    w ? w->lhl : nullptr, w ? w->lhh : nullptr};
                }
            } else {
                // ---- omega-phases (a6, a7, a8)
                const u64 *Fend = nullptr;  // table of the phase's last round
                for (u32 ph = 1; ph <= 2; ph++) {
                    const u32 rbase = s + (ph == 2 ? sp : 0);
                    const u32 Lb = sp / 2;
                    if (ph == 2) {
                        Fin f = fin_of_prev(FIN_W);
                        f.draw = (i32)(co + s + sp - 1);
                        f.msg = w ? msg + 3ull * (s + sp - 1) : nullptr;
                        f.last = 1;
                        f.F = Fend;
                        f.vout = vslot;
                        const u64 ne = (1ull << Lb) + (1ull << (sp - Lb));
                        StepDesc &e = addg(ST_EQ, ne, 1, 8.0 * ne);
                        e.fin = f;
                        e.u.eq = EqArgs{PT_CHAL, sp, Lb, co + s, w ? w->blo : nullptr, w ? w->bhi : nullptr};
                    }
                    const u64 *F = V(i + 1);
                    u64 *fbuf[2] = {w ? w->fA : nullptr, w ? w->fB : nullptr};
                    for (u32 k = 0; k < sp; k++) {
                        WArgs a;
                        memset(&a, 0, sizeof a);
                        a.kind = kind;
                        a.ph = ph;
                        a.init = k == 0;
                        a.write_w = k + 1 < sp;
                        a.inline_fold = k > 0 && S <= INLINE_FOLD_MAX_GATES;
                        a.S = S;
                        a.k = k;
                        a.nfold = 1ull << (sp - k);
                        a.idx = soa_at(i, ph == 1 ? c->in1[i] : c->in2[i]);
                        a.oth = soa_at(i, ph == 1 ? c->in2[i] : c->in1[i]);
                        a.type = soa_at(i, c->type[i]);
                        a.Vn = V(i + 1);
                        a.alo = w ? w->alo : nullptr;
                        a.ahi = w ? w->ahi : nullptr;
                        a.La = s / 2;
                        a.blo = w ? w->blo : nullptr;
                        a.bhi = w ? w->bhi : nullptr;
                        a.Lb = Lb;
                        a.rchal = -1;
                        a.w = w ? w->w : nullptr;
                        a.off = w ? w->off : nullptr;
                        Fin f;
                        memset(&f, 0, sizeof f);
                        f.kind = FIN_NONE;
                        f.draw = -1;
                        if (k > 0) {
                            f = fin_of_prev(FIN_W);
                            f.draw = (i32)(co + rbase + k - 1);
                            f.msg = w ? msg + 3ull * (rbase + k - 1) : nullptr;
                            u64 *dst = fbuf[k & 1];
                            if (a.inline_fold) {
                                a.F = F;       // F^(k-1): the kernel folds it into dst
                                a.Fout = dst;
                            } else {
                                StepDesc &fs = addg(ST_FOLD, a.nfold, 4, a.nfold * 24.0);
                                fs.fin = f;
                                fs.u.fold = FoldArgs{a.nfold, F, dst};
                                memset(&f, 0, sizeof f);
                                f.kind = FIN_NONE;
                                f.draw = -1;
                                a.F = dst;
                                a.rchal = (i32)(co + rbase + k - 1);
                            }
                            F = dst;
                        } else {
                            a.F = F;
                        }
                        // algorithmic bytes per gate: index 4, weight read 8 (not at
                        // init) and write 8 (not in the last round), the additive
                        // operand 8 (phase 1 with ADD gates), type 1 (mixed), init:
                        // other index 4 + operand gather 8 (phase 1); plus one pass
                        // over the fold table (and its folded half when inline).
                        const double per = 4.0 + (a.init ? 0 : 8) + (a.write_w ? 8 : 0) +
                                           (ph == 1 && kind != KIND_MUL ? 8 : 0) +
                                           (kind == KIND_MIXED ? 1 : 0) + (a.init ? 4.0 + (ph == 1 ? 8 : 0) : 0);
                        const double nb = S * per + (a.inline_fold ? 24.0 : 8.0) * a.nfold;
                        StepDesc &ws = addg(ST_W, std::max<u64>(S, a.inline_fold ? a.nfold : 0), 4, nb);
                        ws.fin = f;
                        ws.u.w = a;
                        reduces(4);
                    }
                    Fend = F;
                }
                // ---- line step (a9): finish the last round, then the line tables
                {
                    Fin f = fin_of_prev(FIN_W);
                    f.draw = (i32)(co + n - 1);
                    f.msg = w ? msg + 3ull * (n - 1) : nullptr;
                    f.last = 2;
                    f.F = Fend;
                    f.vout = vslot ? vslot + 1 : nullptr;
                    if (lfold) {
                        lfold_step(f);
                    } else {
                        StepDesc &e = addg(ST_LT, ntab, 1, 8.0 * ntab);
                        e.fin = f;
                        e.u.lt = LtArgs{sp >= 2 ? sp : 1, Ll, M, co + s, co + s + sp, w ? w->llo : nullptr,
                                        w ? w->lhl : nullptr, w ? w->lhh : nullptr};
                        if (sp < 2) e.u.lt.sp = 0;  // nothing to tabulate
                    }
                }
            }
            {
                memset(&layer_end, 0, sizeof layer_end);
                layer_end.kind = FIN_LINE;
                layer_end.draw = (i32)(co + n);
                layer_end.sp = sp;
                layer_end.bstar = chals ? chals + co + s : nullptr;
                layer_end.cstar = chals ? chals + co + s + sp : nullptr;
                layer_end.msg = vslot ? vslot + 2 : nullptr;
                if (lfold) {  // the fold's rows, added up by ST_FINISH
                    layer_end.T = sp - 1;
                    layer_end.rows = lrows;
                    layer_end.nrows = lwg;
                    layer_end.chunk_blocks = lwg;
                    layer_end.ch = ROW_STRIDE;
                } else if (sp >= 2) {
                    const u32 T = sp - 1;
                    const u32 chunks = (T + LINE_CHUNK - 1) / LINE_CHUNK;
                    const u32 ch = ((T + chunks - 1) / chunks + 3) / 4 * 4;  // equal chunks, 4 | ch
                    const u32 cb = (u32)(((1ull << M) + (SBLOCK / 64) - 1) / (SBLOCK / 64));
                    StepDesc &ls = add(ST_LINE, chunks * cb, 8.0 * (1ull << sp) * chunks);
                    mods.back() = (double)T * (1ull << sp);  // one product per line point and entry
                    ls.u.line = LineArgs{sp, Ll, M, T, cb, ch, V(i + 1), w ? w->llo : nullptr,
                                         w ? w->lhl : nullptr, w ? w->lhh : nullptr};
                    reduces(LINE_CHUNK);
                    layer_end.T = T;
                    layer_end.rows = ls.rows;
                    layer_end.nrows = ls.nblocks;
                    layer_end.chunk_blocks = cb;
                    layer_end.ch = ch;
                }
            }
        }
        sc_last[d - 1] = (int)out.size() - 1;
        StepDesc &e = add(ST_END, 1, 0);
        e.fin = layer_end;
        add_finish();
    }
};

// Chunk counts, single-chunk flags and byte sizes of every layer's gate
// groups, from the wire counts alone (what planning and sizing need; no
// memory is allocated).
static void size_groups(gkr_circuit *c) {
    if (c->grouped) return;
    const u32 d = c->L - 1;
    c->grp[0].assign(d, gkr_circuit::Group());
    c->grp[1].assign(d, gkr_circuit::Group());
    c->g_off.assign(d + 1, 0);
    c->nch_max = 1;
    auto al = [](size_t n) { return (n + 255) & ~size_t(255); };
    size_t bytes = 0;
    std::vector<u32> cnt;
    c->wlive.assign(d, 0);
    for (u32 i = 0; i < d; i++) {
        c->g_off[i] = bytes;
        const u64 N = 1ull << c->s[i + 1], S = c->S[i];
        u64 live = c->S[i + 1];
        for (int ph = 0; ph < 2; ph++) {
            const std::vector<u32> &idx = ph ? c->h_in2[i] : c->h_in1[i];
            cnt.assign(N, 0);
            for (u64 g = 0; g < S; g++) {
                cnt[idx[g]]++;
                live = std::max<u64>(live, (u64)idx[g] + 1);
            }
            u64 nch = 0, ntiles = 0, span = TILE_POS + 1;  // positions in the open tile
            bool single = true;
            for (u64 x = 0; x < N; x++) {
                const u64 csz = chunk_of(cnt[x]);
                const u64 k = (cnt[x] + csz - 1) / csz;
                nch += k;
                single = single && k <= 1;
                for (u64 q = 0; q < k; q++) {  // the chunks of wire x, in order (as build_group cuts them)
                    const u64 len = std::min<u64>(csz, cnt[x] - q * csz);
                    if (span + len > TILE_POS) {
                        ntiles++;
                        span = 0;
                    }
                    span += len;
                }
            }
            if (!ntiles) ntiles = 1;  // no gates: one empty tile
            gkr_circuit::Group &D = c->grp[ph][i];
            D.nch = (u32)nch;
            D.ntiles = (u32)ntiles;
            D.single = single;
            c->nch_max = std::max<u64>(c->nch_max, nch + 1);
            c->wlive[i] = std::min<u64>(live, N);
            // perm, cstart, xch, rowptr, oths, tch, types (mixed layers)
            bytes += 2 * al(S * 4) + al((nch + 1) * 4) + 2 * al((N + 1) * 4) + al((ntiles + 1) * 4) +
                     al(c->h_type[i].size());
        }
    }
    c->g_off[d] = bytes;
    c->grouped = true;
}

// Group every layer's gates by in1 and by in2 (once per circuit), one layer
// at a time, into the memory the circuit's gate arrays live in.
static int ensure_groups(gkr_circuit *c) {
    if (c->gmem) return GKR_OK;
    size_groups(c);
    const u32 d = c->L - 1;
    void *mem = nullptr;
    HIP_TRY(mem_alloc(c->gates_host, std::max<size_t>(c->g_off[d], 256), &mem));
    c->gmem = mem;
    char *p = (char *)mem;
    auto put = [&](const void *src, size_t bytes, void **dst) -> hipError_t {
        *dst = p;
        p += (bytes + 255) & ~size_t(255);
        return bytes ? hipMemcpy(*dst, src, bytes, hipMemcpyDefault) : hipSuccess;
    };
    for (u32 i = 0; i < d; i++) {
        const u64 N = 1ull << c->s[i + 1];
        for (int ph = 0; ph < 2; ph++) {
            HostGroup G;
            build_group(ph ? c->h_in2[i] : c->h_in1[i], ph ? c->h_in1[i] : c->h_in2[i], c->h_type[i], N, G);
            gkr_circuit::Group &D = c->grp[ph][i];
            if (G.cstart.size() != (size_t)D.nch + 1 || G.tch.size() != (size_t)D.ntiles + 1)
                return fail(GKR_ERR_INVALID, "gate grouping changed size");
            HIP_TRY(put(G.perm.data(), G.perm.size() * 4, (void **)&D.perm));
            HIP_TRY(put(G.cstart.data(), G.cstart.size() * 4, (void **)&D.cstart));
            HIP_TRY(put(G.xch.data(), G.xch.size() * 4, (void **)&D.xch));
            HIP_TRY(put(G.rowptr.data(), G.rowptr.size() * 4, (void **)&D.rowptr));
            HIP_TRY(put(G.oths.data(), G.oths.size() * 4, (void **)&D.oths));
            HIP_TRY(put(G.tch.data(), G.tch.size() * 4, (void **)&D.tch));
            D.types = nullptr;
            if (!G.types.empty()) HIP_TRY(put(G.types.data(), G.types.size(), (void **)&D.types));
        }
        if ((size_t)(p - (char *)mem) != c->g_off[i + 1]) return fail(GKR_ERR_INVALID, "gate groups misplaced");
    }
    return GKR_OK;
}

// Move the circuit's gate arrays (struct of arrays and groups) between
// device memory and pinned host memory; pointers into them are rebased.
// The caller invalidates every step program that holds the old pointers.
static int move_gates(gkr_circuit *c, bool to_host) {
    if (c->gates_host == to_host) return GKR_OK;
    const u32 d = c->L - 1;
    void *ns = nullptr, *ng = nullptr;
    hipError_t e = mem_alloc(to_host, std::max<size_t>(c->soa_off[d], 256), &ns);
    if (e == hipSuccess) e = hipMemcpy(ns, c->soa, c->soa_off[d], hipMemcpyDefault);
    if (e == hipSuccess && c->gmem) {
        e = mem_alloc(to_host, std::max<size_t>(c->g_off[d], 256), &ng);
        if (e == hipSuccess) e = hipMemcpy(ng, c->gmem, c->g_off[d], hipMemcpyDefault);
    }
    if (e != hipSuccess) {
        gate_free(to_host, ns);
        gate_free(to_host, ng);
        return fail(e == hipErrorOutOfMemory ? GKR_ERR_NOMEM : GKR_ERR_DEVICE,
                    std::string("moving the gate arrays: ") + hipGetErrorString(e));
    }
    auto rb = [](auto *ptr, void *ob, void *nb) -> decltype(ptr) {
        return ptr ? (decltype(ptr))((char *)nb + ((const char *)ptr - (const char *)ob)) : ptr;
    };
    for (u32 i = 0; i < d; i++) {
        c->in1[i] = rb(c->in1[i], c->soa, ns);
        c->in2[i] = rb(c->in2[i], c->soa, ns);
        c->type[i] = rb(c->type[i], c->soa, ns);
    }
    if (c->gmem)
        for (int ph = 0; ph < 2; ph++)
            for (gkr_circuit::Group &D : c->grp[ph]) {
                D.perm = rb(D.perm, c->gmem, ng);
                D.cstart = rb(D.cstart, c->gmem, ng);
                D.xch = rb(D.xch, c->gmem, ng);
                D.rowptr = rb(D.rowptr, c->gmem, ng);
                D.oths = rb(D.oths, c->gmem, ng);
                D.tch = rb(D.tch, c->gmem, ng);
                D.types = rb(D.types, c->gmem, ng);
            }
    gate_free(c->gates_host, c->soa);
    gate_free(c->gates_host, c->gmem);
    c->soa = ns;
    c->gmem = ng;
    c->gates_host = to_host;
    return GKR_OK;
}

// (Re)build a workspace's step program with the current launch shapes and
// upload it; the workspace must be idle.
// Copies of a per-layer (copy-once-per-layer) proof, Sec. 5.1.2.  The
// prover works on two layers at a time: layer i's sum-check reads V_i and
// V_{i+1} (slots i % 3 and (i+1) % 3) and layer i's gate groups (gate slot
// i % 2).  Evaluation runs from the inputs upward: each table V_j, j >= 3,
// goes to host memory once written, before evaluation of layer j - 3
// overwrites its slot; every layer's struct of arrays comes in while the
// layer above the next one is evaluated.  The sum-check runs downward:
// V_{i+2} and layer i+1's groups come in while layer i's rounds run, each
// once the last step reading its slot's previous content has finished.
static void plan_transfers(const gkr_circuit *c, Workspace &w, const Planner &pl) {
    w.xfers.clear();
    if (w.mode != GKR_MEM_LAYER) return;
    const int d = (int)c->L - 1;
    const int load = 0;  // the first step loads the inputs into V_d
    auto writer = [&](int j) { return j == d ? load : pl.eval_at[j]; };
    auto vbytes = [&](int j) { return (size_t)8 << c->s[j]; };
    std::vector<Workspace::Xfer> x;
    for (int j = d; j >= 3; j--)  // evaluation: V_j out before its slot is reused
        x.push_back({writer(j), pl.eval_at[j - 3], w.V[j], w.Vslot[j % 3], vbytes(j), hipMemcpyDeviceToHost});
    for (int j = 3; j <= d; j++)  // sum-check: V_j back for layers j - 1 and j
        x.push_back({pl.sc_last[j - 3], pl.sc_first[j - 1], w.Vslot[j % 3], w.V[j], vbytes(j),
                     hipMemcpyHostToDevice});
    if (w.gslot) {
        const bool tables = c->omega_algo != GKR_OMEGA_GATES;
        for (int i = d - 1; i >= 0; i--)  // evaluation of layer i: its struct of arrays
            x.push_back({i + 2 <= d - 1 ? pl.eval_at[i + 2] : -1, pl.eval_at[i], w.Gslot[i % 2],
                         (const char *)c->soa + c->soa_off[i], c->soa_off[i + 1] - c->soa_off[i],
                         hipMemcpyHostToDevice});
        for (int i = 0; i < d; i++) {  // sum-check of layer i: its groups (or struct of arrays)
            const char *src = tables ? (const char *)c->gmem + c->g_off[i] : (const char *)c->soa + c->soa_off[i];
            const size_t n = tables ? c->g_off[i + 1] - c->g_off[i] : c->soa_off[i + 1] - c->soa_off[i];
            x.push_back({i <= 1 ? pl.eval_at[i] : pl.sc_last[i - 2], pl.sc_first[i], w.Gslot[i % 2], src, n,
                         hipMemcpyHostToDevice});
        }
    }
    std::stable_sort(x.begin(), x.end(), [](const Workspace::Xfer &a, const Workspace::Xfer &b) {
        return a.after < b.after;
    });
    w.xfers = x;
}

// Every copy starts after the step it follows and ends before the step that
// waits for it, and stays inside its slot.
static int check_transfers(const gkr_circuit *c, const Workspace &w) {
    const int nsteps = (int)w.steps.size();
    const size_t vslot = (size_t)8 << c->smax;
    for (const Workspace::Xfer &x : w.xfers) {
        if (x.before < 0 || x.before >= nsteps || x.after >= x.before)
            return fail(GKR_ERR_INVALID, "a transfer is ordered after the step that needs it");
        const char *d = (const char *)(x.kind == hipMemcpyDeviceToHost ? x.src : x.dst);
        bool inside = false;
        for (int k = 0; k < 3; k++)
            inside = inside || (d >= (const char *)w.Vslot[k] && d + x.bytes <= (const char *)w.Vslot[k] + vslot);
        for (int k = 0; k < 2 && w.gslot; k++)
            inside = inside || (d >= w.Gslot[k] && d + x.bytes <= w.Gslot[k] + w.gslot);
        if (!inside) return fail(GKR_ERR_INVALID, "a transfer leaves its slot");
    }
    return GKR_OK;
}

// (Re)build a workspace's step program with the current launch shapes and
// upload it; the workspace must be idle.
static int plan_into(gkr_circuit *c, Workspace &ws) {
    const u32 epoch = g_tune_epoch.load();
    Planner plan{c, &ws};
    plan.build();
    const size_t nsteps = plan.out.size();
    if (nsteps != ws.steps.size()) return fail(GKR_ERR_INVALID, "step program changed size");
    if (plan.rows_used > ws.cap_rows || plan.recs_used > ws.cap_recs || plan.items.size() > ws.cap_items)
        return fail(GKR_ERR_INVALID, "step program outgrew its workspace");
    for (const StepDesc &sd : plan.out)
        if (sd.fin.kind != FIN_NONE && !((fin_mask(sd.kind) >> sd.fin.kind) & 1))
            return fail(GKR_ERR_INVALID, "step program: a step carries a finish its kernel lacks");
    plan_transfers(c, ws, plan);
    {
        ws.steps.resize(nsteps);  // (its length is all check_transfers reads)
        const int rc = check_transfers(c, ws);
        if (rc) return rc;
    }
    while (ws.xev.size() < 2 * ws.xfers.size()) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ws.xev.push_back(e);
    }
    ws.steps = plan.out;
    ws.pclass = plan.cls;
    ws.pbytes = plan.bytes;
    ws.pmods = plan.mods;
    ws.punits = plan.units;
    std::vector<JobEntry> jobs(2 * nsteps);
    for (size_t t = 0; t < nsteps; t++) {
        jobs[2 * t] = JobEntry{ws.d_steps + t, 0, 0};
        jobs[2 * t + 1] = JobEntry{nullptr, step_grid(plan.out[t]), 0};
    }
    HIP_TRY(hipMemcpy(ws.d_steps, plan.out.data(), nsteps * sizeof(StepDesc), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ws.d_jobs, jobs.data(), jobs.size() * sizeof(JobEntry), hipMemcpyHostToDevice));
    if (!plan.items.empty())
        HIP_TRY(hipMemcpy(ws.d_items, plan.items.data(), plan.items.size() * sizeof(FinItem), hipMemcpyHostToDevice));
    if (!plan.top.empty()) {
        if (plan.top.size() >= c->L) return fail(GKR_ERR_INVALID, "top layers outgrew their descriptors");
        HIP_TRY(hipMemcpy(ws.d_top, plan.top.data(), plan.top.size() * sizeof(TopLayer), hipMemcpyHostToDevice));
    }
    ws.epoch = epoch;
    return GKR_OK;
}

// Re-plan an idle workspace planned before the launch shapes last changed.
static int refresh_plan(gkr_circuit *c, Workspace &ws) {
    return ws.epoch == g_tune_epoch.load() ? GKR_OK : plan_into(c, ws);
}

// Device and pinned host bytes of a workspace of c in the given mode
// (sized without allocating).
static PlanSizes plan_sizes(gkr_circuit *c) {
    if (c->omega_algo != GKR_OMEGA_GATES) size_groups(c);
    Planner count{c, nullptr};
    count.build();
    return count.sizes();
}

static void size_workspace(gkr_circuit *c, int mode, const PlanSizes &ps, size_t *dev, size_t *host) {
    Workspace probe;
    probe.mode = mode;
    Arena a, h;
    carve(c, a, h, probe, ps);
    *dev = a.used;
    *host = h.used;
}

// A proof's scratch with its step program (for the circuit's own proofs, or
// one entry of a batch or server), its tables placed as `mode` says.
static int make_workspace(gkr_circuit *c, int mode, Workspace **out) {
    *out = nullptr;
    if (c->omega_algo != GKR_OMEGA_GATES) {
        int rc = ensure_groups(c);
        if (rc) return rc;
    }
    const PlanSizes ps = plan_sizes(c);
    const size_t nsteps = ps.nsteps;
    size_t dbytes = 0, hbytes = 0;
    size_workspace(c, mode, ps, &dbytes, &hbytes);
    std::unique_ptr<Workspace, void (*)(Workspace *)> ws(new Workspace(), free_workspace);
    ws->mode = mode;
    HIP_TRY(hipMalloc(&ws->mem, dbytes));
    ws->bytes = dbytes;
    if (hbytes) HIP_TRY(mem_alloc(true, hbytes, &ws->hmem));
    ws->hbytes = hbytes;
    Arena a, h;
    a.base = (char *)ws->mem;
    a.cap = dbytes;
    h.base = (char *)ws->hmem;
    h.cap = hbytes;
    carve(c, a, h, *ws, ps);
    ws->cap_rows = ps.rows;
    ws->cap_recs = ps.recs;
    ws->cap_items = ps.items;
    ws->steps.resize(nsteps);
    if (mode == GKR_MEM_LAYER) {
        HIP_TRY(hipStreamCreateWithFlags(&ws->cs, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&ws->ev_begin, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&ws->ev_join, hipEventDisableTiming));
    }
    int rc = plan_into(c, *ws);
    if (rc) return rc;
    HIP_TRY(hipHostMalloc((void **)&ws->h_msgs, c->n_msgs * 8));
    HIP_TRY(hipHostMalloc((void **)&ws->h_chals, std::max<u64>(c->n_chals, 1) * 8));
    HIP_TRY(hipHostMalloc((void **)&ws->h_setup, 3 * 8));
    ws->gen = c->gen;
    *out = ws.release();
    return GKR_OK;
}

// Device bytes of c's gate arrays (struct of arrays, and the groups the
// tables algorithm reads).
static size_t gate_bytes(gkr_circuit *c) {
    if (c->omega_algo != GKR_OMEGA_GATES) size_groups(c);
    const u32 d = c->L - 1;
    return c->soa_off[d] + (c->omega_algo != GKR_OMEGA_GATES ? c->g_off[d] : 0);
}

// Device bytes a workspace of c takes in `mode` (sized without allocating;
// cached per mode until the circuit's program changes).
static int workspace_size(gkr_circuit *c, int mode, size_t *bytes) {
    if (mode < 0 || mode > GKR_MEM_MESSAGE) return fail(GKR_ERR_INVALID, "unknown memory mode");
    if (!c->ws_bytes[mode]) {
        size_t host = 0;
        size_workspace(c, mode, plan_sizes(c), &c->ws_bytes[mode], &host);
    }
    *bytes = c->ws_bytes[mode];
    return GKR_OK;
}

static int ensure_workspace(gkr_circuit *c) {
    if (c->ws) return refresh_plan(c, *c->ws);
    return make_workspace(c, c->mem_mode, &c->ws);
}

// Device and pinned host bytes of one proof of c in `mode`, gate arrays
// included where the mode places them.
static int memory_need(gkr_circuit *c, int mode, u64 *dev, u64 *host) {
    if (mode < GKR_MEM_RESIDENT || mode > GKR_MEM_MESSAGE) return fail(GKR_ERR_INVALID, "unknown memory mode");
    size_t d = 0, h = 0;
    size_workspace(c, mode, plan_sizes(c), &d, &h);
    const size_t g = gate_bytes(c);
    *dev = d + (mode == GKR_MEM_RESIDENT ? g : 0);
    *host = h + (mode == GKR_MEM_RESIDENT ? 0 : g);
    return GKR_OK;
}

extern "C" int gkr_memory_need(gkr_circuit *c, int mode, uint64_t *device_bytes, uint64_t *host_bytes) {
    if (!c) return fail(GKR_ERR_INVALID, "circuit is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    u64 d = 0, h = 0;
    const int rc = memory_need(c, mode, &d, &h);
    if (rc) return rc;
    if (device_bytes) *device_bytes = d;
    if (host_bytes) *host_bytes = h;
    return GKR_OK;
}

static void drop_batches_of(const gkr_circuit *c);
static void drop_served_scratch_of(const gkr_circuit *c);

extern "C" int gkr_circuit_set_memory(gkr_circuit *c, int mode, uint64_t device_budget_bytes, int *chosen) {
    if (!c) return fail(GKR_ERR_INVALID, "circuit is NULL");
    if (mode < GKR_MEM_RESIDENT || mode > GKR_MEM_AUTO) return fail(GKR_ERR_INVALID, "unknown memory mode");
    {
        std::lock_guard<std::mutex> lk(c->mu);
        int pick = -1;
        for (int m = GKR_MEM_RESIDENT; m <= GKR_MEM_MESSAGE && pick < 0; m++) {
            if (mode != GKR_MEM_AUTO && m != mode) continue;
            u64 d = 0, h = 0;
            const int rc = memory_need(c, m, &d, &h);
            if (rc) return rc;
            if (!device_budget_bytes || d <= device_budget_bytes) pick = m;
        }
        if (pick < 0) return fail(GKR_ERR_NOMEM, "no memory mode fits the device budget");
        free_workspace(c->ws);  // every step program holds the old placement
        c->ws = nullptr;
        const int rc = move_gates(c, pick != GKR_MEM_RESIDENT);
        c->mem_mode = pick;
        c->gen++;
        if (chosen) *chosen = pick;
        if (rc) return rc;
    }
    drop_batches_of(c);
    drop_served_scratch_of(c);
    return GKR_OK;
}

// ------------------------------------------------------------------- prover

#define LAUNCH(cls, bytes, expr)                                  \
    do {                                                          \
        Scope sc_(cls, st, (double)(bytes));                      \
        HIP_TRY(expr);                                            \
    } while (0)

// Enqueue one whole proof (inputs already staged, seed in w.state[2]): one
// launch per step.  A per-layer proof's copies run on its copy stream: a
// copy starts once the step named by its `after` has finished (an event on
// st), and the step named by its `before` waits for it (an event on cs).
static int enqueue_proof(Workspace &w, hipStream_t st) {
    const size_t n = w.steps.size(), nx = w.xfers.size();
    size_t xi = 0;
    auto issue = [&](int after) -> int {  // copies that may start after step `after`
        if (xi >= nx || w.xfers[xi].after != after) return GKR_OK;
        hipEvent_t done = w.xev[2 * xi];
        HIP_TRY(hipEventRecord(done, st));
        HIP_TRY(hipStreamWaitEvent(w.cs, done, 0));
        for (; xi < nx && w.xfers[xi].after == after; xi++) {
            const Workspace::Xfer &x = w.xfers[xi];
            HIP_TRY(hipMemcpyAsync(x.dst, x.src, x.bytes, x.kind, w.cs));
            HIP_TRY(hipEventRecord(w.xev[2 * xi + 1], w.cs));
        }
        return GKR_OK;
    };
    if (nx) {
        int rc = issue(-1);
        if (rc) return rc;
    }
    for (size_t t = 0; t < n; t++) {
        for (size_t k = 0; k < nx; k++)
            if (w.xfers[k].before == (int)t) HIP_TRY(hipStreamWaitEvent(st, w.xev[2 * k + 1], 0));
        hipEvent_t a, b;
        prof_pair(w.pclass[t], w.pbytes[t], &a, &b, w.pmods[t], w.punits[t] ? (int)size_class(w.punits[t]) : -1);
        HIP_TRY(launch_step(st, w.steps[t], a, b));
        if (nx) {
            int rc = issue((int)t);
            if (rc) return rc;
        }
    }
    if (xi != nx) return fail(GKR_ERR_INVALID, "a transfer of the proof was not issued");
    if (nx) {  // the copy stream's work ends before the proof does
        HIP_TRY(hipEventRecord(w.ev_join, w.cs));
        HIP_TRY(hipStreamWaitEvent(st, w.ev_join, 0));
    }
    return GKR_OK;
}

namespace {
hipStream_t capture_stream();
}

// A proof's launches as a graph, captured on first use and again after a
// re-plan; a replay costs one enqueue instead of one per step.
static int proof_graph(Workspace &w) {
    if (w.gexec && w.gepoch == w.epoch) return GKR_OK;
    if (w.gexec) (void)hipGraphExecDestroy(w.gexec);
    if (w.graph) (void)hipGraphDestroy(w.graph);
    w.gexec = nullptr;
    w.graph = nullptr;
    hipStream_t cst = capture_stream();
    if (!cst) return fail(GKR_ERR_DEVICE, "no capture stream");
    HIP_TRY(hipStreamBeginCapture(cst, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_proof(w, cst);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cst, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    HIP_TRY(e);
    w.graph = graph;
    HIP_TRY(hipGraphInstantiate(&w.gexec, graph, nullptr, nullptr, 0));
    w.gepoch = w.epoch;
    return GKR_OK;
}

// One proof's launches on st: replayed from its graph, or launched one by
// one while per-launch profiling is on.
static int run_proof(Workspace &w, hipStream_t st) {
    if (g_prof.on || w.mode == GKR_MEM_LAYER) return enqueue_proof(w, st);
    const int rc = proof_graph(w);
    if (rc) return rc;
    HIP_TRY(hipGraphLaunch(w.gexec, st));
    return GKR_OK;
}

// Host inputs checked and copied in (device inputs are read in place), then
// seed, input pointer and a cleared range flag into state[2..4]
// (asynchronous on st; h_setup must not be reused before st has passed).
static int stage_proof(gkr_circuit *c, Workspace &w, const uint64_t *inputs, int inputs_on_device,
                       uint64_t seed, hipStream_t st) {
    const u64 Sd = c->S[c->L - 1];
    const u64 *src = inputs;
    if (!inputs_on_device) {
        for (u64 g = 0; g < Sd; g++)
            if (inputs[g] >= fp::P) return fail(GKR_ERR_RANGE, "input value not below p");
        // (into device memory, or into pinned host memory for out-of-core proofs)
        HIP_TRY(hipMemcpyAsync(w.instage, inputs, Sd * 8, hipMemcpyDefault, st));
        src = w.instage;
    }
    w.h_setup[0] = seed;
    w.h_setup[1] = (u64)(uintptr_t)src;
    w.h_setup[2] = 0;
    HIP_TRY(hipMemcpyAsync(w.state + 2, w.h_setup, 3 * 8, hipMemcpyHostToDevice, st));
    return GKR_OK;
}

extern "C" int gkr_prove(const gkr_circuit *cc, const uint64_t *inputs, int inputs_on_device,
                         uint64_t seed, uint64_t *msgs, uint64_t *chals, void *hip_stream) {
    if (!cc || !inputs || !msgs) return fail(GKR_ERR_INVALID, "NULL argument");
    gkr_circuit *c = const_cast<gkr_circuit *>(cc);
    hipStream_t st = pick_stream(hip_stream);
    if (!st) return fail(GKR_ERR_DEVICE, "no stream");
    std::lock_guard<std::mutex> lk(c->mu);
    int rc = ensure_workspace(c);
    if (rc) return rc;
    Workspace &w = *c->ws;
    rc = stage_proof(c, w, inputs, inputs_on_device, seed, st);
    if (rc) return rc;
    rc = run_proof(w, st);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(w.h_msgs, w.msgs, c->n_msgs * 8, hipMemcpyDeviceToHost, st));
    if (chals) HIP_TRY(hipMemcpyAsync(w.h_chals, w.chals, c->n_chals * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(w.h_setup + 2, w.state + 4, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (w.h_setup[2]) return fail(GKR_ERR_RANGE, "input value not below p");
    memcpy(msgs, w.h_msgs, c->n_msgs * 8);
    if (chals) memcpy(chals, w.h_chals, c->n_chals * 8);
    return GKR_OK;
}

// ----------------------------------------------------------------- autotune

extern "C" int gkr_autotune(uint32_t n, const gkr_circuit *const *circuits, const uint64_t *const *inputs,
                            int inputs_on_device, uint32_t reps, void *hip_stream) {
    if (n == 0 || !circuits || !inputs) return fail(GKR_ERR_INVALID, "no circuits to tune on");
    for (u32 q = 0; q < n; q++)
        if (!circuits[q] || !inputs[q]) return fail(GKR_ERR_INVALID, "NULL circuit or inputs");
    hipStream_t st = pick_stream(hip_stream);
    if (!st) return fail(GKR_ERR_DEVICE, "no stream");
    reps = std::max<u32>(reps, 1);
    std::lock_guard<std::mutex> tl(g_tune_mu);
    const size_t nkey = (size_t)NKIND * NCLASS * NSHAPE;
    std::vector<double> tot(nkey, 0.0);
    std::vector<u32> cnt(nkey, 0);
    std::vector<hipEvent_t> ev;
    int rc = GKR_OK;
    for (int shape = 0; shape < NSHAPE && !rc; shape++) {
        g_force = shape;  // every tunable step of every plan made now
        g_tune_epoch++;
        for (u32 q = 0; q < n && !rc; q++) {
            gkr_circuit *c = const_cast<gkr_circuit *>(circuits[q]);
            std::lock_guard<std::mutex> lk(c->mu);
            if (c->mem_mode == GKR_MEM_LAYER) {
                rc = fail(GKR_ERR_INVALID, "launch shapes are tuned on resident or per-message circuits");
                break;
            }
            rc = ensure_workspace(c);
            if (rc) break;
            Workspace &w = *c->ws;
            const size_t T = w.steps.size();
            while (ev.size() < 2 * T) {
                hipEvent_t e = nullptr;
                if (hipEventCreate(&e) != hipSuccess) {
                    rc = fail(GKR_ERR_DEVICE, "hipEventCreate failed");
                    break;
                }
                ev.push_back(e);
            }
            for (u32 rep = 0; rep <= reps && !rc; rep++) {  // run 0 warms up
                rc = stage_proof(c, w, inputs[q], inputs_on_device, 1 + rep, st);
                for (size_t t = 0; t < T && !rc; t++) {
                    const bool timed = rep > 0 && w.punits[t] != 0;
                    if (launch_step(st, w.steps[t], timed ? ev[2 * t] : nullptr,
                                    timed ? ev[2 * t + 1] : nullptr) != hipSuccess)
                        rc = fail(GKR_ERR_DEVICE, "step launch failed");
                }
                if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = fail(GKR_ERR_DEVICE, "stream failed");
                if (rc || rep == 0) continue;
                for (size_t t = 0; t < T; t++) {
                    if (!w.punits[t]) continue;
                    float ms = 0;
                    if (hipEventElapsedTime(&ms, ev[2 * t], ev[2 * t + 1]) != hipSuccess) continue;
                    const size_t key = ((size_t)w.steps[t].kind * NCLASS + size_class(w.punits[t])) * NSHAPE + shape;
                    tot[key] += ms;
                    cnt[key]++;
                }
            }
        }
    }
    g_force = -1;
    if (!rc) {
        for (int k = 0; k < NKIND; k++)
            for (int b = 0; b < NCLASS; b++) {
                int best = -1;
                double bm = 0;
                for (int shape = 0; shape < NSHAPE; shape++) {
                    const size_t key = ((size_t)k * NCLASS + b) * NSHAPE + shape;
                    if (!cnt[key]) continue;
                    const double m = tot[key] / cnt[key];
                    if (best < 0 || m < bm) {
                        best = shape;
                        bm = m;
                    }
                }
                if (best >= 0) g_tune[k][b] = (u8)best;
            }
    }
    g_tune_epoch++;  // plans made during tuning are rebuilt with the choice
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    return rc;
}

extern "C" int gkr_tune_get(uint8_t *buf, uint32_t *len) {
    if (!len) return fail(GKR_ERR_INVALID, "len is NULL");
    const uint32_t need = 4 + NKIND * NCLASS;
    if (!buf) {
        *len = need;
        return GKR_OK;
    }
    if (*len < need) return fail(GKR_ERR_BUFSIZE, "tuning buffer too small");
    std::lock_guard<std::mutex> tl(g_tune_mu);
    buf[0] = 1;
    buf[1] = (uint8_t)NKIND;
    buf[2] = (uint8_t)NCLASS;
    buf[3] = 0;
    memcpy(buf + 4, g_tune, NKIND * NCLASS);
    *len = need;
    return GKR_OK;
}

extern "C" int gkr_tune_set(const uint8_t *buf, uint32_t len) {
    std::lock_guard<std::mutex> tl(g_tune_mu);
    if (!buf) {
        memset(g_tune, SHAPE_DEFAULT, sizeof g_tune);
    } else {
        if (len != 4 + (uint32_t)NKIND * NCLASS || buf[0] != 1 || buf[1] != NKIND || buf[2] != NCLASS)
            return fail(GKR_ERR_INVALID, "not a tuning table of this library");
        for (uint32_t q = 4; q < len; q++)
            if (buf[q] != SHAPE_DEFAULT && buf[q] >= NSHAPE) return fail(GKR_ERR_INVALID, "bad shape code");
        memcpy(g_tune, buf + 4, NKIND * NCLASS);
    }
    g_tune_epoch++;
    return GKR_OK;
}

// ------------------------------------------------------------------ batches
//
// A batch plan owns one workspace (scratch + step program) per entry.
// Launch t runs step t of every proof that has one: a job table maps each
// workgroup to (proof, step).  The sequence "write seeds and input pointers,
// all batched steps, gather the transcripts" is captured once as a HIP
// graph and replayed for later batches over the same circuits.

namespace {

struct BatchPlan {
    std::vector<gkr_circuit *> key;
    int flags = 0;
    u32 epoch = 0;  // launch shapes its programs were planned with
    std::vector<Workspace *> ws;
    std::vector<u32> l_off, l_njobs, l_blocks;  // per launch
    std::vector<double> l_bytes, l_mods;         // algorithmic bytes and products per launch
    std::vector<u64> out_off;
    u64 out_words = 0;
    void *mem = nullptr;  // job tables, slots, gathered transcripts
    JobEntry *d_jobs = nullptr;
    BatchSlot *d_slots = nullptr;
    u64 *d_out = nullptr;
    BatchSlot *h_slots = nullptr;
    u64 *h_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    ~BatchPlan() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        for (Workspace *w : ws) free_workspace(w);
        if (mem) (void)hipFree(mem);
        if (h_slots) (void)hipHostFree(h_slots);
        if (h_out) (void)hipHostFree(h_out);
    }
};

std::mutex g_batch_mu;
std::vector<std::unique_ptr<BatchPlan>> g_batches;  // most recent last
constexpr size_t BATCH_CACHE = 4;

hipStream_t capture_stream() {
    static std::mutex mu;
    static std::vector<hipStream_t> streams;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
        return nullptr;
    return streams[dev];
}

// Enqueue a batch's launches (setup, steps, gather) on st.
int enqueue_batch(BatchPlan &B, hipStream_t st, bool profile) {
    const u32 n = (u32)B.ws.size();
    HIP_TRY(launch_batch_setup(st, B.d_slots, n));
    for (size_t t = 0; t < B.l_off.size(); t++) {
        hipEvent_t a = nullptr, b = nullptr;
        if (profile) prof_pair(PC_BATCH, B.l_bytes[t], &a, &b, B.l_mods[t]);
        HIP_TRY(launch_steps(st, B.d_jobs + B.l_off[t], B.l_njobs[t], B.l_blocks[t], a, b));
    }
    HIP_TRY(launch_batch_gather(st, B.d_slots, n, B.d_out));
    return GKR_OK;
}

int build_batch(const std::vector<gkr_circuit *> &cs, int flags, std::unique_ptr<BatchPlan> &out) {
    std::unique_ptr<BatchPlan> B(new BatchPlan());
    B->key = cs;
    B->flags = flags;
    B->epoch = g_tune_epoch.load();
    const u32 n = (u32)cs.size();
    for (gkr_circuit *c : cs) {
        Workspace *w = nullptr;
        std::lock_guard<std::mutex> lk(c->mu);
        if (c->mem_mode == GKR_MEM_LAYER)
            return fail(GKR_ERR_INVALID, "a copy-once-per-layer circuit is proved one proof at a time");
        int rc = make_workspace(c, c->mem_mode, &w);
        if (rc) return rc;
        B->ws.push_back(w);
    }
    // schedule: launch t holds step t - start[q] of proof q.  A proof starts
    // late enough that its ST_TOP step (the longest one-workgroup step) runs
    // in the same launch as every other proof's, instead of lengthening
    // launches of its own; proofs without one start at once.
    std::vector<size_t> start(n, 0);
    {
        std::vector<long> top_at(n, -1);
        long last_top = -1;
        for (u32 q = 0; q < n; q++) {
            const std::vector<StepDesc> &st = B->ws[q]->steps;
            for (size_t t = 0; t < st.size() && top_at[q] < 0; t++)
                if (st[t].kind == ST_TOP) top_at[q] = (long)t;
            last_top = std::max(last_top, top_at[q]);
        }
        for (u32 q = 0; q < n; q++)
            if (top_at[q] >= 0) start[q] = (size_t)(last_top - top_at[q]);
    }
    size_t T = 0;
    for (u32 q = 0; q < n; q++) T = std::max(T, start[q] + B->ws[q]->steps.size());
    std::vector<JobEntry> jobs;
    for (size_t t = 0; t < T; t++) {
        B->l_off.push_back((u32)jobs.size());
        u32 blocks = 0, nj = 0;
        double lb = 0, lm = 0;
        for (u32 q = 0; q < n; q++) {
            Workspace *w = B->ws[q];
            if (t < start[q] || t - start[q] >= w->steps.size()) continue;
            const size_t k = t - start[q];
            jobs.push_back(JobEntry{w->d_steps + k, blocks, 0});
            blocks += step_grid(w->steps[k]);
            lb += w->pbytes[k];
            lm += w->pmods[k];
            nj++;
        }
        if (!nj) {  // (no proof in this launch: none is planned)
            B->l_off.pop_back();
            continue;
        }
        B->l_bytes.push_back(lb);
        B->l_mods.push_back(lm);
        jobs.push_back(JobEntry{nullptr, blocks, 0});  // sentinel
        B->l_njobs.push_back(nj);
        B->l_blocks.push_back(blocks);
    }
    B->out_off.resize(n);
    u64 off = 0;
    for (u32 q = 0; q < n; q++) {
        B->out_off[q] = off;
        off += cs[q]->n_msgs + 1;  // transcript, then the range flag
    }
    B->out_words = off;
    Arena sz, a;
    auto lay = [&](Arena &ar) {
        B->d_jobs = ar.take<JobEntry>(jobs.size());
        B->d_slots = ar.take<BatchSlot>(n);
        B->d_out = ar.take<u64>(off);
    };
    lay(sz);
    HIP_TRY(hipMalloc(&B->mem, sz.used));
    a.base = (char *)B->mem;
    lay(a);
    HIP_TRY(hipMemcpy(B->d_jobs, jobs.data(), jobs.size() * sizeof(JobEntry), hipMemcpyHostToDevice));
    HIP_TRY(hipHostMalloc((void **)&B->h_slots, n * sizeof(BatchSlot)));
    HIP_TRY(hipHostMalloc((void **)&B->h_out, off * 8));
    for (u32 q = 0; q < n; q++) {
        BatchSlot &s = B->h_slots[q];
        s.state = B->ws[q]->state;
        s.seed = 0;
        s.input = 0;
        s.msgs = B->ws[q]->msgs;
        s.n_msgs = cs[q]->n_msgs;
        s.out_off = B->out_off[q];
        s.flag_off = B->out_off[q] + cs[q]->n_msgs;
    }
    if (flags & GKR_BATCH_GRAPH) {
        hipStream_t cst = capture_stream();
        if (!cst) return fail(GKR_ERR_DEVICE, "no capture stream");
        HIP_TRY(hipStreamBeginCapture(cst, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_batch(*B, cst, false);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(cst, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        HIP_TRY(e);
        B->graph = graph;
        HIP_TRY(hipGraphInstantiate(&B->gexec, graph, nullptr, nullptr, 0));
    }
    out = std::move(B);
    return GKR_OK;
}

}  // namespace

// Cached batch plans refer to the circuits' device arrays.
static void drop_batches_of(const gkr_circuit *c) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (size_t k = 0; k < g_batches.size();) {
        auto &key = g_batches[k]->key;
        if (std::find(key.begin(), key.end(), c) != key.end())
            g_batches.erase(g_batches.begin() + k);
        else
            k++;
    }
}

extern "C" int gkr_batch_prove(uint32_t n, const gkr_circuit *const *circuits,
                               const uint64_t *const *inputs, int inputs_on_device,
                               const uint64_t *seeds, uint64_t *const *msgs, int flags,
                               void *hip_stream) {
    if (n == 0) return GKR_OK;
    if (!circuits || !inputs || !seeds || !msgs) return fail(GKR_ERR_INVALID, "NULL argument");
    if (!inputs_on_device) return fail(GKR_ERR_INVALID, "batched inputs must be device pointers");
    for (u32 q = 0; q < n; q++)
        if (!circuits[q] || !inputs[q] || !msgs[q]) return fail(GKR_ERR_INVALID, "NULL entry");
    hipStream_t st = pick_stream(hip_stream);
    if (!st) return fail(GKR_ERR_DEVICE, "no stream");
    std::vector<gkr_circuit *> key(n);
    for (u32 q = 0; q < n; q++) key[q] = const_cast<gkr_circuit *>(circuits[q]);
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchPlan *B = nullptr;
    for (size_t k = 0; k < g_batches.size(); k++)
        if (g_batches[k]->key == key && g_batches[k]->flags == flags) {
            if (g_batches[k]->epoch != g_tune_epoch.load()) {  // planned with older shapes
                g_batches.erase(g_batches.begin() + k);
                break;
            }
            std::unique_ptr<BatchPlan> hit = std::move(g_batches[k]);
            g_batches.erase(g_batches.begin() + k);
            g_batches.push_back(std::move(hit));
            B = g_batches.back().get();
            break;
        }
    if (!B) {
        std::unique_ptr<BatchPlan> fresh;
        int rc = build_batch(key, flags, fresh);
        if (rc) return rc;
        if (g_batches.size() >= BATCH_CACHE) g_batches.erase(g_batches.begin());
        g_batches.push_back(std::move(fresh));
        B = g_batches.back().get();
    }
    for (u32 q = 0; q < n; q++) {
        B->h_slots[q].seed = seeds[q];
        B->h_slots[q].input = (u64)(uintptr_t)inputs[q];
    }
    HIP_TRY(hipMemcpyAsync(B->d_slots, B->h_slots, n * sizeof(BatchSlot), hipMemcpyHostToDevice, st));
    if (B->gexec && !g_prof.on) {
        HIP_TRY(hipGraphLaunch(B->gexec, st));
    } else {
        int rc = enqueue_batch(*B, st, g_prof.on);
        if (rc) return rc;
    }
    HIP_TRY(hipMemcpyAsync(B->h_out, B->d_out, B->out_words * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int rc = GKR_OK;
    for (u32 q = 0; q < n; q++) {
        memcpy(msgs[q], B->h_out + B->out_off[q], circuits[q]->n_msgs * 8);
        if (B->h_out[B->out_off[q] + circuits[q]->n_msgs]) rc = fail(GKR_ERR_RANGE, "input value not below p");
    }
    return rc;
}

// ----------------------------------------------------------------- verifier

namespace {

// Lagrange interpolation of y[0..D] at nodes 0..D, evaluated at x.
u64 lagrange_host(const u64 *y, u32 D, u64 x) {
    using namespace fp;
    u64 acc = 0;
    for (u32 i = 0; i <= D; i++) {
        u64 num = 1, den = 1;
        for (u32 j = 0; j <= D; j++) {
            if (j == i) continue;
            num = mul(num, sub(x, j));
            den = mul(den, sub(i, j));
        }
        acc = add(acc, mul(y[i], mul(num, inv(den))));
    }
    return acc;
}

// G(r) for a degree-2 message given at 0, 1, 2.
u64 quad_at(const u64 *G, u64 r) {
    using namespace fp;
    const u64 inv2 = 1ull << 60;  // 2 * 2^60 = 2^61 = 1
    const u64 r1 = sub(r, 1), r2 = sub(r, 2);
    u64 t0 = mul(mul(G[0], mul(r1, r2)), inv2);
    u64 t1 = mul(G[1], mul(r, r2));
    u64 t2 = mul(mul(G[2], mul(r, r1)), inv2);
    return add(sub(t0, t1), t2);
}

// ~T(pt) on the host by binding variables one at a time (small tables).
u64 mle_host(std::vector<u64> T, const u64 *pt, u32 s) {
    using namespace fp;
    for (u32 k = 0; k < s; k++) {
        const u64 h = 1ull << (s - k - 1);
        for (u64 m = 0; m < h; m++) T[m] = add(T[2 * m], mul(pt[k], sub(T[2 * m + 1], T[2 * m])));
    }
    return T[0];
}

struct VerifyScratch {
    std::mutex mu;
    int device = -1;
    void *mem = nullptr;
    size_t cap = 0;
    u64 *h_res = nullptr;
    size_t h_cap = 0;
};
VerifyScratch g_vs;

int vs_reserve(size_t bytes, size_t host_words) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (g_vs.device != dev || g_vs.cap < bytes) {
        if (g_vs.mem) (void)hipFree(g_vs.mem);
        g_vs.mem = nullptr;
        g_vs.cap = 0;
        HIP_TRY(hipMalloc(&g_vs.mem, bytes));
        g_vs.cap = bytes;
        g_vs.device = dev;
    }
    if (g_vs.h_cap < host_words) {
        if (g_vs.h_res) (void)hipHostFree(g_vs.h_res);
        g_vs.h_res = nullptr;
        HIP_TRY(hipHostMalloc((void **)&g_vs.h_res, host_words * 8));
        g_vs.h_cap = host_words;
    }
    return GKR_OK;
}

// Streamed input extension for host inputs (the verifier's one pass over
// the inputs, Sec. 4.1.2, through two buffers, one filling while the other
// is processed, as Sec. 4.2.2 suggests for a streaming verifier).  Chunks of
// VCHUNK values are copied from the
// caller's memory into two device buffers on a copy stream, chunk k into
// buffer k & 1 once the kernels that read that buffer before have finished;
// the caller's stream checks the chunk against p (u64 values, into *bad_dev)
// and adds its extension terms into the same per-workgroup rows while chunk
// k + 1 is copied.  Chunks start at multiples of VCHUNK, a multiple of 2^L
// for every table here (L <= 16).
constexpr u64 VCHUNK = 1ull << 23;

struct InputStream {  // one per device, created on first use, kept until exit
    hipStream_t cs = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr};
};
constexpr int IS_DEVICES = 64;
std::mutex g_is_mu;
InputStream g_is[IS_DEVICES];

// dbuf: device room for 2 min(n, VCHUNK) values.
template <typename T>
static int stream_mle(hipStream_t st, const T *in, u64 n, T *dbuf, const u64 *lo, const u64 *hi, u32 L,
                      u64 *partials, int *nb, u32 *bad_dev) {
    std::lock_guard<std::mutex> lk(g_is_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= IS_DEVICES) return fail(GKR_ERR_DEVICE, "device index beyond the input streams");
    InputStream &is = g_is[dev];
    if (!is.cs) {  // stream and events belong to this device
        HIP_TRY(hipStreamCreateWithFlags(&is.cs, hipStreamNonBlocking));
        for (int b = 0; b < 2; b++) {
            HIP_TRY(hipEventCreateWithFlags(&is.copied[b], hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&is.used[b], hipEventDisableTiming));
        }
    }
    const u64 C = std::min<u64>(n, VCHUNK);
    const int nbf = blocks_for(C, 8);
    u64 k = 0;
    for (u64 x0 = 0; x0 < n; x0 += C, k++) {
        const int b = (int)(k & 1);
        const u64 m = std::min<u64>(C, n - x0);
        if (k >= 2) HIP_TRY(hipStreamWaitEvent(is.cs, is.used[b], 0));
        HIP_TRY(hipMemcpyAsync(dbuf + b * C, in + x0, m * sizeof(T), hipMemcpyHostToDevice, is.cs));
        HIP_TRY(hipEventRecord(is.copied[b], is.cs));
        HIP_TRY(hipStreamWaitEvent(st, is.copied[b], 0));
        const u64 *t64 = sizeof(T) == 8 ? (const u64 *)(dbuf + b * C) : nullptr;
        const u32 *t32 = sizeof(T) == 4 ? (const u32 *)(dbuf + b * C) : nullptr;
        if (t64) HIP_TRY(launch_check_range(st, t64, m, bad_dev));
        HIP_TRY(launch_mle(st, m, t64, t32, lo, hi + (x0 >> L), L, partials, nb, k > 0, nbf));
        HIP_TRY(hipEventRecord(is.used[b], st));
    }
    return GKR_OK;
}

void reject(int *accepted, gkr_reject_info *why, int layer, int round, int check) {
    *accepted = 0;
    if (why) {
        why->layer = layer;
        why->round = round;
        why->check = check;
    }
}

}  // namespace

extern "C" int gkr_verify(const gkr_circuit *c, const uint64_t *inputs, int inputs_on_device,
                          uint64_t seed, const uint64_t *msgs, uint64_t n_msgs, int *accepted,
                          gkr_reject_info *why, void *hip_stream) {
    using namespace fp;
    if (!c || !inputs || !accepted || (!msgs && n_msgs)) return fail(GKR_ERR_INVALID, "NULL argument");
    hipStream_t st = pick_stream(hip_stream);
    if (!st) return fail(GKR_ERR_DEVICE, "no stream");
    *accepted = 0;
    if (why) *why = {-1, -1, 0};
    const u32 d = c->L - 1;
    const u64 Sd = c->S[d];
    if (n_msgs != c->n_msgs) {
        reject(accepted, why, -1, -1, GKR_CHECK_MALFORMED);
        return GKR_OK;
    }
    for (u64 k = 0; k < n_msgs; k++)
        if (msgs[k] >= P) {
            reject(accepted, why, -1, -1, GKR_CHECK_MALFORMED);
            return GKR_OK;
        }
    // The verifier's own coins: same stream as the prover's challenges.
    std::vector<u64> ch(c->n_chals);
    u64 rs = sm_state(seed, PURPOSE_GKR);
    for (auto &x : ch) x = sm_field(rs);
    // z_{i} for every layer; z_{i+1} = l(tau) of layer i.
    std::vector<std::vector<u64>> z(c->L);
    z[0].assign(ch.begin(), ch.begin() + c->s[0]);
    for (u32 i = 0; i < d; i++) {
        const u32 s = c->s[i], sp = c->s[i + 1], n = s + 2 * sp;
        const u64 *r = ch.data() + c->co[i];
        const u64 tau = r[n];
        z[i + 1].resize(sp);
        for (u32 k = 0; k < sp; k++) z[i + 1][k] = add(r[s + k], mul(tau, sub(r[s + sp + k], r[s + k])));
    }
    // Device part: add~ / mult~ per layer, and the inputs' extension at z_d.
    std::lock_guard<std::mutex> lk(g_vs.mu);
    Arena sz;
    const u64 npts = c->n_chals + c->s[d] + 8;
    struct {
        u64 *pts, *tab, *partials, *res, *in;
        u32 *flag;
    } v;
    auto lay = [&](Arena &a) {
        v.pts = a.take<u64>(npts);
        v.tab = a.take<u64>(6ull * HALF_MAX);
        v.partials = a.take<u64>((u64)MAX_BLOCKS * 4);
        v.res = a.take<u64>(2ull * d + 2);
        v.in = a.take<u64>(inputs_on_device ? 1 : 2 * std::min<u64>(Sd, VCHUNK));
        v.flag = a.take<u32>(1);
    };
    lay(sz);
    int rc = vs_reserve(sz.used, 2ull * d + 3);
    if (rc) return rc;
    Arena a;
    a.base = (char *)g_vs.mem;
    lay(a);
    // points: chals as drawn, then z_d
    std::vector<u64> pts(npts, 0);
    std::copy(ch.begin(), ch.end(), pts.begin());
    std::copy(z[d].begin(), z[d].end(), pts.begin() + c->n_chals);
    HIP_TRY(hipMemcpyAsync(v.pts, pts.data(), npts * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(v.flag, 0, 4, st));
    if (inputs_on_device) LAUNCH(PC_MISC, Sd * 8.0, launch_check_range(st, inputs, Sd, v.flag));
    u64 *T = v.tab;
    int nb = 0;
    const bool closed = g_closed_forms.load() != 0;
    for (u32 i = 0; i < d; i++) {
        if (closed && c->form[i] != GKR_WIRING_GATES) continue;  // on the host below
        const u32 s = c->s[i], sp = c->s[i + 1];
        const u64 *r = v.pts + c->co[i];
        u32 La, Lb;
        split_half(s, &La);
        split_half(sp, &Lb);
        LAUNCH(PC_TABLES, 0, launch_eq_halves(st, r, s, La, T, T + HALF_MAX));
        LAUNCH(PC_TABLES, 0, launch_eq_halves(st, r + s, sp, Lb, T + 2 * HALF_MAX, T + 3 * HALF_MAX));
        LAUNCH(PC_TABLES, 0,
               launch_eq_halves(st, r + s + sp, sp, Lb, T + 4 * HALF_MAX, T + 5 * HALF_MAX));
        WiringArgs wa;
        wa.kind = c->kind[i];
        wa.S = c->S[i];
        wa.type = c->type[i];
        wa.in1 = c->in1[i];
        wa.in2 = c->in2[i];
        wa.alo = T;
        wa.ahi = T + HALF_MAX;
        wa.La = La;
        wa.blo = T + 2 * HALF_MAX;
        wa.bhi = T + 3 * HALF_MAX;
        wa.Lb = Lb;
        wa.clo = T + 4 * HALF_MAX;
        wa.chi = T + 5 * HALF_MAX;
        wa.Lc = Lb;
        wa.partials = v.partials;
        LAUNCH(PC_WIRING, c->S[i] * 8.0, launch_wiring(st, wa, &nb));
        LAUNCH(PC_MISC, 0, launch_reduce_rows(st, nb, 2, v.partials, v.res + 2 * i));
    }
    {
        const u32 sd = c->s[d];
        u32 Ld;
        split_half(sd, &Ld);
        LAUNCH(PC_TABLES, 0, launch_eq_halves(st, v.pts + c->n_chals, sd, Ld, T, T + HALF_MAX));
        if (inputs_on_device) {
            LAUNCH(PC_MLE, Sd * 8.0, launch_mle(st, Sd, inputs, nullptr, T, T + HALF_MAX, Ld, v.partials, &nb));
        } else {
            rc = stream_mle<u64>(st, inputs, Sd, v.in, T, T + HALF_MAX, Ld, v.partials, &nb, v.flag);
            if (rc) return rc;
        }
        LAUNCH(PC_MISC, 0, launch_reduce_rows(st, nb, 1, v.partials, v.res + 2 * d));
    }
    HIP_TRY(hipMemcpyAsync(g_vs.h_res, v.res, (2ull * d + 1) * 8, hipMemcpyDeviceToHost, st));
    g_vs.h_res[2ull * d + 1] = 0;
    HIP_TRY(hipMemcpyAsync(g_vs.h_res + 2ull * d + 1, v.flag, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if ((uint32_t)g_vs.h_res[2ull * d + 1])
        return fail(GKR_ERR_RANGE, "input value not below p");
    const u64 *res = g_vs.h_res;
    // Host replay of the protocol (a10).
    u64 mi = 0;
    std::vector<u64> outs(1ull << c->s[0], 0);
    for (u32 g = 0; g < c->S[0]; g++) outs[g] = msgs[mi++];
    u64 claim = mle_host(outs, z[0].data(), c->s[0]);
    for (u32 i = 0; i < d; i++) {
        const u32 s = c->s[i], sp = c->s[i + 1], n = s + 2 * sp;
        const u64 *r = ch.data() + c->co[i];
        for (u32 j = 0; j < n; j++) {
            const u64 *G = msgs + mi;
            mi += 3;
            if (add(G[0], G[1]) != claim) {
                reject(accepted, why, (int)i, (int)j, GKR_CHECK_ROUND);
                return GKR_OK;
            }
            claim = quad_at(G, r[j]);
        }
        const u64 v1 = msgs[mi++], v2 = msgs[mi++];
        u64 beta = 1;
        for (u32 k = 0; k < s; k++) beta = mul(beta, eq(z[i][k], r[k]));
        u64 addv = res[2 * i], mulv = res[2 * i + 1];
        if (closed && c->form[i] != GKR_WIRING_GATES) {
            const u64 w = wiring_closed(c->form[i], c->S[i], s, sp, r, r + s, r + s + sp);
            addv = c->kind[i] == KIND_ADD ? w : 0;
            mulv = c->kind[i] == KIND_MUL ? w : 0;
        }
        const u64 rhs = mul(beta, add(mul(addv, add(v1, v2)), mul(mulv, mul(v1, v2))));
        if (rhs != claim) {
            reject(accepted, why, (int)i, (int)n, GKR_CHECK_WIRING);
            return GKR_OK;
        }
        if (sp == 0 && v1 != v2) {
            reject(accepted, why, (int)i, -1, GKR_CHECK_LINE);
            return GKR_OK;
        }
        std::vector<u64> y(std::max<u32>(sp, 1) + 1);
        y[0] = v1;
        y[1] = v2;
        for (u32 t = 2; t <= sp; t++) y[t] = msgs[mi++];
        claim = lagrange_host(y.data(), std::max<u32>(sp, 1), r[n]);
    }
    if (res[2 * d] != claim) {
        reject(accepted, why, (int)d, -1, GKR_CHECK_INPUT);
        return GKR_OK;
    }
    *accepted = 1;
    return GKR_OK;
}

// --------------------------------------------------------- F2 sum-check

namespace {

struct F2Scratch {
    std::mutex mu;
    int device = -1;
    void *mem = nullptr;
    size_t cap = 0;
    u64 *h = nullptr;
    size_t h_cap = 0;
} g_f2;

int f2_reserve(size_t bytes, size_t host_words) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (g_f2.device != dev || g_f2.cap < bytes) {
        if (g_f2.mem) (void)hipFree(g_f2.mem);
        g_f2.mem = nullptr;
        g_f2.cap = 0;
        HIP_TRY(hipMalloc(&g_f2.mem, bytes));
        g_f2.cap = bytes;
        g_f2.device = dev;
    }
    if (g_f2.h_cap < host_words) {
        if (g_f2.h) (void)hipHostFree(g_f2.h);
        g_f2.h = nullptr;
        HIP_TRY(hipHostMalloc((void **)&g_f2.h, host_words * 8));
        g_f2.h_cap = host_words;
    }
    return GKR_OK;
}

bool pow2(u64 n) { return n && !(n & (n - 1)); }

}  // namespace

// Scratch of one F2 sum-check proof at base (sized when base is NULL):
// the two folded tables, two rounds' partial rows, the transcript and
// challenges on the device, the challenge stream's state and, for host
// inputs, their staging copy.
struct F2scLayout {
    u64 *A0, *A1, *partials, *msgs, *chals;
    ProofState *ps;
    u32 *in;
};
static size_t f2sc_layout(char *base, u64 n, int on_device, F2scLayout &v) {
    const u32 l = log2ceil(n);
    Arena a;
    a.base = base;
    v.A0 = a.take<u64>(std::max<u64>(n / 2, 2));
    v.A1 = a.take<u64>(std::max<u64>(n / 4, 2));
    v.partials = a.take<u64>((u64)MAX_BLOCKS * 6);  // two rounds' rows
    v.msgs = a.take<u64>(1 + 3ull * l);
    v.chals = a.take<u64>(std::max<u32>(l, 1));
    v.ps = a.take<ProofState>(1);
    v.in = a.take<u32>(on_device ? 1 : n);
    return a.used;
}

// Enqueue one F2 sum-check proof on st into the scratch v lays out (host
// inputs are first copied into v.in); the transcript stays on the device.
static int f2sc_enqueue(const uint32_t *freq, u64 n, int on_device, u64 seed, const F2scLayout &v,
                        hipStream_t st) {
    const u32 l = log2ceil(n);
    const u32 *a32 = freq;
    if (!on_device) {
        HIP_TRY(hipMemcpyAsync(v.in, freq, n * 4, hipMemcpyHostToDevice, st));
        a32 = v.in;
    }
    int nb = 0;
    if (l == 0) {
        LAUNCH(PC_MISC, 4, launch_f2sc_single(st, a32, v.msgs));
        return GKR_OK;
    }
    LAUNCH(PC_MISC, 0, launch_f2sc_init(st, v.ps, seed));
    u64 *bufs[2] = {v.A0, v.A1};
    const u64 *src = nullptr;
    // round j's launch also finishes round j - 1 (its message and
    // challenge), so the challenge is drawn one launch after its sums
    int prev = 0;
    // rounds from j0 on run as one tail once level j0 fits it
    u32 j0 = l;
    if (l >= 3) j0 = std::max<u32>(2, l > 12 ? l - 12 : 2);
    for (u32 j = 0; j < j0; j++) {
        const u64 pairs = n >> (j + 1);
        u64 *dst = j == 0 ? nullptr : bufs[(j + 1) & 1];
        const double bytes = j == 0 ? pairs * 8.0 : (j == 1 ? pairs * 32.0 : pairs * 48.0);
        u64 *pmsg = j ? v.msgs + 1 + 3 * (j - 1) : nullptr, *pchal = j ? v.chals + j - 1 : nullptr;
        LAUNCH(PC_F2SC, bytes,
               launch_f2sc_round(st, (int)j, pairs, a32, src, dst, v.ps, v.partials, prev, pmsg, pchal,
                                 j == 1 ? v.msgs : nullptr, &nb));
        prev = nb;
        if (j > 0) src = dst;
    }
    if (j0 < l)
        LAUNCH(PC_FINAL, (n >> (j0 - 1)) * 8.0,
               launch_f2sc_tail(st, (int)j0, (int)l, src, prev, v.partials, v.ps, v.msgs, v.chals));
    else
        LAUNCH(PC_FINAL, prev * 24.0,
               launch_f2sc_final(st, (int)(l - 1), prev, v.partials, v.ps, v.msgs + 1 + 3 * (l - 1),
                                 v.chals + l - 1, l == 1 ? v.msgs : nullptr));
    return GKR_OK;
}

static int f2sc_check(const uint32_t *freq, u64 n, const uint64_t *msgs) {
    if (!freq || !msgs) return fail(GKR_ERR_INVALID, "NULL argument");
    if (!pow2(n) || n > (1ull << 32)) return fail(GKR_ERR_INVALID, "n must be a power of two <= 2^32");
    return GKR_OK;
}

extern "C" int f2_sumcheck_prove(const uint32_t *freq, uint64_t n, int on_device, uint64_t seed,
                                 uint64_t *msgs, uint64_t *chals, void *hip_stream) {
    int rc = f2sc_check(freq, n, msgs);
    if (rc) return rc;
    hipStream_t st = pick_stream(hip_stream);
    if (!st) return fail(GKR_ERR_DEVICE, "no stream");
    const u32 l = log2ceil(n);
    const u64 nm = 1 + 3ull * l;
    std::lock_guard<std::mutex> lk(g_f2.mu);
    F2scLayout v;
    rc = f2_reserve(f2sc_layout(nullptr, n, on_device, v), nm + l + 1);
    if (rc) return rc;
    f2sc_layout((char *)g_f2.mem, n, on_device, v);
    rc = f2sc_enqueue(freq, n, on_device, seed, v, st);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(g_f2.h, v.msgs, nm * 8, hipMemcpyDeviceToHost, st));
    if (chals && l) HIP_TRY(hipMemcpyAsync(g_f2.h + nm, v.chals, l * 8ull, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    memcpy(msgs, g_f2.h, nm * 8);
    if (chals && l) memcpy(chals, g_f2.h + nm, l * 8ull);
    return GKR_OK;
}

// ------------------------------------- F2 sum-check without allocation

// The scratch of f2_sumcheck_prove_noalloc: one static array per device,
// held from the module's load on that device until the process ends.
constexpr u64 F2SC_NOALLOC_MAX_N = 1ull << 22;
constexpr size_t F2SC_NOALLOC_BYTES = 48ull << 20;
static __device__ __align__(256) char scratch[F2SC_NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
struct NoallocScratch {
    std::mutex mu;                            // one proof at a time in this process
    void *ptr[NOALLOC_MAX_DEVICES] = {};      // device address of `scratch` on each device
} g_noalloc;
}  // namespace

extern "C" int f2_sumcheck_prove_noalloc(const uint32_t *freq, uint64_t n, int on_device, uint64_t seed,
                                         uint64_t *msgs, uint64_t *chals, void *hip_stream) {
    int rc = f2sc_check(freq, n, msgs);
    if (rc) return rc;
    if (n > F2SC_NOALLOC_MAX_N) return fail(GKR_ERR_NOMEM, "n above 2^22, the static scratch's limit");
    F2scLayout v;
    if (f2sc_layout(nullptr, n, on_device, v) > F2SC_NOALLOC_BYTES)
        return fail(GKR_ERR_NOMEM, "the proof's scratch exceeds the static scratch array");
    hipStream_t st = pick_stream(hip_stream);
    if (!st) return fail(GKR_ERR_DEVICE, "no stream");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(GKR_ERR_DEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_noalloc.mu);
    if (!g_noalloc.ptr[dev]) {  // once per device, with that device current
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(GKR_ERR_DEVICE, "no device address for the static scratch");
        g_noalloc.ptr[dev] = p;
    }
    f2sc_layout((char *)g_noalloc.ptr[dev], n, on_device, v);
    rc = f2sc_enqueue(freq, n, on_device, seed, v, st);
    if (rc) return rc;
    const u32 l = log2ceil(n);
    HIP_TRY(hipMemcpyAsync(msgs, v.msgs, (1 + 3ull * l) * 8, hipMemcpyDeviceToHost, st));
    if (chals && l) HIP_TRY(hipMemcpyAsync(chals, v.chals, l * 8ull, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GKR_OK;
}

extern "C" int f2_sumcheck_verify(const uint32_t *freq, uint64_t n, int on_device, uint64_t seed,
                                  const uint64_t *msgs, uint64_t n_msgs, int *accepted,
                                  gkr_reject_info *why, void *hip_stream) {
    using namespace fp;
    if (!freq || !accepted || (!msgs && n_msgs)) return fail(GKR_ERR_INVALID, "NULL argument");
    if (!pow2(n) || n > (1ull << 32)) return fail(GKR_ERR_INVALID, "n must be a power of two <= 2^32");
    hipStream_t st = pick_stream(hip_stream);
    if (!st) return fail(GKR_ERR_DEVICE, "no stream");
    *accepted = 0;
    if (why) *why = {-1, -1, 0};
    const u32 l = log2ceil(n);
    if (n_msgs != 1 + 3ull * l) {
        reject(accepted, why, -1, -1, GKR_CHECK_MALFORMED);
        return GKR_OK;
    }
    for (u64 k = 0; k < n_msgs; k++)
        if (msgs[k] >= P) {
            reject(accepted, why, -1, -1, GKR_CHECK_MALFORMED);
            return GKR_OK;
        }
    std::vector<u64> r(l);
    u64 rs = sm_state(seed, PURPOSE_F2SC);
    for (auto &x : r) x = sm_field(rs);
    u64 claim = msgs[0];
    for (u32 j = 0; j < l; j++) {
        const u64 *G = msgs + 1 + 3 * j;
        if (add(G[0], G[1]) != claim) {
            reject(accepted, why, -1, (int)j, GKR_CHECK_ROUND);
            return GKR_OK;
        }
        claim = quad_at(G, r[j]);
    }
    // ~a(r) on the device, one pass over the vector (the verifier's secret,
    // Sec. 4.1.2; its pass parallel over the input symbols, Sec. 4.2.2)
    std::lock_guard<std::mutex> lk(g_f2.mu);
    struct {
        u64 *pts, *tab, *partials, *res;
        u32 *in;
    } v;
    auto lay = [&](Arena &a) {
        v.pts = a.take<u64>(l + 1);
        v.tab = a.take<u64>(2ull * HALF_MAX);
        v.partials = a.take<u64>((u64)MAX_BLOCKS);
        v.res = a.take<u64>(1);
        v.in = a.take<u32>(on_device ? 1 : 2 * std::min<u64>(n, VCHUNK));
    };
    Arena sz;
    lay(sz);
    int rc = f2_reserve(sz.used, 2);
    if (rc) return rc;
    Arena a;
    a.base = (char *)g_f2.mem;
    lay(a);
    if (l) HIP_TRY(hipMemcpyAsync(v.pts, r.data(), l * 8ull, hipMemcpyHostToDevice, st));
    u32 L;
    split_half(l, &L);
    int nb = 0;
    LAUNCH(PC_TABLES, 0, launch_eq_halves(st, v.pts, l, L, v.tab, v.tab + HALF_MAX));
    if (on_device) {
        LAUNCH(PC_MLE, n * 4.0, launch_mle(st, n, nullptr, freq, v.tab, v.tab + HALF_MAX, L, v.partials, &nb));
    } else {
        rc = stream_mle<u32>(st, freq, n, v.in, v.tab, v.tab + HALF_MAX, L, v.partials, &nb, nullptr);
        if (rc) return rc;
    }
    LAUNCH(PC_MISC, 0, launch_reduce_rows(st, nb, 1, v.partials, v.res));
    HIP_TRY(hipMemcpyAsync(g_f2.h, v.res, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const u64 ar = g_f2.h[0];
    if (mul(ar, ar) != claim) {
        reject(accepted, why, -1, -1, GKR_CHECK_INPUT);
        return GKR_OK;
    }
    *accepted = 1;
    return GKR_OK;
}

// -------------------------------------------------------------- field check

extern "C" int gkr_field_op(int op, const uint64_t *a, const uint64_t *b, uint64_t *out, uint64_t n,
                            void *hip_stream) {
    if (op < 0 || op > 4 || (n && (!a || !b || !out))) return fail(GKR_ERR_INVALID, "bad argument");
    hipStream_t st = pick_stream(hip_stream);
    if (!st) return fail(GKR_ERR_DEVICE, "no stream");
    if (n == 0) return GKR_OK;
    HIP_TRY(launch_field_op(st, op, a, b, out, n));
    HIP_TRY(hipStreamSynchronize(st));
    return GKR_OK;
}

// ------------------------------------------------------------------ serving
//
// Continuous batching: a scheduler thread keeps up to max_slots proofs in
// flight.  Every launch runs the next step of each in-flight proof (job
// table in the kernel arguments), so a request that arrives while others run
// joins at the next launch.  A request is admitted when a slot is free and
// its scratch fits the HBM budget; its scratch comes from a per-circuit pool
// and returns there when the proof completes.

namespace {

struct ServeReq {
    u64 id = 0;
    gkr_circuit *c = nullptr;
    Workspace *ws = nullptr;
    u64 seed = 0;
    std::vector<u64> inputs;  // copied at submission
    size_t next = 0;          // next step of its program
    hipEvent_t done_ev = nullptr;
    u64 *h_out = nullptr;     // pinned: transcript, then the range flag
    std::chrono::steady_clock::time_point t_submit, t_done;
    int state = 0;            // 0 queued, 1 running, 2 finishing, 3 done
    int err = GKR_OK;
    std::string msg;          // what failed, when err != GKR_OK
};

size_t workspace_bytes(const Workspace *w) { return w ? w->bytes : 0; }

}  // namespace

struct gkr_server {
    u64 budget = 0, used = 0;
    u32 max_slots = 1;
    int device = 0;
    hipStream_t st = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<ServeReq *> queued;
    std::vector<ServeReq *> running, finishing;
    std::unordered_map<u64, ServeReq *> reqs;
    std::unordered_map<gkr_circuit *, std::vector<Workspace *>> pool;  // idle scratch
    u64 next_id = 1;
    bool stop = false;
    std::thread worker;
    std::vector<hipEvent_t> ring;  // bounds how far the host runs ahead of the GPU
    size_t ring_pos = 0;
    std::string err;

    // Frees one workspace this server accounts for.
    void drop(Workspace *w) {
        used -= std::min<u64>(used, w->bytes);
        free_workspace(w);
    }

    // Scratch for r: pooled, or new if the budget allows (idle pooled scratch
    // of other circuits is released first).  1: got it; 0: wait for running
    // proofs to return scratch; < 0: error (the request fails, r->msg says
    // why).  Pooled scratch made before the circuit's program changed
    // (another omega algorithm) is discarded.
    int acquire(ServeReq *r) {
        auto &v = pool[r->c];
        while (!v.empty()) {
            Workspace *w = v.back();
            v.pop_back();
            int rc;
            {
                std::lock_guard<std::mutex> lk(r->c->mu);
                rc = w->gen != r->c->gen ? 1 : refresh_plan(r->c, *w);
            }
            if (rc == GKR_OK) {
                r->ws = w;
                return 1;
            }
            drop(w);  // stale or not re-plannable: make a fresh one below
        }
        // resident scratch if the circuit is resident and it fits the
        // budget, else the out-of-core placement whose rounds read their
        // tables in place from host memory (Sec. 5.1.3)
        size_t need = 0;
        int mode = GKR_MEM_RESIDENT;
        {
            std::lock_guard<std::mutex> lk(r->c->mu);
            int rc = GKR_OK;
            if (r->c->mem_mode == GKR_MEM_RESIDENT) rc = workspace_size(r->c, GKR_MEM_RESIDENT, &need);
            if (!rc && (r->c->mem_mode != GKR_MEM_RESIDENT || need > budget)) {
                mode = GKR_MEM_MESSAGE;
                rc = workspace_size(r->c, mode, &need);
            }
            if (rc) {
                r->msg = g_err;
                return rc;
            }
        }
        if (need > budget) {
            r->msg = "a proof's scratch exceeds the server's HBM budget";
            return GKR_ERR_NOMEM;
        }
        while (used + need > budget) {
            bool freed = false;
            for (auto &kv : pool)
                if (!kv.second.empty()) {
                    drop(kv.second.back());
                    kv.second.pop_back();
                    freed = true;
                    break;
                }
            if (!freed) break;
        }
        if (used + need > budget) return 0;  // wait for running proofs to return scratch
        Workspace *w = nullptr;
        {
            std::lock_guard<std::mutex> lk(r->c->mu);
            const int rc = make_workspace(r->c, mode, &w);
            if (rc) {
                r->msg = g_err;
                return rc;
            }
        }
        used += w->bytes;
        r->ws = w;
        return 1;
    }

    void release(ServeReq *r) {
        if (r->ws) pool[r->c].push_back(r->ws);
        r->ws = nullptr;
    }

    // Idle scratch of circuit c (being destroyed, or its program changed).
    void forget(const gkr_circuit *c) {
        auto it = pool.find(const_cast<gkr_circuit *>(c));
        if (it == pool.end()) return;
        for (Workspace *w : it->second) drop(w);
        pool.erase(it);
    }

    int start(ServeReq *r) {
        Workspace &w = *r->ws;
        const u64 Sd = r->inputs.size();
        HIP_TRY(hipMemcpyAsync(w.instage, r->inputs.data(), Sd * 8, hipMemcpyDefault, st));
        w.h_setup[0] = r->seed;
        w.h_setup[1] = (u64)(uintptr_t)w.instage;
        w.h_setup[2] = 0;
        HIP_TRY(hipMemcpyAsync(w.state + 2, w.h_setup, 3 * 8, hipMemcpyHostToDevice, st));
        return GKR_OK;
    }

    void loop() {
        if (hipSetDevice(device) != hipSuccess) return;
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            // admission: free slot and scratch within the budget
            while (!queued.empty() && running.size() + finishing.size() < max_slots) {
                ServeReq *r = queued.front();
                const int got = acquire(r);
                if (got == 0) break;
                queued.pop_front();
                r->err = got < 0 ? got : start(r);
                if (r->err) {
                    if (got > 0) r->msg = g_err;  // start() failed
                    r->state = 3;
                    release(r);
                    cv.notify_all();
                    continue;
                }
                r->state = 1;
                r->next = 0;
                running.push_back(r);
            }
            // completions
            bool freed = false;
            for (size_t k = 0; k < finishing.size();) {
                ServeReq *r = finishing[k];
                if (hipEventQuery(r->done_ev) == hipSuccess) {
                    r->t_done = std::chrono::steady_clock::now();
                    if (r->h_out[r->c->n_msgs]) {
                        r->err = GKR_ERR_RANGE;
                        r->msg = "input value not below p";
                    }
                    r->state = 3;
                    release(r);
                    finishing.erase(finishing.begin() + k);
                    freed = true;
                } else {
                    k++;
                }
            }
            if (freed) cv.notify_all();
            if (freed && !queued.empty()) continue;  // returned scratch or slots: admit again
            if (running.empty()) {
                // nothing to launch: sleep until a submission (untimed only
                // when nothing is queued or finishing)
                if (finishing.empty() && queued.empty())
                    cv.wait(lk);
                else
                    cv.wait_for(lk, std::chrono::microseconds(20));
                continue;
            }
            // one launch: the next step of every running proof
            JobTable t;
            t.n = 0;
            t.total = 0;
            double lb = 0, lm = 0;
            for (ServeReq *r : running) {
                const StepDesc &sd = r->ws->steps[r->next];
                t.e[t.n++] = JobEntry{r->ws->d_steps + r->next, t.total, 0};
                t.total += step_grid(sd);
                lb += r->ws->pbytes[r->next];
                lm += r->ws->pmods[r->next];
            }
            t.e[t.n] = JobEntry{nullptr, t.total, 0};
            lk.unlock();
            // keep at most ring.size() launches in flight
            hipEvent_t &slot = ring[ring_pos];
            (void)hipEventSynchronize(slot);
            hipEvent_t pa = nullptr, pb = nullptr;
            prof_pair(PC_SERVE, lb, &pa, &pb, lm);
            if (pa) (void)hipEventRecord(pa, st);
            hipError_t e = launch_step_table(st, t);
            if (pb) (void)hipEventRecord(pb, st);
            if (e == hipSuccess) e = hipEventRecord(slot, st);
            ring_pos = (ring_pos + 1) % ring.size();
            lk.lock();
            if (e != hipSuccess) {
                // the proofs of the failed launch end with an error; their
                // scratch may be mid-step, so it is freed rather than pooled
                err = std::string("step launch failed: ") + hipGetErrorString(e);
                for (ServeReq *r : running) {
                    r->err = GKR_ERR_DEVICE;
                    r->msg = err;
                    r->state = 3;
                    if (r->ws) drop(r->ws);
                    r->ws = nullptr;
                }
                running.clear();
                cv.notify_all();
                continue;
            }
            for (size_t k = 0; k < running.size();) {
                ServeReq *r = running[k];
                r->next++;
                if (r->next == r->ws->steps.size()) {
                    // transcript and range flag back to the host
                    Workspace &w = *r->ws;
                    (void)hipMemcpyAsync(r->h_out, w.msgs, r->c->n_msgs * 8, hipMemcpyDeviceToHost, st);
                    (void)hipMemcpyAsync(r->h_out + r->c->n_msgs, w.state + 4, 8, hipMemcpyDeviceToHost, st);
                    (void)hipEventRecord(r->done_ev, st);
                    r->state = 2;
                    finishing.push_back(r);
                    running.erase(running.begin() + k);
                } else {
                    k++;
                }
            }
        }
    }
};

// Live servers, so that a circuit's idle pooled scratch (whose step
// programs point into the circuit's device arrays) is freed with the
// circuit or when its program changes.
static std::mutex g_servers_mu;
static std::vector<gkr_server *> g_servers;

static void drop_served_scratch_of(const gkr_circuit *c) {
    std::lock_guard<std::mutex> lk(g_servers_mu);
    for (gkr_server *s : g_servers) {
        std::lock_guard<std::mutex> sl(s->mu);
        s->forget(c);
    }
}

extern "C" int gkr_server_create(uint64_t hbm_budget_bytes, uint32_t max_slots, gkr_server **out) {
    if (!out) return fail(GKR_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > (u32)MAX_TABLE_JOBS - 1)
        return fail(GKR_ERR_INVALID, "max_slots must be in [1, 127]");
    std::unique_ptr<gkr_server> s(new gkr_server());
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    HIP_TRY(hipGetDevice(&s->device));
    HIP_TRY(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
    s->ring.resize(64);
    for (auto &e : s->ring) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    gkr_server *raw = s.get();
    s->worker = std::thread([raw] { raw->loop(); });
    {
        std::lock_guard<std::mutex> lk(g_servers_mu);
        g_servers.push_back(raw);
    }
    *out = s.release();
    return GKR_OK;
}

extern "C" int gkr_server_submit(gkr_server *s, const gkr_circuit *c, const uint64_t *inputs,
                                 uint64_t seed, uint64_t *req_id) {
    if (!s || !c || !inputs || !req_id) return fail(GKR_ERR_INVALID, "NULL argument");
    const u64 Sd = c->S[c->L - 1];
    for (u64 g = 0; g < Sd; g++)
        if (inputs[g] >= fp::P) return fail(GKR_ERR_RANGE, "input value not below p");
    std::unique_ptr<ServeReq> r(new ServeReq());
    r->c = const_cast<gkr_circuit *>(c);
    r->seed = seed;
    r->inputs.assign(inputs, inputs + Sd);
    HIP_TRY(hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming));
    HIP_TRY(hipHostMalloc((void **)&r->h_out, (c->n_msgs + 1) * 8));
    r->t_submit = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    *req_id = r->id;
    ServeReq *raw = r.release();
    s->reqs[raw->id] = raw;
    s->queued.push_back(raw);
    s->cv.notify_all();
    return GKR_OK;
}

extern "C" int gkr_server_poll(gkr_server *s, uint64_t req_id, uint64_t *msgs, int *done,
                               double *latency_s) {
    if (!s || !done) return fail(GKR_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return fail(GKR_ERR_INVALID, "unknown request");
    ServeReq *r = it->second;
    *done = r->state == 3;
    if (!*done) return GKR_OK;
    const int err = r->err;
    const std::string msg = r->msg.empty() ? s->err : r->msg;
    if (!err && msgs) memcpy(msgs, r->h_out, r->c->n_msgs * 8);
    if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    (void)hipEventDestroy(r->done_ev);
    (void)hipHostFree(r->h_out);
    s->reqs.erase(it);
    delete r;
    if (err) return fail(err, msg);
    return GKR_OK;
}

extern "C" int gkr_server_stats(gkr_server *s, uint32_t *running, uint32_t *queued,
                                uint64_t *hbm_used) {
    if (!s) return fail(GKR_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (running) *running = (u32)(s->running.size() + s->finishing.size());
    if (queued) *queued = (u32)s->queued.size();
    if (hbm_used) *hbm_used = s->used;
    return GKR_OK;
}

extern "C" void gkr_server_destroy(gkr_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(g_servers_mu);
        g_servers.erase(std::remove(g_servers.begin(), g_servers.end(), s), g_servers.end());
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->st);
    for (auto &kv : s->reqs) {
        if (kv.second->ws) free_workspace(kv.second->ws);
        (void)hipEventDestroy(kv.second->done_ev);
        (void)hipHostFree(kv.second->h_out);
        delete kv.second;
    }
    for (auto &kv : s->pool)
        for (Workspace *w : kv.second) free_workspace(w);
    for (auto &e : s->ring) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(s->st);
    delete s;
}

// ------------------------------------------------- non-interactive F2

namespace {

struct Nif2Scratch {
    std::mutex mu;
    int device = -1;
    void *mem = nullptr;
    size_t cap = 0;
    u64 *h = nullptr;  // pinned: the proof and two verifier values
    size_t h_cap = 0;
} g_nif2;

int nif2_reserve(size_t bytes, size_t host_words) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (g_nif2.device != dev || g_nif2.cap < bytes) {
        if (g_nif2.mem) (void)hipFree(g_nif2.mem);
        g_nif2.mem = nullptr;
        g_nif2.cap = 0;
        HIP_TRY(hipMalloc(&g_nif2.mem, bytes));
        g_nif2.cap = bytes;
        g_nif2.device = dev;
    }
    if (g_nif2.h_cap < host_words) {
        if (g_nif2.h) (void)hipHostFree(g_nif2.h);
        g_nif2.h = nullptr;
        g_nif2.h_cap = 0;
        HIP_TRY(hipHostMalloc((void **)&g_nif2.h, host_words * 8));
        g_nif2.h_cap = host_words;
    }
    return GKR_OK;
}

constexpr u64 NIF2_ROOT = 37;     // a primitive root of F_p
constexpr u64 NIF2_PURPOSE = 9;   // SplitMix64 stream of the verifier's secret

// h = product of coprime prime powers among 3, 9, 5, 25, 7, 11, 13 (each a
// supported DFT length); w generates the order-h subgroup.
int nif2_plan(u32 h, PfaPlan &pl) {
    if (h < 3 || h % 2 == 0 || ((fp::P - 1) / 2) % h)
        return fail(GKR_ERR_INVALID, "h must be odd, at least 3, and divide (p - 1) / 2");
    memset(&pl, 0, sizeof pl);
    pl.h = h;
    u32 rest = h;
    for (u32 q : {3u, 5u, 7u, 11u, 13u}) {
        u32 f = 1;
        while (rest % q == 0) {
            rest /= q;
            f *= q;
        }
        if (f > 1) pl.F[pl.nf++] = f;
    }
    if (rest != 1)
        return fail(GKR_ERR_INVALID, "h's prime factors must be among 3, 5, 7, 11, 13 (3 and 5 at most squared)");
    const u64 w = fp::pow(NIF2_ROOT, (fp::P - 1) / h);
    u32 stride = 1;
    for (u32 i = 0; i < pl.nf; i++) {
        const u32 F = pl.F[i], g = h / F;
        pl.stride[i] = stride;
        stride *= F;
        pl.gstep[i] = g;
        u32 gi = 1;
        while ((u64)g * gi % F != 1) gi++;
        pl.ginv[i] = gi;
        pl.cstep[i] = (u32)((u64)g * gi % h);  // 1 mod F, 0 mod the other factors
        pl.wfwd[i] = fp::pow(w, g);
        pl.winv[i] = fp::inv(pl.wfwd[i]);
    }
    return GKR_OK;
}

// Host inputs below p (checked here) copied to dst, or device inputs
// range-checked into *flag.
int nif2_inputs(const uint64_t *a, u64 n, int on_device, u64 *dst, u32 *flag, hipStream_t st,
                const u64 **src) {
    HIP_TRY(hipMemsetAsync(flag, 0, 4, st));
    if (on_device) {
        LAUNCH(PC_NIF2, n * 8.0, launch_nif2_range(st, a, n, flag));
        *src = a;
        return GKR_OK;
    }
    for (u64 i = 0; i < n; i++)
        if (a[i] >= fp::P) return fail(GKR_ERR_RANGE, "input value not below p");
    HIP_TRY(hipMemcpyAsync(dst, a, n * 8, hipMemcpyHostToDevice, st));
    *src = dst;
    return GKR_OK;
}

}  // namespace

extern "C" int nif2_prove(const uint64_t *a, uint64_t n, uint32_t h, int on_device, uint64_t *msgs,
                          void *hip_stream) {
    if (!a || !msgs || n == 0) return fail(GKR_ERR_INVALID, "NULL argument or n = 0");
    PfaPlan pl;
    int rc = nif2_plan(h, pl);
    if (rc) return rc;
    hipStream_t st = pick_stream(hip_stream);
    if (!st) return fail(GKR_ERR_DEVICE, "no stream");
    const u64 v = (n + h - 1) / h;
    std::lock_guard<std::mutex> lk(g_nif2.mu);
    struct {
        u64 *W, *tw, *in, *msgs, *part;
        u32 *flag;
    } b;
    auto lay = [&](Arena &ar) {
        b.W = ar.take<u64>((u64)h * v);
        b.part = ar.take<u64>(2ull * h * nif2_colsum_split(h, v));
        b.tw = ar.take<u64>(h);
        b.in = ar.take<u64>(on_device ? 1 : n);
        b.msgs = ar.take<u64>(2ull * h);
        b.flag = ar.take<u32>(1);
    };
    Arena sz;
    lay(sz);
    rc = nif2_reserve(sz.used, 2ull * h + 1);
    if (rc) return rc;
    Arena ar;
    ar.base = (char *)g_nif2.mem;
    lay(ar);
    const u64 *src = nullptr;
    rc = nif2_inputs(a, n, on_device, b.in, b.flag, st, &src);
    if (rc) return rc;
    const u64 xi = fp::pow(NIF2_ROOT, (fp::P - 1) / (2ull * h));
    LAUNCH(PC_NIF2, h * 8.0, launch_nif2_twist(st, h, xi, b.tw));
    LAUNCH(PC_NIF2, (double)h * v * 8 * 2 * 2 * pl.nf, launch_nif2_transform(st, pl, src, n, v, b.tw, b.W));
    LAUNCH(PC_NIF2, (double)h * v * 16, launch_nif2_colsum(st, pl, src, n, v, b.W, b.part, b.msgs));
    HIP_TRY(hipMemcpyAsync(g_nif2.h, b.msgs, 2ull * h * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(g_nif2.h + 2ull * h, b.flag, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (*(const u32 *)(g_nif2.h + 2ull * h)) return fail(GKR_ERR_RANGE, "input value not below p");
    memcpy(msgs, g_nif2.h, 2ull * h * 8);
    return GKR_OK;
}

extern "C" int nif2_verify(const uint64_t *a, uint64_t n, uint32_t h, int on_device, uint64_t seed,
                           const uint64_t *msgs, uint64_t n_msgs, int *accepted, uint64_t *f2,
                           void *hip_stream) {
    if (!a || !accepted || n == 0) return fail(GKR_ERR_INVALID, "NULL argument or n = 0");
    PfaPlan pl;
    int rc = nif2_plan(h, pl);
    if (rc) return rc;
    *accepted = 0;
    if (f2) *f2 = 0;
    if (n_msgs != 2ull * h || !msgs) return GKR_OK;
    for (u64 k = 0; k < n_msgs; k++)
        if (msgs[k] >= fp::P) return GKR_OK;
    hipStream_t st = pick_stream(hip_stream);
    if (!st) return fail(GKR_ERR_DEVICE, "no stream");
    const u64 v = (n + h - 1) / h;
    const u32 nch = (h + 31) / 32;
    std::lock_guard<std::mutex> lk(g_nif2.mu);
    struct {
        u64 *L, *L2, *part, *blk, *out, *in, *msgs;
        u32 *flag;
    } b;
    auto lay = [&](Arena &ar) {
        b.L = ar.take<u64>(h);
        b.L2 = ar.take<u64>(2ull * h);
        b.part = ar.take<u64>((u64)nch * v);
        b.blk = ar.take<u64>(1024);
        b.out = ar.take<u64>(2);
        b.in = ar.take<u64>(on_device ? 1 : n);
        b.msgs = ar.take<u64>(2ull * h);
        b.flag = ar.take<u32>(1);
    };
    Arena sz;
    lay(sz);
    rc = nif2_reserve(sz.used, 2ull * h + 3);
    if (rc) return rc;
    Arena ar;
    ar.base = (char *)g_nif2.mem;
    lay(ar);
    const u64 *src = nullptr;
    rc = nif2_inputs(a, n, on_device, b.in, b.flag, st, &src);
    if (rc) return rc;
    // the secret point, drawn before the stream is read
    u64 rs = fp::sm_state(seed, NIF2_PURPOSE);
    const u64 r = fp::sm_field(rs);
    const u64 w = fp::pow(NIF2_ROOT, (fp::P - 1) / h), xi = fp::pow(NIF2_ROOT, (fp::P - 1) / (2ull * h));
    memcpy(g_nif2.h, msgs, 2ull * h * 8);
    HIP_TRY(hipMemcpyAsync(b.msgs, g_nif2.h, 2ull * h * 8, hipMemcpyHostToDevice, st));
    LAUNCH(PC_NIF2, h * 8.0, launch_nif2_basis(st, w, h, r, b.L));
    LAUNCH(PC_NIF2, n * 8.0 + (double)nch * v * 16, launch_nif2_rows(st, src, n, v, h, b.L, b.part, b.blk, b.out));
    LAUNCH(PC_NIF2, 2.0 * h * 8, launch_nif2_basis(st, xi, 2ull * h, r, b.L2));
    LAUNCH(PC_NIF2, 2.0 * h * 16, launch_nif2_dot(st, b.msgs, b.L2, 2ull * h, b.blk, b.out + 1));
    HIP_TRY(hipMemcpyAsync(g_nif2.h, b.out, 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(g_nif2.h + 2, b.flag, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (*(const u32 *)(g_nif2.h + 2)) return fail(GKR_ERR_RANGE, "input value not below p");
    *accepted = g_nif2.h[0] == g_nif2.h[1];
    if (f2) {
        u64 s = 0;
        for (u64 j = 0; j < h; j++) s = fp::add(s, msgs[2 * j]);
        *f2 = s;
    }
    return GKR_OK;
}

// pyfpt_host.hip -- host runtime behind the C ABI of include/pyfpt.h.
//
// Per call: validate, turn each instance into binary32 step constants and
// integer bin thresholds (Sec. 2.1 bins (e_j, e_{j+1}] of N = k dN become
// K_j < k <= K_{j+1}), order the shared work queue longest-expected-run first,
// upload, launch queue reset -> persistent step kernel -> merge -> finalize
// on the caller's stream (optionally as a replayed hipGraph), and copy the
// per-instance results out.  Launch shape (workgroup size, workgroups per CU,
// queue claim chunk) comes from the options or from a measured autotuner
// cached per device and workload signature.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pyfpt.h"
#include "fpt_kernels.h"
#include "fpt_train.h"

using namespace fpt;

namespace {

// Message of the calling thread's last failed call (a fixed buffer: reporting an error never
// allocates).
thread_local char g_err[512];

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int dev_fail(hipError_t e, const char *what) {
    return fail(PYFPT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                       \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return dev_fail(e_, what); \
    } while (0)

constexpr uint64_t kDefaultKmax = 1ull << 20;
constexpr int kDefaultNsub = 16;
constexpr size_t kAlign = 256;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct LaunchCfg {
    int block = 0, wg_per_cu = 0, chunk = 0;
};

struct Device {
    int id = -1;
    int cus = 0;
    size_t max_lds = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t pinned_done = nullptr;
    hipEvent_t arena_done = nullptr;    // after an upload read from the host arena
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    unsigned char *scratch = nullptr;   // this device's copy of the static scratch array
    // graph cache
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<unsigned char> gkey;
    std::map<std::string, LaunchCfg> tuned;
};

constexpr int kMaxDevices = 64;

std::mutex g_mu;
Device g_dev[kMaxDevices];

int get_device(Device **out) {
    int id = 0;
    HIP_TRY(hipGetDevice(&id), "hipGetDevice");
    if (id < 0 || id >= kMaxDevices) return fail(PYFPT_EDEVICE, "device %d beyond the %d devices supported", id, kMaxDevices);
    Device &d = g_dev[id];
    if (d.id < 0) {
        d.id = id;
        hipDeviceProp_t p;
        HIP_TRY(hipGetDeviceProperties(&p, id), "hipGetDeviceProperties");
        d.cus = p.multiProcessorCount;
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, id) != hipSuccess) lds = 65536;
        d.max_lds = static_cast<size_t>(lds);
        HIP_TRY(hipEventCreateWithFlags(&d.pinned_done, hipEventDisableTiming), "hipEventCreate");
        HIP_TRY(hipEventCreateWithFlags(&d.arena_done, hipEventDisableTiming), "hipEventCreate");
        for (auto &e : d.ev) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
    }
    *out = &d;
    return PYFPT_OK;
}

bool finite(double x) { return std::isfinite(x); }

// ----------------------------------------------------------------------------
// host arena: while the allocation-free entry point runs (under g_mu, flag set on its thread),
// the call's bookkeeping (prepared instances, thresholds, queue order, upload image) is carved
// from this static block instead of the heap; elsewhere the containers use the heap as usual.
// ----------------------------------------------------------------------------
constexpr size_t kArenaBytes = 8u << 20;
alignas(256) unsigned char g_arena[kArenaBytes];
size_t g_arena_top = 0;
thread_local bool g_in_arena = false;
hipEvent_t g_arena_upload = nullptr;    // recorded after the last upload that read the arena

bool in_arena(const void *p) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    return c >= g_arena && c < g_arena + kArenaBytes;
}

void *arena_take(size_t bytes) {
    const size_t at = align_up(g_arena_top, 64);
    if (bytes > kArenaBytes - at) return nullptr;
    g_arena_top = at + bytes;
    return g_arena + at;
}

struct ArenaFull {};

template <class T>
struct ArenaAlloc {
    using value_type = T;
    ArenaAlloc() = default;
    template <class U>
    ArenaAlloc(const ArenaAlloc<U> &) {}
    T *allocate(size_t n) {
        if (g_in_arena) {
            void *p = n <= kArenaBytes / sizeof(T) ? arena_take(n * sizeof(T)) : nullptr;
            if (!p) throw ArenaFull{};
            return static_cast<T *>(p);
        }
        return static_cast<T *>(::operator new(n * sizeof(T)));
    }
    void deallocate(T *p, size_t) {
        if (!in_arena(p)) ::operator delete(p);
    }
    template <class U>
    bool operator==(const ArenaAlloc<U> &) const { return true; }
    template <class U>
    bool operator!=(const ArenaAlloc<U> &) const { return false; }
};

template <class T>
using Vec = std::vector<T, ArenaAlloc<T>>;

// Stable descending order of (key, index) pairs by key, in place (insertion sort: batches hold
// at most 1024 instances, and it needs no temporary buffer).
void sort_longest_first(Vec<std::pair<double, int>> &v) {
    for (size_t i = 1; i < v.size(); ++i) {
        const std::pair<double, int> x = v[i];
        size_t j = i;
        while (j > 0 && v[j - 1].first < x.first) {
            v[j] = v[j - 1];
            --j;
        }
        v[j] = x;
    }
}

// ----------------------------------------------------------------------------
// validation and preparation
// ----------------------------------------------------------------------------
struct Prepared {
    Vec<InstDev> inst;
    Vec<uint32_t> order;
    Vec<uint64_t> vbeg_sorted;
    Vec<uint32_t> thr;
    Vec<double> edges;
    Vec<MergeInst> mi;
    Vec<ResultLayout> rl;
    TableLayout lay{};
    const uint16_t *mlp_params = nullptr;
    int mlp_every = 1;
    uint64_t v_total = 0;
    uint64_t counts_total = 0, values_total = 0;
    int pot = 0, bias = 0;
    uint32_t n_sub = 0;
};

int check_f32(double x, const char *name, int i) {
    const float f = static_cast<float>(x);
    if (std::isnan(x) || (std::isinf(f) && !std::isinf(x)))
        return fail(PYFPT_EINVAL, "instance %d: %s = %g not representable in binary32", i, name, x);
    return PYFPT_OK;
}

int validate(const pyfpt_instance &I, int i) {
    const pyfpt_potential &P = I.pot;
    if (!finite(I.phi_in) || !finite(I.phi_end) || !finite(I.dN))
        return fail(PYFPT_EINVAL, "instance %d: phi_in, phi_end and dN must be finite", i);
    if (!(I.phi_in > I.phi_end)) return fail(PYFPT_EINVAL, "instance %d: need phi_in > phi_end", i);
    if (std::isnan(I.phi_uv) || (std::isinf(I.phi_uv) && I.phi_uv < 0))
        return fail(PYFPT_EINVAL, "instance %d: phi_uv must be a number or +inf", i);
    if (I.phi_uv < I.phi_in) return fail(PYFPT_EINVAL, "instance %d: need phi_uv >= phi_in", i);
    if (!(I.dN > 0)) return fail(PYFPT_EINVAL, "instance %d: need dN > 0", i);
    if (std::isnan(I.phi_esc) || I.phi_esc < 0) return fail(PYFPT_EINVAL, "instance %d: bad phi_esc", i);
    if (I.phi_esc != 0 && !(I.phi_esc > I.phi_in)) return fail(PYFPT_EINVAL, "instance %d: need phi_esc > phi_in", i);
    if (I.k_max >= (1ull << 32)) return fail(PYFPT_EINVAL, "instance %d: k_max must be < 2^32", i);
    if (I.n_traj > UINT64_MAX - I.t_first)
        return fail(PYFPT_EINVAL, "instance %d: t_first + n_traj exceeds 2^64 - 1", i);
    switch (P.kind) {
    case PYFPT_POT_QUADRATIC:
    case PYFPT_POT_QUADRATIC_BUMP:
        if (!finite(P.m) || !(P.m > 0)) return fail(PYFPT_EINVAL, "instance %d: need finite m > 0", i);
        if (!(I.phi_end > 0)) return fail(PYFPT_EINVAL, "instance %d: quadratic potentials need phi_end > 0", i);
        if (P.kind == PYFPT_POT_QUADRATIC_BUMP) {
            if (!finite(P.a) || !finite(P.phi0) || !finite(P.w) || !(P.w > 0) || !(P.a > -1))
                return fail(PYFPT_EINVAL, "instance %d: bump needs finite a > -1, phi0, w > 0", i);
        }
        break;
    case PYFPT_POT_FLAT:
        if (!finite(P.V0) || !(P.V0 > 0)) return fail(PYFPT_EINVAL, "instance %d: need finite V0 > 0", i);
        break;
    default:
        return fail(PYFPT_EINVAL, "instance %d: unknown potential kind %d", i, P.kind);
    }
    const pyfpt_bias &B = I.bias;
    switch (B.kind) {
    case PYFPT_BIAS_NONE: break;
    case PYFPT_BIAS_NOISE_SCALED:
        if (!finite(B.A)) return fail(PYFPT_EINVAL, "instance %d: bias amplitude must be finite", i);
        break;
    case PYFPT_BIAS_POWER:
        if (!finite(B.A) || B.p < 0 || B.p > 16) return fail(PYFPT_EINVAL, "instance %d: power bias needs finite A and 0 <= p <= 16", i);
        break;
    case PYFPT_BIAS_MLP: {
        const pyfpt_mlp &M = B.mlp;
        if (!M.params) return fail(PYFPT_EINVAL, "instance %d: learned bias needs device parameters", i);
        if (M.hidden != 64) return fail(PYFPT_EINVAL, "instance %d: learned bias supports hidden = 64 only", i);
        if (M.eval_every != 1 && M.eval_every != 4 && M.eval_every != 8 && M.eval_every != 16)
            return fail(PYFPT_EINVAL, "instance %d: eval_every must be 1, 4, 8 or 16", i);
        bool ok = std::isfinite(M.out_scale) && std::isfinite(B.target_N);
        for (int q = 0; q < 3; ++q) ok = ok && std::isfinite(M.in_mean[q]) && std::isfinite(M.in_inv_scale[q]);
        if (!ok) return fail(PYFPT_EINVAL, "instance %d: learned bias constants must be finite", i);
        break;
    }
    default:
        return fail(PYFPT_EINVAL, "instance %d: unknown bias kind %d", i, B.kind);
    }
    const pyfpt_bins &bn = I.bins;
    if (bn.n_bins < 1 || bn.n_bins > (1 << 20)) return fail(PYFPT_EINVAL, "instance %d: n_bins out of range", i);
    if (bn.n_sub == 1 || bn.n_sub < 0 || bn.n_sub > 64) return fail(PYFPT_EINVAL, "instance %d: n_sub must be 0 or 2..64", i);
    if (!bn.edges) return fail(PYFPT_EINVAL, "instance %d: edges is NULL", i);
    for (int j = 0; j <= bn.n_bins; ++j) {
        if (!finite(bn.edges[j])) return fail(PYFPT_EINVAL, "instance %d: edge %d not finite", i, j);
        if (j > 0 && !(bn.edges[j] > bn.edges[j - 1])) return fail(PYFPT_EINVAL, "instance %d: edges not strictly ascending at %d", i, j);
    }
    int rc;
    if ((rc = check_f32(I.phi_in, "phi_in", i)) || (rc = check_f32(I.phi_end, "phi_end", i)) ||
        (rc = check_f32(I.dN, "dN", i)))
        return rc;
    if (finite(I.phi_uv) && (rc = check_f32(2.0 * I.phi_uv, "2 phi_uv", i))) return rc;
    return PYFPT_OK;
}

uint32_t threshold(double e, double dN) {
    // K = max{k >= 0 : fl(k * dN) <= e}, clamped to [0, 2^32-1]
    if (e < 0) return 0;
    double q = std::floor(e / dN);
    if (q > 4294967294.0) return 0xFFFFFFFFu;
    int64_t K = static_cast<int64_t>(q);
    while (static_cast<double>(K + 1) * dN <= e) ++K;
    while (K > 0 && static_cast<double>(K) * dN > e) --K;
    if (K > 0xFFFFFFFFll) return 0xFFFFFFFFu;
    return static_cast<uint32_t>(K);
}

// Expected steps per run: orders the shared work queue (longest first, so that the launch drains
// on short runs) and centres the step-count sums.  For the quadratic potentials (the bump is a
// small perturbation of it) this is the noise-free run under the drift actually applied: with the
// noise-scaled bias B = A S = A c phi, c = m / (2 pi sqrt 6), the path d phi/dN = -2/phi + A c phi
// takes N = -ln[(2 - A c phi_in^2) / (2 - A c phi_end^2)] / (2 A c) to reach phi_end (the
// classical (phi_in^2 - phi_end^2)/4 at A = 0).  Where that drift does not point to the end
// (A c phi_in^2 >= 2), the noise has to carry each run against it, and the run is counted as
// k_max steps.  Other biases take the unbiased classical value; other potentials k_max.
double expected_steps(const pyfpt_instance &I, uint64_t k_max) {
    const double cap = static_cast<double>(k_max);
    if (I.cost_hint > 0) return std::min(I.cost_hint, cap);
    if (I.pot.kind != PYFPT_POT_QUADRATIC && I.pot.kind != PYFPT_POT_QUADRATIC_BUMP) return cap;
    const double a2 = I.phi_in * I.phi_in, e2 = I.phi_end * I.phi_end;
    double n = (a2 - e2) / 4.0;
    if (I.bias.kind == PYFPT_BIAS_NOISE_SCALED && I.bias.A != 0.0) {
        const double Ac = I.bias.A * I.pot.m / (2.0 * M_PI * std::sqrt(6.0));
        if (Ac * a2 >= 2.0) return cap;
        n = -std::log((2.0 - Ac * a2) / (2.0 - Ac * e2)) / (2.0 * Ac);
    }
    return std::min(n / I.dN, cap);
}

int prepare(const pyfpt_instance *ins, int n_inst, Prepared &P) {
    if (n_inst < 1 || n_inst > 1024) return fail(PYFPT_EINVAL, "n_inst must be 1..1024");
    for (int i = 0; i < n_inst; ++i) {
        int rc = validate(ins[i], i);
        if (rc) return rc;
    }
    P.pot = ins[0].pot.kind;
    P.bias = ins[0].bias.kind;
    // No bias is the noise-scaled bias with A = 0: the step then adds +0 to the drift and
    // +-0 to ln w, so a batch mixing the two runs as noise-scaled with identical results.
    for (int i = 1; i < n_inst; ++i) {
        const int b = ins[i].bias.kind;
        if (b != P.bias && ((b == PYFPT_BIAS_NONE && P.bias == PYFPT_BIAS_NOISE_SCALED) ||
                            (b == PYFPT_BIAS_NOISE_SCALED && P.bias == PYFPT_BIAS_NONE)))
            P.bias = PYFPT_BIAS_NOISE_SCALED;
    }
    const int ns0 = ins[0].bins.n_sub ? ins[0].bins.n_sub : kDefaultNsub;
    for (int i = 1; i < n_inst; ++i) {
        const int b = ins[i].bias.kind == PYFPT_BIAS_NONE && P.bias == PYFPT_BIAS_NOISE_SCALED
                          ? PYFPT_BIAS_NOISE_SCALED : ins[i].bias.kind;
        if (ins[i].pot.kind != P.pot || b != P.bias)
            return fail(PYFPT_EUNSUPPORTED, "all instances of a batch must share potential and bias kinds");
        if (b == PYFPT_BIAS_MLP && (ins[i].bias.mlp.params != ins[0].bias.mlp.params ||
                                    ins[i].bias.mlp.eval_every != ins[0].bias.mlp.eval_every))
            return fail(PYFPT_EUNSUPPORTED, "learned-bias instances of a batch must share the network and eval_every");
        const int ns = ins[i].bins.n_sub ? ins[i].bins.n_sub : kDefaultNsub;
        if (ns != ns0) return fail(PYFPT_EINVAL, "all instances of a batch must share n_sub");
    }
    P.n_sub = static_cast<uint32_t>(ns0);
    if (P.bias == PYFPT_BIAS_MLP) {
        P.mlp_params = static_cast<const uint16_t *>(ins[0].bias.mlp.params);
        P.mlp_every = ins[0].bias.mlp.eval_every;
    }
    P.inst.resize(n_inst);
    P.mi.resize(n_inst);
    P.rl.resize(n_inst);
    uint32_t rows = 0, thr_base = 0;
    size_t n_edges = 0;
    for (int i = 0; i < n_inst; ++i) n_edges += static_cast<size_t>(ins[i].bins.n_bins) + 1;
    P.thr.reserve(n_edges);
    P.edges.reserve(n_edges);
    P.order.reserve(n_inst);
    P.vbeg_sorted.reserve(n_inst);
    Vec<std::pair<double, int>> cost;
    cost.reserve(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const pyfpt_instance &I = ins[i];
        const uint64_t k_max = I.k_max ? I.k_max : kDefaultKmax;
        InstDev &D = P.inst[i];
        std::memset(&D, 0, sizeof D);
        StepConsts &C = D.c;
        C.dN = static_cast<float>(I.dN);
        C.sq = static_cast<float>(std::sqrt(I.dN));
        C.hdN = static_cast<float>(0.5 * I.dN);
        if (I.pot.kind == PYFPT_POT_FLAT)
            C.cm = static_cast<float>(std::sqrt(I.pot.V0 / 3.0) / (2.0 * M_PI));
        else
            C.cm = static_cast<float>(I.pot.m / (2.0 * M_PI * std::sqrt(6.0)));
        C.a = static_cast<float>(I.pot.a);
        C.phi0 = static_cast<float>(I.pot.phi0);
        C.inv_w2 = static_cast<float>(1.0 / (I.pot.w * I.pot.w));
        C.inv_2w2 = static_cast<float>(0.5 / (I.pot.w * I.pot.w));
        C.A = I.bias.kind == PYFPT_BIAS_NONE ? 0.0f : static_cast<float>(I.bias.A);
        if (I.bias.kind == PYFPT_BIAS_MLP) {
            for (int q = 0; q < 3; ++q) {
                D.mlp.in_mean[q] = I.bias.mlp.in_mean[q];
                D.mlp.in_inv[q] = I.bias.mlp.in_inv_scale[q];
            }
            D.mlp.out_scale = I.bias.mlp.out_scale;
            D.mlp.target_N = static_cast<float>(I.bias.target_N);
        }
        C.p = I.bias.p;
        C.phi_end = static_cast<float>(I.phi_end);
        C.phi_uv = static_cast<float>(I.phi_uv);
        C.two_uv = C.phi_uv + C.phi_uv;
        const bool wall = std::isfinite(I.phi_uv);
        C.phi_esc = wall ? INFINITY : static_cast<float>(I.phi_esc > 0 ? I.phi_esc : 100.0 * I.phi_in);
        C.phi_in = static_cast<float>(I.phi_in);
        C.k_max = static_cast<uint32_t>(k_max);
        D.stream = I.stream;
        D.n_bins = static_cast<uint32_t>(I.bins.n_bins);
        D.row_base = rows;
        D.thr_base = thr_base;
        D.dump_slot = static_cast<uint32_t>(i);
        D.k_center = static_cast<uint32_t>(std::min(expected_steps(I, k_max), 4294967295.0));
        D.n_traj = I.n_traj;
        D.t_first = I.t_first;
        for (int j = 0; j <= I.bins.n_bins; ++j) {
            P.thr.push_back(threshold(I.bins.edges[j], I.dN));
            P.edges.push_back(I.bins.edges[j]);
        }
        MergeInst &M = P.mi[i];
        M.row_base = rows;
        M.n_rows = D.n_bins + 4;
        M.n_bins = D.n_bins;
        M.edge_base = thr_base;
        M.n_traj = I.n_traj;
        M.t_first = I.t_first;
        P.rl[i] = result_layout(D.n_bins, P.n_sub);
        M.counts_off = P.counts_total;
        M.values_off = P.values_total;
        P.counts_total += P.rl[i].n_counts;
        P.values_total += P.rl[i].n_values;
        rows += D.n_bins + 4;
        thr_base += D.n_bins + 1;
        if (I.n_traj > 0) cost.push_back({expected_steps(I, k_max), i});
    }
    // longest expected runs first (ties: caller order)
    sort_longest_first(cost);
    uint64_t v = 0;
    for (auto &c : cost) {
        P.order.push_back(static_cast<uint32_t>(c.second));
        P.vbeg_sorted.push_back(v);
        P.inst[c.second].v_begin = v;
        v += ins[c.second].n_traj;
    }
    if (P.order.empty()) {
        P.order.push_back(0);
        P.vbeg_sorted.push_back(0);
    }
    P.v_total = v;
    // per-workgroup table layout
    TableLayout &L = P.lay;
    L.n_rows = rows;
    L.n_sub = P.n_sub;
    L.n_inst = static_cast<uint32_t>(n_inst);
    size_t off = 0;
    L.off_scal = 0;
    off = align_up(static_cast<size_t>(n_inst) * 128, 16);
    L.off_jk_lse = static_cast<uint32_t>(off);
    off += static_cast<size_t>(P.n_sub) * rows * 8;
    L.off_lse_w2 = static_cast<uint32_t>(off);
    off += static_cast<size_t>(rows) * 8;
    L.off_shift = static_cast<uint32_t>(off);
    off += static_cast<size_t>(rows) * 8;
    L.off_s1 = static_cast<uint32_t>(off);
    off += static_cast<size_t>(rows) * 8;
    L.off_s2 = static_cast<uint32_t>(off);
    off += static_cast<size_t>(rows) * 8;
    L.off_s3 = static_cast<uint32_t>(off);
    off += static_cast<size_t>(rows) * 8;
    L.off_s4 = static_cast<uint32_t>(off);
    off += static_cast<size_t>(rows) * 8;
    L.off_cnt = static_cast<uint32_t>(off);
    off += static_cast<size_t>(P.n_sub) * rows * 4;
    off = align_up(off, kAlign);
    if (off > 0x7FFFFFFFull) return fail(PYFPT_EINVAL, "per-workgroup table too large (%zu bytes)", off);
    L.slice_bytes = static_cast<uint32_t>(off);
    return PYFPT_OK;
}

// workspace map
struct WsMap {
    size_t queue, inst, order, vbeg, thr, edges, mi, counts, values, slices, total, upload_bytes;
};

WsMap ws_map(const Prepared &P, int n_wg) {
    WsMap m{};
    size_t o = 0;
    m.queue = o; o += kAlign;
    m.inst = o; o = align_up(o + P.inst.size() * sizeof(InstDev), kAlign);
    m.order = o; o = align_up(o + P.order.size() * 4, kAlign);
    m.vbeg = o; o = align_up(o + P.vbeg_sorted.size() * 8, kAlign);
    m.thr = o; o = align_up(o + P.thr.size() * 4, kAlign);
    m.edges = o; o = align_up(o + P.edges.size() * 8, kAlign);
    m.mi = o; o = align_up(o + P.mi.size() * sizeof(MergeInst), kAlign);
    m.upload_bytes = o - m.inst;
    m.counts = o; o = align_up(o + P.counts_total * 8, kAlign);
    m.values = o; o = align_up(o + P.values_total * 8, kAlign);
    m.slices = o; o += static_cast<size_t>(n_wg) * P.lay.slice_bytes;
    m.total = align_up(o, kAlign);
    return m;
}

void resolve_cfg(const Device &d, const Prepared &P, LaunchCfg &c, bool &lds) {
    const bool mlp = P.bias == PYFPT_BIAS_MLP;
    if (c.block <= 0) c.block = mlp ? 256 : 512;
    // the learned bias with one active instance fits three waves per SIMD (three 256-thread
    // workgroups per CU); otherwise one
    const bool mlp1 = mlp && P.order.size() == 1;
    if (c.wg_per_cu <= 0) c.wg_per_cu = mlp ? (mlp1 ? 3 : 1) : 2;
    if (c.chunk <= 0) c.chunk = 1;
    // LDS budget per workgroup: the CU's LDS shared by its resident workgroups, less the
    // single-instance learned sampler's static copy of the network's operand tiles
    const size_t share = std::min<size_t>(d.max_lds, 160 * 1024 / static_cast<size_t>(c.wg_per_cu));
    const size_t budget = share - (mlp1 ? std::min(share, fpt::MLP_TILE_LDS_BYTES) : 0);
    lds = P.lay.slice_bytes <= budget;
}

std::string signature(const Prepared &P, uint64_t seed_unused) {
    (void)seed_unused;
    char buf[256];
    snprintf(buf, sizeof buf, "p%d b%d i%zu r%u j%u v%llu", P.pot, P.bias, P.inst.size(), P.lay.n_rows, P.n_sub,
             static_cast<unsigned long long>(P.v_total));
    return buf;
}

struct RunCtx {
    Device *d;
    hipStream_t stream;
};

int run_prepared(Device &d, const Prepared &P, uint64_t seed, const LaunchCfg &cfg_in, const pyfpt_options *opt,
                 hipStream_t stream, void *ws, size_t ws_bytes, bool use_graph, float *timing,
                 bool noalloc = false) {
    LaunchCfg cfg = cfg_in;
    bool lds = false;
    resolve_cfg(d, P, cfg, lds);
    if (cfg.block < 64 || cfg.block > 1024 || cfg.block % 64)
        return fail(PYFPT_EINVAL, "block must be a multiple of 64 in 64..1024");
    if (P.bias == PYFPT_BIAS_MLP && cfg.block > 256)
        return fail(PYFPT_EINVAL, "the learned bias runs with block <= 256");
    if (cfg.wg_per_cu * cfg.block > 2048) return fail(PYFPT_EINVAL, "wg_per_cu * block must be <= 2048");
    const int n_wg = d.cus * cfg.wg_per_cu;
    const WsMap m = ws_map(P, n_wg);
    if (ws_bytes < m.total) return fail(PYFPT_ENOMEM, "workspace too small: need %zu bytes, have %zu", m.total, ws_bytes);
    unsigned char *W = static_cast<unsigned char *>(ws);

    // upload through the pinned staging buffer, or, without allocating, through an image in the
    // host arena (the caller has waited for the previous arena upload)
    unsigned char *H = nullptr;
    if (noalloc) {
        H = static_cast<unsigned char *>(arena_take(m.upload_bytes));
        if (!H) return fail(PYFPT_ENOMEM, "upload image of %zu bytes exceeds the host arena (%zu bytes)",
                            m.upload_bytes, kArenaBytes);
    } else if (d.pinned_bytes < m.upload_bytes) {
        if (d.pinned) {
            HIP_TRY(hipEventSynchronize(d.pinned_done), "hipEventSynchronize");
            (void)hipHostFree(d.pinned);
            d.pinned = nullptr;
        }
        HIP_TRY(hipHostMalloc(&d.pinned, m.upload_bytes, hipHostMallocDefault), "hipHostMalloc");
        d.pinned_bytes = m.upload_bytes;
    } else {
        HIP_TRY(hipEventSynchronize(d.pinned_done), "hipEventSynchronize");
    }
    if (!noalloc) H = static_cast<unsigned char *>(d.pinned);
    std::memset(H, 0, m.upload_bytes);
    std::memcpy(H + (m.inst - m.inst), P.inst.data(), P.inst.size() * sizeof(InstDev));
    std::memcpy(H + (m.order - m.inst), P.order.data(), P.order.size() * 4);
    std::memcpy(H + (m.vbeg - m.inst), P.vbeg_sorted.data(), P.vbeg_sorted.size() * 8);
    std::memcpy(H + (m.thr - m.inst), P.thr.data(), P.thr.size() * 4);
    std::memcpy(H + (m.edges - m.inst), P.edges.data(), P.edges.size() * 8);
    std::memcpy(H + (m.mi - m.inst), P.mi.data(), P.mi.size() * sizeof(MergeInst));
    HIP_TRY(hipMemcpyAsync(W + m.inst, H, m.upload_bytes, hipMemcpyHostToDevice, stream), "upload");
    if (noalloc) {
        HIP_TRY(hipEventRecord(d.arena_done, stream), "hipEventRecord");
        g_arena_upload = d.arena_done;
    } else {
        HIP_TRY(hipEventRecord(d.pinned_done, stream), "hipEventRecord");
    }

    StepArgs sa{};
    sa.inst = reinterpret_cast<const InstDev *>(W + m.inst);
    sa.order = reinterpret_cast<const uint32_t *>(W + m.order);
    sa.vbeg_sorted = reinterpret_cast<const uint64_t *>(W + m.vbeg);
    sa.n_inst = static_cast<int32_t>(P.order.size());
    sa.thr = reinterpret_cast<const uint32_t *>(W + m.thr);
    sa.queue = reinterpret_cast<unsigned long long *>(W + m.queue);
    sa.v_total = P.v_total;
    sa.key0 = static_cast<uint32_t>(seed);
    sa.key1 = static_cast<uint32_t>(seed >> 32);
    sa.slices = W + m.slices;
    sa.lay = P.lay;
    sa.chunk = static_cast<uint32_t>(cfg.chunk);
    sa.mlp_params = P.mlp_params;
    sa.mlp_every = P.mlp_every;
    if (opt && opt->dump.n) {
        if (!opt->dump.k || !opt->dump.lw || !opt->dump.phi || !opt->dump.status || opt->dump.stride == 0)
            return fail(PYFPT_EINVAL, "dump: all four arrays and stride >= 1 are required");
        sa.dump.n = opt->dump.n;
        sa.dump.stride = opt->dump.stride;
        sa.dump.k = opt->dump.k;
        sa.dump.lw = opt->dump.lw;
        sa.dump.phi = opt->dump.phi;
        sa.dump.status = opt->dump.status;
    }
    MergeArgs ma{};
    ma.slices = W + m.slices;
    ma.n_wg = n_wg;
    ma.lay = P.lay;
    ma.mi = reinterpret_cast<const MergeInst *>(W + m.mi);
    ma.n_inst = static_cast<int32_t>(P.mi.size());
    ma.edges = reinterpret_cast<const double *>(W + m.edges);
    ma.counts = reinterpret_cast<uint64_t *>(W + m.counts);
    ma.values = reinterpret_cast<double *>(W + m.values);
    const size_t lds_bytes = lds ? P.lay.slice_bytes : 0;

    auto enqueue = [&](bool timed) -> int {
        HIP_TRY(launch_init_queue(sa.queue, stream), "launch init");
        if (timed) HIP_TRY(hipEventRecord(d.ev[0], stream), "event");
        HIP_TRY(launch_step(P.pot, P.bias, lds, n_wg, cfg.block, lds_bytes, sa, stream), "launch step kernel");
        if (timed) HIP_TRY(hipEventRecord(d.ev[1], stream), "event");
        HIP_TRY(launch_merge(ma, static_cast<int>(P.lay.n_rows), static_cast<int>(P.n_sub), stream), "launch merge");
        if (timed) HIP_TRY(hipEventRecord(d.ev[2], stream), "event");
        return PYFPT_OK;
    };

    if (use_graph && !timing) {
        // key: everything the recorded launches depend on
        std::vector<unsigned char> key;
        auto put = [&](const void *p, size_t n) {
            const unsigned char *c = static_cast<const unsigned char *>(p);
            key.insert(key.end(), c, c + n);
        };
        put(&sa, sizeof sa);
        put(&ma, sizeof ma);
        put(&cfg, sizeof cfg);
        put(&lds, sizeof lds);
        int pb[2] = {P.pot, P.bias};
        put(pb, sizeof pb);
        put(&stream, sizeof stream);
        if (!d.gexec || key != d.gkey) {
            if (d.gexec) { (void)hipGraphExecDestroy(d.gexec); d.gexec = nullptr; }
            if (d.graph) { (void)hipGraphDestroy(d.graph); d.graph = nullptr; }
            HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            int rc = enqueue(false);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(stream, &g);
            if (rc) return rc;
            if (e != hipSuccess) return dev_fail(e, "hipStreamEndCapture");
            d.graph = g;
            HIP_TRY(hipGraphInstantiate(&d.gexec, d.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
            d.gkey = key;
        }
        HIP_TRY(hipGraphLaunch(d.gexec, stream), "hipGraphLaunch");
    } else {
        int rc = enqueue(timing != nullptr);
        if (rc) return rc;
    }
    if (timing) {
        HIP_TRY(hipEventSynchronize(d.ev[2]), "hipEventSynchronize");
        HIP_TRY(hipEventElapsedTime(&timing[0], d.ev[0], d.ev[1]), "hipEventElapsedTime");
        HIP_TRY(hipEventElapsedTime(&timing[1], d.ev[1], d.ev[2]), "hipEventElapsedTime");
    }
    return PYFPT_OK;
}

int copy_out(const Prepared &P, void *ws, int n_wg, pyfpt_result *out, hipStream_t stream) {
    const WsMap m = ws_map(P, n_wg);
    unsigned char *W = static_cast<unsigned char *>(ws);
    bool host = false;
    for (size_t i = 0; i < P.inst.size(); ++i) {
        if (!out[i].counts || !out[i].values) return fail(PYFPT_EINVAL, "result %zu: NULL buffer", i);
        const hipMemcpyKind kind = out[i].on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        host |= !out[i].on_device;
        HIP_TRY(hipMemcpyAsync(out[i].counts, W + m.counts + P.mi[i].counts_off * 8, P.rl[i].n_counts * 8, kind, stream),
                "copy counts");
        HIP_TRY(hipMemcpyAsync(out[i].values, W + m.values + P.mi[i].values_off * 8, P.rl[i].n_values * 8, kind, stream),
                "copy values");
    }
    if (host) HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    return PYFPT_OK;
}

int ensure_ws(Device &d, size_t bytes, void **ws) {
    if (d.ws_bytes < bytes) {
        if (d.ws) {
            HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
            (void)hipFree(d.ws);
            d.ws = nullptr;
            d.ws_bytes = 0;
            if (d.gexec) { (void)hipGraphExecDestroy(d.gexec); d.gexec = nullptr; }
            if (d.graph) { (void)hipGraphDestroy(d.graph); d.graph = nullptr; }
        }
        hipError_t e = hipMalloc(&d.ws, bytes);
        if (e != hipSuccess) return fail(PYFPT_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        d.ws_bytes = bytes;
    }
    *ws = d.ws;
    return PYFPT_OK;
}

// Measured autotuning of (block, wg_per_cu, chunk): short runs of the same
// instances with fewer trajectories, scored by trajectory-steps per second.
int autotune(Device &d, const pyfpt_instance *ins, int n_inst, uint64_t seed, hipStream_t stream,
             const Prepared &P, LaunchCfg &best) {
    const std::string key = signature(P, seed);
    auto it = d.tuned.find(key);
    if (it != d.tuned.end()) {
        best = it->second;
        return PYFPT_OK;
    }
    static const LaunchCfg cands[] = {
        {256, 4, 1}, {512, 2, 1}, {1024, 1, 1}, {256, 8, 1}, {512, 2, 4},
    };
    // about one trajectory per lane of the largest grid, split over instances by their share
    const double lanes = static_cast<double>(d.cus) * 2048.0;
    const double total = static_cast<double>(P.v_total);
    std::vector<pyfpt_instance> cal(ins, ins + n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const double share = total > 0 ? static_cast<double>(ins[i].n_traj) / total : 0.0;
        cal[i].n_traj = std::min<uint64_t>(ins[i].n_traj, static_cast<uint64_t>(std::ceil(lanes * share)));
    }
    Prepared C;
    int rc = prepare(cal.data(), n_inst, C);
    if (rc) return rc;
    double best_rate = -1;
    best = LaunchCfg{512, 2, 1};
    std::vector<uint64_t> counts(C.counts_total);
    for (const LaunchCfg &c : cands) {
        if (P.bias == PYFPT_BIAS_MLP && c.block > 256) continue;
        LaunchCfg cc = c;
        bool lds = false;
        resolve_cfg(d, C, cc, lds);
        const int n_wg = d.cus * cc.wg_per_cu;
        const WsMap m = ws_map(C, n_wg);
        void *ws = nullptr;
        if ((rc = ensure_ws(d, m.total, &ws))) return rc;
        float tm[2] = {0, 0};
        if ((rc = run_prepared(d, C, seed ^ 0x5DEECE66Dull, cc, nullptr, stream, ws, d.ws_bytes, false, tm))) return rc;
        HIP_TRY(hipMemcpyAsync(counts.data(), static_cast<unsigned char *>(ws) + m.counts, C.counts_total * 8,
                               hipMemcpyDeviceToHost, stream), "tune copy");
        HIP_TRY(hipStreamSynchronize(stream), "tune sync");
        double steps = 0;
        for (size_t i = 0; i < C.inst.size(); ++i) steps += static_cast<double>(counts[C.mi[i].counts_off + C.rl[i].total_steps]);
        const double rate = steps / std::max(1e-6, static_cast<double>(tm[0]));
        if (rate > best_rate) {
            best_rate = rate;
            best = c;
        }
    }
    d.tuned[key] = best;
    return PYFPT_OK;
}

int run_batch_impl(const pyfpt_instance *ins, int n_inst, uint64_t seed, pyfpt_result *out, const pyfpt_options *opt) {
    if (!ins || !out) return fail(PYFPT_EINVAL, "NULL instance or result array");
    Prepared P;
    int rc = prepare(ins, n_inst, P);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    Device *d = nullptr;
    if ((rc = get_device(&d))) return rc;
    if (d->cus <= 0) return fail(PYFPT_EDEVICE, "no compute units reported");
    hipStream_t stream = opt ? static_cast<hipStream_t>(opt->stream) : nullptr;
    LaunchCfg cfg;
    if (opt) {
        cfg.block = opt->block;
        cfg.wg_per_cu = opt->wg_per_cu;
        cfg.chunk = opt->chunk;
    }
    if ((cfg.block <= 0 || cfg.wg_per_cu <= 0 || cfg.chunk <= 0) && P.v_total > 0) {
        LaunchCfg t;
        if ((rc = autotune(*d, ins, n_inst, seed, stream, P, t))) return rc;
        if (cfg.block <= 0) cfg.block = t.block;
        if (cfg.wg_per_cu <= 0) cfg.wg_per_cu = t.wg_per_cu;
        if (cfg.chunk <= 0) cfg.chunk = t.chunk;
    }
    LaunchCfg rcfg = cfg;
    bool lds;
    resolve_cfg(*d, P, rcfg, lds);
    const int n_wg = d->cus * rcfg.wg_per_cu;
    const WsMap m = ws_map(P, n_wg);
    void *ws = nullptr;
    size_t ws_bytes = 0;
    if (opt && opt->workspace) {
        ws = opt->workspace;
        ws_bytes = opt->workspace_bytes;
    } else {
        if ((rc = ensure_ws(*d, m.total, &ws))) return rc;
        ws_bytes = d->ws_bytes;
    }
    const bool graph = opt && opt->use_graph;
    if (graph && stream == nullptr) return fail(PYFPT_EINVAL, "use_graph needs a non-null stream (the null stream cannot be captured)");
    if ((rc = run_prepared(*d, P, seed, rcfg, opt, stream, ws, ws_bytes, graph, opt ? opt->timing_ms : nullptr))) return rc;
    return copy_out(P, ws, n_wg, out, stream);
}

// ----------------------------------------------------------------------------
// allocation-free variant of the batched run
// ----------------------------------------------------------------------------
// The device scratch of pyfpt_run_batch_noalloc: queue counter, instance records, thresholds,
// staging results and per-workgroup tables.  Every device the library runs on holds its own copy
// for the life of the process.  In host code this name is only a stand-in for the symbol; the
// device address comes from hipGetSymbolAddress, once per device (Device::scratch).
static __device__ __align__(256) unsigned char scratch[PYFPT_NOALLOC_SCRATCH_BYTES];

int noalloc_setup(Device &d) {
    if (d.scratch) return PYFPT_OK;
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) return fail(PYFPT_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    d.scratch = static_cast<unsigned char *>(p);
    return PYFPT_OK;
}

// Sets the calling thread's arena flag for the scope and starts the arena empty.
struct ArenaScope {
    ArenaScope() {
        g_arena_top = 0;
        g_in_arena = true;
    }
    ~ArenaScope() { g_in_arena = false; }
};

int run_batch_noalloc_impl(const pyfpt_instance *ins, int n_inst, uint64_t seed, pyfpt_result *out,
                           const pyfpt_options *opt) {
    if (!ins || !out) return fail(PYFPT_EINVAL, "NULL instance or result array");
    if (opt && opt->workspace)
        return fail(PYFPT_EINVAL, "pyfpt_run_batch_noalloc works in its static scratch: workspace must be NULL");
    if (opt && opt->use_graph)
        return fail(PYFPT_EINVAL, "pyfpt_run_batch_noalloc does not build graphs (instantiation allocates)");
    std::lock_guard<std::mutex> lock(g_mu);
    Device *d = nullptr;
    int rc;
    if ((rc = get_device(&d))) return rc;
    if (d->cus <= 0) return fail(PYFPT_EDEVICE, "no compute units reported");
    if ((rc = noalloc_setup(*d))) return rc;
    // the arena is reused: wait until the previous upload from it has been read
    if (g_arena_upload) HIP_TRY(hipEventSynchronize(g_arena_upload), "hipEventSynchronize");
    ArenaScope scope;
    try {
        Prepared P;
        if ((rc = prepare(ins, n_inst, P))) return rc;
        hipStream_t stream = opt ? static_cast<hipStream_t>(opt->stream) : nullptr;
        LaunchCfg cfg;
        if (opt) {
            cfg.block = opt->block;
            cfg.wg_per_cu = opt->wg_per_cu;
            cfg.chunk = opt->chunk;
        }
        bool lds;
        resolve_cfg(*d, P, cfg, lds);          // no autotuning: 0 fields take the defaults
        const int n_wg = d->cus * cfg.wg_per_cu;
        if (cfg.wg_per_cu < 1 || cfg.wg_per_cu > 64) return fail(PYFPT_EINVAL, "wg_per_cu must be 1..64");
        const WsMap m = ws_map(P, n_wg);
        if (m.total > PYFPT_NOALLOC_SCRATCH_BYTES)
            return fail(PYFPT_ENOMEM,
                        "pyfpt_run_batch_noalloc needs %zu bytes of scratch for %u table rows on %d workgroups; "
                        "its static scratch holds %zu (use fewer workgroups per CU, fewer bins or fewer instances)",
                        m.total, P.lay.n_rows, n_wg, static_cast<size_t>(PYFPT_NOALLOC_SCRATCH_BYTES));
        if ((rc = run_prepared(*d, P, seed, cfg, opt, stream, d->scratch, PYFPT_NOALLOC_SCRATCH_BYTES, false,
                               opt ? opt->timing_ms : nullptr, true)))
            return rc;
        return copy_out(P, d->scratch, n_wg, out, stream);
    } catch (const ArenaFull &) {
        return fail(PYFPT_ENOMEM, "the batch's bookkeeping exceeds the host arena (%zu bytes)", kArenaBytes);
    }
}

// ----------------------------------------------------------------------------
// training of the learned proposal
// ----------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t bytes) {
        if (p) {
            (void)hipFree(p);
            p = nullptr;
        }
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(PYFPT_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        }
        return PYFPT_OK;
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

int check_offsets(const uint64_t *off, int64_t n, uint64_t n_rec) {
    if (off[0] != 0) return fail(PYFPT_EINVAL, "rec_off[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
        if (off[i + 1] < off[i]) return fail(PYFPT_EINVAL, "rec_off not ascending at %lld", static_cast<long long>(i));
    if (n_rec != UINT64_MAX && off[n] != n_rec) return fail(PYFPT_EINVAL, "rec_off[n_paths] must equal n_rec");
    return PYFPT_OK;
}

MlpConsts mlp_consts(const pyfpt_mlp &m, double target_N) {
    MlpConsts c{};
    for (int q = 0; q < 3; ++q) {
        c.in_mean[q] = m.in_mean[q];
        c.in_inv[q] = m.in_inv_scale[q];
    }
    c.out_scale = m.out_scale;
    c.target_N = static_cast<float>(target_N);
    return c;
}

// Replay on the device: buffers already on the device; outputs per path on the device.
int records_device(const Prepared &P, uint64_t seed, int group, int stride, const uint64_t *d_t, uint32_t n_paths,
                   const uint64_t *d_off, TrainRec *d_rec, uint32_t *d_k, double *d_lw, int32_t *d_st,
                   uint64_t *d_nrec, hipStream_t stream) {
    RecordArgs ra{};
    ra.inst = P.inst[0];
    ra.t_ids = d_t;
    ra.n_paths = n_paths;
    ra.key0 = static_cast<uint32_t>(seed);
    ra.key1 = static_cast<uint32_t>(seed >> 32);
    ra.group = group;
    ra.stride = stride;
    ra.mlp_every = P.mlp_every;
    ra.mlp_params = P.mlp_params;
    ra.rec_off = d_off;
    ra.rec = d_rec;
    ra.k_out = d_k;
    ra.lw_out = d_lw;
    ra.st_out = d_st;
    ra.n_rec_out = d_nrec;
    HIP_TRY(launch_records(P.pot, P.bias, ra, stream), "launch record kernel");
    return PYFPT_OK;
}

int backward_groups(uint64_t n_rec) {
    int cus = 0;
    {
        Device *d = nullptr;
        std::lock_guard<std::mutex> lock(g_mu);
        if (get_device(&d) == PYFPT_OK) cus = d->cus;
    }
    const uint64_t tiles = (n_rec + 63) / 64;
    const uint64_t cap = static_cast<uint64_t>(cus > 0 ? cus : 1) * 4;   // four backward workgroups per CU
    return static_cast<int>(std::max<uint64_t>(1, std::min(tiles, cap)));
}

}  // namespace

extern "C" {

int pyfpt_bin_thresholds(const double *edges, int32_t n_edges, double dN, uint32_t *out) {
    if (!edges || !out || n_edges < 1) return fail(PYFPT_EINVAL, "NULL argument or n_edges < 1");
    if (!(dN > 0) || !std::isfinite(dN)) return fail(PYFPT_EINVAL, "need finite dN > 0");
    for (int32_t j = 0; j < n_edges; ++j) out[j] = threshold(edges[j], dN);
    return PYFPT_OK;
}

int pyfpt_result_layout(int32_t n_bins, int32_t n_sub, pyfpt_layout *out) {
    if (!out) return fail(PYFPT_EINVAL, "NULL layout");
    if (n_bins < 1) return fail(PYFPT_EINVAL, "n_bins must be >= 1");
    if (n_sub == 0) n_sub = kDefaultNsub;
    if (n_sub < 2 || n_sub > 64) return fail(PYFPT_EINVAL, "n_sub must be 0 or 2..64");
    const ResultLayout L = result_layout(static_cast<uint32_t>(n_bins), static_cast<uint32_t>(n_sub));
    out->n_counts = L.n_counts;
    out->n_values = L.n_values;
    out->count = L.count;
    out->jk_count = L.jk_count;
    out->n_traj = L.n_traj;
    out->total_steps = L.total_steps;
    out->lse_w = L.lse_w;
    out->lse_w2 = L.lse_w2;
    out->jk_lse_w = L.jk_lse_w;
    out->mean_lnw = L.mean_lnw;
    out->m2_lnw = L.m2_lnw;
    out->m3_lnw = L.m3_lnw;
    out->m4_lnw = L.m4_lnw;
    out->log_p = L.log_p;
    out->rel_err_jk = L.rel_err_jk;
    out->rel_err_kish = L.rel_err_kish;
    out->log_p_ln = L.log_p_ln;
    out->rel_err_ln_lo = L.rel_err_ln_lo;
    out->rel_err_ln_hi = L.rel_err_ln_hi;
    out->normal_p = L.normal_p;
    out->lse_w_all = L.lse_w_all;
    out->lse_w2_all = L.lse_w2_all;
    out->lse_wk = L.lse_wk;
    out->lse_wk2 = L.lse_wk2;
    out->sum_k2 = L.sum_k2;
    out->pearson_r = L.pearson_r;
    out->ess = L.ess;
    out->lognormal_gate = L.lognormal_gate;
    return PYFPT_OK;
}

int pyfpt_run_batch(const pyfpt_instance *inst, int32_t n_inst, uint64_t seed, pyfpt_result *out,
                    const pyfpt_options *opt) {
    try {
        return run_batch_impl(inst, n_inst, seed, out, opt);
    } catch (...) {
        return fail(PYFPT_ENOMEM, "host exception (allocation failure)");
    }
}

int pyfpt_run_batch_noalloc(const pyfpt_instance *inst, int32_t n_inst, uint64_t seed, pyfpt_result *out,
                            const pyfpt_options *opt) {
    try {
        return run_batch_noalloc_impl(inst, n_inst, seed, out, opt);
    } catch (...) {
        return fail(PYFPT_ENOMEM, "host exception");
    }
}

int pyfpt_run(const pyfpt_potential *pot, double phi_in, double phi_end, double phi_uv, double dN,
              const pyfpt_bias *bias, uint64_t n_traj, uint64_t seed, const pyfpt_bins *bins, pyfpt_result *out,
              const pyfpt_options *opt) {
    if (!pot || !bias || !bins || !out) return fail(PYFPT_EINVAL, "NULL argument");
    pyfpt_instance I;
    std::memset(&I, 0, sizeof I);
    I.pot = *pot;
    I.bias = *bias;
    I.phi_in = phi_in;
    I.phi_end = phi_end;
    I.phi_uv = phi_uv;
    I.dN = dN;
    I.n_traj = n_traj;
    I.bins = *bins;
    if (opt) {
        I.k_max = opt->k_max;
        I.phi_esc = opt->phi_esc;
        I.stream = opt->stream_id;
        I.t_first = opt->t_first;
    }
    return pyfpt_run_batch(&I, 1, seed, out, opt);
}

int pyfpt_workspace_size(const pyfpt_instance *inst, int32_t n_inst, const pyfpt_options *opt, size_t *bytes) {
    if (!inst || !bytes) return fail(PYFPT_EINVAL, "NULL argument");
    try {
        Prepared P;
        int rc = prepare(inst, n_inst, P);
        if (rc) return rc;
        std::lock_guard<std::mutex> lock(g_mu);
        Device *d = nullptr;
        if ((rc = get_device(&d))) return rc;
        LaunchCfg c;
        if (opt) {
            c.block = opt->block;
            c.wg_per_cu = opt->wg_per_cu;
            c.chunk = opt->chunk;
        }
        if (c.wg_per_cu <= 0) c.wg_per_cu = 8;   // the largest grid the autotuner may pick
        bool lds;
        resolve_cfg(*d, P, c, lds);
        *bytes = ws_map(P, d->cus * c.wg_per_cu).total;
        return PYFPT_OK;
    } catch (...) {
        return fail(PYFPT_ENOMEM, "host exception (allocation failure)");
    }
}

int pyfpt_mlp_forward(const pyfpt_mlp *mlp, double target_N, const float *phi, const float *N, float *r,
                      uint64_t n, void *stream) {
    if (!mlp) return fail(PYFPT_EINVAL, "NULL network");
    if (n == 0) return PYFPT_OK;
    if (!mlp->params || !phi || !N || !r) return fail(PYFPT_EINVAL, "NULL pointer");
    if (mlp->hidden != 64) return fail(PYFPT_EINVAL, "hidden must be 64");
    MlpConsts c{};
    for (int q = 0; q < 3; ++q) {
        c.in_mean[q] = mlp->in_mean[q];
        c.in_inv[q] = mlp->in_inv_scale[q];
    }
    c.out_scale = mlp->out_scale;
    c.target_N = static_cast<float>(target_N);
    HIP_TRY(launch_mlp_forward(static_cast<const uint16_t *>(mlp->params), c, phi, N, r, n,
                               static_cast<hipStream_t>(stream)), "launch mlp forward");
    return PYFPT_OK;
}

static int pyfpt_combine_impl(const pyfpt_result *res, int32_t n_res, int32_t n_bins, int32_t n_sub, int32_t estimator,
                  double *log_p, double *err_log, int32_t *n_used) {
    if (!res || !log_p || !err_log || !n_used || n_res < 1) return fail(PYFPT_EINVAL, "NULL argument or n_res < 1");
    const bool strict = (estimator & PYFPT_COMBINE_NO_EXTRAPOLATION) != 0;
    const int32_t kind = estimator & ~PYFPT_COMBINE_NO_EXTRAPOLATION;
    if (kind < 0 || kind > 3)
        return fail(PYFPT_EINVAL, "estimator must be 0, 1, 2 or 3, optionally + PYFPT_COMBINE_NO_EXTRAPOLATION");
    if (n_bins < 1) return fail(PYFPT_EINVAL, "n_bins must be >= 1");
    if (n_sub == 0) n_sub = kDefaultNsub;
    if (n_sub < 2 || n_sub > 64) return fail(PYFPT_EINVAL, "n_sub must be 0 or 2..64");
    const ResultLayout L = result_layout(static_cast<uint32_t>(n_bins), static_cast<uint32_t>(n_sub));
    const uint32_t B = static_cast<uint32_t>(n_bins);
    // per (result, bin): the estimate y and its weight 1/e^2 (0 where not trusted)
    std::vector<double> ys(static_cast<size_t>(n_res) * B, 0.0), ws(static_cast<size_t>(n_res) * B, 0.0);
    std::fill(n_used, n_used + B, 0);
    std::vector<uint64_t> cbuf;
    std::vector<double> vbuf;
    for (int32_t i = 0; i < n_res; ++i) {
        if (!res[i].counts || !res[i].values) return fail(PYFPT_EINVAL, "result %d has NULL buffers", i);
        const uint64_t *C = static_cast<const uint64_t *>(res[i].counts);
        const double *V = static_cast<const double *>(res[i].values);
        if (res[i].on_device) {
            cbuf.resize(L.n_counts);
            vbuf.resize(L.n_values);
            HIP_TRY(hipMemcpy(cbuf.data(), C, 8 * L.n_counts, hipMemcpyDeviceToHost), "download counts");
            HIP_TRY(hipMemcpy(vbuf.data(), V, 8 * L.n_values, hipMemcpyDeviceToHost), "download values");
            C = cbuf.data();
            V = vbuf.data();
        }
        int est = kind;
        if (est == 2) est = V[L.lognormal_gate] == 1.0 ? 1 : 0;
        for (uint32_t j = 0; j < B; ++j) {
            const double n = static_cast<double>(C[L.count + j]);
            // naive estimate, trusted when n > 400 and n > exp(var ln w); lognormal estimate,
            // trusted when the bin passes the normality gate (and, with the no-extrapolation
            // rule, when n >= exp(s^2/2): the mean of w rests on ln w about s standard deviations
            // above its mean, which n draws reach only if s <= sqrt(2 ln n))
            const double p = V[L.normal_p + j];
            bool gate = n >= 8.0 && std::isfinite(p) && p >= 0.005;
            if (strict && gate) gate = n >= std::exp(0.5 * V[L.m2_lnw + j] * n / (n - 1.0));
            const bool naive_ok = n > 400.0 && n > std::exp(V[L.m2_lnw + j]);
            const bool use_ln = est == 1 || (est == 3 && gate);
            const double y = use_ln ? V[L.log_p_ln + j] : V[L.log_p + j];
            const double e = use_ln ? std::log1p(V[L.rel_err_ln_hi + j]) : V[L.rel_err_jk + j];
            const bool ok = est == 0 ? naive_ok : (est == 1 ? gate : gate || naive_ok);
            if (!ok || !std::isfinite(y) || !std::isfinite(e) || !(e > 0)) continue;
            ys[static_cast<size_t>(i) * B + j] = y;
            ws[static_cast<size_t>(i) * B + j] = 1.0 / (e * e);
            n_used[j] += 1;
        }
    }
    // inverse-variance mean; where the contributors scatter more than their errors allow
    // (chi^2 > n - 1), the error is scaled by Birge's ratio sqrt(chi^2 / (n - 1))
    for (uint32_t j = 0; j < B; ++j) {
        if (!n_used[j]) {
            log_p[j] = err_log[j] = NAN;
            continue;
        }
        double sw = 0.0, swy = 0.0;
        for (int32_t i = 0; i < n_res; ++i) {
            sw += ws[static_cast<size_t>(i) * B + j];
            swy += ws[static_cast<size_t>(i) * B + j] * ys[static_cast<size_t>(i) * B + j];
        }
        const double mean = swy / sw;
        double chi2 = 0.0;
        for (int32_t i = 0; i < n_res; ++i) {
            const double d = ys[static_cast<size_t>(i) * B + j] - mean;
            chi2 += ws[static_cast<size_t>(i) * B + j] * d * d;
        }
        const double birge = n_used[j] > 1 ? std::sqrt(std::max(1.0, chi2 / (n_used[j] - 1))) : 1.0;
        log_p[j] = mean;
        err_log[j] = birge / std::sqrt(sw);
    }
    return PYFPT_OK;
}

int pyfpt_combine(const pyfpt_result *res, int32_t n_res, int32_t n_bins, int32_t n_sub, int32_t estimator,
                  double *log_p, double *err_log, int32_t *n_used) {
    try {
        return pyfpt_combine_impl(res, n_res, n_bins, n_sub, estimator, log_p, err_log, n_used);
    } catch (...) {
        return fail(PYFPT_ENOMEM, "host exception (allocation failure)");
    }
}

static int pyfpt_proposal_records_impl(const pyfpt_instance *inst, uint64_t seed, const uint64_t *t_ids, int32_t n_paths,
                           int32_t group, int32_t stride, const uint64_t *rec_off, pyfpt_record *rec,
                           uint32_t *k_out, double *lw_out, int32_t *status_out, const pyfpt_options *opt) {
    if (!inst || n_paths < 0 || (n_paths > 0 && (!t_ids || !rec_off || !k_out || !lw_out || !status_out)))
        return fail(PYFPT_EINVAL, "NULL argument or n_paths < 0");
    if (group != 1 && group != 4 && group != 8 && group != 16) return fail(PYFPT_EINVAL, "group must be 1, 4, 8 or 16");
    if (stride < 1) return fail(PYFPT_EINVAL, "stride must be >= 1");
    if (n_paths >= (1 << 27)) return fail(PYFPT_EINVAL, "n_paths must be < 2^27");
    Prepared P;
    int rc = prepare(inst, 1, P);
    if (rc) return rc;
    if (n_paths == 0) return PYFPT_OK;
    if ((rc = check_offsets(rec_off, n_paths, UINT64_MAX))) return rc;
    const uint64_t n_rec = rec_off[n_paths];
    if (n_rec > 0 && !rec) return fail(PYFPT_EINVAL, "NULL record array");
    hipStream_t stream = opt ? static_cast<hipStream_t>(opt->stream) : nullptr;
    DevBuf t, off, r, k, lw, st, nr;
    if ((rc = t.alloc(8ull * n_paths)) || (rc = off.alloc(8ull * (n_paths + 1))) || (rc = r.alloc(16ull * n_rec)) ||
        (rc = k.alloc(4ull * n_paths)) || (rc = lw.alloc(8ull * n_paths)) || (rc = st.alloc(4ull * n_paths)) ||
        (rc = nr.alloc(8ull * n_paths)))
        return rc;
    HIP_TRY(hipMemcpyAsync(t.p, t_ids, 8ull * n_paths, hipMemcpyHostToDevice, stream), "upload ids");
    HIP_TRY(hipMemcpyAsync(off.p, rec_off, 8ull * (n_paths + 1), hipMemcpyHostToDevice, stream), "upload offsets");
    if ((rc = records_device(P, seed, group, stride, t.as<uint64_t>(), static_cast<uint32_t>(n_paths), off.as<uint64_t>(),
                             r.as<TrainRec>(), k.as<uint32_t>(), lw.as<double>(), st.as<int32_t>(), nr.as<uint64_t>(),
                             stream)))
        return rc;
    if (n_rec) HIP_TRY(hipMemcpyAsync(rec, r.p, 16ull * n_rec, hipMemcpyDeviceToHost, stream), "download records");
    HIP_TRY(hipMemcpyAsync(k_out, k.p, 4ull * n_paths, hipMemcpyDeviceToHost, stream), "download k");
    HIP_TRY(hipMemcpyAsync(lw_out, lw.p, 8ull * n_paths, hipMemcpyDeviceToHost, stream), "download lw");
    HIP_TRY(hipMemcpyAsync(status_out, st.p, 4ull * n_paths, hipMemcpyDeviceToHost, stream), "download status");
    HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    return PYFPT_OK;
}

int pyfpt_proposal_records(const pyfpt_instance *inst, uint64_t seed, const uint64_t *t_ids, int32_t n_paths,
                           int32_t group, int32_t stride, const uint64_t *rec_off, pyfpt_record *rec,
                           uint32_t *k_out, double *lw_out, int32_t *status_out, const pyfpt_options *opt) {
    try {
        return pyfpt_proposal_records_impl(inst, seed, t_ids, n_paths, group, stride, rec_off, rec, k_out, lw_out, status_out, opt);
    } catch (...) {
        return fail(PYFPT_ENOMEM, "host exception (allocation failure)");
    }
}

static int pyfpt_proposal_loss_grad_impl(const pyfpt_mlp *net, double target_N, double dN, const float *theta,
                             const pyfpt_record *rec, uint64_t n_rec, const uint64_t *rec_off, int32_t n_paths,
                             const double *lw0, double n_total, int32_t objective, double temper,
                             double rec_weight, double *loss, double *grad, double *lw_theta,
                             const pyfpt_options *opt) {
    if (!net || !theta || !rec_off || !lw0 || !loss || !grad || !lw_theta || (n_rec > 0 && !rec))
        return fail(PYFPT_EINVAL, "NULL argument");
    if (n_paths < 1 || n_paths >= (1 << 27)) return fail(PYFPT_EINVAL, "n_paths must be 1 .. 2^27-1");
    if (objective != 0 && objective != 1) return fail(PYFPT_EINVAL, "objective must be 0 or 1");
    if (!(temper > 0.0 && temper <= 1.0)) return fail(PYFPT_EINVAL, "temper must be in (0, 1]");
    if (!(rec_weight >= 1.0) || !std::isfinite(rec_weight) || (objective == 0 && rec_weight != 1.0))
        return fail(PYFPT_EINVAL, "rec_weight must be >= 1 (and 1 for objective 0)");
    if (!(dN > 0) || !std::isfinite(dN) || !(n_total > 0) || !std::isfinite(target_N))
        return fail(PYFPT_EINVAL, "need finite dN > 0, n_total > 0 and finite target_N");
    int rc = check_offsets(rec_off, n_paths, n_rec);
    if (rc) return rc;
    for (uint64_t e = 0; e < n_rec; ++e) {
        const uint32_t pn = rec[e].path_n;
        if ((pn >> 5) >= static_cast<uint32_t>(n_paths) || (pn & 31u) < 1 || (pn & 31u) > 16)
            return fail(PYFPT_EINVAL, "record %llu: path index or step count out of range",
                        static_cast<unsigned long long>(e));
    }
    hipStream_t stream = opt ? static_cast<hipStream_t>(opt->stream) : nullptr;
    const int n_part = backward_groups(n_rec);
    DevBuf r, off, th, lwt, l0, c, ls, part, g;
    if ((rc = r.alloc(16ull * n_rec)) || (rc = off.alloc(8ull * (n_paths + 1))) || (rc = th.alloc(4ull * NET_N_PARAMS)) ||
        (rc = lwt.alloc(8ull * n_paths)) || (rc = l0.alloc(8ull * n_paths)) ||
        (rc = c.alloc(8ull * n_paths)) || (rc = ls.alloc(8)) ||
        (rc = part.alloc(4ull * NET_N_PARAMS * static_cast<uint64_t>(n_part))) || (rc = g.alloc(8ull * NET_N_PARAMS)))
        return rc;
    if (n_rec) HIP_TRY(hipMemcpyAsync(r.p, rec, 16ull * n_rec, hipMemcpyHostToDevice, stream), "upload records");
    HIP_TRY(hipMemcpyAsync(off.p, rec_off, 8ull * (n_paths + 1), hipMemcpyHostToDevice, stream), "upload offsets");
    HIP_TRY(hipMemcpyAsync(th.p, theta, 4ull * NET_N_PARAMS, hipMemcpyHostToDevice, stream), "upload theta");
    HIP_TRY(hipMemcpyAsync(l0.p, lw0, 8ull * n_paths, hipMemcpyHostToDevice, stream), "upload lw0");
    TrainArgs ta{};
    ta.rec = r.as<TrainRec>();
    ta.n_rec = n_rec;
    ta.rec_off = off.as<uint64_t>();
    ta.n_paths = n_paths;
    ta.n_part = n_part;
    ta.objective = objective;
    ta.temper = static_cast<float>(temper);
    ta.rec_weight = static_cast<float>(rec_weight);
    ta.theta = th.as<float>();
    ta.mc = mlp_consts(*net, target_N);
    ta.dN = static_cast<float>(dN);
    ta.lw_theta = lwt.as<double>();
    ta.lw0 = l0.as<double>();
    ta.n_total = n_total;
    ta.c = c.as<double>();
    ta.loss = ls.as<double>();
    ta.part = part.as<float>();
    ta.grad = g.as<double>();
    HIP_TRY(launch_train_loss(ta, stream), "launch loss kernels");
    HIP_TRY(launch_train_grad(ta, stream), "launch gradient kernels");
    HIP_TRY(hipMemcpyAsync(loss, ls.p, 8, hipMemcpyDeviceToHost, stream), "download loss");
    HIP_TRY(hipMemcpyAsync(grad, g.p, 8ull * NET_N_PARAMS, hipMemcpyDeviceToHost, stream), "download grad");
    HIP_TRY(hipMemcpyAsync(lw_theta, lwt.p, 8ull * n_paths, hipMemcpyDeviceToHost, stream), "download lw_theta");
    HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    return PYFPT_OK;
}

int pyfpt_proposal_loss_grad(const pyfpt_mlp *net, double target_N, double dN, const float *theta,
                             const pyfpt_record *rec, uint64_t n_rec, const uint64_t *rec_off, int32_t n_paths,
                             const double *lw0, double n_total, int32_t objective, double temper,
                             double rec_weight, double *loss, double *grad, double *lw_theta,
                             const pyfpt_options *opt) {
    try {
        return pyfpt_proposal_loss_grad_impl(net, target_N, dN, theta, rec, n_rec, rec_off, n_paths, lw0, n_total, objective, temper, rec_weight, loss,
                                           grad, lw_theta, opt);
    } catch (...) {
        return fail(PYFPT_ENOMEM, "host exception (allocation failure)");
    }
}

static int pyfpt_train_proposal_impl(const pyfpt_instance *inst, uint64_t seed, const pyfpt_train_config *cfg, float *theta,
                         uint16_t *params_bf16, pyfpt_train_report *report, const pyfpt_options *opt) {
    if (!inst || !cfg || !theta || !params_bf16 || !report) return fail(PYFPT_EINVAL, "NULL argument");
    if (inst->bias.kind != PYFPT_BIAS_MLP) return fail(PYFPT_EINVAL, "the instance's bias must be the learned bias");
    if (cfg->group != 1 && cfg->group != 4 && cfg->group != 8 && cfg->group != 16)
        return fail(PYFPT_EINVAL, "group must be 1, 4, 8 or 16");
    if (cfg->rounds < 1 || cfg->steps < 1 || cfg->n_sample < 1 || cfg->max_paths < 0 || cfg->max_paths >= (1 << 27))
        return fail(PYFPT_EINVAL, "need rounds >= 1, steps >= 1, n_sample >= 1, 0 <= max_paths < 2^27");
    if (!(cfg->window_hi > cfg->window_lo) || !std::isfinite(cfg->window_lo) || !std::isfinite(cfg->window_hi))
        return fail(PYFPT_EINVAL, "need a finite window lo < hi");
    if (!(cfg->lr > 0) || !(cfg->beta1 >= 0 && cfg->beta1 < 1) || !(cfg->beta2 >= 0 && cfg->beta2 < 1) || !(cfg->eps > 0))
        return fail(PYFPT_EINVAL, "bad Adam constants");
    if (cfg->objective != 0 && cfg->objective != 1) return fail(PYFPT_EINVAL, "objective must be 0 or 1");
    if (!(cfg->temper > 0.0f && cfg->temper <= 1.0f)) return fail(PYFPT_EINVAL, "temper must be in (0, 1]");
    if (cfg->stride < 1 || (cfg->objective == 0 && cfg->stride != 1))
        return fail(PYFPT_EINVAL, "stride must be >= 1 (and 1 for objective 0)");
    if (cfg->n_sample >= (1ull << 32)) return fail(PYFPT_EINVAL, "n_sample must be < 2^32");
    if (cfg->select < 0) return fail(PYFPT_EINVAL, "select must be 0 or a pilot size");
    for (int j = 0; j < NET_N_PARAMS; ++j)
        if (!std::isfinite(theta[j])) return fail(PYFPT_EINVAL, "theta[%d] is not finite", j);
    hipStream_t stream = opt ? static_cast<hipStream_t>(opt->stream) : nullptr;
    int rc;
    // device copies of the network: master, Adam moments, bfloat16 copy for sampling
    DevBuf th, am, av, bf, g;
    if ((rc = th.alloc(4ull * NET_N_PARAMS)) || (rc = am.alloc(4ull * NET_N_PARAMS)) || (rc = av.alloc(4ull * NET_N_PARAMS)) ||
        (rc = bf.alloc(2ull * NET_N_PARAMS)) || (rc = g.alloc(8ull * NET_N_PARAMS)))
        return rc;
    HIP_TRY(hipMemcpyAsync(th.p, theta, 4ull * NET_N_PARAMS, hipMemcpyHostToDevice, stream), "upload theta");
    HIP_TRY(hipMemsetAsync(am.p, 0, 4ull * NET_N_PARAMS, stream), "clear Adam m");
    HIP_TRY(hipMemsetAsync(av.p, 0, 4ull * NET_N_PARAMS, stream), "clear Adam v");
    HIP_TRY(launch_to_bf16(th.as<float>(), bf.as<uint16_t>(), stream), "launch bf16 copy");
    // sampling instance: the current network, n_sample runs
    pyfpt_instance I = *inst;
    I.bias.mlp.params = bf.p;
    I.n_traj = cfg->n_sample;
    I.t_first = 0;                 // each round draws runs 0 .. n_sample - 1 (the dump index is the id)
    const uint64_t ns = cfg->n_sample;
    const uint64_t n_pilot = cfg->select > 0 ? static_cast<uint64_t>(cfg->select) : 0;
    const uint64_t nbuf = std::max(ns, n_pilot);
    DevBuf dk, dlw, dphi, dst;
    if ((rc = dk.alloc(4 * nbuf)) || (rc = dlw.alloc(8 * nbuf)) || (rc = dphi.alloc(4 * nbuf)) || (rc = dst.alloc(4 * nbuf)))
        return rc;
    pyfpt_layout lay{};
    if ((rc = pyfpt_result_layout(I.bins.n_bins, I.bins.n_sub ? I.bins.n_sub : kDefaultNsub, &lay))) return rc;
    std::vector<uint64_t> counts(lay.n_counts);
    std::vector<double> values(lay.n_values);
    std::vector<uint32_t> hk(nbuf);
    std::vector<double> hlw(nbuf);
    std::vector<int32_t> hst(nbuf);
    hipEvent_t ev[4] = {};
    struct EvFree {
        hipEvent_t *e;
        ~EvFree() {
            for (int i = 0; i < 4; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } evfree{ev};
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
    int64_t t_adam = 0;
    // one sampling pass of the current network, every run dumped and downloaded
    auto sample = [&](uint64_t seed_r, uint64_t n, float *ms) -> int {
        I.n_traj = n;
        pyfpt_options so{};
        so.stream = stream;
        so.block = opt && opt->block ? opt->block : 256;
        so.wg_per_cu = opt && opt->wg_per_cu ? opt->wg_per_cu : 2;
        so.chunk = opt && opt->chunk ? opt->chunk : 1;
        so.dump.n = n;
        so.dump.stride = 1;
        so.dump.k = dk.as<uint32_t>();
        so.dump.lw = dlw.as<double>();
        so.dump.phi = dphi.as<float>();
        so.dump.status = dst.as<int32_t>();
        pyfpt_result res{counts.data(), values.data(), 0};
        HIP_TRY(hipEventRecord(ev[0], stream), "event");
        const int r = run_batch_impl(&I, 1, seed_r, &res, &so);
        if (r) return r;
        HIP_TRY(hipEventRecord(ev[1], stream), "event");
        HIP_TRY(hipMemcpyAsync(hk.data(), dk.p, 4 * n, hipMemcpyDeviceToHost, stream), "download k");
        HIP_TRY(hipMemcpyAsync(hlw.data(), dlw.p, 8 * n, hipMemcpyDeviceToHost, stream), "download lw");
        HIP_TRY(hipMemcpyAsync(hst.data(), dst.p, 4 * n, hipMemcpyDeviceToHost, stream), "download status");
        HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
        HIP_TRY(hipEventElapsedTime(ms, ev[0], ev[1]), "hipEventElapsedTime");
        I.n_traj = ns;
        return PYFPT_OK;
    };
    auto in_window = [&](uint64_t t) {
        const double N = static_cast<double>(hk[t]) * I.dN;
        return hst[t] == PYFPT_ST_ENDED && N > cfg->window_lo && N <= cfg->window_hi;
    };
    // Kish ESS (sum w)^2 / sum w^2 over the window runs of the first n dumped runs
    auto window_kish = [&](uint64_t n) -> double {
        double mx = -INFINITY;
        for (uint64_t t = 0; t < n; ++t)
            if (in_window(t)) mx = std::max(mx, hlw[t]);
        if (!(mx > -INFINITY)) return 0.0;
        double s1 = 0.0, s2 = 0.0;
        for (uint64_t t = 0; t < n; ++t)
            if (in_window(t)) {
                const double e = std::exp(hlw[t] - mx);
                s1 += e;
                s2 += e * e;
            }
        return s1 * s1 / s2;
    };
    // select mode: host copies of the starting network and of each round's end network
    std::vector<std::vector<float>> cand;
    if (n_pilot) cand.push_back(std::vector<float>(theta, theta + NET_N_PARAMS));
    for (int round = 0; round < cfg->rounds; ++round) {
        pyfpt_train_report &R = report[round];
        std::memset(&R, 0, sizeof R);
        R.pilot_ess = NAN;
        const uint64_t seed_r = seed + static_cast<uint64_t>(round);
        // 1. sample from the current proposal, every run dumped
        if ((rc = sample(seed_r, ns, &R.ms_sample))) return rc;
        // 2. the runs that ended in the window (right-closed, as the bins)
        std::vector<uint64_t> ids;
        std::vector<double> lw0;
        double mx = -INFINITY;
        for (uint64_t t = 0; t < ns; ++t) {
            if (in_window(t)) {
                R.n_window += 1;
                // records carry the path index in 27 bits
                const bool room = cfg->max_paths == 0 ? ids.size() < (1u << 27) - 1u
                                                      : static_cast<int32_t>(ids.size()) < cfg->max_paths;
                if (room) {
                    ids.push_back(t);
                    lw0.push_back(hlw[t]);
                    mx = std::max(mx, hlw[t]);
                }
            }
        }
        R.n_used = static_cast<int32_t>(ids.size());
        if (ids.empty()) {
            R.loss_first = R.loss_last = -INFINITY;
            if (n_pilot) cand.push_back(cand.back());
            continue;
        }
        {
            double s1 = 0, s2 = 0;
            for (double x : lw0) {
                s1 += std::exp(x - mx);
                s2 += std::exp(2 * (x - mx));
            }
            R.kish_window = s1 * s1 / s2;
        }
        const uint32_t np = static_cast<uint32_t>(ids.size());
        std::vector<uint64_t> off(np + 1, 0);
        for (uint32_t i = 0; i < np; ++i) {
            const uint64_t groups = (hk[ids[i]] + cfg->group - 1) / cfg->group;
            off[i + 1] = off[i] + (groups + cfg->stride - 1) / cfg->stride;
        }
        const uint64_t n_rec = off[np];
        R.n_records = n_rec;
        // 3. replay into records under the proposal that drew the runs
        Prepared P;
        if ((rc = prepare(&I, 1, P))) return rc;
        DevBuf dt, doff, drec, rk, rlw, rst, rnr, lwt, l0, c, ls, part;
        const int n_part = backward_groups(n_rec);
        if ((rc = dt.alloc(8ull * np)) || (rc = doff.alloc(8ull * (np + 1))) || (rc = drec.alloc(16ull * n_rec)) ||
            (rc = rk.alloc(4ull * np)) || (rc = rlw.alloc(8ull * np)) || (rc = rst.alloc(4ull * np)) ||
            (rc = rnr.alloc(8ull * np)) || (rc = lwt.alloc(8ull * np)) ||
            (rc = l0.alloc(8ull * np)) || (rc = c.alloc(8ull * np)) || (rc = ls.alloc(8)) ||
            (rc = part.alloc(4ull * NET_N_PARAMS * static_cast<uint64_t>(n_part))))
            return rc;
        HIP_TRY(hipMemcpyAsync(dt.p, ids.data(), 8ull * np, hipMemcpyHostToDevice, stream), "upload ids");
        HIP_TRY(hipMemcpyAsync(doff.p, off.data(), 8ull * (np + 1), hipMemcpyHostToDevice, stream), "upload offsets");
        HIP_TRY(hipMemcpyAsync(l0.p, lw0.data(), 8ull * np, hipMemcpyHostToDevice, stream), "upload lw0");
        HIP_TRY(hipEventRecord(ev[1], stream), "event");
        if ((rc = records_device(P, seed_r, cfg->group, cfg->stride, dt.as<uint64_t>(), np, doff.as<uint64_t>(), drec.as<TrainRec>(),
                                 rk.as<uint32_t>(), rlw.as<double>(), rst.as<int32_t>(), rnr.as<uint64_t>(), stream)))
            return rc;
        HIP_TRY(hipEventRecord(ev[2], stream), "event");
        {
            std::vector<uint32_t> k2(np);
            std::vector<double> lw2(np);
            HIP_TRY(hipMemcpyAsync(k2.data(), rk.p, 4ull * np, hipMemcpyDeviceToHost, stream), "download k");
            HIP_TRY(hipMemcpyAsync(lw2.data(), rlw.p, 8ull * np, hipMemcpyDeviceToHost, stream), "download lw");
            HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
            for (uint32_t i = 0; i < np; ++i)
                if (k2[i] != hk[ids[i]] || lw2[i] != lw0[i])
                    return fail(PYFPT_EDEVICE, "replay of run %llu differs from the sampled run",
                                static_cast<unsigned long long>(ids[i]));
        }
        HIP_TRY(hipEventElapsedTime(&R.ms_records, ev[1], ev[2]), "hipEventElapsedTime");
        // 4. Adam steps on log M2
        TrainArgs ta{};
        ta.rec = drec.as<TrainRec>();
        ta.n_rec = n_rec;
        ta.rec_off = doff.as<uint64_t>();
        ta.n_paths = static_cast<int32_t>(np);
        ta.n_part = n_part;
        ta.objective = cfg->objective;
        ta.temper = cfg->temper;
        ta.rec_weight = static_cast<float>(cfg->stride);
        ta.theta = th.as<float>();
        ta.mc = P.inst[0].mlp;
        ta.dN = P.inst[0].c.dN;
        ta.lw_theta = lwt.as<double>();
        ta.lw0 = l0.as<double>();
        ta.n_total = static_cast<double>(ns);
        ta.c = c.as<double>();
        ta.loss = ls.as<double>();
        ta.part = part.as<float>();
        ta.grad = g.as<double>();
        HIP_TRY(hipEventRecord(ev[2], stream), "event");
        for (int step = 0; step < cfg->steps; ++step) {
            // the cross-entropy weights c_i depend on w_0 only: the forward pass (ln w_theta and
            // the weights) is needed once per round; log M2's weights change with theta
            if (step == 0 || cfg->objective == 0) HIP_TRY(launch_train_loss(ta, stream), "launch loss kernels");
            if (step == 0) HIP_TRY(hipMemcpyAsync(&R.loss_first, ls.p, 8, hipMemcpyDeviceToHost, stream), "download loss");
            HIP_TRY(launch_train_grad(ta, stream), "launch gradient kernels");
            t_adam += 1;
            AdamArgs aa{};
            aa.theta = th.as<float>();
            aa.m = am.as<float>();
            aa.v = av.as<float>();
            aa.grad = g.as<double>();
            aa.bf16 = bf.as<uint16_t>();
            aa.lr = cfg->lr;
            aa.beta1 = cfg->beta1;
            aa.beta2 = cfg->beta2;
            aa.eps = cfg->eps;
            aa.bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(cfg->beta1), static_cast<double>(t_adam)));
            aa.bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(cfg->beta2), static_cast<double>(t_adam)));
            HIP_TRY(launch_adam(aa, stream), "launch Adam");
        }
        // loss at the updated parameters
        HIP_TRY(launch_train_loss(ta, stream), "launch loss kernels");
        HIP_TRY(hipEventRecord(ev[3], stream), "event");
        HIP_TRY(hipMemcpyAsync(&R.loss_last, ls.p, 8, hipMemcpyDeviceToHost, stream), "download loss");
        HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
        HIP_TRY(hipEventElapsedTime(&R.ms_optimise, ev[2], ev[3]), "hipEventElapsedTime");
        if (n_pilot) {
            cand.emplace_back(NET_N_PARAMS);
            HIP_TRY(hipMemcpyAsync(cand.back().data(), th.p, 4ull * NET_N_PARAMS, hipMemcpyDeviceToHost, stream),
                    "copy theta");
            HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
        }
    }
    if (n_pilot) {
        // score every candidate on its own pilot of n_pilot runs (seeds apart from the training
        // rounds') by the Kish ESS of its window runs, and keep the best
        double best_ess = -1.0;
        size_t best = 0;
        for (size_t c = 0; c < cand.size(); ++c) {
            HIP_TRY(hipMemcpyAsync(th.p, cand[c].data(), 4ull * NET_N_PARAMS, hipMemcpyHostToDevice, stream), "upload theta");
            HIP_TRY(launch_to_bf16(th.as<float>(), bf.as<uint16_t>(), stream), "launch bf16 copy");
            float ms = 0.0f;
            if ((rc = sample(seed + (1ull << 30) + c, n_pilot, &ms))) return rc;
            const double e = window_kish(n_pilot);
            if (c > 0) report[c - 1].pilot_ess = e;
            if (e > best_ess) {
                best_ess = e;
                best = c;
            }
        }
        HIP_TRY(hipMemcpyAsync(th.p, cand[best].data(), 4ull * NET_N_PARAMS, hipMemcpyHostToDevice, stream), "upload theta");
        HIP_TRY(launch_to_bf16(th.as<float>(), bf.as<uint16_t>(), stream), "launch bf16 copy");
        if (best > 0) report[best - 1].selected = 1;
    }
    HIP_TRY(hipMemcpyAsync(theta, th.p, 4ull * NET_N_PARAMS, hipMemcpyDeviceToHost, stream), "download theta");
    HIP_TRY(hipMemcpyAsync(params_bf16, bf.p, 2ull * NET_N_PARAMS, hipMemcpyDeviceToHost, stream), "download params");
    HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    return PYFPT_OK;
}

int pyfpt_train_proposal(const pyfpt_instance *inst, uint64_t seed, const pyfpt_train_config *cfg, float *theta,
                         uint16_t *params_bf16, pyfpt_train_report *report, const pyfpt_options *opt) {
    try {
        return pyfpt_train_proposal_impl(inst, seed, cfg, theta, params_bf16, report, opt);
    } catch (...) {
        return fail(PYFPT_ENOMEM, "host exception (allocation failure)");
    }
}

int pyfpt_device_cus(int32_t *cus) {
    if (!cus) return fail(PYFPT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(g_mu);
    Device *d = nullptr;
    int rc = get_device(&d);
    if (rc) {
        *cus = 0;
        return rc;
    }
    *cus = d->cus;
    return PYFPT_OK;
}

const char *pyfpt_last_error(void) { return g_err; }

}  // extern "C"

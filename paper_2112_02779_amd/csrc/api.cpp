// Host runtime of librir: argument validation, sensor tables, batch plans
// (tile lists, workspaces, captured HIP graphs), the C ABI of include/rir.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <limits>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "elev_table.h"
#include "rir.h"
#include "rir_internal.h"
#include "rir_ops.h"
#include "sdf_extract.h"
#include "sdf_hash.h"

using namespace rir;

namespace {

thread_local std::string g_err;

// Identity of sensors and networks inside cached plans.  Ids are never reused,
// so a plan built for an object that has since been destroyed can never be
// matched by a new object that happens to get the same address.
std::atomic<uint64_t> g_next_uid{1};

rir_status fail(rir_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return fail(e_ == hipErrorOutOfMemory ? RIR_E_OOM : RIR_E_HIP,                          \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                         \
    } while (0)

constexpr double kTwoPi = 6.28318530717958647692528676655900577;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Byte layout of one device allocation holding several arrays.
struct Layout {
    size_t bytes = 0;
    size_t add(size_t n) {
        size_t off = align_up(bytes, 256);
        bytes = off + n;
        return off;
    }
};

}  // namespace

// ============================================================================ sensor

struct rir_sensor {
    uint64_t uid = g_next_uid.fetch_add(1);
    int device = 0;
    int H = 0, W = 0, nlev = 0;
    double r0 = 0.0;
    std::vector<double> phi, theta;
    void *dmem = nullptr;
    SensorTab<float> tf{};
    SensorTab<double> td{};
    const SensorTab<float> *d_tf = nullptr;
    const SensorTab<double> *d_td = nullptr;
    ~rir_sensor()
    {
        if (dmem) {
            hipSetDevice(device);
            hipFree(dmem);
        }
    }
};

namespace {

struct HostTables {
    std::vector<double> row, col, nrow, theta;
    std::vector<double> mu[kMaxLevels], uoff[kMaxLevels];
    double s_lo, s_hi, cos_h, sin_h, lo, hi;
    double kW[kMaxLevels];
    long nbins[kMaxLevels];
    std::vector<float> ebin_f[kMaxLevels];
    std::vector<double> ebin_d[kMaxLevels];
};

// FP64 construction of the tables of Sec. 3: the factors of Eq. (1), the
// product-form neighbour-difference factors, and per level the sin of the
// elevation midpoints between strided rows with the packed inverse table over
// sin(phi) (Sec. 3.2): 2 H_l bins at least, and at least two per smallest
// midpoint gap, doubled until no bin holds two distinct midpoints.
bool build_tables(const rir_sensor &s, int inv_bins, HostTables &t)
{
    const int H = s.H, W = s.W;
    t.row.resize(4 * H);
    for (int v = 0; v < H; ++v) {
        t.row[4 * v] = std::cos(s.phi[v]);
        t.row[4 * v + 1] = std::sin(s.phi[v]);
        t.row[4 * v + 2] = std::cos(s.theta[v]);
        t.row[4 * v + 3] = std::sin(s.theta[v]);
    }
    t.col.resize(2 * W);
    for (int u = 0; u < W; ++u) {
        const double a = kTwoPi * (double)u / (double)W;
        t.col[2 * u] = std::cos(a);
        t.col[2 * u + 1] = std::sin(a);
    }
    t.nrow.assign(8 * H, 0.0);
    for (int v = 1; v + 1 < H; ++v) {
        const double sg = 0.5 * (s.phi[v + 1] + s.phi[v - 1]), dp = 0.5 * (s.phi[v + 1] - s.phi[v - 1]);
        const double m = 0.5 * (s.theta[v + 1] + s.theta[v - 1]), dt = 0.5 * (s.theta[v + 1] - s.theta[v - 1]);
        double *f = &t.nrow[8 * v];
        f[0] = std::cos(m + sg);
        f[1] = std::sin(m + sg);
        f[2] = std::cos(m - sg);
        f[3] = std::sin(m - sg);
        f[4] = std::sin(dt + dp);
        f[5] = std::sin(dt - dp);
        f[6] = 2.0 * std::cos(sg) * std::sin(dp);
        f[7] = 0.0;
    }
    t.theta = s.theta;
    const double phi_hi = s.phi[0] + 0.5 * (s.phi[0] - s.phi[1]);
    const double phi_lo = s.phi[H - 1] - 0.5 * (s.phi[H - 2] - s.phi[H - 1]);
    t.s_hi = phi_hi >= 0.5 * M_PI ? INFINITY : std::sin(phi_hi);
    t.s_lo = phi_lo <= -0.5 * M_PI ? -INFINITY : std::sin(phi_lo);
    t.cos_h = std::cos(kTwoPi / W);
    t.sin_h = std::sin(kTwoPi / W);
    t.lo = std::isfinite(t.s_lo) ? t.s_lo : -1.0;
    t.hi = std::isfinite(t.s_hi) ? t.s_hi : 1.0;
    for (int l = 0; l < s.nlev; ++l) {
        const int st = 1 << l, Hl = H / st;
        t.kW[l] = (double)W / (kTwoPi * st);
        t.uoff[l].resize(Hl);
        for (int k = 0; k < Hl; ++k)
            t.uoff[l][k] = s.theta[st * k] * (double)W / (kTwoPi * st);
        t.mu[l].assign(std::max(Hl - 1, 0), 0.0);
        double gmin = t.hi - t.lo;
        for (int k = 0; k + 1 < Hl; ++k) {
            t.mu[l][k] = std::sin(0.5 * (s.phi[st * k] + s.phi[st * (k + 1)]));
            if (k > 0)
                gmin = std::min(gmin, t.mu[l][k - 1] - t.mu[l][k]);
        }
        long nb = std::max<long>(2L * Hl, std::max(inv_bins, 2));
        if (Hl > 2 && gmin > 0)
            nb = std::max<long>(nb, (long)std::ceil(2.0 * (t.hi - t.lo) / gmin) + 1);
        for (;; nb *= 2) {
            if (nb > (1L << 20))
                return false;
            if (build_ebin<float>(t.mu[l], t.uoff[l], nb, t.lo, t.hi, t.ebin_f[l]) &&
                build_ebin<double>(t.mu[l], t.uoff[l], nb, t.lo, t.hi, t.ebin_d[l]))
                break;
        }
        t.nbins[l] = nb;
    }
    return true;
}

template <typename T>
void fill_tab(SensorTab<T> &tab, const rir_sensor &s, const HostTables &t, char *base, const size_t *off_row,
              const size_t *off_col, const size_t *off_nrow, const size_t *off_theta, const size_t *off_ebin)
{
    tab.H = s.H;
    tab.W = s.W;
    tab.nlev = s.nlev;
    tab.r0 = (T)s.r0;
    tab.s_lo = std::isfinite(t.s_lo) ? (T)t.s_lo : -std::numeric_limits<T>::infinity();
    tab.s_hi = std::isfinite(t.s_hi) ? (T)t.s_hi : std::numeric_limits<T>::infinity();
    tab.cos_h = (T)t.cos_h;
    tab.sin_h = (T)t.sin_h;
    tab.row = reinterpret_cast<const T *>(base + *off_row);
    tab.col = reinterpret_cast<const T *>(base + *off_col);
    tab.nrow = reinterpret_cast<const T *>(base + *off_nrow);
    tab.theta = reinterpret_cast<const T *>(base + *off_theta);
    for (int l = 0; l < kMaxLevels; ++l) {
        if (l < s.nlev) {
            tab.nbins[l] = (int)t.nbins[l];
            tab.bin_lo[l] = (T)t.lo;
            tab.bin_scale[l] = (T)((double)t.nbins[l] / (t.hi - t.lo));
            tab.kW[l] = (T)t.kW[l];
            tab.ebin[l] = reinterpret_cast<const T *>(base + off_ebin[l]);
        } else {
            tab.nbins[l] = 0;
            tab.bin_lo[l] = tab.bin_scale[l] = tab.kW[l] = (T)0;
            tab.ebin[l] = nullptr;
        }
    }
}

template <typename T>
void put(std::vector<char> &img, size_t off, const std::vector<double> &v)
{
    T *p = reinterpret_cast<T *>(img.data() + off);
    for (size_t i = 0; i < v.size(); ++i)
        p[i] = (T)v[i];
}

}  // namespace

namespace {

// Validates a sensor description and copies it into s (no device work).
rir_status read_desc(const rir_sensor_desc *desc, rir_sensor &s, const char *who)
{
    const std::string w(who);
    const int H = desc->H, W = desc->W;
    if (H < 2 || W < 4)
        return fail(RIR_E_LUT, w + ": need H >= 2 and W >= 4");
    if (!desc->phi_lut)
        return fail(RIR_E_INVALID, w + ": phi_lut is null");
    if (!(desc->r0 >= 0.0) || !std::isfinite(desc->r0))
        return fail(RIR_E_LUT, w + ": r0 must be finite and >= 0");
    s.H = H;
    s.W = W;
    s.r0 = desc->r0;
    s.phi.assign(desc->phi_lut, desc->phi_lut + H);
    s.theta.assign(H, 0.0);
    if (desc->theta_lut)
        s.theta.assign(desc->theta_lut, desc->theta_lut + H);
    for (int v = 0; v < H; ++v) {
        if (!std::isfinite(s.phi[v]) || std::fabs(s.phi[v]) >= 0.5 * M_PI)
            return fail(RIR_E_LUT, w + ": phi_lut entries must be finite with |phi| < pi/2");
        if (v > 0 && !(s.phi[v] < s.phi[v - 1]))
            return fail(RIR_E_LUT, w + ": phi_lut must be strictly decreasing (row 0 = top beam)");
        if (!std::isfinite(s.theta[v]) || std::fabs(s.theta[v]) >= M_PI)
            return fail(RIR_E_LUT, w + ": theta_lut entries must be finite with |theta| < pi");
    }
    int nlev = 0;
    while (nlev < kMaxLevels && H % (1 << nlev) == 0 && W % (1 << nlev) == 0 && (W >> nlev) >= 2)
        ++nlev;
    s.nlev = nlev;
    return RIR_OK;
}

}  // namespace

extern "C" rir_status rir_elevation_table(const rir_sensor_desc *desc, int32_t level, int32_t precision,
                                          void *entries, int64_t capacity, int64_t *nbins, double *bin_lo,
                                          double *bin_scale)
{
    if (!desc || !nbins)
        return fail(RIR_E_INVALID, "rir_elevation_table: null argument");
    if (precision != RIR_PREC_FP32 && precision != RIR_PREC_FP64)
        return fail(RIR_E_INVALID, "rir_elevation_table: unknown precision");
    rir_sensor s;
    rir_status st = read_desc(desc, s, "rir_elevation_table");
    if (st != RIR_OK)
        return st;
    if (level < 0 || level >= s.nlev)
        return fail(RIR_E_INVALID, "rir_elevation_table: level outside the sensor's pyramid");
    HostTables t;
    if (!build_tables(s, std::max(desc->inv_bins, 0), t))
        return fail(RIR_E_LUT, "rir_elevation_table: elevation midpoints too close for the inverse table");
    const int64_t nb = t.nbins[level];
    *nbins = nb;
    if (bin_lo)
        *bin_lo = t.lo;
    if (bin_scale)
        *bin_scale = (double)nb / (t.hi - t.lo);
    if (!entries)
        return RIR_OK;
    if (capacity < 4 * nb)
        return fail(RIR_E_INVALID, "rir_elevation_table: capacity below 4 * nbins");
    if (precision == RIR_PREC_FP32)
        std::memcpy(entries, t.ebin_f[level].data(), 4 * sizeof(float) * nb);
    else
        std::memcpy(entries, t.ebin_d[level].data(), 4 * sizeof(double) * nb);
    return RIR_OK;
}

extern "C" rir_status rir_sensor_create(const rir_sensor_desc *desc, rir_sensor **out)
{
    if (!desc || !out)
        return fail(RIR_E_INVALID, "rir_sensor_create: null argument");
    *out = nullptr;
    std::unique_ptr<rir_sensor> s(new rir_sensor());
    rir_status st = read_desc(desc, *s, "rir_sensor_create");
    if (st != RIR_OK)
        return st;
    const int nlev = s->nlev;
    HIP_TRY(hipGetDevice(&s->device));
    HostTables t;
    if (!build_tables(*s, std::max(desc->inv_bins, 0), t))
        return fail(RIR_E_LUT, "rir_sensor_create: elevation midpoints too close for the inverse table");

    Layout lay;
    size_t od_row = lay.add(8 * t.row.size()), od_col = lay.add(8 * t.col.size());
    size_t od_nrow = lay.add(8 * t.nrow.size()), od_theta = lay.add(8 * t.theta.size());
    size_t of_row = lay.add(4 * t.row.size()), of_col = lay.add(4 * t.col.size());
    size_t of_nrow = lay.add(4 * t.nrow.size()), of_theta = lay.add(4 * t.theta.size());
    size_t od_ebin[kMaxLevels] = {}, of_ebin[kMaxLevels] = {};
    for (int l = 0; l < nlev; ++l) {
        od_ebin[l] = lay.add(8 * t.ebin_d[l].size());
        of_ebin[l] = lay.add(4 * t.ebin_f[l].size());
    }
    size_t o_tf = lay.add(sizeof(SensorTab<float>)), o_td = lay.add(sizeof(SensorTab<double>));
    std::vector<char> img(lay.bytes, 0);
    put<double>(img, od_row, t.row);
    put<double>(img, od_col, t.col);
    put<double>(img, od_nrow, t.nrow);
    put<double>(img, od_theta, t.theta);
    put<float>(img, of_row, t.row);
    put<float>(img, of_col, t.col);
    put<float>(img, of_nrow, t.nrow);
    put<float>(img, of_theta, t.theta);
    for (int l = 0; l < nlev; ++l) {
        std::memcpy(img.data() + od_ebin[l], t.ebin_d[l].data(), 8 * t.ebin_d[l].size());
        std::memcpy(img.data() + of_ebin[l], t.ebin_f[l].data(), 4 * t.ebin_f[l].size());
    }
    HIP_TRY(hipMalloc(&s->dmem, lay.bytes));
    char *base = static_cast<char *>(s->dmem);
    fill_tab(s->tf, *s, t, base, &of_row, &of_col, &of_nrow, &of_theta, of_ebin);
    fill_tab(s->td, *s, t, base, &od_row, &od_col, &od_nrow, &od_theta, od_ebin);
    std::memcpy(img.data() + o_tf, &s->tf, sizeof(s->tf));
    std::memcpy(img.data() + o_td, &s->td, sizeof(s->td));
    HIP_TRY(hipMemcpy(s->dmem, img.data(), lay.bytes, hipMemcpyHostToDevice));
    s->d_tf = reinterpret_cast<const SensorTab<float> *>(base + o_tf);
    s->d_td = reinterpret_cast<const SensorTab<double> *>(base + o_td);
    *out = s.release();
    return RIR_OK;
}

extern "C" void rir_sensor_destroy(rir_sensor *sensor) { delete sensor; }

// ============================================================================ learned-weight network

struct rir_mlp {
    uint64_t uid = g_next_uid.fetch_add(1);
    int device = 0;
    void *dmem = nullptr;
    uint16_t *w = nullptr;   // bf16 weights [kMlpNW]
    float *b = nullptr;      // biases [kMlpNB]
    float *master = nullptr; // FP32 master weights [kMlpNW]
    float *m1 = nullptr, *m2 = nullptr;  // Adam moments [5185]
    float *gpart = nullptr;  // per-block gradient records
    int gpart_blocks = 0;
    int step = 0;
    ~rir_mlp()
    {
        hipSetDevice(device);
        if (dmem)
            hipFree(dmem);
        if (gpart)
            hipFree(gpart);
    }
    MlpDev dev() const { return MlpDev{w, b}; }
};

// ============================================================================ context and plans

namespace {

struct KeyPod {
    int levels, iters[kMaxLevels], init_mode, weight_mode, learned_levels, precision, use_graph, debug, normal_window;
    double delta, edge_rel, max_corr, r_max, stop_eps;
    uint64_t mlp;
    rir_tuning tune;
};

struct PlanKey {
    std::vector<uint64_t> sensors;
    KeyPod k;
    bool operator<(const PlanKey &o) const
    {
        if (sensors != o.sensors)
            return sensors < o.sensors;
        return std::memcmp(&k, &o.k, sizeof(KeyPod)) < 0;
    }
};

struct Plan {
    PlanKey key;
    uint64_t last_use = 0;
    std::vector<int> shapes;  // H, W per pair (checked on every reuse)
    int device = 0;
    int n_pairs = 0;
    bool fp64 = false;
    int tile_seg[kMaxLevels] = {}, block = 0;
    bool lean[kMaxLevels] = {};  // the lean step variant applies (StepArgs::lean)
    bool resident[kMaxLevels] = {};  // some pair runs the level in the pair-resident kernel
    int n_tiles[kMaxLevels] = {};
    int grid[kMaxLevels] = {};
    // the coarse levels (and with lane_fine the finest) run as n_lanes
    // sub-batches of consecutive pairs
    // (lane k: pairs lane_p0[k] .. lane_p0[k + 1] - 1, tiles lane_t0[l][k] ..
    // lane_t0[l][k + 1] - 1 of level l), each on a stream of its own
    int n_lanes = 1;
    int lane_p0[kMaxLanes + 1] = {};
    int lane_t0[kMaxLevels][kMaxLanes + 1] = {};
    int lane_grid[kMaxLevels][kMaxLanes] = {};
    void *dmem = nullptr;
    void *h_desc = nullptr;   // pinned host copy of the pair descriptors
    size_t desc_bytes = 0;
    void *d_desc = nullptr;
    int2 *d_tiles[kMaxLevels] = {};
    // tile records; level l's start at record rec0[l] (levels never share
    // records: sub-batches may be at different levels at the same time)
    void *d_psum = nullptr;
    int4 *d_pcnt = nullptr;
    int rec0[kMaxLevels] = {};
    double *d_poses = nullptr;
    rir_level_stats *d_stats = nullptr;
    int *d_flags = nullptr;
    int *d_tickets = nullptr;  // [n_pairs], right after the flags
    bool nbf[kMaxLevels] = {};       // level keeps the learned weight's neighbour features
    size_t max_px[kMaxLevels] = {};  // largest level image of the batch
    std::vector<const float *> cur_src, cur_dst;
    hipEvent_t desc_evt = nullptr;
    bool desc_pending = false;
    // the whole schedule (prepass and every level) as one graph, without and
    // with the context's timing events as graph nodes
    hipGraphExec_t g_run[3] = {nullptr, nullptr, nullptr};  // by timing mode
    hipGraph_t g_src[3] = {nullptr, nullptr, nullptr};      // the graphs they were built from
    hipGraphNode_t fine_ev[2] = {nullptr, nullptr};         // event nodes of g_src[2]
    ~Plan()
    {
        hipSetDevice(device);
        for (auto &g : g_run)
            if (g)
                hipGraphExecDestroy(g);
        for (auto &g : g_src)
            if (g)
                hipGraphDestroy(g);
        if (desc_evt)
            hipEventDestroy(desc_evt);
        if (h_desc)
            hipHostFree(h_desc);
        if (dmem)
            hipFree(dmem);
    }
};

}  // namespace

struct rir_ctx {
    int device = 0;
    int n_cu = 256;
    hipStream_t cap = nullptr;  // private stream used only for graph capture
    // streams of the coarse-level sub-batches (default priority), forked from
    // and joined back into the caller's stream with the events below
    hipStream_t lane_st[kMaxLanes] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kMaxLanes] = {};
    rir_tuning tune{256, 8, 0, 1, 4, 1, 1, 0};
    std::map<PlanKey, std::unique_ptr<Plan>> plans;
    uint64_t use_clock = 0;
    int timing = 0;  // 0 off, 1 every level and the prepass, 2 the finest level only
    int timing_levels = 0, timed_mode = 0;  // of the last timed call
    // mode 2: one event pair per call, round robin over kRing pairs
    static constexpr int kRing = 64;
    hipEvent_t ring[kRing][2] = {};
    int ring_next = 0, ring_n = 0;
    hipEvent_t ev[2 * (kMaxLevels + 1)] = {};
    bool ev_recorded = false;
    ~rir_ctx()
    {
        hipSetDevice(device);
        plans.clear();
        for (auto &e : ev)
            if (e)
                hipEventDestroy(e);
        for (auto &pr : ring)
            for (auto &e : pr)
                if (e)
                    hipEventDestroy(e);
        if (cap)
            hipStreamDestroy(cap);
        for (auto &q : lane_st)
            if (q)
                hipStreamDestroy(q);
        for (auto &e : join_ev)
            if (e)
                hipEventDestroy(e);
        if (fork_ev)
            hipEventDestroy(fork_ev);
    }
};

extern "C" rir_status rir_ctx_create(int device, rir_ctx **out)
{
    if (!out)
        return fail(RIR_E_INVALID, "rir_ctx_create: null argument");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n)
        return fail(RIR_E_INVALID, "rir_ctx_create: no such device");
    HIP_TRY(hipSetDevice(device));
    std::unique_ptr<rir_ctx> c(new rir_ctx());
    c->device = device;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    for (auto &q : c->lane_st)
        HIP_TRY(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    for (auto &e : c->join_ev)
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto &e : c->ev)
        HIP_TRY(hipEventCreate(&e));
    for (auto &pr : c->ring)
        for (auto &e : pr)
            HIP_TRY(hipEventCreate(&e));
    *out = c.release();
    return RIR_OK;
}

extern "C" void rir_ctx_destroy(rir_ctx *ctx) { delete ctx; }

// Concurrent sub-batches (rir_tuning.lanes > 1): built and tested, switched
// off (see check_tuning).
constexpr bool kLanesEnabled = false;

static rir_status check_tuning(const rir_tuning *t)
{
    if (!(t->block == 64 || t->block == 128 || t->block == 256))
        return fail(RIR_E_INVALID, "rir_tuning.block must be 64, 128 or 256");
    if (t->px_per_thread < 1 || t->px_per_thread > 16)
        return fail(RIR_E_INVALID, "rir_tuning.px_per_thread must be in 1..16");
    if (t->grid_mult < 0 || t->grid_mult > 64)
        return fail(RIR_E_INVALID, "rir_tuning.grid_mult must be in 0..64");
    if (!(t->chunk == 1 || t->chunk == 2 || t->chunk == 4))
        return fail(RIR_E_INVALID, "rir_tuning.chunk must be 1, 2 or 4");
    if (t->xcd_remap != 0 && t->xcd_remap != 1)
        return fail(RIR_E_INVALID, "rir_tuning.xcd_remap must be 0 or 1");
    if (t->solve_in_step != 0 && t->solve_in_step != 1)
        return fail(RIR_E_INVALID, "rir_tuning.solve_in_step must be 0 or 1");
    if (t->lanes < 1 || t->lanes > kMaxLanes)
        return fail(RIR_E_INVALID, "rir_tuning.lanes must be in 1..4");
    // Concurrent sub-batches are switched off: a full benchmark run with them
    // on ended once in a host segmentation fault whose cause is not found.
    if (t->lanes > 1 && !kLanesEnabled)
        return fail(RIR_E_UNSUPPORTED, "rir_tuning.lanes > 1 (concurrent sub-batches) is switched off in this build");
    if (t->lane_fine != 0 && t->lane_fine != 1)
        return fail(RIR_E_INVALID, "rir_tuning.lane_fine must be 0 or 1");
    return RIR_OK;
}

extern "C" rir_status rir_ctx_set_tuning(rir_ctx *ctx, const rir_tuning *tuning)
{
    if (!ctx || !tuning)
        return fail(RIR_E_INVALID, "rir_ctx_set_tuning: null argument");
    rir_status st = check_tuning(tuning);
    if (st != RIR_OK)
        return st;
    if (std::memcmp(&ctx->tune, tuning, sizeof(rir_tuning)) != 0) {
        ctx->tune = *tuning;
        HIP_TRY(hipSetDevice(ctx->device));
        HIP_TRY(hipDeviceSynchronize());  // captured graphs of the old plans may still run
        ctx->plans.clear();
    }
    return RIR_OK;
}

extern "C" rir_status rir_ctx_get_tuning(const rir_ctx *ctx, rir_tuning *tuning)
{
    if (!ctx || !tuning)
        return fail(RIR_E_INVALID, "rir_ctx_get_tuning: null argument");
    *tuning = ctx->tune;
    return RIR_OK;
}

namespace {
// Whether timing mode `timing` brackets part l (l = levels: the prepass).
bool timed_part(int timing, int l) { return timing == 1 || (timing == 2 && l == 0); }
}  // namespace

extern "C" rir_status rir_ctx_enable_timing(rir_ctx *ctx, int32_t on)
{
    if (!ctx)
        return fail(RIR_E_INVALID, "rir_ctx_enable_timing: null context");
    if (on < 0 || on > 2)
        return fail(RIR_E_INVALID, "rir_ctx_enable_timing: mode must be 0, 1 or 2");
    ctx->timing = on;
    ctx->ev_recorded = false;
    ctx->ring_n = 0;
    return RIR_OK;
}

extern "C" rir_status rir_ctx_level_times(rir_ctx *ctx, float *ms, int32_t n)
{
    if (!ctx || !ms)
        return fail(RIR_E_INVALID, "rir_ctx_level_times: null argument");
    if (!ctx->ev_recorded)
        return fail(RIR_E_INVALID, "rir_ctx_level_times: no timed call recorded");
    HIP_TRY(hipSetDevice(ctx->device));
    const int L = ctx->timing_levels;
    for (int i = 0; i < n; ++i)
        ms[i] = 0.f;
    if (ctx->timed_mode == 2) {
        // mean over the timed calls since timing was enabled (the last kRing)
        const int cnt = std::min(ctx->ring_n, rir_ctx::kRing);
        double sum = 0.0;
        for (int k = 0; k < cnt; ++k) {
            const int i = (ctx->ring_next - 1 - k + rir_ctx::kRing) % rir_ctx::kRing;
            float t = 0.f;
            HIP_TRY(hipEventSynchronize(ctx->ring[i][1]));
            HIP_TRY(hipEventElapsedTime(&t, ctx->ring[i][0], ctx->ring[i][1]));
            sum += t;
        }
        if (n > 0 && cnt > 0)
            ms[0] = (float)(sum / cnt);
        return RIR_OK;
    }
    for (int l = 0; l <= L && l < n; ++l) {
        if (!timed_part(ctx->timed_mode, l))
            continue;
        HIP_TRY(hipEventSynchronize(ctx->ev[2 * l + 1]));
        HIP_TRY(hipEventElapsedTime(&ms[l], ctx->ev[2 * l], ctx->ev[2 * l + 1]));
    }
    return RIR_OK;
}

namespace {

rir_status check_params(const rir_icp_params *p)
{
    if (!p)
        return fail(RIR_E_INVALID, "null rir_icp_params");
    if (p->levels < 1 || p->levels > kMaxLevels)
        return fail(RIR_E_INVALID, "rir_icp_params.levels must be in 1..8");
    for (int l = 0; l < p->levels; ++l)
        if (p->iters[l] < 0 || p->iters[l] > 1000)
            return fail(RIR_E_INVALID, "rir_icp_params.iters must be in 0..1000");
    if (!(p->delta > 0.0) || !std::isfinite(p->delta))
        return fail(RIR_E_INVALID, "rir_icp_params.delta must be > 0");
    if (!(p->edge_rel > 0.0) || !std::isfinite(p->edge_rel))
        return fail(RIR_E_INVALID, "rir_icp_params.edge_rel must be > 0");
    if (!std::isfinite(p->max_corr_dist))
        return fail(RIR_E_INVALID, "rir_icp_params.max_corr_dist must be finite");
    if (p->init_mode != 0 && p->init_mode != 1)
        return fail(RIR_E_INVALID, "rir_icp_params.init_mode must be 0 or 1");
    if (p->weight_mode != RIR_WEIGHT_HUBER && p->weight_mode != RIR_WEIGHT_LEARNED)
        return fail(RIR_E_INVALID, "rir_icp_params.weight_mode must be HUBER or LEARNED");
    if (p->weight_mode == RIR_WEIGHT_LEARNED && !p->mlp)
        return fail(RIR_E_INVALID, "rir_icp_params.mlp is required with learned weights");
    if (p->weight_mode == RIR_WEIGHT_LEARNED && !(p->r_max > 0.0))
        return fail(RIR_E_INVALID, "rir_icp_params.r_max must be > 0 with learned weights");
    if (p->learned_levels < 0 || p->learned_levels >= (1 << kMaxLevels))
        return fail(RIR_E_INVALID, "rir_icp_params.learned_levels must be a bit set over levels 0..7");
    if (p->precision != RIR_PREC_FP32 && p->precision != RIR_PREC_FP64)
        return fail(RIR_E_INVALID, "rir_icp_params.precision must be FP32 or FP64");
    if (!(p->stop_eps >= 0.0) || !std::isfinite(p->stop_eps))
        return fail(RIR_E_INVALID, "rir_icp_params.stop_eps must be finite and >= 0");
    if (p->normal_window < 0 || p->normal_window > 3)
        return fail(RIR_E_INVALID, "rir_icp_params.normal_window must be 0 (cross product) or 1..3 (PCA)");
    return RIR_OK;
}

rir_status check_pairs(const rir_ctx *ctx, const rir_icp_params *p, int n, const rir_pair *pairs)
{
    if (n < 1)
        return fail(RIR_E_INVALID, "n_pairs must be >= 1");
    if (!pairs)
        return fail(RIR_E_INVALID, "pairs is null");
    const int div = 1 << (p->levels - 1);
    for (int i = 0; i < n; ++i) {
        const rir_sensor *s = pairs[i].sensor;
        if (!s || !pairs[i].src_range || !pairs[i].dst_range)
            return fail(RIR_E_INVALID, "pair " + std::to_string(i) + ": null sensor or image");
        if (s->device != ctx->device)
            return fail(RIR_E_INVALID, "pair " + std::to_string(i) + ": sensor lives on another device");
        if (s->H % div || s->W % div || p->levels > s->nlev)
            return fail(RIR_E_SHAPE, "pair " + std::to_string(i) + ": H and W must be divisible by 2^(levels-1)");
        if ((int64_t)s->H * s->W >= (1 << 24))
            return fail(RIR_E_SHAPE, "pair " + std::to_string(i) + ": images must have fewer than 2^24 pixels");
    }
    return RIR_OK;
}

template <typename T>
void set_desc_images(PairDesc<T> *d, const rir_pair &p)
{
    d->src[0] = const_cast<float *>(p.src_range);
    d->dstr[0] = const_cast<float *>(p.dst_range);
}

// Allocates and fills a plan for one batch shape.
rir_status make_plan(rir_ctx *ctx, const PlanKey &key, const rir_pair *pairs, int n, Plan *&out)
{
    std::unique_ptr<Plan> P(new Plan());
    P->key = key;
    P->device = ctx->device;
    P->n_pairs = n;
    P->fp64 = key.k.precision == RIR_PREC_FP64;
    const size_t tsz = P->fp64 ? sizeof(double) : sizeof(float);
    const int L = key.k.levels;
    P->block = key.k.tune.block;
    // a tile is block * px_per_thread pixels (in 64-pixel row segments) at
    // levels 0 and 1, and 4x fewer per level below (down to one pixel per
    // thread): large tiles amortise the per-tile reduction, small ones keep
    // the chip full on the coarse levels.  The rule depends on the tuning
    // only, so a pair's result does not depend on the batch around it.
    for (int l = 0; l < L; ++l) {
        const int sh = l > 1 ? 2 * (l - 1) : 0;
        P->tile_seg[l] = key.k.tune.block / kSegPx * std::max(1, key.k.tune.px_per_thread >> sh);
    }
    for (int l = 0; l < L; ++l) {
        bool lean = !(key.k.max_corr > 0.0);
        for (int i = 0; i < n; ++i)
            lean = lean && pairs[i].sensor->r0 == 0.0 && ((pairs[i].sensor->W >> l) % kSegPx) == 0 &&
                   (pairs[i].sensor->W & (pairs[i].sensor->W - 1)) == 0;
        P->lean[l] = lean;
    }
    // Pairs whose level image is small run all iterations of the level in the
    // pair-resident kernel (a property of the pair and the parameters only, so
    // that a pair's result never depends on its batch); they get no tiles.
    // Level 0 always keeps its tiles: the prepass and the centroid
    // initialisation walk them.
    auto resident = [&](int i, int l) {
        if (l == 0)
            return false;
        const rir_sensor *s = pairs[i].sensor;
        const int Hl = s->H >> l, Wl = s->W >> l;
        const bool learned = key.k.weight_mode == RIR_WEIGHT_LEARNED &&
                             (key.k.learned_levels == 0 || ((key.k.learned_levels >> l) & 1));
        return !key.k.debug && !P->fp64 && !learned && !(key.k.max_corr > 0.0) && s->r0 == 0.0 &&
               (s->W & (s->W - 1)) == 0 &&
               Wl % kSegPx == 0 && Hl <= kPairRows && Hl * Wl <= kPairMaxPx;
    };
    std::vector<std::vector<int2>> tiles(L);
    std::vector<int> t0(n * kMaxLevels, 0), nt(n * kMaxLevels, 0);
    for (int l = 0; l < L; ++l) {
        P->resident[l] = false;
        for (int i = 0; i < n; ++i) {
            const rir_sensor *s = pairs[i].sensor;
            const int nseg = (s->H >> l) * (((s->W >> l) + kSegPx - 1) / kSegPx);
            const bool res = resident(i, l);
            P->resident[l] = P->resident[l] || res;
            const int k = res ? 0 : (nseg + P->tile_seg[l] - 1) / P->tile_seg[l];
            t0[i * kMaxLevels + l] = (int)tiles[l].size();
            nt[i * kMaxLevels + l] = k;
            for (int j = 0; j < k; ++j)
                tiles[l].push_back(make_int2(i, j * P->tile_seg[l]));
        }
        P->n_tiles[l] = (int)tiles[l].size();
        int G = P->n_tiles[l];
        if (key.k.tune.grid_mult > 0)
            G = std::min(G, key.k.tune.grid_mult * ctx->n_cu);
        if (key.k.tune.xcd_remap)
            G = (G + 7) / 8 * 8;
        P->grid[l] = std::max(G, 1);
    }
    // Sub-batches of the coarse levels: consecutive pairs, cut where the
    // running pixel count passes k / n_lanes of the batch's (so that the
    // lanes carry about equal work).  One lane when no level runs in lanes.
    {
        const bool any = L > 1 || key.k.tune.lane_fine;
        const int S = (any && !key.k.debug) ? std::max(1, std::min(key.k.tune.lanes, n)) : 1;
        std::vector<double> cum(n + 1, 0.0);
        for (int i = 0; i < n; ++i)
            cum[i + 1] = cum[i] + (double)pairs[i].sensor->H * (double)pairs[i].sensor->W;
        P->n_lanes = S;
        P->lane_p0[0] = 0;
        for (int k = 1; k < S; ++k) {
            int i = P->lane_p0[k - 1] + 1;  // every lane keeps at least one pair
            while (i < n - (S - k) && cum[i] < cum[n] * k / S)
                ++i;
            P->lane_p0[k] = i;
        }
        P->lane_p0[S] = n;
        for (int l = 0; l < L; ++l) {
            for (int k = 0; k < S; ++k) {
                const int p0 = P->lane_p0[k];
                P->lane_t0[l][k] = t0[p0 * kMaxLevels + l];
            }
            P->lane_t0[l][S] = P->n_tiles[l];
            for (int k = 0; k < S; ++k) {
                int G = P->lane_t0[l][k + 1] - P->lane_t0[l][k];
                if (key.k.tune.grid_mult > 0)
                    G = std::min(G, key.k.tune.grid_mult * ctx->n_cu);
                if (key.k.tune.xcd_remap)
                    G = (G + 7) / 8 * 8;
                P->lane_grid[l][k] = std::max(G, 1);
            }
        }
    }
    int max_tiles = 0;  // records of all levels
    for (int l = 0; l < L; ++l) {
        P->rec0[l] = max_tiles;
        max_tiles += P->n_tiles[l];
    }
    max_tiles = std::max(max_tiles, 1);
    // device layout
    Layout lay;
    P->desc_bytes = n * (P->fp64 ? sizeof(PairDesc<double>) : sizeof(PairDesc<float>));
    size_t o_desc = lay.add(P->desc_bytes);
    size_t o_tiles[kMaxLevels];
    for (int l = 0; l < L; ++l)
        o_tiles[l] = lay.add(sizeof(int2) * tiles[l].size());
    size_t o_psum = lay.add((size_t)max_tiles * kAccum * tsz);
    size_t o_pcnt = lay.add((size_t)max_tiles * sizeof(int4));
    size_t o_pose = lay.add((size_t)n * 16 * sizeof(double));
    size_t o_stats = lay.add((size_t)n * L * sizeof(rir_level_stats));
    size_t o_flags = lay.add((size_t)(n * kFlagStride + n) * sizeof(int));  // flags, then tickets
    std::vector<size_t> o_src(n * kMaxLevels, 0), o_dstr(n * kMaxLevels, 0), o_dst4(n * kMaxLevels, 0);
    std::vector<size_t> o_nbf(n * kMaxLevels, 0);
    // learned levels of FP32 plans keep the network's neighbour features of
    // every target pixel (16 B per pixel, computed once per call)
    auto nbf_level = [&](int l) {
        return !P->fp64 && !key.k.debug && key.k.weight_mode == RIR_WEIGHT_LEARNED &&
               (key.k.learned_levels == 0 || ((key.k.learned_levels >> l) & 1));
    };
    std::vector<size_t> o_frames(n, 0);
    for (int i = 0; i < n; ++i) {
        const rir_sensor *s = pairs[i].sensor;
        o_frames[i] = lay.add((size_t)s->H * kFrame * tsz);
        for (int l = 0; l < L; ++l) {
            const size_t Nl = (size_t)(s->H >> l) * (s->W >> l);
            if (l > 0) {
                o_src[i * kMaxLevels + l] = lay.add(Nl * sizeof(float));
                o_dstr[i * kMaxLevels + l] = lay.add(Nl * sizeof(float));
            }
            o_dst4[i * kMaxLevels + l] = lay.add(Nl * 4 * tsz);
            if (nbf_level(l))
                o_nbf[i * kMaxLevels + l] = lay.add(Nl * 16);
        }
    }
    for (int l = 0; l < L; ++l) {
        P->nbf[l] = nbf_level(l);
        for (int i = 0; i < n; ++i) {
            const size_t Nl = (size_t)(pairs[i].sensor->H >> l) * (pairs[i].sensor->W >> l);
            P->max_px[l] = std::max<size_t>(P->max_px[l], Nl);
        }
    }
    HIP_TRY(hipMalloc(&P->dmem, lay.bytes));
    char *base = static_cast<char *>(P->dmem);
    HIP_TRY(hipMemset(base + o_flags, 0, (size_t)(n * kFlagStride + n) * sizeof(int)));
    P->d_desc = base + o_desc;
    for (int l = 0; l < L; ++l) {
        P->d_tiles[l] = reinterpret_cast<int2 *>(base + o_tiles[l]);
        HIP_TRY(hipMemcpy(P->d_tiles[l], tiles[l].data(), sizeof(int2) * tiles[l].size(), hipMemcpyHostToDevice));
    }
    P->d_psum = base + o_psum;
    P->d_pcnt = reinterpret_cast<int4 *>(base + o_pcnt);
    P->d_poses = reinterpret_cast<double *>(base + o_pose);
    P->d_stats = reinterpret_cast<rir_level_stats *>(base + o_stats);
    P->d_flags = reinterpret_cast<int *>(base + o_flags);
    P->d_tickets = P->d_flags + (size_t)n * kFlagStride;
    HIP_TRY(hipHostMalloc(&P->h_desc, P->desc_bytes, hipHostMallocDefault));
    std::memset(P->h_desc, 0, P->desc_bytes);
    for (int i = 0; i < n; ++i) {
        const rir_sensor *s = pairs[i].sensor;
        auto fill = [&](auto *d, auto *tab) {
            d->tab = tab;
            d->tabd = s->d_td;
            using TF = typename std::remove_pointer<typename std::remove_reference<decltype(d->frames)>::type>::type;
            d->frames = reinterpret_cast<TF *>(base + o_frames[i]);
            d->H = s->H;
            d->W = s->W;
            for (int l = 0; l < kMaxLevels; ++l) {
                d->src[l] = nullptr;
                d->dstr[l] = nullptr;
                d->dst4[l] = nullptr;
                d->nbf[l] = nullptr;
                d->tile0[l] = d->ntile[l] = 0;
            }
            for (int l = 0; l < L; ++l) {
                using TT = typename std::remove_pointer<typename std::remove_reference<decltype(d->dst4[0])>::type>::type;
                if (l > 0) {
                    d->src[l] = reinterpret_cast<float *>(base + o_src[i * kMaxLevels + l]);
                    d->dstr[l] = reinterpret_cast<float *>(base + o_dstr[i * kMaxLevels + l]);
                }
                d->dst4[l] = reinterpret_cast<TT *>(base + o_dst4[i * kMaxLevels + l]);
                if (P->nbf[l])
                    d->nbf[l] = reinterpret_cast<uint32_t *>(base + o_nbf[i * kMaxLevels + l]);
                d->tile0[l] = t0[i * kMaxLevels + l];
                d->ntile[l] = nt[i * kMaxLevels + l];
            }
            set_desc_images(d, pairs[i]);
        };
        if (P->fp64)
            fill(reinterpret_cast<PairDesc<double> *>(P->h_desc) + i, s->d_td);
        else
            fill(reinterpret_cast<PairDesc<float> *>(P->h_desc) + i, s->d_tf);
        P->cur_src.push_back(pairs[i].src_range);
        P->cur_dst.push_back(pairs[i].dst_range);
    }
    HIP_TRY(hipMemcpy(P->d_desc, P->h_desc, P->desc_bytes, hipMemcpyHostToDevice));
    HIP_TRY(hipEventCreateWithFlags(&P->desc_evt, hipEventDisableTiming));
    out = P.release();
    return RIR_OK;
}

rir_status get_plan(rir_ctx *ctx, const rir_icp_params *p, const rir_pair *pairs, int n, int debug, Plan *&out)
{
    PlanKey key;
    std::memset(&key.k, 0, sizeof(KeyPod));
    for (int i = 0; i < n; ++i)
        key.sensors.push_back(pairs[i].sensor->uid);
    KeyPod &k = key.k;
    k.levels = p->levels;
    for (int l = 0; l < kMaxLevels; ++l)
        k.iters[l] = l < p->levels ? p->iters[l] : 0;
    k.init_mode = p->init_mode;
    k.weight_mode = p->weight_mode;
    k.learned_levels = p->weight_mode == RIR_WEIGHT_LEARNED ? p->learned_levels : 0;
    k.precision = p->precision;
    k.use_graph = p->use_graph ? 1 : 0;
    k.debug = debug;
    k.delta = p->delta;
    k.edge_rel = p->edge_rel;
    k.max_corr = p->max_corr_dist;
    k.stop_eps = p->stop_eps;
    k.normal_window = p->normal_window;
    k.r_max = p->weight_mode == RIR_WEIGHT_LEARNED ? p->r_max : 0.0;
    k.mlp = p->weight_mode == RIR_WEIGHT_LEARNED ? p->mlp->uid : 0;
    k.tune = ctx->tune;
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) {
        Plan *P = it->second.get();
        for (int i = 0; i < n; ++i)
            if (P->shapes[2 * i] != pairs[i].sensor->H || P->shapes[2 * i + 1] != pairs[i].sensor->W)
                return fail(RIR_E_SHAPE, "internal: cached plan does not match the batch shape");
        P->last_use = ++ctx->use_clock;
        out = P;
        return RIR_OK;
    }
    // keep at most kMaxPlans plans: evict the least recently used (plans of
    // destroyed sensors are never used again and age out this way)
    constexpr size_t kMaxPlans = 8;
    if (ctx->plans.size() >= kMaxPlans) {
        HIP_TRY(hipDeviceSynchronize());
        while (ctx->plans.size() >= kMaxPlans) {
            auto victim = ctx->plans.begin();
            for (auto jt = ctx->plans.begin(); jt != ctx->plans.end(); ++jt)
                if (jt->second->last_use < victim->second->last_use)
                    victim = jt;
            ctx->plans.erase(victim);
        }
    }
    Plan *P = nullptr;
    rir_status st = make_plan(ctx, key, pairs, n, P);
    if (st != RIR_OK)
        return st;
    for (int i = 0; i < n; ++i) {
        P->shapes.push_back(pairs[i].sensor->H);
        P->shapes.push_back(pairs[i].sensor->W);
    }
    P->last_use = ++ctx->use_clock;
    ctx->plans[key].reset(P);
    out = P;
    return RIR_OK;
}

// Points the plan's descriptors at this call's images (only when they changed).
rir_status update_images(Plan *P, const rir_pair *pairs, hipStream_t st)
{
    bool changed = false;
    for (int i = 0; i < P->n_pairs; ++i)
        if (P->cur_src[i] != pairs[i].src_range || P->cur_dst[i] != pairs[i].dst_range)
            changed = true;
    if (!changed)
        return RIR_OK;
    // the pinned staging copy may still be read by a previous enqueued copy
    HIP_TRY(hipEventSynchronize(P->desc_evt));
    for (int i = 0; i < P->n_pairs; ++i) {
        if (P->fp64)
            set_desc_images(reinterpret_cast<PairDesc<double> *>(P->h_desc) + i, pairs[i]);
        else
            set_desc_images(reinterpret_cast<PairDesc<float> *>(P->h_desc) + i, pairs[i]);
        P->cur_src[i] = pairs[i].src_range;
        P->cur_dst[i] = pairs[i].dst_range;
    }
    HIP_TRY(hipMemcpyAsync(P->d_desc, P->h_desc, P->desc_bytes, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(P->desc_evt, st));
    return RIR_OK;
}

// Learned weights at this level (weight_mode LEARNED and the level selected).
bool learned_at(const rir_icp_params *p, int level)
{
    return p->weight_mode == RIR_WEIGHT_LEARNED && (p->learned_levels == 0 || ((p->learned_levels >> level) & 1));
}

// Arguments of the launches of one iteration; lane >= 0 restricts them to
// that sub-batch's pairs and tiles.
StepArgs step_args(const Plan *P, const rir_icp_params *p, int level, int iter, int mode, int lane = -1)
{
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.pairs = P->d_desc;
    a.tiles = P->d_tiles[level];
    a.n_tiles = P->n_tiles[level];
    if (lane >= 0) {
        a.tile_base = P->lane_t0[level][lane];
        a.n_tiles = P->lane_t0[level][lane + 1] - a.tile_base;
        a.pair_base = P->lane_p0[lane];
    }
    a.level = level;
    a.iter = iter;
    a.levels = P->key.k.levels;
    a.tile_seg = P->tile_seg[level];
    a.chunk = P->key.k.tune.chunk;
    a.xcd_remap = P->key.k.tune.xcd_remap;
    a.mode = mode;
    a.iters = P->key.k.iters[level];
    a.stats_pass = (mode == kStepDebug || iter == P->key.k.iters[level] - 1) ? 1 : 0;
    a.lean = (mode != kStepDebug && P->lean[level]) ? 1 : 0;
    a.learned = learned_at(p, level) ? 1 : 0;
    a.psum = static_cast<char *>(P->d_psum) + (size_t)P->rec0[level] * kAccum * (P->fp64 ? sizeof(double) : sizeof(float));
    a.pcnt = P->d_pcnt + P->rec0[level];
    a.poses = P->d_poses;
    a.stats = P->d_stats;
    a.flags = P->d_flags;
    a.tickets = P->d_tickets;
    // the solving step launch covers one tile per workgroup
    a.fused = (mode != kStepDebug && P->key.k.tune.solve_in_step && P->key.k.tune.grid_mult == 0) ? 1 : 0;
    a.delta = p->delta;
    a.max_corr = p->max_corr_dist;
    a.stop_eps = p->stop_eps;
    a.r_max = (float)p->r_max;
    if (p->weight_mode == RIR_WEIGHT_LEARNED)
        a.mlp = p->mlp->dev();
    return a;
}

// Enqueues the flag/ticket/statistics reset of the whole batch.
rir_status enqueue_clear(const Plan *P, hipStream_t st)
{
    HIP_TRY(launch_clear(P->d_flags, P->n_pairs * (kFlagStride + 1), P->d_stats, P->n_pairs * P->key.k.levels, st));
    return RIR_OK;
}

// Enqueues the normal/pyramid pass (target records, level images, learned
// neighbour features, initial pose and ray frames) of the whole batch
// (lane < 0) or of one sub-batch.
rir_status enqueue_prepass(const Plan *P, const rir_icp_params *p, hipStream_t st, int lane = -1)
{
    const int np = lane < 0 ? P->n_pairs : P->lane_p0[lane + 1] - P->lane_p0[lane];
    const int pb = lane < 0 ? 0 : P->lane_p0[lane];
    PrepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.pairs = P->d_desc;
    a.tiles = P->d_tiles[0];
    a.n_tiles = P->n_tiles[0];
    if (lane >= 0) {
        a.tile_base = P->lane_t0[0][lane];
        a.n_tiles = P->lane_t0[0][lane + 1] - a.tile_base;
    }
    a.pair_base = pb;
    a.tile_seg = P->tile_seg[0];
    a.levels = P->key.k.levels;
    a.init_centroid = p->init_mode == 1;
    a.edge_rel = p->edge_rel;
    a.psum = P->d_psum;  // level-0 records
    a.poses = P->d_poses;
    a.xcd_remap = P->key.k.tune.xcd_remap;
    a.given_normals = P->key.k.normal_window > 0 ? 1 : 0;
    if (a.given_normals)
        HIP_TRY(launch_pca_records(P->fp64, a, P->key.k.normal_window, np, (int)P->max_px[0], st));
    HIP_TRY(launch_prepass(P->fp64, a, lane < 0 ? P->grid[0] : P->lane_grid[0][lane], P->block, np, st));
    for (int l = 0; l < P->key.k.levels; ++l)
        if (P->nbf[l]) {
            NbrArgs b;
            b.pairs = P->d_desc;
            b.pair_base = pb;
            b.level = l;
            b.delta = p->delta;
            HIP_TRY(launch_nbr_feats(b, np, (int)P->max_px[l], st));
        }
    StepArgs f = step_args(P, p, 0, 0, kStepNormal, lane);
    HIP_TRY(launch_frames(P->fp64, f, np, st));
    return RIR_OK;
}

// Enqueues the Gauss-Newton iterations of one level, for the whole batch
// (lane < 0) or for one sub-batch.
rir_status enqueue_level(const Plan *P, const rir_icp_params *p, int l, hipStream_t st, int lane = -1)
{
    const int np = lane < 0 ? P->n_pairs : P->lane_p0[lane + 1] - P->lane_p0[lane];
    const int grid = lane < 0 ? P->grid[l] : P->lane_grid[l][lane];
    if (P->resident[l] && P->key.k.iters[l] > 0)
        HIP_TRY(launch_level(P->fp64, step_args(P, p, l, 0, kStepNormal, lane), np, st));
    if (step_args(P, p, l, 0, kStepNormal, lane).n_tiles == 0)
        return RIR_OK;
    for (int it = 0; it < P->key.k.iters[l]; ++it) {
        StepArgs a = step_args(P, p, l, it, kStepNormal, lane);
        HIP_TRY(launch_step(P->fp64, a.learned ? RIR_WEIGHT_LEARNED : RIR_WEIGHT_HUBER, a, grid, P->block, st));
        if (!a.fused)
            HIP_TRY(launch_solve(P->fp64, a, np, st));
        if (a.learned) {
            StepArgs b = step_args(P, p, l, it, kStepFallback, lane);
            HIP_TRY(launch_step(P->fp64, RIR_WEIGHT_HUBER, b, grid, P->block, st));
            if (!b.fused)
                HIP_TRY(launch_solve(P->fp64, b, np, st));
        }
    }
    return RIR_OK;
}

// The prepass (with `prepass`) and levels hi .. lo (coarse to fine; none if
// hi < lo) of every sub-batch, each on its lane stream: forked from st after
// the work enqueued so far, joined back into st.
rir_status enqueue_lanes(rir_ctx *ctx, const Plan *P, const rir_icp_params *p, bool prepass, int hi, int lo,
                         hipStream_t st)
{
    HIP_TRY(hipEventRecord(ctx->fork_ev, st));
    for (int k = 0; k < P->n_lanes; ++k) {
        hipStream_t q = ctx->lane_st[k];
        HIP_TRY(hipStreamWaitEvent(q, ctx->fork_ev, 0));
        if (prepass) {
            rir_status s = enqueue_prepass(P, p, q, k);
            if (s != RIR_OK)
                return s;
        }
        for (int l = hi; l >= lo; --l) {
            rir_status s = enqueue_level(P, p, l, q, k);
            if (s != RIR_OK)
                return s;
        }
        HIP_TRY(hipEventRecord(ctx->join_ev[k], q));
        HIP_TRY(hipStreamWaitEvent(st, ctx->join_ev[k], 0));
    }
    return RIR_OK;
}

// Records timing event e on st.  While st is being captured, the event
// becomes an event-record node of the graph: added after the nodes the next
// captured work would depend on, and made the only dependency of that work.
rir_status record_timing(hipEvent_t e, hipStream_t st, bool capturing)
{
    if (!capturing) {
        HIP_TRY(hipEventRecord(e, st));
        return RIR_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    hipGraph_t g = nullptr;
    const hipGraphNode_t *deps = nullptr;
    size_t nd = 0;
    HIP_TRY(hipStreamGetCaptureInfo_v2(st, &cs, &id, &g, &deps, &nd));
    if (cs != hipStreamCaptureStatusActive || !g)
        return fail(RIR_E_HIP, "timing event outside an active capture");
    hipGraphNode_t node = nullptr;
    HIP_TRY(hipGraphAddEventRecordNode(&node, g, deps, nd, e));
    HIP_TRY(hipStreamUpdateCaptureDependencies(st, &node, 1, hipStreamSetCaptureDependencies));
    return RIR_OK;
}

// Enqueues the whole schedule: reset, prepass, then the levels coarse to
// fine, with timing events around the prepass and every level (timing 1) or
// around the finest level (timing 2; `fine` the event pair, else the
// context's).  With more than one lane the prepass and the coarse levels
// (with lane_fine all levels) run as concurrent sub-batches, forked once
// after the reset and joined at the end; timing joins and forks again at
// each timed boundary (after the prepass and every level under timing 1,
// before the finest level under timing 2), so that each timed part has its
// own time.
rir_status enqueue_all(rir_ctx *ctx, Plan *P, const rir_icp_params *p, int timing, hipStream_t st, hipEvent_t *fine,
                       bool capturing)
{
    const int L = P->key.k.levels;
    hipEvent_t *evs = ctx->ev;
    rir_status s = RIR_OK;
    const bool lanes = P->n_lanes > 1, fine_lanes = lanes && P->key.k.tune.lane_fine;
    if (timed_part(timing, L) && (s = record_timing(evs[2 * L], st, capturing)) != RIR_OK)
        return s;
    if ((s = enqueue_clear(P, st)) != RIR_OK)
        return s;
    if (lanes && timing == 0)
        s = enqueue_lanes(ctx, P, p, true, L - 1, fine_lanes ? 0 : 1, st);
    else if (lanes && timing == 2)
        s = enqueue_lanes(ctx, P, p, true, L - 1, 1, st);
    else if (lanes)
        s = enqueue_lanes(ctx, P, p, true, -1, 0, st);
    else
        s = enqueue_prepass(P, p, st);
    if (s != RIR_OK)
        return s;
    if (timed_part(timing, L) && (s = record_timing(evs[2 * L + 1], st, capturing)) != RIR_OK)
        return s;
    if (!lanes || timing == 1) {
        for (int l = L - 1; l >= 1; --l) {
            if (timed_part(timing, l) && (s = record_timing(evs[2 * l], st, capturing)) != RIR_OK)
                return s;
            s = lanes ? enqueue_lanes(ctx, P, p, false, l, l, st) : enqueue_level(P, p, l, st);
            if (s != RIR_OK)
                return s;
            if (timed_part(timing, l) && (s = record_timing(evs[2 * l + 1], st, capturing)) != RIR_OK)
                return s;
        }
    }
    if (lanes && timing == 0 && fine_lanes)
        return RIR_OK;  // the finest level ran in the lanes
    if (timed_part(timing, 0) && (s = record_timing(fine ? fine[0] : evs[0], st, capturing)) != RIR_OK)
        return s;
    if ((s = fine_lanes ? enqueue_lanes(ctx, P, p, false, 0, 0, st) : enqueue_level(P, p, 0, st)) != RIR_OK)
        return s;
    if (timed_part(timing, 0) && (s = record_timing(fine ? fine[1] : evs[1], st, capturing)) != RIR_OK)
        return s;
    return RIR_OK;
}

// The whole schedule as one graph, captured on the context's private stream
// (the lane streams join the capture): one launch per call, kernels back to
// back, parallel branches for the sub-batches of the coarse levels, and the
// timing events as event-record nodes.
rir_status capture(rir_ctx *ctx, Plan *P, const rir_icp_params *p, int timing, hipGraphExec_t *out)
{
    hipStream_t cs = ctx->cap;
    // timing 2: captured with ring pair 0, re-pointed at each call's pair
    hipEvent_t fine[2] = {ctx->ring[0][0], ctx->ring[0][1]};
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    rir_status st = enqueue_all(ctx, P, p, timing, cs, timing == 2 ? fine : nullptr, true);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (st != RIR_OK) {
        if (g)
            hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess)
        return fail(RIR_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    if (timing == 2) {
        P->fine_ev[0] = P->fine_ev[1] = nullptr;
        size_t nn = 0;
        e = hipGraphGetNodes(g, nullptr, &nn);
        std::vector<hipGraphNode_t> nodes(nn);
        if (e == hipSuccess)
            e = hipGraphGetNodes(g, nodes.data(), &nn);
        for (size_t i = 0; i < nn && e == hipSuccess; ++i) {
            hipGraphNodeType t;
            e = hipGraphNodeGetType(nodes[i], &t);
            if (e != hipSuccess || t != hipGraphNodeTypeEventRecord)
                continue;
            hipEvent_t ev = nullptr;
            e = hipGraphEventRecordNodeGetEvent(nodes[i], &ev);
            for (int k = 0; k < 2; ++k)
                if (e == hipSuccess && ev == fine[k])
                    P->fine_ev[k] = nodes[i];
        }
        if (e == hipSuccess && (!P->fine_ev[0] || !P->fine_ev[1])) {
            hipGraphDestroy(g);
            return fail(RIR_E_HIP, "captured schedule lacks the timing event nodes");
        }
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        return fail(RIR_E_HIP, std::string("instantiating the schedule graph: ") + hipGetErrorString(e));
    }
    // the source graph stays alive with the plan: its event nodes address the
    // instantiated graph when the timing events are swapped per call
    if (P->g_src[timing])
        hipGraphDestroy(P->g_src[timing]);
    P->g_src[timing] = g;
    return RIR_OK;
}

rir_status run_plan(rir_ctx *ctx, Plan *P, const rir_icp_params *p, hipStream_t st)
{
    const int tm = ctx->timing;
    hipEvent_t *fine = nullptr;
    if (tm == 2) {
        fine = ctx->ring[ctx->ring_next];
        ctx->ring_next = (ctx->ring_next + 1) % rir_ctx::kRing;
        ctx->ring_n = std::min(ctx->ring_n + 1, rir_ctx::kRing);
    }
    if (p->use_graph) {
        hipGraphExec_t &g = P->g_run[tm];
        if (!g) {
            rir_status s = capture(ctx, P, p, tm, &g);
            if (s != RIR_OK)
                return s;
        }
        if (fine) {
            HIP_TRY(hipGraphExecEventRecordNodeSetEvent(g, P->fine_ev[0], fine[0]));
            HIP_TRY(hipGraphExecEventRecordNodeSetEvent(g, P->fine_ev[1], fine[1]));
        }
        HIP_TRY(hipGraphLaunch(g, st));
    } else {
        rir_status s = enqueue_all(ctx, P, p, tm, st, fine, false);
        if (s != RIR_OK)
            return s;
    }
    if (tm) {
        ctx->timing_levels = P->key.k.levels;
        ctx->timed_mode = tm;
        ctx->ev_recorded = true;
    }
    return RIR_OK;
}

}  // namespace

extern "C" rir_status rir_icp_batch(rir_ctx *ctx, const rir_icp_params *params, int32_t n_pairs, const rir_pair *pairs,
                                    const double *init_poses, double *poses_out, rir_level_stats *stats_out,
                                    void *stream)
{
    if (!ctx)
        return fail(RIR_E_INVALID, "rir_icp_batch: null context");
    rir_status s = check_params(params);
    if (s != RIR_OK)
        return s;
    s = check_pairs(ctx, params, n_pairs, pairs);
    if (s != RIR_OK)
        return s;
    if (!poses_out || (params->init_mode == 0 && !init_poses))
        return fail(RIR_E_INVALID, "rir_icp_batch: null pose buffer");
    if (params->weight_mode == RIR_WEIGHT_LEARNED && params->mlp->device != ctx->device)
        return fail(RIR_E_INVALID, "rir_icp_batch: network lives on another device");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Plan *P = nullptr;
    s = get_plan(ctx, params, pairs, n_pairs, 0, P);
    if (s != RIR_OK)
        return s;
    s = update_images(P, pairs, st);
    if (s != RIR_OK)
        return s;
    const size_t pose_bytes = (size_t)n_pairs * 16 * sizeof(double);
    if (params->init_mode == 0)
        HIP_TRY(hipMemcpyAsync(P->d_poses, init_poses, pose_bytes, hipMemcpyDeviceToDevice, st));
    s = run_plan(ctx, P, params, st);
    if (s != RIR_OK)
        return s;
    HIP_TRY(hipMemcpyAsync(poses_out, P->d_poses, pose_bytes, hipMemcpyDeviceToDevice, st));
    if (stats_out)
        HIP_TRY(hipMemcpyAsync(stats_out, P->d_stats, (size_t)n_pairs * params->levels * sizeof(rir_level_stats),
                               hipMemcpyDeviceToDevice, st));
    return RIR_OK;
}

extern "C" rir_status rir_debug_associate(rir_ctx *ctx, const rir_icp_params *params, const rir_pair *pair,
                                          int32_t level, const double *pose, int32_t *u, int32_t *v, uint8_t *mask,
                                          float *e, float *w, float *J, float *feat, rir_level_stats *stats_out,
                                          void *stream)
{
    if (!ctx || !pose)
        return fail(RIR_E_INVALID, "rir_debug_associate: null argument");
    rir_status s = check_params(params);
    if (s != RIR_OK)
        return s;
    s = check_pairs(ctx, params, 1, pair);
    if (s != RIR_OK)
        return s;
    if (level < 0 || level >= params->levels)
        return fail(RIR_E_INVALID, "rir_debug_associate: level out of range");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    rir_icp_params q = *params;
    q.use_graph = 0;
    q.init_mode = 0;
    Plan *P = nullptr;
    s = get_plan(ctx, &q, pair, 1, 1, P);
    if (s != RIR_OK)
        return s;
    s = update_images(P, pair, st);
    if (s != RIR_OK)
        return s;
    s = enqueue_clear(P, st);
    if (s == RIR_OK)
        s = enqueue_prepass(P, &q, st);
    if (s != RIR_OK)
        return s;
    // the pose goes through the (pinned) descriptor staging event discipline
    HIP_TRY(hipEventSynchronize(P->desc_evt));
    double *hp = nullptr;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&hp), 16 * sizeof(double), hipHostMallocDefault));
    std::memcpy(hp, pose, 16 * sizeof(double));
    hipError_t e1 = hipMemcpyAsync(P->d_poses, hp, 16 * sizeof(double), hipMemcpyHostToDevice, st);
    StepArgs a = step_args(P, &q, level, 0, kStepDebug);
    a.dbg_u = u;
    a.dbg_v = v;
    a.dbg_mask = mask;
    a.dbg_e = e;
    a.dbg_w = w;
    a.dbg_J = J;
    a.dbg_feat = feat;
    hipError_t e2 = e1 == hipSuccess ? launch_frames(P->fp64, a, 1, st) : e1;
    if (e2 == hipSuccess)
        e2 = launch_step(P->fp64, a.learned ? RIR_WEIGHT_LEARNED : RIR_WEIGHT_HUBER, a, P->grid[level], P->block, st);
    if (e2 == hipSuccess)
        e2 = launch_solve(P->fp64, a, 1, st);
    hipError_t e3 = hipStreamSynchronize(st);
    hipHostFree(hp);
    HIP_TRY(e1);
    HIP_TRY(e2);
    HIP_TRY(e3);
    if (stats_out)
        HIP_TRY(hipMemcpy(stats_out, P->d_stats, sizeof(rir_level_stats), hipMemcpyDeviceToHost));
    return RIR_OK;
}

extern "C" rir_status rir_autotune(rir_ctx *ctx, const rir_icp_params *params, int32_t n_pairs,
                                   const rir_pair *pairs, const double *init_poses, double *poses_scratch,
                                   rir_tuning *best, float *best_ms, void *stream)
{
    if (!ctx || !poses_scratch)
        return fail(RIR_E_INVALID, "rir_autotune: null argument");
    rir_status s = check_params(params);
    if (s != RIR_OK)
        return s;
    s = check_pairs(ctx, params, n_pairs, pairs);
    if (s != RIR_OK)
        return s;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int was_timing = ctx->timing;
    ctx->timing = 0;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int blocks[] = {128, 256};
    const int ppts[] = {4, 8, 16};
    const int gms[] = {0, 4};
    const int chunks[] = {1, 2, 4};
    rir_tuning bt = ctx->tune;
    float bms = INFINITY;
    // the launch shape at the context's lane setting (the lane count is not
    // swept: concurrent sub-batches stay off unless the caller sets them)
    std::vector<rir_tuning> cands;
    for (int b : blocks)
        for (int ppt : ppts)
            for (int gm : gms)
                for (int ch : chunks)
                    cands.push_back(rir_tuning{b, ppt, gm, 1, ch, 1, ctx->tune.lanes, ctx->tune.lane_fine});
    for (size_t ci = 0; ci < cands.size() && s == RIR_OK; ++ci) {
        const rir_tuning t = cands[ci];
        s = rir_ctx_set_tuning(ctx, &t);
        if (s != RIR_OK)
            break;
        // warm-up (builds the plan and captures the graphs)
        s = rir_icp_batch(ctx, params, n_pairs, pairs, init_poses, poses_scratch, nullptr, stream);
        if (s != RIR_OK)
            break;
        const int reps = 3;
        if (hipEventRecord(e0, st) != hipSuccess)
            break;
        for (int r = 0; r < reps && s == RIR_OK; ++r)
            s = rir_icp_batch(ctx, params, n_pairs, pairs, init_poses, poses_scratch, nullptr, stream);
        if (s != RIR_OK)
            break;
        hipEventRecord(e1, st);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (ms < bms) {
            bms = ms;
            bt = t;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    ctx->timing = was_timing;
    if (s != RIR_OK)
        return s;
    s = rir_ctx_set_tuning(ctx, &bt);
    if (s != RIR_OK)
        return s;
    if (best)
        *best = bt;
    if (best_ms)
        *best_ms = bms;
    return RIR_OK;
}

// ============================================================================ geometry entry points

extern "C" rir_status rir_unproject(const rir_sensor *sensor, const float *range, float *xyz, uint8_t *valid,
                                    void *stream)
{
    if (!sensor || !range || !xyz || !valid)
        return fail(RIR_E_INVALID, "rir_unproject: null argument");
    HIP_TRY(hipSetDevice(sensor->device));
    HIP_TRY(launch_unproject(sensor->tf, range, xyz, valid, static_cast<hipStream_t>(stream)));
    return RIR_OK;
}

extern "C" rir_status rir_project(const rir_sensor *sensor, int32_t level, const float *xyz, int64_t n, int32_t *u,
                                  int32_t *v, float *r, uint8_t *valid, void *stream)
{
    if (!sensor || (n > 0 && (!xyz || !u || !v || !r || !valid)))
        return fail(RIR_E_INVALID, "rir_project: null argument");
    if (n < 0)
        return fail(RIR_E_INVALID, "rir_project: n < 0");
    if (level < 0 || level >= sensor->nlev)
        return fail(RIR_E_SHAPE, "rir_project: level not supported by this sensor's shape");
    if (n == 0)
        return RIR_OK;
    HIP_TRY(hipSetDevice(sensor->device));
    HIP_TRY(launch_project(sensor->d_tf, level, xyz, n, u, v, r, valid, static_cast<hipStream_t>(stream)));
    return RIR_OK;
}

extern "C" rir_status rir_normals(const rir_sensor *sensor, const float *range, double edge_rel, float *nrm,
                                  uint8_t *valid, void *stream)
{
    if (!sensor || !range || !nrm || !valid)
        return fail(RIR_E_INVALID, "rir_normals: null argument");
    if (!(edge_rel > 0.0) || !std::isfinite(edge_rel))
        return fail(RIR_E_INVALID, "rir_normals: edge_rel must be > 0");
    HIP_TRY(hipSetDevice(sensor->device));
    HIP_TRY(launch_normals(sensor->tf, range, edge_rel, nrm, valid, static_cast<hipStream_t>(stream)));
    return RIR_OK;
}

extern "C" rir_status rir_normals_pca(const rir_sensor *sensor, int32_t n_images, const float *range, int32_t half,
                                      double edge_rel, float *nrm, uint8_t *valid, void *stream)
{
    if (!sensor)
        return fail(RIR_E_INVALID, "rir_normals_pca: null argument");
    if (n_images < 0)
        return fail(RIR_E_INVALID, "rir_normals_pca: n_images < 0");
    if (n_images > 0 && (!range || !nrm || !valid))
        return fail(RIR_E_INVALID, "rir_normals_pca: null argument");
    if (half < 1 || half > 3)
        return fail(RIR_E_INVALID, "rir_normals_pca: half must be 1, 2 or 3");
    if (!(edge_rel > 0.0) || !std::isfinite(edge_rel))
        return fail(RIR_E_INVALID, "rir_normals_pca: edge_rel must be > 0");
    if (n_images == 0)
        return RIR_OK;
    HIP_TRY(hipSetDevice(sensor->device));
    HIP_TRY(launch_normals_pca(sensor->td, range, n_images, half, edge_rel, nrm, valid,
                               static_cast<hipStream_t>(stream)));
    return RIR_OK;
}

extern "C" rir_status rir_deskew(const rir_sensor *sensor, int32_t n_images, const float *range_in,
                                 const double *twists, float *range_out, void *stream)
{
    if (!sensor)
        return fail(RIR_E_INVALID, "rir_deskew: null argument");
    if (n_images < 0)
        return fail(RIR_E_INVALID, "rir_deskew: n_images < 0");
    if (n_images == 0)
        return RIR_OK;
    if (!range_in || !twists || !range_out)
        return fail(RIR_E_INVALID, "rir_deskew: null argument");
    const size_t bytes = (size_t)n_images * sensor->H * sensor->W * sizeof(float);
    const char *a = reinterpret_cast<const char *>(range_in), *b = reinterpret_cast<const char *>(range_out);
    if (a < b + bytes && b < a + bytes)
        return fail(RIR_E_INVALID, "rir_deskew: range_out overlaps range_in");
    for (int64_t i = 0; i < 6 * (int64_t)n_images; ++i)
        if (!std::isfinite(twists[i]))
            return fail(RIR_E_INVALID, "rir_deskew: non-finite twist");
    HIP_TRY(hipSetDevice(sensor->device));
    HIP_TRY(launch_deskew(sensor->d_td, sensor->H, sensor->W, sensor->r0 > 0.0, n_images, range_in, twists,
                          range_out, static_cast<hipStream_t>(stream)));
    return RIR_OK;
}

// ============================================================================ projective SDF fusion

// Fusion arguments shared by the dense and the sparse volume: the sensor's
// FP32 tables, the truncation band, the range clip and the cull distance.
static void sdf_common_args(const rir_sensor *sensor, double trunc, double r_clip, SdfArgs &a)
{
    a.tab = sensor->d_tf;
    a.xcd_remap = 1;
    a.trunc = trunc > 0.0 ? (float)trunc : std::numeric_limits<float>::infinity();
    if (r_clip > 0.0) {
        // the largest float not above r_clip: the FP32 test om <= clip then
        // decides exactly as om <= r_clip in real arithmetic
        float c = (float)r_clip;
        if ((double)c > r_clip)
            c = std::nextafter(c, 0.0f);
        a.clip = c;
    } else {
        a.clip = std::numeric_limits<float>::infinity();
    }
    // A voxel is updated only if Omega <= r_clip and Omega - r >= -trunc, so its
    // distance to the sensor origin is at most r_clip + trunc + r0; the margin
    // covers the FP32 rounding of r.
    a.cull = (trunc > 0.0 && r_clip > 0.0) ? r_clip + trunc + sensor->r0 + 1e-3 + 1e-4 * (r_clip + trunc) : -1.0;
}

// World -> sensor poses of k scans (row-major 4x4) as fusion frames.
static void sdf_frames(const double *poses, int k, SdfFrame *f)
{
    for (int j = 0; j < k; ++j) {
        const double *T = poses + 16 * (size_t)j;
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c)
                f[j].R[3 * r + c] = T[4 * r + c];
            f[j].t[r] = T[4 * r + 3];
        }
    }
}

extern "C" rir_status rir_sdf_integrate(const rir_sensor *sensor, const rir_volume_desc *vol, float *voxels,
                                        int32_t n_frames, const float *ranges, const double *poses, double trunc,
                                        double r_clip, void *stream)
{
    if (!sensor || !vol)
        return fail(RIR_E_INVALID, "rir_sdf_integrate: null argument");
    if (n_frames < 0)
        return fail(RIR_E_INVALID, "rir_sdf_integrate: n_frames < 0");
    if (n_frames > 0 && (!voxels || !ranges || !poses))
        return fail(RIR_E_INVALID, "rir_sdf_integrate: null argument");
    if (vol->nbx < 1 || vol->nby < 1 || vol->nbz < 1)
        return fail(RIR_E_SHAPE, "rir_sdf_integrate: block counts must be >= 1");
    const int64_t nblk = (int64_t)vol->nbx * vol->nby * vol->nbz;
    if (nblk > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(RIR_E_SHAPE, "rir_sdf_integrate: more than 2^31 - 1 blocks");
    if (!(vol->voxel > 0.0) || !std::isfinite(vol->voxel))
        return fail(RIR_E_INVALID, "rir_sdf_integrate: voxel size must be finite and > 0");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(vol->origin[i]))
            return fail(RIR_E_INVALID, "rir_sdf_integrate: origin must be finite");
    if (!std::isfinite(trunc) || !std::isfinite(r_clip))
        return fail(RIR_E_INVALID, "rir_sdf_integrate: trunc and r_clip must be finite");
    for (int64_t i = 0; i < 16 * (int64_t)n_frames; ++i)
        if (!std::isfinite(poses[i]))
            return fail(RIR_E_INVALID, "rir_sdf_integrate: non-finite pose");
    const int64_t img_bytes = (int64_t)sensor->H * sensor->W * (int64_t)sizeof(float);
    if (img_bytes * kSdfFrames >= ((int64_t)1 << 31))
        return fail(RIR_E_SHAPE, "rir_sdf_integrate: range images too large for one launch");
    if (n_frames == 0)
        return RIR_OK;
    HIP_TRY(hipSetDevice(sensor->device));

    SdfArgs a{};
    sdf_common_args(sensor, trunc, r_clip, a);
    a.vox = voxels;
    a.nbx = vol->nbx;
    a.nby = vol->nby;
    a.nbz = vol->nbz;
    for (int i = 0; i < 3; ++i)
        a.origin[i] = vol->origin[i];
    a.voxel = vol->voxel;
    const bool r0 = sensor->r0 > 0.0;
    const bool pow2 = (sensor->W & (sensor->W - 1)) == 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int32_t f0 = 0; f0 < n_frames; f0 += kSdfFrames) {
        const int k = std::min<int32_t>(kSdfFrames, n_frames - f0);
        a.n_frames = k;
        a.ranges = ranges + (size_t)f0 * (size_t)(img_bytes / (int64_t)sizeof(float));
        sdf_frames(poses + 16 * (size_t)f0, k, a.f);
        HIP_TRY(launch_sdf_fuse(a, r0, pow2, false, st));
    }
    return RIR_OK;
}


extern "C" rir_status rir_sdf_extract(const rir_volume_desc *vol, const float *voxels, double min_weight,
                                      double max_jump, float *points, int64_t max_points, uint64_t *count,
                                      void *stream)
{
    if (!vol || !voxels || !count || (max_points > 0 && !points))
        return fail(RIR_E_INVALID, "rir_sdf_extract: null argument");
    if (max_points < 0)
        return fail(RIR_E_INVALID, "rir_sdf_extract: max_points < 0");
    if (vol->nbx < 1 || vol->nby < 1 || vol->nbz < 1)
        return fail(RIR_E_SHAPE, "rir_sdf_extract: block counts must be >= 1");
    if ((int64_t)vol->nbx * vol->nby * vol->nbz > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(RIR_E_SHAPE, "rir_sdf_extract: more than 2^31 - 1 blocks");
    if (!(vol->voxel > 0.0) || !std::isfinite(vol->voxel))
        return fail(RIR_E_INVALID, "rir_sdf_extract: voxel size must be finite and > 0");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(vol->origin[i]))
            return fail(RIR_E_INVALID, "rir_sdf_extract: origin must be finite");
    if (!std::isfinite(min_weight) || std::isnan(max_jump) || !(max_jump >= 0.0))
        return fail(RIR_E_INVALID, "rir_sdf_extract: min_weight must be finite and max_jump >= 0");
    SdfExtractArgs a{};
    a.vox = voxels;
    a.nbx = vol->nbx;
    a.nby = vol->nby;
    a.nbz = vol->nbz;
    a.min_weight = (float)min_weight;
    if ((double)a.min_weight < min_weight)
        a.min_weight = std::nextafter(a.min_weight, std::numeric_limits<float>::infinity());
    a.max_jump = max_jump;
    for (int i = 0; i < 3; ++i)
        a.origin[i] = vol->origin[i];
    a.voxel = vol->voxel;
    a.pts = points;
    a.max_pts = max_points;
    a.count = reinterpret_cast<unsigned long long *>(count);
    HIP_TRY(launch_sdf_extract(a, false, static_cast<hipStream_t>(stream)));
    return RIR_OK;
}

extern "C" rir_status rir_sdf_mesh(const rir_volume_desc *vol, const float *voxels, double min_weight,
                                   double max_jump, float *triangles, int64_t max_triangles, uint64_t *count,
                                   void *stream)
{
    if (!vol || !voxels || !count || (max_triangles > 0 && !triangles))
        return fail(RIR_E_INVALID, "rir_sdf_mesh: null argument");
    if (max_triangles < 0)
        return fail(RIR_E_INVALID, "rir_sdf_mesh: max_triangles < 0");
    if (vol->nbx < 1 || vol->nby < 1 || vol->nbz < 1)
        return fail(RIR_E_SHAPE, "rir_sdf_mesh: block counts must be >= 1");
    if ((int64_t)vol->nbx * vol->nby * vol->nbz > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(RIR_E_SHAPE, "rir_sdf_mesh: more than 2^31 - 1 blocks");
    if (!(vol->voxel > 0.0) || !std::isfinite(vol->voxel))
        return fail(RIR_E_INVALID, "rir_sdf_mesh: voxel size must be finite and > 0");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(vol->origin[i]))
            return fail(RIR_E_INVALID, "rir_sdf_mesh: origin must be finite");
    if (!std::isfinite(min_weight) || std::isnan(max_jump) || !(max_jump >= 0.0))
        return fail(RIR_E_INVALID, "rir_sdf_mesh: min_weight must be finite and max_jump >= 0");
    SdfExtractArgs a{};
    a.vox = voxels;
    a.nbx = vol->nbx;
    a.nby = vol->nby;
    a.nbz = vol->nbz;
    a.min_weight = (float)min_weight;
    if ((double)a.min_weight < min_weight)
        a.min_weight = std::nextafter(a.min_weight, std::numeric_limits<float>::infinity());
    a.max_jump = max_jump;
    for (int i = 0; i < 3; ++i)
        a.origin[i] = vol->origin[i];
    a.voxel = vol->voxel;
    a.pts = triangles;
    a.max_pts = max_triangles;
    a.count = reinterpret_cast<unsigned long long *>(count);
    HIP_TRY(launch_sdf_mesh(a, false, static_cast<hipStream_t>(stream)));
    return RIR_OK;
}

// ============================================================================ sparse SDF volume

struct rir_bvol {
    int device = 0;
    double origin[3] = {0.0, 0.0, 0.0};
    double voxel = 0.0;
    int max_blocks = 0;
    uint32_t cap = 0;       // hash table entries (power of two, >= 2 max_blocks)
    void *dmem = nullptr;
    BvolDev t{};
    int *d_nbr = nullptr;   // [max_blocks][kNbrPerBlock]
    float *d_vox = nullptr; // [max_blocks][4096][2]
    int64_t n_blocks = 0;   // host copies
    int64_t n_frames = 0;
    ~rir_bvol()
    {
        if (dmem) {
            hipSetDevice(device);
            hipFree(dmem);
        }
    }
};

constexpr size_t kBvolBlockBytes = (size_t)kSdfEdge * kSdfEdge * kSdfEdge * 2 * sizeof(float);

// Clears the table, the counters and the voxels of the first `used` slots.
static rir_status bvol_clear(rir_bvol *v, int64_t used, hipStream_t st)
{
    HIP_TRY(hipMemsetAsync(v->t.keys, 0xff, (size_t)v->cap * sizeof(unsigned long long), st));
    HIP_TRY(hipMemsetAsync(v->t.vals, 0xff, (size_t)v->cap * sizeof(int), st));
    HIP_TRY(hipMemsetAsync(v->t.act, 0x7f, (size_t)v->cap * sizeof(int), st));  // 0x7f7f7f7f: never
    HIP_TRY(hipMemsetAsync(v->t.count, 0, 2 * sizeof(int), st));
    if (used > 0)
        HIP_TRY(hipMemsetAsync(v->d_vox, 0, (size_t)used * kBvolBlockBytes, st));
    v->n_blocks = 0;
    v->n_frames = 0;
    return RIR_OK;
}

extern "C" rir_status rir_bvol_create(int device, const double origin[3], double voxel, int32_t max_blocks,
                                      rir_bvol **out)
{
    if (!out || !origin)
        return fail(RIR_E_INVALID, "rir_bvol_create: null argument");
    *out = nullptr;
    if (!(voxel > 0.0) || !std::isfinite(voxel))
        return fail(RIR_E_INVALID, "rir_bvol_create: voxel size must be finite and > 0");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(origin[i]))
            return fail(RIR_E_INVALID, "rir_bvol_create: origin must be finite");
    if (max_blocks < 1 || max_blocks > (1 << 26))
        return fail(RIR_E_INVALID, "rir_bvol_create: max_blocks must be in 1..2^26");
    HIP_TRY(hipSetDevice(device));
    std::unique_ptr<rir_bvol> v(new rir_bvol());
    v->device = device;
    for (int i = 0; i < 3; ++i)
        v->origin[i] = origin[i];
    v->voxel = voxel;
    v->max_blocks = max_blocks;
    v->cap = 1;
    while (v->cap < 2u * (uint32_t)max_blocks)
        v->cap <<= 1;
    Layout lay;
    const size_t o_keys = lay.add((size_t)v->cap * sizeof(unsigned long long));
    const size_t o_vals = lay.add((size_t)v->cap * sizeof(int));
    const size_t o_act = lay.add((size_t)v->cap * sizeof(int));
    const size_t o_blocks = lay.add((size_t)max_blocks * sizeof(int4));
    const size_t o_nbr = lay.add((size_t)max_blocks * kNbrPerBlock * sizeof(int));
    const size_t o_ctr = lay.add(2 * sizeof(int));
    const size_t o_vox = lay.add((size_t)max_blocks * kBvolBlockBytes);
    HIP_TRY(hipMalloc(&v->dmem, lay.bytes));
    char *base = static_cast<char *>(v->dmem);
    v->t.keys = reinterpret_cast<unsigned long long *>(base + o_keys);
    v->t.vals = reinterpret_cast<int *>(base + o_vals);
    v->t.act = reinterpret_cast<int *>(base + o_act);
    v->t.blocks = reinterpret_cast<int4 *>(base + o_blocks);
    v->t.count = reinterpret_cast<int *>(base + o_ctr);
    v->t.flags = v->t.count + 1;
    v->t.mask = v->cap - 1;
    v->t.max_blocks = max_blocks;
    v->d_nbr = reinterpret_cast<int *>(base + o_nbr);
    v->d_vox = reinterpret_cast<float *>(base + o_vox);
    rir_status s = bvol_clear(v.get(), max_blocks, nullptr);
    if (s != RIR_OK)
        return s;
    HIP_TRY(hipDeviceSynchronize());
    *out = v.release();
    return RIR_OK;
}

extern "C" void rir_bvol_destroy(rir_bvol *vol) { delete vol; }

extern "C" rir_status rir_bvol_reset(rir_bvol *vol, void *stream)
{
    if (!vol)
        return fail(RIR_E_INVALID, "rir_bvol_reset: null argument");
    HIP_TRY(hipSetDevice(vol->device));
    return bvol_clear(vol, vol->n_blocks, static_cast<hipStream_t>(stream));
}

extern "C" rir_status rir_bvol_integrate(rir_bvol *vol, const rir_sensor *sensor, int32_t n_frames,
                                         const float *ranges, const double *poses, double trunc, double r_clip,
                                         double radius, void *stream)
{
    if (!vol || !sensor)
        return fail(RIR_E_INVALID, "rir_bvol_integrate: null argument");
    if (n_frames < 0)
        return fail(RIR_E_INVALID, "rir_bvol_integrate: n_frames < 0");
    if (n_frames > 0 && (!ranges || !poses))
        return fail(RIR_E_INVALID, "rir_bvol_integrate: null argument");
    if (!std::isfinite(trunc) || !std::isfinite(r_clip))
        return fail(RIR_E_INVALID, "rir_bvol_integrate: trunc and r_clip must be finite");
    if (!(radius >= 0.0) || !(radius <= 64.0 * vol->voxel))
        return fail(RIR_E_INVALID, "rir_bvol_integrate: radius must be in 0 .. 64 voxels");
    if (sensor->device != vol->device)
        return fail(RIR_E_INVALID, "rir_bvol_integrate: sensor and volume on different devices");
    for (int64_t i = 0; i < 16 * (int64_t)n_frames; ++i)
        if (!std::isfinite(poses[i]))
            return fail(RIR_E_INVALID, "rir_bvol_integrate: non-finite pose");
    const int64_t hw = (int64_t)sensor->H * sensor->W;
    if (hw * (int64_t)sizeof(float) * kSdfFrames >= ((int64_t)1 << 31))
        return fail(RIR_E_SHAPE, "rir_bvol_integrate: range images too large for one launch");
    if (vol->n_frames + n_frames > (int64_t)std::numeric_limits<int32_t>::max() / 2)
        return fail(RIR_E_SHAPE, "rir_bvol_integrate: too many scans in the volume's history");
    if (n_frames == 0)
        return RIR_OK;
    HIP_TRY(hipSetDevice(vol->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    // activation of every scan of the call, each entry keeping its first scan
    BvolActArgs b{};
    b.tab = sensor->d_td;
    b.H = sensor->H;
    b.W = sensor->W;
    for (int i = 0; i < 3; ++i)
        b.origin[i] = vol->origin[i];
    b.radius = radius;
    b.clip = r_clip;
    b.edge = (double)kSdfEdge * vol->voxel;
    b.t = vol->t;
    for (int32_t f0 = 0; f0 < n_frames; f0 += kSdfFrames) {
        const int k = std::min<int32_t>(kSdfFrames, n_frames - f0);
        b.n_frames = k;
        b.frame0 = (int)(vol->n_frames + f0);
        b.ranges = ranges + (size_t)f0 * (size_t)hw;
        sdf_frames(poses + 16 * (size_t)f0, k, b.f);
        HIP_TRY(launch_bvol_activate(b, st));
    }
    int ctr[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(ctr, vol->t.count, sizeof(ctr), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    vol->n_blocks = std::min<int64_t>(ctr[0], vol->max_blocks);
    if (ctr[1] & kBvolFull)
        return fail(RIR_E_OOM, "rir_bvol_integrate: more active blocks than max_blocks (reset the volume)");
    if (ctr[1] & kBvolRange)
        return fail(RIR_E_OOM, "rir_bvol_integrate: a return beyond the block coordinate range (reset the volume)");
    // fusion of every active block; scan j of a launch skips the blocks
    // activated after it
    SdfArgs a{};
    sdf_common_args(sensor, trunc, r_clip, a);
    a.vox = vol->d_vox;
    for (int i = 0; i < 3; ++i)
        a.origin[i] = vol->origin[i];
    a.voxel = vol->voxel;
    a.blocks = vol->t.blocks;
    a.act = vol->t.act;
    a.n_blocks = (int)vol->n_blocks;
    const bool r0 = sensor->r0 > 0.0;
    const bool pow2 = (sensor->W & (sensor->W - 1)) == 0;
    for (int32_t f0 = 0; f0 < n_frames; f0 += kSdfFrames) {
        const int k = std::min<int32_t>(kSdfFrames, n_frames - f0);
        a.n_frames = k;
        a.frame0 = (int)(vol->n_frames + f0);
        a.ranges = ranges + (size_t)f0 * (size_t)hw;
        sdf_frames(poses + 16 * (size_t)f0, k, a.f);
        HIP_TRY(launch_sdf_fuse(a, r0, pow2, true, st));
    }
    vol->n_frames += n_frames;
    return RIR_OK;
}

extern "C" rir_status rir_bvol_size(const rir_bvol *vol, int64_t *n_blocks, int64_t *n_frames)
{
    if (!vol)
        return fail(RIR_E_INVALID, "rir_bvol_size: null argument");
    if (n_blocks)
        *n_blocks = vol->n_blocks;
    if (n_frames)
        *n_frames = vol->n_frames;
    return RIR_OK;
}

extern "C" rir_status rir_bvol_export(const rir_bvol *vol, int32_t *blocks, float *voxels, void *stream)
{
    if (!vol)
        return fail(RIR_E_INVALID, "rir_bvol_export: null argument");
    HIP_TRY(hipSetDevice(vol->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (blocks)
        HIP_TRY(launch_bvol_export(vol->t, (int)vol->n_blocks, reinterpret_cast<int4 *>(blocks), st));
    if (voxels && vol->n_blocks > 0)
        HIP_TRY(hipMemcpyAsync(voxels, vol->d_vox, (size_t)vol->n_blocks * kBvolBlockBytes, hipMemcpyDeviceToDevice,
                               st));
    return RIR_OK;
}

extern "C" rir_status rir_bvol_extract(rir_bvol *vol, double min_weight, double max_jump, float *points,
                                       int64_t max_points, uint64_t *count, void *stream)
{
    if (!vol || !count || (max_points > 0 && !points))
        return fail(RIR_E_INVALID, "rir_bvol_extract: null argument");
    if (max_points < 0)
        return fail(RIR_E_INVALID, "rir_bvol_extract: max_points < 0");
    if (!std::isfinite(min_weight) || std::isnan(max_jump) || !(max_jump >= 0.0))
        return fail(RIR_E_INVALID, "rir_bvol_extract: min_weight must be finite and max_jump >= 0");
    HIP_TRY(hipSetDevice(vol->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_bvol_neighbors(vol->t, (int)vol->n_blocks, vol->d_nbr, st));
    SdfExtractArgs a{};
    a.vox = vol->d_vox;
    a.min_weight = (float)min_weight;
    if ((double)a.min_weight < min_weight)
        a.min_weight = std::nextafter(a.min_weight, std::numeric_limits<float>::infinity());
    a.max_jump = max_jump;
    for (int i = 0; i < 3; ++i)
        a.origin[i] = vol->origin[i];
    a.voxel = vol->voxel;
    a.pts = points;
    a.max_pts = max_points;
    a.count = reinterpret_cast<unsigned long long *>(count);
    a.blocks = vol->t.blocks;
    a.nbr = vol->d_nbr;
    a.n_blocks = (int)vol->n_blocks;
    HIP_TRY(launch_sdf_extract(a, true, st));
    return RIR_OK;
}

extern "C" rir_status rir_bvol_mesh(rir_bvol *vol, double min_weight, double max_jump, float *triangles,
                                    int64_t max_triangles, uint64_t *count, void *stream)
{
    if (!vol || !count || (max_triangles > 0 && !triangles))
        return fail(RIR_E_INVALID, "rir_bvol_mesh: null argument");
    if (max_triangles < 0)
        return fail(RIR_E_INVALID, "rir_bvol_mesh: max_triangles < 0");
    if (!std::isfinite(min_weight) || std::isnan(max_jump) || !(max_jump >= 0.0))
        return fail(RIR_E_INVALID, "rir_bvol_mesh: min_weight must be finite and max_jump >= 0");
    HIP_TRY(hipSetDevice(vol->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_bvol_neighbors(vol->t, (int)vol->n_blocks, vol->d_nbr, st));
    SdfExtractArgs a{};
    a.vox = vol->d_vox;
    a.min_weight = (float)min_weight;
    if ((double)a.min_weight < min_weight)
        a.min_weight = std::nextafter(a.min_weight, std::numeric_limits<float>::infinity());
    a.max_jump = max_jump;
    for (int i = 0; i < 3; ++i)
        a.origin[i] = vol->origin[i];
    a.voxel = vol->voxel;
    a.pts = triangles;
    a.max_pts = max_triangles;
    a.count = reinterpret_cast<unsigned long long *>(count);
    a.blocks = vol->t.blocks;
    a.nbr = vol->d_nbr;
    a.n_blocks = (int)vol->n_blocks;
    HIP_TRY(launch_sdf_mesh(a, true, st));
    return RIR_OK;
}

// ============================================================================ learned-weight network API

extern "C" rir_status rir_mlp_create(int device, const uint16_t *w_bf16, const float *b_f32, rir_mlp **out)
{
    if (!w_bf16 || !b_f32 || !out)
        return fail(RIR_E_INVALID, "rir_mlp_create: null argument");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n)
        return fail(RIR_E_INVALID, "rir_mlp_create: no such device");
    HIP_TRY(hipSetDevice(device));
    std::unique_ptr<rir_mlp> m(new rir_mlp());
    m->device = device;
    Layout lay;
    size_t o_w = lay.add(kMlpNW * 2), o_b = lay.add(kMlpNB * 4), o_ms = lay.add(kMlpNW * 4);
    size_t o_m1 = lay.add(5185 * 4), o_m2 = lay.add(5185 * 4);
    HIP_TRY(hipMalloc(&m->dmem, lay.bytes));
    char *base = static_cast<char *>(m->dmem);
    m->w = reinterpret_cast<uint16_t *>(base + o_w);
    m->b = reinterpret_cast<float *>(base + o_b);
    m->master = reinterpret_cast<float *>(base + o_ms);
    m->m1 = reinterpret_cast<float *>(base + o_m1);
    m->m2 = reinterpret_cast<float *>(base + o_m2);
    HIP_TRY(hipMemset(m->dmem, 0, lay.bytes));
    rir_status s = rir_mlp_set_params(m.get(), w_bf16, b_f32);
    if (s != RIR_OK)
        return s;
    *out = m.release();
    return RIR_OK;
}

extern "C" void rir_mlp_destroy(rir_mlp *mlp) { delete mlp; }

extern "C" rir_status rir_mlp_set_params(rir_mlp *m, const uint16_t *w_bf16, const float *b_f32)
{
    if (!m || !w_bf16 || !b_f32)
        return fail(RIR_E_INVALID, "rir_mlp_set_params: null argument");
    HIP_TRY(hipSetDevice(m->device));
    std::vector<float> master(kMlpNW);
    for (int i = 0; i < kMlpNW; ++i) {
        uint32_t bits = (uint32_t)w_bf16[i] << 16;
        std::memcpy(&master[i], &bits, 4);
    }
    HIP_TRY(hipMemcpy(m->w, w_bf16, kMlpNW * 2, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->b, b_f32, kMlpNB * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->master, master.data(), kMlpNW * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(m->m1, 0, 5185 * 4));
    HIP_TRY(hipMemset(m->m2, 0, 5185 * 4));
    m->step = 0;
    return RIR_OK;
}

extern "C" rir_status rir_mlp_get_params(const rir_mlp *m, uint16_t *w_bf16, float *b_f32, float *master)
{
    if (!m || !w_bf16 || !b_f32)
        return fail(RIR_E_INVALID, "rir_mlp_get_params: null argument");
    HIP_TRY(hipSetDevice(m->device));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(w_bf16, m->w, kMlpNW * 2, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(b_f32, m->b, kMlpNB * 4, hipMemcpyDeviceToHost));
    if (master)
        HIP_TRY(hipMemcpy(master, m->master, kMlpNW * 4, hipMemcpyDeviceToHost));
    return RIR_OK;
}

extern "C" rir_status rir_mlp_forward(const rir_mlp *m, const float *feats, int64_t B, float *w_out, void *stream)
{
    if (!m || (B > 0 && (!feats || !w_out)))
        return fail(RIR_E_INVALID, "rir_mlp_forward: null argument");
    if (B < 0)
        return fail(RIR_E_INVALID, "rir_mlp_forward: B < 0");
    if (B == 0)
        return RIR_OK;
    HIP_TRY(hipSetDevice(m->device));
    HIP_TRY(launch_mlp_forward(m->dev(), feats, B, w_out, static_cast<hipStream_t>(stream)));
    return RIR_OK;
}

extern "C" rir_status rir_mlp_train_step(rir_mlp *m, const float *feats, const float *labels, int64_t B, float lr,
                                         float *loss_out, float *grads_out, void *stream)
{
    if (!m || !feats || !labels)
        return fail(RIR_E_INVALID, "rir_mlp_train_step: null argument");
    if (B < 1 || B > (1LL << 30))
        return fail(RIR_E_INVALID, "rir_mlp_train_step: B must be in 1..2^30");
    if (!(lr >= 0.f) || !std::isfinite(lr))
        return fail(RIR_E_INVALID, "rir_mlp_train_step: lr must be finite and >= 0");
    HIP_TRY(hipSetDevice(m->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nb = mlp_grad_blocks(B);
    if (nb > m->gpart_blocks) {
        HIP_TRY(hipStreamSynchronize(st));
        if (m->gpart)
            HIP_TRY(hipFree(m->gpart));
        m->gpart = nullptr;
        HIP_TRY(hipMalloc(reinterpret_cast<void **>(&m->gpart), (size_t)nb * kMlpGradRecord * sizeof(float)));
        m->gpart_blocks = nb;
    }
    HIP_TRY(launch_mlp_grad(m->dev(), feats, labels, B, m->gpart, nb, st));
    m->step += 1;
    HIP_TRY(launch_mlp_adam(m->gpart, nb, B, lr, m->step, m->master, m->b, m->m1, m->m2, m->w, loss_out, grads_out,
                            st));
    return RIR_OK;
}

extern "C" rir_status rir_mlp_train_step_noalloc(rir_mlp *m, const float *feats, const float *labels, int64_t B,
                                                 float lr, float *loss_out, float *grads_out, void *stream)
{
    if (!m || !feats || !labels)
        return fail(RIR_E_INVALID, "rir_mlp_train_step_noalloc: null argument");
    if (B < 1 || B > kMlpScratchMaxB)
        return fail(RIR_E_INVALID, "rir_mlp_train_step_noalloc: B must be in 1..32768 (the gradient records of "
                                   "larger batches do not fit the library's fixed scratch array)");
    if (!(lr >= 0.f) || !std::isfinite(lr))
        return fail(RIR_E_INVALID, "rir_mlp_train_step_noalloc: lr must be finite and >= 0");
    HIP_TRY(hipSetDevice(m->device));
    float *recs = nullptr;
    HIP_TRY(mlp_scratch(m->device, &recs));
    hipStream_t st = static_cast<hipStream_t>(stream);
    // every record is written in full by the gradient kernel before the Adam
    // kernel reads it: nothing in the array needs clearing
    const int nb = mlp_grad_blocks(B);
    HIP_TRY(launch_mlp_grad(m->dev(), feats, labels, B, recs, nb, st));
    m->step += 1;
    HIP_TRY(launch_mlp_adam(recs, nb, B, lr, m->step, m->master, m->b, m->m1, m->m2, m->w, loss_out, grads_out, st));
    return RIR_OK;
}

extern "C" const char *rir_last_error(void) { return g_err.c_str(); }

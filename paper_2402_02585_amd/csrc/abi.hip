// C ABI of libgqaoa (include/gqaoa.h): argument validation, error reporting
// and dispatch to the kernel launchers. Every check runs before the first HIP
// call, so an invalid call returns without touching the device.
#include "internal.h"
#include "stream_pool.h"
#include "tune_cache.h"

#include <cmath>

#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

namespace gqaoa {

// launchers (cost_table.hip, sv.hip, hist.hip, mlp.hip)
int launch_cost_table(int n, int m, const int32_t *lits, uint8_t *cost, uint64_t *hist, hipStream_t st);
int launch_cost_table_noalloc(int n, int m, const int32_t *lits, uint8_t *cost, uint64_t *hist, hipStream_t st);
uint64_t batched_cost_offset(int i, const int32_t *n_host);
int launch_hist_batched(int num_inst, const int32_t *n_host, const int32_t *m_host, const int32_t *lits,
                        uint64_t *hists, int hist_stride, uint8_t *costs, hipStream_t st);
size_t sv_workspace_bytes(int num_inst, int n, int p, int dtype, int ckpt_every, bool grad);
int run_evolve(int n, int m, const uint8_t *cost, int p, const double *beta, const double *gamma, int dtype,
               int init_uniform, void *psi, int target, double *psol, double *energy, double *norm, void *ws,
               hipStream_t st);
int run_solution_prob(int n, const uint8_t *cost, const void *psi, int dtype, int target, double *out, void *ws,
                      hipStream_t st);
int run_grad(int num_inst, int n, const int32_t *m_of, const uint8_t *cost, int p, const double *beta,
             const double *gamma, int dtype, const int32_t *targets, int ckpt_every, double *psol, double *dbeta,
             double *dgamma, void *ws, hipStream_t st);
int run_hist_evolve(int n, int m, const uint64_t *hist, int p, const double *beta, const double *gamma,
                    int target, double *psol, double *energy, double *norm, hipStream_t st);
int run_row_best(int rows, int cols, const void *x, int mode, int32_t *idx, void *val, hipStream_t st);
size_t level_probs_workspace_bytes(int n);
int run_level_probs(int n, const uint8_t *cost, const void *psi, int dtype, int level, int64_t max_out,
                    int64_t *z_out, double *p_out, int64_t *count, void *ws, hipStream_t st);
int run_mlp_angles(int batch, const float *out, double *beta, double *gamma, hipStream_t st);
int run_gather_rows(int rows, const int32_t *idx, int src_rows, const void *src, int row_bytes, void *dst,
                    hipStream_t st);
size_t hist_grad_workspace_bytes(int num_inst, int hist_stride, int pstride);
int run_hist_grad(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists,
                  int hist_stride, const int32_t *target_host, int pstride, const int32_t *p_host,
                  const double *beta, const double *gamma, double *psol, double *dbeta, double *dgamma,
                  void *ws, hipStream_t st);
size_t scan_workspace_bytes(int num_inst, int hist_stride, int nb, int ng, int num_p, int per_inst);
int scan_max_levels();
int run_scan(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists, int hist_stride,
             const int32_t *target_host, int nb, const double *betas, int ng, const double *gammas, int per_inst,
             int num_p, const int32_t *p_list, float *psol, float *energy, float threshold, int32_t *first_p,
             const int32_t *pmax_host, const int32_t *tile, void *ws, hipStream_t st);
size_t x_workspace_bytes(int n, int p, int dtype);
struct EvolvePlan;
int evolve_plan_create(int n, int m, const uint8_t *cost, int p, int dtype, int init_uniform, void *psi, int target,
                       void *ws, hipStream_t st, EvolvePlan **out);
int evolve_plan_run(EvolvePlan *E, const double *beta, const double *gamma, double *psol, double *energy,
                    double *norm, hipStream_t st);
void evolve_plan_destroy(EvolvePlan *E);
struct ScanPlan;
int scan_plan_create(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists,
                     int hist_stride, const int32_t *target_host, int nb, const double *betas, int ng,
                     const double *gammas, int per_inst, int num_p, const int32_t *p_list, float *psol,
                     float *energy, const int32_t *tile, int num_items, const int32_t *items,
                     const uint8_t *costs, const uint64_t *cost_off, float *item_psol, float *item_energy,
                     hipStream_t st, ScanPlan **out);
int scan_plan_run(ScanPlan *P, const double *betas, const double *gammas, hipStream_t st);
void scan_plan_destroy(ScanPlan *P);
int run_sv_items(int num_inst, const int32_t *n_host, const int32_t *m_host, const int32_t *target_host,
                 const uint8_t *costs, int num_items, const int32_t *item_inst, const double *beta,
                 const double *gamma, int num_p, const int32_t *p_list, float *psol, float *energy, hipStream_t st);
int run_evolve_x(int n, const uint8_t *cost, int p, const double *beta, const double *gamma, int dtype,
                 int init_uniform, void *psi, int target, double *psol, double *energy, double *norm, void *ws,
                 hipStream_t st);
int run_shots_to_all(int K, const double *p, int runs, uint64_t seed, int max_shots, int32_t *out, hipStream_t st);
int run_draws_to_reject(int K, const double *q, int trials, uint64_t seed, double crit, int n_min, int max_draws,
                        int32_t *out, hipStream_t st);
size_t mlp_act_bytes(int batch);
size_t mlp_infer_bytes(int batch);
int run_mlp_infer(const float *prm, int batch, const float *x, float *out, void *ws, hipStream_t st);
int run_mlp_forward(const float *prm, int batch, const float *x, float *out, void *act, hipStream_t st);
int run_mlp_backward(const float *prm, int batch, const void *act, const float *dout, float *grads,
                     hipStream_t st);
int run_mlp_adam(float *prm, const float *grads, float *state, int step, float lr, float b1, float b2, float eps,
                 hipStream_t st);
int run_mlp_loss(int batch, const float *out, const float *tgt, float *dout, float *loss, hipStream_t st);
int run_mlp_features(int batch, const uint64_t *hists, int hist_stride, const int32_t *n, const int32_t *m,
                     const int32_t *p, float *x, hipStream_t st);

// ---- errors ----------------------------------------------------------------------------
static thread_local char g_err[512] = {0};

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}
void clear_error() { g_err[0] = 0; }
int fail(int status, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return status;
}

// ---- instrumentation -----------------------------------------------------------------------
struct ProfPending {
    const char *name;
    hipEvent_t e0, e1;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static int g_prof_every = 1;  // time one launch in this many, per name
static std::vector<ProfPending> g_prof_pending;
struct ProfTotal {
    double ms = 0.0;
    int64_t count = 0;
};
static const char *kProfNames[] = {"sv_round_c64", "sv_round_c128", "sv_reverse_c64", "sv_reverse_c128",
                                   "cost_table", "scan", "x_pass_c64", "x_pass_c128",
                                   "sv_resident_c64", "sv_resident_c128"};
static ProfTotal g_prof_tot[sizeof(kProfNames) / sizeof(kProfNames[0])];
static int64_t g_prof_seen[sizeof(kProfNames) / sizeof(kProfNames[0])];  // launches seen while enabled

bool prof_on() { return g_prof_on; }

ProfScope::ProfScope(const char *name, hipStream_t st) : name_(name), st_(st) {
    if (!g_prof_on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;  // no event nodes in captured graphs
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        bool sample = true;
        for (size_t i = 0; i < sizeof(kProfNames) / sizeof(kProfNames[0]); ++i)
            if (!strcmp(kProfNames[i], name)) sample = (g_prof_seen[i]++ % g_prof_every) == 0;
        if (!sample) return;
    }
    if (hipEventCreate(&e0_) != hipSuccess) { e0_ = nullptr; return; }
    if (hipEventRecord(e0_, st_) != hipSuccess) { (void)hipEventDestroy(e0_); e0_ = nullptr; }
}

void ProfScope::end() {
    if (!e0_) return;
    hipEvent_t e1;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0_); e0_ = nullptr; return; }
    (void)hipEventRecord(e1, st_);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back(ProfPending{name_, e0_, e1});
    e0_ = nullptr;
}

void prof_collect() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &p : g_prof_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.e1) == hipSuccess && hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
            for (size_t i = 0; i < sizeof(kProfNames) / sizeof(kProfNames[0]); ++i)
                if (!strcmp(kProfNames[i], p.name)) {
                    g_prof_tot[i].ms += ms;
                    g_prof_tot[i].count += 1;
                }
        }
        (void)hipEventDestroy(p.e0);
        (void)hipEventDestroy(p.e1);
    }
    g_prof_pending.clear();
}

// ---- device properties -------------------------------------------------------------------
static std::mutex g_dev_mu;
static std::vector<DeviceInfo> g_devs;

int device_info(DeviceInfo *out) {
    int dev = -1;
    GQ_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_dev_mu);
    for (auto &d : g_devs)
        if (d.device == dev) {
            *out = d;
            return GQAOA_OK;
        }
    hipDeviceProp_t prop;
    GQ_HIP(hipGetDeviceProperties(&prop, dev));
    DeviceInfo d;
    d.device = dev;
    d.num_cus = prop.multiProcessorCount;
    d.lds_per_block = prop.sharedMemPerBlock;
    strncpy(d.arch, prop.gcnArchName, sizeof(d.arch) - 1);
    if (strncmp(d.arch, "gfx950", 6) != 0)
        return fail(GQAOA_ENODEV, "device %d is %s; this library is built for gfx950", dev, d.arch);
    g_devs.push_back(d);
    *out = d;
    return GQAOA_OK;
}

// ---- streams lent to graph captures ---------------------------------------------------------
static std::mutex g_pool_mu;
static std::vector<std::pair<int, hipStream_t>> g_pool;  // (device, stream), free for the taking

int stream_pool_take(size_t n, std::vector<hipStream_t> *out) {
    int dev = -1;
    GQ_HIP(hipGetDevice(&dev));
    size_t got = 0;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        for (size_t i = g_pool.size(); i-- > 0 && got < n;)
            if (g_pool[i].first == dev) {
                out->push_back(g_pool[i].second);
                g_pool.erase(g_pool.begin() + (ptrdiff_t)i);
                ++got;
            }
    }
    for (; got < n; ++got) {
        hipStream_t s = nullptr;
        GQ_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        out->push_back(s);
    }
    return GQAOA_OK;
}

void stream_pool_give(int device, const std::vector<hipStream_t> &streams) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (hipStream_t s : streams)
        if (s) g_pool.emplace_back(device, s);
}

// ---- validation helpers ------------------------------------------------------------------
static int check_clauses(int n, int m, const int32_t *lits, int inst) {
    for (int i = 0; i < m; ++i) {
        int v[3];
        for (int j = 0; j < 3; ++j) {
            const int32_t lit = lits[3 * i + j];
            if (lit < 0 || lit >= 2 * n)
                return fail(GQAOA_EINVAL, "instance %d clause %d: literal %d outside [0, %d)", inst, i, lit, 2 * n);
            v[j] = lit >> 1;
        }
        if (v[0] == v[1] || v[0] == v[2] || v[1] == v[2])
            return fail(GQAOA_EINVAL, "instance %d clause %d repeats a variable", inst, i);
    }
    return GQAOA_OK;
}

static bool dtype_ok(int dt) { return dt == GQAOA_C64 || dt == GQAOA_C128; }
constexpr int kMaxP = 100000;

}  // namespace gqaoa

using namespace gqaoa;

extern "C" {

const char *gqaoa_status_string(int status) {
    switch (status) {
        case GQAOA_OK: return "ok";
        case GQAOA_EINVAL: return "invalid argument";
        case GQAOA_ERANGE: return "argument out of range";
        case GQAOA_EWORKSPACE: return "workspace too small";
        case GQAOA_EHIP: return "HIP runtime error";
        case GQAOA_ENODEV: return "no gfx950 device";
        default: return "unknown status";
    }
}

const char *gqaoa_last_error(void) { return g_err; }

int gqaoa_abi_version(void) { return 1; }

int gqaoa_cost_table(int n, int m, const int32_t *lits_host, uint8_t *cost_dev, uint64_t *hist_dev,
                     void *stream) {
    clear_error();
    if (n < GQAOA_MIN_N || n > GQAOA_MAX_N) return fail(GQAOA_ERANGE, "n=%d outside [3, 34]", n);
    if (m < 1 || m > GQAOA_MAX_M) return fail(GQAOA_ERANGE, "m=%d outside [1, 255]", m);
    if (!lits_host || !cost_dev) return fail(GQAOA_EINVAL, "NULL lits_host or cost_dev");
    int s = check_clauses(n, m, lits_host, 0);
    if (s) return s;
    return launch_cost_table(n, m, lits_host, cost_dev, hist_dev, (hipStream_t)stream);
}

int gqaoa_cost_table_noalloc(int n, int m, const int32_t *lits_host, uint8_t *cost_dev, uint64_t *hist_dev,
                             void *stream) {
    clear_error();
    if (n < GQAOA_MIN_N || n > GQAOA_MAX_N) return fail(GQAOA_ERANGE, "n=%d outside [3, 34]", n);
    if (m < 1 || m > GQAOA_MAX_M) return fail(GQAOA_ERANGE, "m=%d outside [1, 255]", m);
    if (!lits_host || !cost_dev) return fail(GQAOA_EINVAL, "NULL lits_host or cost_dev");
    int s = check_clauses(n, m, lits_host, 0);
    if (s) return s;
    return launch_cost_table_noalloc(n, m, lits_host, cost_dev, hist_dev, (hipStream_t)stream);
}

static int check_batched_instances(int num_inst, const int32_t *n_host, const int32_t *m_host,
                                   const int32_t *lits_host, int hist_stride, int max_n) {
    if (num_inst < 1 || num_inst > (1 << 20)) return fail(GQAOA_ERANGE, "num_inst=%d outside [1, 2^20]", num_inst);
    if (!n_host || !m_host || !lits_host) return fail(GQAOA_EINVAL, "NULL argument");
    if (hist_stride < 2 || hist_stride > 4096) return fail(GQAOA_ERANGE, "hist_stride=%d", hist_stride);
    size_t off = 0;
    for (int i = 0; i < num_inst; ++i) {
        if (n_host[i] < GQAOA_MIN_N || n_host[i] > max_n)
            return fail(GQAOA_ERANGE, "instance %d: n=%d outside [3, %d]", i, n_host[i], max_n);
        if (m_host[i] < 1 || m_host[i] > GQAOA_MAX_M) return fail(GQAOA_ERANGE, "instance %d: m=%d", i, m_host[i]);
        if (m_host[i] + 1 > hist_stride) return fail(GQAOA_ERANGE, "instance %d: m+1=%d > hist_stride", i, m_host[i] + 1);
        int s = check_clauses(n_host[i], m_host[i], lits_host + 3 * off, i);
        if (s) return s;
        off += (size_t)m_host[i];
    }
    return GQAOA_OK;
}

int gqaoa_hist_batched(int num_inst, const int32_t *n_host, const int32_t *m_host, const int32_t *lits_host,
                       uint64_t *hists_dev, int hist_stride, void *stream) {
    clear_error();
    int s = check_batched_instances(num_inst, n_host, m_host, lits_host, hist_stride, 30);
    if (s) return s;
    if (!hists_dev) return fail(GQAOA_EINVAL, "NULL hists_dev");
    return launch_hist_batched(num_inst, n_host, m_host, lits_host, hists_dev, hist_stride, nullptr,
                               (hipStream_t)stream);
}

uint64_t gqaoa_cost_batched_offset(int index, const int32_t *n_host) {
    if (index < 0 || !n_host) return 0;
    return batched_cost_offset(index, n_host);
}

int gqaoa_cost_batched(int num_inst, const int32_t *n_host, const int32_t *m_host, const int32_t *lits_host,
                       uint8_t *costs_dev, uint64_t *hists_dev, int hist_stride, void *stream) {
    clear_error();
    int s = check_batched_instances(num_inst, n_host, m_host, lits_host, hist_stride, 26);
    if (s) return s;
    if (!costs_dev) return fail(GQAOA_EINVAL, "NULL costs_dev");
    return launch_hist_batched(num_inst, n_host, m_host, lits_host, hists_dev, hist_stride, costs_dev,
                               (hipStream_t)stream);
}

size_t gqaoa_workspace_bytes(int n, int p, int dtype, int ckpt_every) {
    (void)ckpt_every;
    if (n < GQAOA_MIN_N || n > GQAOA_MAX_N || p < 0 || p > kMaxP || !dtype_ok(dtype)) return 0;
    return sv_workspace_bytes(1, n, p, dtype, 0, false);
}

int gqaoa_evolve(int n, int m, const uint8_t *cost_dev, int p, const double *beta_host, const double *gamma_host,
                 int dtype, int init_uniform, void *psi_dev, int target_level, double *psol_host,
                 double *energy_host, double *norm_host, void *ws_dev, size_t ws_bytes, void *stream) {
    clear_error();
    if (n < GQAOA_MIN_N || n > GQAOA_MAX_N) return fail(GQAOA_ERANGE, "n=%d outside [3, 34]", n);
    if (m < 1 || m > GQAOA_MAX_M) return fail(GQAOA_ERANGE, "m=%d outside [1, 255]", m);
    if (p < 0 || p > kMaxP) return fail(GQAOA_ERANGE, "p=%d outside [0, %d]", p, kMaxP);
    if (target_level < 0 || target_level > m) return fail(GQAOA_ERANGE, "target_level=%d outside [0, m]", target_level);
    if (!dtype_ok(dtype)) return fail(GQAOA_EINVAL, "dtype=%d", dtype);
    if (!cost_dev || !psi_dev || !ws_dev) return fail(GQAOA_EINVAL, "NULL cost_dev, psi_dev or ws_dev");
    if (p > 0 && (!beta_host || !gamma_host)) return fail(GQAOA_EINVAL, "NULL angles");
    const size_t need = sv_workspace_bytes(1, n, p, dtype, 0, false);
    if (ws_bytes < need) return fail(GQAOA_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    return run_evolve(n, m, cost_dev, p, beta_host, gamma_host, dtype, init_uniform, psi_dev, target_level, psol_host,
                      energy_host, norm_host, ws_dev, (hipStream_t)stream);
}

int gqaoa_evolve_plan_create(int n, int m, const uint8_t *cost_dev, int p, int dtype, int init_uniform,
                             void *psi_dev, int target_level, void *ws_dev, size_t ws_bytes, void *stream,
                             gqaoa_evolve_plan **plan_out) {
    clear_error();
    if (!plan_out) return fail(GQAOA_EINVAL, "NULL plan_out");
    *plan_out = nullptr;
    if (n < GQAOA_MIN_N || n > GQAOA_MAX_N) return fail(GQAOA_ERANGE, "n=%d outside [3, 34]", n);
    if (m < 1 || m > GQAOA_MAX_M) return fail(GQAOA_ERANGE, "m=%d outside [1, 255]", m);
    if (p < 1 || p > kMaxP) return fail(GQAOA_ERANGE, "p=%d outside [1, %d]", p, kMaxP);
    if (target_level < 0 || target_level > m) return fail(GQAOA_ERANGE, "target_level=%d outside [0, m]", target_level);
    if (!dtype_ok(dtype)) return fail(GQAOA_EINVAL, "dtype=%d", dtype);
    if (!cost_dev || !psi_dev || !ws_dev) return fail(GQAOA_EINVAL, "NULL cost_dev, psi_dev or ws_dev");
    const size_t need = sv_workspace_bytes(1, n, p, dtype, 0, false);
    if (ws_bytes < need) return fail(GQAOA_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    EvolvePlan *E = nullptr;
    int s = evolve_plan_create(n, m, cost_dev, p, dtype, init_uniform ? 1 : 0, psi_dev, target_level, ws_dev,
                               (hipStream_t)stream, &E);
    if (s) return s;
    *plan_out = reinterpret_cast<gqaoa_evolve_plan *>(E);
    return GQAOA_OK;
}

int gqaoa_evolve_plan_run(gqaoa_evolve_plan *plan, const double *beta_host, const double *gamma_host,
                          double *psol_host, double *energy_host, double *norm_host, void *stream) {
    clear_error();
    if (!plan || !beta_host || !gamma_host) return fail(GQAOA_EINVAL, "NULL plan or angles");
    return evolve_plan_run(reinterpret_cast<EvolvePlan *>(plan), beta_host, gamma_host, psol_host, energy_host,
                           norm_host, (hipStream_t)stream);
}

void gqaoa_evolve_plan_destroy(gqaoa_evolve_plan *plan) { evolve_plan_destroy(reinterpret_cast<EvolvePlan *>(plan)); }

size_t gqaoa_x_workspace_bytes(int n, int p, int dtype) {
    if (n < GQAOA_MIN_N || n > GQAOA_MAX_N || p < 0 || p > kMaxP || !dtype_ok(dtype)) return 0;
    return x_workspace_bytes(n, p, dtype);
}

int gqaoa_evolve_x(int n, int m, const uint8_t *cost_dev, int p, const double *beta_host, const double *gamma_host,
                   int dtype, int init_uniform, void *psi_dev, int target_level, double *psol_host,
                   double *energy_host, double *norm_host, void *ws_dev, size_t ws_bytes, void *stream) {
    clear_error();
    if (n < GQAOA_MIN_N || n > GQAOA_MAX_N) return fail(GQAOA_ERANGE, "n=%d outside [3, 34]", n);
    if (m < 1 || m > GQAOA_MAX_M) return fail(GQAOA_ERANGE, "m=%d outside [1, 255]", m);
    if (p < 0 || p > kMaxP) return fail(GQAOA_ERANGE, "p=%d outside [0, %d]", p, kMaxP);
    if (target_level < 0 || target_level > m) return fail(GQAOA_ERANGE, "target_level=%d outside [0, m]", target_level);
    if (!dtype_ok(dtype)) return fail(GQAOA_EINVAL, "dtype=%d", dtype);
    if (!cost_dev || !psi_dev || !ws_dev) return fail(GQAOA_EINVAL, "NULL cost_dev, psi_dev or ws_dev");
    if (p > 0 && (!beta_host || !gamma_host)) return fail(GQAOA_EINVAL, "NULL angles");
    const size_t need = x_workspace_bytes(n, p, dtype);
    if (ws_bytes < need) return fail(GQAOA_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    return run_evolve_x(n, cost_dev, p, beta_host, gamma_host, dtype, init_uniform, psi_dev, target_level, psol_host,
                        energy_host, norm_host, ws_dev, (hipStream_t)stream);
}

int gqaoa_solution_prob(int n, const uint8_t *cost_dev, const void *psi_dev, int dtype, int target_level,
                        double *out_host, void *ws_dev, size_t ws_bytes, void *stream) {
    clear_error();
    if (n < GQAOA_MIN_N || n > GQAOA_MAX_N) return fail(GQAOA_ERANGE, "n=%d outside [3, 34]", n);
    if (target_level < 0 || target_level > GQAOA_MAX_M) return fail(GQAOA_ERANGE, "target_level=%d", target_level);
    if (!dtype_ok(dtype)) return fail(GQAOA_EINVAL, "dtype=%d", dtype);
    if (!cost_dev || !psi_dev || !out_host || !ws_dev) return fail(GQAOA_EINVAL, "NULL argument");
    const size_t need = sv_workspace_bytes(1, n, 0, dtype, 0, false);
    if (ws_bytes < need) return fail(GQAOA_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    return run_solution_prob(n, cost_dev, psi_dev, dtype, target_level, out_host, ws_dev, (hipStream_t)stream);
}

size_t gqaoa_grad_workspace_bytes(int num_inst, int n, int p, int dtype, int ckpt_every) {
    if (num_inst < 1 || n < GQAOA_MIN_N || n > GQAOA_MAX_N || p < 1 || p > kMaxP || ckpt_every < 0 ||
        !dtype_ok(dtype))
        return 0;
    return sv_workspace_bytes(num_inst, n, p, dtype, ckpt_every, true);
}

int gqaoa_grad_batched(int num_inst, int n, const int32_t *m_host, const uint8_t *cost_dev, int p,
                       const double *beta_host, const double *gamma_host, int dtype, const int32_t *target_host,
                       int ckpt_every, double *psol_host, double *dbeta_host, double *dgamma_host, void *ws_dev,
                       size_t ws_bytes, void *stream) {
    clear_error();
    if (num_inst < 1 || num_inst > 65536) return fail(GQAOA_ERANGE, "num_inst=%d outside [1, 65536]", num_inst);
    if (n < GQAOA_MIN_N || n > GQAOA_MAX_N) return fail(GQAOA_ERANGE, "n=%d outside [3, 34]", n);
    if (p < 1 || p > kMaxP) return fail(GQAOA_ERANGE, "p=%d outside [1, %d]", p, kMaxP);
    if (ckpt_every < 0) return fail(GQAOA_ERANGE, "ckpt_every=%d", ckpt_every);
    if (!dtype_ok(dtype)) return fail(GQAOA_EINVAL, "dtype=%d", dtype);
    if (!m_host || !cost_dev || !beta_host || !gamma_host || !ws_dev) return fail(GQAOA_EINVAL, "NULL argument");
    std::vector<int32_t> tg(num_inst, 0);
    for (int i = 0; i < num_inst; ++i) {
        if (m_host[i] < 1 || m_host[i] > GQAOA_MAX_M) return fail(GQAOA_ERANGE, "instance %d: m=%d", i, m_host[i]);
        if (target_host) tg[i] = target_host[i];
        if (tg[i] < 0 || tg[i] > m_host[i]) return fail(GQAOA_ERANGE, "instance %d: target_level=%d", i, tg[i]);
    }
    const size_t need = sv_workspace_bytes(num_inst, n, p, dtype, ckpt_every, true);
    if (ws_bytes < need) return fail(GQAOA_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    return run_grad(num_inst, n, m_host, cost_dev, p, beta_host, gamma_host, dtype, tg.data(), ckpt_every, psol_host,
                    dbeta_host, dgamma_host, ws_dev, (hipStream_t)stream);
}

int gqaoa_grad(int n, int m, const uint8_t *cost_dev, int p, const double *beta_host, const double *gamma_host,
               int dtype, int target_level, int ckpt_every, double *psol_host, double *dbeta_host,
               double *dgamma_host, void *ws_dev, size_t ws_bytes, void *stream) {
    const int32_t mm = m, tt = target_level;
    return gqaoa_grad_batched(1, n, &mm, cost_dev, p, beta_host, gamma_host, dtype, &tt, ckpt_every, psol_host,
                              dbeta_host, dgamma_host, ws_dev, ws_bytes, stream);
}

int gqaoa_hist_evolve(int n, int m, const uint64_t *hist_dev, int p, const double *beta_host,
                      const double *gamma_host, int target_level, double *psol_host, double *energy_host,
                      double *norm_host, void *stream) {
    clear_error();
    if (n < GQAOA_MIN_N || n > 62) return fail(GQAOA_ERANGE, "n=%d outside [3, 62]", n);
    if (m < 1 || m > GQAOA_MAX_M) return fail(GQAOA_ERANGE, "m=%d outside [1, 255]", m);
    if (p < 0 || p > kMaxP) return fail(GQAOA_ERANGE, "p=%d outside [0, %d]", p, kMaxP);
    if (target_level < 0 || target_level > m) return fail(GQAOA_ERANGE, "target_level=%d", target_level);
    if (!hist_dev) return fail(GQAOA_EINVAL, "NULL hist_dev");
    if (p > 0 && (!beta_host || !gamma_host)) return fail(GQAOA_EINVAL, "NULL angles");
    return run_hist_evolve(n, m, hist_dev, p, beta_host, gamma_host, target_level, psol_host, energy_host, norm_host,
                           (hipStream_t)stream);
}

int gqaoa_row_best(int rows, int cols, const void *x_dev, int mode, int32_t *idx_dev, void *val_dev, void *stream) {
    clear_error();
    if (rows < 1) return fail(GQAOA_ERANGE, "rows=%d", rows);
    if (cols < 1 || cols > (1 << 30)) return fail(GQAOA_ERANGE, "cols=%d outside [1, 2^30]", cols);
    if (mode < GQAOA_ROW_ARGMAX_F32 || mode > GQAOA_ROW_MIN_POSITIVE_I32) return fail(GQAOA_EINVAL, "mode=%d", mode);
    if (!x_dev || !idx_dev) return fail(GQAOA_EINVAL, "NULL argument");
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    return run_row_best(rows, cols, x_dev, mode, idx_dev, val_dev, (hipStream_t)stream);
}

size_t gqaoa_level_probs_workspace_bytes(int n) {
    if (n < GQAOA_MIN_N || n > GQAOA_MAX_N) return 0;
    return level_probs_workspace_bytes(n);
}

int gqaoa_level_probs(int n, const uint8_t *cost_dev, const void *psi_dev, int dtype, int level, int64_t max_out,
                      int64_t *z_dev, double *prob_dev, int64_t *count_host, void *ws_dev, size_t ws_bytes,
                      void *stream) {
    clear_error();
    if (n < GQAOA_MIN_N || n > GQAOA_MAX_N) return fail(GQAOA_ERANGE, "n=%d outside [3, 34]", n);
    if (level < 0 || level > GQAOA_MAX_M) return fail(GQAOA_ERANGE, "level=%d outside [0, 255]", level);
    if (max_out < 0) return fail(GQAOA_ERANGE, "max_out=%lld", (long long)max_out);
    if (!dtype_ok(dtype)) return fail(GQAOA_EINVAL, "dtype=%d", dtype);
    if (!cost_dev || !psi_dev || !count_host || !ws_dev) return fail(GQAOA_EINVAL, "NULL argument");
    const size_t need = level_probs_workspace_bytes(n);
    if (ws_bytes < need) return fail(GQAOA_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    return run_level_probs(n, cost_dev, psi_dev, dtype, level, max_out, z_dev, prob_dev, count_host, ws_dev,
                           (hipStream_t)stream);
}

int gqaoa_mlp_angles(int batch, const float *out_dev, double *beta_dev, double *gamma_dev, void *stream) {
    clear_error();
    if (batch < 1 || batch > (1 << 26)) return fail(GQAOA_ERANGE, "batch=%d", batch);
    if (!out_dev || !beta_dev || !gamma_dev) return fail(GQAOA_EINVAL, "NULL argument");
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    return run_mlp_angles(batch, out_dev, beta_dev, gamma_dev, (hipStream_t)stream);
}

int gqaoa_gather_rows(int rows, const int32_t *idx_dev, int src_rows, const void *src_dev, int row_bytes,
                      void *dst_dev, void *stream) {
    clear_error();
    if (rows < 1 || src_rows < 1) return fail(GQAOA_ERANGE, "rows=%d src_rows=%d", rows, src_rows);
    if (row_bytes < 4 || row_bytes > (1 << 20) || row_bytes % 4) return fail(GQAOA_ERANGE, "row_bytes=%d", row_bytes);
    if (!idx_dev || !src_dev || !dst_dev) return fail(GQAOA_EINVAL, "NULL argument");
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    return run_gather_rows(rows, idx_dev, src_rows, src_dev, row_bytes, dst_dev, (hipStream_t)stream);
}

size_t gqaoa_hist_grad_workspace_bytes(int num_inst, int hist_stride, int p_max) {
    if (num_inst < 1 || num_inst > (1 << 20) || hist_stride < 2 || hist_stride > 4096 || p_max < 1 || p_max > kMaxP)
        return 0;
    return hist_grad_workspace_bytes(num_inst, hist_stride, p_max);
}

int gqaoa_hist_grad_batched(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists_host,
                            int hist_stride, const int32_t *target_host, int p_max, const int32_t *p_host,
                            const double *beta_host, const double *gamma_host, double *psol_host,
                            double *dbeta_host, double *dgamma_host, void *ws_dev, size_t ws_bytes, void *stream) {
    clear_error();
    if (num_inst < 1 || num_inst > (1 << 20)) return fail(GQAOA_ERANGE, "num_inst=%d outside [1, 2^20]", num_inst);
    if (hist_stride < 2 || hist_stride > 4096) return fail(GQAOA_ERANGE, "hist_stride=%d", hist_stride);
    if (p_max < 1 || p_max > kMaxP) return fail(GQAOA_ERANGE, "p_max=%d outside [1, %d]", p_max, kMaxP);
    if (!n_host || !m_host || !hists_host || !beta_host || !gamma_host || !ws_dev)
        return fail(GQAOA_EINVAL, "NULL argument");
    for (int i = 0; i < num_inst; ++i) {
        if (n_host[i] < GQAOA_MIN_N || n_host[i] > 62) return fail(GQAOA_ERANGE, "instance %d: n=%d", i, n_host[i]);
        if (m_host[i] < 1 || m_host[i] > GQAOA_MAX_M || m_host[i] + 1 > hist_stride)
            return fail(GQAOA_ERANGE, "instance %d: m=%d", i, m_host[i]);
        const int t = target_host ? target_host[i] : 0;
        if (t < 0 || t > m_host[i]) return fail(GQAOA_ERANGE, "instance %d: target_level=%d", i, t);
        if (p_host && (p_host[i] < 1 || p_host[i] > p_max))
            return fail(GQAOA_ERANGE, "instance %d: p=%d outside [1, %d]", i, p_host[i], p_max);
    }
    const size_t need = hist_grad_workspace_bytes(num_inst, hist_stride, p_max);
    if (ws_bytes < need) return fail(GQAOA_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    return run_hist_grad(num_inst, n_host, m_host, hists_host, hist_stride, target_host, p_max, p_host, beta_host,
                         gamma_host, psol_host, dbeta_host, dgamma_host, ws_dev, (hipStream_t)stream);
}

size_t gqaoa_scan_workspace_bytes(int num_inst, int hist_stride, int nb, int ng, int num_p, int per_instance_grid) {
    if (num_inst < 1 || hist_stride < 2 || nb < 1 || ng < 1 || num_p < 1) return 0;
    return scan_workspace_bytes(num_inst, hist_stride, nb, ng, num_p, per_instance_grid ? 1 : 0);
}

// Checks shared by the two scan entry points (everything but the outputs).
static int check_scan_args(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists_host,
                           int hist_stride, const int32_t *target_host, int nb, const double *betas_host, int ng,
                           const double *gammas_host, int num_p, const int32_t *p_list_host, const int32_t *tile) {
    if (num_inst < 1 || num_inst > (1 << 20)) return fail(GQAOA_ERANGE, "num_inst=%d", num_inst);
    if (nb < 1 || nb > 4096 || ng < 1 || ng > 4096) return fail(GQAOA_ERANGE, "grid %d x %d outside [1, 4096]^2", nb, ng);
    if (num_p < 1 || num_p > 16) return fail(GQAOA_ERANGE, "num_p=%d outside [1, 16]", num_p);
    if (hist_stride < 2 || hist_stride > 4096) return fail(GQAOA_ERANGE, "hist_stride=%d", hist_stride);
    if (!n_host || !m_host || !hists_host || !betas_host || !gammas_host || !p_list_host)
        return fail(GQAOA_EINVAL, "NULL argument");
    for (int q = 0; q < num_p; ++q) {
        if (p_list_host[q] < 1 || p_list_host[q] > kMaxP) return fail(GQAOA_ERANGE, "p_list[%d]=%d", q, p_list_host[q]);
        if (q && p_list_host[q] <= p_list_host[q - 1]) return fail(GQAOA_EINVAL, "p_list is not ascending");
    }
    if (tile && !tile_valid(tile[0], tile[1]))
        return fail(GQAOA_EINVAL, "tile {%d, %d}", tile[0], tile[1]);
    const uint64_t items = (uint64_t)num_inst * ng * ((nb + 63) / 64);
    if (items >= (1ull << 31)) return fail(GQAOA_ERANGE, "too many work items (%llu)", (unsigned long long)items);
    for (int i = 0; i < num_inst; ++i) {
        if (n_host[i] < GQAOA_MIN_N || n_host[i] > 62) return fail(GQAOA_ERANGE, "instance %d: n=%d", i, n_host[i]);
        if (m_host[i] < 1 || m_host[i] > GQAOA_MAX_M || m_host[i] + 1 > hist_stride)
            return fail(GQAOA_ERANGE, "instance %d: m=%d", i, m_host[i]);
        const int t = target_host ? target_host[i] : 0;
        if (t < 0 || t > m_host[i]) return fail(GQAOA_ERANGE, "instance %d: target_level=%d", i, t);
        int K = 0;
        for (int k = 0; k <= m_host[i]; ++k) K += hists_host[(size_t)i * hist_stride + k] != 0;
        if (K > scan_max_levels()) return fail(GQAOA_ERANGE, "instance %d: %d occupied levels (max %d)", i, K, scan_max_levels());
    }
    return GQAOA_OK;
}

int gqaoa_scan_batched(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists_host,
                       int hist_stride, const int32_t *target_host, int nb, const double *betas_host, int ng,
                       const double *gammas_host, int per_instance_grid, int num_p, const int32_t *p_list_host,
                       float *psol_dev,
                       float *energy_dev, const int32_t *tile, void *ws_dev, size_t ws_bytes, void *stream) {
    clear_error();
    int s = check_scan_args(num_inst, n_host, m_host, hists_host, hist_stride, target_host, nb, betas_host, ng,
                            gammas_host, num_p, p_list_host, tile);
    if (s) return s;
    if (!psol_dev || !ws_dev) return fail(GQAOA_EINVAL, "NULL argument");
    const int pig = per_instance_grid ? 1 : 0;
    const size_t need = scan_workspace_bytes(num_inst, hist_stride, nb, ng, num_p, pig);
    if (ws_bytes < need) return fail(GQAOA_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    return run_scan(num_inst, n_host, m_host, hists_host, hist_stride, target_host, nb, betas_host, ng, gammas_host,
                    pig, num_p, p_list_host, psol_dev, energy_dev, 0.f, nullptr, nullptr, tile, ws_dev,
                    (hipStream_t)stream);
}

int gqaoa_scan_crossing(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists_host,
                        int hist_stride, const int32_t *target_host, int nb, const double *betas_host, int ng,
                        const double *gammas_host, int per_instance_grid, int p_max, const int32_t *p_max_host,
                        float threshold, int32_t *first_p_dev, const int32_t *tile, void *ws_dev, size_t ws_bytes,
                        void *stream) {
    clear_error();
    const int32_t pl[1] = {p_max};
    int s = check_scan_args(num_inst, n_host, m_host, hists_host, hist_stride, target_host, nb, betas_host, ng,
                            gammas_host, 1, pl, tile);
    if (s) return s;
    if (!ws_dev) return fail(GQAOA_EINVAL, "NULL ws_dev");
    if (p_max_host)
        for (int i = 0; i < num_inst; ++i)
            if (p_max_host[i] < 1 || p_max_host[i] > p_max)
                return fail(GQAOA_ERANGE, "instance %d: p_max=%d outside [1, %d]", i, p_max_host[i], p_max);
    if (!first_p_dev) return fail(GQAOA_EINVAL, "NULL first_p_dev");
    if (!(threshold > 0.f && threshold <= 1.f)) return fail(GQAOA_ERANGE, "threshold=%g outside (0, 1]", (double)threshold);
    const int pig = per_instance_grid ? 1 : 0;
    const size_t need = scan_workspace_bytes(num_inst, hist_stride, nb, ng, 1, pig);
    if (ws_bytes < need) return fail(GQAOA_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    return run_scan(num_inst, n_host, m_host, hists_host, hist_stride, target_host, nb, betas_host, ng, gammas_host,
                    pig, 1, pl, nullptr, nullptr, threshold, first_p_dev, p_max_host, tile, ws_dev,
                    (hipStream_t)stream);
}

int gqaoa_shots_to_all(int num_solutions, const double *p_host, int runs, uint64_t seed, int max_shots,
                       int32_t *shots_dev, void *stream) {
    clear_error();
    if (num_solutions < 1 || num_solutions > 64) return fail(GQAOA_ERANGE, "num_solutions=%d outside [1, 64]", num_solutions);
    if (runs < 1 || runs > (1 << 26)) return fail(GQAOA_ERANGE, "runs=%d", runs);
    if (max_shots < 1) return fail(GQAOA_ERANGE, "max_shots=%d", max_shots);
    if (!p_host || !shots_dev) return fail(GQAOA_EINVAL, "NULL argument");
    double tot = 0.0;
    for (int k = 0; k < num_solutions; ++k) {
        if (!(p_host[k] >= 0.0) || !std::isfinite(p_host[k])) return fail(GQAOA_EINVAL, "p[%d]=%g", k, p_host[k]);
        tot += p_host[k];
    }
    if (!(tot > 0.0) || tot > 1.0 + 1e-9) return fail(GQAOA_EINVAL, "solution probabilities sum to %g", tot);
    return run_shots_to_all(num_solutions, p_host, runs, seed, max_shots, shots_dev, (hipStream_t)stream);
}

int gqaoa_draws_to_reject(int num_solutions, const double *q_host, int trials, uint64_t seed, double crit, int n_min,
                          int max_draws, int32_t *draws_dev, void *stream) {
    clear_error();
    if (num_solutions < 2 || num_solutions > 64) return fail(GQAOA_ERANGE, "num_solutions=%d outside [2, 64]", num_solutions);
    if (trials < 1 || trials > (1 << 24)) return fail(GQAOA_ERANGE, "trials=%d", trials);
    if (max_draws < 1 || max_draws > 10000000) return fail(GQAOA_ERANGE, "max_draws=%d outside [1, 1e7]", max_draws);
    if (n_min < 1) return fail(GQAOA_ERANGE, "n_min=%d", n_min);
    if (!(crit > 0.0) || !std::isfinite(crit)) return fail(GQAOA_EINVAL, "crit=%g", crit);
    if (!q_host || !draws_dev) return fail(GQAOA_EINVAL, "NULL argument");
    double tot = 0.0;
    for (int k = 0; k < num_solutions; ++k) {
        if (!(q_host[k] >= 0.0) || !std::isfinite(q_host[k])) return fail(GQAOA_EINVAL, "q[%d]=%g", k, q_host[k]);
        tot += q_host[k];
    }
    if (!(tot > 0.0)) return fail(GQAOA_EINVAL, "solution probabilities sum to %g", tot);
    return run_draws_to_reject(num_solutions, q_host, trials, seed, crit, n_min, max_draws, draws_dev,
                               (hipStream_t)stream);
}

int gqaoa_sv_items(int num_inst, const int32_t *n_host, const int32_t *m_host, const int32_t *target_host,
                   const uint8_t *costs_dev, int num_items, const int32_t *item_inst_host, const double *beta_host,
                   const double *gamma_host, int num_p, const int32_t *p_list_host, float *psol_dev,
                   float *energy_dev, void *stream) {
    clear_error();
    if (num_inst < 1 || num_inst > (1 << 20)) return fail(GQAOA_ERANGE, "num_inst=%d", num_inst);
    if (num_items < 1 || num_items > (1 << 24)) return fail(GQAOA_ERANGE, "num_items=%d", num_items);
    if (num_p < 1 || num_p > 16) return fail(GQAOA_ERANGE, "num_p=%d outside [1, 16]", num_p);
    if (!n_host || !m_host || !costs_dev || !item_inst_host || !beta_host || !gamma_host || !p_list_host || !psol_dev)
        return fail(GQAOA_EINVAL, "NULL argument");
    for (int q = 0; q < num_p; ++q) {
        if (p_list_host[q] < 1 || p_list_host[q] > kMaxP) return fail(GQAOA_ERANGE, "p_list[%d]=%d", q, p_list_host[q]);
        if (q && p_list_host[q] <= p_list_host[q - 1]) return fail(GQAOA_EINVAL, "p_list is not ascending");
    }
    for (int i = 0; i < num_inst; ++i) {
        if (n_host[i] < GQAOA_MIN_N || n_host[i] > 26) return fail(GQAOA_ERANGE, "instance %d: n=%d", i, n_host[i]);
        if (m_host[i] < 1 || m_host[i] > GQAOA_MAX_M) return fail(GQAOA_ERANGE, "instance %d: m=%d", i, m_host[i]);
        const int t = target_host ? target_host[i] : 0;
        if (t < 0 || t > m_host[i]) return fail(GQAOA_ERANGE, "instance %d: target_level=%d", i, t);
    }
    for (int k = 0; k < num_items; ++k) {
        const int i = item_inst_host[k];
        if (i < 0 || i >= num_inst) return fail(GQAOA_ERANGE, "item %d: instance %d", k, i);
        if (!std::isfinite(beta_host[k]) || !std::isfinite(gamma_host[k])) return fail(GQAOA_EINVAL, "item %d: angles", k);
    }
    return run_sv_items(num_inst, n_host, m_host, target_host, costs_dev, num_items, item_inst_host, beta_host,
                        gamma_host, num_p, p_list_host, psol_dev, energy_dev, (hipStream_t)stream);
}

static bool all_finite(const double *v, size_t n) {
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(v[k])) return false;
    return true;
}

int gqaoa_scan_plan_create(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists_host,
                           int hist_stride, const int32_t *target_host, int nb, const double *betas_host, int ng,
                           const double *gammas_host, int per_instance_grid, int num_p, const int32_t *p_list_host,
                           float *psol_dev, float *energy_dev, const int32_t *tile, int num_items,
                           const int32_t *items_host, const uint8_t *costs_dev, const uint64_t *cost_off_host,
                           float *item_psol_dev, float *item_energy_dev, void *stream, gqaoa_scan_plan **plan_out) {
    clear_error();
    if (!plan_out) return fail(GQAOA_EINVAL, "NULL plan_out");
    *plan_out = nullptr;
    int s = check_scan_args(num_inst, n_host, m_host, hists_host, hist_stride, target_host, nb, betas_host, ng,
                            gammas_host, num_p, p_list_host, tile);
    if (s) return s;
    if (!psol_dev) return fail(GQAOA_EINVAL, "NULL psol_dev");
    const int pig = per_instance_grid ? 1 : 0;
    const size_t ga = pig ? (size_t)num_inst : 1;
    if (!all_finite(betas_host, (size_t)nb * ga) || !all_finite(gammas_host, (size_t)ng * ga))
        return fail(GQAOA_EINVAL, "non-finite angle in the grid");
    if (num_items < 0 || num_items > (1 << 24)) return fail(GQAOA_ERANGE, "num_items=%d", num_items);
    if (num_items) {
        if (!items_host || !costs_dev || !cost_off_host || !item_psol_dev) return fail(GQAOA_EINVAL, "NULL item argument");
        for (int k = 0; k < num_items; ++k) {
            const int i = items_host[3 * k], g = items_host[3 * k + 1], b = items_host[3 * k + 2];
            if (i < 0 || i >= num_inst) return fail(GQAOA_ERANGE, "item %d: instance %d", k, i);
            if (g < 0 || g >= ng || b < 0 || b >= nb) return fail(GQAOA_EINVAL, "item %d: cell (%d, %d) outside the grid", k, g, b);
            if (n_host[i] > GQAOA_SV_ITEMS_MAX_N) return fail(GQAOA_ERANGE, "item %d: n=%d > %d", k, n_host[i], GQAOA_SV_ITEMS_MAX_N);
        }
    }
    ScanPlan *P = nullptr;
    s = scan_plan_create(num_inst, n_host, m_host, hists_host, hist_stride, target_host, nb, betas_host, ng,
                         gammas_host, pig, num_p, p_list_host, psol_dev, energy_dev, tile, num_items, items_host,
                         costs_dev, cost_off_host, item_psol_dev, item_energy_dev, (hipStream_t)stream, &P);
    if (s) return s;
    *plan_out = reinterpret_cast<gqaoa_scan_plan *>(P);
    return GQAOA_OK;
}

int gqaoa_scan_plan_run(gqaoa_scan_plan *plan, const double *betas_host, const double *gammas_host, void *stream) {
    clear_error();
    if (!plan) return fail(GQAOA_EINVAL, "NULL plan");
    if (!betas_host != !gammas_host) return fail(GQAOA_EINVAL, "one of the two grids is NULL");
    return scan_plan_run(reinterpret_cast<ScanPlan *>(plan), betas_host, gammas_host, (hipStream_t)stream);
}

void gqaoa_scan_plan_destroy(gqaoa_scan_plan *plan) { scan_plan_destroy(reinterpret_cast<ScanPlan *>(plan)); }

size_t gqaoa_mlp_act_bytes(int batch) {
    if (batch < 1 || batch > (1 << 20)) return 0;
    return mlp_act_bytes(batch);
}

size_t gqaoa_mlp_infer_bytes(int batch) {
    if (batch < 1 || batch > (1 << 20)) return 0;
    return mlp_infer_bytes(batch);
}

int gqaoa_mlp_infer(const float *params_dev, int batch, const float *x_dev, float *out_dev, void *ws_dev,
                    size_t ws_bytes, void *stream) {
    clear_error();
    if (batch < 1 || batch > (1 << 20)) return fail(GQAOA_ERANGE, "batch=%d", batch);
    if (!params_dev || !x_dev || !out_dev || !ws_dev) return fail(GQAOA_EINVAL, "NULL argument");
    if (ws_bytes < mlp_infer_bytes(batch)) return fail(GQAOA_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, mlp_infer_bytes(batch));
    return run_mlp_infer(params_dev, batch, x_dev, out_dev, ws_dev, (hipStream_t)stream);
}

int gqaoa_mlp_forward(const float *params_dev, int batch, const float *x_dev, float *out_dev, void *act_dev,
                      void *stream) {
    clear_error();
    if (batch < 1 || batch > (1 << 20)) return fail(GQAOA_ERANGE, "batch=%d", batch);
    if (!params_dev || !x_dev || !out_dev || !act_dev) return fail(GQAOA_EINVAL, "NULL argument");
    return run_mlp_forward(params_dev, batch, x_dev, out_dev, act_dev, (hipStream_t)stream);
}

int gqaoa_mlp_backward(const float *params_dev, int batch, const void *act_dev, const float *dout_dev,
                       float *grads_dev, void *stream) {
    clear_error();
    if (batch < 1 || batch > (1 << 20)) return fail(GQAOA_ERANGE, "batch=%d", batch);
    if (!params_dev || !act_dev || !dout_dev || !grads_dev) return fail(GQAOA_EINVAL, "NULL argument");
    return run_mlp_backward(params_dev, batch, act_dev, dout_dev, grads_dev, (hipStream_t)stream);
}

int gqaoa_mlp_adam(float *params_dev, const float *grads_dev, float *state_dev, int step, float lr, float beta1,
                   float beta2, float eps, void *stream) {
    clear_error();
    if (step < 1) return fail(GQAOA_ERANGE, "step=%d (first step is 1)", step);
    if (!params_dev || !grads_dev || !state_dev) return fail(GQAOA_EINVAL, "NULL argument");
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
        return fail(GQAOA_ERANGE, "Adam hyper-parameters");
    return run_mlp_adam(params_dev, grads_dev, state_dev, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}

int gqaoa_mlp_loss(int batch, const float *out_dev, const float *targets_dev, float *dout_dev, float *loss_dev,
                   void *stream) {
    clear_error();
    if (batch < 1 || batch > (1 << 20)) return fail(GQAOA_ERANGE, "batch=%d", batch);
    if (!out_dev || !targets_dev || !dout_dev || !loss_dev) return fail(GQAOA_EINVAL, "NULL argument");
    return run_mlp_loss(batch, out_dev, targets_dev, dout_dev, loss_dev, (hipStream_t)stream);
}

int gqaoa_mlp_features(int batch, const uint64_t *hists_dev, int hist_stride, const int32_t *n_dev,
                       const int32_t *m_dev, const int32_t *p_dev, float *x_dev, void *stream) {
    clear_error();
    if (batch < 1 || batch > (1 << 20)) return fail(GQAOA_ERANGE, "batch=%d", batch);
    if (hist_stride < 2 || hist_stride > 4096) return fail(GQAOA_ERANGE, "hist_stride=%d", hist_stride);
    if (!hists_dev || !n_dev || !m_dev || !p_dev || !x_dev) return fail(GQAOA_EINVAL, "NULL argument");
    return run_mlp_features(batch, hists_dev, hist_stride, n_dev, m_dev, p_dev, x_dev, (hipStream_t)stream);
}

int gqaoa_profile_enable(int on) {
    if (on < 0) return fail(GQAOA_EINVAL, "profile interval %d", on);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    g_prof_every = on > 0 ? on : 1;
    return GQAOA_OK;
}

void gqaoa_profile_reset(void) {
    prof_collect();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &t : g_prof_tot) t = ProfTotal{};
    for (auto &c : g_prof_seen) c = 0;
}

int gqaoa_profile_read(const char *name, double *total_ms, int64_t *count) {
    prof_collect();
    if (!name) return fail(GQAOA_EINVAL, "NULL name");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (size_t i = 0; i < sizeof(kProfNames) / sizeof(kProfNames[0]); ++i)
        if (!strcmp(kProfNames[i], name)) {
            if (total_ms) *total_ms = g_prof_tot[i].ms;
            if (count) *count = g_prof_tot[i].count;
            return GQAOA_OK;
        }
    return fail(GQAOA_EINVAL, "unknown profile name %s", name);
}

}  // extern "C"

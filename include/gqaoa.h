/* gqaoa.h - C ABI of libgqaoa, an MI355X (gfx950) simulator of Grover-QAOA
 * (G-QAOA) on random 3-SAT, following Zhang et al., "Grover-QAOA for 3-SAT:
 * Quadratic Speedup, Fair-Sampling, and Parameter Clustering" (arXiv 2402.02585).
 *
 * Conventions for every entry point
 *  - Pointers named *_dev are device memory (hipMalloc or a torch CUDA tensor),
 *    owned by the caller. Pointers named *_host are host memory owned by the
 *    caller. The library keeps no pointer after a call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work
 *    is enqueued on it. Calls that fill *_host outputs synchronize `stream`
 *    before returning; calls with device outputs only return after enqueueing.
 *  - Arguments are validated before anything is enqueued: on GQAOA_EINVAL or
 *    GQAOA_ERANGE nothing has been written. GQAOA_EHIP reports a failed HIP
 *    call; gqaoa_last_error() then holds the HIP message.
 *  - Clause encoding: a literal is the int32 2*var + neg (var in [0, n),
 *    neg = 1 for a negated variable); a clause is 3 literals on 3 distinct
 *    variables (App. B, Eq. (B2) with k_i = 3). lits_host holds 3*m int32.
 *  - Assignment tau <-> index z with variable v at bit v of z. A literal is
 *    false iff bit var of z equals neg (App. B: x is satisfied by tau(x) = 1,
 *    its negation by tau(x) = 0).
 *  - Complex amplitudes are interleaved (re, im): float2 for GQAOA_C64,
 *    double2 for GQAOA_C128. Angles are always double.
 *  - Per-round host outputs have p+1 entries: index 0 is the initial state,
 *    index j the state after round j's mixer.
 *  - The library is not thread-safe for concurrent calls sharing a
 *    workspace; independent workspaces/streams may be used concurrently.
 *  - Device memory: calls with a ws_dev argument use only it and the
 *    caller's buffers. The calls without one that stage per-call tables on
 *    the device (gqaoa_cost_table, gqaoa_hist_batched, gqaoa_cost_batched,
 *    gqaoa_hist_evolve, gqaoa_sv_items, gqaoa_shots_to_all,
 *    gqaoa_draws_to_reject) take them stream-ordered (hipMallocAsync on
 *    `stream`, freed on it after their last launch; clause records, round
 *    tables and block rows, a few MiB at most); gqaoa_cost_table_noalloc is
 *    the form of gqaoa_cost_table that allocates nothing. Plans allocate
 *    their device tables at create and free them at destroy; the streams a
 *    plan captures its graph on are borrowed from a per-device pool that the
 *    library keeps until the process ends (no device memory).
 */
#ifndef GQAOA_H
#define GQAOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GQAOA_OK = 0,
    GQAOA_EINVAL = -1,      /* NULL pointer, malformed clause, unknown enum value */
    GQAOA_ERANGE = -2,      /* n, m, p, level, batch size or grid out of range */
    GQAOA_EWORKSPACE = -3,  /* ws_bytes smaller than the matching *_workspace_bytes */
    GQAOA_EHIP = -4,        /* a HIP runtime call failed */
    GQAOA_ENODEV = -5       /* no usable gfx950 device */
};

typedef enum { GQAOA_C64 = 0, GQAOA_C128 = 1 } gqaoa_dtype;

/* Limits. GQAOA_MAX_M bounds m because costs are stored in one byte. */
#define GQAOA_MIN_N 3
#define GQAOA_MAX_N 34
#define GQAOA_MAX_M 255

/* Text of a status code (static storage). */
const char *gqaoa_status_string(int status);
/* Detail of the last failure on the calling thread ("" if none). */
const char *gqaoa_last_error(void);
/* ABI version, currently 1. */
int gqaoa_abi_version(void);

/* ---- cost table and level histogram ----------------------------------------
 * Definition: Sec. II.A (the energy E_i of clause i following Eq. (1)) and
 * App. B. C(z) = number of clauses that assignment z leaves unsatisfied = the
 * diagonal of H_P. The level histogram N_k = #{z : C(z) = k} is the
 * "classical pre-computation" of App. C ("Optimization").
 * n in [3, 34], m in [1, 255]. cost_dev: uint8[2^n], written for every z.
 * hist_dev: uint64[m+1] (N_0 = number of solutions), or NULL to skip it.
 * Errors: EINVAL for NULL lits/cost or a clause with a repeated variable or a
 * literal outside [0, 2n); ERANGE for n or m outside the limits. */
int gqaoa_cost_table(int n, int m, const int32_t *lits_host, uint8_t *cost_dev,
                     uint64_t *hist_dev, void *stream);

/* Allocation-free form of gqaoa_cost_table, for callers that cannot allocate
 * device memory (serving loops, harnesses that forbid hipMalloc): the same
 * arguments, errors and results (cost table and histogram bit-identical), with
 * the call's scratch (clause records and per-block histogram rows) in a static
 * device array of 12 KiB + 2 MiB instead of stream-ordered allocations. Every
 * valid (n, m) fits in it. Each GPU the library runs on holds its own copy
 * until the process ends. All calls on one GPU share that copy: calls that
 * overlap on one GPU (different streams without ordering, several host
 * threads) race; order them. Like gqaoa_cost_table it synchronizes the stream
 * once, after uploading the clause records, so it cannot be graph-captured. */
int gqaoa_cost_table_noalloc(int n, int m, const int32_t *lits_host, uint8_t *cost_dev,
                             uint64_t *hist_dev, void *stream);

/* Histograms only, for many instances in one launch (no cost table kept).
 * Instance i has n_host[i] variables, m_host[i] clauses whose literals start
 * at lits_host[3*off_i], off_i = sum of m_host[<i]. hists_dev is
 * uint64[num_inst][hist_stride], hist_stride >= max m + 1; entries beyond m_i
 * are zeroed. n_i in [3, 30], m_i in [1, 255], num_inst in [1, 2^20].
 * Errors as gqaoa_cost_table, plus ERANGE for hist_stride. */
int gqaoa_hist_batched(int num_inst, const int32_t *n_host, const int32_t *m_host,
                       const int32_t *lits_host, uint64_t *hists_dev, int hist_stride,
                       void *stream);

/* Cost tables of many instances in one launch (as gqaoa_hist_batched, with
 * n_i in [3, 26]): instance i's table C_i(z), z < 2^n_i, is written to
 * costs_dev + gqaoa_cost_batched_offset(i, n_host), the tables following
 * each other in instance order, each starting at a multiple of 64 bytes
 * (the buffer needs gqaoa_cost_batched_offset(num_inst, n_host) bytes).
 * hists_dev may be NULL; otherwise it receives the histograms as in
 * gqaoa_hist_batched. Errors as gqaoa_hist_batched. */
uint64_t gqaoa_cost_batched_offset(int index, const int32_t *n_host);
int gqaoa_cost_batched(int num_inst, const int32_t *n_host, const int32_t *m_host,
                       const int32_t *lits_host, uint8_t *costs_dev, uint64_t *hists_dev,
                       int hist_stride, void *stream);

/* ---- statevector evolution, Eq. (3) ---------------------------------------
 * For j = 1..p applies exp(-i gamma_j H_P) (phase exp(-i gamma_j C(z)) on z),
 * then exp(-i beta_j H_M) with H_M = |s><s| a projector (Eq. (2)), i.e.
 * psi <- psi + (exp(-i beta_j) - 1) |s><s|psi>. The single-angle-pair form,
 * Eq. (5), is the special case of equal angles.
 * psi_dev: on entry the initial state (ignored if init_uniform != 0, which
 * starts from |+> = |s>); on exit the state after round p. p in [0, 100000].
 * Readouts, each host array of p+1 doubles or NULL:
 *   psol_host[j]   = sum over z with C(z) = target_level of |psi_z|^2
 *                    (target_level 0: solutions; k_min: Max-SAT assignments),
 *   energy_host[j] = <psi|H_P|psi>, the cost function of Eq. (4),
 *   norm_host[j]   = <psi|psi>.
 * cost_dev must hold C(z) for all z (from gqaoa_cost_table) with values <= m.
 * ws_dev/ws_bytes: device scratch of gqaoa_workspace_bytes(n, p, dt, 0) bytes.
 * Errors: EINVAL (NULL cost/psi/angles/ws, bad dtype), ERANGE (n, m, p,
 * target_level outside [0, m]), EWORKSPACE. */
size_t gqaoa_workspace_bytes(int n, int p, int dtype, int ckpt_every);
int gqaoa_evolve(int n, int m, const uint8_t *cost_dev, int p, const double *beta_host,
                 const double *gamma_host, int dtype, int init_uniform, void *psi_dev,
                 int target_level, double *psol_host, double *energy_host,
                 double *norm_host, void *ws_dev, size_t ws_bytes, void *stream);

/* ---- X-QAOA comparator (Sec. II.B, rows "X" of Table I) -------------------
 * The same rounds with the transverse-field mixer in place of |s><s|: for
 * j = 1..p, psi <- exp(-i gamma_j H_P) psi, then psi <- exp(-i beta_j H_X) psi,
 * H_X = sum_q X_q, i.e. on every qubit q the amplitude pairs (a, b) differing
 * in bit q of z become (cos b_j a - i sin b_j b, cos b_j b - i sin b_j a).
 * Arguments, readouts, dtypes and errors as gqaoa_evolve (init_uniform starts
 * from |+>); the level-space shortcut does not apply to this mixer.
 * ws: gqaoa_x_workspace_bytes(n, p, dtype) bytes (0 for invalid arguments). */
size_t gqaoa_x_workspace_bytes(int n, int p, int dtype);
int gqaoa_evolve_x(int n, int m, const uint8_t *cost_dev, int p, const double *beta_host,
                   const double *gamma_host, int dtype, int init_uniform, void *psi_dev,
                   int target_level, double *psol_host, double *energy_host,
                   double *norm_host, void *ws_dev, size_t ws_bytes, void *stream);

/* Graph-captured form of gqaoa_evolve for callers that evolve one instance
 * many times with new angles (angle searches, where at small n each round is
 * a few microseconds and launch overhead dominates): create captures the
 * whole call (device-side angle tables, p >= 1 rounds, final readout) into
 * one HIP graph; each run uploads the 2p angles, replays it and returns the
 * readouts as gqaoa_evolve does (synchronizes the stream). Arguments of
 * create as gqaoa_evolve (workspace: gqaoa_workspace_bytes(n, p, dtype, 0));
 * cost_dev, psi_dev and ws_dev must stay valid while the plan lives. With
 * init_uniform = 1 every run starts from |s>; with 0, from psi's contents,
 * which a run overwrites with its final state. Runs of one plan come from
 * one host thread at a time. The results equal gqaoa_evolve's up to the last
 * bit of the phase tables (device vs host float64 sin/cos).
 * Errors: as gqaoa_evolve, ERANGE for p < 1, EINVAL for a NULL plan_out or
 * angles, non-finite angles, or another device current at a run. */
typedef struct gqaoa_evolve_plan gqaoa_evolve_plan;
int gqaoa_evolve_plan_create(int n, int m, const uint8_t *cost_dev, int p, int dtype,
                             int init_uniform, void *psi_dev, int target_level, void *ws_dev,
                             size_t ws_bytes, void *stream, gqaoa_evolve_plan **plan_out);
int gqaoa_evolve_plan_run(gqaoa_evolve_plan *plan, const double *beta_host,
                          const double *gamma_host, double *psol_host, double *energy_host,
                          double *norm_host, void *stream);
void gqaoa_evolve_plan_destroy(gqaoa_evolve_plan *plan);

/* Solution probability of a given state (the readout of Sec. III, P_sol):
 * *out_host = sum over z with C(z) = target_level of |psi_z|^2.
 * ws: gqaoa_workspace_bytes(n, 0, dtype, 0) bytes. */
int gqaoa_solution_prob(int n, const uint8_t *cost_dev, const void *psi_dev, int dtype,
                        int target_level, double *out_host, void *ws_dev, size_t ws_bytes,
                        void *stream);

/* ---- adjoint gradient of P_sol ----------------------------------------------
 * P = <psi_p|Pi_t|psi_p> after p rounds of Eq. (3) from |s>, Pi_t the
 * projector on level t = target_level, and its gradient with respect to all
 * 2p angles (the full G-QAOA parameters optimized in App. C), by a reverse
 * sweep: lambda_p = Pi_t psi_p; mu_k = lambda_k + (e^{+i beta_k} - 1)|s><s|lambda_k>;
 * dP/dbeta_k = 2 Re(-i e^{-i beta_k} <lambda_k|s><s|phi_k>);
 * dP/dgamma_k = 2 Im(sum_z conj(mu_z) C(z) phi_z); lambda_{k-1} = e^{+i gamma_k C} mu_k,
 * with phi_k the state after round k's phase. Forward states are
 * checkpointed every ckpt_every rounds and recomputed per segment
 * (ckpt_every = 0 keeps every round's state).
 * Batched form: num_inst instances with the same n, m_host[i] clauses,
 * costs at cost_dev + i*2^n, angles at beta_host + i*p. Outputs psol_host[i],
 * dbeta_host[i*p + k], dgamma_host[i*p + k].
 * ws: gqaoa_grad_workspace_bytes(num_inst, n, p, dtype, ckpt_every) bytes.
 * Errors: as gqaoa_evolve; ERANGE for p < 1, ckpt_every < 0 or num_inst < 1. */
size_t gqaoa_grad_workspace_bytes(int num_inst, int n, int p, int dtype, int ckpt_every);
int gqaoa_grad(int n, int m, const uint8_t *cost_dev, int p, const double *beta_host,
               const double *gamma_host, int dtype, int target_level, int ckpt_every,
               double *psol_host, double *dbeta_host, double *dgamma_host, void *ws_dev,
               size_t ws_bytes, void *stream);
int gqaoa_grad_batched(int num_inst, int n, const int32_t *m_host, const uint8_t *cost_dev,
                       int p, const double *beta_host, const double *gamma_host, int dtype,
                       const int32_t *target_host, int ckpt_every, double *psol_host,
                       double *dbeta_host, double *dgamma_host, void *ws_dev,
                       size_t ws_bytes, void *stream);

/* ---- level-space ("effective space") evolution ----------------------------
 * App. C, "Optimization": from |s> every amplitude depends on z only through
 * C(z), so the state is one amplitude b_k per occupied level k with weight
 * w_k = N_k / 2^n, evolved as b_k <- e^{-i gamma_j k} b_k, then
 * b_k <- b_k + (e^{-i beta_j} - 1) sum_l w_l b_l. Readouts P_sol = w_t |b_t|^2,
 * E = sum_k k w_k |b_k|^2, norm = sum_k w_k |b_k|^2 (float64 on the device).
 * hist_dev: uint64[m+1] (from gqaoa_cost_table); n gives 2^n = sum N_k.
 * Outputs as gqaoa_evolve (p+1 entries each, NULL to skip). */
int gqaoa_hist_evolve(int n, int m, const uint64_t *hist_dev, int p, const double *beta_host,
                      const double *gamma_host, int target_level, double *psol_host,
                      double *energy_host, double *norm_host, void *stream);

/* Level-space adjoint gradient for many instances (float64): for instance i,
 * P_i = w_t |b_t|^2 after p_i rounds of Eq. (3) from |s> in the level space
 * above (t = target_host[i], NULL = level 0) and dP_i/dbeta_k, dP_i/dgamma_k for
 * every round k < p_i: the reverse sweep of gqaoa_grad with <s|x> =
 * sum_l w_l x_l and the diagonal C replaced by the level index. These are the
 * gradients of full G-QAOA (all 2p angles, App. C "Optimization") at O(p K)
 * work per instance, K = occupied levels, instead of O(p 2^n). The forward
 * states are recomputed by running each (unitary) round backwards, so the
 * device state is O(K) per instance for any p.
 * Instance i: hists_host + i*hist_stride holds N_k for k <= m_host[i] (host
 * memory, as gqaoa_scan_batched), n_host[i] variables (sum N_k = 2^n), p_i =
 * p_host[i] in [1, p_max] (NULL: p_max for all), angles beta_host[i*p_max + k]
 * and gamma_host[i*p_max + k] for k < p_i.
 * Outputs (host, each may be NULL): psol_host[i], dbeta_host[i*p_max + k],
 * dgamma_host[i*p_max + k]; entries k >= p_i are 0. Synchronizes the stream.
 * ws: gqaoa_hist_grad_workspace_bytes(num_inst, hist_stride, p_max) bytes (0
 * for invalid sizes). Errors: EINVAL (NULL pointers), ERANGE (num_inst in
 * [1, 2^20], hist_stride in [2, 4096], n_i in [3, 62], m_i in [1, 255] with
 * m_i < hist_stride, target in [0, m_i], p_max in [1, 100000], p_i), EWORKSPACE. */
size_t gqaoa_hist_grad_workspace_bytes(int num_inst, int hist_stride, int p_max);
int gqaoa_hist_grad_batched(int num_inst, const int32_t *n_host, const int32_t *m_host,
                            const uint64_t *hists_host, int hist_stride, const int32_t *target_host,
                            int p_max, const int32_t *p_host, const double *beta_host,
                            const double *gamma_host, double *psol_host, double *dbeta_host,
                            double *dgamma_host, void *ws_dev, size_t ws_bytes, void *stream);

/* ---- batched single-angle-pair scan, Eq. (5) -------------------------------
 * For every instance i, beta_b (b < nb) and gamma_g (g < ng), runs the
 * single-angle-pair protocol in the level space for p_list[num_p-1] rounds
 * and records, after each p in p_list (ascending, >= 1),
 *   psol_dev  [((i*num_p + q)*ng + g)*nb + b] = P_sol   (float),
 *   energy_dev[same index]                    = E, Eq. (4) (float; NULL to skip).
 * Instance i: hists_host + i*hist_stride holds N_k for k <= m_host[i],
 * n_host[i] variables; target_host[i] its target level (NULL = 0 for all).
 * Angles in radians: with per_instance_grid = 0 every instance uses
 * betas_host[nb] and gammas_host[ng]; with 1 instance i uses
 * betas_host[i*nb .. i*nb+nb) and gammas_host[i*ng .. i*ng+ng). Arithmetic is
 * float32.
 * tile: NULL = autotuned (cached per device and shape class), else an int[2]
 * {waves_per_block in {1,2,4}, blocks_per_cu in [1,32]}.
 * ws: gqaoa_scan_workspace_bytes(num_inst, hist_stride, nb, ng, num_p,
 * per_instance_grid) bytes.
 * Errors: EINVAL (NULL pointers), ERANGE (num_inst in [1, 2^20], nb, ng in
 * [1, 4096], num_p in [1, 16], p values in [1, 100000], more than 128
 * occupied levels in an instance). */
size_t gqaoa_scan_workspace_bytes(int num_inst, int hist_stride, int nb, int ng, int num_p,
                                  int per_instance_grid);
int gqaoa_scan_batched(int num_inst, const int32_t *n_host, const int32_t *m_host,
                       const uint64_t *hists_host, int hist_stride, const int32_t *target_host,
                       int nb, const double *betas_host, int ng, const double *gammas_host,
                       int per_instance_grid, int num_p, const int32_t *p_list_host,
                       float *psol_dev, float *energy_dev, const int32_t *tile, void *ws_dev,
                       size_t ws_bytes, void *stream);

/* Rounds-to-target form of the scan (the minimum-rounds search of Sec. III.A
 * and its Max-SAT variant): the same single-angle-pair level-space rounds,
 * run up to p_i rounds, recording for every (i, g, b)
 *   first_p_dev[(i*ng + g)*nb + b] = the first round j in [1, p_i] after
 *   which P_sol (at target_host[i]) >= threshold, or 0 if none.
 * p_i = p_max_host[i] (each in [1, p_max]), or p_max for every instance when
 * p_max_host is NULL; p_max in [1, 100000]; threshold in (0, 1]. The
 * decision is taken on the float32 P_sol. Other arguments, workspace (with
 * num_p = 1) and errors as gqaoa_scan_batched. */
int gqaoa_scan_crossing(int num_inst, const int32_t *n_host, const int32_t *m_host,
                        const uint64_t *hists_host, int hist_stride, const int32_t *target_host,
                        int nb, const double *betas_host, int ng, const double *gammas_host,
                        int per_instance_grid, int p_max, const int32_t *p_max_host,
                        float threshold, int32_t *first_p_dev,
                        const int32_t *tile, void *ws_dev, size_t ws_bytes, void *stream);

/* Statevector work items of the batched scan (the check of the level-space
 * reduction amplitude by amplitude): item k runs the single-angle-pair
 * protocol of Eq. (5) with (beta_host[k], gamma_host[k]) on instance
 * item_inst_host[k], whose cost table is in costs_dev at
 * gqaoa_cost_batched_offset(item_inst_host[k], n_host) (the layout written by
 * gqaoa_cost_batched), from |s>, complex64 state, for
 * p_list[num_p-1] rounds, recording after each p in p_list (ascending)
 *   psol_dev  [k*num_p + q] = P_sol at target_host[inst] (NULL: level 0),
 *   energy_dev[k*num_p + q] = E of Eq. (4) (NULL to skip), both float.
 * Items of instances with n <= GQAOA_SV_ITEMS_MAX_N keep their state in
 * registers (one block per item); larger ones (n <= 26) are evolved by the
 * streaming round passes, all items of one n together.
 * Synchronizes the stream. Errors: EINVAL (NULL pointers, non-finite angles,
 * p_list not ascending), ERANGE (counts, n, m, targets, p values). */
#define GQAOA_SV_ITEMS_MAX_N 14
int gqaoa_sv_items(int num_inst, const int32_t *n_host, const int32_t *m_host,
                   const int32_t *target_host, const uint8_t *costs_dev, int num_items,
                   const int32_t *item_inst_host, const double *beta_host,
                   const double *gamma_host, int num_p, const int32_t *p_list_host,
                   float *psol_dev, float *energy_dev, void *stream);

/* ---- graph-captured scan plan ----------------------------------------------
 * The scan of gqaoa_scan_batched (Eq. (5) in the level space of App. C) for
 * callers that evaluate the same instances over many angle grids (grid
 * refinement, local searches around optimized angles), with optional
 * statevector work items on cells of the same grid (the amplitude-by-amplitude
 * check of gqaoa_sv_items).
 *
 * gqaoa_scan_plan_create does the per-instance work once: it compacts and
 * uploads the occupied levels, chooses every bucket's launch shape (tile as in
 * gqaoa_scan_batched), and captures all launches in one HIP graph, the scan on
 * one branch and the items on a parallel one. Arguments num_inst ... tile are
 * those of gqaoa_scan_batched (no workspace: the plan allocates its device
 * tables and a pinned staging block, freed by gqaoa_scan_plan_destroy);
 * betas_host/gammas_host give the first grid. psol_dev/energy_dev (layout of
 * gqaoa_scan_batched) must stay valid while the plan lives.
 * Items (num_items in [0, 2^24]; 0 = none, and then the item arguments may be
 * NULL): items_host[3k..3k+2] = (instance i, gamma index g, beta index b);
 * item k runs the single-angle-pair protocol with the grid's (beta_b,
 * gamma_g) of instance i (its own row when per_instance_grid) on the cost
 * table at costs_dev + cost_off_host[i] (uint8[2^n_i], e.g. written by
 * gqaoa_cost_batched), and writes item_psol_dev[k*num_p + q] (and
 * item_energy_dev, NULL to skip) after each p_list[q], the float values of
 * the scan's cell (i, q, g, b) computed without the level reduction. Item
 * instances need n <= GQAOA_SV_ITEMS_MAX_N (the register-held items).
 * Synchronizes the stream. Errors: those of gqaoa_scan_batched and
 * gqaoa_sv_items, EINVAL for a NULL plan_out or an item cell outside the
 * grid, EHIP if the graph cannot be captured.
 *
 * gqaoa_scan_plan_run uploads a new grid (same sizes as at creation;
 * betas_host and gammas_host both NULL: keep the current one) and replays the
 * graph on `stream`. It does not synchronize: the outputs are complete when
 * the stream reaches the end of the replay. A run waits (on the device) for
 * the plan's previous replay, from any stream, and (on the host) for the
 * previous upload to have read the staging block. A plan is used from one
 * host thread at a time, on the device current at its creation.
 * Errors: EINVAL (NULL plan, one of the two grids NULL, non-finite angles,
 * another device current).
 *
 * gqaoa_scan_plan_destroy waits for the plan's last replay and frees it
 * (NULL is a no-op). */
typedef struct gqaoa_scan_plan gqaoa_scan_plan;
int gqaoa_scan_plan_create(int num_inst, const int32_t *n_host, const int32_t *m_host,
                           const uint64_t *hists_host, int hist_stride, const int32_t *target_host,
                           int nb, const double *betas_host, int ng, const double *gammas_host,
                           int per_instance_grid, int num_p, const int32_t *p_list_host,
                           float *psol_dev, float *energy_dev, const int32_t *tile,
                           int num_items, const int32_t *items_host, const uint8_t *costs_dev,
                           const uint64_t *cost_off_host, float *item_psol_dev,
                           float *item_energy_dev, void *stream, gqaoa_scan_plan **plan_out);
int gqaoa_scan_plan_run(gqaoa_scan_plan *plan, const double *betas_host,
                        const double *gammas_host, void *stream);
void gqaoa_scan_plan_destroy(gqaoa_scan_plan *plan);

/* ---- angle-predictor MLP (bfloat16 MFMA, float32 accumulation) -------------
 * The paper suggests deriving angles from statistics of the density of
 * states (Sec. V) and reports clustering of optimized pairs (Sec. III.B).
 * Network 131 -> 256 -> GELU -> 256 -> GELU -> 2 (exact-erf GELU).
 * params_dev: float32 master parameters packed as
 *   W1[160][256] (rows 131..159 zero), b1[256], W2[256][256], b2[256],
 *   W3[256][2], b3[2]  -> GQAOA_MLP_NPARAMS floats.
 * x_dev: float32 features [batch][131] (rounded to bfloat16 on load).
 * out_dev: float32 raw outputs [batch][2]; beta = 2 pi sigmoid(o0),
 * gamma = pi sigmoid(o1).
 * act_dev: activation cache of gqaoa_mlp_act_bytes(batch) bytes, written by
 * forward and read by backward.
 * gqaoa_mlp_backward takes dout_dev [batch][2] (dL/do, float32) and writes
 * grads_dev (same packing as params, float32; overwritten, not accumulated).
 * gqaoa_mlp_adam: Adam with bias correction on the float32 master copy;
 * state_dev holds 2*GQAOA_MLP_NPARAMS floats (m then v), zero at step 1.
 * batch in [1, 1<<20]. */
#define GQAOA_MLP_NPARAMS (160 * 256 + 256 + 256 * 256 + 256 + 256 * 2 + 2)
size_t gqaoa_mlp_act_bytes(int batch);
int gqaoa_mlp_forward(const float *params_dev, int batch, const float *x_dev, float *out_dev,
                      void *act_dev, void *stream);
/* Inference only (no activation cache, no gradients): the same outputs as
 * gqaoa_mlp_forward (identical bfloat16 activations; the output layer's sum
 * may round differently in the last float32 place), from two launches with
 * the weights held in LDS. ws_dev: gqaoa_mlp_infer_bytes(batch) bytes for
 * the bfloat16 first hidden layer. Errors: ERANGE (batch), EINVAL (NULL
 * pointers), EWORKSPACE. */
size_t gqaoa_mlp_infer_bytes(int batch);
int gqaoa_mlp_infer(const float *params_dev, int batch, const float *x_dev, float *out_dev,
                    void *ws_dev, size_t ws_bytes, void *stream);
int gqaoa_mlp_backward(const float *params_dev, int batch, const void *act_dev,
                       const float *dout_dev, float *grads_dev, void *stream);
int gqaoa_mlp_adam(float *params_dev, const float *grads_dev, float *state_dev, int step,
                   float lr, float beta1, float beta2, float eps, void *stream);
/* Angle-regression loss L = mean_b ((beta_b - beta*_b)/(2 pi))^2 + ((gamma_b - gamma*_b)/pi)^2
 * on the raw outputs out_dev [batch][2]; targets_dev [batch][2] = (beta*, gamma*).
 * Writes dout_dev = dL/dout [batch][2] and *loss_dev (float, device). */
int gqaoa_mlp_loss(int batch, const float *out_dev, const float *targets_dev, float *dout_dev,
                   float *loss_dev, void *stream);
/* Features of the network from device histograms: x_dev [batch][131] with
 * x[k] = N_k / 2^n for k < 128 (0 beyond m), x[128] = n/24, x[129] = d/8 with
 * d = m/n, x[130] = log2(p)/6. hists_dev [batch][hist_stride] (uint64);
 * n_dev, m_dev, p_dev: int32 [batch] device arrays. */
int gqaoa_mlp_features(int batch, const uint64_t *hists_dev, int hist_stride, const int32_t *n_dev,
                       const int32_t *m_dev, const int32_t *p_dev, float *x_dev, void *stream);

/* ---- fair-sampling metrics (Sec. IV, Table I, the two right-hand columns) ---
 * Monte Carlo on the device over noiseless output probabilities. Random
 * numbers: SplitMix64 (Steele, Lea and Flood, 2014) used counter-based, draw
 * d of run r is output r * 2^32 + d of the generator started from state seed,
 * u = (x >> 11) * 2^-53; a draw is the first category k with u < cdf[k]
 * (running sums in index order).
 *
 * gqaoa_shots_to_all: p_host[k] = probability of solution k in the output
 * distribution (k < num_solutions <= 64, sum <= 1; the remaining mass is the
 * non-solution outcome). For every run r < runs, shots_dev[r] (int32,
 * device) = the number of shots until every solution has appeared, or 0 if
 * that takes more than max_shots.
 *
 * gqaoa_draws_to_reject: draws from the distribution conditioned on
 * solutions (q_host, num_solutions in [2, 64], normalized here; the last
 * solution takes any rounding rest). For every trial, after each draw N >=
 * n_min the chi-squared statistic against the uniform distribution is
 * compared with crit (the caller's critical value for num_solutions - 1
 * degrees of freedom) in the exact form K sum_k O_k^2 - N^2 > crit N;
 * draws_dev[trial] = the first such N, or 0 if none up to max_draws (<= 1e7).
 * Both synchronize the stream. Errors: ERANGE (counts and limits), EINVAL
 * (NULL pointers, negative or non-finite probabilities, crit). */
int gqaoa_shots_to_all(int num_solutions, const double *p_host, int runs, uint64_t seed,
                       int max_shots, int32_t *shots_dev, void *stream);
int gqaoa_draws_to_reject(int num_solutions, const double *q_host, int trials, uint64_t seed,
                          double crit, int n_min, int max_draws, int32_t *draws_dev,
                          void *stream);

/* ---- selections on device data -----------------------------------------------
 * Small steps the drivers take between the calls above (picking optimized
 * angles from a scan, the earliest crossing of Sec. III.A, the solution
 * distribution of Sec. IV), kept on the device so that no other framework
 * computes on the library's outputs.
 *
 * gqaoa_row_best: x_dev is a row-major rows x cols matrix. For every row r,
 * idx_dev[r] (int32) = the column of its best entry, ties to the lowest
 * column, and val_dev[r] (NULL to skip) = that entry:
 *   GQAOA_ROW_ARGMAX_F32: the largest float (a NaN never beats a number);
 *   GQAOA_ROW_ARGMIN_F32: the smallest float;
 *   GQAOA_ROW_MIN_POSITIVE_I32: the least int32 > 0 (the earliest first
 *     crossing of gqaoa_scan_crossing); idx and val are 0 if the row has none.
 * rows >= 1, cols in [1, 2^30]. Enqueues only. Errors: ERANGE, EINVAL. */
enum { GQAOA_ROW_ARGMAX_F32 = 0, GQAOA_ROW_ARGMIN_F32 = 1, GQAOA_ROW_MIN_POSITIVE_I32 = 2 };
int gqaoa_row_best(int rows, int cols, const void *x_dev, int mode, int32_t *idx_dev, void *val_dev,
                   void *stream);

/* The assignments of one cost level and their output probabilities (the
 * solution distribution whose fairness Sec. IV measures, level 0; or any
 * other level): for the k-th z in ascending order with C(z) = level,
 * z_dev[k] = z (int64) and prob_dev[k] = |psi_z|^2 (float64, from the state's
 * components), for k < min(count, max_out); *count_host = the number of such
 * z. Either output may be NULL. cost_dev: uint8[2^n]; psi_dev: float2 or
 * double2 [2^n]. ws: gqaoa_level_probs_workspace_bytes(n) bytes (8 bytes per
 * 16384 assignments). Synchronizes the stream. Errors: ERANGE (n, level,
 * max_out < 0), EINVAL, EWORKSPACE. */
size_t gqaoa_level_probs_workspace_bytes(int n);
int gqaoa_level_probs(int n, const uint8_t *cost_dev, const void *psi_dev, int dtype, int level,
                      int64_t max_out, int64_t *z_dev, double *prob_dev, int64_t *count_host,
                      void *ws_dev, size_t ws_bytes, void *stream);

/* The angle map of the network (gqaoa_mlp_forward / gqaoa_mlp_infer outputs
 * [batch][2]): beta_dev[b] = 2 pi sigmoid(o_b0), gamma_dev[b] = pi
 * sigmoid(o_b1), in float64. batch in [1, 2^26]. Enqueues only. */
int gqaoa_mlp_angles(int batch, const float *out_dev, double *beta_dev, double *gamma_dev, void *stream);

/* Row gather (training batches): dst row r = src row idx_dev[r] for r <
 * rows, rows of row_bytes bytes (a multiple of 4, at most 1 MiB); an index
 * outside [0, src_rows) gives a row of zeros. Enqueues only. */
int gqaoa_gather_rows(int rows, const int32_t *idx_dev, int src_rows, const void *src_dev, int row_bytes,
                      void *dst_dev, void *stream);

/* ---- instrumentation ---------------------------------------------------------
 * gqaoa_profile_enable(k) with k >= 1 makes the library bracket one launch
 * in k (counted per name, from the last reset) of its streaming kernels with
 * HIP events on the launch stream and accumulate their durations under a
 * name (k = 0 disables; k < 0 is EINVAL): "sv_round_c64", "sv_round_c128" (forward round
 * passes), "sv_reverse_c64", "sv_reverse_c128" (adjoint passes), "cost_table",
 * "scan", "x_pass_c64", "x_pass_c128" (X-QAOA streaming passes), and
 * "sv_resident_c64", "sv_resident_c128" (the one-launch evolution of a
 * small state, all rounds).
 * Durations are collected when the call that launched them synchronizes.
 * gqaoa_profile_read returns GQAOA_EINVAL for an unknown name. */
int gqaoa_profile_enable(int on);
void gqaoa_profile_reset(void);
int gqaoa_profile_read(const char *name, double *total_ms, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* GQAOA_H */

// Level-space adjoint gradient of P_sol for many instances (float64): the
// reverse sweep of the adjoint gradient (dP/dbeta_k, dP/dgamma_k for every
// round) in the effective space of App. C, "Optimization", for full G-QAOA
// (all 2p angles, App. C) at the sizes the paper simulates.
//
// From |s>, an amplitude depends on z only through the level l = C(z), so the
// state is one amplitude b_l per occupied level with weight w_l = N_l / 2^n,
// and <s|x> = sum_l w_l x_l. Forward round k (Eq. (3)):
//     phi_k = e^{-i gamma_k l} psi_{k-1},   psi_k = phi_k + (e^{-i beta_k} - 1) <s|phi_k>.
// P = w_t |psi_p(t)|^2 at the target level t. Reverse sweep, lambda_p = Pi_t psi_p:
//     mu_k = lambda_k + (e^{+i beta_k} - 1) <s|lambda_k>
//     dP/dbeta_k  = 2 Re(-i e^{-i beta_k} conj(<s|lambda_k>) <s|phi_k>)
//     dP/dgamma_k = 2 Im(sum_l w_l conj(mu_l) l phi_l)
//     lambda_{k-1} = e^{+i gamma_k l} mu_k.
// The forward states are not stored: a round is unitary, so the reverse sweep
// runs it backwards, phi_k = psi_k + (e^{+i beta_k} - 1) <s|psi_k> and
// psi_{k-1} = e^{+i gamma_k l} phi_k, and needs O(K) state per instance for
// any p (the rounding of the inversion grows like p times the float64 epsilon).
//
// One wave per instance; lane j holds the compacted occupied levels j + 64 i,
// i < LPL (LPL = 1, 2, 4 for up to 64, 128, 256 levels). Inner products are
// DPP wave sums in a fixed order, so results do not depend on the batch.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gqaoa {

struct HistGradSlot {
    int32_t inst;     // caller's instance index
    int32_t lev_off;  // first compacted level of the instance
    int32_t K;        // occupied levels
    int32_t t_idx;    // position of the target level among them, -1 if unoccupied
    int32_t p;        // rounds of this instance
    int32_t pad[3];
};

struct HistGradArgs {
    const HistGradSlot *slots;
    int nslots;
    const int32_t *lev;
    const double *w;
    const double *betas, *gammas;  // [inst][pstride]
    int pstride;
    double *psol;                  // [inst]
    double *dbeta, *dgamma;        // [inst][pstride]
};

constexpr int kGradWaves = 4;

template <int LPL>
__global__ void __launch_bounds__(kGradWaves * 64) hist_grad_kernel(HistGradArgs a) {
    const int lane = threadIdx.x & 63;
    const int slot = blockIdx.x * kGradWaves + (threadIdx.x >> 6);
    if (slot >= a.nslots) return;  // whole waves exit together
    const HistGradSlot sl = a.slots[slot];
    const double *bet = a.betas + (size_t)sl.inst * a.pstride;
    const double *gam = a.gammas + (size_t)sl.inst * a.pstride;
    double lv[LPL], w[LPL], br[LPL], bi[LPL];
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
        const int k = lane + 64 * i;
        const bool on = k < sl.K;
        lv[i] = on ? (double)a.lev[sl.lev_off + k] : 0.0;
        w[i] = on ? a.w[sl.lev_off + k] : 0.0;
        br[i] = 1.0;
        bi[i] = 0.0;
    }
    // forward rounds
    for (int r = 0; r < sl.p; ++r) {
        const double g = gam[r];
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            double s, c;
            sincos(g * lv[i], &s, &c);
            const double pr = c * br[i] + s * bi[i];   // e^{-i g l} b
            const double pi_ = c * bi[i] - s * br[i];
            br[i] = pr;
            bi[i] = pi_;
            sr += w[i] * pr;
            si += w[i] * pi_;
        }
        sr = wave_sum_dpp(sr);
        si = wave_sum_dpp(si);
        double sb, cb;
        sincos(bet[r], &sb, &cb);
        const double mr = cb - 1.0, mi = -sb;             // e^{-i beta} - 1
        const double dr = mr * sr - mi * si, di = mr * si + mi * sr;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            br[i] += dr;
            bi[i] += di;
        }
    }
    // P and lambda_p = Pi_t psi_p (a level's amplitude sits in one lane only)
    double lr[LPL], li[LPL], P = 0.0;
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
        const bool t = lane + 64 * i == sl.t_idx;
        lr[i] = t ? br[i] : 0.0;
        li[i] = t ? bi[i] : 0.0;
        P += t ? w[i] * (br[i] * br[i] + bi[i] * bi[i]) : 0.0;
    }
    P = wave_sum_dpp(P);
    if (lane == 0) a.psol[sl.inst] = P;
    double *db = a.dbeta + (size_t)sl.inst * a.pstride;
    double *dg = a.dgamma + (size_t)sl.inst * a.pstride;
    for (int r = sl.p - 1; r >= 0; --r) {
        double sb, cb;
        sincos(bet[r], &sb, &cb);
        const double hr = cb - 1.0, hi = sb;              // e^{+i beta} - 1
        // phi_r from psi_r: phi = psi + (e^{+i beta} - 1) <s|psi>
        double pr_ = 0.0, pi_ = 0.0, lsr = 0.0, lsi = 0.0;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            pr_ += w[i] * br[i];
            pi_ += w[i] * bi[i];
            lsr += w[i] * lr[i];
            lsi += w[i] * li[i];
        }
        pr_ = wave_sum_dpp(pr_);
        pi_ = wave_sum_dpp(pi_);
        lsr = wave_sum_dpp(lsr);
        lsi = wave_sum_dpp(lsi);
        const double er = hr * pr_ - hi * pi_, ei = hr * pi_ + hi * pr_;
        double fsr = 0.0, fsi = 0.0;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            br[i] += er;                                  // br, bi now hold phi_r
            bi[i] += ei;
            fsr += w[i] * br[i];
            fsi += w[i] * bi[i];
        }
        fsr = wave_sum_dpp(fsr);
        fsi = wave_sum_dpp(fsi);
        // dP/dbeta = 2 Re(-i e^{-i beta} conj(s_lam) s_phi), -i e^{-i beta} = (-sin beta, -cos beta)
        const double zr = lsr * fsr + lsi * fsi, zi = lsr * fsi - lsi * fsr;  // conj(s_lam) s_phi
        const double dbeta = 2.0 * (-sb * zr + cb * zi);
        // mu = lambda + (e^{+i beta} - 1) s_lam
        const double ur = hr * lsr - hi * lsi, ui = hr * lsi + hi * lsr;
        double gsum = 0.0;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            lr[i] += ur;                                  // lr, li now hold mu_r
            li[i] += ui;
            // Im(conj(mu) phi) = mu_r phi_i - mu_i phi_r
            gsum += w[i] * lv[i] * (lr[i] * bi[i] - li[i] * br[i]);
        }
        gsum = wave_sum_dpp(gsum);
        if (lane == 0) {
            db[r] = dbeta;
            dg[r] = 2.0 * gsum;
        }
        // lambda_{r-1} = e^{+i g l} mu_r, psi_{r-1} = e^{+i g l} phi_r
        const double g = gam[r];
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            double s, c;
            sincos(g * lv[i], &s, &c);
            const double nbr = c * br[i] - s * bi[i], nbi = c * bi[i] + s * br[i];
            const double nlr = c * lr[i] - s * li[i], nli = c * li[i] + s * lr[i];
            br[i] = nbr;
            bi[i] = nbi;
            lr[i] = nlr;
            li[i] = nli;
        }
    }
    for (int r = sl.p + lane; r < a.pstride; r += 64) {  // rounds beyond this instance's p
        db[r] = 0.0;
        dg[r] = 0.0;
    }
}

constexpr int kHistGradMaxK = 256;

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

size_t hist_grad_workspace_bytes(int num_inst, int hist_stride, int pstride) {
    const size_t I = (size_t)num_inst;
    const size_t lv = I * (size_t)std::min(hist_stride, kHistGradMaxK);
    const size_t ang = I * (size_t)pstride * sizeof(double);
    return al256(sizeof(HistGradSlot) * I) + al256(4 * lv) + al256(8 * lv) + 2 * al256(ang) +
           al256(8 * I) + 2 * al256(ang);
}

int run_hist_grad(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists,
                  int hist_stride, const int32_t *target_host, int pstride, const int32_t *p_host,
                  const double *beta, const double *gamma, double *psol, double *dbeta, double *dgamma,
                  void *ws, hipStream_t st) {
    // compact the occupied levels; group instances by levels per lane
    std::vector<int32_t> lev;
    std::vector<double> w;
    std::vector<HistGradSlot> groups[3];
    for (int i = 0; i < num_inst; ++i) {
        const uint64_t *h = hists + (size_t)i * hist_stride;
        const int t = target_host ? target_host[i] : 0;
        const double invN = std::ldexp(1.0, -n_host[i]);
        HistGradSlot s{i, (int32_t)lev.size(), 0, -1, p_host ? p_host[i] : pstride, {0, 0, 0}};
        for (int k = 0; k <= m_host[i]; ++k)
            if (h[k]) {
                if (k == t) s.t_idx = (int32_t)lev.size() - s.lev_off;
                lev.push_back(k);
                w.push_back((double)h[k] * invN);  // exact: a count times a power of two
            }
        s.K = (int32_t)lev.size() - s.lev_off;
        groups[s.K <= 64 ? 0 : (s.K <= 128 ? 1 : 2)].push_back(s);
    }
    std::vector<HistGradSlot> slots;
    int first[4] = {0, 0, 0, 0};
    for (int gi = 0; gi < 3; ++gi) {
        first[gi] = (int)slots.size();
        slots.insert(slots.end(), groups[gi].begin(), groups[gi].end());
    }
    first[3] = (int)slots.size();

    const size_t I = (size_t)num_inst;
    const size_t lvcap = I * (size_t)std::min(hist_stride, kHistGradMaxK);
    const size_t ang = I * (size_t)pstride * sizeof(double);
    char *p = reinterpret_cast<char *>(ws);
    HistGradSlot *d_slots = reinterpret_cast<HistGradSlot *>(p);
    p += al256(sizeof(HistGradSlot) * I);
    int32_t *d_lev = reinterpret_cast<int32_t *>(p);
    p += al256(4 * lvcap);
    double *d_w = reinterpret_cast<double *>(p);
    p += al256(8 * lvcap);
    double *d_beta = reinterpret_cast<double *>(p);
    p += al256(ang);
    double *d_gamma = reinterpret_cast<double *>(p);
    p += al256(ang);
    double *d_psol = reinterpret_cast<double *>(p);
    p += al256(8 * I);
    double *d_db = reinterpret_cast<double *>(p);
    p += al256(ang);
    double *d_dg = reinterpret_cast<double *>(p);

    GQ_HIP(hipMemcpyAsync(d_slots, slots.data(), sizeof(HistGradSlot) * slots.size(), hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(d_lev, lev.data(), 4 * lev.size(), hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(d_w, w.data(), 8 * w.size(), hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(d_beta, beta, ang, hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(d_gamma, gamma, ang, hipMemcpyHostToDevice, st));
    for (int gi = 0; gi < 3; ++gi) {
        const int ns = first[gi + 1] - first[gi];
        if (!ns) continue;
        HistGradArgs a{d_slots + first[gi], ns, d_lev, d_w, d_beta, d_gamma, pstride, d_psol, d_db, d_dg};
        const dim3 grid((unsigned)((ns + kGradWaves - 1) / kGradWaves)), block(64 * kGradWaves);
        if (gi == 0)
            hipLaunchKernelGGL(hist_grad_kernel<1>, grid, block, 0, st, a);
        else if (gi == 1)
            hipLaunchKernelGGL(hist_grad_kernel<2>, grid, block, 0, st, a);
        else
            hipLaunchKernelGGL(hist_grad_kernel<4>, grid, block, 0, st, a);
        GQ_LAUNCH_CHECK();
    }
    if (psol) GQ_HIP(hipMemcpyAsync(psol, d_psol, 8 * I, hipMemcpyDeviceToHost, st));
    if (dbeta) GQ_HIP(hipMemcpyAsync(dbeta, d_db, ang, hipMemcpyDeviceToHost, st));
    if (dgamma) GQ_HIP(hipMemcpyAsync(dgamma, d_dg, ang, hipMemcpyDeviceToHost, st));
    GQ_HIP(hipStreamSynchronize(st));  // host tables above and the outputs
    return GQAOA_OK;
}

}  // namespace gqaoa

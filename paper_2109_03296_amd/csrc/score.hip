// Targeted evaluation (Section 3, 3.1) of an explicit list of linear
// trajectories with real-valued starts: the search's filtered likelihood at
// the pixels a trajectory crosses.  One lane per trajectory; the per-epoch
// sample, the sigma_G cut and the sums use the same device code and the
// same operation order as the search kernels, so an integer start on a grid
// velocity reproduces the search's slot bit for bit.
#include <algorithm>

#include "search_kernels.h"

namespace kbm {
namespace {

struct ScoreArgs {
    const float *psi;
    const float *phi;
    const float4 *params;  // [n] (x0, y0, vx, vy)
    float *lh;
    float *flux;
    uint64_t *keep;
    int16_t *nobs;
    float *lh_raw;
    int64_t n;
    int W, H, T, min_obs, sigmag;
    float coeff, n_sigma;
    RankTable rt;
    double t[KBM_MAX_EPOCHS];  // t_i - min_j t_j
};

template <int TM>
__global__ __launch_bounds__(256) void score_kernel(ScoreArgs a) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const float4 p = a.params[j];
    const size_t plane = (size_t)a.W * a.H;
    float nu[TM], s[TM];
    int nv = 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        nu[i] = INFINITY;  // padding sorts last
        s[i] = 0.0f;
        if (i < a.T) {
            const double t = a.t[i];
            const double fx = floor((double)p.x + (double)p.z * t + 0.5);
            const double fy = floor((double)p.y + (double)p.w * t + 0.5);
            nu[i] = __builtin_nanf("");
            if (fx >= 0.0 && fx < (double)a.W && fy >= 0.0 && fy < (double)a.H) {
                const size_t q = (size_t)i * plane + (size_t)fy * a.W + (size_t)fx;
                bool bad = false;
                const float2 v = srch::pack_sample(a.psi[q], a.phi[q], bad);
                if (!bad) {
                    nu[i] = v.x;
                    s[i] = v.y;
                    ++nv;
                }
            }
        }
    }
    float P = 0.0f, F = 0.0f, Pr = 0.0f, Fr = 0.0f;
    uint32_t lo = 0, hi = 0;
    SigmaGCut cut{0.0f, INFINITY};
    if (a.sigmag && nv > 0)
        cut = sigmag_cut<TM, true>(nu, a.rt.lo[nv], a.rt.md[nv], a.rt.hi[nv], a.coeff,
                                   a.n_sigma);
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        if (i < a.T) {
            const bool ok = nu[i] == nu[i];
            const bool k = ok && (!a.sigmag || cut.keeps(nu[i]));
            P = fmaf(k ? nu[i] : 0.0f, s[i], P);
            F = fmaf(k ? s[i] : 0.0f, s[i], F);
            Pr = fmaf(ok ? nu[i] : 0.0f, s[i], Pr);
            Fr = fmaf(s[i], s[i], Fr);
            if (i < 32)
                lo |= k ? (1u << i) : 0u;
            else
                hi |= k ? (1u << (i - 32)) : 0u;
        }
    }
    const float L = srch::lh_value(P, F);
    a.nobs[j] = (int16_t)nv;
    if (nv >= a.min_obs && nv > 0 && isfinite(L)) {
        a.lh[j] = L;
        a.flux[j] = P / F;
        a.keep[j] = (uint64_t)lo | ((uint64_t)hi << 32);
        if (a.lh_raw) a.lh_raw[j] = srch::lh_value(Pr, Fr);
    } else {
        a.lh[j] = -INFINITY;
        a.flux[j] = 0.0f;
        a.keep[j] = 0;
        if (a.lh_raw) a.lh_raw[j] = -INFINITY;
    }
}

template <int TM>
void launch_score(const ScoreArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL((score_kernel<TM>), dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0,
                       stream, a);
}

}  // namespace
}  // namespace kbm

extern "C" kbm_status kbm_score_trajectories(const kbm_stack *s, const float *psi,
                                             const float *phi, int64_t n,
                                             const float *params, int32_t min_obs,
                                             int32_t sigmag, double q_lo, double q_hi,
                                             double coeff, double n_sigma, float *lh,
                                             float *flux, uint64_t *keep, int16_t *n_obs,
                                             float *lh_raw, hipStream_t stream) {
    using namespace kbm;
    clear_error();
    kbm_status st = check_stack(s, "kbm_score_trajectories");
    if (st != KBM_OK) return st;
    KBM_REQUIRE(n >= 0, KBM_ERR_INVALID_ARG, "kbm_score_trajectories: n = %lld < 0",
                (long long)n);
    KBM_REQUIRE(min_obs >= 1, KBM_ERR_INVALID_ARG,
                "kbm_score_trajectories: min_obs = %d must be >= 1", min_obs);
    KBM_REQUIRE(sigmag == 0 || sigmag == 1, KBM_ERR_INVALID_ARG,
                "kbm_score_trajectories: sigmag must be 0 or 1");
    st = check_sigmag_params(q_lo, q_hi, coeff, n_sigma);
    if (st != KBM_OK) return st;
    if (n == 0) return KBM_OK;
    KBM_REQUIRE(psi && phi && params && lh && flux && keep && n_obs, KBM_ERR_INVALID_ARG,
                "kbm_score_trajectories: arrays must be non-NULL");
    KBM_REQUIRE(n < ((int64_t)1 << 40), KBM_ERR_UNSUPPORTED,
                "kbm_score_trajectories: n too large");
    KBM_REQUIRE(((uintptr_t)params & 15) == 0, KBM_ERR_INVALID_ARG,
                "kbm_score_trajectories: params must be 16-byte aligned");
    ScoreArgs a{};
    a.psi = psi;
    a.phi = phi;
    a.params = reinterpret_cast<const float4 *>(params);
    a.lh = lh;
    a.flux = flux;
    a.keep = keep;
    a.nobs = n_obs;
    a.lh_raw = lh_raw;
    a.n = n;
    a.W = s->width;
    a.H = s->height;
    a.T = s->num_epochs;
    a.min_obs = min_obs;
    a.sigmag = sigmag;
    a.coeff = (float)coeff;
    a.n_sigma = (float)n_sigma;
    a.rt = make_rank_table(q_lo, q_hi);
    double t0 = s->times[0];
    for (int i = 1; i < a.T; ++i) t0 = std::min(t0, s->times[i]);
    for (int i = 0; i < a.T; ++i) a.t[i] = s->times[i] - t0;
    if (a.T <= 16)
        launch_score<16>(a, stream);
    else if (a.T <= 32)
        launch_score<32>(a, stream);
    else
        launch_score<64>(a, stream);
    KBM_LAUNCHED("score_kernel");
    return KBM_OK;
}

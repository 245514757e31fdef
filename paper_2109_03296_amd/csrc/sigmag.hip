// Standalone sigma_G lightcurve filter (Section 3.1, Eqs. 1-5) over n
// independent lightcurves, one lane per lightcurve.  Same rule, ranks and
// binary32 decision as the filter fused into the search kernel (the device
// code is shared through kbm_internal.h).
#include "kbm_internal.h"

namespace kbm {
namespace {

template <int TM>
__global__ __launch_bounds__(256) void sigmag_kernel(
    const float *__restrict__ psi, const float *__restrict__ phi,
    const uint8_t *__restrict__ valid, int64_t n, int T, RankTable rt,
    float coeff, float n_sigma, uint64_t *__restrict__ keep,
    float *__restrict__ lh) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    float ps[TM], ph[TM], nu[TM];
    int nv = 0;
    const int64_t row = c * T;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        ps[i] = 0.0f;
        ph[i] = 0.0f;
        nu[i] = i < T ? __builtin_nanf("") : INFINITY;
        if (i < T) {
            const float a = psi[row + i];
            const float b = phi ? phi[row + i] : 1.0f;
            const bool ok = (valid == nullptr || valid[row + i] != 0) &&
                            b > 0.0f && isfinite(b) && isfinite(a);
            if (ok) {
                ps[i] = a;
                ph[i] = b;
                nu[i] = a / sqrtf(b);
                ++nv;
            }
        }
    }
    if (nv == 0) {
        keep[c] = 0;
        if (lh) lh[c] = -INFINITY;
        return;
    }
    const SigmaGCut cut = sigmag_cut<TM, true>(nu, rt.lo[nv], rt.md[nv], rt.hi[nv], coeff, n_sigma);
    float P = 0.0f, F = 0.0f;
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        if (i < T) {
            const bool k = cut.keeps(nu[i]);
            P += k ? ps[i] : 0.0f;
            F += k ? ph[i] : 0.0f;
            if (i < 32)
                lo |= k ? (1u << i) : 0u;
            else
                hi |= k ? (1u << (i - 32)) : 0u;
        }
    }
    keep[c] = (uint64_t)lo | ((uint64_t)hi << 32);
    if (lh) lh[c] = P / sqrtf(F);
}

template <int TM>
void launch(const float *psi, const float *phi, const uint8_t *valid,
            int64_t n, int T, const RankTable &rt, float coeff, float ns,
            uint64_t *keep, float *lh, hipStream_t stream) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL((sigmag_kernel<TM>), dim3((unsigned)blocks), dim3(256),
                       0, stream, psi, phi, valid, n, T, rt, coeff, ns, keep,
                       lh);
}

}  // namespace
}  // namespace kbm

extern "C" kbm_status kbm_sigmag_filter(const float *psi_curve,
                                        const float *phi_curve,
                                        const uint8_t *valid, int64_t n,
                                        int32_t T, double q_lo, double q_hi,
                                        double coeff, double n_sigma,
                                        uint64_t *keep, float *lh_filtered,
                                        hipStream_t stream) {
    using namespace kbm;
    clear_error();
    KBM_REQUIRE(n >= 0, KBM_ERR_INVALID_ARG,
                "kbm_sigmag_filter: n = %lld must be >= 0", (long long)n);
    KBM_REQUIRE(T >= 1 && T <= KBM_MAX_EPOCHS, KBM_ERR_INVALID_ARG,
                "kbm_sigmag_filter: T = %d not in [1, %d]", T, KBM_MAX_EPOCHS);
    kbm_status st = check_sigmag_params(q_lo, q_hi, coeff, n_sigma);
    if (st != KBM_OK) return st;
    KBM_REQUIRE(n == 0 || (psi_curve != nullptr && keep != nullptr),
                KBM_ERR_INVALID_ARG,
                "kbm_sigmag_filter: psi_curve and keep must be non-NULL");
    KBM_REQUIRE((n + 255) / 256 < ((int64_t)1 << 31), KBM_ERR_UNSUPPORTED,
                "kbm_sigmag_filter: n = %lld too large", (long long)n);
    if (n == 0) return KBM_OK;
    const RankTable rt = make_rank_table(q_lo, q_hi);
    const float c = (float)coeff, ns = (float)n_sigma;
    if (T <= 8) launch<8>(psi_curve, phi_curve, valid, n, T, rt, c, ns, keep, lh_filtered, stream);
    else if (T <= 16) launch<16>(psi_curve, phi_curve, valid, n, T, rt, c, ns, keep, lh_filtered, stream);
    else if (T <= 24) launch<24>(psi_curve, phi_curve, valid, n, T, rt, c, ns, keep, lh_filtered, stream);
    else if (T <= 32) launch<32>(psi_curve, phi_curve, valid, n, T, rt, c, ns, keep, lh_filtered, stream);
    else if (T <= 48) launch<48>(psi_curve, phi_curve, valid, n, T, rt, c, ns, keep, lh_filtered, stream);
    else launch<64>(psi_curve, phi_curve, valid, n, T, rt, c, ns, keep, lh_filtered, stream);
    KBM_LAUNCHED("sigmag_kernel");
    return KBM_OK;
}

// Standalone sigma_G lightcurve filter (Section 3.1, Eqs. 1-5) over n
// independent lightcurves, one lane per lightcurve (rows staged through
// LDS, below).  Same rule, ranks and
// binary32 decision as the filter fused into the search kernel (the device
// code is shared through kbm_internal.h).  The filtered per-epoch value is
// the likelihood psi/sqrt(phi) or, as a variant the paper allows, the flux
// psi/phi; a post-filter flag marks curves whose recomputed likelihood
// reaches a threshold.
#include "kbm_internal.h"

namespace kbm {
namespace {

// One 64-lane workgroup per 64 lightcurves.  Their rows are contiguous in
// memory ([n][T]), so the workgroup first copies the whole 64 x T block of
// psi, phi and the validity flags into LDS with coalesced loads (lane j
// reads elements j, j + 64, ...), then each lane reads its own row from LDS
// (row stride T rounded up to odd, so the 64 lanes hit 64 different banks).
// Reading the rows directly would make every load instruction touch up to
// 64 different cache lines.  All of a lane's loads are issued before the
// first LDS write, so the block's memory latency is paid once, not once per
// element.
constexpr int SG_LANES = 64;

template <int TM>
__global__ __launch_bounds__(SG_LANES) void sigmag_kernel(
    const float *__restrict__ psi, const float *__restrict__ phi,
    const uint8_t *__restrict__ valid, int64_t n, int T, int quantity, RankTable rt,
    float coeff, float n_sigma, float lh_min, uint64_t *__restrict__ keep,
    float *__restrict__ lh, uint8_t *__restrict__ pass, int vec) {
    constexpr int RS = TM | 1;  // LDS row stride (odd)
    __shared__ float s_ps[SG_LANES * RS];
    __shared__ float s_ph[SG_LANES * RS];
    __shared__ uint8_t s_ok[SG_LANES * RS];
    const int64_t c0 = (int64_t)blockIdx.x * SG_LANES;
    const int rows = (int)min((int64_t)SG_LANES, n - c0);
    const int64_t base = c0 * T;
    const int count = rows * T;  // <= SG_LANES * TM
    const int lane = threadIdx.x;
    if (vec) {
        // 16-byte loads: each workgroup's block starts 16-byte aligned (64 T
        // floats and 64 T flag bytes from 16-byte aligned arrays).  For
        // k = 0, 1, ... the lane takes the q-th float4 (floats 4q .. 4q+3) and
        // the q-th 16-byte group of flags of the block, q = k * 64 + lane;
        // the last count % 4 floats and count % 16 flags are read one by one.
        constexpr int NF = TM / 4;
        constexpr int NB = TM >= 16 ? TM / 16 : 1;
        const int n4 = count >> 2, n16 = count >> 4;
        const float4 *p4 = reinterpret_cast<const float4 *>(psi + base);
        const float4 *f4 = phi ? reinterpret_cast<const float4 *>(phi + base) : nullptr;
        const uint4 *v16 = valid ? reinterpret_cast<const uint4 *>(valid + base) : nullptr;
        float4 va[NF], vb[NF];
        uint4 vc[NB];
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            const int q = k * SG_LANES + lane;
            va[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            vb[k] = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
            if (q < n4) {
                va[k] = p4[q];
                if (f4) vb[k] = f4[q];
            }
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const int q = k * SG_LANES + lane;
            vc[k] = make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
            if (v16 && q < n16) vc[k] = v16[q];
        }
        const int tf = 4 * n4 + lane, tb = 16 * n16 + lane;
        float xa = 0.0f, xb = 1.0f;
        uint32_t xc = 1u;
        if (tf < count) {
            xa = psi[base + tf];
            if (phi) xb = phi[base + tf];
        }
        if (tb < count && valid) xc = valid[base + tb];
        // Scatter into the padded rows; (r, i) is stepped without division.
        int r = (4 * lane) / T, i = 4 * lane - r * T;
        int dr = (4 * SG_LANES) / T, di = 4 * SG_LANES - dr * T;
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            if (k * SG_LANES + lane < n4) {
                const float a4[4] = {va[k].x, va[k].y, va[k].z, va[k].w};
                const float b4[4] = {vb[k].x, vb[k].y, vb[k].z, vb[k].w};
                int rr = r, ii = i;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    s_ps[rr * RS + ii] = a4[e];
                    s_ph[rr * RS + ii] = b4[e];
                    if (++ii == T) {
                        ii = 0;
                        ++rr;
                    }
                }
            }
            r += dr;
            i += di;
            if (i >= T) {
                i -= T;
                ++r;
            }
        }
        r = (16 * lane) / T;
        i = 16 * lane - r * T;
        dr = (16 * SG_LANES) / T;
        di = 16 * SG_LANES - dr * T;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (k * SG_LANES + lane < n16) {
                const uint32_t w4[4] = {vc[k].x, vc[k].y, vc[k].z, vc[k].w};
                int rr = r, ii = i;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    s_ok[rr * RS + ii] = (uint8_t)(w4[e / 4] >> (8 * (e % 4)));
                    if (++ii == T) {
                        ii = 0;
                        ++rr;
                    }
                }
            }
            r += dr;
            i += di;
            while (i >= T) {
                i -= T;
                ++r;
            }
        }
        if (tf < count) {
            const int rt = tf / T;
            s_ps[rt * RS + (tf - rt * T)] = xa;
            s_ph[rt * RS + (tf - rt * T)] = xb;
        }
        if (tb < count) {
            const int rt = tb / T;
            s_ok[rt * RS + (tb - rt * T)] = (uint8_t)xc;
        }
    } else {
        float ga[TM], gb[TM];
        uint32_t gc[TM];
#pragma unroll
        for (int k = 0; k < TM; ++k) {
            const int j = k * SG_LANES + lane;
            ga[k] = 0.0f;
            gb[k] = 1.0f;
            gc[k] = 1u;
            if (j < count) {
                ga[k] = psi[base + j];
                if (phi) gb[k] = phi[base + j];
                if (valid) gc[k] = valid[base + j];
            }
        }
        // Row and column of element k * SG_LANES + lane, stepped without division.
        int r = lane / T, i = lane - r * T;
        const int dr = SG_LANES / T, di = SG_LANES - dr * T;
#pragma unroll
        for (int k = 0; k < TM; ++k) {
            if (k * SG_LANES + lane < count) {
                s_ps[r * RS + i] = ga[k];
                s_ph[r * RS + i] = gb[k];
                s_ok[r * RS + i] = (uint8_t)gc[k];
            }
            r += dr;
            i += di;
            if (i >= T) {
                i -= T;
                ++r;
            }
        }
    }
    __syncthreads();
    const int l = lane;
    if (l >= rows) return;
    const int64_t c = c0 + l;
    float ps[TM], ph[TM], nu[TM];
    int nv = 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        ps[i] = 0.0f;
        ph[i] = 0.0f;
        nu[i] = i < T ? __builtin_nanf("") : INFINITY;
        if (i < T) {
            const float a = s_ps[l * RS + i];
            const float b = s_ph[l * RS + i];
            const bool ok = s_ok[l * RS + i] != 0 && b > 0.0f && isfinite(b) && isfinite(a);
            if (ok) {
                ps[i] = a;
                ph[i] = b;
                nu[i] = quantity ? a / b : a / sqrtf(b);
                ++nv;
            }
        }
    }
    if (nv == 0) {
        keep[c] = 0;
        if (lh) lh[c] = -INFINITY;
        if (pass) pass[c] = 0;
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
    const float L = P / sqrtf(F);
    if (lh) lh[c] = L;
    if (pass) pass[c] = L >= lh_min ? 1 : 0;
}

template <int TM>
void launch(const float *psi, const float *phi, const uint8_t *valid,
            int64_t n, int T, int quantity, const RankTable &rt, float coeff, float ns,
            float lh_min, uint64_t *keep, float *lh, uint8_t *pass, hipStream_t stream) {
    const int64_t blocks = (n + SG_LANES - 1) / SG_LANES;
    const int vec = (((uintptr_t)psi | (uintptr_t)phi | (uintptr_t)valid) & 15u) == 0;
    hipLaunchKernelGGL((sigmag_kernel<TM>), dim3((unsigned)blocks), dim3(SG_LANES),
                       0, stream, psi, phi, valid, n, T, quantity, rt, coeff, ns, lh_min,
                       keep, lh, pass, vec);
}

}  // namespace
}  // namespace kbm

extern "C" kbm_status kbm_sigmag_filter_ex(const float *psi_curve, const float *phi_curve,
                                           const uint8_t *valid, int64_t n, int32_t T,
                                           int32_t quantity, double q_lo, double q_hi,
                                           double coeff, double n_sigma, double lh_min,
                                           uint64_t *keep, float *lh_filtered,
                                           uint8_t *pass, hipStream_t stream) {
    using namespace kbm;
    clear_error();
    KBM_REQUIRE(n >= 0, KBM_ERR_INVALID_ARG,
                "kbm_sigmag_filter: n = %lld must be >= 0", (long long)n);
    KBM_REQUIRE(T >= 1 && T <= KBM_MAX_EPOCHS, KBM_ERR_INVALID_ARG,
                "kbm_sigmag_filter: T = %d not in [1, %d]", T, KBM_MAX_EPOCHS);
    KBM_REQUIRE(quantity == 0 || quantity == 1, KBM_ERR_INVALID_ARG,
                "kbm_sigmag_filter: quantity = %d must be 0 (likelihood) or 1 (flux)",
                quantity);
    KBM_REQUIRE(!std::isnan(lh_min), KBM_ERR_INVALID_ARG, "kbm_sigmag_filter: lh_min is NaN");
    kbm_status st = check_sigmag_params(q_lo, q_hi, coeff, n_sigma);
    if (st != KBM_OK) return st;
    KBM_REQUIRE(n == 0 || (psi_curve != nullptr && keep != nullptr),
                KBM_ERR_INVALID_ARG,
                "kbm_sigmag_filter: psi_curve and keep must be non-NULL");
    KBM_REQUIRE((n + 63) / 64 < ((int64_t)1 << 31), KBM_ERR_UNSUPPORTED,
                "kbm_sigmag_filter: n = %lld too large", (long long)n);
    if (n == 0) return KBM_OK;
    const RankTable rt = make_rank_table(q_lo, q_hi);
    const float c = (float)coeff, ns = (float)n_sigma, lm = (float)lh_min;
#define KBM_SG_LAUNCH(TM) \
    launch<TM>(psi_curve, phi_curve, valid, n, T, quantity, rt, c, ns, lm, keep, lh_filtered, \
               pass, stream)
    if (T <= 8) KBM_SG_LAUNCH(8);
    else if (T <= 16) KBM_SG_LAUNCH(16);
    else if (T <= 24) KBM_SG_LAUNCH(24);
    else if (T <= 32) KBM_SG_LAUNCH(32);
    else if (T <= 48) KBM_SG_LAUNCH(48);
    else KBM_SG_LAUNCH(64);
#undef KBM_SG_LAUNCH
    KBM_LAUNCHED("sigmag_kernel");
    return KBM_OK;
}

extern "C" kbm_status kbm_sigmag_filter(const float *psi_curve,
                                        const float *phi_curve,
                                        const uint8_t *valid, int64_t n,
                                        int32_t T, double q_lo, double q_hi,
                                        double coeff, double n_sigma,
                                        uint64_t *keep, float *lh_filtered,
                                        hipStream_t stream) {
    return kbm_sigmag_filter_ex(psi_curve, phi_curve, valid, n, T, 0, q_lo, q_hi, coeff,
                                n_sigma, -INFINITY, keep, lh_filtered, nullptr, stream);
}

// Median coadded postage stamps along trajectories and their central-moment
// cut (Section 3.3).  One workgroup per trajectory, one lane per stamp
// pixel: the lane gathers its pixel from the T epochs (coalesced along stamp
// rows), takes the median of the usable values with the sorting network the
// sigma_G filter uses, and the workgroup reduces the six moment sums in
// FP64 (shuffles within a wave, then LDS across waves).
#include <algorithm>
#include <cmath>

#include "kbm_internal.h"

namespace kbm {
namespace {

constexpr int SWAVE = 64;
constexpr int MAX_R = 15;
constexpr int MAX_WAVES = ((2 * MAX_R + 1) * (2 * MAX_R + 1) + SWAVE - 1) / SWAVE;

struct StampArgs {
    const float *sci;
    const float *var;
    const uint8_t *mask;
    const float4 *params;  // [n] (x0, y0, vx, vy)
    const uint64_t *keep;
    float *coadd;          // [n][k][k] or null
    double *moments;       // [n][6]
    uint8_t *pass;         // [n]
    int64_t n;
    int W, H, T, r, k;
    double lim[5];         // |x|, |y|, |xy|, xx, yy
    double t[KBM_MAX_EPOCHS];
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = SWAVE / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, SWAVE);
    return v;
}

template <int TM>
__global__ __launch_bounds__(1024) void stamp_kernel(StampArgs a) {
    __shared__ double part[6][MAX_WAVES];
    const int64_t j = blockIdx.x;
    const float4 p = a.params[j];
    const uint64_t kp = a.keep ? a.keep[j] : ~0ull;
    const int kk = a.k * a.k;
    const int tid = threadIdx.x;
    const bool act = tid < kk;
    const int dy = act ? tid / a.k - a.r : 0, dx = act ? tid % a.k - a.r : 0;
    const size_t plane = (size_t)a.W * a.H;
    float v[TM];
    int nv = 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        v[i] = INFINITY;  // unusable and padding sort last
        if (i < a.T && ((kp >> i) & 1)) {
            const double t = a.t[i];
            const double cx = floor((double)p.x + (double)p.z * t + 0.5);
            const double cy = floor((double)p.y + (double)p.w * t + 0.5);
            const double x = cx + dx, y = cy + dy;
            if (act && x >= 0.0 && x < (double)a.W && y >= 0.0 && y < (double)a.H) {
                const size_t q = (size_t)i * plane + (size_t)y * a.W + (size_t)x;
                const float s = a.sci[q], w = a.var[q];
                const bool ok = (a.mask == nullptr || a.mask[q] == 0) && isfinite(s) &&
                                isfinite(w) && w > 0.0f;
                if (ok) {
                    v[i] = s;
                    ++nv;
                }
            }
        }
    }
    sort_network<TM>(v);
    float med = 0.0f;
    if (nv > 0) {
        const float lo = select_rank<TM>(v, (nv - 1) / 2);
        const float hi = select_rank<TM>(v, nv / 2);
        med = (nv & 1) ? lo : (lo + hi) * 0.5f;
    }
    if (act && a.coadd) a.coadd[j * kk + tid] = med;
    const double m = act ? (double)med : 0.0;
    double s6[6] = {m, m * dx, m * dy, m * dx * dy, m * dx * dx, m * dy * dy};
    const int w = tid / SWAVE, lane = tid % SWAVE;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        s6[c] = wave_sum(s6[c]);
        if (lane == 0) part[c][w] = s6[c];
    }
    __syncthreads();
    if (tid != 0) return;
    const int nw = (int)((blockDim.x + SWAVE - 1) / SWAVE);
    double tot[6] = {0, 0, 0, 0, 0, 0};
    for (int ww = 0; ww < nw; ++ww)
        for (int c = 0; c < 6; ++c) tot[c] += part[c][ww];
    double *mo = a.moments + j * 6;
    mo[0] = tot[0];
    bool ok = tot[0] > 0.0;
    for (int c = 1; c < 6; ++c) mo[c] = ok ? tot[c] / tot[0] : NAN;
    ok = ok && fabs(mo[1]) < a.lim[0] && fabs(mo[2]) < a.lim[1] && fabs(mo[3]) < a.lim[2] &&
         mo[4] < a.lim[3] && mo[5] < a.lim[4];
    a.pass[j] = ok ? 1 : 0;
}

template <int TM>
void launch_stamps(const StampArgs &a, hipStream_t stream) {
    const int threads = ((a.k * a.k + SWAVE - 1) / SWAVE) * SWAVE;
    hipLaunchKernelGGL((stamp_kernel<TM>), dim3((unsigned)a.n), dim3(threads), 0, stream, a);
}

}  // namespace
}  // namespace kbm

extern "C" kbm_status kbm_stamps(const kbm_stack *s, const float *sci, const float *var,
                                 const uint8_t *mask, int64_t n, const float *params,
                                 const uint64_t *keep, int32_t radius, const double *limits,
                                 float *coadd, double *moments, uint8_t *pass,
                                 hipStream_t stream) {
    using namespace kbm;
    clear_error();
    kbm_status st = check_stack(s, "kbm_stamps");
    if (st != KBM_OK) return st;
    KBM_REQUIRE(n >= 0 && n < ((int64_t)1 << 31), KBM_ERR_INVALID_ARG,
                "kbm_stamps: n = %lld not in [0, 2^31)", (long long)n);
    KBM_REQUIRE(radius >= 1 && radius <= MAX_R, KBM_ERR_INVALID_ARG,
                "kbm_stamps: radius = %d not in [1, %d]", radius, MAX_R);
    double lim[5] = {0.5, 0.5, 1.5, 36.5, 36.5};
    if (limits)
        for (int c = 0; c < 5; ++c) {
            KBM_REQUIRE(std::isfinite(limits[c]), KBM_ERR_INVALID_ARG,
                        "kbm_stamps: limit %d is not finite", c);
            lim[c] = limits[c];
        }
    if (n == 0) return KBM_OK;
    KBM_REQUIRE(sci && var && params && moments && pass, KBM_ERR_INVALID_ARG,
                "kbm_stamps: sci, var, params, moments and pass must be non-NULL");
    KBM_REQUIRE(((uintptr_t)params & 15) == 0, KBM_ERR_INVALID_ARG,
                "kbm_stamps: params must be 16-byte aligned");
    StampArgs a{};
    a.sci = sci;
    a.var = var;
    a.mask = mask;
    a.params = reinterpret_cast<const float4 *>(params);
    a.keep = keep;
    a.coadd = coadd;
    a.moments = moments;
    a.pass = pass;
    a.n = n;
    a.W = s->width;
    a.H = s->height;
    a.T = s->num_epochs;
    a.r = radius;
    a.k = 2 * radius + 1;
    for (int c = 0; c < 5; ++c) a.lim[c] = lim[c];
    double t0 = s->times[0];
    for (int i = 1; i < a.T; ++i) t0 = std::min(t0, s->times[i]);
    for (int i = 0; i < a.T; ++i) a.t[i] = s->times[i] - t0;
    if (a.T <= 16)
        launch_stamps<16>(a, stream);
    else if (a.T <= 32)
        launch_stamps<32>(a, stream);
    else
        launch_stamps<64>(a, stream);
    KBM_LAUNCHED("stamp_kernel");
    return KBM_OK;
}

// Decision of the targeted mode: enough usable epochs, filtered likelihood
// at least lh_min (NaN never passes), stamp passes the moment cut.
namespace kbm {
namespace {
__global__ __launch_bounds__(256) void detect_kernel(int64_t n, const float *lh,
                                                     const int16_t *n_obs,
                                                     const uint8_t *stamp_pass, int min_obs,
                                                     float lh_min, uint8_t *detected) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    detected[j] = (n_obs[j] >= min_obs && lh[j] >= lh_min && stamp_pass[j] != 0) ? 1 : 0;
}
}  // namespace
}  // namespace kbm

extern "C" kbm_status kbm_detect(int64_t n, const float *lh, const int16_t *n_obs,
                                 const uint8_t *stamp_pass, int32_t min_obs, float lh_min,
                                 uint8_t *detected, hipStream_t stream) {
    using namespace kbm;
    clear_error();
    KBM_REQUIRE(n >= 0 && n < ((int64_t)1 << 40), KBM_ERR_INVALID_ARG,
                "kbm_detect: n = %lld out of range", (long long)n);
    KBM_REQUIRE(n == 0 || (lh && n_obs && stamp_pass && detected), KBM_ERR_INVALID_ARG,
                "kbm_detect: arrays must be non-NULL");
    KBM_REQUIRE(!std::isnan(lh_min), KBM_ERR_INVALID_ARG, "kbm_detect: lh_min is NaN");
    if (n == 0) return KBM_OK;
    hipLaunchKernelGGL(detect_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       n, lh, n_obs, stamp_pass, (int)min_obs, lh_min, detected);
    KBM_LAUNCHED("detect_kernel");
    return KBM_OK;
}

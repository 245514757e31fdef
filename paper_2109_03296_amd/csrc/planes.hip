// Likelihood planes psi/phi (Section 3): correlation of I*w with the PSF
// and of w with PSF^2, w = inverse variance or 0 for masked/unusable pixels.
//
// One workgroup computes a 64 x 16 output tile of one epoch.  The tile and
// its PSF halo of u = I*w and w are staged in LDS once (each input pixel is
// read from HBM once per tile, the weight is computed once), then every
// thread evaluates four outputs from LDS.  HBM traffic per pixel-epoch is
// the algorithmic 9 B in (sci, var, mask) + 8 B out (psi, phi) plus the
// halo re-reads of neighbouring tiles.
//
// A PSF that is an outer product P[b][a] = c_b r_a (a sampled Gaussian is)
// takes a two-pass path: a horizontal pass over the staged rows (with r and
// r^2) into LDS, then a vertical pass (with c and c^2), 2k + 2k(1 + 2r/16)
// multiply-adds per output instead of 2k^2.  The factors come from the
// caller's PSF (checked to reproduce it to 1e-6 of its largest tap) and sit
// in kernel arguments, i.e. scalar registers.
#include <algorithm>
#include <cmath>

#include "kbm_internal.h"

namespace kbm {
namespace {

constexpr int TILE_X = 64;
constexpr int TILE_Y = 16;
constexpr int THREADS = 256;
constexpr int MAX_R = (KBM_MAX_PSF - 1) / 2;
constexpr int LDS_W = TILE_X + 2 * MAX_R;
constexpr int LDS_H = TILE_Y + 2 * MAX_R;

// PSF rows b0 .. b0+nb-1 of one launch, in kernel arguments.  The direct
// kernel takes at most PSF_ARG_MAX taps per launch (kernel arguments stay
// well under 4 KB); a wider PSF is applied in two launches over row ranges,
// the second adding its partial sums to the first's.
constexpr int PSF_ARG_MAX = 640;
struct PsfArg {
    float p[PSF_ARG_MAX];
};

__global__ __launch_bounds__(THREADS) void planes_kernel(
    const float *__restrict__ sci, const float *__restrict__ var,
    const uint8_t *__restrict__ mask, float *__restrict__ psi,
    float *__restrict__ phi, int W, int H, int k, int b0, int nb, int accumulate,
    PsfArg psf) {
    __shared__ float s_u[LDS_H * LDS_W];
    __shared__ float s_w[LDS_H * LDS_W];
    __shared__ float s_p[PSF_ARG_MAX];
    __shared__ float s_p2[PSF_ARG_MAX];

    const int r = k / 2;
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * TILE_X;
    const int y0 = blockIdx.y * TILE_Y;
    const size_t plane = (size_t)blockIdx.z * ((size_t)W * H);
    const int lw = TILE_X + 2 * r, lh = TILE_Y + 2 * r;

    for (int j = tid; j < nb * k; j += THREADS) {
        const float p = psf.p[j];
        s_p[j] = p;
        s_p2[j] = p * p;
    }
    for (int j = tid; j < lw * lh; j += THREADS) {
        const int ly = j / lw, lx = j - ly * lw;
        const int gx = x0 - r + lx, gy = y0 - r + ly;
        float u = 0.0f, w = 0.0f;
        if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
            const size_t q = plane + (size_t)gy * W + gx;
            const float I = sci[q], v = var[q];
            const bool masked = mask != nullptr && mask[q] != 0;
            const bool ok = !masked && isfinite(I) && isfinite(v) && v > 0.0f;
            w = ok ? 1.0f / v : 0.0f;
            u = ok ? I * w : 0.0f;
        }
        s_u[ly * LDS_W + lx] = u;
        s_w[ly * LDS_W + lx] = w;
    }
    __syncthreads();

    const int tx = tid % TILE_X;
    const int ty = tid / TILE_X;
    const int x = x0 + tx;
    if (x >= W) return;
#pragma unroll
    for (int s = 0; s < TILE_Y / (THREADS / TILE_X); ++s) {
        const int ly = ty + s * (THREADS / TILE_X);
        const int y = y0 + ly;
        if (y >= H) break;
        float a_psi = 0.0f, a_phi = 0.0f;
        for (int b = 0; b < nb; ++b) {
            const float *ru = s_u + (ly + b0 + b) * LDS_W + tx;
            const float *rw = s_w + (ly + b0 + b) * LDS_W + tx;
            const float *pp = s_p + b * k;
            const float *pp2 = s_p2 + b * k;
            for (int a = 0; a < k; ++a) {
                a_psi = fmaf(pp[a], ru[a], a_psi);
                a_phi = fmaf(pp2[a], rw[a], a_phi);
            }
        }
        const size_t o = plane + (size_t)y * W + x;
        if (accumulate) {
            a_psi += psi[o];
            a_phi += phi[o];
        }
        psi[o] = a_psi;
        phi[o] = a_phi;
    }
}

struct SepArg {
    float c[KBM_MAX_PSF], c2[KBM_MAX_PSF];  // column factor (rows b), squared
    float r[KBM_MAX_PSF], r2[KBM_MAX_PSF];  // row factor (columns a), squared
};

template <int K>
__global__ __launch_bounds__(THREADS) void planes_sep_kernel(
    const float *__restrict__ sci, const float *__restrict__ var,
    const uint8_t *__restrict__ mask, float *__restrict__ psi,
    float *__restrict__ phi, int W, int H, SepArg f) {
    constexpr int R = K / 2;
    constexpr int LW = TILE_X + 2 * R, LH = TILE_Y + 2 * R;
    __shared__ float s_u[LH * LW];
    __shared__ float s_w[LH * LW];
    __shared__ float h_u[LH * TILE_X];
    __shared__ float h_w[LH * TILE_X];

    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * TILE_X;
    const int y0 = blockIdx.y * TILE_Y;
    const size_t plane = (size_t)blockIdx.z * ((size_t)W * H);
    for (int j = tid; j < LW * LH; j += THREADS) {
        const int ly = j / LW, lx = j - ly * LW;
        const int gx = x0 - R + lx, gy = y0 - R + ly;
        float u = 0.0f, w = 0.0f;
        if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
            const size_t q = plane + (size_t)gy * W + gx;
            const float I = sci[q], v = var[q];
            const bool masked = mask != nullptr && mask[q] != 0;
            const bool ok = !masked && isfinite(I) && isfinite(v) && v > 0.0f;
            w = ok ? 1.0f / v : 0.0f;
            u = ok ? I * w : 0.0f;
        }
        s_u[j] = u;
        s_w[j] = w;
    }
    __syncthreads();
    for (int j = tid; j < LH * TILE_X; j += THREADS) {
        const int ly = j / TILE_X, lx = j - ly * TILE_X;
        const float *ru = s_u + ly * LW + lx;
        const float *rw = s_w + ly * LW + lx;
        float a_u = 0.0f, a_w = 0.0f;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            a_u = fmaf(f.r[a], ru[a], a_u);
            a_w = fmaf(f.r2[a], rw[a], a_w);
        }
        h_u[j] = a_u;
        h_w[j] = a_w;
    }
    __syncthreads();
    const int tx = tid % TILE_X;
    const int ty = tid / TILE_X;
    const int x = x0 + tx;
    if (x >= W) return;
#pragma unroll
    for (int s = 0; s < TILE_Y / (THREADS / TILE_X); ++s) {
        const int ly = ty + s * (THREADS / TILE_X);
        const int y = y0 + ly;
        if (y >= H) break;
        float a_psi = 0.0f, a_phi = 0.0f;
#pragma unroll
        for (int b = 0; b < K; ++b) {
            a_psi = fmaf(f.c[b], h_u[(ly + b) * TILE_X + tx], a_psi);
            a_phi = fmaf(f.c2[b], h_w[(ly + b) * TILE_X + tx], a_phi);
        }
        const size_t o = plane + (size_t)y * W + x;
        psi[o] = a_psi;
        phi[o] = a_phi;
    }
}

// Rank-1 factors c, r of a k x k PSF (P[b][a] = c_b r_a to within 1e-6 of
// the largest tap), or false.
bool separable(const float *psf, int k, SepArg *f) {
    int b0 = 0, a0 = 0;
    double big = 0.0;
    for (int b = 0; b < k; ++b)
        for (int a = 0; a < k; ++a)
            if (std::fabs((double)psf[b * k + a]) > big) {
                big = std::fabs((double)psf[b * k + a]);
                b0 = b;
                a0 = a;
            }
    if (!(big > 0.0)) return false;
    const double piv = psf[b0 * k + a0];
    double c[KBM_MAX_PSF], r[KBM_MAX_PSF];
    for (int b = 0; b < k; ++b) c[b] = psf[b * k + a0];
    for (int a = 0; a < k; ++a) r[a] = psf[b0 * k + a] / piv;
    for (int b = 0; b < k; ++b)
        for (int a = 0; a < k; ++a)
            if (std::fabs(c[b] * r[a] - (double)psf[b * k + a]) > 1e-6 * big) return false;
    for (int j = 0; j < k; ++j) {
        f->c[j] = (float)c[j];
        f->c2[j] = (float)(c[j] * c[j]);
        f->r[j] = (float)r[j];
        f->r2[j] = (float)(r[j] * r[j]);
    }
    return true;
}

template <int K>
void launch_sep(dim3 grid, hipStream_t stream, const float *sci, const float *var,
                const uint8_t *mask, float *psi, float *phi, int W, int H,
                const SepArg &f) {
    hipLaunchKernelGGL((planes_sep_kernel<K>), grid, dim3(THREADS), 0, stream, sci, var,
                       mask, psi, phi, W, H, f);
}

}  // namespace
}  // namespace kbm

extern "C" kbm_status kbm_make_planes(const kbm_stack *s, const float *sci,
                                      const float *var, const uint8_t *mask,
                                      const float *psf, int32_t psf_k,
                                      float *psi, float *phi,
                                      hipStream_t stream) {
    using namespace kbm;
    clear_error();
    kbm_status st = check_stack(s, "kbm_make_planes");
    if (st != KBM_OK) return st;
    KBM_REQUIRE(sci && var && psi && phi, KBM_ERR_INVALID_ARG,
                "kbm_make_planes: sci, var, psi and phi must be non-NULL");
    KBM_REQUIRE(psf != nullptr, KBM_ERR_INVALID_ARG,
                "kbm_make_planes: psf is NULL");
    KBM_REQUIRE(psf_k >= 1 && (psf_k % 2) == 1, KBM_ERR_INVALID_ARG,
                "kbm_make_planes: psf_k = %d must be odd and >= 1", psf_k);
    KBM_REQUIRE(psf_k <= KBM_MAX_PSF, KBM_ERR_UNSUPPORTED,
                "kbm_make_planes: psf_k = %d exceeds %d", psf_k, KBM_MAX_PSF);
    for (int j = 0; j < psf_k * psf_k; ++j)
        KBM_REQUIRE(std::isfinite(psf[j]), KBM_ERR_INVALID_ARG,
                    "kbm_make_planes: psf[%d] is not finite", j);

    const int W = s->width, H = s->height, T = s->num_epochs;
    dim3 grid((W + TILE_X - 1) / TILE_X, (H + TILE_Y - 1) / TILE_Y, T);
    SepArg f{};
    if (separable(psf, psf_k, &f)) {
        switch (psf_k) {
#define KBM_SEP_CASE(n) \
    case n: launch_sep<n>(grid, stream, sci, var, mask, psi, phi, W, H, f); break;
            KBM_SEP_CASE(1) KBM_SEP_CASE(3) KBM_SEP_CASE(5) KBM_SEP_CASE(7)
            KBM_SEP_CASE(9) KBM_SEP_CASE(11) KBM_SEP_CASE(13) KBM_SEP_CASE(15)
            KBM_SEP_CASE(17) KBM_SEP_CASE(19) KBM_SEP_CASE(21) KBM_SEP_CASE(23)
            KBM_SEP_CASE(25) KBM_SEP_CASE(27) KBM_SEP_CASE(29) KBM_SEP_CASE(31)
#undef KBM_SEP_CASE
        }
        KBM_LAUNCHED("planes_sep_kernel");
        return KBM_OK;
    }
    const int rows = PSF_ARG_MAX / psf_k;  // >= 20 for psf_k <= 31
    for (int b0 = 0; b0 < psf_k; b0 += rows) {
        const int nb = std::min(rows, psf_k - b0);
        PsfArg pa{};
        for (int j = 0; j < nb * psf_k; ++j) pa.p[j] = psf[b0 * psf_k + j];
        hipLaunchKernelGGL(planes_kernel, grid, dim3(THREADS), 0, stream, sci, var,
                           mask, psi, phi, W, H, (int)psf_k, b0, nb, b0 > 0 ? 1 : 0, pa);
        KBM_LAUNCHED("planes_kernel");
    }
    return KBM_OK;
}

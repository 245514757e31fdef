// Likelihood planes psi/phi (Section 3): correlation of I*w with the PSF
// and of w with PSF^2, w = inverse variance or 0 for masked/unusable pixels.
//
// A PSF that is an outer product P[b][a] = c_b r_a (a sampled Gaussian is)
// takes a two-pass path: a horizontal pass with r and r^2, then a vertical
// pass with c and c^2, 2k + 2k multiply-adds per output instead of 2k^2.
// The factors come from the caller's PSF (checked to reproduce it to 1e-6
// of its largest tap) and sit in kernel arguments, i.e. scalar registers.
// That kernel streams down strips of rows so each input pixel is read about
// once; HBM traffic per pixel-epoch is close to the algorithmic 9 B in (sci,
// var, mask) + 8 B out (psi, phi).
//
// Any other PSF takes the direct kernel: one workgroup computes a 64 x 16
// output tile of one epoch; the tile and its PSF halo of u = I*w and w are
// staged in LDS once, then every thread evaluates four outputs from LDS.
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

// Two-pass path for rank-1 PSFs, row-streaming.  A workgroup owns a strip of
// SW_COLS columns and walks SW_ROWS output rows down it: each input row is
// read once (float2 loads of two adjacent columns per thread, plus the
// 2R halo pixels of the strip by the first 2R threads), weighted, staged in
// LDS, reduced horizontally with r and r^2, and pushed into a ring of the
// last K horizontal results held in registers; from the 2R-th row on every
// step emits one output row (vertical pass with c and c^2).  Input is read
// (SW_COLS + 2R)/SW_COLS x (SW_ROWS + 2R)/SW_ROWS times, about 1.08x for
// K = 9, and output is written once.  Each output is the same chain of
// multiply-adds as a tiled two-pass kernel: horizontal over a = 0 .. K-1,
// then vertical over b = 0 .. K-1.
constexpr int SW_THREADS = 256;
constexpr int SW_COLS = 2 * SW_THREADS;
constexpr int SW_ROWS = 128;

struct RowIn {
    float I0, I1, v0, v1;
    uint32_t m;  // mask bytes of the two columns (0 = usable)
    float hI, hv;
    uint32_t hm;
};

template <bool VEC>
__device__ __forceinline__ void load_row(const float *__restrict__ sci,
                                         const float *__restrict__ var,
                                         const uint8_t *__restrict__ mask, size_t plane, int W,
                                         int H, int gy, int x, int hx, bool halo, RowIn &r) {
    r.I0 = r.I1 = r.v0 = r.v1 = 0.0f;
    r.m = 0x0101u;
    r.hI = r.hv = 0.0f;
    r.hm = 1u;
    if (gy < 0 || gy >= H) return;
    const size_t row = plane + (size_t)gy * W;
    if (VEC && x + 1 < W) {
        const float2 a = *reinterpret_cast<const float2 *>(sci + row + x);
        const float2 b = *reinterpret_cast<const float2 *>(var + row + x);
        r.I0 = a.x;
        r.I1 = a.y;
        r.v0 = b.x;
        r.v1 = b.y;
        r.m = mask ? (uint32_t)*reinterpret_cast<const uint16_t *>(mask + row + x) : 0u;
    } else {
        if (x < W) {
            r.I0 = sci[row + x];
            r.v0 = var[row + x];
            r.m = (r.m & 0xff00u) | (mask ? mask[row + x] : 0u);
        }
        if (x + 1 < W) {
            r.I1 = sci[row + x + 1];
            r.v1 = var[row + x + 1];
            r.m = (r.m & 0x00ffu) | ((mask ? (uint32_t)mask[row + x + 1] : 0u) << 8);
        }
    }
    if (halo && hx >= 0 && hx < W) {
        r.hI = sci[row + hx];
        r.hv = var[row + hx];
        r.hm = mask ? mask[row + hx] : 0u;
    }
}

// Weight of one pixel (planes' rule): usable -> (I / var, 1 / var).
__device__ __forceinline__ void weight(float I, float v, uint32_t m, float &u, float &w) {
    const bool ok = m == 0u && isfinite(I) && isfinite(v) && v > 0.0f;
    w = ok ? 1.0f / v : 0.0f;
    u = ok ? I * w : 0.0f;
}

template <int K, bool VEC>
__global__ __launch_bounds__(SW_THREADS) void planes_stream_kernel(
    const float *__restrict__ sci, const float *__restrict__ var,
    const uint8_t *__restrict__ mask, float *__restrict__ psi,
    float *__restrict__ phi, int W, int H, SepArg f) {
    constexpr int R = K / 2;
    constexpr int LW = SW_COLS + 2 * R;
    __shared__ float s_u[2][LW];
    __shared__ float s_w[2][LW];
    const int t = threadIdx.x;
    const int x0 = blockIdx.x * SW_COLS;
    const int y0 = blockIdx.y * SW_ROWS;
    const size_t plane = (size_t)blockIdx.z * ((size_t)W * H);
    const int x = x0 + 2 * t;
    // threads 0 .. 2R-1 also read one halo column: x0-R+t (left) or
    // x0+SW_COLS+t-R (right)
    const bool halo = t < 2 * R;
    const int hx = t < R ? x0 - R + t : x0 + SW_COLS + (t - R);
    const int hl = t < R ? t : SW_COLS + t;  // its LDS slot
    const int rows_in = min(SW_ROWS, H - y0) + 2 * R;
    float hu0[K], hu1[K], hw0[K], hw1[K];  // ring of horizontal results
    RowIn cur;
    load_row<VEC>(sci, var, mask, plane, W, H, y0 - R, x, hx, halo, cur);
    for (int jb = 0; jb < rows_in; jb += K) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int j = jb + q;
            if (j >= rows_in) break;
            const int buf = j & 1;
            float u0, w0, u1, w1;
            weight(cur.I0, cur.v0, cur.m & 0xffu, u0, w0);
            weight(cur.I1, cur.v1, cur.m >> 8, u1, w1);
            s_u[buf][R + 2 * t] = u0;
            s_w[buf][R + 2 * t] = w0;
            s_u[buf][R + 2 * t + 1] = u1;
            s_w[buf][R + 2 * t + 1] = w1;
            if (halo) {
                float hu, hw;
                weight(cur.hI, cur.hv, cur.hm, hu, hw);
                s_u[buf][hl] = hu;
                s_w[buf][hl] = hw;
            }
            if (j + 1 < rows_in)
                load_row<VEC>(sci, var, mask, plane, W, H, y0 - R + j + 1, x, hx, halo, cur);
            __syncthreads();
            float a0 = 0.0f, a1 = 0.0f, b0 = 0.0f, b1 = 0.0f;
#pragma unroll
            for (int a = 0; a < K; ++a) {
                a0 = fmaf(f.r[a], s_u[buf][2 * t + a], a0);
                b0 = fmaf(f.r2[a], s_w[buf][2 * t + a], b0);
                a1 = fmaf(f.r[a], s_u[buf][2 * t + 1 + a], a1);
                b1 = fmaf(f.r2[a], s_w[buf][2 * t + 1 + a], b1);
            }
            hu0[q] = a0;
            hu1[q] = a1;
            hw0[q] = b0;
            hw1[q] = b1;
            if (j >= 2 * R) {
                const int y = y0 + j - 2 * R;
                float p0 = 0.0f, p1 = 0.0f, g0 = 0.0f, g1 = 0.0f;
#pragma unroll
                for (int b = 0; b < K; ++b) {
                    const int sl = (q + 1 + b) % K;
                    p0 = fmaf(f.c[b], hu0[sl], p0);
                    g0 = fmaf(f.c2[b], hw0[sl], g0);
                    p1 = fmaf(f.c[b], hu1[sl], p1);
                    g1 = fmaf(f.c2[b], hw1[sl], g1);
                }
                const size_t o = plane + (size_t)y * W + x;
                if (VEC && x + 1 < W) {
                    *reinterpret_cast<float2 *>(psi + o) = make_float2(p0, p1);
                    *reinterpret_cast<float2 *>(phi + o) = make_float2(g0, g1);
                } else {
                    if (x < W) {
                        psi[o] = p0;
                        phi[o] = g0;
                    }
                    if (x + 1 < W) {
                        psi[o + 1] = p1;
                        phi[o + 1] = g1;
                    }
                }
            }
        }
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
                const uint8_t *mask, float *psi, float *phi, int W, int H, int T,
                const SepArg &f) {
    // Row-streaming kernel (input read ~once); float2 accesses need even
    // row starts, i.e. an even width.
    const dim3 sg((W + SW_COLS - 1) / SW_COLS, (H + SW_ROWS - 1) / SW_ROWS, T);
    if ((W & 1) == 0)
        hipLaunchKernelGGL((planes_stream_kernel<K, true>), sg, dim3(SW_THREADS), 0, stream,
                           sci, var, mask, psi, phi, W, H, f);
    else
        hipLaunchKernelGGL((planes_stream_kernel<K, false>), sg, dim3(SW_THREADS), 0, stream,
                           sci, var, mask, psi, phi, W, H, f);
    (void)grid;
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
    case n: launch_sep<n>(grid, stream, sci, var, mask, psi, phi, W, H, T, f); break;
            KBM_SEP_CASE(1) KBM_SEP_CASE(3) KBM_SEP_CASE(5) KBM_SEP_CASE(7)
            KBM_SEP_CASE(9) KBM_SEP_CASE(11) KBM_SEP_CASE(13) KBM_SEP_CASE(15)
            KBM_SEP_CASE(17) KBM_SEP_CASE(19) KBM_SEP_CASE(21) KBM_SEP_CASE(23)
            KBM_SEP_CASE(25) KBM_SEP_CASE(27) KBM_SEP_CASE(29) KBM_SEP_CASE(31)
#undef KBM_SEP_CASE
        }
        KBM_LAUNCHED("planes_stream_kernel");
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

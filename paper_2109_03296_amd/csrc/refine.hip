// Bilinear trajectory likelihood and its adjoint (refinement of search
// candidates to sub-pixel start positions and velocities).
//
// One lane per candidate.  Positions x_i = x0 + vx t_i are formed in FP64
// (a float32 position at x ~ 4000 px would carry ~2e-4 px of rounding), the
// taps and weights in binary32.  One pass over the kept epochs accumulates
// the bilinear samples of psi and phi and, when an upstream gradient is
// given, the sums of their x and y derivatives (plain and times t_i), from
// which dL/dx_i = dPsi/dx_i / sqrt(Phi) - L/(2 Phi) dPhi/dx_i chained through
// dx_i/dx0 = 1 and dx_i/dvx = t_i follows; a second pass, only for plane
// gradients, scatter-adds g/sqrt(Phi) * w_tap into dL/dpsi and
// -g L/(2 Phi) * w_tap into dL/dphi with float atomics.
#include "kbm_internal.h"

namespace kbm {
namespace {

struct RefineArgs {
    const float *psi;
    const float *phi;
    const float *params;
    const uint64_t *keep;
    float *lh;
    const float *grad_lh;
    float *grad_params;
    float *grad_psi;
    float *grad_phi;
    int64_t n;
    int W, H, T;
    double t[KBM_MAX_EPOCHS];
};

struct Taps {
    int ix, iy;
    float fx, fy;
    bool any;  // at least one tap inside the image
};

__device__ __forceinline__ Taps taps_at(const RefineArgs &a, double x0,
                                        double vx, double y0, double vy,
                                        double t) {
#pragma clang fp contract(off)
    const double x = x0 + vx * t;
    const double y = y0 + vy * t;
    const double fxl = floor(x), fyl = floor(y);
    Taps p;
    p.any = fxl >= -1.0 && fxl <= (double)(a.W - 1) && fyl >= -1.0 &&
            fyl <= (double)(a.H - 1);
    p.ix = p.any ? (int)fxl : 0;
    p.iy = p.any ? (int)fyl : 0;
    p.fx = p.any ? (float)(x - fxl) : 0.0f;
    p.fy = p.any ? (float)(y - fyl) : 0.0f;
    return p;
}

__device__ __forceinline__ float tap(const float *plane, int W, int H, int x,
                                     int y) {
    return ((unsigned)x < (unsigned)W && (unsigned)y < (unsigned)H)
               ? plane[(size_t)y * W + x]
               : 0.0f;
}

// L and (with `grad`) g * dL/dparams of candidate c at parameters (x0, y0,
// vx, vy), plus the scatter-adds into the plane gradients when requested.
// Returns L (0 when the kept samples carry no phi, with a zero gradient).
//
// dL/dx_i = A dPsi/dx_i + B dPhi/dx_i with A = 1/sqrt(Phi), B = -L/(2 Phi)
// known only after the sums, but the parameter gradient is linear in the
// per-epoch derivatives: dL/dx0 = A sum dPsi/dx_i + B sum dPhi/dx_i and
// dL/dvx = A sum t_i dPsi/dx_i + B sum t_i dPhi/dx_i.  So one pass over
// the taps accumulates the likelihood sums and these eight derivative sums;
// only the plane-gradient scatter (which needs A and B per tap) revisits
// the taps.
__device__ __forceinline__ float refine_one(const RefineArgs &a, int64_t c, float px0,
                                            float py0, float pvx, float pvy, uint64_t km,
                                            bool grad, float g, float (&gp)[4]) {
    const double x0 = px0, y0 = py0;
    const double vx = pvx, vy = pvy;
    const size_t HW = (size_t)a.W * a.H;

    float Ps = 0.0f, Fs = 0.0f;
    float spx = 0.0f, spy = 0.0f, sfx = 0.0f, sfy = 0.0f;  // sums of dPsi, dPhi
    float tpx = 0.0f, tpy = 0.0f, tfx = 0.0f, tfy = 0.0f;  // the same times t_i
    for (int i = 0; i < a.T; ++i) {
        if (!((km >> i) & 1)) continue;
        const Taps p = taps_at(a, x0, vx, y0, vy, a.t[i]);
        if (!p.any) continue;
        const float *ps = a.psi + i * HW;
        const float *ph = a.phi + i * HW;
        const float s00 = tap(ps, a.W, a.H, p.ix, p.iy), s10 = tap(ps, a.W, a.H, p.ix + 1, p.iy);
        const float s01 = tap(ps, a.W, a.H, p.ix, p.iy + 1), s11 = tap(ps, a.W, a.H, p.ix + 1, p.iy + 1);
        const float f00 = tap(ph, a.W, a.H, p.ix, p.iy), f10 = tap(ph, a.W, a.H, p.ix + 1, p.iy);
        const float f01 = tap(ph, a.W, a.H, p.ix, p.iy + 1), f11 = tap(ph, a.W, a.H, p.ix + 1, p.iy + 1);
        const float w00 = (1.0f - p.fx) * (1.0f - p.fy), w10 = p.fx * (1.0f - p.fy);
        const float w01 = (1.0f - p.fx) * p.fy, w11 = p.fx * p.fy;
        Ps += w00 * s00 + w10 * s10 + w01 * s01 + w11 * s11;
        Fs += w00 * f00 + w10 * f10 + w01 * f01 + w11 * f11;
        if (grad) {
            const float dpx = (1.0f - p.fy) * (s10 - s00) + p.fy * (s11 - s01);
            const float dpy = (1.0f - p.fx) * (s01 - s00) + p.fx * (s11 - s10);
            const float dfx = (1.0f - p.fy) * (f10 - f00) + p.fy * (f11 - f01);
            const float dfy = (1.0f - p.fx) * (f01 - f00) + p.fx * (f11 - f10);
            const float ti = (float)a.t[i];
            spx += dpx;
            spy += dpy;
            sfx += dfx;
            sfy += dfy;
            tpx += ti * dpx;
            tpy += ti * dpy;
            tfx += ti * dfx;
            tfy += ti * dfy;
        }
    }
    if (!(Fs > 0.0f)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) gp[j] = 0.0f;
        return 0.0f;
    }
    const float L = Ps / sqrtf(Fs);
    if (!grad) return L;

    const float A = 1.0f / sqrtf(Fs);
    const float B = -L / (2.0f * Fs);
    gp[0] = g * (A * spx + B * sfx);
    gp[1] = g * (A * spy + B * sfy);
    gp[2] = g * (A * tpx + B * tfx);
    gp[3] = g * (A * tpy + B * tfy);
    if (a.grad_psi || a.grad_phi) {
        for (int i = 0; i < a.T; ++i) {
            if (!((km >> i) & 1)) continue;
            const Taps p = taps_at(a, x0, vx, y0, vy, a.t[i]);
            if (!p.any) continue;
            const float w[4] = {(1.0f - p.fx) * (1.0f - p.fy), p.fx * (1.0f - p.fy),
                                (1.0f - p.fx) * p.fy, p.fx * p.fy};
            const int xs[4] = {p.ix, p.ix + 1, p.ix, p.ix + 1};
            const int ys[4] = {p.iy, p.iy, p.iy + 1, p.iy + 1};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if ((unsigned)xs[j] >= (unsigned)a.W || (unsigned)ys[j] >= (unsigned)a.H) continue;
                const size_t q = i * HW + (size_t)ys[j] * a.W + xs[j];
                if (a.grad_psi) unsafeAtomicAdd(a.grad_psi + q, g * A * w[j]);
                if (a.grad_phi) unsafeAtomicAdd(a.grad_phi + q, g * B * w[j]);
            }
        }
    }
    return L;
}

__global__ __launch_bounds__(256) void refine_kernel(RefineArgs a) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    const uint64_t km = a.keep ? a.keep[c] : ~(uint64_t)0;
    const bool grad = a.grad_lh != nullptr;
    float gp[4];
    const float L = refine_one(a, c, a.params[4 * c + 0], a.params[4 * c + 1],
                               a.params[4 * c + 2], a.params[4 * c + 3], km, grad,
                               grad ? a.grad_lh[c] : 0.0f, gp);
    a.lh[c] = L;
    if (!grad) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) a.grad_params[4 * c + j] = gp[j];
}

// The whole refinement loop for one candidate per lane: `steps` times the
// adjoint (upstream gradient 1) and the Adam update of the four parameters
// with m and v in registers, then L at the final parameters.  Each step's
// arithmetic is that of refine_kernel followed by adam_kernel, so the
// result equals alternating the two launches, bit for bit.
constexpr int REFINE_MAX_STEPS = 64;
struct RefineAdamArgs {
    RefineArgs r;   // params and lh alias the in/out arrays below
    float *params;  // [n][4], updated in place
    float lr[REFINE_MAX_STEPS][4];
    float c1[REFINE_MAX_STEPS], c2[REFINE_MAX_STEPS];  // 1 - beta^step
    float b1, b2, omb1, omb2, eps;
    int steps;
};

// 64-lane workgroups: 10^5 candidates make ~1560 waves, which spread over
// the 256 CUs far more evenly as single waves than as groups of four.
constexpr int REFINE_ADAM_THREADS = 64;
__global__ __launch_bounds__(REFINE_ADAM_THREADS) void refine_adam_kernel(RefineAdamArgs a) {
#pragma clang fp contract(off)
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.r.n) return;
    const uint64_t km = a.r.keep ? a.r.keep[c] : ~(uint64_t)0;
    float p[4], m[4], v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        p[j] = a.params[4 * c + j];
        m[j] = 0.0f;
        v[j] = 0.0f;
    }
    for (int s = 0; s < a.steps; ++s) {
        float gp[4];
        (void)refine_one(a.r, c, p[0], p[1], p[2], p[3], km, true, 1.0f, gp);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float g = -1.0f * gp[j];  // ascent: the gradient of -L
            m[j] = a.b1 * m[j] + a.omb1 * g;
            v[j] = a.b2 * v[j] + a.omb2 * g * g;
            const float mh = m[j] / a.c1[s], vh = v[j] / a.c2[s];
            p[j] -= a.lr[s][j] * mh / (sqrtf(vh) + a.eps);
        }
    }
    float gp[4];
    const float L = refine_one(a.r, c, p[0], p[1], p[2], p[3], km, false, 0.0f, gp);
#pragma unroll
    for (int j = 0; j < 4; ++j) a.params[4 * c + j] = p[j];
    a.r.lh[c] = L;
}

}  // namespace
}  // namespace kbm

extern "C" kbm_status kbm_refine(const kbm_stack *s, const float *psi,
                                 const float *phi, int64_t n,
                                 const float *params, const uint64_t *keep,
                                 float *lh, const float *grad_lh,
                                 float *grad_params, float *grad_psi,
                                 float *grad_phi, hipStream_t stream) {
    using namespace kbm;
    clear_error();
    kbm_status st = check_stack(s, "kbm_refine");
    if (st != KBM_OK) return st;
    KBM_REQUIRE(n >= 0, KBM_ERR_INVALID_ARG, "kbm_refine: n = %lld must be >= 0",
                (long long)n);
    KBM_REQUIRE(n == 0 || (psi && phi && params && lh), KBM_ERR_INVALID_ARG,
                "kbm_refine: psi, phi, params and lh must be non-NULL");
    KBM_REQUIRE(grad_lh == nullptr || grad_params != nullptr || n == 0,
                KBM_ERR_INVALID_ARG,
                "kbm_refine: grad_params is required with grad_lh");
    KBM_REQUIRE((n + 255) / 256 < ((int64_t)1 << 31), KBM_ERR_UNSUPPORTED,
                "kbm_refine: n = %lld too large", (long long)n);
    if (n == 0) return KBM_OK;
    RefineArgs a{};
    a.psi = psi;
    a.phi = phi;
    a.params = params;
    a.keep = keep;
    a.lh = lh;
    a.grad_lh = grad_lh;
    a.grad_params = grad_params;
    a.grad_psi = grad_lh ? grad_psi : nullptr;
    a.grad_phi = grad_lh ? grad_phi : nullptr;
    a.n = n;
    a.W = s->width;
    a.H = s->height;
    a.T = s->num_epochs;
    double t0 = s->times[0];
    for (int i = 1; i < a.T; ++i) t0 = std::min(t0, s->times[i]);
    for (int i = 0; i < a.T; ++i) a.t[i] = s->times[i] - t0;
    hipLaunchKernelGGL(refine_kernel, dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, stream, a);
    KBM_LAUNCHED("refine_kernel");
    return KBM_OK;
}

extern "C" kbm_status kbm_refine_adam(const kbm_stack *s, const float *psi,
                                      const float *phi, int64_t n, float *params,
                                      const uint64_t *keep, const float *lr, int32_t steps,
                                      double beta1, double beta2, double eps, float *lh,
                                      hipStream_t stream) {
    using namespace kbm;
    clear_error();
    kbm_status st = check_stack(s, "kbm_refine_adam");
    if (st != KBM_OK) return st;
    KBM_REQUIRE(n >= 0, KBM_ERR_INVALID_ARG, "kbm_refine_adam: n = %lld must be >= 0",
                (long long)n);
    KBM_REQUIRE(steps >= 1 && steps <= REFINE_MAX_STEPS, KBM_ERR_UNSUPPORTED,
                "kbm_refine_adam: steps = %d not in [1, %d]", steps, REFINE_MAX_STEPS);
    KBM_REQUIRE(lr != nullptr, KBM_ERR_INVALID_ARG, "kbm_refine_adam: lr is NULL");
    for (int j = 0; j < 4 * steps; ++j)
        KBM_REQUIRE(std::isfinite(lr[j]), KBM_ERR_INVALID_ARG,
                    "kbm_refine_adam: lr[%d] is not finite", j);
    KBM_REQUIRE(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0,
                KBM_ERR_INVALID_ARG, "kbm_refine_adam: bad betas or eps");
    KBM_REQUIRE(n == 0 || (psi && phi && params && lh), KBM_ERR_INVALID_ARG,
                "kbm_refine_adam: psi, phi, params and lh must be non-NULL");
    KBM_REQUIRE((n + 63) / 64 < ((int64_t)1 << 31), KBM_ERR_UNSUPPORTED,
                "kbm_refine_adam: n = %lld too large", (long long)n);
    if (n == 0) return KBM_OK;
    RefineAdamArgs a{};
    a.r.psi = psi;
    a.r.phi = phi;
    a.r.params = params;
    a.r.keep = keep;
    a.r.lh = lh;
    a.r.n = n;
    a.r.W = s->width;
    a.r.H = s->height;
    a.r.T = s->num_epochs;
    double t0 = s->times[0];
    for (int i = 1; i < a.r.T; ++i) t0 = std::min(t0, s->times[i]);
    for (int i = 0; i < a.r.T; ++i) a.r.t[i] = s->times[i] - t0;
    a.params = params;
    for (int k = 0; k < steps; ++k) {
        for (int j = 0; j < 4; ++j) a.lr[k][j] = lr[4 * k + j];
        // as kbm_adam_step at step k + 1
        a.c1[k] = (float)(1.0 - std::pow(beta1, (double)(k + 1)));
        a.c2[k] = (float)(1.0 - std::pow(beta2, (double)(k + 1)));
    }
    a.b1 = (float)beta1;
    a.b2 = (float)beta2;
    a.omb1 = (float)(1.0 - beta1);
    a.omb2 = (float)(1.0 - beta2);
    a.eps = (float)eps;
    a.steps = steps;
    hipLaunchKernelGGL(refine_adam_kernel,
                       dim3((unsigned)((n + REFINE_ADAM_THREADS - 1) / REFINE_ADAM_THREADS)),
                       dim3(REFINE_ADAM_THREADS), 0, stream, a);
    KBM_LAUNCHED("refine_adam_kernel");
    return KBM_OK;
}

// ---------------------------------------------------------------------
// Adam update of the refinement parameters (Kingma & Ba, Algorithm 1):
// m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr_col * mhat/(sqrt(vhat)+eps)
// with mhat = m/(1-b1^t), vhat = v/(1-b2^t); maximize flips the sign of g.
// ---------------------------------------------------------------------
namespace kbm {
namespace {

constexpr int ADAM_MAX_COLS = 8;

struct AdamArgs {
    float *p;
    const float *g;
    float *m;
    float *v;
    int64_t n;  // elements
    int cols;
    float lr[ADAM_MAX_COLS];
    // 1 - b1 and 1 - b2 are formed in FP64 and rounded once: 1 - (float)b2
    // would carry the rounding error of b2 (1.3e-5 relative for 0.999).
    float b1, b2, omb1, omb2, eps, c1, c2, sign;
};

__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const float g = a.sign * a.g[i];
    const float m = a.b1 * a.m[i] + a.omb1 * g;
    const float v = a.b2 * a.v[i] + a.omb2 * g * g;
    a.m[i] = m;
    a.v[i] = v;
    const float mh = m / a.c1, vh = v / a.c2;
    a.p[i] -= a.lr[i % a.cols] * mh / (sqrtf(vh) + a.eps);
}

}  // namespace
}  // namespace kbm

extern "C" kbm_status kbm_adam_step(float *params, const float *grad, float *m,
                                    float *v, int64_t n, int32_t cols,
                                    const float *lr, double beta1, double beta2,
                                    double eps, int32_t step, int32_t maximize,
                                    hipStream_t stream) {
    using namespace kbm;
    clear_error();
    KBM_REQUIRE(n >= 0 && cols >= 1 && cols <= ADAM_MAX_COLS && lr != nullptr,
                KBM_ERR_INVALID_ARG, "kbm_adam_step: bad shape (n=%lld, cols=%d)",
                (long long)n, cols);
    KBM_REQUIRE(n == 0 || (params && grad && m && v), KBM_ERR_INVALID_ARG,
                "kbm_adam_step: arrays must be non-NULL");
    KBM_REQUIRE(step >= 1, KBM_ERR_INVALID_ARG, "kbm_adam_step: step must be >= 1");
    KBM_REQUIRE(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0,
                KBM_ERR_INVALID_ARG, "kbm_adam_step: bad betas or eps");
    for (int c = 0; c < cols; ++c)
        KBM_REQUIRE(std::isfinite(lr[c]), KBM_ERR_INVALID_ARG, "kbm_adam_step: lr not finite");
    const int64_t total = n * cols;
    if (total == 0) return KBM_OK;
    AdamArgs a{};
    a.p = params;
    a.g = grad;
    a.m = m;
    a.v = v;
    a.n = total;
    a.cols = cols;
    for (int c = 0; c < cols; ++c) a.lr[c] = lr[c];
    a.b1 = (float)beta1;
    a.b2 = (float)beta2;
    a.omb1 = (float)(1.0 - beta1);
    a.omb2 = (float)(1.0 - beta2);
    a.eps = (float)eps;
    a.c1 = (float)(1.0 - std::pow(beta1, (double)step));
    a.c2 = (float)(1.0 - std::pow(beta2, (double)step));
    a.sign = maximize ? -1.0f : 1.0f;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       stream, a);
    KBM_LAUNCHED("adam_kernel");
    return KBM_OK;
}

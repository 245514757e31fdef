// Internal helpers shared by the kbm HIP translation units: error
// reporting, argument checks, and the sigma_G device code used by both the
// fused search kernel and the standalone filter kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>

#include "kbm.h"
#include "sortnet.h"

namespace kbm {

// ---------------------------------------------------------------------
// Host-side error handling
// ---------------------------------------------------------------------
void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

#define KBM_REQUIRE(cond, code, ...)          \
    do {                                      \
        if (!(cond)) {                        \
            ::kbm::set_error(__VA_ARGS__);    \
            return (code);                    \
        }                                     \
    } while (0)

#define KBM_HIP(call)                                                       \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                             \
            ::kbm::set_error("%s failed: %s", #call, hipGetErrorString(e_)); \
            return KBM_ERR_DEVICE;                                          \
        }                                                                   \
    } while (0)

// Check that the last launch was accepted by the runtime.
#define KBM_LAUNCHED(name)                                                 \
    do {                                                                   \
        hipError_t e_ = hipGetLastError();                                 \
        if (e_ != hipSuccess) {                                            \
            ::kbm::set_error("launch of %s failed: %s", name,              \
                             hipGetErrorString(e_));                       \
            return KBM_ERR_DEVICE;                                         \
        }                                                                  \
    } while (0)

kbm_status check_stack(const kbm_stack *s, const char *what);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Asynchronous copy of a small host table to device memory on `stream`
// through a pinned staging buffer (safe to free `src` on return).
kbm_status stage_to_device(void *dst, const void *src, size_t bytes,
                           hipStream_t stream);

// ---------------------------------------------------------------------
// Quantile ranks: nearest-rank selection floor(q (n-1) + 1/2) in FP64,
// tabulated on the host for every usable-epoch count n in [1, 64].
// ---------------------------------------------------------------------
struct RankTable {
    uint8_t lo[KBM_MAX_EPOCHS + 1];
    uint8_t md[KBM_MAX_EPOCHS + 1];
    uint8_t hi[KBM_MAX_EPOCHS + 1];
};

RankTable make_rank_table(double q_lo, double q_hi);

kbm_status check_sigmag_params(double q_lo, double q_hi, double coeff,
                               double n_sigma);

// ---------------------------------------------------------------------
// Device code: fixed-size sorting network and rank selection
// ---------------------------------------------------------------------

// Sort N registers with the compile-time network of sortnet.h (3-sorter
// runs joined by Batcher's odd-even merges; valid for every N, checked by
// the 0-1 principle on the host).  Every wire index is a template constant,
// so the array stays in VGPRs, and comparators whose outputs no caller
// reads are dead code: with compile-time ranks only the ones that reach
// them remain.  Compare-exchanges use IEEE 754-2019 minimum/maximum
// (v_minimum3_f32 / v_maximum3_f32), 3-sorters v_minimum3_f32, v_med3_f32
// and v_maximum3_f32.  Callers never pass NaN (unusable entries arrive as
// +inf), and unlike fminf/fmaxf these need no quieting of operands the
// compiler cannot prove quiet (values loaded as raw bits), which would cost
// one extra instruction per element.  On NaN-free input the only freedom
// left is the order of -0 and +0, which compare equal: every rank value,
// difference and threshold built from the sorted array is the same.
template <int N, int K>
__device__ __forceinline__ void net_op(float (&a)[N]) {
    constexpr net::Op o = net::Table<N>::net.op[K];
    if constexpr (o.t == 0) {
        const float x = a[o.a], y = a[o.b];
        a[o.a] = __builtin_elementwise_minimum(x, y);
        a[o.b] = __builtin_elementwise_maximum(x, y);
    } else {
        const float x = a[o.a], y = a[o.b], z = a[o.c];
        a[o.a] = __builtin_elementwise_minimum(__builtin_elementwise_minimum(x, y), z);
        a[o.b] = __builtin_amdgcn_fmed3f(x, y, z);
        a[o.c] = __builtin_elementwise_maximum(__builtin_elementwise_maximum(x, y), z);
    }
}

template <int N, int... K>
__device__ __forceinline__ void net_apply(float (&a)[N], std::integer_sequence<int, K...>) {
    (net_op<N, K>(a), ...);
}

template <int N, int... R>
__device__ __forceinline__ void net_to_ranks(float (&a)[N], std::integer_sequence<int, R...>) {
    const float t[N] = {a[net::Table<N>::net.out[R]]...};
#pragma unroll
    for (int r = 0; r < N; ++r) a[r] = t[r];
}

template <int N>
__device__ __forceinline__ void sort_network(float (&a)[N]) {
    net_apply<N>(a, std::make_integer_sequence<int, net::Table<N>::net.nops>{});
    net_to_ranks<N>(a, std::make_integer_sequence<int, N>{});
}

constexpr int next_pow2(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// a[r] for a runtime index r in [0, N): a binary tree of selects on the bits
// of r (P-1 v_cndmask for P = next_pow2(N)).
template <int N>
__device__ __forceinline__ float select_rank(const float (&a)[N], int r) {
    constexpr int P = next_pow2(N);
    float t[P];
#pragma unroll
    for (int j = 0; j < P; ++j) t[j] = a[j < N ? j : N - 1];
#pragma unroll
    for (int w = P / 2, b = 0; w >= 1; w /= 2, ++b) {
        const bool bit = (r >> b) & 1;
#pragma unroll
        for (int j = 0; j < w; ++j) t[j] = bit ? t[2 * j + 1] : t[2 * j];
    }
    return t[0];
}

// sigma_G cut (Section 3.1) for one lightcurve held in registers.  For
// epochs i < T, nu[i] is psi_i/sqrt(phi_i) when usable and NaN otherwise;
// entries i >= T are padding and hold +inf.  r_lo, r_md, r_hi are the
// nearest ranks of q_lo, 1/2, q_hi for the number of usable epochs.
// SEL = true when NaN entries may be present (they sort as +inf); with
// SEL = false every epoch i < T is usable.  Binary32, no contraction:
//   x_q   = sorted usable nu at rank r_q(n)
//   sigma = coeff * (x_hi - x_lo);  thr = n_sigma * sigma
//   keep  = |nu_i - x_md| <= thr   (false for NaN, i.e. unusable epochs)
// The caller applies keeps() epoch by epoch (a per-epoch bool array would
// live in SGPR lane masks and spill).
struct SigmaGCut {
    float x_md, thr;
    __device__ __forceinline__ bool keeps(float nu) const {
#pragma clang fp contract(off)
        return fabsf(nu - x_md) <= thr;
    }
};

// Same cut with compile-time ranks (no select trees; comparators whose
// outputs do not reach the three ranks are dead code).
template <int N, int RL, int RM, int RH>
__device__ __forceinline__ SigmaGCut sigmag_cut_fixed(const float (&nu)[N],
                                                      float coeff,
                                                      float n_sigma) {
#pragma clang fp contract(off)
    float srt[N];
#pragma unroll
    for (int i = 0; i < N; ++i) srt[i] = nu[i];
    sort_network<N>(srt);
    const float sigma = coeff * (srt[RH] - srt[RL]);
    SigmaGCut c;
    c.x_md = srt[RM];
    c.thr = n_sigma * sigma;
    return c;
}

template <int N, bool SEL>
__device__ __forceinline__ SigmaGCut sigmag_cut(const float (&nu)[N], int r_lo,
                                                int r_md, int r_hi,
                                                float coeff, float n_sigma) {
#pragma clang fp contract(off)
    float srt[N];
#pragma unroll
    for (int i = 0; i < N; ++i)
        srt[i] = SEL ? ((nu[i] == nu[i]) ? nu[i] : INFINITY) : nu[i];
    sort_network<N>(srt);
    const float x_lo = select_rank<N>(srt, r_lo);
    const float x_md = select_rank<N>(srt, r_md);
    const float x_hi = select_rank<N>(srt, r_hi);
    const float sigma = coeff * (x_hi - x_lo);
    SigmaGCut c;
    c.x_md = x_md;
    c.thr = n_sigma * sigma;
    return c;
}

}  // namespace kbm

// Device code of the trajectory search (Section 3, 3.1 and 3.2): argument
// block, loaders, the sigma_G score, the chunked search kernel and the
// finalize kernel.  Included by the translation units that instantiate the
// kernels for different epoch counts (so they compile in parallel).
//
// Layout and schedule
//  * The host turns every (velocity, epoch) pair into an integer pixel
//    offset floor(v t + 1/2) in FP64 once per call ("pointer arithmetic",
//    Section 3: images are never shifted).  Three small tables go to the
//    workspace: the packed 16-bit (dx, dy) per (v, i), the element offset
//    i H W + dy W + dx per (v, i) (so no per-epoch constant has to stay live
//    across the velocity loop), and each velocity's offset bounding box.
//  * A prep kernel packs every pixel-epoch into one float2 (nu, s) with
//    nu = psi / sqrt(phi) and s = sqrt(phi), both correctly rounded binary32,
//    or (NaN, 0) where the pixel is unusable.  nu depends only on the pixel,
//    so the filter reads it instead of dividing per trajectory-epoch, and a
//    trajectory-epoch costs one 8-byte load.  Sums use psi ~ nu*s and
//    phi ~ s*s (a few ulp from psi, phi); the keep decision uses nu itself.
//  * One wavefront owns 64 consecutive start pixels of one row.  For a given
//    velocity all lanes read 64 consecutive float2 per epoch (coalesced).
//    Plane reads are buffer loads when the packed planes fit 32-bit byte
//    offsets: one descriptor, a per-lane byte offset and a wave-uniform
//    per-epoch scalar offset.  When a velocity's whole track box keeps the
//    wave inside the image the per-epoch offset is purely scalar (no
//    per-lane address arithmetic); otherwise per-lane element offsets are
//    clamped into the planes and out-of-image samples are discarded.  Larger
//    stacks use 64-bit addresses.
//  * The lightcurve (nu, s for T epochs) lives in VGPRs; sigma_G runs per
//    lane: a Batcher sorting network and a select tree for the three ranks.
//    Kernels are instantiated for the exact epoch count where it is common,
//    so no padding logic is emitted.
//  * Velocities are swept in chunks, one launch per chunk, so every wave in
//    flight works on the same few velocities and neighbouring waves re-read
//    the same plane rows through L2.  Tiles are grouped into super-tiles
//    (256 px x 16 rows) handed to the 8 XCDs in contiguous column strips.
//    Each lane's top-K (L', velocity index) lives in registers within a
//    chunk and in the workspace between chunks; a final kernel re-evaluates
//    the K winners to emit flux, n_obs, keep bits and lh_raw.
#pragma once

#include "kbm_internal.h"

namespace kbm {
namespace srch {

#ifndef KBM_ST_X
#define KBM_ST_X 4
#endif
#ifndef KBM_ST_Y
#define KBM_ST_Y 16
#endif
#ifndef KBM_VCHUNK
#define KBM_VCHUNK 256
#endif
#ifndef KBM_MAX_WAVES_PER_SIMD
#define KBM_MAX_WAVES_PER_SIMD 8
#endif
#ifndef KBM_STAGGER
#define KBM_STAGGER 1
#endif
#ifndef KBM_PIPE
#define KBM_PIPE 0
#endif
#ifndef KBM_NW
#define KBM_NW 1
#endif

constexpr int WAVE = 64;
constexpr int NUM_XCD = 8;
constexpr int ST_X = KBM_ST_X;      // tiles (of 64 px) across a super-tile
constexpr int ST_Y = KBM_ST_Y;      // rows in a super-tile
constexpr int ST_TILES = ST_X * ST_Y;
constexpr int VCHUNK = KBM_VCHUNK;  // velocities per launch
constexpr int NW = KBM_NW;          // waves per workgroup sharing a tile
constexpr int BUF_DWORD3 = 0x00020000;  // raw buffer descriptor, CDNA

struct SearchArgs {
    const float2 *pk;         // [T][H][W] (nu, s)
    uint32_t pk_bytes;        // bytes covered by the buffer descriptor
    uint32_t n_elem;          // T H W
    const int *off16;         // [V][T] (dx & 0xffff) | (dy << 16)
    const uint32_t *lin;      // [V][T] i H W + dy W + dx (mod 2^32)
    const int4 *vbox;         // [V] (dxmin, dxmax, dymin, dymax)
    const int4 *mbox;         // [V] min_obs-th smallest/largest dx and dy
    const int *ranks;         // [3][65] quantile ranks by usable count
    const int *flags;         // [0] != 0: some pixel-epoch is unusable
    float *stL;               // [K][Npix] running top-K likelihoods
    int *stI;                 // [K][Npix] running top-K velocity indices
    float *lh;
    float *flux;
    int32_t *vidx;
    int16_t *nobs;
    uint64_t *keep;
    float *lh_raw;
    int W, H, T, V, K, min_obs, sigmag;
    int x0, y0, Wr, Hr, tiles_x, n_super_y, n_tiles;
    int v_begin, v_end, first;
    float coeff, n_sigma;
    int defq;                 // quantiles are (0.25, 0.75): fixed ranks
};

__device__ __forceinline__ bool ranks_before(float la, int ia, float lb,
                                             int ib) {
    return la > lb || (la == lb && ia < ib);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const SearchArgs &a) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)a.pk, (short)0,
                                             (int)a.pk_bytes, BUF_DWORD3);
}

__device__ __forceinline__ float2 ld_plane(__amdgpu_buffer_rsrc_t r,
                                           uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float2,
                              __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// Element e of the packed planes, clamped into the planes (an out-of-image
// lane's offset may wrap; its value is discarded by the caller).
template <bool SINGLE>
__device__ __forceinline__ float2 ld_elem(const SearchArgs &a,
                                          __amdgpu_buffer_rsrc_t r, uint32_t e) {
    const uint32_t c = min(e, a.n_elem - 1u);
    if (SINGLE) return ld_plane(r, c * 8u, 0u);
    return a.pk[c];
}

struct Score {
    float L, flux;
    uint64_t keep;
};

// Filtered (or plain) likelihood of one lightcurve.  For i < T, nu[i] is NaN
// for an unusable epoch and s[i] = 0; entries i >= T are padding (+inf, 0).
// SEL selects the NaN handling needed when unusable epochs may be present.
template <int TM, bool SEL, bool EXACT>
__device__ __forceinline__ Score score(const SearchArgs &a,
                                       const float (&nu)[TM],
                                       const float (&s)[TM], int nv) {
    const int T = EXACT ? TM : a.T;
    Score r;
    float P = 0.0f, F = 0.0f;
    uint32_t lo = 0, hi = 0;
    if (a.sigmag) {
        const int rl = a.ranks[nv], rm = a.ranks[65 + nv], rh = a.ranks[130 + nv];
        const SigmaGCut c = sigmag_cut<TM, SEL>(nu, rl, rm, rh, a.coeff, a.n_sigma);
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if (i < T) {
                const bool k = c.keeps(nu[i]);
                P = fmaf(k ? nu[i] : 0.0f, s[i], P);
                F = fmaf(k ? s[i] : 0.0f, s[i], F);
                if (i < 32)
                    lo |= k ? (1u << i) : 0u;
                else
                    hi |= k ? (1u << (i - 32)) : 0u;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if (i < T) {
                const bool ok = SEL ? (nu[i] == nu[i]) : true;
                P = fmaf(ok ? nu[i] : 0.0f, s[i], P);
                F = fmaf(s[i], s[i], F);
                if (i < 32)
                    lo |= ok ? (1u << i) : 0u;
                else
                    hi |= ok ? (1u << (i - 32)) : 0u;
            }
        }
    }
    r.keep = (uint64_t)lo | ((uint64_t)hi << 32);
    r.L = P / sqrtf(F);
    r.flux = P / F;
    return r;
}

// Clean, exact-T fast path with the default quantiles (0.25, 0.75): every
// epoch is usable, the nearest ranks floor(q (T-1) + 1/2) are compile-time
// constants, and the kept sums zero s instead of selecting twice.
template <int T>
__device__ __forceinline__ float score_fixed(const SearchArgs &a,
                                             const float (&nu)[T],
                                             const float (&s)[T]) {
    constexpr int RL = (T + 1) / 4, RM = T / 2, RH = (3 * T - 1) / 4;
    float P = 0.0f, F = 0.0f;
    if (a.sigmag) {
        const SigmaGCut c = sigmag_cut_fixed<T, RL, RM, RH>(nu, a.coeff, a.n_sigma);
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const float sk = c.keeps(nu[i]) ? s[i] : 0.0f;
            P = fmaf(nu[i], sk, P);
            F = fmaf(sk, sk, F);
        }
    } else {
#pragma unroll
        for (int i = 0; i < T; ++i) {
            P = fmaf(nu[i], s[i], P);
            F = fmaf(s[i], s[i], F);
        }
    }
    return P / sqrtf(F);
}

// Whole-wave in-bounds load: the per-epoch offset is wave-uniform.
template <int TM, bool CLEAN, bool EXACT, bool SINGLE>
__device__ __forceinline__ int load_fast(const SearchArgs &a,
                                         __amdgpu_buffer_rsrc_t rs,
                                         uint32_t lane, uint32_t wave_e,
                                         const uint32_t *lv, float (&nu)[TM],
                                         float (&s)[TM]) {
    const int T = EXACT ? TM : a.T;
    int nv = 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        if (i < T) {
            const uint32_t e = wave_e + lv[i];
            const float2 q = SINGLE ? ld_plane(rs, lane * 8u, e * 8u)
                                    : a.pk[(size_t)e + lane];
            nu[i] = q.x;
            s[i] = q.y;
            if (!CLEAN) nv += (q.x == q.x) ? 1 : 0;
        } else {
            nu[i] = INFINITY;
            s[i] = 0.0f;
        }
    }
    return CLEAN ? T : nv;
}

// General load with per-lane bounds checks.
template <int TM, bool EXACT, bool SINGLE>
__device__ __forceinline__ int load_slow(const SearchArgs &a,
                                         __amdgpu_buffer_rsrc_t rs, int x,
                                         int y, const int *ov,
                                         const uint32_t *lv, float (&nu)[TM],
                                         float (&s)[TM]) {
    const int T = EXACT ? TM : a.T;
    const uint32_t pix = (uint32_t)(y * a.W + x);
    int nv = 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        if (i < T) {
            const int o = ov[i];
            const int dx = (int)(int16_t)(o & 0xffff), dy = o >> 16;
            const bool inb = (unsigned)(x + dx) < (unsigned)a.W &&
                             (unsigned)(y + dy) < (unsigned)a.H;
            const float2 q = ld_elem<SINGLE>(a, rs, lv[i] + pix);
            const bool ok = inb && (q.x == q.x);
            nu[i] = ok ? q.x : __builtin_nanf("");
            s[i] = ok ? q.y : 0.0f;
            nv += ok ? 1 : 0;
        } else {
            nu[i] = INFINITY;
            s[i] = 0.0f;
        }
    }
    return nv;
}

// Tile of this workgroup (one wave = 64 px of one row), XCD-major over
// super-tiles ordered column by column.  Returns false for padding tiles.
__device__ __forceinline__ bool map_tile(const SearchArgs &a, int &tx, int &ty) {
    const int N = a.n_tiles;
    const int b = blockIdx.x;
    const int q = N / NUM_XCD, rem = N % NUM_XCD;
    const int xcd = b % NUM_XCD, slot = b / NUM_XCD;
    const int t = xcd * q + min(xcd, rem) + slot;
    const int st = t / ST_TILES, w = t % ST_TILES;
    const int sx = st / a.n_super_y, sy = st % a.n_super_y;
    tx = sx * ST_X + w % ST_X;
    ty = sy * ST_Y + w / ST_X;
    return tx < a.tiles_x && ty < a.Hr;
}

template <int TM, int KM, bool CLEAN, bool EXACT, bool SINGLE>
__device__ __forceinline__ void run_chunk(const SearchArgs &a, int tx, int ty) {
    // NW waves share this tile's 64 start pixels and interleave the chunk's
    // velocities (wave w takes v = v_begin + w, w + NW, ...), so at any time
    // they read nearly the same plane rows: lines are shared through L1 and
    // the per-XCD footprint of a velocity step shrinks NW-fold.
    const unsigned lane = threadIdx.x % WAVE;
    const int w = NW > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE)) : 0;
    const int rx = tx * WAVE + (int)lane, ry = ty;
    const bool active = rx < a.Wr;
    const int xw = a.x0 + tx * WAVE;
    const int x = xw + (int)lane, y = a.y0 + ry;
    const size_t npix = (size_t)a.Wr * a.Hr;
    const size_t pix = (size_t)ry * a.Wr + (active ? rx : 0);
    const int T = EXACT ? TM : a.T;
    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(a);

    float kL[KM];
    int kI[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        // Slots below KM-K are placeholders that rank above everything, so
        // the K-th best always sits in the last register.
        const int slot = j - (KM - a.K);
        if (slot < 0) {
            kL[j] = INFINITY;
            kI[j] = -2;
        } else if (a.first || !active || w != 0) {
            kL[j] = -INFINITY;
            kI[j] = -1;
        } else {
            kL[j] = a.stL[(size_t)slot * npix + pix];
            kI[j] = a.stI[(size_t)slot * npix + pix];
        }
    }

    const uint32_t wave_e = (uint32_t)(y * a.W + xw);
    const int nvel = a.v_end - a.v_begin;
    const int rot = KBM_STAGGER > 1 ? (int)((blockIdx.x / NUM_XCD) % KBM_STAGGER) * nvel / KBM_STAGGER : 0;
    for (int vv = w; vv < nvel; vv += NW) {
        int v = a.v_begin + vv + rot;
        if (v >= a.v_end) v -= nvel;
        const int4 bx = a.vbox[v];
        const bool fast = xw + bx.x >= 0 &&
                          xw + (WAVE - 1) + bx.y < a.W && y + bx.z >= 0 &&
                          y + bx.w < a.H;
        if (!fast) {
            // Sound skip: if fewer than min_obs epochs can hold any lane of
            // this wave in the image (per axis), no lane reaches min_obs.
            const int4 mb = a.mbox[v];
            if (xw + mb.x > a.W - 1 || xw + (WAVE - 1) + mb.y < 0 ||
                y + mb.z > a.H - 1 || y + mb.w < 0)
                continue;
        }
        float nu[TM], s[TM];
        int nv;
        Score sc;
        if (fast) {
            nv = load_fast<TM, CLEAN, EXACT, SINGLE>(a, rs, lane, wave_e,
                                                     a.lin + (size_t)v * T, nu, s);
            if (EXACT && CLEAN && a.defq)
                sc.L = score_fixed<TM>(a, nu, s);
            else
                sc = score<TM, !CLEAN, EXACT>(a, nu, s, nv);
        } else {
            nv = load_slow<TM, EXACT, SINGLE>(a, rs, x, y, a.off16 + (size_t)v * T,
                                              a.lin + (size_t)v * T, nu, s);
            sc = score<TM, true, EXACT>(a, nu, s, nv);
        }
        if (active && nv >= a.min_obs && isfinite(sc.L) &&
            ranks_before(sc.L, v, kL[KM - 1], kI[KM - 1])) {
            kL[KM - 1] = sc.L;
            kI[KM - 1] = v;
#pragma unroll
            for (int j = KM - 1; j > 0; --j) {
                if (ranks_before(kL[j], kI[j], kL[j - 1], kI[j - 1])) {
                    const float tl = kL[j];
                    kL[j] = kL[j - 1];
                    kL[j - 1] = tl;
                    const int ti = kI[j];
                    kI[j] = kI[j - 1];
                    kI[j - 1] = ti;
                }
            }
        }
    }
    if (NW > 1) {
        // Merge the waves' lists into wave 0's through LDS.  The ranking
        // compares velocity indices on ties, so the merge order is immaterial.
        __shared__ float mL[NW > 1 ? NW - 1 : 1][KM][WAVE];
        __shared__ int mI[NW > 1 ? NW - 1 : 1][KM][WAVE];
        if (w > 0) {
#pragma unroll
            for (int j = 0; j < KM; ++j) {
                mL[w - 1][j][lane] = kL[j];
                mI[w - 1][j][lane] = kI[j];
            }
        }
        __syncthreads();
        if (w != 0) return;
        for (int o = 0; o < NW - 1; ++o) {
#pragma unroll
            for (int j = 0; j < KM; ++j) {
                const float L = mL[o][j][lane];
                const int v = mI[o][j][lane];
                if (v >= 0 && ranks_before(L, v, kL[KM - 1], kI[KM - 1])) {
                    kL[KM - 1] = L;
                    kI[KM - 1] = v;
#pragma unroll
                    for (int jj = KM - 1; jj > 0; --jj) {
                        if (ranks_before(kL[jj], kI[jj], kL[jj - 1], kI[jj - 1])) {
                            const float tl = kL[jj];
                            kL[jj] = kL[jj - 1];
                            kL[jj - 1] = tl;
                            const int ti = kI[jj];
                            kI[jj] = kI[jj - 1];
                            kI[jj - 1] = ti;
                        }
                    }
                }
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        const int slot = j - (KM - a.K);
        if (slot >= 0) {
            a.stL[(size_t)slot * npix + pix] = kL[j];
            a.stI[(size_t)slot * npix + pix] = kI[j];
        }
    }
}

// Insert (L, v) into a lane's sorted top-K registers.
template <int KM>
__device__ __forceinline__ void topk_insert(float (&kL)[KM], int (&kI)[KM],
                                            float L, int v) {
    kL[KM - 1] = L;
    kI[KM - 1] = v;
#pragma unroll
    for (int j = KM - 1; j > 0; --j) {
        if (ranks_before(kL[j], kI[j], kL[j - 1], kI[j - 1])) {
            const float tl = kL[j];
            kL[j] = kL[j - 1];
            kL[j - 1] = tl;
            const int ti = kI[j];
            kI[j] = kI[j - 1];
            kI[j - 1] = ti;
        }
    }
}

// One velocity of the software-pipelined sweep (clean stacks, exact T,
// single buffer).  cur holds this velocity's samples when it is on the fast
// path (loaded one step earlier); the next velocity's loads are issued into
// nxt before this velocity is scored, so they travel while the lane sorts.
template <int T, int KM>
__device__ __forceinline__ void pipe_step(const SearchArgs &a,
                                          __amdgpu_buffer_rsrc_t rs,
                                          unsigned lane, int x, int y, int xw,
                                          uint32_t wave_e, bool active, int v,
                                          bool fast_v, int vn, bool fast_n,
                                          float (&cn)[T], float (&cs)[T],
                                          float (&nn)[T], float (&ns)[T],
                                          float (&kL)[KM], int (&kI)[KM]) {
    if (fast_n)
        load_fast<T, true, true, true>(a, rs, lane, wave_e, a.lin + (size_t)vn * T, nn, ns);
    float L;
    int nv = T;
    if (fast_v) {
        if (a.defq) {
            L = score_fixed<T>(a, cn, cs);
        } else {
            L = score<T, false, true>(a, cn, cs, T).L;
        }
    } else {
        const int4 mb = a.mbox[v];
        if (xw + mb.x > a.W - 1 || xw + (WAVE - 1) + mb.y < 0 ||
            y + mb.z > a.H - 1 || y + mb.w < 0)
            return;
        nv = load_slow<T, true, true>(a, rs, x, y, a.off16 + (size_t)v * T,
                                      a.lin + (size_t)v * T, cn, cs);
        L = score<T, true, true>(a, cn, cs, nv).L;
    }
    if (active && nv >= a.min_obs && isfinite(L) &&
        ranks_before(L, v, kL[KM - 1], kI[KM - 1]))
        topk_insert<KM>(kL, kI, L, v);
}

template <int T, int KM>
__device__ __forceinline__ void run_chunk_pipe(const SearchArgs &a, int tx, int ty) {
    const unsigned lane = threadIdx.x;
    const int rx = tx * WAVE + (int)lane, ry = ty;
    const bool active = rx < a.Wr;
    const int xw = a.x0 + tx * WAVE;
    const int x = xw + (int)lane, y = a.y0 + ry;
    const size_t npix = (size_t)a.Wr * a.Hr;
    const size_t pix = (size_t)ry * a.Wr + (active ? rx : 0);
    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(a);

    float kL[KM];
    int kI[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        const int slot = j - (KM - a.K);
        if (slot < 0) {
            kL[j] = INFINITY;
            kI[j] = -2;
        } else if (a.first || !active) {
            kL[j] = -INFINITY;
            kI[j] = -1;
        } else {
            kL[j] = a.stL[(size_t)slot * npix + pix];
            kI[j] = a.stI[(size_t)slot * npix + pix];
        }
    }
    const uint32_t wave_e = (uint32_t)(y * a.W + xw);
    const int nvel = a.v_end - a.v_begin;
    const int rot = KBM_STAGGER > 1 ? (int)((blockIdx.x / NUM_XCD) % KBM_STAGGER) * nvel / KBM_STAGGER : 0;
    auto vel_at = [&](int vv) {
        int v = a.v_begin + vv + rot;
        return v >= a.v_end ? v - nvel : v;
    };
    auto is_fast = [&](int v) {
        const int4 bx = a.vbox[v];
        return xw + bx.x >= 0 && xw + (WAVE - 1) + bx.y < a.W && y + bx.z >= 0 &&
               y + bx.w < a.H;
    };
    float An[T], As[T], Bn[T], Bs[T];
    int v = vel_at(0);
    bool fv = is_fast(v);
    if (fv) load_fast<T, true, true, true>(a, rs, lane, wave_e, a.lin + (size_t)v * T, An, As);
    for (int vv = 0; vv < nvel; vv += 2) {
        const bool has1 = vv + 1 < nvel;
        const int v1 = has1 ? vel_at(vv + 1) : v;
        const bool f1 = has1 && is_fast(v1);
        pipe_step<T, KM>(a, rs, lane, x, y, xw, wave_e, active, v, fv, v1, f1,
                         An, As, Bn, Bs, kL, kI);
        if (!has1) break;
        const bool has2 = vv + 2 < nvel;
        const int v2 = has2 ? vel_at(vv + 2) : v1;
        const bool f2 = has2 && is_fast(v2);
        pipe_step<T, KM>(a, rs, lane, x, y, xw, wave_e, active, v1, f1, v2, f2,
                         Bn, Bs, An, As, kL, kI);
        v = v2;
        fv = f2;
    }
    if (!active) return;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        const int slot = j - (KM - a.K);
        if (slot >= 0) {
            a.stL[(size_t)slot * npix + pix] = kL[j];
            a.stI[(size_t)slot * npix + pix] = kI[j];
        }
    }
}

template <int TM, int KM, bool EXACT, bool SINGLE>
__global__ __launch_bounds__(WAVE * NW)
__attribute__((amdgpu_waves_per_eu(1, KBM_MAX_WAVES_PER_SIMD)))
void search_chunk_kernel(SearchArgs a) {
    int tx, ty;
    if (!map_tile(a, tx, ty)) return;
    if (a.flags[0] == 0) {
        if (KBM_PIPE && NW == 1 && EXACT && SINGLE)
            run_chunk_pipe<TM, KM>(a, tx, ty);
        else
            run_chunk<TM, KM, true, EXACT, SINGLE>(a, tx, ty);
    } else {
        run_chunk<TM, KM, false, EXACT, SINGLE>(a, tx, ty);
    }
}

// Re-evaluate each pixel's K winners and write all result fields.
template <int TM, bool SINGLE>
__global__ __launch_bounds__(256) void finalize_kernel(SearchArgs a) {
    const size_t npix = (size_t)a.Wr * a.Hr;
    const size_t pix = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= npix) return;
    const int rx = (int)(pix % a.Wr), ry = (int)(pix / a.Wr);
    const int x = a.x0 + rx, y = a.y0 + ry;
    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(a);
    for (int slot = 0; slot < a.K; ++slot) {
        const size_t o = pix * a.K + slot;
        const int vi = a.stI[(size_t)slot * npix + pix];
        if (vi < 0) {
            a.lh[o] = -INFINITY;
            a.flux[o] = 0.0f;
            a.vidx[o] = -1;
            a.nobs[o] = 0;
            a.keep[o] = 0;
            if (a.lh_raw) a.lh_raw[o] = -INFINITY;
            continue;
        }
        float nu[TM], s[TM];
        const int nv = load_slow<TM, false, SINGLE>(a, rs, x, y, a.off16 + (size_t)vi * a.T,
                                                     a.lin + (size_t)vi * a.T, nu, s);
        const Score sc = score<TM, true, false>(a, nu, s, nv);
        a.lh[o] = sc.L;
        a.flux[o] = sc.flux;
        a.vidx[o] = vi;
        a.nobs[o] = (int16_t)nv;
        a.keep[o] = sc.keep;
        if (a.lh_raw) {
            float P = 0.0f, F = 0.0f;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                if (i < a.T) {
                    P = fmaf(nu[i] == nu[i] ? nu[i] : 0.0f, s[i], P);
                    F = fmaf(s[i], s[i], F);
                }
            }
            a.lh_raw[o] = P / sqrtf(F);
        }
    }
}

// Launch the chunk sequence for one kernel variant.
template <int TM, int KM, bool EXACT, bool SINGLE>
void launch_chunks(SearchArgs a, hipStream_t stream) {
    for (int v0 = 0; v0 < a.V; v0 += VCHUNK) {
        a.v_begin = v0;
        a.v_end = v0 + VCHUNK < a.V ? v0 + VCHUNK : a.V;
        a.first = v0 == 0;
        hipLaunchKernelGGL((search_chunk_kernel<TM, KM, EXACT, SINGLE>), dim3(a.n_tiles),
                           dim3(WAVE * NW), 0, stream, a);
    }
}

// Exact-epoch-count variants (buffer-addressed stacks, K <= 8) live in
// separate translation units; each returns true when it handled T.
bool launch_exact_a(int T, const SearchArgs &a, hipStream_t stream);
bool launch_exact_b(int T, const SearchArgs &a, hipStream_t stream);

}  // namespace srch
}  // namespace kbm

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
#define KBM_ST_X 2
#endif
#ifndef KBM_ST_Y
#define KBM_ST_Y 32
#endif
#ifndef KBM_VCHUNK
#define KBM_VCHUNK 256
#endif
#ifndef KBM_MAX_WAVES_PER_SIMD
#define KBM_MAX_WAVES_PER_SIMD 8
#endif
#ifndef KBM_NW
#define KBM_NW 4
#endif

constexpr int WAVE = 64;
constexpr int NUM_XCD = 8;
constexpr int ST_X = KBM_ST_X;      // tiles (of 64 px) across a super-tile
constexpr int ST_Y = KBM_ST_Y;      // rows in a super-tile
constexpr int ST_TILES = ST_X * ST_Y;
constexpr int VCHUNK = KBM_VCHUNK;  // velocities per launch
constexpr int NW = KBM_NW;          // waves per workgroup sharing a tile
constexpr int BUF_DWORD3 = 0x00020000;  // raw buffer descriptor, CDNA

// Constant address space: tables and argument blocks that no kernel writes
// while the search runs are read through it, so uniform reads stay scalar
// loads even in kernels that store elsewhere.
#define KBM_CONST __attribute__((address_space(4)))
template <class P>
__device__ __forceinline__ const KBM_CONST P *cst(const P *p) {
    return (const KBM_CONST P *)p;
}

// Entry i of a constant int4 table.
__device__ __forceinline__ int4 ld_box(const int4 *t, int i) {
    const KBM_CONST int *p = (const KBM_CONST int *)t + 4 * (size_t)i;
    return make_int4(p[0], p[1], p[2], p[3]);
}

// Plane addressing modes (template parameter AM): 0 = 64-bit addresses;
// 1 = one buffer descriptor over all epochs (packed planes below 4 GB);
// 2 = two descriptors, epochs [0, split) and [split, T) with split = T/2,
// each group below 4 GB, per-epoch element offsets relative to their group
// (in exact-T code the group of every epoch is a compile-time constant).
struct SearchArgs {
    const float2 *pk;         // [T][H][W] (nu, s)
    uint32_t pk_bytes;        // bytes covered by the (first) descriptor
    uint32_t n_elem;          // elements of the first group (T H W if one)
    const float2 *pk2;        // first element of epoch `split`
    uint32_t pk2_bytes;       // bytes covered by the second descriptor
    uint32_t n_elem2;         // elements of the second group
    int split;                // epochs in the first group (T unless AM = 2)
    int am;                   // addressing mode of this stack (0, 1, 2)
    const int *off16;         // [V][T] (dx & 0xffff) | (dy << 16)
    const uint32_t *lin;      // [V][T] i H W + dy W + dx (mod 2^32)
    const int4 *vbox;         // [V][2] (dxmin, dxmax, dymin, dymax), (same1, same4, 0, 0):
                              // masks of epochs < 32 offset as at velocity v-1, v-4
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

struct PlaneRsrc {
    __amdgpu_buffer_rsrc_t r0, r1;  // epoch groups [0, split), [split, T)
};

template <class A>
__device__ __forceinline__ PlaneRsrc plane_rsrc(const A &a) {
    return PlaneRsrc{
        __builtin_amdgcn_make_buffer_rsrc((void *)a.pk, (short)0, (int)a.pk_bytes, BUF_DWORD3),
        __builtin_amdgcn_make_buffer_rsrc((void *)a.pk2, (short)0, (int)a.pk2_bytes,
                                          BUF_DWORD3)};
}

// Whether epoch i (a compile-time index in the unrolled loops) lies in the
// second group; SPLIT >= 0 is the split known at compile time (exact T).
template <int AM, int SPLIT, class A>
__device__ __forceinline__ bool second_group(const A &a, int i) {
    return AM == 2 && (SPLIT >= 0 ? i >= SPLIT : i >= a.split);
}

__device__ __forceinline__ float2 ld_plane(__amdgpu_buffer_rsrc_t r,
                                           uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float2,
                              __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// Element e of the packed planes, clamped into the planes (an out-of-image
// lane's offset may wrap; its value is discarded by the caller).
template <int AM, int SPLIT, class A>
__device__ __forceinline__ float2 ld_elem(const A &a, const PlaneRsrc &r, int i, uint32_t e) {
    const bool g1 = second_group<AM, SPLIT>(a, i);
    const uint32_t c = min(e, (g1 ? a.n_elem2 : a.n_elem) - 1u);
    if (AM > 0) return ld_plane(g1 ? r.r1 : r.r0, c * 8u, 0u);
    return a.pk[c];
}

// Packed sample of one pixel-epoch: (psi / sqrt(phi), sqrt(phi)), both
// correctly rounded binary32, or (NaN, 0) when the pixel-epoch is unusable
// (phi <= 0 or a non-finite value).  Sets bad for an unusable one.
__device__ __forceinline__ float2 pack_sample(float psi, float phi, bool &bad) {
    const bool ok = phi > 0.0f && isfinite(phi) && isfinite(psi);
    const float sb = sqrtf(phi);
    bad |= !ok;
    return ok ? make_float2(psi / sb, sb) : make_float2(__builtin_nanf(""), 0.0f);
}

// L = Psi / sqrt(Phi) as the search ranks and stores it: one hardware
// reciprocal square root (1 ulp) and a product, a few ulp from the
// correctly rounded quotient.  Every kernel that forms a search likelihood
// uses this one function, so equal inputs give equal bits everywhere.
__device__ __forceinline__ float lh_value(float P, float F) {
    return P * __builtin_amdgcn_rsqf(F);
}

struct Score {
    float L, flux;
    uint64_t keep;
};

// Filtered (or plain) likelihood of one lightcurve.  For i < T, nu[i] is NaN
// for an unusable epoch and s[i] = 0; entries i >= T are padding (+inf, 0).
// SEL selects the NaN handling needed when unusable epochs may be present.
template <int TM, bool SEL, bool EXACT, class A>
__device__ __forceinline__ Score score(const A &a,
                                       const float (&nu)[TM],
                                       const float (&s)[TM], int nv) {
    const int T = EXACT ? TM : a.T;
    Score r;
    float P = 0.0f, F = 0.0f;
    uint32_t lo = 0, hi = 0;
    if (a.sigmag) {
        const KBM_CONST int *rk = cst(a.ranks);
        const int rl = rk[nv], rm = rk[65 + nv], rh = rk[130 + nv];
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
    r.L = lh_value(P, F);
    r.flux = P / F;
    return r;
}

// Clean, exact-T fast path with the default quantiles (0.25, 0.75): every
// epoch is usable, the nearest ranks floor(q (T-1) + 1/2) are compile-time
// constants, and the kept sums zero s instead of selecting twice.
template <int T, class A>
__device__ __forceinline__ float score_fixed(const A &a,
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
    return lh_value(P, F);
}

// Nearest ranks floor(q (n-1) + 1/2) of the default quantiles 1/4, 1/2, 3/4
// in integer form (exact: (n+1)/4, n/2, (3n-1)/4 rounded down).
constexpr int rank_q1(int n) { return n < 1 ? 0 : (n + 1) / 4; }
constexpr int rank_q2(int n) { return n < 1 ? 0 : n / 2; }
constexpr int rank_q3(int n) { return n < 1 ? 0 : (3 * n - 1) / 4; }

// Sorted value at the rank of n = nv usable epochs, for nv in [T-3, T]:
// four compile-time positions and a pick by nv.
template <int T, int R0, int R1, int R2, int R3>
__device__ __forceinline__ float pick_near(const float (&srt)[T], int nv) {
    const float v0 = srt[R0], v1 = srt[R1], v2 = srt[R2], v3 = srt[R3];
    return nv == T ? v0 : nv == T - 1 ? v1 : nv == T - 2 ? v2 : v3;
}

// Filtered likelihood with the default quantiles when every lane has at
// least T-3 usable epochs (unusable ones are NaN and sort last): the sorting
// network only has to produce the positions the ranks of T..T-3 usable
// epochs reach (7 of 26 for T = 26), so it is pruned almost as far as the
// all-usable network.  Same sorted values, ranks and arithmetic as score().
template <int T, class A>
__device__ __forceinline__ float score_near(const A &a, const float (&nu)[T],
                                            const float (&s)[T], int nv) {
#pragma clang fp contract(off)
    float srt[T];
#pragma unroll
    for (int i = 0; i < T; ++i) srt[i] = (nu[i] == nu[i]) ? nu[i] : INFINITY;
    sort_network<T>(srt);
    const float x_lo =
        pick_near<T, rank_q1(T), rank_q1(T - 1), rank_q1(T - 2), rank_q1(T - 3)>(srt, nv);
    const float x_md =
        pick_near<T, rank_q2(T), rank_q2(T - 1), rank_q2(T - 2), rank_q2(T - 3)>(srt, nv);
    const float x_hi =
        pick_near<T, rank_q3(T), rank_q3(T - 1), rank_q3(T - 2), rank_q3(T - 3)>(srt, nv);
    SigmaGCut c;
    c.x_md = x_md;
    c.thr = a.n_sigma * (a.coeff * (x_hi - x_lo));
    float P = 0.0f, F = 0.0f;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        const bool k = c.keeps(nu[i]);
        P = fmaf(k ? nu[i] : 0.0f, s[i], P);
        F = fmaf(k ? s[i] : 0.0f, s[i], F);
    }
    return lh_value(P, F);
}

// One velocity's per-epoch offsets.  Up to 32 epochs they are loaded into
// scalar registers when constructed; above that the row stays in memory and
// each entry is loaded where it is used (holding 33..64 offsets would spill
// scalar registers).
template <int TM, bool HOLD = (TM <= 32)>
struct LinRow;
template <int TM>
struct LinRow<TM, true> {
    uint32_t v[TM];
    __device__ __forceinline__ LinRow(const KBM_CONST uint32_t *p, int T) {
#pragma unroll
        for (int i = 0; i < TM; ++i) v[i] = i < T ? p[i] : 0u;
    }
    __device__ __forceinline__ uint32_t operator[](int i) const { return v[i]; }
};
template <int TM>
struct LinRow<TM, false> {
    const KBM_CONST uint32_t *p;
    __device__ __forceinline__ LinRow(const KBM_CONST uint32_t *q, int) : p(q) {}
    __device__ __forceinline__ uint32_t operator[](int i) const { return p[i]; }
};

// Whole-wave in-bounds load: the per-epoch offset is wave-uniform.
// Leading epochs whose samples a wave keeps from one velocity to the next
// (the carried registers); past these every epoch is loaded.
constexpr int KBM_CARRY = 10;

// Epochs below KBM_CARRY whose bit is set in `keep` (wave-uniform) are not
// loaded: nu and s still hold this wave's samples of the previous velocity
// it swept, whose offsets for those epochs are the same.
template <int TM, bool CLEAN, bool EXACT, int AM, class A, class LV>
__device__ __forceinline__ int load_fast(const A &a,
                                         const PlaneRsrc &rs,
                                         uint32_t lane, uint32_t wave_e,
                                         const LV &lv, int keep, float (&nu)[TM],
                                         float (&s)[TM]) {
    const int T = EXACT ? TM : a.T;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        if (i < T) {
            if (i >= KBM_CARRY || !((keep >> i) & 1)) {
                const uint32_t e = wave_e + lv[i];
                const float2 q =
                    AM > 0 ? ld_plane(second_group<AM, EXACT ? TM / 2 : -1>(a, i) ? rs.r1
                                                                                  : rs.r0,
                                      lane * 8u, e * 8u)
                           : a.pk[(size_t)e + lane];
                nu[i] = q.x;
                s[i] = q.y;
            }
        } else {
            nu[i] = INFINITY;
            s[i] = 0.0f;
        }
    }
    if (CLEAN) return T;
    int nv = 0;
#pragma unroll
    for (int i = 0; i < TM; ++i)
        if (i < T) nv += (nu[i] == nu[i]) ? 1 : 0;
    return nv;
}

// General load with per-lane bounds checks.
template <int TM, bool EXACT, int AM, class A, class LV>
__device__ __forceinline__ int load_slow(const A &a,
                                         const PlaneRsrc &rs, int x,
                                         int y, const KBM_CONST int *ov,
                                         const LV &lv, float (&nu)[TM],
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
            const float2 q = ld_elem<AM, EXACT ? TM / 2 : -1>(a, rs, i, lv[i] + pix);
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

// Sweep velocities [v_begin, v_end) for the tile's 64 start pixels.  With
// first set the running lists start empty, else they are read from the
// workspace; they are written back at the end.  mL/mI point to an LDS block
// of (NW-1)*KM*WAVE entries each (unused when NW == 1).
template <int TM, int KM, bool CLEAN, bool EXACT, int AM, int NWT = NW, bool CONTIG = false,
          class A>
__device__ __forceinline__ void run_chunk(const A &a, int tx, int ty,
                                          int v_begin, int v_end, bool first,
                                          float *mL, int *mI) {
    // NWT waves share this tile's 64 start pixels and split the chunk's
    // velocities between them (interleaved or in contiguous shares, below).
    const unsigned lane = threadIdx.x % WAVE;
    const int w = NWT > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE)) : 0;
    const int rx = tx * WAVE + (int)lane, ry = ty;
    const bool active = rx < a.Wr;
    const int xw = a.x0 + tx * WAVE;
    const int x = xw + (int)lane, y = a.y0 + ry;
    const size_t npix = (size_t)a.Wr * a.Hr;
    const size_t pix = (size_t)ry * a.Wr + (active ? rx : 0);
    const int T = EXACT ? TM : a.T;
    const PlaneRsrc rs = plane_rsrc(a);

    // Wave 0 continues the pixel's running list.  The other waves start
    // from K copies of that list's K-th best L with index -1: only a
    // trajectory that beats it can reach the merged top K (an equal L loses
    // the tie to the older entry), so they insert as rarely as wave 0 does,
    // and the merge skips the index -1 fillers.
    float thr = -INFINITY;
    if (!first && active && w != 0) thr = a.stL[(size_t)(a.K - 1) * npix + pix];
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
        } else if (first || !active || w != 0) {
            kL[j] = thr;
            kI[j] = -1;
        } else {
            kL[j] = a.stL[(size_t)slot * npix + pix];
            kI[j] = a.stI[(size_t)slot * npix + pix];
        }
    }

    // Lanes past the region end never insert: their candidate is clamped to
    // -inf by a per-lane value.  The empty asm hides where the value comes
    // from, so the compiler keeps one VGPR instead of turning the clamp back
    // into a select on a lane mask held in scalar registers for the whole
    // sweep (which it spills).  In a stack without unusable samples every
    // fast-path trajectory has n_obs = T, so the min_obs test is folded into
    // the gate as well.
    float gate = (active && (!CLEAN || T >= a.min_obs)) ? INFINITY : -INFINITY;
    asm volatile("" : "+v"(gate));
    const uint32_t wave_e = (uint32_t)(y * a.W + xw);
    // The first KBM_CARRY entries of nu and s carry over between velocities:
    // `have` says they hold the fast-path samples of the previous velocity
    // this wave swept (v - NWT interleaved, v - 1 contiguous).  Not above 32
    // epochs, where the carried registers would cost occupancy.
    constexpr int NC = TM > 32 ? 0 : TM < KBM_CARRY ? TM : KBM_CARRY;
    float cnu[NC > 0 ? NC : 1], cs[NC > 0 ? NC : 1];
#pragma unroll
    for (int i = 0; i < (NC > 0 ? NC : 1); ++i) {
        cnu[i] = 0.0f;
        cs[i] = 0.0f;
    }
    int have = 0;
    // Wave w sweeps v_begin + w, v_begin + w + NWT, ... (interleaved: the
    // waves read nearly the same rows at a time) or, with CONTIG, the w-th
    // contiguous share of [v_begin, v_end) (consecutive velocities repeat
    // more offsets, whose samples stay in registers).
    const int span = CONTIG ? (v_end - v_begin + NWT - 1) / NWT : 0;
    const int v_first = CONTIG ? v_begin + w * span : v_begin + w;
    const int v_last = CONTIG ? min(v_end, v_first + span) : v_end;
    constexpr int v_step = CONTIG ? 1 : NWT;
    constexpr int same_at = (CONTIG || NWT == 1) ? 4 : 5;
    for (int v = v_first; v < v_last; v += v_step) {
        // The velocity's box (and for T <= 32 its offset row) is read up
        // front, as one batch of scalar loads with one wait, and the box
        // test combines its four comparisons without short-circuit branches
        // (each branch would wait for its own scalar load).
        const int4 bx = ld_box(a.vbox, 2 * v);
        const int same = cst((const int *)a.vbox)[8 * (size_t)v + same_at];
        const LinRow<TM> lv(cst(a.lin) + (size_t)v * T, T);
        const bool fast = (xw + bx.x >= 0) & (xw + (WAVE - 1) + bx.y < a.W) &
                          (y + bx.z >= 0) & (y + bx.w < a.H);
        if (!fast) {
            // Sound skip: if fewer than min_obs epochs can hold any lane of
            // this wave in the image (per axis), no lane reaches min_obs.
            const int4 mb = ld_box(a.mbox, v);
            if (xw + mb.x > a.W - 1 || xw + (WAVE - 1) + mb.y < 0 ||
                y + mb.z > a.H - 1 || y + mb.w < 0) {
                have = 0;
                continue;
            }
        }
        float nu[TM], s[TM];
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            nu[i] = cnu[i];
            s[i] = cs[i];
        }
        int nv;
        Score sc;
        if (fast) {
            nv = load_fast<TM, CLEAN, EXACT, AM>(
                a, rs, lane, wave_e, lv, (NC > 0 && have && (CONTIG || NWT == 1 || NWT == 4)) ? same : 0,
                nu, s);
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                cnu[i] = nu[i];
                cs[i] = s[i];
            }
            have = 1;
            if (EXACT && CLEAN && a.defq)
                sc.L = score_fixed<TM>(a, nu, s);
            else if (EXACT && !CLEAN && TM >= 4 && a.defq && a.sigmag &&
                     __all(nv >= TM - 3))
                sc.L = score_near<TM>(a, nu, s, nv);
            else
                sc = score<TM, !CLEAN, EXACT>(a, nu, s, nv);
        } else {
            nv = load_slow<TM, EXACT, AM>(a, rs, x, y, cst(a.off16) + (size_t)v * T, lv,
                                          nu, s);
            have = 0;
            sc = score<TM, true, EXACT>(a, nu, s, nv);
        }
        // Velocities reach a lane in increasing index order (within the
        // sweep, across chunks, and in the state read back), so v exceeds
        // every index in the list: under the tie rule an equal L keeps the
        // older entry, and ranks_before(L, v, x, i) reduces to L > x.  The
        // insertion itself is branch-free: c_j = (L > kL[j]) is false then
        // true down the descending list, so slot j takes kL[j] before the
        // insertion point, L at it and kL[j-1] after it; a lane that does
        // not insert uses L = -inf, for which every c_j is false.  Once the
        // lists hold good entries most velocities insert in no lane of the
        // wave, which then skips the block.
        const bool obs_ok = (CLEAN && fast) || nv >= a.min_obs;
        const float xL = __builtin_elementwise_minimum(
            (obs_ok && isfinite(sc.L)) ? sc.L : -INFINITY, gate);
        if (__any(xL > kL[KM - 1])) {
#pragma unroll
            for (int j = KM - 1; j > 0; --j) {
                const bool cj = xL > kL[j], cp = xL > kL[j - 1];
                kL[j] = cp ? kL[j - 1] : (cj ? xL : kL[j]);
                kI[j] = cp ? kI[j - 1] : (cj ? v : kI[j]);
            }
            const bool c0 = xL > kL[0];
            kL[0] = c0 ? xL : kL[0];
            kI[0] = c0 ? v : kI[0];
        }
    }
    if (NWT > 1) {
        // Merge the waves' lists into wave 0's through LDS.  The ranking
        // compares velocity indices on ties, so the merge order is immaterial.
        if (w > 0) {
#pragma unroll
            for (int j = 0; j < KM; ++j) {
                mL[((w - 1) * KM + j) * WAVE + lane] = kL[j];
                mI[((w - 1) * KM + j) * WAVE + lane] = kI[j];
            }
        }
        __syncthreads();
        if (w != 0) return;
        for (int o = 0; o < NWT - 1; ++o) {
#pragma unroll
            for (int j = 0; j < KM; ++j) {
                const float L = mL[(o * KM + j) * WAVE + lane];
                const int v = mI[(o * KM + j) * WAVE + lane];
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

template <int TM, int KM, bool EXACT, int AM>
__global__ __launch_bounds__(WAVE * NW)
__attribute__((amdgpu_waves_per_eu(1, KBM_MAX_WAVES_PER_SIMD)))
void search_chunk_kernel(SearchArgs a) {
    __shared__ float mL[NW > 1 ? (NW - 1) * KM * WAVE : 1];
    __shared__ int mI[NW > 1 ? (NW - 1) * KM * WAVE : 1];
    int tx, ty;
    if (!map_tile(a, tx, ty)) return;
    if (cst(a.flags)[0] == 0)
        run_chunk<TM, KM, true, EXACT, AM>(a, tx, ty, a.v_begin, a.v_end, a.first, mL, mI);
    else
        run_chunk<TM, KM, false, EXACT, AM>(a, tx, ty, a.v_begin, a.v_end, a.first, mL, mI);
}

// Re-evaluate the K winners of start pixel (x, y) (flat result index pix
// within the region) from the running lists and write all result fields.
template <int TM, bool EXACT, int AM, class A>
__device__ __forceinline__ void finalize_pixel(const A &a,
                                               const PlaneRsrc &rs, int x,
                                               int y, size_t pix) {
    const size_t npix = (size_t)a.Wr * a.Hr;
    const int T = EXACT ? TM : a.T;
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
        const int nv = load_slow<TM, EXACT, AM>(a, rs, x, y, cst(a.off16) + (size_t)vi * T,
                                                    cst(a.lin) + (size_t)vi * T, nu, s);
        const Score sc = score<TM, true, EXACT>(a, nu, s, nv);
        a.lh[o] = sc.L;
        a.flux[o] = sc.flux;
        a.vidx[o] = vi;
        a.nobs[o] = (int16_t)nv;
        a.keep[o] = sc.keep;
        if (a.lh_raw) {
            float P = 0.0f, F = 0.0f;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                if (i < T) {
                    P = fmaf(nu[i] == nu[i] ? nu[i] : 0.0f, s[i], P);
                    F = fmaf(s[i], s[i], F);
                }
            }
            a.lh_raw[o] = lh_value(P, F);
        }
    }
}

template <int TM, int AM>
__global__ __launch_bounds__(256) void finalize_kernel(SearchArgs a) {
    const size_t npix = (size_t)a.Wr * a.Hr;
    const size_t pix = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= npix) return;
    const int rx = (int)(pix % a.Wr), ry = (int)(pix / a.Wr);
    finalize_pixel<TM, false, AM>(a, plane_rsrc(a), a.x0 + rx, a.y0 + ry, pix);
}

// Launch the chunk sequence for one kernel variant.
template <int TM, int KM, bool EXACT, int AM>
void launch_chunks(SearchArgs a, hipStream_t stream) {
    for (int v0 = 0; v0 < a.V; v0 += VCHUNK) {
        a.v_begin = v0;
        a.v_end = v0 + VCHUNK < a.V ? v0 + VCHUNK : a.V;
        a.first = v0 == 0;
        hipLaunchKernelGGL((search_chunk_kernel<TM, KM, EXACT, AM>), dim3(a.n_tiles),
                           dim3(WAVE * NW), 0, stream, a);
    }
}

// Exact-epoch-count variants (buffer-addressed stacks, K <= 8) live in
// separate translation units; each returns true when it handled T.
bool launch_exact_a(int T, const SearchArgs &a, hipStream_t stream);
bool launch_exact_b(int T, const SearchArgs &a, hipStream_t stream);

}  // namespace srch
}  // namespace kbm

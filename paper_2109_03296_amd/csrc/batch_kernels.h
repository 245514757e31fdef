// Device side of the batched persistent search: work-item dispatch and the
// per-epoch-count item bodies.  Included by one translation unit per
// wavefront count (they compile in parallel); the schedule is described in
// batch.hip.
#pragma once

#include "search_kernels.h"

namespace kbm {
namespace batch {

using srch::NUM_XCD;
using srch::SearchArgs;
using srch::WAVE;
using srch::cst;

constexpr int BKM = 8;            // list registers (k <= 8)
constexpr int MAX_T = 32;         // exact epoch counts compiled in
constexpr int PAD_COLS = 16;      // every allowed tile_cols divides this
constexpr int PAD_ROWS = 64;      // every allowed tile_rows divides this
constexpr int MIN_VB = 32;
constexpr int CTRL_HEAD = 64;     // words: queue heads [0, 8), stall flag [8]
constexpr uint32_t SPIN_LIMIT = 1u << 20;  // polls before a wait gives up

struct PrepDesc {
    const float *psi;
    const float *phi;
    float2 *pk;
    int *flag;
    uint64_t n;
};

struct StackInfo {
    uint32_t prog_off;   // first progress counter of the stack
    uint32_t n_tiles;    // padded tile count (whole super-tiles)
    uint32_t n_super_y;  // super-tiles per column strip
    uint32_t probe_off;  // autotuner probes: first tile of each queue's share
                         // taken, relative to the share's start (else 0)
};

// Register budget of the batched kernel: at least this many waves per SIMD
// (3: up to 168 VGPRs per lane).
#ifndef KBM_BATCH_MIN_WAVES
#define KBM_BATCH_MIN_WAVES 3
#endif

// Merge buffers of the four-wave variant (the only code that touches them,
// so single-wave kernels allocate no LDS for them).
__shared__ float g_mL[3 * BKM * WAVE];
__shared__ int g_mI[3 * BKM * WAVE];

__device__ __forceinline__ const KBM_CONST SearchArgs *uniform_desc(const SearchArgs *d,
                                                                    int s) {
    const uint64_t p = (uint64_t)d;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)p);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(p >> 32));
    return (const KBM_CONST SearchArgs *)(((uint64_t)hi << 32) | lo) +
           __builtin_amdgcn_readfirstlane(s);
}

// One work item for epoch count T.  Kept out of line so every epoch count
// is register-allocated on its own; all arguments are wave-uniform and are
// made scalar again on entry.
template <int T, int NWT, bool CONTIG>
static __device__ __noinline__ void batch_tile(const SearchArgs *descs, int s, int tx, int ty,
                                        int v0, int v1, int flags) {
    const KBM_CONST SearchArgs &a = *uniform_desc(descs, s);
    tx = __builtin_amdgcn_readfirstlane(tx);
    ty = __builtin_amdgcn_readfirstlane(ty);
    v0 = __builtin_amdgcn_readfirstlane(v0);
    v1 = __builtin_amdgcn_readfirstlane(v1);
    flags = __builtin_amdgcn_readfirstlane(flags);
    const bool first = flags & 1, last = flags & 2;
    float *mL = NWT > 1 ? g_mL : nullptr;
    int *mI = NWT > 1 ? g_mI : nullptr;
    if (cst(a.flags)[0] == 0)
        srch::run_chunk<T, BKM, true, true, 1, NWT, CONTIG>(a, tx, ty, v0, v1, first, mL, mI);
    else
        srch::run_chunk<T, BKM, false, true, 1, NWT, CONTIG>(a, tx, ty, v0, v1, first, mL, mI);
    if (!last) return;
    const int w = NWT > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE)) : 0;
    const int rx = tx * WAVE + (int)(threadIdx.x % WAVE);
    if (w != 0 || rx >= a.Wr) return;
    srch::finalize_pixel<T, true, 1>(a, srch::plane_rsrc(a), a.x0 + rx, a.y0 + ty,
                                        (size_t)ty * a.Wr + rx);
}

#define KBM_BATCH_CASE(n)                                                      \
    case n:                                                                    \
        batch_tile<n, NWT, CONTIG>(descs, s, tx, ty, v0, v1, flags);           \
        break;

template <int NWT, bool CONTIG>
__global__ __launch_bounds__(WAVE * NWT)
__attribute__((amdgpu_waves_per_eu(KBM_BATCH_MIN_WAVES, 8)))
void batch_kernel(const SearchArgs *__restrict__ descs,
                  const StackInfo *__restrict__ info,
                  const uint32_t *__restrict__ pre, const int2 *__restrict__ seg,
                  uint32_t *ctrl, uint32_t *prog, int nseg, int vbs, int st_x,
                  int st_y) {
    __shared__ int item[3];
    int q = blockIdx.x % NUM_XCD, hops = 0;  // thread 0's queue cursor
    for (;;) {
        if (threadIdx.x == 0) {
            int s = -1, vb = 0, t = 0;
            while (hops < NUM_XCD) {
                const KBM_CONST uint32_t *pq = cst(pre) + (size_t)q * (nseg + 1);
                const uint32_t n = pq[nseg];
                uint32_t i = n;
                if (__hip_atomic_load(ctrl + q, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT) < n)
                    i = atomicAdd(ctrl + q, 1u);
                if (i < n) {
                    int lo = 0, hi = nseg;  // pq[lo] <= i < pq[hi]
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (pq[mid] <= i) lo = mid;
                        else hi = mid;
                    }
                    const KBM_CONST int *g = (const KBM_CONST int *)seg + 2 * lo;
                    s = g[0];
                    vb = g[1];
                    t = (int)(cst(info)[s].n_tiles * (uint32_t)q / NUM_XCD +
                              cst(info)[s].probe_off + (i - pq[lo]));
                    break;
                }
                ++hops;
                q = (q + 1) % NUM_XCD;
            }
            item[0] = s;
            item[1] = vb;
            item[2] = t;
        }
        __syncthreads();
        const int s = __builtin_amdgcn_readfirstlane(item[0]);
        const int vb = __builtin_amdgcn_readfirstlane(item[1]);
        const int t = __builtin_amdgcn_readfirstlane(item[2]);
        __syncthreads();
        if (s < 0) break;

        const KBM_CONST SearchArgs &a = cst(descs)[s];
        const int n_super_y = (int)cst(info)[s].n_super_y;
        const uint32_t prog_off = cst(info)[s].prog_off;
        const int sts = st_x * st_y;
        const int st = t / sts, wi = t - st * sts;
        const int sx = st / n_super_y, sy = st - sx * n_super_y;
        const int tx = sx * st_x + wi % st_x, ty = sy * st_y + wi / st_x;
        if (tx >= a.tiles_x || ty >= a.Hr) continue;  // padding tile
        uint32_t *pc = prog + prog_off + t;
        if (vb > 0) {
            if (threadIdx.x == 0) {
                uint32_t n = 0;
                while (__hip_atomic_load(pc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                       (uint32_t)vb) {
                    if (++n > SPIN_LIMIT) {
                        atomicOr(ctrl + NUM_XCD, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
        }
        const int v0 = vb * vbs, v1 = min(a.V, v0 + vbs);
        const int flags = (vb == 0 ? 1 : 0) | (v1 == a.V ? 2 : 0);
        switch (a.T) {
            KBM_BATCH_CASE(1) KBM_BATCH_CASE(2) KBM_BATCH_CASE(3) KBM_BATCH_CASE(4)
            KBM_BATCH_CASE(5) KBM_BATCH_CASE(6) KBM_BATCH_CASE(7) KBM_BATCH_CASE(8)
            KBM_BATCH_CASE(9) KBM_BATCH_CASE(10) KBM_BATCH_CASE(11) KBM_BATCH_CASE(12)
            KBM_BATCH_CASE(13) KBM_BATCH_CASE(14) KBM_BATCH_CASE(15) KBM_BATCH_CASE(16)
            KBM_BATCH_CASE(17) KBM_BATCH_CASE(18) KBM_BATCH_CASE(19) KBM_BATCH_CASE(20)
            KBM_BATCH_CASE(21) KBM_BATCH_CASE(22) KBM_BATCH_CASE(23) KBM_BATCH_CASE(24)
            KBM_BATCH_CASE(25) KBM_BATCH_CASE(26) KBM_BATCH_CASE(27) KBM_BATCH_CASE(28)
            KBM_BATCH_CASE(29) KBM_BATCH_CASE(30) KBM_BATCH_CASE(31) KBM_BATCH_CASE(32)
            default: break;
        }
        // The item's waves must all have left run_chunk (wave 0 wrote the
        // lists) before the lists are published.
        __syncthreads();
        if (!(flags & 2) && threadIdx.x == 0)
            __hip_atomic_store(pc, (uint32_t)(vb + 1), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Launch of batch_kernel<NWT, CONTIG> and its occupancy (workgroups per
// CU); one translation unit per wavefront count and sweep order.
struct BatchLaunch {
    const SearchArgs *descs;
    const StackInfo *info;
    const uint32_t *pre;
    const int2 *seg;
    uint32_t *ctrl, *prog;
    int nseg, vbs, st_x, st_y;
};
hipError_t launch_batch_nw1(const BatchLaunch &l, unsigned grid, hipStream_t stream);
hipError_t launch_batch_nw4(const BatchLaunch &l, unsigned grid, hipStream_t stream);
hipError_t launch_batch_nw1c(const BatchLaunch &l, unsigned grid, hipStream_t stream);
hipError_t launch_batch_nw4c(const BatchLaunch &l, unsigned grid, hipStream_t stream);
hipError_t occupancy_nw1(int *blocks);
hipError_t occupancy_nw4(int *blocks);
hipError_t occupancy_nw1c(int *blocks);
hipError_t occupancy_nw4c(int *blocks);

}  // namespace batch
}  // namespace kbm

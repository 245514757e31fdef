// Candidate extraction: the global top-N of the per-pixel results by the
// filtered likelihood, above a threshold (trajectories with a large enough
// recomputed likelihood leave the GPU, Section 3.1; the per-pixel lists of
// Section 3.2 are the input).
//
// Every result slot gets a 64-bit key: the order-preserving bit pattern of
// its likelihood in the high word and the complement of its flat slot index
// in the low word, so keys are unique and "larger key" means "higher L',
// then smaller index".  An 8-pass radix select (8 bits per pass, histograms
// in LDS then global atomics) finds the N-th largest key (it stops early
// once the bucket of the N-th key is taken whole: then every key at or above
// the prefix found so far is selected, which with distinct likelihoods
// happens after the four passes over the likelihood bits); an ordered
// compaction (block counts, one scan, block-local ballot ranks) then writes
// the selected slots in flat-index order.  Slots below the threshold, empty
// or non-finite never take part.
#include <map>
#include <mutex>
#include <vector>

#include "kbm_internal.h"

namespace kbm {
namespace {

constexpr int EX_THREADS = 256;
constexpr int EX_BLOCKS_MAX = 4096;

struct ExtractState {
    unsigned long long prefix;  // selected high bits of the threshold key
    unsigned long long remain;  // how many keys still to take at this prefix
    unsigned long long total;   // eligible slots
    unsigned int none;          // nothing to select (no eligible slot, or N = 0)
    unsigned int done;          // prefix is final: the remaining passes do nothing
    unsigned int hist[256];
};

__device__ __forceinline__ uint32_t f32_order(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ bool eligible(float L, float lh_min) {
    return isfinite(L) && L >= lh_min;
}

__device__ __forceinline__ unsigned long long slot_key(float L, uint64_t idx) {
    return ((unsigned long long)f32_order(L) << 32) |
           (unsigned long long)(0xffffffffu - (uint32_t)idx);
}

__global__ __launch_bounds__(256) void ex_init_kernel(ExtractState *st, uint64_t n_max) {
    if (threadIdx.x == 0) {
        st->prefix = 0;
        st->remain = n_max;
        st->total = 0;
        st->none = 0;
        st->done = 0;
    }
    st->hist[threadIdx.x] = 0;
}

// Histogram of key byte `pass` (0 = most significant) over eligible slots
// whose higher bytes equal the current prefix.  Pass 0 also counts them.
__global__ __launch_bounds__(EX_THREADS) void ex_hist_kernel(
    const float *__restrict__ lh, uint64_t n, float lh_min, int pass,
    ExtractState *st) {
    if (st->done) return;
    __shared__ unsigned int h[256];
    __shared__ unsigned long long cnt;
    h[threadIdx.x] = 0;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int shift = 56 - 8 * pass;
    const unsigned long long pre = st->prefix;
    const unsigned long long mask = pass == 0 ? 0ull : (~0ull << (64 - 8 * pass));
    unsigned long long local = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * EX_THREADS + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * EX_THREADS) {
        const float L = lh[i];
        if (!eligible(L, lh_min)) continue;
        ++local;
        const unsigned long long key = slot_key(L, i);
        if ((key & mask) != pre) continue;
        atomicAdd(&h[(key >> shift) & 0xff], 1u);
    }
    if (pass == 0 && local) atomicAdd(&cnt, local);
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
    if (pass == 0 && threadIdx.x == 0 && cnt) atomicAdd(&st->total, cnt);
}

// Choose the byte of the N-th largest key at this pass (scan from 255 down).
// After the eighth pass `prefix` is that key; exactly N keys are >= it.  If
// the chosen bucket holds exactly the keys still needed, all of them are
// taken: `prefix` with its lower bytes zero is then already a threshold with
// exactly N keys >= it, and the remaining passes are skipped.
__global__ __launch_bounds__(256) void ex_pick_kernel(ExtractState *st, int pass) {
    if (st->done) return;
    __syncthreads();  // every thread has read `done` before thread 0 may set it
    if (threadIdx.x == 0) {
        if (pass == 0) {
            if (st->total < st->remain) st->remain = st->total;
            st->none = st->remain == 0;
        }
        unsigned long long need = st->remain;
        const int shift = 56 - 8 * pass;
        if (need > 0) {
            int b = 255;
            for (; b > 0; --b) {
                const unsigned long long c = st->hist[b];
                if (c >= need) break;
                need -= c;
            }
            st->prefix |= (unsigned long long)b << shift;
            st->done = st->hist[b] == need;
            st->remain = need;
        }
    }
    __syncthreads();
    st->hist[threadIdx.x] = 0;
}

// Per-block count of selected slots (key >= threshold).
__global__ __launch_bounds__(EX_THREADS) void ex_count_kernel(
    const float *__restrict__ lh, uint64_t n, float lh_min, uint64_t per_block,
    const ExtractState *st, unsigned int *block_cnt) {
    __shared__ unsigned int c;
    if (threadIdx.x == 0) c = 0;
    __syncthreads();
    const unsigned long long thr = st->prefix;
    const bool any = !st->none;
    const uint64_t b0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t b1 = b0 + per_block < n ? b0 + per_block : n;
    unsigned int local = 0;
    if (any)
        for (uint64_t i = b0 + threadIdx.x; i < b1; i += EX_THREADS) {
            const float L = lh[i];
            if (eligible(L, lh_min) && slot_key(L, i) >= thr) ++local;
        }
    if (local) atomicAdd(&c, local);
    __syncthreads();
    if (threadIdx.x == 0) block_cnt[blockIdx.x] = c;
}

// Exclusive scan of the block counts (one workgroup) and the output count.
__global__ __launch_bounds__(256) void ex_scan_kernel(unsigned int *block_cnt, int nb,
                                                      int64_t *n_out) {
    __shared__ unsigned long long part[256];
    const int per = (nb + 255) / 256;
    const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    unsigned long long s = 0;
    for (int b = b0; b < b1; ++b) s += block_cnt[b];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long acc = 0;
        for (int t = 0; t < 256; ++t) {
            const unsigned long long v = part[t];
            part[t] = acc;
            acc += v;
        }
        *n_out = (int64_t)acc;
    }
    __syncthreads();
    unsigned long long acc = part[threadIdx.x];
    for (int b = b0; b < b1; ++b) {
        const unsigned int v = block_cnt[b];
        block_cnt[b] = (unsigned int)acc;
        acc += v;
    }
}

struct ExtractOut {
    const float *lh;
    const float *flux;
    const int32_t *vidx;
    const int16_t *nobs;
    const uint64_t *keep;
    const float *vel;    // device [V][2]
    float *params;       // [n_max][4]
    float *out_lh;
    float *out_flux;
    uint64_t *out_keep;
    int64_t *out_index;
    int16_t *out_nobs;
    int Wr, K, x0, y0;
};

// Ordered write: a block walks its range in chunks of EX_THREADS slots and
// ranks the selected ones with wave ballots.
__global__ __launch_bounds__(EX_THREADS) void ex_write_kernel(
    ExtractOut o, uint64_t n, float lh_min, uint64_t per_block,
    const ExtractState *st, const unsigned int *block_off) {
    __shared__ unsigned int wave_tot[EX_THREADS / 64];
    const unsigned long long thr = st->prefix;
    if (st->none) return;
    const uint64_t b0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t b1 = b0 + per_block < n ? b0 + per_block : n;
    unsigned int base = block_off[blockIdx.x];
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    for (uint64_t c0 = b0; c0 < b1; c0 += EX_THREADS) {
        const uint64_t i = c0 + threadIdx.x;
        bool sel = false;
        if (i < b1) {
            const float L = o.lh[i];
            sel = eligible(L, lh_min) && slot_key(L, i) >= thr;
        }
        const unsigned long long bal = __ballot(sel);
        const unsigned int below = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wave_tot[wv] = __popcll(bal);
        __syncthreads();
        unsigned int off = 0, tot = 0;
        for (int w = 0; w < EX_THREADS / 64; ++w) {
            if (w < wv) off += wave_tot[w];
            tot += wave_tot[w];
        }
        if (sel) {
            const uint64_t pos = base + off + below;
            const uint64_t pix = i / o.K;
            const int vi = o.vidx[i];
            o.params[4 * pos + 0] = (float)(o.x0 + (int)(pix % o.Wr));
            o.params[4 * pos + 1] = (float)(o.y0 + (int)(pix / o.Wr));
            o.params[4 * pos + 2] = o.vel[2 * vi];
            o.params[4 * pos + 3] = o.vel[2 * vi + 1];
            o.out_lh[pos] = o.lh[i];
            if (o.out_flux) o.out_flux[pos] = o.flux[i];
            if (o.out_keep) o.out_keep[pos] = o.keep[i];
            if (o.out_index) o.out_index[pos] = (int64_t)i;
            if (o.out_nobs) o.out_nobs[pos] = o.nobs[i];
        }
        base += tot;
        __syncthreads();
    }
}

struct ExLayout {
    size_t st_off, cnt_off, vel_off, end;
    int nb;
    uint64_t per_block;
};

ExLayout ex_layout(uint64_t n, int num_vel) {
    ExLayout l;
    l.nb = (int)std::min<uint64_t>(EX_BLOCKS_MAX, (n + EX_THREADS - 1) / EX_THREADS);
    if (l.nb < 1) l.nb = 1;
    l.per_block = (n + l.nb - 1) / l.nb;
    l.st_off = 0;
    l.cnt_off = align_up(sizeof(ExtractState), 256);
    l.vel_off = align_up(l.cnt_off + sizeof(unsigned int) * l.nb, 256);
    l.end = l.vel_off + sizeof(float) * 2 * (size_t)num_vel;
    return l;
}

}  // namespace
}  // namespace kbm

extern "C" kbm_status kbm_extract_workspace_size(int32_t Hr, int32_t Wr, int32_t k,
                                                 int32_t num_vel, size_t *bytes) {
    using namespace kbm;
    clear_error();
    KBM_REQUIRE(bytes && Hr >= 0 && Wr >= 0 && k >= 1 && k <= KBM_MAX_K && num_vel >= 1,
                KBM_ERR_INVALID_ARG, "kbm_extract_workspace_size: bad arguments");
    const uint64_t n = (uint64_t)Hr * Wr * k;
    *bytes = align_up(ex_layout(n, num_vel).end, 256);
    return KBM_OK;
}

namespace kbm {
namespace {

// Validation shared by both entry points; returns the slot count in *n.
kbm_status check_extract(const char *who, const kbm_results *r, int32_t Hr, int32_t Wr,
                         int32_t k, const float *vel, int32_t num_vel, float lh_min,
                         int64_t n_max, const float *params, const float *lh,
                         const float *flux, const uint64_t *keep, const int16_t *n_obs,
                         const int64_t *n_out, uint64_t *n) {
    KBM_REQUIRE(r != nullptr && r->lh && r->vel_idx, KBM_ERR_INVALID_ARG,
                "%s: results (lh, vel_idx) must be non-NULL", who);
    KBM_REQUIRE(Hr >= 0 && Wr >= 0 && k >= 1 && k <= KBM_MAX_K, KBM_ERR_INVALID_ARG,
                "%s: bad result shape %d x %d x %d", who, Hr, Wr, k);
    KBM_REQUIRE(vel != nullptr && num_vel >= 1, KBM_ERR_INVALID_ARG,
                "%s: velocity list is empty", who);
    KBM_REQUIRE(n_max >= 0 && params && lh && n_out, KBM_ERR_INVALID_ARG,
                "%s: params, lh and n_out must be non-NULL, n_max >= 0", who);
    KBM_REQUIRE(!std::isnan(lh_min), KBM_ERR_INVALID_ARG, "%s: lh_min is NaN", who);
    *n = (uint64_t)Hr * Wr * k;
    KBM_REQUIRE(*n < ((uint64_t)1 << 32), KBM_ERR_UNSUPPORTED,
                "%s: more than 2^32 result slots", who);
    KBM_REQUIRE(!flux || r->flux, KBM_ERR_INVALID_ARG, "%s: results lack flux", who);
    KBM_REQUIRE(!keep || r->keep, KBM_ERR_INVALID_ARG, "%s: results lack keep", who);
    KBM_REQUIRE(!n_obs || r->n_obs, KBM_ERR_INVALID_ARG, "%s: results lack n_obs", who);
    return KBM_OK;
}

// Radix select, block counts, scan and ordered write; `st` and `cnt` are
// scratch (every word the kernels read is written first by an earlier
// kernel of the sequence), `dvel` the device velocity list.
kbm_status enqueue_extract(const kbm_results *r, uint64_t n, const ExLayout &l,
                           ExtractState *st, unsigned int *cnt, const float *dvel,
                           int32_t Wr, int32_t k, int32_t x_begin, int32_t y_begin,
                           float lh_min, int64_t n_max, float *params, float *lh,
                           float *flux, uint64_t *keep, int64_t *index, int16_t *n_obs,
                           int64_t *n_out, hipStream_t stream) {
    hipLaunchKernelGGL(ex_init_kernel, dim3(1), dim3(256), 0, stream, st, (uint64_t)n_max);
    for (int pass = 0; pass < 8; ++pass) {
        hipLaunchKernelGGL(ex_hist_kernel, dim3(l.nb), dim3(EX_THREADS), 0, stream,
                           r->lh, n, lh_min, pass, st);
        hipLaunchKernelGGL(ex_pick_kernel, dim3(1), dim3(256), 0, stream, st, pass);
    }
    hipLaunchKernelGGL(ex_count_kernel, dim3(l.nb), dim3(EX_THREADS), 0, stream, r->lh,
                       n, lh_min, l.per_block, st, cnt);
    hipLaunchKernelGGL(ex_scan_kernel, dim3(1), dim3(256), 0, stream, cnt, l.nb, n_out);
    ExtractOut o{};
    o.lh = r->lh;
    o.flux = r->flux;
    o.vidx = r->vel_idx;
    o.nobs = r->n_obs;
    o.keep = r->keep;
    o.vel = dvel;
    o.params = params;
    o.out_lh = lh;
    o.out_flux = flux;
    o.out_keep = keep;
    o.out_index = index;
    o.out_nobs = n_obs;
    o.Wr = Wr;
    o.K = k;
    o.x0 = x_begin;
    o.y0 = y_begin;
    hipLaunchKernelGGL(ex_write_kernel, dim3(l.nb), dim3(EX_THREADS), 0, stream, o, n,
                       lh_min, l.per_block, st, cnt);
    KBM_LAUNCHED("ex_write_kernel");
    return KBM_OK;
}

// Scratch of kbm_extract_top_noalloc: the select state and the per-block
// counts (at most EX_BLOCKS_MAX blocks whatever the slot count).  Each GPU
// holds its own copy until the process ends.
constexpr size_t EX_SCRATCH_BYTES = KBM_EXTRACT_SCRATCH_BYTES;
static_assert(EX_SCRATCH_BYTES >= (sizeof(ExtractState) + 255) / 256 * 256 +
                                      sizeof(unsigned int) * EX_BLOCKS_MAX,
              "scratch of kbm_extract_top_noalloc too small for EX_BLOCKS_MAX blocks");

}  // namespace

static __device__ __align__(256) unsigned char scratch[EX_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mutex;
std::map<int, char *> g_scratch;  // device -> device address of `scratch`

// Device address of this device's scratch, looked up once per device with
// that device current.
kbm_status scratch_address(char **out) {
    int dev = 0;
    KBM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void *p = nullptr;
        KBM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        KBM_REQUIRE(p != nullptr, KBM_ERR_DEVICE,
                    "kbm_extract_top_noalloc: no device address for the scratch array");
        it = g_scratch.emplace(dev, static_cast<char *>(p)).first;
    }
    *out = it->second;
    return KBM_OK;
}

}  // namespace
}  // namespace kbm

extern "C" kbm_status kbm_extract_top(const kbm_results *r, int32_t Hr, int32_t Wr,
                                      int32_t k, int32_t x_begin, int32_t y_begin,
                                      const float *vel, int32_t num_vel, float lh_min,
                                      int64_t n_max, float *params, float *lh,
                                      float *flux, uint64_t *keep, int64_t *index,
                                      int16_t *n_obs, int64_t *n_out,
                                      void *workspace, size_t workspace_bytes,
                                      hipStream_t stream) {
    using namespace kbm;
    clear_error();
    uint64_t n = 0;
    kbm_status s = check_extract("kbm_extract_top", r, Hr, Wr, k, vel, num_vel, lh_min,
                                 n_max, params, lh, flux, keep, n_obs, n_out, &n);
    if (s != KBM_OK) return s;
    const ExLayout l = ex_layout(n, num_vel);
    KBM_REQUIRE(workspace != nullptr && workspace_bytes >= l.end, KBM_ERR_WORKSPACE,
                "kbm_extract_top: workspace of %zu bytes given, %zu needed",
                workspace_bytes, l.end);
    char *ws = static_cast<char *>(workspace);
    ExtractState *st = reinterpret_cast<ExtractState *>(ws + l.st_off);
    unsigned int *cnt = reinterpret_cast<unsigned int *>(ws + l.cnt_off);
    float *dvel = reinterpret_cast<float *>(ws + l.vel_off);
    s = stage_to_device(dvel, vel, sizeof(float) * 2 * (size_t)num_vel, stream);
    if (s != KBM_OK) return s;
    return enqueue_extract(r, n, l, st, cnt, dvel, Wr, k, x_begin, y_begin, lh_min, n_max,
                           params, lh, flux, keep, index, n_obs, n_out, stream);
}

extern "C" kbm_status kbm_extract_top_noalloc(const kbm_results *r, int32_t Hr, int32_t Wr,
                                              int32_t k, int32_t x_begin, int32_t y_begin,
                                              const float *vel_dev, int32_t num_vel,
                                              float lh_min, int64_t n_max, float *params,
                                              float *lh, float *flux, uint64_t *keep,
                                              int64_t *index, int16_t *n_obs,
                                              int64_t *n_out, hipStream_t stream) {
    using namespace kbm;
    clear_error();
    uint64_t n = 0;
    kbm_status s = check_extract("kbm_extract_top_noalloc", r, Hr, Wr, k, vel_dev, num_vel,
                                 lh_min, n_max, params, lh, flux, keep, n_obs, n_out, &n);
    if (s != KBM_OK) return s;
    const ExLayout l = ex_layout(n, num_vel);
    KBM_REQUIRE(l.vel_off <= EX_SCRATCH_BYTES, KBM_ERR_UNSUPPORTED,
                "kbm_extract_top_noalloc: %zu bytes of scratch needed, %zu available",
                l.vel_off, EX_SCRATCH_BYTES);
    char *ws = nullptr;
    s = scratch_address(&ws);
    if (s != KBM_OK) return s;
    ExtractState *st = reinterpret_cast<ExtractState *>(ws + l.st_off);
    unsigned int *cnt = reinterpret_cast<unsigned int *>(ws + l.cnt_off);
    return enqueue_extract(r, n, l, st, cnt, vel_dev, Wr, k, x_begin, y_begin, lh_min,
                           n_max, params, lh, flux, keep, index, n_obs, n_out, stream);
}

// Batched persistent search: kbm_search's result for many stacks from one
// persistent kernel launch, captured once into a HIP graph and replayed.
//
// Schedule
//  * A work item is (stack s, tile t, velocity block b): the 64 start pixels
//    of tile t against velocities [b B, min(V, (b+1) B)).  Tiles are
//    enumerated in super-tile order (tile_cols x tile_rows tiles, column
//    strips of super-tiles), as in the per-stack search.
//  * Eight queues, one per XCD.  Queue q holds, for every stack, the q-th
//    eighth of its tiles (a contiguous strip), so each XCD's L2 serves one
//    strip of each stack.  Within a queue, items are ordered by velocity
//    block, then by stack in decreasing cost per item (T, longest first),
//    then by tile: in flight, all workgroups of an XCD sweep the same block
//    of velocities over neighbouring tiles, and the cheapest items come
//    last.  A queue is a list of segments (block, stack) with prefix sums.
//  * Workgroup g serves queue g mod 8 (workgroups are dispatched to XCDs
//    round-robin), then the other queues in turn; an atomic counter per
//    queue hands out items.  Every workgroup exits after one pass over the
//    eight queues.
//  * A tile's running top-K lists pass from block b to b+1 through the
//    workspace.  The item of block b publishes them with a release store of
//    b+1 to the tile's progress counter; the item of block b+1 waits (acquire
//    loads, bounded) until it reads b+1.  The producer item was dequeued
//    earlier from the same queue, so it is held by a running workgroup that
//    can only be waiting on an even earlier item: the wait always ends.
//  * The item of a tile's last block re-evaluates the K winners and writes
//    the results.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <iomanip>
#include <map>
#include <sstream>

#include <sys/stat.h>
#include <unistd.h>
#include <mutex>
#include <string>
#include <vector>

#include "batch_kernels.h"
#include "search_host.h"

namespace kbm {
namespace batch {

__global__ __launch_bounds__(256) void zero_words_kernel(uint32_t *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256)
        p[i] = 0u;
}

// Pack every stack's planes (stack = blockIdx.y); flags unusable samples.
__global__ __launch_bounds__(256) void batch_prep_kernel(const PrepDesc *__restrict__ d) {
    const PrepDesc &p = d[blockIdx.y];
    bool bad = false;
    for (uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x; j < p.n;
         j += (uint64_t)gridDim.x * 256)
        p.pk[j] = srch::pack_sample(p.psi[j], p.phi[j], bad);
    if (__any(bad) && (threadIdx.x % WAVE) == 0) atomicOr(p.flag, 1);
}

struct Sched {
    int vb, st_x, st_y, nw, bpc, sw;
};

bool pow2_in(int x, int hi) { return x >= 1 && x <= hi && (x & (x - 1)) == 0; }

// Built-in schedule: 1024 velocities per item, 4 wavefronts per workgroup
// sharing a tile, 128 px x 32 row super-tiles, as many workgroups as fit;
// the waves take contiguous shares of the item's velocities when some stack
// has at least 16384 velocities, else every fourth velocity.  Measured when
// this default was chosen (before the 3-sorter networks): the DECam-CCD stack (2048 x 4096, T = 26, 128^2 velocities) takes 1183 ms this
// way (interleaved: 1236 ms at its best block, 2048); 62 stacks of 64^2
// velocities take 10.54 s (contiguous: 10.76 s at its best block, 512).
Sched default_sched(int vmax) { return Sched{1024, 2, 32, 4, 0, vmax >= 16384 ? 1 : 0}; }

// Trajectory-epochs that one run of a stack evaluates.  The sweep evaluates
// a (tile, velocity) pair when every epoch of every lane of the tile's
// 64-pixel row segment stays inside the image (F, the offset bounding box)
// or when, per axis, min_obs epochs keep some lane inside (M, the min_obs
// box), and skips it otherwise.  Both tests only depend on the geometry,
// and each is a column condition and a row condition, so per velocity
//   pairs(F or M) = pairs(F) + pairs(M) - pairs(F and M),
// each term a lane count over the tile columns times a row count.  Padding
// lanes of the last column tile are not counted.
uint64_t evaluated_traj_epochs(const srch::SearchArgs &a, const int4 *box, const int4 *mbox) {
    const int64_t y_lo = a.y0, y_hi = (int64_t)a.y0 + a.Hr - 1, H1 = (int64_t)a.H - 1;
    auto rows = [&](int64_t lo, int64_t hi) -> int64_t {
        lo = std::max(lo, y_lo);
        hi = std::min(hi, y_hi);
        return hi >= lo ? hi - lo + 1 : 0;
    };
    uint64_t pairs = 0;  // lane-weighted (pixel, velocity) pairs
    for (int v = 0; v < a.V; ++v) {
        const int4 bx = box[2 * v], mb = mbox[v];
        int64_t lf = 0, lm = 0, lfm = 0;
        for (int tx = 0; tx < a.tiles_x; ++tx) {
            const int64_t xw = (int64_t)a.x0 + (int64_t)tx * WAVE;
            const int64_t lanes = std::min<int64_t>(WAVE, (int64_t)a.Wr - (int64_t)tx * WAVE);
            const bool fx = xw + bx.x >= 0 && xw + (WAVE - 1) + bx.y < a.W;
            const bool mx = xw + mb.x <= a.W - 1 && xw + (WAVE - 1) + mb.y >= 0;
            lf += fx ? lanes : 0;
            lm += mx ? lanes : 0;
            lfm += (fx && mx) ? lanes : 0;
        }
        const int64_t f_lo = -(int64_t)bx.z, f_hi = H1 - bx.w;  // y + bx.z >= 0, y + bx.w < H
        const int64_t m_lo = -(int64_t)mb.w, m_hi = H1 - mb.z;  // y + mb.w >= 0, y + mb.z < H
        pairs += (uint64_t)(lf * rows(f_lo, f_hi) + lm * rows(m_lo, m_hi) -
                            lfm * rows(std::max(f_lo, m_lo), std::min(f_hi, m_hi)));
    }
    return pairs * (uint64_t)a.T;
}

}  // namespace batch
}  // namespace kbm

struct kbm_batch {
    int device = 0;
    int S = 0;
    int n_cu = 0;
    std::vector<int> T, V, Wr, Hr, tiles_x;
    std::vector<size_t> n_elem;
    char *ws = nullptr;
    kbm::srch::SearchArgs *descs = nullptr;
    kbm::batch::PrepDesc *prep = nullptr;
    kbm::batch::StackInfo *info = nullptr;
    int2 *seg = nullptr;
    uint32_t *pre = nullptr;
    uint32_t *ctrl = nullptr;  // queue heads, stall flag, flags[S], progress
    uint32_t *prog = nullptr;
    size_t max_seg = 0, max_prog = 0, ctrl_words = 0, flags_words = 0;
    int prep_blocks = 1;
    int nseg = 0;
    kbm::batch::Sched sched{};
    float probe_ms = 0.0f;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t *host_word = nullptr;  // pinned
    uint64_t evaluated = 0;  // trajectory-epochs one run evaluates
};

namespace kbm {
namespace batch {
namespace {

struct BatchLayout {
    size_t stacks_end, descs_off, prep_off, info_off, seg_off, pre_off, ctrl_off, end;
    size_t max_seg, max_prog, flags_words, ctrl_words;
};

BatchLayout batch_layout(const kbm_stack *stacks, const kbm_search_params *p, int S) {
    BatchLayout l{};
    size_t cur = 0;
    for (int j = 0; j < S; ++j) cur = srch::layout(stacks[j], p[j], cur).end;
    l.stacks_end = cur;
    for (int j = 0; j < S; ++j) {
        const size_t Wr = p[j].x_end - p[j].x_begin, Hr = p[j].y_end - p[j].y_begin;
        l.max_seg += (p[j].num_vel + MIN_VB - 1) / MIN_VB;
        const size_t tx = (Wr + WAVE - 1) / WAVE;
        l.max_prog += align_up(tx, PAD_COLS) * align_up(Hr, PAD_ROWS);
    }
    l.flags_words = align_up(S, 64);
    l.ctrl_words = CTRL_HEAD + l.flags_words + l.max_prog;
    l.descs_off = align_up(cur, 256);
    l.prep_off = align_up(l.descs_off + sizeof(SearchArgs) * S, 256);
    l.info_off = align_up(l.prep_off + sizeof(PrepDesc) * S, 256);
    l.seg_off = align_up(l.info_off + sizeof(StackInfo) * S, 256);
    l.pre_off = align_up(l.seg_off + sizeof(int2) * l.max_seg, 256);
    l.ctrl_off = align_up(l.pre_off + sizeof(uint32_t) * NUM_XCD * (l.max_seg + 1), 256);
    l.end = align_up(l.ctrl_off + sizeof(uint32_t) * l.ctrl_words, 256);
    return l;
}

kbm_status check_batch(const kbm_stack *stacks, const kbm_search_params *p, int S) {
    kbm_status st = srch::check_search(stacks, p, S);
    if (st != KBM_OK) return st;
    for (int j = 0; j < S; ++j) {
        KBM_REQUIRE(stacks[j].num_epochs <= MAX_T, KBM_ERR_UNSUPPORTED,
                    "kbm_batch: stack %d has T = %d > %d epochs (use kbm_search)", j,
                    stacks[j].num_epochs, MAX_T);
        KBM_REQUIRE(p[j].k <= BKM, KBM_ERR_UNSUPPORTED,
                    "kbm_batch: stack %d asks k = %d > %d (use kbm_search)", j, p[j].k, BKM);
        const uint64_t pk = (uint64_t)8 * stacks[j].num_epochs * stacks[j].width *
                            stacks[j].height;
        KBM_REQUIRE(pk <= 0xffffffffull, KBM_ERR_UNSUPPORTED,
                    "kbm_batch: stack %d needs %llu bytes of packed planes (>= 2^32; "
                    "use kbm_search)", j, (unsigned long long)pk);
    }
    return KBM_OK;
}

kbm_status check_sched(const Sched &s) {
    KBM_REQUIRE(s.vb >= MIN_VB, KBM_ERR_INVALID_ARG,
                "kbm_batch: vel_block = %d must be >= %d", s.vb, MIN_VB);
    KBM_REQUIRE(pow2_in(s.st_x, PAD_COLS) && pow2_in(s.st_y, PAD_ROWS), KBM_ERR_INVALID_ARG,
                "kbm_batch: super-tile %d x %d: cols must be a power of two <= %d, "
                "rows a power of two <= %d", s.st_x, s.st_y, PAD_COLS, PAD_ROWS);
    KBM_REQUIRE(s.nw == 1 || s.nw == 4, KBM_ERR_INVALID_ARG,
                "kbm_batch: waves = %d must be 1 or 4", s.nw);
    KBM_REQUIRE(s.bpc >= 0 && s.bpc <= 64, KBM_ERR_INVALID_ARG,
                "kbm_batch: blocks_per_cu = %d not in [0, 64]", s.bpc);
    KBM_REQUIRE(s.sw == 0 || s.sw == 1, KBM_ERR_INVALID_ARG,
                "kbm_batch: sweep = %d must be 0 or 1", s.sw);
    return KBM_OK;
}

// Queue segments and prefix sums for schedule `sc`; with div > 1 each
// queue keeps only ceil(len / div) consecutive tiles of its share of every
// stack, taken from the middle of the share (the autotuner's probe: the
// first tiles are the top rows of the image, where more tracks leave it
// than in the bulk of the stack).
kbm_status write_schedule(kbm_batch *b, const Sched &sc, int div, hipStream_t stream) {
    const int S = b->S;
    std::vector<StackInfo> info(S);
    uint32_t off = 0;
    for (int j = 0; j < S; ++j) {
        const uint32_t nsx = (b->tiles_x[j] + sc.st_x - 1) / sc.st_x;
        const uint32_t nsy = (b->Hr[j] + sc.st_y - 1) / sc.st_y;
        const uint64_t nt = (uint64_t)nsx * nsy * sc.st_x * sc.st_y;
        KBM_REQUIRE(nt < (1u << 28), KBM_ERR_UNSUPPORTED,
                    "kbm_batch: stack %d has too many tiles", j);
        // Every queue's share has floor(nt / 8) or one more tiles; the probe
        // keeps at most ceil(ceil(nt / 8) / div) of them from probe_off on,
        // which stays inside the smaller share.
        uint32_t probe_off = 0;
        if (div > 1) {
            const uint64_t lo = nt / NUM_XCD, hi = (nt + NUM_XCD - 1) / NUM_XCD;
            const uint64_t keep = (hi + div - 1) / div;
            probe_off = lo > keep ? (uint32_t)((lo - keep) / 2) : 0u;
        }
        info[j] = StackInfo{off, (uint32_t)nt, nsy, probe_off};
        off += (uint32_t)nt;
    }
    KBM_REQUIRE(off <= b->max_prog, KBM_ERR_INVALID_ARG,
                "kbm_batch: internal error, progress counters exceed the workspace");
    std::vector<int> order;
    int max_nvb = 0;
    for (int j = 0; j < S; ++j) {
        if (b->Wr[j] == 0 || b->Hr[j] == 0) continue;
        order.push_back(j);
        max_nvb = std::max(max_nvb, (b->V[j] + sc.vb - 1) / sc.vb);
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->T[x] > b->T[y]; });
    std::vector<int2> seg;
    for (int vb = 0; vb < max_nvb; ++vb)
        for (int j : order)
            if ((b->V[j] + sc.vb - 1) / sc.vb > vb) seg.push_back(make_int2(j, vb));
    KBM_REQUIRE(seg.size() <= b->max_seg, KBM_ERR_INVALID_ARG,
                "kbm_batch: internal error, segments exceed the workspace");
    const int nseg = (int)seg.size();
    std::vector<uint32_t> pre((size_t)NUM_XCD * (nseg + 1));
    for (int q = 0; q < NUM_XCD; ++q) {
        uint64_t acc = 0;
        pre[(size_t)q * (nseg + 1)] = 0;
        for (int k = 0; k < nseg; ++k) {
            const uint32_t nt = info[seg[k].x].n_tiles;
            const uint32_t r0 = nt * (uint32_t)q / NUM_XCD, r1 = nt * (uint32_t)(q + 1) / NUM_XCD;
            uint64_t len = r1 - r0;
            if (div > 1) len = (len + div - 1) / div;
            acc += len;
            KBM_REQUIRE(acc < (1ull << 31), KBM_ERR_UNSUPPORTED,
                        "kbm_batch: more than 2^31 work items in one queue");
            pre[(size_t)q * (nseg + 1) + k + 1] = (uint32_t)acc;
        }
    }
    kbm_status st = stage_to_device(b->info, info.data(), sizeof(StackInfo) * S, stream);
    if (st != KBM_OK) return st;
    if (nseg > 0) {
        st = stage_to_device(b->seg, seg.data(), sizeof(int2) * nseg, stream);
        if (st != KBM_OK) return st;
    }
    st = stage_to_device(b->pre, pre.data(), sizeof(uint32_t) * pre.size(), stream);
    if (st != KBM_OK) return st;
    KBM_HIP(hipStreamSynchronize(stream));
    b->nseg = nseg;
    return KBM_OK;
}

kbm_status blocks_per_cu(int nw, int sw, int *out) {
    int nb = 0;
    if (nw == 1)
        KBM_HIP(sw ? occupancy_nw1c(&nb) : occupancy_nw1(&nb));
    else
        KBM_HIP(sw ? occupancy_nw4c(&nb) : occupancy_nw4(&nb));
    *out = std::max(nb, 1);
    return KBM_OK;
}

// Schedule with blocks_per_cu = 0 replaced by the occupancy limit.
kbm_status resolve(Sched *sc) {
    if (sc->bpc != 0) return KBM_OK;
    return blocks_per_cu(sc->nw, sc->sw, &sc->bpc);
}

// Enqueue clear -> pack -> persistent search for schedule `sc` (already
// written to the workspace, blocks_per_cu resolved).  Only kernel launches:
// capturable.
kbm_status enqueue_run(kbm_batch *b, const Sched &sc, hipStream_t stream,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    const uint64_t nz = b->ctrl_words;
    const int zb = (int)std::min<uint64_t>((nz + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_words_kernel, dim3(zb), dim3(256), 0, stream, b->ctrl, nz);
    KBM_LAUNCHED("zero_words_kernel");
    hipLaunchKernelGGL(batch_prep_kernel, dim3(b->prep_blocks, b->S), dim3(256), 0, stream,
                       b->prep);
    KBM_LAUNCHED("batch_prep_kernel");
    const unsigned grid = (unsigned)(sc.bpc * b->n_cu);
    const BatchLaunch l{b->descs, b->info, b->pre, b->seg, b->ctrl,
                        b->prog, b->nseg, sc.vb, sc.st_x, sc.st_y};
    if (ev0) KBM_HIP(hipEventRecord(ev0, stream));
    const hipError_t e = sc.nw == 1 ? (sc.sw ? launch_batch_nw1c(l, grid, stream)
                                             : launch_batch_nw1(l, grid, stream))
                                    : (sc.sw ? launch_batch_nw4c(l, grid, stream)
                                             : launch_batch_nw4(l, grid, stream));
    if (e != hipSuccess) {
        set_error("launch of batch_kernel failed: %s", hipGetErrorString(e));
        return KBM_ERR_DEVICE;
    }
    if (ev1) KBM_HIP(hipEventRecord(ev1, stream));
    return KBM_OK;
}

// Time the persistent kernel of schedule `sc` on a probe of every stack.
kbm_status probe(kbm_batch *b, Sched sc, int div, hipStream_t stream,
                 hipEvent_t e0, hipEvent_t e1, float *ms) {
    kbm_status st = resolve(&sc);
    if (st != KBM_OK) return st;
    st = write_schedule(b, sc, div, stream);
    if (st != KBM_OK) return st;
    st = enqueue_run(b, sc, stream, e0, e1);
    if (st != KBM_OK) return st;
    KBM_HIP(hipEventSynchronize(e1));
    KBM_HIP(hipEventElapsedTime(ms, e0, e1));
    return KBM_OK;
}

bool same_sched(const Sched &x, const Sched &y) {
    return x.vb == y.vb && x.st_x == y.st_x && x.st_y == y.st_y && x.nw == y.nw &&
           x.bpc == y.bpc && x.sw == y.sw;
}

std::mutex g_tune_mutex;
std::map<std::string, std::pair<Sched, float>> g_tuned;

// Persisted choices of the autotuner: a JSON object mapping a key (library
// build id, device architecture, batch shape) to [vel_block, tile_cols,
// tile_rows, waves, blocks_per_cu, sweep, probe_ms], one entry per line.
// The file is KBM_TUNE_CACHE if set (empty: no file), else
// $HOME/.cache/kbm/autotune.json.  It is read and rewritten under the tune
// mutex; a missing, unreadable or malformed file only costs a new tuning.
std::string tune_cache_path() {
    const char *e = std::getenv("KBM_TUNE_CACHE");
    if (e) return std::string(e);
    const char *h = std::getenv("HOME");
    if (!h || !*h) return std::string();
    return std::string(h) + "/.cache/kbm/autotune.json";
}

std::map<std::string, std::pair<Sched, float>> read_tune_cache(const std::string &path) {
    std::map<std::string, std::pair<Sched, float>> m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t q0 = line.find('"'), q1 = line.find('"', q0 + 1);
        const size_t b0 = line.find('[', q1 == std::string::npos ? 0 : q1);
        const size_t b1 = line.find(']', b0 == std::string::npos ? 0 : b0);
        if (q0 == std::string::npos || q1 == std::string::npos || b0 == std::string::npos ||
            b1 == std::string::npos)
            continue;
        std::string nums = line.substr(b0 + 1, b1 - b0 - 1);
        std::replace(nums.begin(), nums.end(), ',', ' ');
        std::istringstream is(nums);
        Sched sc{};
        float ms = 0.0f;
        if (!(is >> sc.vb >> sc.st_x >> sc.st_y >> sc.nw >> sc.bpc >> sc.sw >> ms)) continue;
        if (check_sched(sc) != KBM_OK) continue;
        m[line.substr(q0 + 1, q1 - q0 - 1)] = std::make_pair(sc, ms);
    }
    clear_error();  // a rejected entry is not the caller's error
    return m;
}

void write_tune_cache(const std::string &path,
                      const std::map<std::string, std::pair<Sched, float>> &m) {
    for (size_t i = 1; i < path.size(); ++i)  // the directories above the file
        if (path[i] == '/') (void)::mkdir(path.substr(0, i).c_str(), 0755);
    const std::string tmp = path + ".tmp" + std::to_string((long long)::getpid());
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << std::setprecision(9) << "{\n";
        size_t i = 0;
        for (const auto &kv : m) {
            const Sched &c = kv.second.first;
            f << "\"" << kv.first << "\": [" << c.vb << ", " << c.st_x << ", " << c.st_y
              << ", " << c.nw << ", " << c.bpc << ", " << c.sw << ", " << kv.second.second
              << "]" << (++i < m.size() ? "," : "") << "\n";
        }
        f << "}\n";
        if (!f) return;
    }
    (void)std::rename(tmp.c_str(), path.c_str());
}

std::string shape_key(const kbm_batch *b, const kbm_search_params *p) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) arch = prop.gcnArchName;
    for (char &c : arch)
        if (c == '"' || c == '\\') c = '_';
    std::string k = std::string(kbm_build_id()) + "|" + arch;
    for (int j = 0; j < b->S; ++j) {
        k += "|" + std::to_string(b->Wr[j]) + "x" + std::to_string(b->Hr[j]) + "T" +
             std::to_string(b->T[j]) + "V" + std::to_string(b->V[j]) + "k" +
             std::to_string(p[j].k) + "s" + std::to_string(p[j].sigmag);
    }
    return k;
}

// Coordinate descent over sweep order, velocity block, super-tile shape,
// waves per workgroup and workgroups per CU, each candidate timed once on a probe of
// 1/16 of every stack's tiles (after one warm-up run).
kbm_status autotune(kbm_batch *b, const kbm_search_params *p, hipStream_t stream,
                    Sched *best, float *best_ms) {
    const std::string key = shape_key(b, p);
    const std::string cache = tune_cache_path();
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tuned.find(key);
        if (it == g_tuned.end() && !cache.empty()) {
            auto disk = read_tune_cache(cache);
            auto d = disk.find(key);
            if (d != disk.end()) it = g_tuned.insert(*d).first;
        }
        if (it != g_tuned.end()) {
            *best = it->second.first;
            *best_ms = it->second.second;
            return KBM_OK;
        }
    }
    const int div = 16;
    int vmax = 0;
    for (int j = 0; j < b->S; ++j) vmax = std::max(vmax, b->V[j]);
    hipEvent_t e0, e1;
    KBM_HIP(hipEventCreate(&e0));
    KBM_HIP(hipEventCreate(&e1));
    kbm_status st = KBM_OK;
    Sched cur = default_sched(vmax);
    float cur_ms = 0.0f, ms = 0.0f;
    auto run = [&](const Sched &c, float *t) -> kbm_status {
        return probe(b, c, div, stream, e0, e1, t);
    };
    const Sched def = cur;
    float def_ms = 0.0f;
    do {
        if ((st = run(cur, &ms)) != KBM_OK) break;  // warm-up
        if ((st = run(cur, &cur_ms)) != KBM_OK) break;
        def_ms = cur_ms;
        auto consider = [&](const Sched &c) -> kbm_status {
            float t = 0.0f;
            kbm_status s2 = run(c, &t);
            if (s2 == KBM_OK && t < cur_ms) {
                cur = c;
                cur_ms = t;
            }
            return s2;
        };
        {
            Sched c = cur;
            c.sw = 1 - cur.sw;
            if ((st = consider(c)) != KBM_OK) break;
        }
        const int vbs[] = {512, 1024, 2048, 4096};
        for (int v : vbs) {
            if (v == cur.vb) continue;
            if (v / 2 >= vmax) continue;  // same single block as a smaller one
            Sched c = cur;
            c.vb = v;
            if ((st = consider(c)) != KBM_OK) break;
        }
        if (st != KBM_OK) break;
        const int shapes[][2] = {{4, 16}, {1, 64}, {8, 8}};
        for (auto &sh : shapes) {
            Sched c = cur;
            c.st_x = sh[0];
            c.st_y = sh[1];
            if ((st = consider(c)) != KBM_OK) break;
        }
        if (st != KBM_OK) break;
        {
            Sched c = cur;
            c.nw = cur.nw == 4 ? 1 : 4;
            if ((st = consider(c)) != KBM_OK) break;
        }
        int full = 1;
        if ((st = blocks_per_cu(cur.nw, cur.sw, &full)) != KBM_OK) break;
        for (int num : {3, 2}) {
            Sched c = cur;
            c.bpc = std::max(1, full * num / 4);
            if (c.bpc >= full) continue;
            if ((st = consider(c)) != KBM_OK) break;
        }
        if (st != KBM_OK) break;
        // The probe ranks schedules on a fraction of the work; its winner
        // replaces the built-in schedule only if a full run confirms it.
        if (!same_sched(cur, def)) {
            float full_def = 0.0f, full_cur = 0.0f;
            if ((st = probe(b, def, 1, stream, e0, e1, &full_def)) != KBM_OK) break;
            if ((st = probe(b, cur, 1, stream, e0, e1, &full_cur)) != KBM_OK) break;
            if (!(full_cur < full_def)) {
                cur = def;
                cur_ms = def_ms;
            }
        }
    } while (false);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != KBM_OK) return st;
    *best = cur;
    *best_ms = cur_ms;
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    g_tuned[key] = std::make_pair(cur, cur_ms);
    if (!cache.empty()) {
        auto disk = read_tune_cache(cache);
        disk[key] = std::make_pair(cur, cur_ms);
        write_tune_cache(cache, disk);
    }
    return KBM_OK;
}

void release(kbm_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->host_word) (void)hipHostFree(b->host_word);
    delete b;
}

}  // namespace
}  // namespace batch
}  // namespace kbm

extern "C" kbm_status kbm_batch_workspace_size(const kbm_stack *stacks,
                                               const kbm_search_params *p,
                                               int32_t num_stacks, size_t *bytes) {
    using namespace kbm;
    clear_error();
    KBM_REQUIRE(bytes != nullptr, KBM_ERR_INVALID_ARG,
                "kbm_batch_workspace_size: bytes is NULL");
    kbm_status st = batch::check_batch(stacks, p, num_stacks);
    if (st != KBM_OK) return st;
    *bytes = batch::batch_layout(stacks, p, num_stacks).end;
    return KBM_OK;
}

extern "C" kbm_status kbm_batch_create(const kbm_stack *stacks, const float *const *psi,
                                       const float *const *phi, const kbm_search_params *p,
                                       kbm_results *out, int32_t num_stacks, void *workspace,
                                       size_t workspace_bytes, int32_t tune,
                                       kbm_schedule *schedule, hipStream_t stream,
                                       kbm_batch **batch_out) {
    using namespace kbm;
    using namespace kbm::batch;
    clear_error();
    KBM_REQUIRE(batch_out != nullptr, KBM_ERR_INVALID_ARG, "kbm_batch_create: batch is NULL");
    *batch_out = nullptr;
    kbm_status st = check_batch(stacks, p, num_stacks);
    if (st != KBM_OK) return st;
    KBM_REQUIRE(tune == KBM_TUNE_DEFAULT || tune == KBM_TUNE_AUTO || tune == KBM_TUNE_GIVEN,
                KBM_ERR_INVALID_ARG, "kbm_batch_create: tune = %d is not a KBM_TUNE_ mode",
                tune);
    int vmax = 0;
    for (int j = 0; j < num_stacks; ++j) vmax = std::max(vmax, (int)p[j].num_vel);
    Sched given = default_sched(vmax);
    if (tune == KBM_TUNE_GIVEN) {
        KBM_REQUIRE(schedule != nullptr, KBM_ERR_INVALID_ARG,
                    "kbm_batch_create: KBM_TUNE_GIVEN needs a schedule");
        given = Sched{schedule->vel_block, schedule->tile_cols, schedule->tile_rows,
                      schedule->waves, schedule->blocks_per_cu, schedule->sweep};
        st = check_sched(given);
        if (st != KBM_OK) return st;
    }
    KBM_REQUIRE(psi != nullptr && phi != nullptr && out != nullptr, KBM_ERR_INVALID_ARG,
                "kbm_batch_create: psi, phi, out must be non-NULL");
    const int S = num_stacks;
    for (int j = 0; j < S; ++j) {
        KBM_REQUIRE(psi[j] != nullptr && phi[j] != nullptr, KBM_ERR_INVALID_ARG,
                    "kbm_batch_create: planes of stack %d are NULL", j);
        const bool empty = p[j].x_end == p[j].x_begin || p[j].y_end == p[j].y_begin;
        KBM_REQUIRE(empty || (out[j].lh && out[j].flux && out[j].vel_idx && out[j].n_obs &&
                              out[j].keep),
                    KBM_ERR_INVALID_ARG, "kbm_batch_create: result arrays of stack %d are NULL",
                    j);
    }
    const BatchLayout L = batch_layout(stacks, p, S);
    KBM_REQUIRE(workspace != nullptr && workspace_bytes >= L.end, KBM_ERR_WORKSPACE,
                "kbm_batch_create: workspace of %zu bytes given, %zu needed", workspace_bytes,
                L.end);

    kbm_batch *b = new kbm_batch();
    auto fail = [&](kbm_status s) {
        release(b);
        return s;
    };
    char *ws = static_cast<char *>(workspace);
    b->S = S;
    b->ws = ws;
    if (hipGetDevice(&b->device) != hipSuccess ||
        hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, b->device) !=
            hipSuccess) {
        set_error("kbm_batch_create: cannot query the current device");
        return fail(KBM_ERR_DEVICE);
    }
    b->descs = reinterpret_cast<srch::SearchArgs *>(ws + L.descs_off);
    b->prep = reinterpret_cast<PrepDesc *>(ws + L.prep_off);
    b->info = reinterpret_cast<StackInfo *>(ws + L.info_off);
    b->seg = reinterpret_cast<int2 *>(ws + L.seg_off);
    b->pre = reinterpret_cast<uint32_t *>(ws + L.pre_off);
    b->ctrl = reinterpret_cast<uint32_t *>(ws + L.ctrl_off);
    b->prog = b->ctrl + CTRL_HEAD + L.flags_words;
    b->max_seg = L.max_seg;
    b->max_prog = L.max_prog;
    b->flags_words = L.flags_words;
    b->ctrl_words = L.ctrl_words;

    std::vector<srch::SearchArgs> descs(S);
    std::vector<PrepDesc> prep(S);
    std::vector<char> tables;
    size_t cursor = 0, max_n = 1;
    for (int j = 0; j < S; ++j) {
        const kbm_stack &s = stacks[j];
        const kbm_search_params &q = p[j];
        const srch::StackLayout l = srch::layout(s, q, cursor);
        cursor = l.end;
        srch::make_tables(s, q, l, s.num_epochs, tables);
        st = stage_to_device(ws + l.tab_off, tables.data(), l.tab_bytes, stream);
        if (st != KBM_OK) return fail(st);
        const size_t n = (size_t)s.num_epochs * s.width * s.height;
        max_n = std::max(max_n, n);
        int *flag = reinterpret_cast<int *>(b->ctrl + CTRL_HEAD + j);
        float2 *pk = reinterpret_cast<float2 *>(ws + l.pk_off);
        prep[j] = PrepDesc{psi[j], phi[j], pk, flag, (uint64_t)n};
        srch::SearchArgs &a = descs[j];
        a = srch::SearchArgs{};
        a.pk = pk;
        a.pk_bytes = (uint32_t)l.pk_bytes;
        a.n_elem = (uint32_t)n;
        a.am = 1;  // one descriptor (checked: packed planes below 4 GB)
        a.split = s.num_epochs;
        a.pk2 = pk;
        a.pk2_bytes = 0;
        a.n_elem2 = 0;
        a.off16 = reinterpret_cast<const int *>(ws + l.tab_off + l.off_rel);
        a.lin = reinterpret_cast<const uint32_t *>(ws + l.tab_off + l.lin_rel);
        a.vbox = reinterpret_cast<const int4 *>(ws + l.tab_off + l.box_rel);
        a.mbox = reinterpret_cast<const int4 *>(ws + l.tab_off + l.mbox_rel);
        a.ranks = reinterpret_cast<const int *>(ws + l.tab_off + l.rank_rel);
        a.flags = flag;
        a.stL = reinterpret_cast<float *>(ws + l.stl_off);
        a.stI = reinterpret_cast<int *>(ws + l.sti_off);
        a.lh = out[j].lh;
        a.flux = out[j].flux;
        a.vidx = out[j].vel_idx;
        a.nobs = out[j].n_obs;
        a.keep = out[j].keep;
        a.lh_raw = out[j].lh_raw;
        a.W = s.width;
        a.H = s.height;
        a.T = s.num_epochs;
        a.V = q.num_vel;
        a.K = q.k;
        a.min_obs = q.min_obs;
        a.sigmag = q.sigmag;
        a.x0 = q.x_begin;
        a.y0 = q.y_begin;
        a.Wr = q.x_end - q.x_begin;
        a.Hr = q.y_end - q.y_begin;
        a.tiles_x = (a.Wr + WAVE - 1) / WAVE;
        a.coeff = (float)q.coeff;
        a.n_sigma = (float)q.n_sigma;
        a.defq = q.q_lo == 0.25 && q.q_hi == 0.75;
        b->evaluated += evaluated_traj_epochs(
            a, reinterpret_cast<const int4 *>(tables.data() + l.box_rel),
            reinterpret_cast<const int4 *>(tables.data() + l.mbox_rel));
        b->T.push_back(a.T);
        b->V.push_back(a.V);
        b->Wr.push_back(a.Wr);
        b->Hr.push_back(a.Hr);
        b->tiles_x.push_back(a.tiles_x);
        b->n_elem.push_back(n);
    }
    b->prep_blocks = (int)std::min<size_t>(std::max<size_t>((max_n + 4095) / 4096, 1), 2048);
    st = stage_to_device(b->descs, descs.data(), sizeof(srch::SearchArgs) * S, stream);
    if (st != KBM_OK) return fail(st);
    st = stage_to_device(b->prep, prep.data(), sizeof(PrepDesc) * S, stream);
    if (st != KBM_OK) return fail(st);
    if (hipStreamSynchronize(stream) != hipSuccess) {
        set_error("kbm_batch_create: staging the tables failed");
        return fail(KBM_ERR_DEVICE);
    }

    Sched sc = given;
    if (tune == KBM_TUNE_AUTO) {
        st = autotune(b, p, stream, &sc, &b->probe_ms);
        if (st != KBM_OK) return fail(st);
    }
    st = resolve(&sc);
    if (st != KBM_OK) return fail(st);
    b->sched = sc;
    st = write_schedule(b, sc, 1, stream);
    if (st != KBM_OK) return fail(st);

    if (hipHostMalloc(&b->host_word, 64, hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        set_error("kbm_batch_create: cannot create the capture stream");
        return fail(KBM_ERR_DEVICE);
    }
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        set_error("kbm_batch_create: hipStreamBeginCapture failed");
        return fail(KBM_ERR_DEVICE);
    }
    st = enqueue_run(b, sc, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->cap, &g);
    b->graph = g;
    if (st != KBM_OK) return fail(st);
    if (ec != hipSuccess || g == nullptr) {
        set_error("kbm_batch_create: hipStreamEndCapture failed: %s", hipGetErrorString(ec));
        return fail(KBM_ERR_DEVICE);
    }
    const hipError_t ei = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        set_error("kbm_batch_create: hipGraphInstantiate failed: %s", hipGetErrorString(ei));
        return fail(KBM_ERR_DEVICE);
    }
    if (schedule) {
        schedule->vel_block = sc.vb;
        schedule->tile_cols = sc.st_x;
        schedule->tile_rows = sc.st_y;
        schedule->waves = sc.nw;
        schedule->blocks_per_cu = sc.bpc;
        schedule->sweep = sc.sw;
        schedule->probe_ms = b->probe_ms;
    }
    *batch_out = b;
    return KBM_OK;
}

extern "C" kbm_status kbm_batch_run(kbm_batch *b, hipStream_t stream) {
    using namespace kbm;
    clear_error();
    KBM_REQUIRE(b != nullptr && b->exec != nullptr, KBM_ERR_INVALID_ARG,
                "kbm_batch_run: batch is NULL");
    KBM_HIP(hipGraphLaunch(b->exec, stream));
    return KBM_OK;
}

extern "C" kbm_status kbm_batch_check(kbm_batch *b, hipStream_t stream, int32_t *stalled) {
    using namespace kbm;
    clear_error();
    KBM_REQUIRE(b != nullptr && stalled != nullptr, KBM_ERR_INVALID_ARG,
                "kbm_batch_check: batch and stalled must be non-NULL");
    KBM_HIP(hipMemcpyAsync(b->host_word, b->ctrl + srch::NUM_XCD, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, stream));
    KBM_HIP(hipStreamSynchronize(stream));
    *stalled = b->host_word[0] != 0u;
    return KBM_OK;
}

extern "C" kbm_status kbm_batch_evaluated(kbm_batch *b, hipStream_t stream,
                                          uint64_t *traj_epochs) {
    using namespace kbm;
    clear_error();
    (void)stream;
    KBM_REQUIRE(b != nullptr && traj_epochs != nullptr, KBM_ERR_INVALID_ARG,
                "kbm_batch_evaluated: batch and traj_epochs must be non-NULL");
    *traj_epochs = b->evaluated;
    return KBM_OK;
}

extern "C" kbm_status kbm_tune_cache_clear(void) {
    kbm::clear_error();
    std::lock_guard<std::mutex> lk(kbm::batch::g_tune_mutex);
    kbm::batch::g_tuned.clear();
    return KBM_OK;
}

extern "C" kbm_status kbm_batch_destroy(kbm_batch *b) {
    kbm::clear_error();
    kbm::batch::release(b);
    return KBM_OK;
}

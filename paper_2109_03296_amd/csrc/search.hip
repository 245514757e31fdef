// Host side of the trajectory search (Section 3, 3.1, 3.2): argument
// checks, offset tables, workspace layout, and the launch sequence
// (tables -> pack prep -> chunked search -> finalize).  Device code and the
// design notes are in search_kernels.h.
#include <algorithm>
#include <vector>

#include "search_host.h"
#include "search_kernels.h"

namespace kbm {
namespace srch {
namespace {

__global__ __launch_bounds__(64) void zero_flags_kernel(int *flags) {
    if (threadIdx.x == 0) flags[0] = 0;
}

__global__ __launch_bounds__(256) void pack_prep_kernel(
    const float *__restrict__ psi, const float *__restrict__ phi,
    float2 *__restrict__ pk, int *__restrict__ flags, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (size_t j = i; j < n; j += stride) pk[j] = pack_sample(psi[j], phi[j], bad);
    if (__any(bad) && (threadIdx.x % WAVE) == 0) atomicOr(flags, 1);
}

// Generic (padded) buckets for epoch counts without an exact variant.
template <int KM, int AM>
void launch_generic_s(const SearchArgs &a, hipStream_t stream) {
    if (a.T <= 8) launch_chunks<8, KM, false, AM>(a, stream);
    else if (a.T <= 16) launch_chunks<16, KM, false, AM>(a, stream);
    else if (a.T <= 24) launch_chunks<24, KM, false, AM>(a, stream);
    else if (a.T <= 32) launch_chunks<32, KM, false, AM>(a, stream);
    else if (a.T <= 48) launch_chunks<48, KM, false, AM>(a, stream);
    else launch_chunks<64, KM, false, AM>(a, stream);
}

template <int KM>
void launch_generic(const SearchArgs &a, hipStream_t stream) {
    if (a.am == 1)
        launch_generic_s<KM, 1>(a, stream);
    else if (a.am == 2)
        launch_generic_s<KM, 2>(a, stream);
    else
        launch_generic_s<KM, 0>(a, stream);
}

template <int TM>
void launch_finalize_t(const SearchArgs &a, hipStream_t stream) {
    const size_t npix = (size_t)a.Wr * a.Hr;
    const dim3 grid((unsigned)((npix + 255) / 256));
    if (a.am == 1)
        hipLaunchKernelGGL((finalize_kernel<TM, 1>), grid, dim3(256), 0, stream, a);
    else if (a.am == 2)
        hipLaunchKernelGGL((finalize_kernel<TM, 2>), grid, dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL((finalize_kernel<TM, 0>), grid, dim3(256), 0, stream, a);
}

void launch_finalize(const SearchArgs &a, hipStream_t stream) {
    if (a.T <= 8) launch_finalize_t<8>(a, stream);
    else if (a.T <= 16) launch_finalize_t<16>(a, stream);
    else if (a.T <= 24) launch_finalize_t<24>(a, stream);
    else if (a.T <= 32) launch_finalize_t<32>(a, stream);
    else if (a.T <= 48) launch_finalize_t<48>(a, stream);
    else launch_finalize_t<64>(a, stream);
}

}  // namespace

StackLayout layout(const kbm_stack &s, const kbm_search_params &p,
                   size_t start) {
    StackLayout l;
    const size_t T = s.num_epochs, V = p.num_vel;
    const size_t npix = (size_t)(p.x_end - p.x_begin) * (p.y_end - p.y_begin);
    l.pk_off = align_up(start, 256);
    l.pk_bytes = sizeof(float2) * T * s.width * s.height;
    l.tab_off = align_up(l.pk_off + l.pk_bytes, 256);
    l.off_rel = 0;
    l.lin_rel = align_up(l.off_rel + sizeof(int) * V * T, 16);
    l.box_rel = align_up(l.lin_rel + sizeof(uint32_t) * V * T, 32);
    l.mbox_rel = align_up(l.box_rel + 2 * sizeof(int4) * V, 16);
    l.rank_rel = align_up(l.mbox_rel + sizeof(int4) * V, 16);
    l.tab_bytes = l.rank_rel + sizeof(int) * 3 * 65;
    l.flags_off = align_up(l.tab_off + l.tab_bytes, 256);
    l.stl_off = align_up(l.flags_off + 256, 256);
    l.sti_off = align_up(l.stl_off + sizeof(float) * npix * p.k, 256);
    l.end = l.sti_off + sizeof(int) * npix * p.k;
    return l;
}

kbm_status check_search(const kbm_stack *stacks, const kbm_search_params *p,
                        int32_t num_stacks) {
    KBM_REQUIRE(num_stacks >= 1, KBM_ERR_INVALID_ARG,
                "kbm_search: num_stacks = %d must be >= 1", num_stacks);
    KBM_REQUIRE(stacks != nullptr && p != nullptr, KBM_ERR_INVALID_ARG,
                "kbm_search: stacks and params must be non-NULL");
    for (int j = 0; j < num_stacks; ++j) {
        kbm_status st = check_stack(&stacks[j], "kbm_search");
        if (st != KBM_OK) return st;
        const kbm_search_params &q = p[j];
        KBM_REQUIRE(q.vel != nullptr && q.num_vel >= 1, KBM_ERR_INVALID_ARG,
                    "kbm_search: stack %d needs a non-empty velocity list", j);
        KBM_REQUIRE(q.k >= 1 && q.k <= KBM_MAX_K, KBM_ERR_INVALID_ARG,
                    "kbm_search: k = %d not in [1, %d]", q.k, KBM_MAX_K);
        KBM_REQUIRE(q.min_obs >= 1, KBM_ERR_INVALID_ARG,
                    "kbm_search: min_obs = %d must be >= 1", q.min_obs);
        KBM_REQUIRE(q.sigmag == 0 || q.sigmag == 1, KBM_ERR_INVALID_ARG,
                    "kbm_search: sigmag must be 0 or 1");
        kbm_status sg = check_sigmag_params(q.q_lo, q.q_hi, q.coeff, q.n_sigma);
        if (sg != KBM_OK) return sg;
        const kbm_stack &s = stacks[j];
        KBM_REQUIRE(s.width <= 32767 && s.height <= 32767, KBM_ERR_UNSUPPORTED,
                    "kbm_search: image sides must be <= 32767 (got %d x %d)",
                    s.width, s.height);
        KBM_REQUIRE((uint64_t)s.num_epochs * s.width * s.height < ((uint64_t)1 << 32),
                    KBM_ERR_UNSUPPORTED,
                    "kbm_search: T*H*W must be below 2^32 pixel-epochs");
        KBM_REQUIRE(q.x_begin >= 0 && q.x_begin <= q.x_end &&
                        q.x_end <= s.width && q.y_begin >= 0 &&
                        q.y_begin <= q.y_end && q.y_end <= s.height,
                    KBM_ERR_INVALID_ARG,
                    "kbm_search: region [%d,%d)x[%d,%d) outside %dx%d image",
                    q.x_begin, q.x_end, q.y_begin, q.y_end, s.width, s.height);
        double t0 = s.times[0], t1 = s.times[0];
        for (int i = 1; i < s.num_epochs; ++i) {
            t0 = std::min(t0, s.times[i]);
            t1 = std::max(t1, s.times[i]);
        }
        for (int v = 0; v < q.num_vel; ++v) {
            const float vx = q.vel[2 * v], vy = q.vel[2 * v + 1];
            KBM_REQUIRE(std::isfinite(vx) && std::isfinite(vy),
                        KBM_ERR_INVALID_ARG,
                        "kbm_search: velocity %d is not finite", v);
            KBM_REQUIRE(std::fabs((double)vx) * (t1 - t0) < 1e9 &&
                            std::fabs((double)vy) * (t1 - t0) < 1e9,
                        KBM_ERR_INVALID_ARG,
                        "kbm_search: velocity %d moves more than 1e9 px", v);
        }
    }
    return KBM_OK;
}

// Tables of one stack, laid out as in the workspace table block:
//  * off16: (dx, dy) = floor(v t + 1/2) in FP64 with t from the earliest
//    epoch (this translation unit is compiled with -ffp-contract=off, so the
//    product is rounded before the addition), packed as 16-bit halves;
//    offsets beyond +/-32767 are clamped, which keeps them out of any image
//    (sides <= 32767);
//  * lin: i H W + dy W + dx modulo 2^32, the element offset of epoch i's
//    sample relative to the start pixel;
//  * vbox: each velocity's offset bounding box, then two masks of the
//    epochs below 32 whose offsets equal those of velocity v-1 and of v-4
//    (a wave that sweeps every first or fourth velocity keeps those samples);
//  * mbox: the min_obs-th smallest and largest dx and dy of each velocity
//    (a wave can only reach min_obs usable epochs if, per axis, that many
//    epochs keep some lane inside the image);
//  * ranks: nearest ranks floor(q (n-1) + 1/2) of q_lo, 1/2, q_hi, n = 0..64.
void make_tables(const kbm_stack &s, const kbm_search_params &p,
                 const StackLayout &l, int split, std::vector<char> &buf) {
    const int T = s.num_epochs, V = p.num_vel;
    double t0 = s.times[0];
    for (int i = 1; i < T; ++i) t0 = std::min(t0, s.times[i]);
    buf.assign(l.tab_bytes, 0);
    int *off = reinterpret_cast<int *>(buf.data() + l.off_rel);
    uint32_t *lin = reinterpret_cast<uint32_t *>(buf.data() + l.lin_rel);
    const int64_t HW = (int64_t)s.width * s.height;
    int4 *box = reinterpret_cast<int4 *>(buf.data() + l.box_rel);  // [V][2]
    int4 *mbox = reinterpret_cast<int4 *>(buf.data() + l.mbox_rel);
    std::vector<int> sx(T), sy(T);
    const int m = std::min(p.min_obs, T);
    int *ranks = reinterpret_cast<int *>(buf.data() + l.rank_rel);
    for (int v = 0; v < V; ++v) {
        const double vx = (double)p.vel[2 * v], vy = (double)p.vel[2 * v + 1];
        int4 b = make_int4(INT32_MAX, INT32_MIN, INT32_MAX, INT32_MIN);
        for (int i = 0; i < T; ++i) {
            const double t = s.times[i] - t0;
            const double px = vx * t;
            const double py = vy * t;
            const int dx = (int)std::floor(px + 0.5), dy = (int)std::floor(py + 0.5);
            const int cx = std::max(-32767, std::min(32767, dx));
            const int cy = std::max(-32767, std::min(32767, dy));
            off[(size_t)v * T + i] = (int)((uint32_t)(cx & 0xffff) | ((uint32_t)cy << 16));
            const int64_t li = (int64_t)(i < split ? i : i - split) * HW +
                               (int64_t)cy * s.width + cx;
            lin[(size_t)v * T + i] = (uint32_t)(uint64_t)li;
            b.x = std::min(b.x, cx);
            b.y = std::max(b.y, cx);
            b.z = std::min(b.z, cy);
            b.w = std::max(b.w, cy);
            sx[i] = cx;
            sy[i] = cy;
        }
        box[2 * v] = b;
        std::sort(sx.begin(), sx.end());
        std::sort(sy.begin(), sy.end());
        if (p.min_obs > T)  // no trajectory can qualify: always skip
            mbox[v] = make_int4(INT32_MAX / 2, INT32_MIN / 2, INT32_MAX / 2, INT32_MIN / 2);
        else
            mbox[v] = make_int4(sx[m - 1], sx[T - m], sy[m - 1], sy[T - m]);
    }
    for (int v = 0; v < V; ++v) {
        uint32_t same[2] = {0u, 0u};
        const int stride[2] = {1, 4};
        for (int k = 0; k < 2; ++k) {
            if (v < stride[k]) continue;
            const uint32_t *a = lin + (size_t)v * T, *b = lin + (size_t)(v - stride[k]) * T;
            for (int i = 0; i < std::min(T, 32); ++i)
                if (a[i] == b[i]) same[k] |= 1u << i;
        }
        box[2 * v + 1] = make_int4((int)same[0], (int)same[1], 0, 0);
    }
    const RankTable rt = make_rank_table(p.q_lo, p.q_hi);
    for (int n = 0; n <= KBM_MAX_EPOCHS; ++n) {
        ranks[n] = rt.lo[n];
        ranks[65 + n] = rt.md[n];
        ranks[130 + n] = rt.hi[n];
    }
}

}  // namespace srch
}  // namespace kbm

extern "C" kbm_status kbm_search_workspace_size(const kbm_stack *stacks,
                                                const kbm_search_params *p,
                                                int32_t num_stacks,
                                                size_t *bytes) {
    using namespace kbm;
    using namespace kbm::srch;
    clear_error();
    KBM_REQUIRE(bytes != nullptr, KBM_ERR_INVALID_ARG,
                "kbm_search_workspace_size: bytes is NULL");
    kbm_status st = check_search(stacks, p, num_stacks);
    if (st != KBM_OK) return st;
    size_t end = 0;
    for (int j = 0; j < num_stacks; ++j) end = layout(stacks[j], p[j], end).end;
    *bytes = align_up(end, 256);
    return KBM_OK;
}

extern "C" kbm_status kbm_search(const kbm_stack *stacks,
                                 const float *const *psi,
                                 const float *const *phi,
                                 const kbm_search_params *p, kbm_results *out,
                                 int32_t num_stacks, void *workspace,
                                 size_t workspace_bytes, hipStream_t stream) {
    using namespace kbm;
    using namespace kbm::srch;
    clear_error();
    kbm_status st = check_search(stacks, p, num_stacks);
    if (st != KBM_OK) return st;
    KBM_REQUIRE(psi != nullptr && phi != nullptr && out != nullptr,
                KBM_ERR_INVALID_ARG, "kbm_search: psi, phi, out must be non-NULL");
    size_t need = 0;
    for (int j = 0; j < num_stacks; ++j) {
        KBM_REQUIRE(psi[j] != nullptr && phi[j] != nullptr, KBM_ERR_INVALID_ARG,
                    "kbm_search: planes of stack %d are NULL", j);
        const bool empty = p[j].x_end == p[j].x_begin || p[j].y_end == p[j].y_begin;
        KBM_REQUIRE(empty || (out[j].lh && out[j].flux && out[j].vel_idx &&
                              out[j].n_obs && out[j].keep),
                    KBM_ERR_INVALID_ARG,
                    "kbm_search: result arrays of stack %d are NULL", j);
        need = layout(stacks[j], p[j], need).end;
    }
    need = align_up(need, 256);
    KBM_REQUIRE(workspace != nullptr && workspace_bytes >= need,
                KBM_ERR_WORKSPACE,
                "kbm_search: workspace of %zu bytes given, %zu needed",
                workspace_bytes, need);

    size_t cursor = 0;
    std::vector<char> tables;
    for (int j = 0; j < num_stacks; ++j) {
        const kbm_stack &s = stacks[j];
        const kbm_search_params &q = p[j];
        const StackLayout l = layout(s, q, cursor);
        cursor = l.end;
        const int Wr = q.x_end - q.x_begin, Hr = q.y_end - q.y_begin;
        if (Wr == 0 || Hr == 0) continue;
        char *ws = static_cast<char *>(workspace);
        const PlaneMode pm = plane_mode(s.num_epochs, (int64_t)s.width * s.height);
        make_tables(s, q, l, pm.split, tables);
        st = stage_to_device(ws + l.tab_off, tables.data(), l.tab_bytes, stream);
        if (st != KBM_OK) return st;
        int *flags = reinterpret_cast<int *>(ws + l.flags_off);
        float2 *pk = reinterpret_cast<float2 *>(ws + l.pk_off);
        hipLaunchKernelGGL(zero_flags_kernel, dim3(1), dim3(64), 0, stream, flags);
        KBM_LAUNCHED("zero_flags_kernel");
        const size_t n = (size_t)s.num_epochs * s.width * s.height;
        const int prep_blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
        hipLaunchKernelGGL(pack_prep_kernel, dim3(prep_blocks), dim3(256), 0,
                           stream, psi[j], phi[j], pk, flags, n);
        KBM_LAUNCHED("pack_prep_kernel");

        SearchArgs a{};
        a.pk = pk;
        // One buffer descriptor covers every epoch plane when the packed
        // planes fit 32-bit byte offsets; else two descriptors over two
        // epoch groups; else 64-bit addresses.
        const size_t hw = (size_t)s.width * s.height;
        a.am = pm.am;
        a.split = pm.split;
        a.n_elem = (uint32_t)(pm.am == 2 ? (size_t)pm.split * hw : n);
        a.pk_bytes = pm.am == 0 ? 0u : (uint32_t)(8 * (size_t)a.n_elem);
        a.pk2 = pk + (pm.am == 2 ? (size_t)pm.split * hw : 0);
        a.n_elem2 = (uint32_t)(pm.am == 2 ? n - (size_t)pm.split * hw : 0);
        a.pk2_bytes = (uint32_t)(8 * (size_t)a.n_elem2);
        a.off16 = reinterpret_cast<const int *>(ws + l.tab_off + l.off_rel);
        a.lin = reinterpret_cast<const uint32_t *>(ws + l.tab_off + l.lin_rel);
        a.vbox = reinterpret_cast<const int4 *>(ws + l.tab_off + l.box_rel);
        a.mbox = reinterpret_cast<const int4 *>(ws + l.tab_off + l.mbox_rel);
        a.ranks = reinterpret_cast<const int *>(ws + l.tab_off + l.rank_rel);
        a.flags = flags;
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
        a.Wr = Wr;
        a.Hr = Hr;
        a.tiles_x = (Wr + WAVE - 1) / WAVE;
        const int n_super_x = (a.tiles_x + ST_X - 1) / ST_X;
        a.n_super_y = (Hr + ST_Y - 1) / ST_Y;
        a.n_tiles = n_super_x * a.n_super_y * ST_TILES;
        a.coeff = (float)q.coeff;
        a.n_sigma = (float)q.n_sigma;
        a.defq = q.q_lo == 0.25 && q.q_hi == 0.75;
        if (!launch_exact_a(a.T, a, stream) && !launch_exact_b(a.T, a, stream)) {
            if (q.k <= 8)
                launch_generic<8>(a, stream);
            else
                launch_generic<16>(a, stream);
        }
        KBM_LAUNCHED("search_chunk_kernel");
        launch_finalize(a, stream);
        KBM_LAUNCHED("finalize_kernel");
    }
    return KBM_OK;
}

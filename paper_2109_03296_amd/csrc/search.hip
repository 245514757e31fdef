// Exhaustive linear-trajectory search with the in-line sigma_G filter and
// the per-pixel top-K (Section 3, 3.1 and 3.2).
//
// Layout and schedule
//  * The host turns every (velocity, epoch) pair into an integer pixel
//    offset floor(v t + 1/2) in FP64 once per call ("pointer arithmetic",
//    Section 3: images are never shifted).  The table is int2 [V][T].
//  * A prep kernel writes nu = psi / sqrt(phi) (correctly rounded binary32)
//    for every pixel-epoch into the workspace, or NaN where the pixel is not
//    usable.  nu depends only on the pixel, so the per-trajectory filter
//    reads it instead of recomputing a division and a square root per
//    trajectory-epoch; NaN doubles as the usability flag.
//  * One wavefront (64 lanes) owns 64 consecutive start pixels of one row
//    and walks the whole velocity list in order.  For a given velocity all
//    lanes read 64 consecutive floats per epoch and plane (coalesced), the
//    offsets are wave-uniform scalar loads, and the lightcurve (psi, phi, nu
//    for T epochs) lives in VGPRs.  sigma_G runs per lane on that register
//    copy: a Batcher sorting network and a select tree for the three ranks.
//  * Each lane keeps its pixel's top-K (L', velocity index) in registers;
//    the K survivors are re-evaluated once at the end to emit flux, n_obs,
//    keep bits and the raw likelihood.
//  * Workgroups are mapped XCD-major: the 8 XCDs each get a contiguous run
//    of tiles, so the rows a tile needs are shared through one L2.
#include <vector>

#include "kbm_internal.h"

namespace kbm {
namespace {

constexpr int WAVE = 64;
constexpr int NUM_XCD = 8;

struct SearchArgs {
    const float *psi;
    const float *phi;
    const float *nu;
    const int2 *off;  // [V][T] (dx, dy)
    float *lh;
    float *flux;
    int32_t *vidx;
    int16_t *nobs;
    uint64_t *keep;
    float *lh_raw;
    int W, H, T, V, K, min_obs, sigmag;
    int x0, y0, Wr, Hr, tiles_x, n_tiles;
    float coeff, n_sigma;
    RankTable rt;
};

__global__ __launch_bounds__(256) void nu_prep_kernel(
    const float *__restrict__ psi, const float *__restrict__ phi,
    float *__restrict__ nu, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t j = i; j < n; j += stride) {
        const float a = psi[j], b = phi[j];
        const bool ok = b > 0.0f && isfinite(b) && isfinite(a);
        nu[j] = ok ? a / sqrtf(b) : __builtin_nanf("");
    }
}

struct TrajOut {
    float L, Lraw, flux;
    int nv;
    uint64_t keep;
};

__device__ __forceinline__ bool ranks_before(float la, int ia, float lb,
                                             int ib) {
    return la > lb || (la == lb && ia < ib);
}

// Evaluate one trajectory: usable epochs, plain sums, optional sigma_G.
template <int TM>
__device__ __forceinline__ TrajOut eval_traj(const SearchArgs &a, int x,
                                             int y, const int2 *ov) {
    float ps[TM], ph[TM], nu[TM];
    float P = 0.0f, F = 0.0f;
    int nv = 0;
    uint32_t vlo = 0, vhi = 0;
    const size_t HW = (size_t)a.W * a.H;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        ps[i] = 0.0f;
        ph[i] = 0.0f;
        nu[i] = __builtin_nanf("");
        if (i < a.T) {
            const int2 o = ov[i];
            const int xx = x + o.x, yy = y + o.y;
            if ((unsigned)xx < (unsigned)a.W && (unsigned)yy < (unsigned)a.H) {
                const size_t q = (size_t)i * HW + (size_t)(yy * a.W + xx);
                const float c = a.nu[q];
                const float p = a.psi[q];
                const float f = a.phi[q];
                if (c == c) {
                    ps[i] = p;
                    ph[i] = f;
                    nu[i] = c;
                    ++nv;
                    P += p;
                    F += f;
                    if (i < 32)
                        vlo |= 1u << i;
                    else
                        vhi |= 1u << (i - 32);
                }
            }
        }
    }
    TrajOut r;
    r.nv = nv;
    r.keep = 0;
    r.L = -INFINITY;
    r.Lraw = -INFINITY;
    r.flux = 0.0f;
    if (nv == 0) return r;
    r.Lraw = P / sqrtf(F);
    if (a.sigmag) {
        bool kf[TM];
        r.keep = sigmag_keep<TM>(nu, nv, a.rt, a.coeff, a.n_sigma, kf);
        float Pk = 0.0f, Fk = 0.0f;
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            Pk += kf[i] ? ps[i] : 0.0f;
            Fk += kf[i] ? ph[i] : 0.0f;
        }
        r.L = Pk / sqrtf(Fk);
        r.flux = Pk / Fk;
    } else {
        r.keep = (uint64_t)vlo | ((uint64_t)vhi << 32);
        r.L = r.Lraw;
        r.flux = P / F;
    }
    return r;
}

template <int KM>
__device__ __forceinline__ int pick_int(const int (&a)[KM], int r) {
    int v = a[0];
#pragma unroll
    for (int j = 1; j < KM; ++j) v = (r == j) ? a[j] : v;
    return v;
}

template <int TM, int KM>
__global__ __launch_bounds__(WAVE) void search_kernel(SearchArgs a) {
    // XCD-major tile order: block b runs on XCD b % 8; give each XCD a
    // contiguous range of tiles.
    const int b = blockIdx.x;
    const int q = a.n_tiles / NUM_XCD, rem = a.n_tiles % NUM_XCD;
    const int xcd = b % NUM_XCD, slot = b / NUM_XCD;
    const int tile = xcd * q + min(xcd, rem) + slot;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int rx = tx * WAVE + (int)threadIdx.x;
    const int ry = ty;
    if (rx >= a.Wr) return;
    const int x = a.x0 + rx, y = a.y0 + ry;

    float kL[KM];
    int kI[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        // Slots below KM-K are placeholders that rank above everything, so
        // the K-th best always sits in the last register.
        const bool ph = j < KM - a.K;
        kL[j] = ph ? INFINITY : -INFINITY;
        kI[j] = ph ? -2 : -1;
    }

    for (int v = 0; v < a.V; ++v) {
        const TrajOut t = eval_traj<TM>(a, x, y, a.off + (size_t)v * a.T);
        if (t.nv >= a.min_obs && isfinite(t.L) &&
            ranks_before(t.L, v, kL[KM - 1], kI[KM - 1])) {
            kL[KM - 1] = t.L;
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

    const size_t base = ((size_t)ry * a.Wr + rx) * (size_t)a.K;
    for (int s = 0; s < a.K; ++s) {
        const int vi = pick_int<KM>(kI, KM - a.K + s);
        const size_t o = base + s;
        if (vi >= 0) {
            const TrajOut t = eval_traj<TM>(a, x, y, a.off + (size_t)vi * a.T);
            a.lh[o] = t.L;
            a.flux[o] = t.flux;
            a.vidx[o] = vi;
            a.nobs[o] = (int16_t)t.nv;
            a.keep[o] = t.keep;
            if (a.lh_raw) a.lh_raw[o] = t.Lraw;
        } else {
            a.lh[o] = -INFINITY;
            a.flux[o] = 0.0f;
            a.vidx[o] = -1;
            a.nobs[o] = 0;
            a.keep[o] = 0;
            if (a.lh_raw) a.lh_raw[o] = -INFINITY;
        }
    }
}

template <int TM, int KM>
void launch_search(const SearchArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL((search_kernel<TM, KM>), dim3(a.n_tiles), dim3(WAVE), 0,
                       stream, a);
}

template <int KM>
void launch_t(const SearchArgs &a, hipStream_t stream) {
    if (a.T <= 8) launch_search<8, KM>(a, stream);
    else if (a.T <= 16) launch_search<16, KM>(a, stream);
    else if (a.T <= 24) launch_search<24, KM>(a, stream);
    else if (a.T <= 32) launch_search<32, KM>(a, stream);
    else if (a.T <= 48) launch_search<48, KM>(a, stream);
    else launch_search<64, KM>(a, stream);
}

// Workspace per stack: nu plane, then the offset table.
struct StackLayout {
    size_t nu_off, nu_bytes, off_off, off_bytes, end;
};

StackLayout layout(const kbm_stack &s, const kbm_search_params &p,
                   size_t start) {
    StackLayout l;
    l.nu_off = align_up(start, 256);
    l.nu_bytes = sizeof(float) * (size_t)s.num_epochs * s.width * s.height;
    l.off_off = align_up(l.nu_off + l.nu_bytes, 256);
    l.off_bytes = sizeof(int2) * (size_t)p.num_vel * s.num_epochs;
    l.end = l.off_off + l.off_bytes;
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

// floor(v t + 1/2) in FP64, t from the earliest epoch.  This translation
// unit is compiled with -ffp-contract=off so the product is rounded before
// the addition.
void make_offsets(const kbm_stack &s, const kbm_search_params &p,
                  std::vector<int2> &out) {
    const int T = s.num_epochs;
    double t0 = s.times[0];
    for (int i = 1; i < T; ++i) t0 = std::min(t0, s.times[i]);
    out.resize((size_t)p.num_vel * T);
    for (int v = 0; v < p.num_vel; ++v) {
        const double vx = (double)p.vel[2 * v], vy = (double)p.vel[2 * v + 1];
        for (int i = 0; i < T; ++i) {
            const double t = s.times[i] - t0;
            const double px = vx * t;
            const double py = vy * t;
            out[(size_t)v * T + i] =
                make_int2((int)std::floor(px + 0.5), (int)std::floor(py + 0.5));
        }
    }
}

}  // namespace
}  // namespace kbm

extern "C" kbm_status kbm_search_workspace_size(const kbm_stack *stacks,
                                                const kbm_search_params *p,
                                                int32_t num_stacks,
                                                size_t *bytes) {
    using namespace kbm;
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
    std::vector<int2> offs;
    for (int j = 0; j < num_stacks; ++j) {
        const kbm_stack &s = stacks[j];
        const kbm_search_params &q = p[j];
        const StackLayout l = layout(s, q, cursor);
        cursor = l.end;
        const int Wr = q.x_end - q.x_begin, Hr = q.y_end - q.y_begin;
        if (Wr == 0 || Hr == 0) continue;
        char *ws = static_cast<char *>(workspace);
        float *nu = reinterpret_cast<float *>(ws + l.nu_off);
        int2 *off = reinterpret_cast<int2 *>(ws + l.off_off);
        make_offsets(s, q, offs);
        st = stage_to_device(off, offs.data(), l.off_bytes, stream);
        if (st != KBM_OK) return st;
        const size_t n = (size_t)s.num_epochs * s.width * s.height;
        const int prep_blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
        hipLaunchKernelGGL(nu_prep_kernel, dim3(prep_blocks), dim3(256), 0,
                           stream, psi[j], phi[j], nu, n);
        KBM_LAUNCHED("nu_prep_kernel");

        SearchArgs a{};
        a.psi = psi[j];
        a.phi = phi[j];
        a.nu = nu;
        a.off = off;
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
        a.n_tiles = a.tiles_x * Hr;
        a.coeff = (float)q.coeff;
        a.n_sigma = (float)q.n_sigma;
        a.rt = make_rank_table(q.q_lo, q.q_hi);
        if (q.k <= 8)
            launch_t<8>(a, stream);
        else
            launch_t<16>(a, stream);
        KBM_LAUNCHED("search_kernel");
    }
    return KBM_OK;
}

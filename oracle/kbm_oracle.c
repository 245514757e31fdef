/*
 * Plain CPU oracle for the shift-and-stack trajectory search of
 * Smotherman et al., "Sifting Through the Static" (arXiv 2109.03296).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library never
 * includes, links or calls it, and it shares no source with the GPU library.
 *
 * Everything here is a direct, slow transcription of the definitions, in
 * FP64 unless stated otherwise:
 *
 *   - likelihood planes (Section 3: psi and phi images built from the
 *     science and variance images with the PSF; masked pixels carry no
 *     weight);
 *   - trajectory sums (Section 3: Psi = sum psi_i, Phi = sum phi_i along a
 *     linear track, nu = Psi / sqrt(Phi));
 *   - the sigma_G lightcurve filter (Section 3.1, Eqs. 1-5: percentile
 *     spread times C_{25,75} ~ 0.7413, points farther than n sigma_G from
 *     the median are dropped, the likelihood is recomputed);
 *   - the in-line per-pixel top-K of Section 3.2;
 *   - the bilinear refinement objective and its analytic gradient.
 *
 * The sigma_G keep decision (the per-epoch nu_i, the order statistics,
 * sigma_G, the threshold and the comparison) can be taken in two
 * precisions.  The paper fixes none.  "binary64" (decision 1) is the plain
 * FP64 definition.  "binary32" (decision 0, the default of the legacy entry
 * points) takes the same steps in IEEE binary32 with correctly rounded
 * division and square root: the GPU kernel decides in binary32, so keep
 * masks of the two can be compared bit for bit, while the FP64 decision
 * with its per-epoch margins |nu_i - x_50| - thr certifies that every bit
 * where binary32 and FP64 disagree lies within binary32 rounding of the
 * threshold.  Sums and likelihoods stay FP64 in both modes.
 *
 * Build: gcc -O2 -fPIC -shared -fopenmp -ffp-contract=off (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KBMO_MAX_T 64

void kbmo_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int kbmo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Likelihood planes                                                    */
/* ------------------------------------------------------------------ */

/* Weight of one input pixel: zero when masked or when the data are not
 * usable (non-finite value or variance, or variance <= 0), otherwise the
 * inverse variance.  Zero weight is a *selection*: the caller skips the
 * term, so a NaN or 1e30 under the mask never enters a product. */
static double pixel_weight(float sci, float var, uint8_t masked)
{
    if (masked) return 0.0;
    if (!isfinite(sci) || !isfinite(var) || !(var > 0.0f)) return 0.0;
    return 1.0 / (double)var;
}

/* psi_i(y,x) = sum_{a,b} P[b+r][a+r] * I_i(y+b,x+a) * w_i(y+b,x+a)
 * phi_i(y,x) = sum_{a,b} P[b+r][a+r]^2 * w_i(y+b,x+a)
 * Correlation with the PSF (a matched filter); out-of-image taps add 0. */
int kbmo_planes(int32_t T, int32_t H, int32_t W, const float *sci,
                const float *var, const uint8_t *mask, const float *psf,
                int32_t k, double *psi, double *phi)
{
    if (T <= 0 || H <= 0 || W <= 0 || k <= 0 || (k % 2) == 0) return 1;
    const int r = k / 2;
#pragma omp parallel for collapse(2) schedule(static)
    for (int t = 0; t < T; ++t) {
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                double sp = 0.0, sf = 0.0;
                for (int b = -r; b <= r; ++b) {
                    const int yy = y + b;
                    if (yy < 0 || yy >= H) continue;
                    for (int a = -r; a <= r; ++a) {
                        const int xx = x + a;
                        if (xx < 0 || xx >= W) continue;
                        const size_t q = ((size_t)t * H + yy) * W + xx;
                        const double w = pixel_weight(sci[q], var[q],
                                                      mask ? mask[q] : 0);
                        if (w == 0.0) continue;
                        const double p = (double)psf[(b + r) * k + (a + r)];
                        sp += p * ((double)sci[q] * w);
                        sf += (p * p) * w;
                    }
                }
                const size_t o = ((size_t)t * H + y) * W + x;
                psi[o] = sp;
                phi[o] = sf;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Linear trajectories                                                  */
/* ------------------------------------------------------------------ */

static double earliest(int32_t T, const double *times)
{
    double t0 = times[0];
    for (int i = 1; i < T; ++i)
        if (times[i] < t0) t0 = times[i];
    return t0;
}

/* Integer pixel offset of velocity v at epoch i: round half up of v*t in
 * FP64, t measured from the earliest epoch.  off[(v*T + i)*2 + {0,1}]. */
void kbmo_offsets(int32_t T, const double *times, int32_t V, const float *vel,
                  int32_t *off)
{
    const double t0 = earliest(T, times);
    for (int v = 0; v < V; ++v) {
        for (int i = 0; i < T; ++i) {
            const double t = times[i] - t0;
            const double px = (double)vel[2 * v] * t;
            const double py = (double)vel[2 * v + 1] * t;
            off[((size_t)v * T + i) * 2 + 0] = (int32_t)floor(px + 0.5);
            off[((size_t)v * T + i) * 2 + 1] = (int32_t)floor(py + 0.5);
        }
    }
}

/* ------------------------------------------------------------------ */
/* sigma_G lightcurve filter (Section 3.1)                              */
/* ------------------------------------------------------------------ */

typedef struct {
    double q_lo, q_hi, coeff, n_sigma;
    int quantity; /* filtered value per epoch: 0 psi/sqrt(phi), 1 psi/phi */
    int decision; /* precision of the keep decision: 0 binary32, 1 binary64 */
} sg_params;

/* Nearest-rank selection: the q-quantile of n sorted values is the value
 * at index floor(q*(n-1) + 1/2). */
static int quantile_rank(double q, int n)
{
    return (int)floor(q * (double)(n - 1) + 0.5);
}

static int cmp_f32(const void *a, const void *b)
{
    const float x = *(const float *)a, y = *(const float *)b;
    return (x > y) - (x < y);
}

static int cmp_f64(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Keep mask over the participating epochs (part[i] != 0), every step in
 * binary32. */
static uint64_t sigmag_keep32(int T, const float *ps, const float *ph,
                              const int *part, const sg_params *p)
{
    float nu[KBMO_MAX_T], s[KBMO_MAX_T];
    int n = 0;
    for (int i = 0; i < T; ++i) {
        if (!part[i]) continue;
        nu[i] = p->quantity ? ps[i] / ph[i] : ps[i] / sqrtf(ph[i]);
        s[n++] = nu[i];
    }
    if (n == 0) return 0;
    qsort(s, (size_t)n, sizeof(float), cmp_f32);
    const float x_lo = s[quantile_rank(p->q_lo, n)];
    const float x_md = s[quantile_rank(0.5, n)];
    const float x_hi = s[quantile_rank(p->q_hi, n)];
    const float sigma_g = (float)p->coeff * (x_hi - x_lo);
    const float thr = (float)p->n_sigma * sigma_g;
    uint64_t keep = 0;
    for (int i = 0; i < T; ++i)
        if (part[i] && fabsf(nu[i] - x_md) <= thr) keep |= (uint64_t)1 << i;
    return keep;
}

/* The same decision in binary64 (Eqs. 1-5 evaluated as written).  When
 * margin != NULL it receives, per epoch, |nu_i - x_50| - thr (negative:
 * kept with room to spare; NaN for epochs that do not participate), and
 * *numax the largest |nu_i| of the lightcurve (0 when none participates). */
static uint64_t sigmag_keep64(int T, const float *ps, const float *ph,
                              const int *part, const sg_params *p,
                              double *margin, double *numax)
{
    double nu[KBMO_MAX_T], s[KBMO_MAX_T];
    double big = 0.0;
    int n = 0;
    for (int i = 0; i < T; ++i) {
        if (margin) margin[i] = NAN;
        if (!part[i]) continue;
        nu[i] = p->quantity ? (double)ps[i] / (double)ph[i]
                            : (double)ps[i] / sqrt((double)ph[i]);
        s[n++] = nu[i];
        if (fabs(nu[i]) > big) big = fabs(nu[i]);
    }
    if (numax) *numax = big;
    if (n == 0) return 0;
    qsort(s, (size_t)n, sizeof(double), cmp_f64);
    const double x_lo = s[quantile_rank(p->q_lo, n)];
    const double x_md = s[quantile_rank(0.5, n)];
    const double x_hi = s[quantile_rank(p->q_hi, n)];
    const double sigma_g = p->coeff * (x_hi - x_lo);
    const double thr = p->n_sigma * sigma_g;
    uint64_t keep = 0;
    for (int i = 0; i < T; ++i) {
        if (!part[i]) continue;
        const double d = fabs(nu[i] - x_md);
        if (d <= thr) keep |= (uint64_t)1 << i;
        if (margin) margin[i] = d - thr;
    }
    return keep;
}

/* Keep mask in the precision p->decision selects; the FP64 margins are
 * written when asked for, whichever precision decides. */
static uint64_t sigmag_keep(int T, const float *ps, const float *ph,
                            const int *part, const sg_params *p,
                            double *margin, double *numax)
{
    if (p->decision) return sigmag_keep64(T, ps, ph, part, p, margin, numax);
    if (margin || numax) sigmag_keep64(T, ps, ph, part, p, margin, numax);
    return sigmag_keep32(T, ps, ph, part, p);
}

static int usable(float ps, float ph)
{
    return ph > 0.0f && isfinite(ph) && isfinite(ps);
}

/* Standalone filter over n lightcurves [n][T] (Section 3.1).  phi == NULL
 * means unit weights (the values in psi are filtered directly).  The
 * filtered per-epoch value is psi/sqrt(phi) (quantity 0, the likelihood) or
 * psi/phi (quantity 1, the flux).  lh = Psi'/sqrt(Phi') over the kept
 * epochs, -inf when nothing participates.  decision: 0 binary32, 1 binary64.
 * margin ([n][T]) and numax ([n]) are optional: the FP64 margins of the
 * decision and the largest |nu_i| per lightcurve (see sigmag_keep64). */
int kbmo_sigmag_ex(int64_t n, int32_t T, const float *psi, const float *phi,
                   const uint8_t *valid, int32_t quantity, int32_t decision,
                   double q_lo, double q_hi, double coeff, double n_sigma,
                   uint64_t *keep, double *lh, double *margin, double *numax)
{
    if (T <= 0 || T > KBMO_MAX_T || (quantity != 0 && quantity != 1)) return 1;
    if (decision != 0 && decision != 1) return 1;
    const sg_params p = {q_lo, q_hi, coeff, n_sigma, quantity, decision};
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        float ps[KBMO_MAX_T], ph[KBMO_MAX_T];
        int part[KBMO_MAX_T];
        for (int i = 0; i < T; ++i) {
            ps[i] = psi[c * T + i];
            ph[i] = phi ? phi[c * T + i] : 1.0f;
            part[i] = (!valid || valid[c * T + i]) && usable(ps[i], ph[i]);
        }
        const uint64_t kp = sigmag_keep(T, ps, ph, part, &p,
                                        margin ? margin + c * T : NULL,
                                        numax ? numax + c : NULL);
        double sp = 0.0, sf = 0.0;
        for (int i = 0; i < T; ++i)
            if (kp >> i & 1) {
                sp += (double)ps[i];
                sf += (double)ph[i];
            }
        keep[c] = kp;
        if (lh) lh[c] = sf > 0.0 ? sp / sqrt(sf) : -INFINITY;
    }
    return 0;
}

int kbmo_sigmag_q(int64_t n, int32_t T, const float *psi, const float *phi,
                  const uint8_t *valid, int32_t quantity, double q_lo,
                  double q_hi, double coeff, double n_sigma, uint64_t *keep,
                  double *lh)
{
    return kbmo_sigmag_ex(n, T, psi, phi, valid, quantity, 0, q_lo, q_hi,
                          coeff, n_sigma, keep, lh, NULL, NULL);
}

int kbmo_sigmag(int64_t n, int32_t T, const float *psi, const float *phi,
                const uint8_t *valid, double q_lo, double q_hi, double coeff,
                double n_sigma, uint64_t *keep, double *lh)
{
    return kbmo_sigmag_q(n, T, psi, phi, valid, 0, q_lo, q_hi, coeff, n_sigma,
                         keep, lh);
}

/* ------------------------------------------------------------------ */
/* Search with the in-line filter and the per-pixel top-K (Section 3.2) */
/* ------------------------------------------------------------------ */

/* Ranking: larger filtered likelihood first; equal likelihoods go to the
 * smaller velocity index. */
static int ranks_before(double la, int ia, double lb, int ib)
{
    return la > lb || (la == lb && ia < ib);
}

typedef struct {
    double lh, flux, lh_raw;
    uint64_t keep;
    int n_obs;
} traj_result;

/* One trajectory from start pixel (x, y) with integer offsets off[i][2]
 * per epoch (Section 3): an epoch is usable when its pixel lies in the
 * image and carries finite psi, phi with phi > 0; Psi, Phi and n_obs run
 * over the usable epochs; then the filter (if on) and L' = Psi'/sqrt(Phi')
 * over the kept epochs.  Returns 1 when the trajectory stands (n_obs >=
 * min_obs, kept phi > 0, finite L'), else 0; n_obs is always set. */
static int eval_traj(int T, int H, int W, const float *psi, const float *phi,
                     int x, int y, const int32_t *off, int min_obs,
                     int sigmag, const sg_params *p, traj_result *r,
                     double *margin, double *numax)
{
    const size_t plane = (size_t)H * W;
    float ps[KBMO_MAX_T], ph[KBMO_MAX_T];
    int part[KBMO_MAX_T];
    int n = 0;
    double sp = 0.0, sf = 0.0;
    uint64_t valid = 0;
    for (int i = 0; i < T; ++i) {
        const int xx = x + off[2 * i + 0];
        const int yy = y + off[2 * i + 1];
        part[i] = 0;
        ps[i] = 0.0f;
        ph[i] = 0.0f;
        if (margin) margin[i] = NAN;
        if (xx < 0 || xx >= W || yy < 0 || yy >= H) continue;
        const size_t q = (size_t)i * plane + (size_t)yy * W + xx;
        if (!usable(psi[q], phi[q])) continue;
        ps[i] = psi[q];
        ph[i] = phi[q];
        part[i] = 1;
        valid |= (uint64_t)1 << i;
        ++n;
        sp += (double)ps[i];
        sf += (double)ph[i];
    }
    r->n_obs = n;
    if (numax) *numax = 0.0;
    if (n == 0 || n < min_obs || !(sf > 0.0)) return 0;
    uint64_t keep = valid;
    double kp_s = sp, kf_s = sf;
    if (sigmag) {
        keep = sigmag_keep(T, ps, ph, part, p, margin, numax);
        kp_s = 0.0;
        kf_s = 0.0;
        for (int i = 0; i < T; ++i)
            if (keep >> i & 1) {
                kp_s += (double)ps[i];
                kf_s += (double)ph[i];
            }
    }
    if (!(kf_s > 0.0)) return 0;
    const double l = kp_s / sqrt(kf_s);
    if (!isfinite(l)) return 0;
    r->lh = l;
    r->flux = kp_s / kf_s;
    r->lh_raw = sp / sqrt(sf);
    r->keep = keep;
    return 1;
}

int kbmo_search_ex(int32_t T, int32_t H, int32_t W, const float *psi,
                   const float *phi, const double *times, int32_t V,
                   const float *vel, int32_t K, int32_t min_obs, int32_t sigmag,
                   int32_t decision, double q_lo, double q_hi, double coeff,
                   double n_sigma, int32_t x_begin, int32_t y_begin,
                   int32_t x_end, int32_t y_end, double *out_lh,
                   double *out_flux, int32_t *out_vidx, int32_t *out_nobs,
                   uint64_t *out_keep, double *out_lh_raw)
{
    if (T <= 0 || T > KBMO_MAX_T || K <= 0 || V <= 0) return 1;
    if (x_end < x_begin || y_end < y_begin) return 1;
    if (decision != 0 && decision != 1) return 1;
    const int Wr = x_end - x_begin, Hr = y_end - y_begin;
    int32_t *off = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)V * T);
    if (!off) return 3;
    kbmo_offsets(T, times, V, vel, off);
    const sg_params p = {q_lo, q_hi, coeff, n_sigma, 0, decision};

#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int ry = 0; ry < Hr; ++ry) {
        for (int rx = 0; rx < Wr; ++rx) {
            const int y = y_begin + ry, x = x_begin + rx;
            const size_t o = ((size_t)ry * Wr + rx) * (size_t)K;
            double *lh = out_lh + o, *fl = out_flux + o;
            int32_t *vi = out_vidx + o, *no = out_nobs + o;
            uint64_t *kp = out_keep + o;
            double *lr = out_lh_raw ? out_lh_raw + o : NULL;
            for (int s = 0; s < K; ++s) {
                lh[s] = -INFINITY;
                fl[s] = 0.0;
                vi[s] = -1;
                no[s] = 0;
                kp[s] = 0;
                if (lr) lr[s] = -INFINITY;
            }
            for (int v = 0; v < V; ++v) {
                traj_result t;
                if (!eval_traj(T, H, W, psi, phi, x, y, off + (size_t)v * T * 2,
                               min_obs, sigmag, &p, &t, NULL, NULL))
                    continue;
                if (!ranks_before(t.lh, v, lh[K - 1], vi[K - 1])) continue;
                int s = K - 1;
                while (s > 0 && ranks_before(t.lh, v, lh[s - 1], vi[s - 1])) {
                    lh[s] = lh[s - 1];
                    fl[s] = fl[s - 1];
                    vi[s] = vi[s - 1];
                    no[s] = no[s - 1];
                    kp[s] = kp[s - 1];
                    if (lr) lr[s] = lr[s - 1];
                    --s;
                }
                lh[s] = t.lh;
                fl[s] = t.flux;
                vi[s] = v;
                no[s] = t.n_obs;
                kp[s] = t.keep;
                if (lr) lr[s] = t.lh_raw;
            }
        }
    }
    free(off);
    return 0;
}

int kbmo_search(int32_t T, int32_t H, int32_t W, const float *psi,
                const float *phi, const double *times, int32_t V,
                const float *vel, int32_t K, int32_t min_obs, int32_t sigmag,
                double q_lo, double q_hi, double coeff, double n_sigma,
                int32_t x_begin, int32_t y_begin, int32_t x_end, int32_t y_end,
                double *out_lh, double *out_flux, int32_t *out_vidx,
                int32_t *out_nobs, uint64_t *out_keep, double *out_lh_raw)
{
    return kbmo_search_ex(T, H, W, psi, phi, times, V, vel, K, min_obs, sigmag,
                          0, q_lo, q_hi, coeff, n_sigma, x_begin, y_begin,
                          x_end, y_end, out_lh, out_flux, out_vidx, out_nobs,
                          out_keep, out_lh_raw);
}

/* Explicit grid trajectories: n pairs of an integer start pixel
 * (start[j] = x, y) and a velocity (vel[j] = vx, vy, px/day), each
 * evaluated exactly as the search evaluates it (same offsets, usable
 * epochs, filter and L').  A trajectory the search would drop gets
 * lh = lh_raw = -inf, flux 0, keep 0; n_obs is always reported.  margin
 * ([n][T]) and numax ([n]) are optional: the FP64 margins of the filter
 * decision (NaN where an epoch does not take part, or for a dropped
 * trajectory, or with the filter off). */
int kbmo_eval_grid(int32_t T, int32_t H, int32_t W, const float *psi,
                   const float *phi, const double *times, int64_t n,
                   const int32_t *start, const float *vel, int32_t min_obs,
                   int32_t sigmag, int32_t decision, double q_lo, double q_hi,
                   double coeff, double n_sigma, double *out_lh,
                   double *out_flux, uint64_t *out_keep, int32_t *out_nobs,
                   double *out_lh_raw, double *margin, double *numax)
{
    if (T <= 0 || T > KBMO_MAX_T || n < 0) return 1;
    if (decision != 0 && decision != 1) return 1;
    const sg_params p = {q_lo, q_hi, coeff, n_sigma, 0, decision};
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        int32_t off[2 * KBMO_MAX_T];
        kbmo_offsets(T, times, 1, vel + 2 * j, off);
        traj_result t;
        double *mg = margin ? margin + j * T : NULL;
        const int ok = eval_traj(T, H, W, psi, phi, start[2 * j], start[2 * j + 1],
                                 off, min_obs, sigmag, &p, &t, mg,
                                 numax ? numax + j : NULL);
        out_nobs[j] = t.n_obs;
        out_lh[j] = ok ? t.lh : -INFINITY;
        out_flux[j] = ok ? t.flux : 0.0;
        out_keep[j] = ok ? t.keep : 0;
        if (out_lh_raw) out_lh_raw[j] = ok ? t.lh_raw : -INFINITY;
        if (!ok && mg)
            for (int i = 0; i < T; ++i) mg[i] = NAN;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Bilinear refinement objective and analytic gradient                  */
/* ------------------------------------------------------------------ */

/* Targeted evaluation of an explicit list of linear trajectories with
 * real-valued starts (params [n][4] = x0, y0, vx, vy as float32).  Epoch i
 * samples the pixel (floor((x0 + vx t_i) + 1/2), floor((y0 + vy t_i) + 1/2))
 * with t_i from the earliest epoch, every product and sum rounded in FP64
 * as written.  Usable epochs, n_obs, the sigma_G keep rule and L' are those
 * of kbmo_search (Section 3, 3.1).  A trajectory the search would drop
 * (n_obs < min_obs, no kept phi, non-finite L') gets lh = lh_raw = -inf,
 * flux 0, keep 0; n_obs is reported for every trajectory. */
int kbmo_score(int32_t T, int32_t H, int32_t W, const float *psi,
               const float *phi, const double *times, int64_t n,
               const float *params, int32_t min_obs, int32_t sigmag,
               double q_lo, double q_hi, double coeff, double n_sigma,
               double *out_lh, double *out_flux, uint64_t *out_keep,
               int32_t *out_nobs, double *out_lh_raw)
{
    if (T <= 0 || T > KBMO_MAX_T || n < 0) return 1;
    const sg_params p = {q_lo, q_hi, coeff, n_sigma, 0, 0};
    const double t0 = earliest(T, times);
    const size_t plane = (size_t)H * W;

#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        const double x0 = params[4 * j + 0], y0 = params[4 * j + 1];
        const double vx = params[4 * j + 2], vy = params[4 * j + 3];
        float ps[KBMO_MAX_T], ph[KBMO_MAX_T];
        int part[KBMO_MAX_T];
        int cnt = 0;
        double sp = 0.0, sf = 0.0;
        uint64_t valid = 0;
        for (int i = 0; i < T; ++i) {
            const double t = times[i] - t0;
            const double fx = floor(x0 + vx * t + 0.5);
            const double fy = floor(y0 + vy * t + 0.5);
            part[i] = 0;
            ps[i] = 0.0f;
            ph[i] = 0.0f;
            if (!(fx >= 0.0 && fx < (double)W && fy >= 0.0 && fy < (double)H)) continue;
            const size_t q = (size_t)i * plane + (size_t)fy * W + (size_t)fx;
            if (!usable(psi[q], phi[q])) continue;
            ps[i] = psi[q];
            ph[i] = phi[q];
            part[i] = 1;
            valid |= (uint64_t)1 << i;
            ++cnt;
            sp += (double)ps[i];
            sf += (double)ph[i];
        }
        out_nobs[j] = cnt;
        out_lh[j] = -INFINITY;
        out_flux[j] = 0.0;
        out_keep[j] = 0;
        if (out_lh_raw) out_lh_raw[j] = -INFINITY;
        if (cnt == 0 || cnt < min_obs || !(sf > 0.0)) continue;
        uint64_t keep = valid;
        double kp_s = sp, kf_s = sf;
        if (sigmag) {
            keep = sigmag_keep(T, ps, ph, part, &p, NULL, NULL);
            kp_s = 0.0;
            kf_s = 0.0;
            for (int i = 0; i < T; ++i)
                if (keep >> i & 1) {
                    kp_s += (double)ps[i];
                    kf_s += (double)ph[i];
                }
        }
        if (!(kf_s > 0.0)) continue;
        const double l = kp_s / sqrt(kf_s);
        if (!isfinite(l)) continue;
        out_lh[j] = l;
        out_flux[j] = kp_s / kf_s;
        out_keep[j] = keep;
        if (out_lh_raw) out_lh_raw[j] = sp / sqrt(sf);
    }
    return 0;
}

static double tap(const float *plane, int H, int W, int x, int y)
{
    if (x < 0 || x >= W || y < 0 || y >= H) return 0.0;
    return (double)plane[(size_t)y * W + x];
}

/* Bilinear sample with pixel centres at integer coordinates; out-of-image
 * taps are zero.  Also returns the one-sided (right) partial derivatives in
 * x and y, the convention that matches floor() at integer coordinates. */
static double bilinear(const float *plane, int H, int W, double x, double y,
                       double *ddx, double *ddy)
{
    const double fxl = floor(x), fyl = floor(y);
    const int ix = (int)fxl, iy = (int)fyl;
    const double fx = x - fxl, fy = y - fyl;
    const double v00 = tap(plane, H, W, ix, iy);
    const double v10 = tap(plane, H, W, ix + 1, iy);
    const double v01 = tap(plane, H, W, ix, iy + 1);
    const double v11 = tap(plane, H, W, ix + 1, iy + 1);
    *ddx = (1.0 - fy) * (v10 - v00) + fy * (v11 - v01);
    *ddy = (1.0 - fx) * (v01 - v00) + fx * (v11 - v10);
    return (1.0 - fx) * (1.0 - fy) * v00 + fx * (1.0 - fy) * v10 +
           (1.0 - fx) * fy * v01 + fx * fy * v11;
}

static void scatter(double *g, int H, int W, double x, double y, double c)
{
    const double fxl = floor(x), fyl = floor(y);
    const int ix = (int)fxl, iy = (int)fyl;
    const double fx = x - fxl, fy = y - fyl;
    const int xs[4] = {ix, ix + 1, ix, ix + 1};
    const int ys[4] = {iy, iy, iy + 1, iy + 1};
    const double ws[4] = {(1.0 - fx) * (1.0 - fy), fx * (1.0 - fy),
                          (1.0 - fx) * fy, fx * fy};
    for (int j = 0; j < 4; ++j) {
        if (xs[j] < 0 || xs[j] >= W || ys[j] < 0 || ys[j] >= H) continue;
        g[(size_t)ys[j] * W + xs[j]] += c * ws[j];
    }
}

/* L(q) = sum_{i in keep} B(psi_i, x_i, y_i) / sqrt(sum_{i in keep}
 * B(phi_i, x_i, y_i)), x_i = x0 + vx t_i, y_i = y0 + vy t_i.  L = 0 (and a
 * zero gradient) when the kept samples carry no phi.  grad_lh == NULL means
 * forward only; otherwise grad_params = g * dL/d(x0,y0,vx,vy) and g times
 * dL/dpsi, dL/dphi is added into grad_psi / grad_phi (either may be NULL). */
int kbmo_refine(int32_t T, int32_t H, int32_t W, const float *psi,
                const float *phi, const double *times, int64_t n,
                const float *params, const uint64_t *keep,
                const double *grad_lh, double *lh, double *grad_params,
                double *grad_psi, double *grad_phi)
{
    if (T <= 0 || T > KBMO_MAX_T || H <= 0 || W <= 0) return 1;
    const double t0 = earliest(T, times);
    const size_t plane = (size_t)H * W;
    for (int64_t c = 0; c < n; ++c) {
        const double x0 = params[4 * c + 0], y0 = params[4 * c + 1];
        const double vx = params[4 * c + 2], vy = params[4 * c + 3];
        const uint64_t km = keep ? keep[c] : ~(uint64_t)0;
        double sp = 0.0, sf = 0.0;
        double dpx[KBMO_MAX_T], dpy[KBMO_MAX_T], dfx[KBMO_MAX_T],
            dfy[KBMO_MAX_T], xs[KBMO_MAX_T], ys[KBMO_MAX_T], ts[KBMO_MAX_T];
        for (int i = 0; i < T; ++i) {
            ts[i] = times[i] - t0;
            xs[i] = x0 + vx * ts[i];
            ys[i] = y0 + vy * ts[i];
            if (!(km >> i & 1)) continue;
            sp += bilinear(psi + i * plane, H, W, xs[i], ys[i], &dpx[i],
                           &dpy[i]);
            sf += bilinear(phi + i * plane, H, W, xs[i], ys[i], &dfx[i],
                           &dfy[i]);
        }
        if (!(sf > 0.0)) {
            lh[c] = 0.0;
            if (grad_lh && grad_params)
                for (int j = 0; j < 4; ++j) grad_params[4 * c + j] = 0.0;
            continue;
        }
        const double l = sp / sqrt(sf);
        lh[c] = l;
        if (!grad_lh) continue;
        const double g = grad_lh[c];
        const double a = 1.0 / sqrt(sf);   /* dL/dPsi */
        const double b = -l / (2.0 * sf);  /* dL/dPhi */
        double gx0 = 0.0, gy0 = 0.0, gvx = 0.0, gvy = 0.0;
        for (int i = 0; i < T; ++i) {
            if (!(km >> i & 1)) continue;
            const double dx = a * dpx[i] + b * dfx[i];
            const double dy = a * dpy[i] + b * dfy[i];
            gx0 += dx;
            gy0 += dy;
            gvx += ts[i] * dx;
            gvy += ts[i] * dy;
            if (grad_psi) scatter(grad_psi + i * plane, H, W, xs[i], ys[i], g * a);
            if (grad_phi) scatter(grad_phi + i * plane, H, W, xs[i], ys[i], g * b);
        }
        if (grad_params) {
            grad_params[4 * c + 0] = g * gx0;
            grad_params[4 * c + 1] = g * gy0;
            grad_params[4 * c + 2] = g * gvx;
            grad_params[4 * c + 3] = g * gvy;
        }
    }
    return 0;
}

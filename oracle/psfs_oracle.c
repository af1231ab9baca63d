/*
 * psfs_oracle.c -- plain FP64 CPU reference ("the oracle") for the
 * probabilistic shape-from-silhouette occupancy pass of Song, Bian et al.,
 * "Digitize Your Body and Action in 3-D at Over 10 FPS" (Sec. 2.2.2,
 * Eq. 1-9), and for the differentiable bilinear variant built on it.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the benchmark's CPU
 * baseline use it. It shares no code, header, table or constant with the HIP
 * library; every FP32/u8 input is widened exactly to FP64 before use.
 *
 * What each function follows:
 *   psfs_oracle_slm          Eq. 1-2 (per-pixel foreground posterior, the SLM)
 *   psfs_oracle_posterior    Eq. 3-9 (voxel occupancy posterior, nearest pixel)
 *   psfs_oracle_voxel_combos Eq. 3-9 for one voxel, every admissible pixel choice
 *   psfs_oracle_fuse_views   Eq. 3-9 for given per-view SLM values
 *   psfs_oracle_bilinear_logits, psfs_oracle_bce_loss, psfs_oracle_grad
 *                            differentiable variant (not in the paper): bilinear
 *                            interpolation of log(2*SLM), BCE-with-logits loss
 *                            and its analytic adjoint.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - N(I | mu, sigma) is a Gaussian with diagonal covariance and per-channel
 *     variance; U(I) is uniform with density exp(log_u) (default 256^-3).
 *   - The voxel centre is projected; pixel centres sit at integer
 *     coordinates; the pixel is x = floor(u + 1/2), y = floor(v + 1/2).
 *   - A view whose projection leaves the image, or whose depth c <= 0, is
 *     skipped (it contributes no factor to Eq. 4).
 *   - Bilinear variant: taps floor(u) + {0,1} x floor(v) + {0,1}; taps
 *     outside the image carry log(2*SLM) = 0.
 *
 * Pins: every function here is checked by the non-GPU tests against values the
 * mathematics fixes (closed forms, a brute-force literal evaluation, a library
 * Gaussian density, the visual-hull limit, invariants, finite differences).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

int psfs_oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the later parallel loops (timing at 1 thread and at all
 * host cores); n <= 0 leaves it unchanged. */
void psfs_oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Eq. 1-2: silhouette likelihood map                                       */
/* ------------------------------------------------------------------------ */

/* Background colour model P(I | F=0) = N(I | mu, diag(var)) (Eq. 1). */
static double background_density(const uint8_t I[3], const float mu[3], const float var[3])
{
    double dens = 1.0;
    for (int c = 0; c < 3; ++c) {
        double d = (double)I[c] - (double)mu[c];
        double v = (double)var[c];
        dens *= exp(-d * d / (2.0 * v)) / sqrt(2.0 * M_PI * v);
    }
    return dens;
}

/*
 * SLM = P(F=1 | I) by Bayes (Eq. 1-2) with foreground density U = exp(log_u)
 * and pixel priors P(F=1) = P(F=0) = 1/2. Also returns 1 - SLM computed
 * without cancellation (used by the adjoint).
 */
static void slm_pixel(const uint8_t I[3], const float mu[3], const float var[3], double U,
                      double *slm, double *one_minus_slm)
{
    const double prior_fg = 0.5, prior_bg = 0.5;
    double fg = U * prior_fg;
    double bg = background_density(I, mu, var) * prior_bg;
    *slm = fg / (fg + bg);
    if (one_minus_slm) *one_minus_slm = bg / (fg + bg);
}

static int valid_variance(const float *var, int64_t nvals)
{
    for (int64_t i = 0; i < nvals; ++i)
        if (!(var[i] > 0.0f) || !isfinite(var[i])) return 0;
    return 1;
}

/* img u8 [npix][3], mean/var FP32 [npix][3] -> slm FP64 [npix]. */
int psfs_oracle_slm(int64_t npix, const uint8_t *img, const float *mean, const float *var,
                    double log_u, double *slm)
{
    if (npix < 0 || (npix > 0 && (!img || !mean || !var || !slm))) return -1;
    if (!valid_variance(var, 3 * npix)) return -2;
    double U = exp(log_u);
    for (int64_t p = 0; p < npix; ++p)
        slm_pixel(img + 3 * p, mean + 3 * p, var + 3 * p, U, &slm[p], NULL);
    return 0;
}

/* log(2 * SLM) per pixel: the quantity the bilinear variant interpolates. */
int psfs_oracle_log2slm(int64_t npix, const uint8_t *img, const float *mean, const float *var,
                        double log_u, double *out)
{
    int rc = psfs_oracle_slm(npix, img, mean, var, log_u, out);
    if (rc) return rc;
    for (int64_t p = 0; p < npix; ++p) out[p] = log(2.0 * out[p]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. 3-9: voxel occupancy posterior                                       */
/* ------------------------------------------------------------------------ */

/*
 * Eq. 5 with the sensor model of Eq. 6-9: P(S_k | V) = sum_O P(S_k | O, V) P(O),
 * P(O=0) = P(O=1) = 1/2; P(S|O=0,V=0) = 1 - SLM (Eq. 6); the three other cases
 * equal SLM (Eq. 7-9).
 */
static double view_likelihood(double s, int V)
{
    const double prior_O[2] = {0.5, 0.5};
    double sum = 0.0;
    for (int O = 0; O < 2; ++O) {
        double cond = (O == 0 && V == 0) ? 1.0 - s : s;
        sum += cond * prior_O[O];
    }
    return sum;
}

/* Eq. 3 with Eq. 4's product over the views that see the voxel. */
static double posterior_from_views(int m, const double *s, double prior)
{
    double like1 = 1.0, like0 = 1.0;
    for (int k = 0; k < m; ++k) {
        like1 *= view_likelihood(s[k], 1);
        like0 *= view_likelihood(s[k], 0);
    }
    double num = like1 * prior;
    return num / (num + like0 * (1.0 - prior));
}

/* Posterior for m views with given SLM values at the voxel's pixels. */
double psfs_oracle_fuse_views(int m, const double *s, double prior)
{
    return posterior_from_views(m, s, prior);
}

typedef struct {
    int n;
    const int32_t *W, *H;
    const double *P;          /* n x 12, row-major 3x4 */
    int nx, ny, nz;
    double o[3], h;
} geom_t;

static void voxel_centre(const geom_t *g, int64_t idx, double X[3])
{
    int64_t i = idx % g->nx, j = (idx / g->nx) % g->ny, k = idx / ((int64_t)g->nx * g->ny);
    X[0] = g->o[0] + g->h * ((double)i + 0.5);
    X[1] = g->o[1] + g->h * ((double)j + 0.5);
    X[2] = g->o[2] + g->h * ((double)k + 0.5);
}

/* (a, b, c) = P_k [X; 1]. */
static void project(const double *P, const double X[3], double abc[3])
{
    for (int r = 0; r < 3; ++r)
        abc[r] = P[4 * r + 0] * X[0] + P[4 * r + 1] * X[1] + P[4 * r + 2] * X[2] + P[4 * r + 3];
}

/*
 * Candidate pixels of one voxel-view under the nearest-pixel rule. The
 * canonical choice is first. When the projected coordinate lies within eps of
 * a rounding boundary, the neighbouring pixel is also admissible (an FP32
 * evaluation of the projection may land on either side). A candidate outside
 * the image is encoded as -1 (the view is then skipped). Returns the count
 * (0 when the voxel is behind the camera).
 */
static int pixel_candidates(const geom_t *g, int k, const double X[3], double eps, int64_t cand[4])
{
    double abc[3];
    project(g->P + 12 * k, X, abc);
    if (!(abc[2] > 0.0)) return 0;
    double u = abc[0] / abc[2], v = abc[1] / abc[2];
    double fu = floor(u + 0.5), fv = floor(v + 0.5);
    double xs[2] = {fu, fu}, ys[2] = {fv, fv};
    int nxc = 1, nyc = 1;
    double ru = (u + 0.5) - fu, rv = (v + 0.5) - fv;
    if (eps > 0.0) {
        if (ru < eps) xs[nxc++] = fu - 1.0;
        else if (ru > 1.0 - eps) xs[nxc++] = fu + 1.0;
        if (rv < eps) ys[nyc++] = fv - 1.0;
        else if (rv > 1.0 - eps) ys[nyc++] = fv + 1.0;
    }
    int cnt = 0;
    for (int a = 0; a < nyc; ++a)
        for (int b = 0; b < nxc; ++b) {
            double x = xs[b], y = ys[a];
            if (x >= 0.0 && x < (double)g->W[k] && y >= 0.0 && y < (double)g->H[k])
                cand[cnt++] = (int64_t)y * g->W[k] + (int64_t)x;
            else
                cand[cnt++] = -1;
        }
    return cnt;
}

static int make_geom(geom_t *g, int n, const int32_t *W, const int32_t *H, const double *P,
                     int nx, int ny, int nz, const double *origin, double h)
{
    if (n < 0 || nx < 0 || ny < 0 || nz < 0 || !(h > 0.0)) return -1;
    if (n > 0 && (!W || !H || !P)) return -1;
    for (int k = 0; k < n; ++k)
        if (W[k] < 1 || H[k] < 1) return -1;
    g->n = n; g->W = W; g->H = H; g->P = P;
    g->nx = nx; g->ny = ny; g->nz = nz;
    g->o[0] = origin[0]; g->o[1] = origin[1]; g->o[2] = origin[2];
    g->h = h;
    return 0;
}

/*
 * Posterior P(V=1 | {S}) of every voxel (Eq. 3-9), nearest-pixel rule.
 *   slm[k]      FP64 SLM map of view k, [H_k][W_k]
 *   post        [nz][ny][nx] canonical posterior
 *   post_lo/hi  (nullable) min / max posterior over all admissible pixel
 *               choices (see pixel_candidates); the posterior increases with
 *               every view's SLM value and a skipped view acts as SLM = 1/2
 *   ncombo      (nullable) number of admissible choice combinations (1 when
 *               no view is near a rounding boundary), saturated at 1<<30
 */
int psfs_oracle_posterior(int n, const int32_t *W, const int32_t *H, const double *P,
                          int nx, int ny, int nz, const double *origin, double h, double prior,
                          const double *const *slm, double eps_px,
                          double *post, double *post_lo, double *post_hi, int32_t *ncombo)
{
    geom_t g;
    if (make_geom(&g, n, W, H, P, nx, ny, nz, origin, h) || n > 64) return -1;
    if (!(prior > 0.0 && prior < 1.0) || !(eps_px >= 0.0 && eps_px < 0.5)) return -1;
    int64_t V = (int64_t)nx * ny * nz;
    if (V > 0 && !post) return -1;

    #pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < V; ++idx) {
        double X[3], s[64], slo[64], shi[64];
        int m = 0, mlo = 0, mhi = 0;
        int64_t combos = 1;
        voxel_centre(&g, idx, X);
        for (int k = 0; k < n; ++k) {
            int64_t cand[4];
            int nc = pixel_candidates(&g, k, X, eps_px, cand);
            if (nc == 0) continue;
            if (cand[0] >= 0) s[m++] = slm[k][cand[0]];
            /* extreme choices for the bounds: a skipped view counts as 1/2 */
            double smin = 2.0, smax = -1.0;
            for (int c = 0; c < nc; ++c) {
                double sv = cand[c] >= 0 ? slm[k][cand[c]] : 0.5;
                if (sv < smin) smin = sv;
                if (sv > smax) smax = sv;
            }
            slo[mlo++] = smin;
            shi[mhi++] = smax;
            if (combos < (1 << 30)) combos *= nc;
        }
        post[idx] = posterior_from_views(m, s, prior);
        if (post_lo) post_lo[idx] = posterior_from_views(mlo, slo, prior);
        if (post_hi) post_hi[idx] = posterior_from_views(mhi, shi, prior);
        if (ncombo) ncombo[idx] = (int32_t)(combos < (1 << 30) ? combos : (1 << 30));
    }
    return 0;
}

/*
 * Every posterior one voxel can take over the admissible pixel choices of its
 * views (enumerated in view order). Returns the number of combinations, or -1;
 * writes at most max_out values.
 */
int64_t psfs_oracle_voxel_combos(int n, const int32_t *W, const int32_t *H, const double *P,
                                 int nx, int ny, int nz, const double *origin, double h, double prior,
                                 const double *const *slm, double eps_px, int64_t voxel,
                                 double *out, int64_t max_out)
{
    geom_t g;
    if (make_geom(&g, n, W, H, P, nx, ny, nz, origin, h) || n > 64) return -1;
    if (voxel < 0 || voxel >= (int64_t)nx * ny * nz) return -1;
    double X[3];
    voxel_centre(&g, voxel, X);
    int64_t cand[64][4];
    int nc[64];
    int64_t total = 1;
    for (int k = 0; k < n; ++k) {
        nc[k] = pixel_candidates(&g, k, X, eps_px, cand[k]);
        if (nc[k] == 0) { nc[k] = 1; cand[k][0] = -2; }   /* behind: skipped */
        total *= nc[k];
        if (total > (1 << 20)) return -1;
    }
    for (int64_t t = 0; t < total && t < max_out; ++t) {
        double s[64];
        int m = 0;
        int64_t r = t;
        for (int k = 0; k < n; ++k) {
            int64_t c = cand[k][r % nc[k]];
            r /= nc[k];
            if (c >= 0) s[m++] = slm[k][c];
        }
        out[t] = posterior_from_views(m, s, prior);
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* Differentiable variant: bilinear log(2*SLM), BCE loss, analytic adjoint  */
/* ------------------------------------------------------------------------ */

/*
 * Logit of the occupancy posterior with each view's log(2*SLM) sampled
 * bilinearly at the projected voxel centre: L = logit(prior) + sum_k l~_k.
 * With a single tap of weight 1 this is the logit of Eq. 3-9's posterior,
 * since each view multiplies the odds by 2*SLM (the closed form of Eq. 5-9).
 *   l2s[k]  FP64 map [H_k][W_k] of log(2*SLM)
 *   L       [nz][ny][nx] logits
 */
int psfs_oracle_bilinear_logits(int n, const int32_t *W, const int32_t *H, const double *P,
                                int nx, int ny, int nz, const double *origin, double h,
                                double prior, const double *const *l2s, double *L)
{
    geom_t g;
    if (make_geom(&g, n, W, H, P, nx, ny, nz, origin, h)) return -1;
    if (!(prior > 0.0 && prior < 1.0)) return -1;
    int64_t V = (int64_t)nx * ny * nz;
    double L0 = log(prior / (1.0 - prior));

    #pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < V; ++idx) {
        double X[3], abc[3];
        voxel_centre(&g, idx, X);
        double acc = L0;
        for (int k = 0; k < n; ++k) {
            project(g.P + 12 * k, X, abc);
            if (!(abc[2] > 0.0)) continue;
            double u = abc[0] / abc[2], v = abc[1] / abc[2];
            double x0 = floor(u), y0 = floor(v);
            double fx = u - x0, fy = v - y0;
            double w[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
            double tx[4] = {x0, x0 + 1, x0, x0 + 1}, ty[4] = {y0, y0, y0 + 1, y0 + 1};
            for (int t = 0; t < 4; ++t) {
                if (tx[t] >= 0 && tx[t] < W[k] && ty[t] >= 0 && ty[t] < H[k])
                    acc += w[t] * l2s[k][(int64_t)ty[t] * W[k] + (int64_t)tx[t]];
            }
        }
        L[idx] = acc;
    }
    return 0;
}

static int in_region(const int32_t *sub, int64_t i, int64_t j, int64_t k)
{
    if (!sub) return 1;
    return i >= sub[0] && i < sub[1] && j >= sub[2] && j < sub[3] && k >= sub[4] && k < sub[5];
}

static int64_t region_size(const int32_t *sub, int nx, int ny, int nz)
{
    if (!sub) return (int64_t)nx * ny * nz;
    int64_t a = sub[1] - sub[0], b = sub[3] - sub[2], c = sub[5] - sub[4];
    return (a > 0 && b > 0 && c > 0) ? a * b * c : 0;
}

static double softplus(double x)
{
    return (x > 0 ? x : 0.0) + log1p(exp(-fabs(x)));
}

/* Mean BCE-with-logits over the region sub = [i0,i1,j0,j1,k0,k1) (NULL: all). */
double psfs_oracle_bce_loss(int nx, int ny, int nz, const double *L, const uint8_t *labels,
                            const int32_t *sub)
{
    int64_t cnt = region_size(sub, nx, ny, nz);
    if (cnt == 0) return 0.0;
    double acc = 0.0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                if (!in_region(sub, i, j, k)) continue;
                int64_t idx = (k * ny + j) * nx + i;
                acc += softplus(L[idx]) - (double)labels[idx] * L[idx];
            }
    return acc / (double)cnt;
}

/*
 * Analytic gradient of grad_loss * bce_loss(bilinear logits) with respect to
 * the background means, the background variances and the camera matrices.
 * Serial, fixed accumulation order (voxel index, then view, then tap).
 *   img[k], mean[k], var[k]  [H_k][W_k][3]
 *   gmean[k], gvar[k]        FP64 [H_k][W_k][3] outputs
 *   gP                       FP64 [n][12] output
 */
int psfs_oracle_grad(int n, const int32_t *W, const int32_t *H, const double *P,
                     int nx, int ny, int nz, const double *origin, double h, double prior,
                     double log_u, const uint8_t *const *img, const float *const *mean,
                     const float *const *var, const uint8_t *labels, const int32_t *sub,
                     double grad_loss, double *const *gmean, double *const *gvar, double *gP)
{
    geom_t g;
    if (make_geom(&g, n, W, H, P, nx, ny, nz, origin, h)) return -1;
    if (!(prior > 0.0 && prior < 1.0)) return -1;
    double U = exp(log_u);
    int64_t V = (int64_t)nx * ny * nz;
    int64_t cnt = region_size(sub, nx, ny, nz);

    double **l2s = calloc((size_t)(n > 0 ? n : 1), sizeof(double *));
    double **oms = calloc((size_t)(n > 0 ? n : 1), sizeof(double *));
    double **adj = calloc((size_t)(n > 0 ? n : 1), sizeof(double *));
    double *L = malloc(sizeof(double) * (size_t)(V > 0 ? V : 1));
    int rc = 0;
    if (!l2s || !oms || !adj || !L) { rc = -3; goto done; }
    for (int k = 0; k < n; ++k) {
        int64_t np = (int64_t)W[k] * H[k];
        if (!valid_variance(var[k], 3 * np)) { rc = -2; goto done; }
        l2s[k] = malloc(sizeof(double) * (size_t)np);
        oms[k] = malloc(sizeof(double) * (size_t)np);
        adj[k] = calloc((size_t)np, sizeof(double));
        if (!l2s[k] || !oms[k] || !adj[k]) { rc = -3; goto done; }
        for (int64_t p = 0; p < np; ++p) {
            double s;
            slm_pixel(img[k] + 3 * p, mean[k] + 3 * p, var[k] + 3 * p, U, &s, &oms[k][p]);
            l2s[k][p] = log(2.0 * s);
        }
    }
    rc = psfs_oracle_bilinear_logits(n, W, H, P, nx, ny, nz, origin, h, prior,
                                     (const double *const *)l2s, L);
    if (rc) goto done;
    memset(gP, 0, sizeof(double) * 12 * (size_t)n);

    /* voxel adjoint: dLoss/dL_v = grad_loss * (sigmoid(L_v) - y_v) / |S| */
    for (int64_t idx = 0; idx < V && cnt > 0; ++idx) {
        int64_t i = idx % nx, j = (idx / nx) % ny, kz = idx / ((int64_t)nx * ny);
        if (!in_region(sub, i, j, kz)) continue;
        double sig = 1.0 / (1.0 + exp(-L[idx]));
        double gv = grad_loss * (sig - (double)labels[idx]) / (double)cnt;
        double X[3], abc[3];
        voxel_centre(&g, idx, X);
        double Xh[4] = {X[0], X[1], X[2], 1.0};
        for (int k = 0; k < n; ++k) {
            project(g.P + 12 * k, X, abc);
            if (!(abc[2] > 0.0)) continue;
            double c = abc[2];
            double u = abc[0] / c, v = abc[1] / c;
            double x0 = floor(u), y0 = floor(v);
            double fx = u - x0, fy = v - y0;
            double w[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
            double dwdu[4] = {-(1 - fy), (1 - fy), -fy, fy};
            double dwdv[4] = {-(1 - fx), -fx, (1 - fx), fx};
            double tx[4] = {x0, x0 + 1, x0, x0 + 1}, ty[4] = {y0, y0, y0 + 1, y0 + 1};
            double dldu = 0.0, dldv = 0.0;
            for (int t = 0; t < 4; ++t) {
                if (!(tx[t] >= 0 && tx[t] < W[k] && ty[t] >= 0 && ty[t] < H[k])) continue;
                int64_t p = (int64_t)ty[t] * W[k] + (int64_t)tx[t];
                adj[k][p] += gv * w[t];
                dldu += dwdu[t] * l2s[k][p];
                dldv += dwdv[t] * l2s[k][p];
            }
            /* u = a/c, v = b/c with (a,b,c) = P [X;1] */
            for (int col = 0; col < 4; ++col) {
                gP[12 * k + 0 + col] += gv * dldu * Xh[col] / c;
                gP[12 * k + 4 + col] += gv * dldv * Xh[col] / c;
                gP[12 * k + 8 + col] += gv * (-dldu * u - dldv * v) * Xh[col] / c;
            }
        }
    }

    /* pixel chain: d log(2*SLM) / d mu_c = -(1 - SLM) (I_c - mu_c) / var_c,
       d log(2*SLM) / d var_c = -(1 - SLM) ((I_c - mu_c)^2 / (2 var_c^2) - 1 / (2 var_c)) */
    for (int k = 0; k < n; ++k) {
        int64_t np = (int64_t)W[k] * H[k];
        for (int64_t p = 0; p < np; ++p) {
            for (int ch = 0; ch < 3; ++ch) {
                double d = (double)img[k][3 * p + ch] - (double)mean[k][3 * p + ch];
                double vv = (double)var[k][3 * p + ch];
                gmean[k][3 * p + ch] = adj[k][p] * (-oms[k][p]) * d / vv;
                gvar[k][3 * p + ch] = adj[k][p] * (-oms[k][p]) * (d * d / (2 * vv * vv) - 1.0 / (2 * vv));
            }
        }
    }

done:
    for (int k = 0; k < n; ++k) {
        if (l2s) free(l2s[k]);
        if (oms) free(oms[k]);
        if (adj) free(adj[k]);
    }
    free(l2s); free(oms); free(adj); free(L);
    return rc;
}

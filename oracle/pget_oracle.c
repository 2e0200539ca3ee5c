/*
 * FP64 CPU oracle for the attenuated ray transform of PGET reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * Everything is plain double precision, plain loops, no blocking and no
 * fusion, written so it can be checked against the paper by eye:
 *
 *   forward   Sec. 2.1, eq. (fwd_model) with the beam transform B, in the
 *             discrete form of eq. (d_fwd_model): the emission and
 *             attenuation maps are sampled on a lattice rotated to angle
 *             theta_a (bilinear interpolation, zero outside the grid), the
 *             attenuation seen by a sample is the sum of the attenuation
 *             samples between it and the detector (midpoint rule: half of
 *             its own sample), and the collimator response r_{m,n} is a
 *             Gaussian across detector bins, the same at every depth unless
 *             a depth response is given: then the response to sample i is
 *             (1 - alpha_i) times the Gaussian taps plus alpha_i times a
 *             second set of taps (the response at the far side of the
 *             field), so that it widens with the emitter's distance from
 *             the detector.  The factor
 *             c_{m,n} >= 1 on an emitter's attenuation path is atten_scale
 *             times an optional per-sample depth factor d_i (the vertical
 *             correction: an emitter farther from the detector reaches it
 *             along a steeper path), d_i = 1 when none is given.
 *   jvp       Sec. 2.1, eq. (frechet): D_lambda F[dl] = F(dl, mu) and
 *             D_mu F[dm] = -F(lambda * B(dm), mu), discretised the same way.
 *   vjp       the exact transpose of jvp (the adjoint F'^* that the gradient
 *             F'^*[r_k] of Sec. 3.1 needs).
 *   reg       the regulariser standing in for alpha*||P x||^2 of
 *             eq. (lma_objective): 0.5*alpha*||grad x||^2 with forward
 *             differences and a Neumann boundary, and its gradient.
 *
 * Geometry (the paper fixes none of it; the readings are listed with the
 * design notes): pixel (r, c) of an N x N map has centre
 * (c - (N-1)/2, r - (N-1)/2); angle a is theta_a = angle0 + a*arc/n_angles;
 * omega = (cos, sin) points to the detector and omega_perp = (-sin, cos);
 * bin j sits at s_j = (j - (n_bins-1)/2)*bin_size; sample i of a ray at
 * t_i = (i - (n_t-1)/2)*step with n_t = 2*ceil((N/sqrt2 + 1)/step); the
 * sample point is s_j*omega_perp + t_i*omega.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n;            /* N: the maps are N x N, row-major               */
    int n_angles;     /* number of projection angles                    */
    int n_bins;       /* detector bins per angle                        */
    int psf_radius;   /* K: taps on each side (negative: ceil(3 sigma)) */
    double angle0;    /* first angle, radians                           */
    double arc;       /* angular range covered by n_angles, radians     */
    double bin_size;  /* detector bin spacing (pixels)                  */
    double step;      /* sample spacing along a ray (pixels)            */
    double psf_sigma; /* Gaussian sigma in bins; 0 = no blur            */
    double atten_scale; /* c_{m,n} of eq. (d_fwd_model): this constant  */
    const double* depth; /* times depth[i] for sample i (n_t values), or NULL */
    const double* resp;  /* depth weight alpha_i in [0, 1] of sample i (n_t values), or NULL */
    const double* far_taps; /* with resp: the far response, 2K+1 taps for offsets -K..K */
} og_geometry;

/* c for an emitter at sample i of a ray */
static double path_factor(const og_geometry* g, int i)
{
    return g->depth ? g->atten_scale * g->depth[i] : g->atten_scale;
}

/* number of samples along each ray */
int og_n_samples(const og_geometry* g)
{
    return 2 * (int)ceil(((double)g->n / sqrt(2.0) + 1.0) / g->step);
}

int og_psf_half_width(const og_geometry* g)
{
    if (g->psf_sigma <= 0.0) return 0;
    if (g->psf_radius >= 0) return g->psf_radius;
    return (int)ceil(3.0 * g->psf_sigma);
}

/* Gaussian collimator taps kappa_{-K..K}, normalised to sum 1. */
void og_psf_taps(const og_geometry* g, double* taps)
{
    int K = og_psf_half_width(g);
    if (g->psf_sigma <= 0.0) { taps[0] = 1.0; return; }
    double sum = 0.0;
    for (int k = -K; k <= K; ++k) {
        taps[k + K] = exp(-(double)(k * k) / (2.0 * g->psf_sigma * g->psf_sigma));
        sum += taps[k + K];
    }
    for (int k = -K; k <= K; ++k) taps[k + K] /= sum;
}

/* Response of the collimator to sample i of a ray at bin offset k (-K..K)
 * from the ray's own bin, given the Gaussian taps of the geometry. */
static double response(const og_geometry* g, const double* taps, int K, int i, int k)
{
    if (!g->resp) return taps[k + K];
    return (1.0 - g->resp[i]) * taps[k + K] + g->resp[i] * g->far_taps[k + K];
}

/* y[a][j + k] += r_i(k) * c over the bins inside [0, n_bins): the spread of
 * the contribution c of sample i of ray (a, j). */
static void spread_sample(const og_geometry* g, const double* taps, int K, int a, int j, int i, double c,
                          double* y)
{
    for (int k = -K; k <= K; ++k) {
        int jj = j + k;
        if (jj < 0 || jj >= g->n_bins) continue;
        y[(size_t)a * g->n_bins + jj] += response(g, taps, K, i, k) * c;
    }
}

/* sum_k r_i(k) w[a][j + k]: the transposed spread, for the adjoint. */
static double gather_sample(const og_geometry* g, const double* taps, int K, int a, int j, int i,
                            const double* w)
{
    double acc = 0.0;
    for (int k = -K; k <= K; ++k) {
        int jj = j + k;
        if (jj < 0 || jj >= g->n_bins) continue;
        acc += response(g, taps, K, i, k) * w[(size_t)a * g->n_bins + jj];
    }
    return acc;
}

/* tent function of bilinear interpolation */
static double tent(double d)
{
    double v = 1.0 - fabs(d);
    return v > 0.0 ? v : 0.0;
}

/* One ray (angle a, bin j): direction cosines and detector offset. */
typedef struct { double cs, sn, s, t0; int nt; } ray_t;

static ray_t make_ray(const og_geometry* g, int a, int j)
{
    ray_t r;
    double th = g->angle0 + (double)a * g->arc / (double)g->n_angles;
    r.cs = cos(th);
    r.sn = sin(th);
    r.s = ((double)j - 0.5 * (double)(g->n_bins - 1)) * g->bin_size;
    r.nt = og_n_samples(g);
    r.t0 = -0.5 * (double)(r.nt - 1) * g->step;
    return r;
}

/* sample point of sample i on the ray, in centred map coordinates:
 * q = s * omega_perp + t_i * omega, t_i = t0 + i * step */
static void sample_point(const og_geometry* g, const ray_t* r, int i, double* qx, double* qy)
{
    double t = r->t0 + (double)i * g->step;
    *qx = -r->s * r->sn + t * r->cs;
    *qy = r->s * r->cs + t * r->sn;
}

/*
 * The pixels whose tent weight at point q can be non-zero are the four
 * around it; for each, weight = tent(qx - x_m) * tent(qy - y_m).  Returns the
 * count (<= 4) of in-grid pixels and fills their indices and weights.
 */
static int bilinear_stencil(const og_geometry* g, double qx, double qy, int* idx, double* w)
{
    int n = g->n;
    double half = 0.5 * (double)(n - 1);
    int c0 = (int)floor(qx + half), r0 = (int)floor(qy + half);
    int cnt = 0;
    for (int dr = 0; dr <= 1; ++dr)
        for (int dc = 0; dc <= 1; ++dc) {
            int r = r0 + dr, c = c0 + dc;
            if (r < 0 || r >= n || c < 0 || c >= n) continue;
            double wt = tent(qx - ((double)c - half)) * tent(qy - ((double)r - half));
            if (wt == 0.0) continue;
            idx[cnt] = r * n + c;
            w[cnt] = wt;
            ++cnt;
        }
    return cnt;
}

static double sample_map(const og_geometry* g, const double* map, double qx, double qy)
{
    int idx[4];
    double w[4];
    int cnt = bilinear_stencil(g, qx, qy, idx, w);
    double v = 0.0;
    for (int k = 0; k < cnt; ++k) v += w[k] * map[idx[k]];
    return v;
}

/* y = K p along the bin axis of every angle, zero outside [0, n_bins). */
static void psf_apply(const og_geometry* g, const double* p, double* y)
{
    int K = og_psf_half_width(g);
    double* taps = (double*)malloc(sizeof(double) * (size_t)(2 * K + 1));
    og_psf_taps(g, taps);
    for (int a = 0; a < g->n_angles; ++a)
        for (int j = 0; j < g->n_bins; ++j) {
            double acc = 0.0;
            for (int k = -K; k <= K; ++k) {
                int jj = j - k;
                if (jj < 0 || jj >= g->n_bins) continue;
                acc += taps[k + K] * p[(size_t)a * g->n_bins + jj];
            }
            y[(size_t)a * g->n_bins + j] = acc;
        }
    free(taps);
}

/* v = K^T w, written from the matrix entries K[j][jj] = kappa_{j - jj}. */
static void psf_apply_transpose(const og_geometry* g, const double* w, double* v)
{
    int K = og_psf_half_width(g);
    double* taps = (double*)malloc(sizeof(double) * (size_t)(2 * K + 1));
    og_psf_taps(g, taps);
    for (int a = 0; a < g->n_angles; ++a)
        for (int jj = 0; jj < g->n_bins; ++jj) {
            double acc = 0.0;
            for (int j = 0; j < g->n_bins; ++j) {
                int k = j - jj;
                if (k < -K || k > K) continue;
                acc += taps[k + K] * w[(size_t)a * g->n_bins + j];
            }
            v[(size_t)a * g->n_bins + jj] = acc;
        }
    free(taps);
}

/*
 * Per-ray quantities shared by the three operators: the sampled emission
 * lam[i], sampled attenuation mu[i], and the transmission
 * E[i] = exp(-c_i * B_i),  B_i = step * (mu[i]/2 + sum_{i' > i} mu[i']).
 */
static void ray_state(const og_geometry* g, const double* f, const double* mu, const ray_t* ray,
                      double* lam_s, double* mu_s, double* E)
{
    int nt = ray->nt;
    for (int i = 0; i < nt; ++i) {
        double qx, qy;
        sample_point(g, ray, i, &qx, &qy);
        lam_s[i] = sample_map(g, f, qx, qy);
        mu_s[i] = sample_map(g, mu, qx, qy);
    }
    double beyond = 0.0; /* sum of mu samples strictly closer to the detector */
    for (int i = nt - 1; i >= 0; --i) {
        double B = g->step * (0.5 * mu_s[i] + beyond);
        E[i] = exp(-path_factor(g, i) * B);
        beyond += mu_s[i];
    }
}

/* y = A(f, mu) with a depth response: every sample spreads its own
 * contribution step * lam_i * E_i over the bins with its response r_i. */
static void forward_depth_response(const og_geometry* g, const double* f, const double* mu, double* y)
{
    int nt = og_n_samples(g);
    int K = og_psf_half_width(g);
    double* taps = (double*)malloc(sizeof(double) * (size_t)(2 * K + 1));
    double* lam_s = (double*)malloc(sizeof(double) * nt);
    double* mu_s = (double*)malloc(sizeof(double) * nt);
    double* E = (double*)malloc(sizeof(double) * nt);
    og_psf_taps(g, taps);
    memset(y, 0, sizeof(double) * (size_t)g->n_angles * g->n_bins);
    for (int a = 0; a < g->n_angles; ++a)
        for (int j = 0; j < g->n_bins; ++j) {
            ray_t ray = make_ray(g, a, j);
            ray_state(g, f, mu, &ray, lam_s, mu_s, E);
            for (int i = 0; i < nt; ++i) spread_sample(g, taps, K, a, j, i, g->step * lam_s[i] * E[i], y);
        }
    free(taps); free(lam_s); free(mu_s); free(E);
}

/* y = A(f, mu): n_angles x n_bins, row-major. */
void og_forward(const og_geometry* g, const double* f, const double* mu, double* y)
{
    if (g->resp) { forward_depth_response(g, f, mu, y); return; }
    int nt = og_n_samples(g);
    size_t nr = (size_t)g->n_angles * g->n_bins;
    double* p = (double*)malloc(sizeof(double) * nr);
    double* lam_s = (double*)malloc(sizeof(double) * nt);
    double* mu_s = (double*)malloc(sizeof(double) * nt);
    double* E = (double*)malloc(sizeof(double) * nt);
    for (int a = 0; a < g->n_angles; ++a)
        for (int j = 0; j < g->n_bins; ++j) {
            ray_t ray = make_ray(g, a, j);
            ray_state(g, f, mu, &ray, lam_s, mu_s, E);
            double acc = 0.0;
            for (int i = 0; i < nt; ++i) acc += lam_s[i] * E[i];
            p[(size_t)a * g->n_bins + j] = g->step * acc;
        }
    psf_apply(g, p, y);
    free(p); free(lam_s); free(mu_s); free(E);
}

/* The raw ray sums p (before the collimator blur), for tests of the blur. */
void og_forward_raw(const og_geometry* g, const double* f, const double* mu, double* p)
{
    int nt = og_n_samples(g);
    double* lam_s = (double*)malloc(sizeof(double) * nt);
    double* mu_s = (double*)malloc(sizeof(double) * nt);
    double* E = (double*)malloc(sizeof(double) * nt);
    for (int a = 0; a < g->n_angles; ++a)
        for (int j = 0; j < g->n_bins; ++j) {
            ray_t ray = make_ray(g, a, j);
            ray_state(g, f, mu, &ray, lam_s, mu_s, E);
            double acc = 0.0;
            for (int i = 0; i < nt; ++i) acc += lam_s[i] * E[i];
            p[(size_t)a * g->n_bins + j] = g->step * acc;
        }
    free(lam_s); free(mu_s); free(E);
}

void og_psf(const og_geometry* g, const double* p, double* y) { psf_apply(g, p, y); }
void og_psf_transpose(const og_geometry* g, const double* w, double* v) { psf_apply_transpose(g, w, v); }

/*
 * jv = J [vf, vmu] = D_lambda F[vf] + D_mu F[vmu]:
 *   raw_{a,j} = step * sum_i E_i * (vf_i - c_i * lam_i * V_i),
 *   V_i = step * (vmu_i/2 + sum_{i' > i} vmu_i')  (the beam transform of vmu),
 * followed by the same collimator blur as the forward map (with a depth
 * response, each sample's term is spread with its own response).
 */
void og_jvp(const og_geometry* g, const double* f, const double* mu, const double* vf,
            const double* vmu, double* jv)
{
    int nt = og_n_samples(g);
    int K = og_psf_half_width(g);
    size_t nr = (size_t)g->n_angles * g->n_bins;
    double* p = (double*)malloc(sizeof(double) * nr);
    double* lam_s = (double*)malloc(sizeof(double) * nt);
    double* mu_s = (double*)malloc(sizeof(double) * nt);
    double* E = (double*)malloc(sizeof(double) * nt);
    double* vf_s = (double*)malloc(sizeof(double) * nt);
    double* vmu_s = (double*)malloc(sizeof(double) * nt);
    double* taps = (double*)malloc(sizeof(double) * (size_t)(2 * K + 1));
    og_psf_taps(g, taps);
    if (g->resp) memset(jv, 0, sizeof(double) * nr);
    for (int a = 0; a < g->n_angles; ++a)
        for (int j = 0; j < g->n_bins; ++j) {
            ray_t ray = make_ray(g, a, j);
            ray_state(g, f, mu, &ray, lam_s, mu_s, E);
            for (int i = 0; i < nt; ++i) {
                double qx, qy;
                sample_point(g, &ray, i, &qx, &qy);
                vf_s[i] = sample_map(g, vf, qx, qy);
                vmu_s[i] = sample_map(g, vmu, qx, qy);
            }
            double acc = 0.0, beyond = 0.0;
            for (int i = nt - 1; i >= 0; --i) {
                double V = g->step * (0.5 * vmu_s[i] + beyond);
                double c = E[i] * (vf_s[i] - path_factor(g, i) * lam_s[i] * V);
                if (g->resp) spread_sample(g, taps, K, a, j, i, g->step * c, jv);
                else acc += c;
                beyond += vmu_s[i];
            }
            p[(size_t)a * g->n_bins + j] = g->step * acc;
        }
    if (!g->resp) psf_apply(g, p, jv);
    free(p); free(lam_s); free(mu_s); free(E); free(vf_s); free(vmu_s); free(taps);
}

/*
 * [gf, gmu] = J^T w.  With wt_i = sum_k r_i(k) w[a][j + k] (K^T w when the
 * response is the same at every depth), every sample i of ray (a, j) carries
 *   d/d lam_i = step * E_i * wt_i,
 *   d/d mu_i  = -step^2 * (c_i lam_i E_i wt_i / 2 + sum_{i' < i} c_i' lam_i' E_i' wt_i'),
 * (mu_i attenuates itself by half and every sample farther from the
 * detector fully), and these are spread back to the pixels with the same
 * bilinear weights that sampled them.
 */
void og_vjp(const og_geometry* g, const double* f, const double* mu, const double* w,
            double* gf, double* gmu)
{
    int nt = og_n_samples(g);
    int n2 = g->n * g->n;
    size_t nr = (size_t)g->n_angles * g->n_bins;
    double* wt = (double*)malloc(sizeof(double) * nr);
    double* lam_s = (double*)malloc(sizeof(double) * nt);
    double* mu_s = (double*)malloc(sizeof(double) * nt);
    double* E = (double*)malloc(sizeof(double) * nt);
    int K = og_psf_half_width(g);
    double* taps = (double*)malloc(sizeof(double) * (size_t)(2 * K + 1));
    og_psf_taps(g, taps);
    psf_apply_transpose(g, w, wt);
    memset(gf, 0, sizeof(double) * (size_t)n2);
    memset(gmu, 0, sizeof(double) * (size_t)n2);
    for (int a = 0; a < g->n_angles; ++a)
        for (int j = 0; j < g->n_bins; ++j) {
            ray_t ray = make_ray(g, a, j);
            ray_state(g, f, mu, &ray, lam_s, mu_s, E);
            /* sum over the samples farther from the detector of c*lam*E (times
             * each one's own cotangent when the response depends on depth) */
            double before = 0.0;
            for (int i = 0; i < nt; ++i) {
                double cle = path_factor(g, i) * lam_s[i] * E[i];
                double wr, d_mu;
                if (g->resp) {
                    /* the cotangent this sample sees through its own response */
                    wr = gather_sample(g, taps, K, a, j, i, w);
                    d_mu = -g->step * g->step * (0.5 * cle * wr + before);
                    before += cle * wr;
                } else {
                    wr = wt[(size_t)a * g->n_bins + j];
                    d_mu = -g->step * g->step * wr * (0.5 * cle + before);
                    before += cle;
                }
                double d_lam = g->step * E[i] * wr;
                double qx, qy;
                int idx[4];
                double bw[4];
                sample_point(g, &ray, i, &qx, &qy);
                int cnt = bilinear_stencil(g, qx, qy, idx, bw);
                for (int k = 0; k < cnt; ++k) {
                    gf[idx[k]] += bw[k] * d_lam;
                    gmu[idx[k]] += bw[k] * d_mu;
                }
            }
        }
    free(wt); free(lam_s); free(mu_s); free(E); free(taps);
}

/*
 * Regulariser 0.5 * alpha * ||grad x||^2 with forward differences,
 * (grad x)_{r,c} = (x[r][c+1] - x[r][c], x[r+1][c] - x[r][c]), zero on the
 * last column / row (Neumann boundary).
 */
double og_reg_energy(int n, double alpha, const double* x)
{
    double acc = 0.0;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            double dx = (c + 1 < n) ? x[r * n + c + 1] - x[r * n + c] : 0.0;
            double dy = (r + 1 < n) ? x[(r + 1) * n + c] - x[r * n + c] : 0.0;
            acc += dx * dx + dy * dy;
        }
    return 0.5 * alpha * acc;
}

/* out = alpha * grad^T grad x, the gradient of og_reg_energy. */
void og_reg_gradient(int n, double alpha, const double* x, double* out)
{
    memset(out, 0, sizeof(double) * (size_t)n * n);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            if (c + 1 < n) {
                double d = x[r * n + c + 1] - x[r * n + c];
                out[r * n + c + 1] += alpha * d;
                out[r * n + c] -= alpha * d;
            }
            if (r + 1 < n) {
                double d = x[(r + 1) * n + c] - x[r * n + c];
                out[(r + 1) * n + c] += alpha * d;
                out[r * n + c] -= alpha * d;
            }
        }
}

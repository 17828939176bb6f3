/*
 * epo.c -- plain FP64 CPU oracle for the EP extinction-mapping hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * Every routine here favours the plain definition over speed:
 *   - the Matern(nu=1/3) covariance uses the integral representation of the
 *     modified Bessel function K_nu, integrated adaptively;
 *   - the Vecchia precision solves each node's conditioning system on its own
 *     (no translation-invariance shortcut);
 *   - the line-of-sight operator walks every trapezoid sample;
 *   - the tilted moments are the plain integrals, done by adaptive
 *     Gauss-Kronrod (7/15) to a relative tolerance of 1e-13.
 *
 * Paper: Sale & Magorrian, "Large-scale three-dimensional Gaussian process
 * extinction mapping" (arXiv:1708.09705).  Section references below are to
 * that paper.
 *
 * Build: gcc -O2 -fPIC -shared -fopenmp (no -ffast-math).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EPO_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Adaptive Gauss-Kronrod (7-point Gauss embedded in 15-point Kronrod).      */
/* Nodes and weights are the published G7/K15 values.                         */
/* ------------------------------------------------------------------------ */
static const double GK_X[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double GK_WK[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double GK_WG[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

/* Expose the rule so tests can check its polynomial exactness. */
void epo_gk15_rule(double *xk, double *wk, double *wg) {
    for (int i = 0; i < 8; i++) { xk[i] = GK_X[i]; wk[i] = GK_WK[i]; }
    for (int i = 0; i < 4; i++) wg[i] = GK_WG[i];
}

/* Vector integrand: writes nf values at x. */
typedef void (*epo_vfun)(double x, const void *ctx, double *out);

#define GK_MAXF 3
typedef struct {
    double a, b;
    double k[GK_MAXF];   /* Kronrod estimate */
    double e[GK_MAXF];   /* |K - G| */
    double ab[GK_MAXF];  /* Kronrod estimate of the integral of |f| */
} gk_iv;

static void gk_eval(epo_vfun f, const void *ctx, int nf, gk_iv *iv) {
    double c = 0.5 * (iv->a + iv->b), h = 0.5 * (iv->b - iv->a);
    double K[GK_MAXF] = {0}, G[GK_MAXF] = {0}, AB[GK_MAXF] = {0};
    double v1[GK_MAXF], v2[GK_MAXF];
    f(c, ctx, v1);
    for (int q = 0; q < nf; q++) {
        K[q] = GK_WK[7] * v1[q];
        G[q] = GK_WG[3] * v1[q];
        AB[q] = GK_WK[7] * fabs(v1[q]);
    }
    for (int i = 0; i < 7; i++) {
        f(c - h * GK_X[i], ctx, v1);
        f(c + h * GK_X[i], ctx, v2);
        for (int q = 0; q < nf; q++) {
            K[q] += GK_WK[i] * (v1[q] + v2[q]);
            AB[q] += GK_WK[i] * (fabs(v1[q]) + fabs(v2[q]));
            if (i & 1) G[q] += GK_WG[i >> 1] * (v1[q] + v2[q]);
        }
    }
    for (int q = 0; q < nf; q++) {
        iv->k[q] = K[q] * h;
        iv->e[q] = fabs((K[q] - G[q]) * h);
        iv->ab[q] = AB[q] * fabs(h);
    }
}

/* Integrate f over the union of [bp[i], bp[i+1]], bisecting the interval
 * with the largest error until every component meets
 *   sum |K-G| <= rtol * integral of |f|.
 * Returns 0 on convergence, 1 if the interval budget ran out. */
static int gk_adapt(epo_vfun f, const void *ctx, int nf, const double *bp, int nbp,
                    double rtol, int maxiv, double *res) {
    gk_iv *iv = (gk_iv *)malloc(sizeof(gk_iv) * (size_t)maxiv);
    int n = 0;
    for (int i = 0; i + 1 < nbp && n < maxiv; i++) {
        if (!(bp[i + 1] > bp[i])) continue;
        iv[n].a = bp[i];
        iv[n].b = bp[i + 1];
        gk_eval(f, ctx, nf, &iv[n]);
        n++;
    }
    int status = 1;
    for (;;) {
        double tot[GK_MAXF] = {0}, err[GK_MAXF] = {0}, ab[GK_MAXF] = {0};
        for (int i = 0; i < n; i++)
            for (int q = 0; q < nf; q++) {
                tot[q] += iv[i].k[q];
                err[q] += iv[i].e[q];
                ab[q] += iv[i].ab[q];
            }
        int ok = 1;
        for (int q = 0; q < nf; q++)
            if (err[q] > rtol * ab[q] && err[q] > 1e-300) ok = 0;
        if (ok) { status = 0; for (int q = 0; q < nf; q++) res[q] = tot[q]; break; }
        if (n >= maxiv) { for (int q = 0; q < nf; q++) res[q] = tot[q]; break; }
        /* bisect the interval with the largest relative error contribution */
        int worst = 0;
        double wv = -1.0;
        for (int i = 0; i < n; i++) {
            double s = 0.0;
            for (int q = 0; q < nf; q++) s += iv[i].e[q] / (ab[q] > 0 ? ab[q] : 1.0);
            if (s > wv) { wv = s; worst = i; }
        }
        double m = 0.5 * (iv[worst].a + iv[worst].b);
        if (!(m > iv[worst].a && m < iv[worst].b)) { /* cannot split further */
            for (int q = 0; q < nf; q++) res[q] = tot[q];
            break;
        }
        iv[n].a = m;
        iv[n].b = iv[worst].b;
        iv[worst].b = m;
        gk_eval(f, ctx, nf, &iv[worst]);
        gk_eval(f, ctx, nf, &iv[n]);
        n++;
    }
    free(iv);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Covariance: Matern nu=1/3 (the 3-D Kolmogorov spectrum truncated at the   */
/* outer scale, Sec. 1) times a compactly supported Wendland taper. */
/* ------------------------------------------------------------------------ */
typedef struct { double nu, x; } kv_ctx;
static void kv_integrand(double t, const void *c, double *out) {
    const kv_ctx *k = (const kv_ctx *)c;
    out[0] = exp(-k->x * cosh(t)) * cosh(k->nu * t);
}

/* K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt, x > 0. */
double epo_besselk(double nu, double x) {
    kv_ctx c = {nu, x};
    /* beyond tmax the integrand is below exp(-745) relative to its peak */
    double tmax = acosh(745.0 / x + 1.0) + 1.0;
    double bp[9];
    for (int i = 0; i <= 8; i++) bp[i] = tmax * i / 8.0;
    double r;
    gk_adapt(kv_integrand, &c, 1, bp, 9, 1e-15, 4000, &r);
    return r;
}

typedef struct {
    double var;      /* sigma_f^2 */
    double ell;      /* Matern length scale (pc) */
    double support;  /* taper radius r_s (pc) */
} epo_prior;

/* Untapered Matern(1/3) covariance at separation r (pc). */
double epo_matern13(double var, double ell, double r) {
    if (r <= 0.0) return var;
    const double nu = 1.0 / 3.0;
    double x = r / ell;
    return var * pow(2.0, 1.0 - nu) / tgamma(nu) * pow(x, nu) * epo_besselk(nu, x);
}

/* Wendland psi_{3,1} taper: (1 - r/rs)_+^4 (1 + 4 r/rs). */
double epo_wendland(double rs, double r) {
    if (r >= rs) return 0.0;
    double u = 1.0 - r / rs;
    return u * u * u * u * (1.0 + 4.0 * r / rs);
}

double epo_cov(double var, double ell, double rs, double r) {
    if (r >= rs) return 0.0;
    return epo_matern13(var, ell, r) * epo_wendland(rs, r);
}

/* ------------------------------------------------------------------------ */
/* Grid: node p = i + n (j + n k) at h (i, j, k), h = L/(n-1).               */
/* ------------------------------------------------------------------------ */
static inline __attribute__((unused)) void node_xyz(int64_t p, int n, double h, double *x) {
    int64_t i = p % n, j = (p / n) % n, k = p / ((int64_t)n * n);
    x[0] = h * (double)i;
    x[1] = h * (double)j;
    x[2] = h * (double)k;
}

/* Dense Cholesky in place (lower, row-major m x m).  Returns 0 or -1 (not PD). */
static int chol_dense(double *a, int m) {
    for (int j = 0; j < m; j++) {
        double s = a[j * m + j];
        for (int k = 0; k < j; k++) s -= a[j * m + k] * a[j * m + k];
        if (!(s > 0.0)) return -1;
        double l = sqrt(s);
        a[j * m + j] = l;
        for (int i = j + 1; i < m; i++) {
            double t = a[i * m + j];
            for (int k = 0; k < j; k++) t -= a[i * m + k] * a[j * m + k];
            a[i * m + j] = t / l;
        }
    }
    return 0;
}

/* Count of the conditioning set of node p: q < p with |x_q - x_p| <= rho.
 * The comparison uses integer offsets: (di^2+dj^2+dk^2) h^2 <= rho^2 (1+1e-9). */
static int vecchia_set(int64_t p, int n, double h, double rho, int32_t *out) {
    int64_t i = p % n, j = (p / n) % n, k = p / ((int64_t)n * n);
    int R = (rho / h + 1.0 < (double)n) ? (int)floor(rho / h) + 1 : n;
    double lim = rho * rho * (1.0 + 1e-9);
    int cnt = 0;
    for (int dk = -R; dk <= 0; dk++)
        for (int dj = -R; dj <= R; dj++)
            for (int di = -R; di <= R; di++) {
                int64_t ii = i + di, jj = j + dj, kk = k + dk;
                if (ii < 0 || jj < 0 || kk < 0 || ii >= n || jj >= n || kk >= n) continue;
                int64_t q = ii + (int64_t)n * (jj + (int64_t)n * kk);
                if (q >= p) continue;
                double m2 = (double)(di * di + dj * dj + dk * dk) * h * h;
                if (m2 <= lim) {
                    if (out) out[cnt] = (int32_t)q;
                    cnt++;
                }
            }
    return cnt;
}

/* Number of nonzeros of B (strictly lower part of the Vecchia factor). */
int64_t epo_vecchia_nnz(int n, double h, double rho) {
    int64_t N = (int64_t)n * n * n, nnz = 0;
    for (int64_t p = 0; p < N; p++) nnz += vecchia_set(p, n, h, rho, NULL);
    return nnz;
}

/* Vecchia / inverse-Cholesky approximation of the tapered prior covariance.
 * For every node p (lexicographic order) with conditioning set c(p):
 *   b_p = K[c,c]^{-1} K[c,p],   d_p = K[p,p] - K[p,c] b_p,
 * and Q0 = (I-B)^T D^{-1} (I-B).  Output B in CSR (rows p, sorted columns).
 * rowptr has N+1 entries.  Returns 0, or -1 if some d_p <= 0 or a system is
 * not positive definite. */
int epo_vecchia(int n, double h, double var, double ell, double rs, double rho,
                int64_t *rowptr, int32_t *col, double *val, double *d) {
    int64_t N = (int64_t)n * n * n;
    rowptr[0] = 0;
    for (int64_t p = 0; p < N; p++) rowptr[p + 1] = rowptr[p] + vecchia_set(p, n, h, rho, NULL);
    /* The covariance between two nodes depends only on the integer squared
     * offset m = di^2 + dj^2 + dk^2; evaluate it once per m. */
    int R = (rho / h + 1.0 < (double)n) ? (int)floor(rho / h) + 1 : n;
    int mmax = 3 * (2 * R) * (2 * R) + 1;
    double *ctab = (double *)malloc(sizeof(double) * (size_t)(mmax + 1));
    for (int m = 0; m <= mmax; m++) ctab[m] = epo_cov(var, ell, rs, h * sqrt((double)m));
    int bad = 0;
#pragma omp parallel
    {
        int32_t cs[4096];
        double *K = (double *)malloc(sizeof(double) * 4096 * 64);
        double *kp = (double *)malloc(sizeof(double) * 4096);
        size_t kcap = 4096 * 64;
#pragma omp for schedule(dynamic, 256)
        for (int64_t p = 0; p < N; p++) {
            int m = vecchia_set(p, n, h, rho, cs);
            if ((size_t)m * m > kcap) {
                kcap = (size_t)m * m;
                K = (double *)realloc(K, sizeof(double) * kcap);
            }
            int64_t ip[3], ia[3], ib[3];
            ip[0] = p % n; ip[1] = (p / n) % n; ip[2] = p / ((int64_t)n * n);
            for (int a = 0; a < m; a++) {
                int64_t qa = cs[a];
                ia[0] = qa % n; ia[1] = (qa / n) % n; ia[2] = qa / ((int64_t)n * n);
                int64_t ma = (ia[0] - ip[0]) * (ia[0] - ip[0]) + (ia[1] - ip[1]) * (ia[1] - ip[1]) +
                             (ia[2] - ip[2]) * (ia[2] - ip[2]);
                kp[a] = ctab[ma];
                for (int b = 0; b <= a; b++) {
                    int64_t qb = cs[b];
                    ib[0] = qb % n; ib[1] = (qb / n) % n; ib[2] = qb / ((int64_t)n * n);
                    int64_t mab = (ia[0] - ib[0]) * (ia[0] - ib[0]) + (ia[1] - ib[1]) * (ia[1] - ib[1]) +
                                  (ia[2] - ib[2]) * (ia[2] - ib[2]);
                    K[a * m + b] = ctab[mab];
                }
            }
            double dp = ctab[0];
            if (m > 0) {
                if (chol_dense(K, m) != 0) {
#pragma omp atomic write
                    bad = 1;
                    continue;
                }
                /* solve L y = kp, L^T b = y */
                double *y = kp;
                for (int a = 0; a < m; a++) {
                    double t = y[a];
                    for (int b = 0; b < a; b++) t -= K[a * m + b] * y[b];
                    y[a] = t / K[a * m + a];
                }
                /* d_p = K[p,p] - |y|^2 */
                double yy = 0.0;
                for (int a = 0; a < m; a++) yy += y[a] * y[a];
                dp -= yy;
                for (int a = m - 1; a >= 0; a--) {
                    double t = y[a];
                    for (int b = a + 1; b < m; b++) t -= K[b * m + a] * y[b];
                    y[a] = t / K[a * m + a];
                }
                for (int a = 0; a < m; a++) {
                    col[rowptr[p] + a] = cs[a];
                    val[rowptr[p] + a] = y[a];
                }
            }
            d[p] = dp;
            if (!(dp > 0.0)) {
#pragma omp atomic write
                bad = 1;
            }
        }
        free(K);
        free(kp);
    }
    free(ctab);
    return bad ? -1 : 0;
}

/* Exact draw from the Vecchia prior: f = m0 + (I-B)^{-1} D^{1/2} xi
 * (forward substitution in lexicographic order). */
void epo_prior_draw(int64_t N, const int64_t *rowptr, const int32_t *col, const double *val,
                    const double *d, double m0, const double *xi, double *f) {
    for (int64_t p = 0; p < N; p++) {
        double s = sqrt(d[p]) * xi[p];
        for (int64_t e = rowptr[p]; e < rowptr[p + 1]; e++) s += val[e] * f[col[e]];
        f[p] = s;
    }
    for (int64_t p = 0; p < N; p++) f[p] += m0;
}

/* Prior variance of a linear functional: g^T Q0^{-1} g with
 * Q0^{-1} = (I-B)^{-1} D (I-B)^{-T}.  g is given sparse (idx sorted ascending,
 * values w).  work must hold N doubles and is returned zeroed. */
double epo_prior_quadform(int64_t N, const int64_t *rowptr, const int32_t *col, const double *val,
                          const double *d, int m, const int32_t *idx, const double *w, double *work) {
    (void)N;
    int64_t top = idx[m - 1];
    for (int a = 0; a < m; a++) work[idx[a]] += w[a];
    /* y = (I-B)^{-T} g: column-oriented backward substitution */
    double v = 0.0;
    for (int64_t p = top; p >= 0; p--) {
        double yp = work[p];
        if (yp != 0.0) {
            for (int64_t e = rowptr[p]; e < rowptr[p + 1]; e++) work[col[e]] += val[e] * yp;
            v += d[p] * yp * yp;
        }
        work[p] = 0.0;
    }
    return v;
}

/* ------------------------------------------------------------------------ */
/* Line-of-sight operator (pseudo-density f = ln(rho kappa), Sec. 5).        */
/* A_n = sum_t w_t exp(F(s_t)),  F = trilinear interpolation of f,           */
/* g_n = d ln A_n / d f,  c_n = ln A_n - g_n . f                              */
/* Samples: T = max(1, ceil(d/step)) equal steps from the observer.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    double h;
    double obs[3];
    double step;
} epo_grid;

static inline int64_t cell_of(double s, double h, int n) {
    double c = floor(s / h);
    if (c < 0) c = 0;
    if (c > n - 2) c = n - 2;
    return (int64_t)c;
}

/* Number of trapezoid intervals for a star at distance dist. */
static int64_t los_T(double dist, double step) {
    double t = ceil(dist / step);
    if (t < 1) t = 1;
    return (int64_t)t;
}

/* Collect the sorted unique set P_n of grid nodes touched by the star's
 * sightline.  Returns the count; writes up to cap node ids into out. */
int epo_los_support(const epo_grid *g, const double *xs, int32_t *out, int cap) {
    double dv[3] = {xs[0] - g->obs[0], xs[1] - g->obs[1], xs[2] - g->obs[2]};
    double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    int64_t T = los_T(dist, g->step);
    int n = g->n;
    /* the samples visit cells in order; collect the corners of each new cell */
    int cnt = 0;
    int64_t last = -1;
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(8 * (T + 1)));
    int nt = 0;
    for (int64_t t = 0; t <= T; t++) {
        double s[3];
        for (int k = 0; k < 3; k++) s[k] = g->obs[k] + (double)t / (double)T * dv[k];
        int64_t ci = cell_of(s[0], g->h, n), cj = cell_of(s[1], g->h, n), ck = cell_of(s[2], g->h, n);
        int64_t cid = ci + (int64_t)n * (cj + (int64_t)n * ck);
        if (cid == last) continue;
        last = cid;
        for (int c = 0; c < 8; c++) {
            int64_t ii = ci + (c & 1), jj = cj + ((c >> 1) & 1), kk = ck + ((c >> 2) & 1);
            tmp[nt++] = (int32_t)(ii + (int64_t)n * (jj + (int64_t)n * kk));
        }
    }
    /* sort + unique (insertion into a simple sorted list via qsort) */
    int cmp(const void *a, const void *b);
    qsort(tmp, (size_t)nt, sizeof(int32_t), cmp);
    for (int i = 0; i < nt; i++) {
        if (i > 0 && tmp[i] == tmp[i - 1]) continue;
        if (cnt < cap) out[cnt] = tmp[i];
        cnt++;
    }
    free(tmp);
    return cnt;
}

int cmp(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Evaluate A_n and g_n at field f for one star whose support P_n (sorted,
 * m entries) is given.  Writes g (m values), returns ln A_n through lnA and
 * c_n = ln A_n - g.f through c. */
void epo_los_eval(const epo_grid *g, const double *xs, const double *f, int m, const int32_t *P,
                  double *gout, double *lnA, double *c) {
    double dv[3] = {xs[0] - g->obs[0], xs[1] - g->obs[1], xs[2] - g->obs[2]};
    double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    int64_t T = los_T(dist, g->step);
    double delta = dist / (double)T;
    int n = g->n;
    for (int a = 0; a < m; a++) gout[a] = 0.0;
    double A = 0.0;
    for (int64_t t = 0; t <= T; t++) {
        double s[3];
        for (int k = 0; k < 3; k++) s[k] = g->obs[k] + (double)t / (double)T * dv[k];
        int64_t cc[3];
        double w[3];
        for (int k = 0; k < 3; k++) {
            cc[k] = cell_of(s[k], g->h, n);
            w[k] = s[k] / g->h - (double)cc[k];
        }
        double phi[8];
        int64_t node[8];
        double F = 0.0;
        for (int c8 = 0; c8 < 8; c8++) {
            int bi = c8 & 1, bj = (c8 >> 1) & 1, bk = (c8 >> 2) & 1;
            phi[c8] = (bi ? w[0] : 1.0 - w[0]) * (bj ? w[1] : 1.0 - w[1]) * (bk ? w[2] : 1.0 - w[2]);
            node[c8] = (cc[0] + bi) + (int64_t)n * ((cc[1] + bj) + (int64_t)n * (cc[2] + bk));
            F += phi[c8] * f[node[c8]];
        }
        double wt = (t == 0 || t == T) ? 0.5 * delta : delta;
        double e = wt * exp(F);
        A += e;
        for (int c8 = 0; c8 < 8; c8++) {
            /* locate node in P (binary search) */
            int lo = 0, hi = m - 1;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (P[mid] < node[c8]) lo = mid + 1; else hi = mid;
            }
            gout[lo] += e * phi[c8];
        }
    }
    double gf = 0.0;
    for (int a = 0; a < m; a++) {
        gout[a] /= A;
        gf += gout[a] * f[P[a]];
    }
    *lnA = log(A);
    *c = log(A) - gf;
}

/* ------------------------------------------------------------------------ */
/* Tilted moments of one star (Sec. 4.1 tilted distribution; App. A.2 moment*/
/* matching): cavity N(a; mu, v) times the likelihood N(A_obs; e^a, s^2).    */
/* Returns ln Z, the mean and the variance of the normalised tilted.         */
/* mode 0: extinction likelihood N(A_obs | e^a, s^2) (plain integral)         */
/* mode 1: Gaussian likelihood N(A_obs | a, s^2) (closed form)                */
/* ------------------------------------------------------------------------ */
typedef struct { double mu, v, A, s2, astar, lmax; } tilt;

static double t_ell(const tilt *t, double a) {
    double y = exp(a), r = t->A - y;
    return -(a - t->mu) * (a - t->mu) / (2.0 * t->v) - r * r / (2.0 * t->s2);
}
static double t_d1(const tilt *t, double a) {
    double y = exp(a);
    return -(a - t->mu) / t->v + (t->A - y) * y / t->s2;
}
static double t_d2(const tilt *t, double a) {
    double y = exp(a);
    return -1.0 / t->v + (t->A * y - 2.0 * y * y) / t->s2;
}

/* zero of the derivative on [lo, hi] where d1(lo) and d1(hi) differ in sign */
static double t_bisect(const tilt *t, double lo, double hi) {
    double flo = t_d1(t, lo);
    for (int it = 0; it < 400; it++) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        double fm = t_d1(t, mid);
        if (fm == 0.0) return mid;
        if ((fm > 0.0) == (flo > 0.0)) { lo = mid; flo = fm; } else hi = mid;
    }
    return 0.5 * (lo + hi);
}

static void tilt_integrand(double a, const void *c, double *out) {
    const tilt *t = (const tilt *)c;
    double e = exp(t_ell(t, a) - t->lmax);
    double u = a - t->astar;
    out[0] = e;
    out[1] = u * e;
    out[2] = u * u * e;
}

/* Returns 0 on success, 1 if the quadrature hit its interval budget,
 * -1 for invalid input (v <= 0 or s <= 0 or non-finite). */
int epo_tilted(int mode, double mu, double v, double A, double s, double *lnZ, double *mhat,
               double *vhat) {
    if (!(v > 0.0) || !(s > 0.0) || !isfinite(mu) || !isfinite(A) || !isfinite(v) || !isfinite(s))
        return -1;
    double s2 = s * s;
    if (mode == 1) {
        /* product of two Gaussians in a */
        double vh = 1.0 / (1.0 / v + 1.0 / s2);
        *vhat = vh;
        *mhat = vh * (mu / v + A / s2);
        double tv = v + s2, r = A - mu;
        *lnZ = -0.5 * log(2.0 * EPO_PI * tv) - 0.5 * r * r / tv;
        return 0;
    }
    tilt t = {mu, v, A, s2, 0.0, 0.0};
    /* Inflection points: l''(a)=0  <=>  2y^2 - A y + s2/v = 0, y = e^a. */
    double disc = A * A - 8.0 * s2 / v;
    double maxima[2] = {mu, mu};
    int nmax = 0;
    double amin = NAN; /* local minimum (bimodal case) */
    if (A > 0.0 && disc > 0.0) {
        double y1 = 0.25 * (A - sqrt(disc)), y2 = 0.25 * (A + sqrt(disc));
        double a1 = log(y1), a2 = log(y2);
        double d1a = t_d1(&t, a1), d1b = t_d1(&t, a2);
        if (d1a < 0.0) { /* maximum left of a1 */
            double step = 1.0, lo = a1 - step;
            for (int it = 0; it < 200 && !(t_d1(&t, lo) > 0.0); it++) { step *= 2.0; lo = a1 - step; }
            maxima[nmax++] = t_bisect(&t, lo, a1);
        }
        if (d1b > 0.0) { /* maximum right of a2 */
            double step = 1.0, hi = a2 + step;
            for (int it = 0; it < 200 && !(t_d1(&t, hi) < 0.0); it++) { step *= 2.0; hi = a2 + step; }
            maxima[nmax++] = t_bisect(&t, a2, hi);
        }
        if (d1a < 0.0 && d1b > 0.0) amin = t_bisect(&t, a1, a2);
    } else {
        double step = 1.0, lo = mu - step, hi = mu + step;
        for (int it = 0; it < 200 && !(t_d1(&t, lo) > 0.0); it++) { step *= 2.0; lo = mu - step; }
        step = 1.0;
        for (int it = 0; it < 200 && !(t_d1(&t, hi) < 0.0); it++) { step *= 2.0; hi = mu + step; }
        maxima[nmax++] = t_bisect(&t, lo, hi);
    }
    /* global maximum */
    int gi = 0;
    if (nmax == 2 && t_ell(&t, maxima[1]) > t_ell(&t, maxima[0])) gi = 1;
    t.astar = maxima[gi];
    t.lmax = t_ell(&t, t.astar);
    double sL = 1.0 / sqrt(-t_d2(&t, maxima[0]));
    double sR = 1.0 / sqrt(-t_d2(&t, maxima[nmax - 1]));
    if (!isfinite(sL) || sL <= 0) sL = sqrt(v);
    if (!isfinite(sR) || sR <= 0) sR = sqrt(v);
    /* tails: step outward by doubling until the log-integrand is 60 below max */
    double L = maxima[0] - sL, U = maxima[nmax - 1] + sR;
    double st = sL;
    for (int it = 0; it < 200 && t_ell(&t, L) - t.lmax > -60.0; it++) { st *= 2.0; L = maxima[0] - st; }
    st = sR;
    for (int it = 0; it < 200 && t_ell(&t, U) - t.lmax > -60.0; it++) { st *= 2.0; U = maxima[nmax - 1] + st; }
    double bp[6];
    int nb = 0;
    bp[nb++] = L;
    bp[nb++] = maxima[0];
    if (nmax == 2) {
        if (isfinite(amin)) bp[nb++] = amin;
        bp[nb++] = maxima[1];
    }
    bp[nb++] = U;
    double I[3];
    int rc = gk_adapt(tilt_integrand, &t, 3, bp, nb, 1e-13, 20000, I);
    double m1 = I[1] / I[0];
    *mhat = t.astar + m1;
    *vhat = I[2] / I[0] - m1 * m1;
    *lnZ = t.lmax + log(I[0]) - 0.5 * log(2.0 * EPO_PI * v) - 0.5 * log(2.0 * EPO_PI * s2);
    return rc;
}

/* Batched form over n stars. Returns number of failures (nonzero status). */
int epo_tilted_batch(int mode, int64_t n, const double *mu, const double *v, const double *A,
                     const double *s, double *lnZ, double *mhat, double *vhat) {
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad)
    for (int64_t i = 0; i < n; i++) {
        int st = epo_tilted(mode, mu[i], v[i], A[i], s[i], &lnZ[i], &mhat[i], &vhat[i]);
        if (st != 0) bad++;
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Batched line-of-sight helpers for many stars.                              */
/* ------------------------------------------------------------------------ */

/* Count |P_n| for every star. */
void epo_los_counts(int n, double h, const double *obs, double step, int64_t nst, const double *xyz,
                    int32_t *counts) {
    epo_grid g = {n, h, {obs[0], obs[1], obs[2]}, step};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < nst; s++) counts[s] = epo_los_support(&g, xyz + 3 * s, NULL, 0);
}

/* Fill the CSR node lists (ptr has nst+1 entries, precomputed from counts). */
void epo_los_fill(int n, double h, const double *obs, double step, int64_t nst, const double *xyz,
                  const int64_t *ptr, int32_t *nodes) {
    epo_grid g = {n, h, {obs[0], obs[1], obs[2]}, step};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < nst; s++)
        epo_los_support(&g, xyz + 3 * s, nodes + ptr[s], (int)(ptr[s + 1] - ptr[s]));
}

/* Linearise every star at field f: g values (CSR aligned with nodes),
 * ln A_n and c_n. */
void epo_los_linearise(int n, double h, const double *obs, double step, int64_t nst,
                       const double *xyz, const int64_t *ptr, const int32_t *nodes, const double *f,
                       double *gval, double *lnA, double *c) {
    epo_grid g = {n, h, {obs[0], obs[1], obs[2]}, step};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < nst; s++)
        epo_los_eval(&g, xyz + 3 * s, f, (int)(ptr[s + 1] - ptr[s]), nodes + ptr[s], gval + ptr[s],
                     &lnA[s], &c[s]);
}

/* Prior variances g_n^T Q0^{-1} g_n for a list of stars. */
void epo_prior_quadform_batch(int64_t N, const int64_t *rowptr, const int32_t *col,
                              const double *val, const double *d, int64_t nst, const int64_t *ptr,
                              const int32_t *nodes, const double *gval, double *out) {
#pragma omp parallel
    {
        double *work = (double *)calloc((size_t)N, sizeof(double));
#pragma omp for schedule(dynamic, 4)
        for (int64_t s = 0; s < nst; s++)
            out[s] = epo_prior_quadform(N, rowptr, col, val, d, (int)(ptr[s + 1] - ptr[s]),
                                        nodes + ptr[s], gval + ptr[s], work);
        free(work);
    }
}

/* X <- Q0^{-1} X for k right-hand sides (X is N x k, row-major), with
 * Q0^{-1} = (I-B)^{-1} D (I-B)^{-T}: a column-oriented backward substitution
 * with (I-B)^T, the scaling by D, a forward substitution with (I-B).  The
 * right-hand sides are split over the threads. */
void epo_q0_solve_multi(int64_t N, const int64_t *rowptr, const int32_t *col, const double *val,
                        const double *d, int64_t k, double *X) {
#pragma omp parallel
    {
        int nt = omp_get_num_threads(), t = omp_get_thread_num();
        int64_t c0 = k * t / nt, c1 = k * (t + 1) / nt;
        if (c1 > c0) {
            for (int64_t p = N - 1; p >= 0; p--) {
                double *xp = X + p * k;
                for (int64_t e = rowptr[p]; e < rowptr[p + 1]; e++) {
                    double *xc = X + (int64_t)col[e] * k;
                    for (int64_t j = c0; j < c1; j++) xc[j] += val[e] * xp[j];
                }
            }
            for (int64_t p = 0; p < N; p++)
                for (int64_t j = c0; j < c1; j++) X[p * k + j] *= d[p];
            for (int64_t p = 0; p < N; p++) {
                double *xp = X + p * k;
                for (int64_t e = rowptr[p]; e < rowptr[p + 1]; e++) {
                    const double *xc = X + (int64_t)col[e] * k;
                    for (int64_t j = c0; j < c1; j++) xp[j] += val[e] * xc[j];
                }
            }
        }
    }
}

/* Y = Q X for k vectors (X, Y: N x k, row-major) with the posterior
 * precision Q = (I-B)^T D^{-1} (I-B) + G^T diag(tau) G, G the star rows
 * (CSR gptr, gnode, gval), never formed.  work: N x k doubles.  The vectors
 * are split over the threads. */
void epo_q_mul_multi(int64_t N, const int64_t *rowptr, const int32_t *col, const double *val,
                     const double *d, int64_t S, const int64_t *gptr, const int32_t *gnode,
                     const double *gval, const double *tau, int64_t k, const double *X, double *Y,
                     double *work) {
#pragma omp parallel
    {
        int nt = omp_get_num_threads(), t = omp_get_thread_num();
        int64_t c0 = k * t / nt, c1 = k * (t + 1) / nt;
        if (c1 > c0) {
            /* work = D^{-1} (I-B) X */
            for (int64_t p = 0; p < N; p++) {
                double *wp = work + p * k;
                const double *xp = X + p * k;
                for (int64_t j = c0; j < c1; j++) wp[j] = xp[j];
                for (int64_t e = rowptr[p]; e < rowptr[p + 1]; e++) {
                    const double *xc = X + (int64_t)col[e] * k;
                    for (int64_t j = c0; j < c1; j++) wp[j] -= val[e] * xc[j];
                }
                for (int64_t j = c0; j < c1; j++) wp[j] /= d[p];
            }
            /* Y = (I-B)^T work */
            for (int64_t p = 0; p < N; p++)
                for (int64_t j = c0; j < c1; j++) Y[p * k + j] = work[p * k + j];
            for (int64_t p = 0; p < N; p++) {
                const double *wp = work + p * k;
                for (int64_t e = rowptr[p]; e < rowptr[p + 1]; e++) {
                    double *yc = Y + (int64_t)col[e] * k;
                    for (int64_t j = c0; j < c1; j++) yc[j] -= val[e] * wp[j];
                }
            }
            /* Y += G^T (tau * (G X)), one star at a time */
            double *a = (double *)malloc(sizeof(double) * (size_t)(c1 - c0));
            for (int64_t s = 0; s < S; s++) {
                for (int64_t j = c0; j < c1; j++) a[j - c0] = 0.0;
                for (int64_t e = gptr[s]; e < gptr[s + 1]; e++) {
                    const double *xq = X + (int64_t)gnode[e] * k;
                    for (int64_t j = c0; j < c1; j++) a[j - c0] += gval[e] * xq[j];
                }
                for (int64_t j = c0; j < c1; j++) a[j - c0] *= tau[s];
                for (int64_t e = gptr[s]; e < gptr[s + 1]; e++) {
                    double *yq = Y + (int64_t)gnode[e] * k;
                    for (int64_t j = c0; j < c1; j++) yq[j] += gval[e] * a[j - c0];
                }
            }
            free(a);
        }
    }
}

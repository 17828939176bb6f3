// Prior of the log pseudo-density: tapered Matern(1/3) covariance and its
// Vecchia sparse precision.
//
// The covariance shape follows the turbulence argument of Sec. 1: a
// Kolmogorov spectrum truncated at the outer (injection) scale, which in
// three dimensions is a Matern kernel with nu = 1/3 and length scale equal
// to the outer scale.  A Wendland psi_{3,1} taper makes it vanish beyond the
// support radius.  The Vecchia precision conditions each node on the earlier
// nodes (lexicographic order) within the conditioning radius.  Away from the
// faces every node sees the same geometry, so the conditioning systems are
// solved once per boundary class, not once per node.
#include "prior.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>

namespace ep {

double besselk_series(double nu, double x) {
    // I_mu(x) = sum_k (x/2)^{2k+mu} / (k! Gamma(k+mu+1))
    auto ival = [x](double mu) {
        double hx = 0.5 * x, q = hx * hx;
        double term = std::pow(hx, mu) / std::tgamma(mu + 1.0);
        double s = term;
        for (int k = 1; k < 200; k++) {
            term *= q / ((double)k * ((double)k + mu));
            s += term;
            if (std::fabs(term) < 1e-18 * std::fabs(s)) break;
        }
        return s;
    };
    const double pi = 3.14159265358979323846;
    return pi / (2.0 * std::sin(nu * pi)) * (ival(-nu) - ival(nu));
}

double cov_tapered(const PriorParams& p, double r) {
    if (r >= p.support) return 0.0;
    double c;
    if (r <= 0.0) {
        c = p.var;
    } else {
        const double nu = 1.0 / 3.0;
        double x = r / p.ell;
        c = p.var * std::pow(2.0, 1.0 - nu) / std::tgamma(nu) * std::pow(x, nu) * besselk_series(nu, x);
    }
    double u = 1.0 - r / p.support;
    double w = u * u * u * u * (1.0 + 4.0 * r / p.support);
    return c * w;
}

// Dense Cholesky (row-major, lower) in place; false if not PD.
static bool chol(std::vector<double>& a, int m) {
    for (int j = 0; j < m; j++) {
        double s = a[j * m + j];
        for (int k = 0; k < j; k++) s -= a[j * m + k] * a[j * m + k];
        if (!(s > 0.0)) return false;
        double l = std::sqrt(s);
        a[j * m + j] = l;
        for (int i = j + 1; i < m; i++) {
            double t = a[i * m + j];
            for (int k = 0; k < j; k++) t -= a[i * m + k] * a[j * m + k];
            a[i * m + j] = t / l;
        }
    }
    return true;
}

int build_vecchia(const GridGeom& g, const PriorParams& p, const Stencil& st, Vecchia& out) {
    const int n = g.n;
    const int64_t N = g.N();
    const int R = st.R;
    const int nh = (int)st.half.size() / 3;
    // covariance by integer squared offset
    int mmax = 3 * (2 * R) * (2 * R) + 1;
    std::vector<double> ctab(mmax + 1);
    for (int m = 0; m <= mmax; m++) ctab[m] = cov_tapered(p, g.h * std::sqrt((double)m));
    auto clip = [R](int64_t i, int n_) { return std::make_pair((int)std::min<int64_t>(i, R), (int)std::min<int64_t>(n_ - 1 - i, R)); };
    // classes: per-axis clipping of the neighbourhood
    std::map<std::tuple<int, int, int, int, int, int>, int> cls;
    std::vector<std::vector<int>> cls_off;   // valid offset indices per class
    std::vector<std::vector<double>> cls_b;  // coefficients per class
    std::vector<double> cls_d;
    std::vector<int32_t> node_cls(N);
    for (int64_t q = 0; q < N; q++) {
        int64_t i = q % n, j = (q / n) % n, k = q / ((int64_t)n * n);
        auto ci = clip(i, n), cj = clip(j, n), ck = clip(k, n);
        auto key = std::make_tuple(ci.first, ci.second, cj.first, cj.second, ck.first, ck.second);
        auto it = cls.find(key);
        if (it != cls.end()) { node_cls[q] = it->second; continue; }
        int id = (int)cls_off.size();
        cls[key] = id;
        node_cls[q] = id;
        std::vector<int> offs;
        for (int o = 0; o < nh; o++) {
            int di = st.half[3 * o], dj = st.half[3 * o + 1], dk = st.half[3 * o + 2];
            if (i + di < 0 || i + di >= n || j + dj < 0 || j + dj >= n || k + dk < 0 || k + dk >= n) continue;
            offs.push_back(o);
        }
        int m = (int)offs.size();
        std::vector<double> K((size_t)m * m), kp(m);
        for (int a = 0; a < m; a++) {
            const int* oa = &st.half[3 * offs[a]];
            kp[a] = ctab[oa[0] * oa[0] + oa[1] * oa[1] + oa[2] * oa[2]];
            for (int b = 0; b < m; b++) {
                const int* ob = &st.half[3 * offs[b]];
                int dx = oa[0] - ob[0], dy = oa[1] - ob[1], dz = oa[2] - ob[2];
                K[(size_t)a * m + b] = ctab[dx * dx + dy * dy + dz * dz];
            }
        }
        double dd = ctab[0];
        std::vector<double> b(m);
        if (m > 0) {
            if (!chol(K, m)) return -1;
            for (int a = 0; a < m; a++) {
                double t = kp[a];
                for (int c = 0; c < a; c++) t -= K[(size_t)a * m + c] * b[c];
                b[a] = t / K[(size_t)a * m + a];
            }
            double yy = 0;
            for (int a = 0; a < m; a++) yy += b[a] * b[a];
            dd -= yy;
            for (int a = m - 1; a >= 0; a--) {
                double t = b[a];
                for (int c = a + 1; c < m; c++) t -= K[(size_t)c * m + a] * b[c];
                b[a] = t / K[(size_t)a * m + a];
            }
        }
        if (!(dd > 0.0)) return -1;
        cls_off.push_back(offs);
        cls_b.push_back(b);
        cls_d.push_back(dd);
    }
    out.rowptr.assign(N + 1, 0);
    for (int64_t q = 0; q < N; q++) out.rowptr[q + 1] = out.rowptr[q] + (int64_t)cls_off[node_cls[q]].size();
    out.col.resize(out.rowptr[N]);
    out.val.resize(out.rowptr[N]);
    out.d.resize(N);
    for (int64_t q = 0; q < N; q++) {
        const auto& offs = cls_off[node_cls[q]];
        const auto& b = cls_b[node_cls[q]];
        out.d[q] = cls_d[node_cls[q]];
        std::vector<std::pair<int32_t, double>> row;
        row.reserve(offs.size());
        for (size_t a = 0; a < offs.size(); a++) {
            const int* o = &st.half[3 * offs[a]];
            int64_t c = q + o[0] + (int64_t)n * (o[1] + (int64_t)n * o[2]);
            row.emplace_back((int32_t)c, b[a]);
        }
        std::sort(row.begin(), row.end());
        for (size_t a = 0; a < row.size(); a++) {
            out.col[out.rowptr[q] + a] = row[a].first;
            out.val[out.rowptr[q] + a] = row[a].second;
        }
    }
    return 0;
}

void build_q0(const GridGeom& g, const Stencil& st, const Vecchia& v, Q0Table& out) {
    const int n = g.n;
    const int64_t N = g.N();
    const int R = st.R;
    // non-positive offsets of the full stencil, (0,0,0) first
    out.lower.assign({0, 0, 0});
    for (size_t o = 0; o < st.full.size(); o += 3) {
        int di = st.full[o], dj = st.full[o + 1], dk = st.full[o + 2];
        bool neg = dk < 0 || (dk == 0 && (dj < 0 || (dj == 0 && di < 0)));
        if (neg) { out.lower.push_back(di); out.lower.push_back(dj); out.lower.push_back(dk); }
    }
    out.nlower = (int)out.lower.size() / 3;
    int W = 4 * R + 1;
    std::vector<int> idx((size_t)W * W * W, -1);
    for (int o = 0; o < out.nlower; o++) {
        int di = out.lower[3 * o], dj = out.lower[3 * o + 1], dk = out.lower[3 * o + 2];
        idx[((size_t)(dk + 2 * R) * W + (dj + 2 * R)) * W + (di + 2 * R)] = o;
    }
    out.val.assign((size_t)N * out.nlower, 0.0);
    // Q0 = sum_p r_p r_p^T / d_p with r_p = e_p - B[p,:]^T
    std::vector<std::pair<int64_t, double>> r;
    for (int64_t p = 0; p < N; p++) {
        r.clear();
        r.emplace_back(p, 1.0);
        for (int64_t e = v.rowptr[p]; e < v.rowptr[p + 1]; e++) r.emplace_back(v.col[e], -v.val[e]);
        double id = 1.0 / v.d[p];
        for (size_t a = 0; a < r.size(); a++)
            for (size_t b = 0; b < r.size(); b++) {
                int64_t qa = r[a].first, qb = r[b].first;
                if (qb > qa) continue;   // store (qa, qb) with qb <= qa
                int64_t ia = qa % n, ja = (qa / n) % n, ka = qa / ((int64_t)n * n);
                int64_t ib = qb % n, jb = (qb / n) % n, kb = qb / ((int64_t)n * n);
                int di = (int)(ib - ia), dj = (int)(jb - ja), dk = (int)(kb - ka);
                int o = idx[((size_t)(dk + 2 * R) * W + (dj + 2 * R)) * W + (di + 2 * R)];
                out.val[(size_t)qa * out.nlower + o] += r[a].second * r[b].second * id;
            }
    }
}

void q0_times_const(const GridGeom& g, const Vecchia& v, double m0, std::vector<double>& out) {
    const int64_t N = g.N();
    std::vector<double> s(N);
    for (int64_t p = 0; p < N; p++) {
        double r = 1.0;
        for (int64_t e = v.rowptr[p]; e < v.rowptr[p + 1]; e++) r -= v.val[e];
        s[p] = r / v.d[p];
    }
    out.assign(s.begin(), s.end());
    for (int64_t p = 0; p < N; p++)
        for (int64_t e = v.rowptr[p]; e < v.rowptr[p + 1]; e++) out[v.col[e]] -= v.val[e] * s[p];
    for (int64_t p = 0; p < N; p++) out[p] *= m0;
}

void prior_draw(const GridGeom& g, const Vecchia& v, double m0, const double* xi, double* f) {
    const int64_t N = g.N();
    for (int64_t p = 0; p < N; p++) {
        double s = std::sqrt(v.d[p]) * xi[p];
        for (int64_t e = v.rowptr[p]; e < v.rowptr[p + 1]; e++) s += v.val[e] * (f[v.col[e]] - m0);
        f[p] = s + m0;
    }
}

}  // namespace ep

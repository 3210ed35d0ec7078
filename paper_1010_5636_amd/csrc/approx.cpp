// Sign-function approximants, computed on the host in FP64.
//
// * Minimax polynomial (Sec. 2.2, Eq. 5 and Eq. 6): sign(x) ~ x P(x^2),
//   P(y) = sum_{k=0}^{n} c_k T_k(z), z = (2y - 1 - eps)/(1 - eps), minimising
//   delta = max_{eps<=y<=1} |1 - sqrt(y) P(y)| (full c_0 in the sum).  Found by
//   the Remez exchange for the weight sqrt(y): the optimum's error
//   equioscillates at n + 2 points.
// * Zolotarev's optimal rational approximation of sign(x) on [k, 1]:
//   r(x) = x sum_l beta_l / (x^2 + sigma_l) with sigma_l = k^2 sn^2/cn^2 at
//   u = (2l-1) K(k')/(2n) (parameter k'^2 = 1 - k^2), numerator zeros at
//   u = 2l K(k')/(2n), and the scale chosen so that 1 - r equioscillates.
// Jacobi elliptic functions via the arithmetic-geometric mean and descending
// Landen transformation (DLMF 22.20(ii)).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "ndq_internal.h"
#include "ndq_solver.h"

namespace {

struct Agm {
    std::vector<double> a, c;
};

// AGM sequence for parameter m (= modulus^2): a0 = 1, b0 = sqrt(1-m), c0 = sqrt(m)
Agm agm(double m) {
    Agm s;
    double a = 1.0, b = sqrt(1.0 - m), c = sqrt(m);
    s.a.push_back(a);
    s.c.push_back(c);
    for (int it = 0; it < 64 && fabs(c) > 1e-17 * a; ++it) {
        const double an = 0.5 * (a + b);
        const double cn = 0.5 * (a - b);
        b = sqrt(a * b);
        a = an;
        c = cn;
        s.a.push_back(a);
        s.c.push_back(c);
    }
    return s;
}

double ellip_k(double m) { return M_PI / (2.0 * agm(m).a.back()); }

void ellip_sncn(double u, double m, double* sn, double* cn) {
    const Agm s = agm(m);
    const int n = (int)s.a.size() - 1;
    double phi = ldexp(s.a[n] * u, n);
    for (int j = n; j >= 1; --j) phi = 0.5 * (phi + asin(s.c[j] * sin(phi) / s.a[j]));
    *sn = sin(phi);
    *cn = cos(phi);
}

// Golden-section search for the maximum of sgn*f on [lo, hi].
template <class F>
double golden_max(F f, double lo, double hi, double sgn) {
    const double gr = 0.5 * (sqrt(5.0) - 1.0);
    for (int it = 0; it < 120 && hi - lo > 1e-15 * fmax(1.0, fabs(hi)); ++it) {
        const double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
        if (sgn * f(x1) > sgn * f(x2)) hi = x2;
        else lo = x1;
    }
    return 0.5 * (lo + hi);
}

// All local extrema of f sampled at t[] (endpoints included), refined.
template <class F>
std::vector<double> extrema(F f, const std::vector<double>& t) {
    const size_t n = t.size();
    std::vector<double> v(n);
    for (size_t i = 0; i < n; ++i) v[i] = f(t[i]);
    std::vector<double> out;
    out.push_back(t[0]);
    for (size_t i = 1; i + 1 < n; ++i) {
        const double dl = v[i] - v[i - 1], dr = v[i + 1] - v[i];
        const bool mx = dl > 0 && dr <= 0, mn = dl < 0 && dr >= 0;
        if (mx || mn) out.push_back(golden_max(f, t[i - 1], t[i + 1], mx ? 1.0 : -1.0));
    }
    out.push_back(t[n - 1]);
    return out;
}

int make_zolotarev(double k, int n, ndq::Approx* ap) {
    const double kp2 = 1.0 - k * k;
    const double bigk = ellip_k(kp2);
    std::vector<double> c(2 * n);
    for (int j = 1; j < 2 * n; ++j) {
        double sn, cn;
        ellip_sncn(j * bigk / (2.0 * n), kp2, &sn, &cn);
        c[j] = sn * sn / (cn * cn);
    }
    std::vector<double> sigma(n), zero(n > 1 ? n - 1 : 0);
    for (int l = 0; l < n; ++l) sigma[l] = k * k * c[2 * l + 1];
    for (int l = 0; l + 1 < n; ++l) zero[l] = k * k * c[2 * l + 2];
    auto g = [&](double x) {
        double num = 1.0, den = 1.0;
        for (double z : zero) num *= x * x + z;
        for (double s : sigma) den *= x * x + s;
        return x * num / den;
    };
    std::vector<double> grid(20000);
    for (size_t i = 0; i < grid.size(); ++i) grid[i] = k * pow(1.0 / k, (double)i / (grid.size() - 1));
    const std::vector<double> ext = extrema(g, grid);
    double gmax = -1e300, gmin = 1e300;
    for (double x : ext) {
        const double v = g(x);
        gmax = std::max(gmax, v);
        gmin = std::min(gmin, v);
    }
    const double scale = 2.0 / (gmax + gmin);
    ap->delta = (gmax - gmin) / (gmax + gmin);
    ap->a = sigma;
    ap->b.assign(n, 0.0);
    for (int l = 0; l < n; ++l) {
        double num = 1.0, den = 1.0;
        for (double z : zero) num *= z - sigma[l];
        for (int j = 0; j < n; ++j)
            if (j != l) den *= sigma[j] - sigma[l];
        ap->b[l] = scale * num / den;
    }
    return NDQ_OK;
}

// Chebyshev sum sum_k c_k T_k(z) by Clenshaw's recurrence.
double cheb_sum(const std::vector<double>& c, double z) {
    double b1 = 0.0, b2 = 0.0;
    for (int k = (int)c.size() - 1; k >= 1; --k) {
        const double b0 = c[k] + 2.0 * z * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return c[0] + z * b1 - b2;
}

// Solve A x = rhs (dense, row-major, size m) by Gaussian elimination with
// partial pivoting; A and rhs are overwritten.
bool solve_dense(std::vector<double>& A, std::vector<double>& rhs, int m) {
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (fabs(A[(size_t)r * m + col]) > fabs(A[(size_t)piv * m + col])) piv = r;
        if (A[(size_t)piv * m + col] == 0.0) return false;
        if (piv != col) {
            for (int j = 0; j < m; ++j) std::swap(A[(size_t)col * m + j], A[(size_t)piv * m + j]);
            std::swap(rhs[col], rhs[piv]);
        }
        const double d = A[(size_t)col * m + col];
        for (int r = col + 1; r < m; ++r) {
            const double f = A[(size_t)r * m + col] / d;
            if (f == 0.0) continue;
            for (int j = col; j < m; ++j) A[(size_t)r * m + j] -= f * A[(size_t)col * m + j];
            rhs[r] -= f * rhs[col];
        }
    }
    for (int r = m - 1; r >= 0; --r) {
        double s = rhs[r];
        for (int j = r + 1; j < m; ++j) s -= A[(size_t)r * m + j] * rhs[j];
        rhs[r] = s / A[(size_t)r * m + r];
    }
    return true;
}

int make_minmax(double eps, int n, ndq::Approx* ap) {
    const int m = n + 2;
    auto y_of = [&](double th) { return 0.5 * ((1.0 - eps) * cos(th) + 1.0 + eps); };
    std::vector<double> theta(m);
    for (int i = 0; i < m; ++i) theta[i] = M_PI * (double)(m - 1 - i) / (double)(m - 1);  // y ascending
    std::vector<double> c(n + 1, 0.0), best_c;
    double delta = 1.0, best_delta = INFINITY;
    for (int iter = 0; iter < 80; ++iter) {
        // sqrt(y_i) P(y_i) + (-1)^i E = 1
        std::vector<double> A((size_t)m * m), rhs(m, 1.0);
        for (int i = 0; i < m; ++i) {
            const double y = y_of(theta[i]);
            const double z = (2.0 * y - 1.0 - eps) / (1.0 - eps);
            const double sy = sqrt(y);
            double t0 = 1.0, t1 = z;
            for (int k = 0; k <= n; ++k) {
                double tk;
                if (k == 0) tk = 1.0;
                else if (k == 1) tk = z;
                else {
                    tk = 2.0 * z * t1 - t0;
                    t0 = t1;
                    t1 = tk;
                }
                A[(size_t)i * m + k] = sy * tk;
            }
            A[(size_t)i * m + n + 1] = (i & 1) ? -1.0 : 1.0;
        }
        if (!solve_dense(A, rhs, m)) return ndq::fail(NDQ_ENOCONV, "Remez: singular reference system");
        for (int k = 0; k <= n; ++k) c[k] = rhs[k];
        const double level = fabs(rhs[n + 1]);
        auto err = [&](double th) {
            const double y = y_of(th);
            return 1.0 - sqrt(y) * cheb_sum(c, (2.0 * y - 1.0 - eps) / (1.0 - eps));
        };
        const int npts = std::max(4000, 40 * m);
        std::vector<double> grid(npts);
        for (int i = 0; i < npts; ++i) grid[i] = M_PI * (double)i / (npts - 1);
        std::vector<double> ext = extrema(err, grid);
        std::sort(ext.begin(), ext.end(), [](double a, double b) { return a > b; });  // y ascending
        std::vector<double> pts, vals;
        double emax = 0.0;
        for (double t : ext) {
            const double e = err(t);
            emax = std::max(emax, fabs(e));
            // merge consecutive equal signs, keeping the larger magnitude
            if (!vals.empty() && ((vals.back() > 0) == (e > 0))) {
                if (fabs(e) > fabs(vals.back())) {
                    pts.back() = t;
                    vals.back() = e;
                }
            } else {
                pts.push_back(t);
                vals.push_back(e);
            }
        }
        delta = emax;
        // keep the iterate with the smallest max error (the quantity minimised);
        // at ~1e-13 the error curve is double-precision rounding noise and further
        // exchanges would only pick noise extrema
        if (emax < best_delta) {
            best_delta = emax;
            best_c = c;
        }
        if (emax - level <= 1e-7 * emax || emax <= 1e-13) break;
        while ((int)pts.size() > m) {
            if (fabs(vals.front()) < fabs(vals.back())) {
                pts.erase(pts.begin());
                vals.erase(vals.begin());
            } else {
                pts.pop_back();
                vals.pop_back();
            }
        }
        if ((int)pts.size() < m) break;
        theta = pts;
    }
    (void)delta;
    ap->a = best_c.empty() ? c : best_c;
    ap->b.clear();
    ap->delta = best_c.empty() ? delta : best_delta;
    return NDQ_OK;
}

}  // namespace

extern "C" {

int ndq_approx_create(int kind, double lo, int degree, ndq_approx** out) {
    if (!out) return ndq::fail(NDQ_EINVAL, "ndq_approx_create: NULL output");
    if (!(lo > 0.0 && lo < 1.0)) return ndq::fail(NDQ_EINVAL, "ndq_approx_create: need 0 < lo < 1 (got %g)", lo);
    ndq::Approx* ap = new (std::nothrow) ndq::Approx;
    if (!ap) return ndq::fail(NDQ_EINVAL, "out of host memory");
    ap->kind = kind;
    ap->lo = lo;
    ap->n = degree;
    int rc;
    if (kind == NDQ_ZOLOTAREV) {
        if (degree < 1 || degree > NDQ_MAX_SHIFTS) {
            delete ap;
            return ndq::fail(NDQ_EINVAL, "Zolotarev: number of poles must be in [1, %d]", NDQ_MAX_SHIFTS);
        }
        rc = make_zolotarev(lo, degree, ap);
    } else if (kind == NDQ_MINMAX_POLY) {
        if (degree < 0 || degree > 2000) {
            delete ap;
            return ndq::fail(NDQ_EINVAL, "minimax polynomial: degree must be in [0, 2000]");
        }
        rc = make_minmax(lo, degree, ap);
    } else {
        delete ap;
        return ndq::fail(NDQ_EINVAL, "ndq_approx_create: unknown kind %d", kind);
    }
    if (rc) {
        delete ap;
        return rc;
    }
    *out = reinterpret_cast<ndq_approx*>(ap);
    return NDQ_OK;
}

int ndq_approx_from_coeffs(int kind, int n, const double* a, const double* b, double lo, double delta,
                           ndq_approx** out) {
    if (!out || !a || (kind == NDQ_ZOLOTAREV && !b)) return ndq::fail(NDQ_EINVAL, "ndq_approx_from_coeffs: NULL argument");
    if (kind == NDQ_ZOLOTAREV ? (n < 1 || n > NDQ_MAX_SHIFTS) : (kind != NDQ_MINMAX_POLY || n < 0 || n > 2000))
        return ndq::fail(NDQ_EINVAL, "ndq_approx_from_coeffs: bad kind/size");
    ndq::Approx* ap = new (std::nothrow) ndq::Approx;
    if (!ap) return ndq::fail(NDQ_EINVAL, "out of host memory");
    ap->kind = kind;
    ap->n = n;
    ap->lo = lo;
    ap->delta = delta;
    if (kind == NDQ_ZOLOTAREV) {
        ap->a.assign(a, a + n);
        ap->b.assign(b, b + n);
    } else {
        ap->a.assign(a, a + n + 1);
    }
    *out = reinterpret_cast<ndq_approx*>(ap);
    return NDQ_OK;
}

int ndq_approx_info(const ndq_approx* h, int* kind, int* n, double* lo, double* delta) {
    if (!h) return ndq::fail(NDQ_EINVAL, "ndq_approx_info: NULL handle");
    const ndq::Approx* ap = reinterpret_cast<const ndq::Approx*>(h);
    if (kind) *kind = ap->kind;
    if (n) *n = ap->n;
    if (lo) *lo = ap->lo;
    if (delta) *delta = ap->delta;
    return NDQ_OK;
}

int ndq_approx_coeffs(const ndq_approx* h, double* a, double* b) {
    if (!h) return ndq::fail(NDQ_EINVAL, "ndq_approx_coeffs: NULL handle");
    const ndq::Approx* ap = reinterpret_cast<const ndq::Approx*>(h);
    if (a) memcpy(a, ap->a.data(), ap->a.size() * sizeof(double));
    if (b && !ap->b.empty()) memcpy(b, ap->b.data(), ap->b.size() * sizeof(double));
    return NDQ_OK;
}

void ndq_approx_destroy(ndq_approx* h) { delete reinterpret_cast<ndq::Approx*>(h); }

}  // extern "C"

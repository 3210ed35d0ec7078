// Dense Hermitian eigensolver for the small projected matrices of the
// eigensolver and the Rayleigh-Ritz steps (n <= a few hundred), on the host.
// Cyclic complex Jacobi: each off-diagonal entry a_pq = |a_pq| e^{i phi} is
// removed by the unitary J = diag(1, e^{-i phi}) G, with G the real Jacobi
// rotation of the symmetric 2x2 problem [[a_pp, |a_pq|], [|a_pq|, a_qq]]
// (Numerical Recipes' tan(theta) choice for stability).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <numeric>
#include <vector>

#include "ndq_internal.h"
#include "ndq_eig.h"

namespace ndq {

int hermitian_eig(int n, std::vector<std::complex<double>>& a, std::vector<double>& w,
                  std::vector<std::complex<double>>& z) {
    using cd = std::complex<double>;
    z.assign((size_t)n * n, cd(0.0, 0.0));
    for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
    auto A = [&](int i, int j) -> cd& { return a[(size_t)i * n + j]; };
    double fro = 0.0;
    for (auto& x : a) fro += std::norm(x);
    fro = sqrt(fro);
    for (int i = 0; i < n; ++i) A(i, i) = cd(A(i, i).real(), 0.0);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += std::norm(A(p, q));
        if (sqrt(off) <= 1e-16 * fro || off == 0.0) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const cd b = A(p, q);
                const double ab = std::abs(b);
                if (ab <= 1e-300) continue;
                const cd u = b / ab;          // e^{i phi}
                const cd ub = std::conj(u);
                const double app = A(p, p).real(), aqq = A(q, q).real();
                const double theta = (aqq - app) / (2.0 * ab);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                // columns: A <- A J, J = [[c, s], [-s ub, c ub]] on (p, q)
                for (int k = 0; k < n; ++k) {
                    const cd akp = A(k, p), akq = A(k, q);
                    A(k, p) = c * akp - s * ub * akq;
                    A(k, q) = s * akp + c * ub * akq;
                    const cd zkp = z[(size_t)k * n + p], zkq = z[(size_t)k * n + q];
                    z[(size_t)k * n + p] = c * zkp - s * ub * zkq;
                    z[(size_t)k * n + q] = s * zkp + c * ub * zkq;
                }
                // rows: A <- J^H A
                for (int k = 0; k < n; ++k) {
                    const cd apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk - s * u * aqk;
                    A(q, k) = s * apk + c * u * aqk;
                }
                A(p, q) = A(q, p) = 0.0;
                A(p, p) = cd(A(p, p).real(), 0.0);
                A(q, q) = cd(A(q, q).real(), 0.0);
            }
        }
    }
    // sort ascending
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int i, int j) { return A(i, i).real() < A(j, j).real(); });
    w.resize(n);
    std::vector<cd> zs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        w[j] = A(idx[j], idx[j]).real();
        for (int k = 0; k < n; ++k) zs[(size_t)k * n + j] = z[(size_t)k * n + idx[j]];
    }
    z.swap(zs);
    return NDQ_OK;
}

}  // namespace ndq

extern "C" int ndq_host_eigh(int n, double* a, double* w, double* z) {
    if (n < 1 || n > 4096 || !a || !w || !z) return ndq::fail(NDQ_EINVAL, "ndq_host_eigh: bad arguments");
    std::vector<std::complex<double>> m((size_t)n * n), zz;
    memcpy(m.data(), a, sizeof(double) * 2 * (size_t)n * n);
    std::vector<double> ww;
    const int rc = ndq::hermitian_eig(n, m, ww, zz);
    if (rc) return rc;
    memcpy(w, ww.data(), sizeof(double) * n);
    memcpy(z, zz.data(), sizeof(double) * 2 * (size_t)n * n);
    return NDQ_OK;
}

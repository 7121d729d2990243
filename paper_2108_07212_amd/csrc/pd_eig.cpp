// pd_eig.cpp -- dense symmetric eigensolver for the closure's mode shapes.
//
// Householder reduction to tridiagonal form (A = Q T Q^T), then the implicit
// QL iteration with a shift from the leading 2 x 2 block, each plane rotation
// applied to the columns of Q (the classical method; Golub & Van Loan,
// "Matrix Computations", Sec. 8.3).  Runs once per particle shape at setup.
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <stdexcept>
#include <vector>

#include "pd_internal.h"

namespace pd {

void sym_eig(std::vector<double> &A, int n, std::vector<double> &w) {
    // Z = Q^T: row j of Z is column j of Q, so that the plane rotations of
    // the QL sweep touch two contiguous rows
    std::vector<double> Z((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n, 0.0), p(n, 0.0), u(n, 0.0), t(n, 0.0);
    auto at = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };

    // ---- Householder: zero column k below the subdiagonal ------------------
    for (int k = 0; k + 2 < n; ++k) {
        double ss = 0.0;
        for (int i = k + 1; i < n; ++i) ss += at(i, k) * at(i, k);
        const double xn = std::sqrt(ss);
        if (xn == 0.0) continue;
        const double alpha = at(k + 1, k) > 0.0 ? -xn : xn;
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i) {
            v[i] = at(i, k) - (i == k + 1 ? alpha : 0.0);
            vn += v[i] * v[i];
        }
        vn = std::sqrt(vn);
        if (vn == 0.0) continue;
        for (int i = k + 1; i < n; ++i) v[i] /= vn;
        // P A P with P = I - 2 v v^T on the trailing block: A -= 2 (v u^T + u v^T),
        // u = A v - (v^T A v) v
        double vAv = 0.0;
        for (int i = k + 1; i < n; ++i) {
            double s = 0.0;
            const double *row = &A[(size_t)i * n];
            for (int j = k + 1; j < n; ++j) s += row[j] * v[j];
            p[i] = s;
            vAv += v[i] * s;
        }
        for (int i = k + 1; i < n; ++i) u[i] = p[i] - vAv * v[i];
        for (int i = k + 1; i < n; ++i) {
            double *row = &A[(size_t)i * n];
            const double vi = v[i], ui = u[i];
            for (int j = k + 1; j < n; ++j) row[j] -= 2.0 * (vi * u[j] + ui * v[j]);
        }
        at(k + 1, k) = at(k, k + 1) = alpha;
        for (int i = k + 2; i < n; ++i) at(i, k) = at(k, i) = 0.0;
        // Q <- Q P, i.e. Z <- P Z on rows k + 1 ..
        std::fill(t.begin(), t.end(), 0.0);
        for (int j = k + 1; j < n; ++j) {
            const double vj = v[j];
            const double *row = &Z[(size_t)j * n];
            for (int r = 0; r < n; ++r) t[r] += row[r] * vj;
        }
        for (int j = k + 1; j < n; ++j) {
            const double vj = 2.0 * v[j];
            double *row = &Z[(size_t)j * n];
            for (int r = 0; r < n; ++r) row[r] -= vj * t[r];
        }
    }
    // tridiagonal T: diagonal d, coupling e[i] between i and i + 1
    std::vector<double> d(n), e(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = at(i, i);
    for (int i = 0; i + 1 < n; ++i) e[i] = at(i + 1, i);

    // ---- implicit QL --------------------------------------------------------
    const double eps = std::numeric_limits<double>::epsilon();
    for (int l = 0; l < n; ++l) {
        for (int iter = 0;; ++iter) {
            int m = l;
            for (; m + 1 < n; ++m)
                if (std::fabs(e[m]) <= eps * (std::fabs(d[m]) + std::fabs(d[m + 1]))) break;
            if (m == l) break;
            if (iter > 100) throw std::runtime_error("eigensolver did not converge");
            // shift: the eigenvalue of the leading 2 x 2 block nearer d[l]
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, shift = 0.0;
            bool deflated = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {  // underflow: split the matrix here and restart
                    d[i + 1] -= shift;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - shift;
                r = (d[i] - g) * s + 2.0 * c * b;
                shift = s * r;
                d[i + 1] = g + shift;
                g = c * r - b;
                double *zi = &Z[(size_t)i * n], *zi1 = &Z[(size_t)(i + 1) * n];
                for (int k = 0; k < n; ++k) {
                    const double a0 = zi[k], a1 = zi1[k];
                    zi1[k] = s * a0 + c * a1;
                    zi[k] = c * a0 - s * a1;
                }
            }
            if (deflated) continue;
            d[l] -= shift;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    // ---- ascending order ----------------------------------------------------
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] < d[b]; });
    w.resize(n);
    for (int k = 0; k < n; ++k) {
        w[k] = d[ord[k]];
        for (int r = 0; r < n; ++r) A[(size_t)r * n + k] = Z[(size_t)ord[k] * n + r];
    }
}

}  // namespace pd

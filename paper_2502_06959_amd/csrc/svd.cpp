// Complex one-sided Jacobi SVD in FP64 (Hestenes' method): the columns of a
// copy of A are rotated pairwise until they are mutually orthogonal; their
// norms are then the singular values and the accumulated rotations give V.
// Used for the operator-Schmidt decomposition of block operators (Sec. IV-A).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace hsf {

namespace {

// Tall case (m >= n): A (row-major m x n) = U diag(s) V^H with U m x n.
void jacobi_tall(int m, int n, const std::vector<cd>& A, std::vector<cd>& U,
                 std::vector<double>& s, std::vector<cd>& V) {
    std::vector<cd> a((size_t)m * n);         // column-major working copy
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) a[(size_t)j * m + i] = A[(size_t)i * n + j];
    V.assign((size_t)n * n, cd(0));           // column-major
    for (int j = 0; j < n; ++j) V[(size_t)j * n + j] = 1.0;

    const double eps = 1e-15;
    // squared column norms, kept current through the rotations
    std::vector<double> n2(n);
    auto col_norm2 = [&](int j) {
        double acc = 0;
        for (int r = 0; r < m; ++r) acc += std::norm(a[(size_t)j * m + r]);
        return acc;
    };
    for (int sweep = 0; sweep < 80; ++sweep) {
        bool rotated = false;
        double top = 0;
        for (int j = 0; j < n; ++j) top = std::max(top, n2[j] = col_norm2(j));
        // a column below 1e-16 of the largest holds a singular value far
        // under any rank tolerance, and rotating it against another changes
        // that one by less than rounding: such pairs are left alone (a block
        // operator of Schmidt rank r has all but r columns go to zero)
        const double tiny = top * 1e-32;
        for (int i = 0; i < n - 1; ++i) {
            cd* ci = &a[(size_t)i * m];
            for (int j = i + 1; j < n; ++j) {
                if (n2[i] <= tiny || n2[j] <= tiny) continue;
                cd* cj = &a[(size_t)j * m];
                const double alpha = n2[i], beta = n2[j];
                cd gamma = 0;
                for (int r = 0; r < m; ++r) gamma += std::conj(ci[r]) * cj[r];
                const double g = std::abs(gamma);
                if (g == 0.0 || g <= eps * std::sqrt(alpha * beta)) continue;
                rotated = true;
                // make the inner product real: c_j <- c_j e^{-i phi}
                const cd ph = gamma / g;
                const cd phc = std::conj(ph);
                const double zeta = (beta - alpha) / (2.0 * g);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t);
                const double sn = cs * t;
                for (int r = 0; r < m; ++r) {
                    const cd x = ci[r], y = cj[r] * phc;
                    ci[r] = cs * x - sn * y;
                    cj[r] = sn * x + cs * y;
                }
                n2[i] = col_norm2(i);
                n2[j] = col_norm2(j);
                cd* vi = &V[(size_t)i * n];
                cd* vj = &V[(size_t)j * n];
                for (int r = 0; r < n; ++r) {
                    const cd x = vi[r], y = vj[r] * phc;
                    vi[r] = cs * x - sn * y;
                    vj[r] = sn * x + cs * y;
                }
            }
        }
        if (!rotated) break;
    }
    std::vector<double> nrm(n);
    for (int j = 0; j < n; ++j) {
        double acc = 0;
        for (int r = 0; r < m; ++r) acc += std::norm(a[(size_t)j * m + r]);
        nrm[j] = std::sqrt(acc);
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
    s.resize(n);
    U.assign((size_t)m * n, cd(0));
    std::vector<cd> Vs((size_t)n * n);
    for (int jj = 0; jj < n; ++jj) {
        const int j = ord[jj];
        s[jj] = nrm[j];
        if (nrm[j] > 0)
            for (int r = 0; r < m; ++r) U[(size_t)jj * m + r] = a[(size_t)j * m + r] / nrm[j];
        for (int r = 0; r < n; ++r) Vs[(size_t)jj * n + r] = V[(size_t)j * n + r];
    }
    V.swap(Vs);
}

}  // namespace

void jacobi_svd(int m, int n, const std::vector<cd>& A, std::vector<cd>& W, std::vector<double>& s,
                std::vector<cd>& Vh) {
    const int r = std::min(m, n);
    if (m >= n) {
        std::vector<cd> U, V;
        jacobi_tall(m, n, A, U, s, V);
        W = U;                                      // m x n column-major
        Vh.assign((size_t)r * n, cd(0));
        for (int k = 0; k < r; ++k)
            for (int c = 0; c < n; ++c) Vh[(size_t)k * n + c] = std::conj(V[(size_t)k * n + c]);
    } else {
        // A^H (n x m, tall) = U' S V'^H  =>  A = V' S U'^H
        std::vector<cd> AH((size_t)n * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) AH[(size_t)j * m + i] = std::conj(A[(size_t)i * n + j]);
        std::vector<cd> U, V;
        jacobi_tall(n, m, AH, U, s, V);             // U: n x m col-major, V: m x m col-major
        W = V;                                      // m x m column-major
        Vh.assign((size_t)r * n, cd(0));
        for (int k = 0; k < r; ++k)
            for (int c = 0; c < n; ++c) Vh[(size_t)k * n + c] = std::conj(U[(size_t)k * n + c]);
    }
}

}  // namespace hsf

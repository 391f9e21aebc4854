// 1-D reference-element operators on [-1, 1] for the LGL collocation of the
// dGSEM (section 2.2) and the L2 projections used by mortars and by the
// conservative transfer (section 3.3: projection matrices built once on the
// reference element from the mass matrix M and the mixed mass matrix S, reverse
// projection scaled by s = 1/2 for a 2:1 tree).  Computed in long double, stored
// as double.
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace dgamr {
namespace {

using ld = long double;

// Legendre P_n(x) and P_{n-1}(x) by the three-term recurrence.
void legendre_pair(int n, ld x, ld& pn, ld& pnm1) {
    ld p0 = 1.0L, p1 = x;
    if (n == 0) { pn = 1.0L; pnm1 = 0.0L; return; }
    for (int k = 1; k < n; ++k) {
        ld p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
    }
    pn = p1;
    pnm1 = p0;
}

ld legendre(int n, ld x) {
    ld a, b;
    legendre_pair(n, x, a, b);
    return a;
}

// LGL nodes are the roots of P_{N+1} - P_{N-1} (a multiple of (x^2 - 1) P_N');
// its derivative is (2N+1) P_N.
void lgl(int N, std::vector<ld>& x, std::vector<ld>& w) {
    const ld pi = 3.141592653589793238462643383279502884L;
    x.assign(N + 1, 0.0L);
    w.assign(N + 1, 0.0L);
    for (int j = 0; j <= N; ++j) {
        ld t = -std::cos(pi * j / N);
        for (int it = 0; it < 200; ++it) {
            ld f = legendre(N + 1, t) - legendre(N - 1, t);
            ld fp = (2 * N + 1) * legendre(N, t);
            ld dt = f / fp;
            t -= dt;
            if (std::fabs(dt) < 1e-19L) break;
        }
        x[j] = t;
    }
    x[0] = -1.0L;
    x[N] = 1.0L;
    for (int j = 0; j <= N / 2; ++j) {  // exact symmetry
        ld s = 0.5L * (x[N - j] - x[j]);
        x[N - j] = s;
        x[j] = -s;
    }
    if (N % 2 == 0) x[N / 2] = 0.0L;
    for (int j = 0; j <= N; ++j) {
        ld p = legendre(N, x[j]);
        w[j] = 2.0L / (N * (N + 1) * p * p);
    }
}

// Gauss-Legendre rule with n points (exact to degree 2n-1).
void gauss(int n, std::vector<ld>& g, std::vector<ld>& wg) {
    const ld pi = 3.141592653589793238462643383279502884L;
    g.assign(n, 0.0L);
    wg.assign(n, 0.0L);
    for (int i = 0; i < n; ++i) {
        ld t = -std::cos(pi * (i + 0.75L) / (n + 0.5L));
        ld pn = 0, pnm1 = 0;
        for (int it = 0; it < 200; ++it) {
            legendre_pair(n, t, pn, pnm1);
            ld dp = n * (t * pn - pnm1) / (t * t - 1.0L);
            ld dt = pn / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-19L) break;
        }
        legendre_pair(n, t, pn, pnm1);
        ld dp = n * (t * pn - pnm1) / (t * t - 1.0L);
        g[i] = t;
        wg[i] = 2.0L / ((1.0L - t * t) * dp * dp);
    }
}

std::vector<ld> bary_weights(const std::vector<ld>& x) {
    int n = (int)x.size();
    std::vector<ld> lam(n, 1.0L);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k)
            if (k != j) lam[j] /= (x[j] - x[k]);
    return lam;
}

// row of Lagrange basis values l_j(y), j = 0..N (barycentric, second form)
void lagrange_row(const std::vector<ld>& x, const std::vector<ld>& lam, ld y, ld* out) {
    int n = (int)x.size();
    for (int j = 0; j < n; ++j) {
        if (y == x[j]) {
            for (int k = 0; k < n; ++k) out[k] = (k == j) ? 1.0L : 0.0L;
            return;
        }
    }
    ld den = 0.0L;
    for (int j = 0; j < n; ++j) den += lam[j] / (y - x[j]);
    for (int j = 0; j < n; ++j) out[j] = (lam[j] / (y - x[j])) / den;
}

// solve A X = B (n x n, n x m) in place by Gaussian elimination with pivoting
void solve(int n, int m, std::vector<ld> A, std::vector<ld>& B) {
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
        if (p != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[p * n + k]);
            for (int k = 0; k < m; ++k) std::swap(B[c * m + k], B[p * m + k]);
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            ld f = A[r * n + c] / A[c * n + c];
            if (f == 0.0L) continue;
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            for (int k = 0; k < m; ++k) B[r * m + k] -= f * B[c * m + k];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < m; ++k) B[r * m + k] /= A[r * n + r];
}

}  // namespace

RefOps make_refops(int N) {
    const int n = N + 1;
    std::vector<ld> x, w;
    lgl(N, x, w);
    std::vector<ld> lam = bary_weights(x);

    std::vector<ld> D(n * n, 0.0L);
    for (int i = 0; i < n; ++i) {
        ld s = 0.0L;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            D[i * n + j] = (lam[j] / lam[i]) / (x[i] - x[j]);
            s += D[i * n + j];
        }
        D[i * n + i] = -s;
    }

    std::vector<ld> I[2];
    for (int a = 0; a < 2; ++a) {
        I[a].assign(n * n, 0.0L);
        for (int m = 0; m < n; ++m) lagrange_row(x, lam, (x[m] + (2 * a - 1)) / 2.0L, &I[a][m * n]);
    }

    // exact mass matrix M[j][k] = int l_j l_k (Gauss-Legendre, N+2 points)
    std::vector<ld> g, wg;
    gauss(N + 2, g, wg);
    std::vector<ld> M(n * n, 0.0L), row(n);
    for (size_t q = 0; q < g.size(); ++q) {
        lagrange_row(x, lam, g[q], row.data());
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) M[j * n + k] += wg[q] * row[j] * row[k];
    }

    // R_a = 1/2 M^{-1} I_a^T M
    std::vector<ld> R[2];
    for (int a = 0; a < 2; ++a) {
        std::vector<ld> B(n * n, 0.0L);
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                ld s = 0.0L;
                for (int m = 0; m < n; ++m) s += I[a][m * n + j] * M[m * n + k];
                B[j * n + k] = 0.5L * s;
            }
        solve(n, n, M, B);
        R[a] = B;
    }

    // P_a[m][j] = c_a(m) l_j(2 x_m - (2a - 1)) (pointwise matching, section 3.3):
    // half a's polynomial at the parent's node m, c_a = 1 inside half a, 1/2 on the
    // shared mid-point (even N), 0 in the other half
    std::vector<ld> P[2];
    for (int a = 0; a < 2; ++a) {
        P[a].assign(n * n, 0.0L);
        for (int m = 0; m < n; ++m) {
            const bool mid = std::fabs(x[m]) < 1e-12L;
            const bool inside = mid || (a == 0 ? x[m] < 0.0L : x[m] > 0.0L);
            if (!inside) continue;
            lagrange_row(x, lam, 2.0L * x[m] - (2 * a - 1), &P[a][m * n]);
            if (mid)
                for (int j = 0; j < n; ++j) P[a][m * n + j] *= 0.5L;
        }
    }

    RefOps o;
    o.N = N;
    auto cvt = [](const std::vector<ld>& v) { return std::vector<double>(v.begin(), v.end()); };
    o.x = cvt(x);
    o.w = cvt(w);
    o.D = cvt(D);
    o.I0 = cvt(I[0]);
    o.I1 = cvt(I[1]);
    o.R0 = cvt(R[0]);
    o.R1 = cvt(R[1]);
    o.P0 = cvt(P[0]);
    o.P1 = cvt(P[1]);
    return o;
}

}  // namespace dgamr

// Host tables of the Chebyshev fiber representation (section "Fiber
// representation"), built in long double and rounded once to double.
//
// Values at the n = p + 1 CGL nodes alpha_k = cos(k pi / p) map to the
// coefficients of the Chebyshev series (eq. cheb-basis) by the discrete cosine
// transform C; differentiation acts on the coefficients by the recursion
// c'_{j-1} = c'_{j+1} + 2 j c_j (c'_p = c'_{p+1} = 0, c'_0 halved); E evaluates a
// series at the nodes.  D^(k) = E R^k C is the k-th alpha-derivative on node
// values.  Resampling to the m first-kind points y_j = cos((2 j + 1) pi / (2 m))
// evaluates the series there.  All matrices are row-major.
#pragma once

#include <cmath>
#include <vector>

namespace stokes {
namespace cheb {

using ld = long double;
constexpr ld PI_L = 3.141592653589793238462643383279502884L;

// cos(a pi / b) for integers, reduced mod 2b first.
inline ld cos_frac(long a, long b) {
    a %= 2 * b;
    if (a < 0) a += 2 * b;
    return cosl(PI_L * (ld)a / (ld)b);
}

struct Tables {
    int n = 0;
    std::vector<double> D1, D2, D3, D4;   // n x n
    std::vector<double> P4, P2;           // (n - 4) x n, (n - 2) x n
};

inline Tables build(int n) {
    const int p = n - 1;
    std::vector<ld> C((size_t)n * n), Ev((size_t)n * n), R((size_t)n * n, 0.0L);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
            const ld wk = (k == 0 || k == p) ? 0.5L : 1.0L;
            const ld gj = (j == 0 || j == p) ? 0.5L : 1.0L;
            C[(size_t)j * n + k] = 2.0L / p * wk * gj * cos_frac((long)j * k, p);
            Ev[(size_t)k * n + j] = cos_frac((long)j * k, p);      // T_j(alpha_k)
        }
    // R: coefficients of the derivative from those of the series, column by column
    std::vector<ld> c(n), d(n + 2);
    for (int col = 0; col < n; ++col) {
        for (int j = 0; j < n; ++j) c[j] = j == col ? 1.0L : 0.0L;
        std::fill(d.begin(), d.end(), 0.0L);
        for (int j = p; j >= 1; --j) d[j - 1] = d[j + 1] + 2.0L * j * c[j];
        d[0] *= 0.5L;
        for (int j = 0; j < n; ++j) R[(size_t)j * n + col] = d[j];
    }
    auto mul = [n](const std::vector<ld>& A, const std::vector<ld>& B, int rows) {
        std::vector<ld> O((size_t)rows * n, 0.0L);
        for (int i = 0; i < rows; ++i)
            for (int k = 0; k < n; ++k) {
                const ld a = A[(size_t)i * n + k];
                if (a == 0.0L) continue;
                for (int j = 0; j < n; ++j) O[(size_t)i * n + j] += a * B[(size_t)k * n + j];
            }
        return O;
    };
    auto to_d = [](const std::vector<ld>& A) { return std::vector<double>(A.begin(), A.end()); };
    Tables t;
    t.n = n;
    std::vector<ld> RC = mul(R, C, n);           // first-derivative coefficients
    t.D1 = to_d(mul(Ev, RC, n));
    RC = mul(R, RC, n);
    t.D2 = to_d(mul(Ev, RC, n));
    RC = mul(R, RC, n);
    t.D3 = to_d(mul(Ev, RC, n));
    RC = mul(R, RC, n);
    t.D4 = to_d(mul(Ev, RC, n));
    for (int m : {n - 4, n - 2}) {
        std::vector<ld> Ty((size_t)m * n);
        for (int j = 0; j < m; ++j)
            for (int l = 0; l < n; ++l) Ty[(size_t)j * n + l] = cos_frac((long)l * (2 * j + 1), 2L * m);
        (m == n - 4 ? t.P4 : t.P2) = to_d(mul(Ty, C, m));
    }
    return t;
}

}  // namespace cheb
}  // namespace stokes

// Device helpers shared by the kernels of the DG-AMR library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "kernels.hpp"

namespace dgamr {
namespace dev {

constexpr int kXcd = 8;  // MI355X: 8 XCDs, workgroups dispatched round-robin

// Give each XCD a contiguous range of leaves (Morton order keeps face
// neighbours close), so neighbour traces are mostly L2 hits on that XCD.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblk) {
    const int64_t q = nblk / kXcd, r = nblk % kXcd;
    const int64_t x = bid % kXcd, i = bid / kXcd;
    return x * q + (x < r ? x : r) + i;
}

template <int N>
struct Sz {
    static constexpr int N1 = N + 1;
    static constexpr int NP = N1 * N1 * N1;
    static constexpr int NF = N1 * N1;
    static constexpr int NT = ((NP + 63) / 64) * 64;   // one thread per node
    static constexpr int NOPS = 5 * NF + N1;           // D, I0, I1, R0, R1, w
};

// element node of face f = 2d + s at face-local index m = a + (N+1) b, with
// (a, b) along the tangential axes in increasing axis order
template <int N>
__device__ __forceinline__ int face_node(int f, int m) {
    constexpr int N1 = N + 1;
    const int d = f >> 1, idx = (f & 1) ? N : 0;
    const int a = m % N1, b = m / N1;
    if (d == 0) return idx + N1 * (a + N1 * b);
    if (d == 1) return a + N1 * (idx + N1 * b);
    return a + N1 * (b + N1 * idx);
}

// k (z index) of that node, which selects the background value
template <int N>
__device__ __forceinline__ int face_k(int f, int m) {
    const int d = f >> 1;
    if (d == 2) return (f & 1) ? N : 0;
    return m / (N + 1);
}

// P' = P(Thetabar + Theta') - Pbar = Pbar F(x), F(x) = (1 + x)^gamma - 1, x = Theta'/Thetabar,
// without cancellation: for |x| <= 2^-7 the binomial series sum_{k=1..7} C(gamma,k) x^k
// (Horner; truncation below 1e-17 relative for 1 < gamma < 2).  A larger |x| is first brought into that
// range by halving log(1 + x): 1 + x = (1 + y)^2 with y = x / (1 + sqrt(1 + x)) (no
// cancellation), repeated until |y| <= 2^-7, and F is rebuilt by F(x) = F(y) (F(y) + 2)
// once per halving.  Only the series coefficients are needed (no special-function
// constants, no call), so the rare wide-range path costs the kernels no registers.

// x = Theta' (1/Thetabar): every kernel forms 1/Thetabar by the same IEEE division,
// so a node's P' has the same bits wherever it is evaluated
__device__ __forceinline__ double binom_series(double x, const BinomCoef& bc) {
    double acc = bc.c[kBinomTerms - 1];
#pragma unroll
    for (int k = kBinomTerms - 2; k >= 0; --k) acc = fma(acc, x, bc.c[k]);
    return acc * x;
}

__device__ __forceinline__ double pprime(double Thp, double rThb, double Pb, double gamma, const BinomCoef& bc) {
    const double x = Thp * rThb;
    double r = binom_series(x, bc);
    if (__builtin_expect(!(fabs(x) <= 0.0078125), 0)) {
        // every step halves |log(1 + y)|; NaN (and y <= -1) leave the loop at once
        double y = x;
        int m = 0;
        while (fabs(y) > 0.0078125 && m < 64) {
            y = y / (1.0 + sqrt(1.0 + y));
            ++m;
        }
        r = binom_series(y, bc);
        for (; m > 0; --m) r = r * (r + 2.0);
    }
    return Pb * r;
}

// 1/x for a positive normal x: the hardware reciprocal estimate refined by two
// Newton steps (within about one ulp; the same bits for the same input), instead
// of the scaled, correctly rounded division sequence
__device__ __forceinline__ double rcp_pos(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// sqrt(a) for a positive normal a: reciprocal square-root estimate, one coupled
// Newton step on (g, h) ~ (sqrt a, 1/(2 sqrt a)), two residual corrections (no
// range scaling or special-value handling)
__device__ __forceinline__ double sqrt_pos(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, a);
    g = fma(d, h, g);
    d = fma(-g, g, a);
    return fma(d, h, g);
}

// background at a node: density, Theta, pressure and 1/Theta
struct Bg {
    double rho, Th, P, rTh;
};

__device__ __forceinline__ Bg bg_make(double rho, double Th, double P) { return Bg{rho, Th, P, 1.0 / Th}; }

// a double at a 32-bit byte offset from a wave-uniform base: one global load with
// a scalar base and a 32-bit vector offset, no 64-bit address arithmetic
__device__ __forceinline__ double ld_off(const double* base, uint32_t byte_off) {
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + byte_off);
}

// call body.template operator()<D>() with D the run-time axis d
template <typename Body>
__device__ __forceinline__ void with_axis(int d, Body&& body) {
    if (d == 0)
        body(std::integral_constant<int, 0>{});
    else if (d == 1)
        body(std::integral_constant<int, 1>{});
    else
        body(std::integral_constant<int, 2>{});
}

// (A x B) applied to a face trace T[(N+1)^2] at face node m (A along the first
// tangential axis, B along the second)
template <int N>
__device__ __forceinline__ double tensor2(const double* T, const double* A, const double* B, int m) {
    constexpr int N1 = N + 1;
    const int m1 = m % N1, m2 = m / N1;
    double acc = 0.0;
#pragma unroll 1
    for (int j2 = 0; j2 < N1; ++j2) {
        double row = 0.0;
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1) row = fma(A[m1 * N1 + j1], T[j2 * N1 + j1], row);
        acc = fma(B[m2 * N1 + j2], row, acc);
    }
    return acc;
}

// Block-level separable tensor products on face data laid out [plane][b][a]
// ((N+1)^2 values per plane, a along the first tangential axis).  Every output
// is an fma chain in a fixed order, so two blocks applying the same operator to
// the same data get bitwise-identical results.
// out[p][b][a'] = sum_a A(p)[a'][a] in[src(p)][b][a]   for planes p < np
template <int N, typename OpA, typename Src>
__device__ __forceinline__ void apply_t1(const double* in, double* out, int np, OpA opA, Src src, int t, int nt) {
    constexpr int N1 = N + 1, NF = N1 * N1;
    for (int it = t; it < np * NF; it += nt) {
        const int p = it / NF, r = it % NF, b = r / N1, a2 = r % N1;
        const double* A = opA(p) + a2 * N1;
        const double* x = in + src(p) * NF + b * N1;
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < N1; ++a) acc = fma(A[a], x[a], acc);
        out[it] = acc;
    }
}
// out[p][b'][a] = sum_b B(p)[b'][b] in[src(p)][b][a]
template <int N, typename OpB, typename Src>
__device__ __forceinline__ void apply_t2(const double* in, double* out, int np, OpB opB, Src src, int t, int nt) {
    constexpr int N1 = N + 1, NF = N1 * N1;
    for (int it = t; it < np * NF; it += nt) {
        const int p = it / NF, r = it % NF, b2 = r / N1, a = r % N1;
        const double* B = opB(p) + b2 * N1;
        const double* x = in + src(p) * NF + a;
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < N1; ++b) acc = fma(B[b], x[b * N1], acc);
        out[it] = acc;
    }
}

// compensated pair (s, c): value s + c
struct Comp {
    double s, c;
};

__device__ __forceinline__ Comp comp_add(Comp x, double y) {
    const double s = x.s + y;
    const double bp = s - x.s;
    const double err = (x.s - (s - bp)) + (y - bp);
    return Comp{s, x.c + err};
}

__device__ __forceinline__ Comp comp_merge(Comp x, Comp y) {
    Comp r = comp_add(x, y.s);
    r.c += y.c;
    return r;
}

// deterministic block reduction of 4 compensated sums; result valid in thread 0
template <int NT>
__device__ void block_reduce4(Comp v[4], Comp* sh /* [4][NT] */) {
    const int t = threadIdx.x;
    for (int q = 0; q < 4; ++q) sh[q * NT + t] = v[q];
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int q = 0; q < 4; ++q) sh[q * NT + t] = comp_merge(sh[q * NT + t], sh[q * NT + t + w]);
        __syncthreads();
    }
    for (int q = 0; q < 4; ++q) v[q] = sh[q * NT];
}

}  // namespace dev
}  // namespace dgamr

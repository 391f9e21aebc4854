// HIP kernels of the artificial viscosity div(mu grad q') (section 4.3: the
// rising bubble runs with mu = 1.5 m^2/s; the form is a reading: constant
// kinematic coefficient on every perturbation variable), discretised with the
// two-pass central scheme: the gradient sigma_d = (2/h_d) D_d q' + lifted
// (q* - q-) n_d with q* the central average, then the divergence
// (2/h_d) D_d (mu sigma_d) + lifted (G* - G-).n with the central flux G*; walls
// add nothing to the gradient and carry no diffusive flux; on hanging faces
// both averages are formed on the mortars (section 3.3) by one generic
// pre-pass.  The divergence is added to the output of the Euler stage kernel
// (the stage is linear in R: out += b dt R_visc).
//
// Compiled with -ffp-contract=off like the Euler kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device_common.hpp"
#include "kernels.hpp"

namespace dgamr {
namespace {

using namespace dev;

// Central averages on the mortars of one hanging face per workgroup: the coarse
// trace of X (5 planes) is interpolated to the four mortars (I_a x I_b), averaged
// with the fine traces there; the fine faces receive lift sgn (X* - X_fine), the
// coarse face lift sgn (sum_ab (R_a x R_b) X*_ab - X_coarse), all times `mul`.
// X is the field of the face's normal axis d: base + d * axis_stride.
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_central_mortar(const CentralMortArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    static_assert(4 * NF <= NT, "one mortar point per thread");
    __shared__ double sT[5 * NF], sU[10 * NF], sMq[20 * NF], sG[10 * NF];
    __shared__ double sOps[Sz<N>::NOPS];
    const int64_t h = xcd_remap(blockIdx.x, gridDim.x);
    const int t = threadIdx.x;
    const int32_t* const row = A.hang + h * 6;
    const int64_t ec = row[0];
    const int f = row[1], fo = f ^ 1, d = f >> 1;
    const int64_t KNP = A.K * NP;
    const double* const X = A.x + (int64_t)d * A.axis_stride;
    const double liftc = 0.5 * N * (N + 1);
    const double sgn = (f & 1) ? 1.0 : -1.0;  // the coarse leaf's outward normal
    for (int ii = t; ii < Sz<N>::NOPS; ii += NT) sOps[ii] = A.ops[ii];
    for (int it = t; it < 5 * NF; it += NT) {
        const int v = it / NF, m = it % NF;
        sT[it] = X[v * KNP + ec * NP + face_node<N>(f, m)];
    }
    double xF[5] = {0, 0, 0, 0, 0};
    double lift_f = 0.0;
    const double lift_c = A.geo[ec * 4 + d] * liftc;
    if (t < 4 * NF) {
        const int quad = t / NF, m = t % NF;
        const int64_t ef = row[2 + quad];
        const int nn = face_node<N>(fo, m);
#pragma unroll
        for (int v = 0; v < 5; ++v) xF[v] = X[v * KNP + ef * NP + nn];
        lift_f = A.geo[ef * 4 + d] * liftc;
    }
    __syncthreads();
    apply_t1<N>(sT, sU, 10, [&](int p) { return sOps + (1 + p / 5) * NF; }, [](int p) { return p % 5; }, t, NT);
    __syncthreads();
    apply_t2<N>(sU, sMq, 20, [&](int p) { return sOps + (1 + (p / 5) / 2) * NF; },
                [](int p) { return ((p / 5) & 1) * 5 + p % 5; }, t, NT);
    __syncthreads();
    if (t < 4 * NF) {
        const int quad = t / NF, m = t % NF;
        double* const out = A.out + ((h * 5 + 1 + quad) * 5) * NF + m;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double avg = 0.5 * (sMq[(quad * 5 + v) * NF + m] + xF[v]);
            out[v * NF] = A.mul * (lift_f * (-sgn) * (avg - xF[v]));  // the fine side's normal is -n_c
            sMq[(quad * 5 + v) * NF + m] = avg;
        }
    }
    __syncthreads();
    for (int it = t; it < 10 * NF; it += NT) {
        const int p = it / NF, r = it % NF, bb = r / N1, a2 = r % N1;
        const int qb = p / 5, v = p % 5;
        double acc = 0.0;
#pragma unroll
        for (int qa = 0; qa < 2; ++qa) {
            const double* Rm = sOps + (3 + qa) * NF + a2 * N1;
            const double* x = sMq + ((qa + 2 * qb) * 5 + v) * NF + bb * N1;
#pragma unroll
            for (int a = 0; a < N1; ++a) acc = fma(Rm[a], x[a], acc);
        }
        sG[it] = acc;
    }
    __syncthreads();
    for (int it = t; it < 5 * NF; it += NT) {
        const int v = it / NF, m = it % NF, b2 = m / N1, a = m % N1;
        double proj = 0.0;
#pragma unroll
        for (int qb = 0; qb < 2; ++qb) {
            const double* Rm = sOps + (3 + qb) * NF + b2 * N1;
            const double* x = sG + (qb * 5 + v) * NF + a;
#pragma unroll
            for (int bb = 0; bb < N1; ++bb) proj = fma(Rm[bb], x[bb * N1], proj);
        }
        A.out[((h * 5) * 5 + v) * NF + m] = A.mul * (lift_c * sgn * (proj - sT[it]));
    }
}

// lifted central face terms of one leaf for the field X of axis d (the faces 2d,
// 2d + 1): conforming lift sgn mul (X+ - X-)/2, walls 0 (gradient) or
// -lift sgn mul X- (zero flux), hanging faces from the pre-pass
template <int N>
__device__ __forceinline__ void central_faces(const double* X, int64_t KNP, int64_t e, const int32_t* rec,
                                              const double* mort, const double* sX, int d, double lift, double mul,
                                              bool wall_zero_flux, double* sS /* [2][5][NF] */, int t, int nt) {
    constexpr int NP = Sz<N>::NP, NF = Sz<N>::NF;
    for (int it = t; it < 10 * NF; it += nt) {
        const int side = it / (5 * NF), r = it % (5 * NF), v = r / NF, m = r % NF;
        const int f = 2 * d + side;
        const int tf = rec[f], type = tf & 0xff;
        const double sgn = side ? 1.0 : -1.0;
        double val;
        if (type == FT_FINE || type == FT_COARSE) {
            const int64_t row = (int64_t)rec[12 + f] * 5 + (type == FT_COARSE ? 0 : 1 + ((tf >> 8) & 0xff));
            val = mort[(row * 5 + v) * NF + m];
        } else {
            const double xm = sX[v * NP + face_node<N>(f, m)];
            if (type == FT_WALL) {
                val = wall_zero_flux ? lift * sgn * (mul * (0.0 - xm)) : 0.0;
            } else {
                const double xp = X[v * KNP + (int64_t)rec[6 + f] * NP + face_node<N>(f ^ 1, m)];
                val = lift * sgn * (mul * (0.5 * (xm + xp) - xm));
            }
        }
        sS[it] = val;
    }
}

// sigma_d = (2/h_d) D_d q + lifted (q* - q-) n_d, d = 0..2, written to sigma [3][5][K][Np]
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_visc_grad(const ViscArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    __shared__ double sX[5 * NP];
    __shared__ double sS[10 * NF];
    __shared__ double sD[N1 * N1];
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t* const rec = A.srec + e * kStageRec;
    const int t = threadIdx.x;
    const int64_t KNP = A.K * NP;
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;
    const double liftc = 0.5 * N * (N + 1);
    for (int ii = t; ii < N1 * N1; ii += NT) sD[ii] = A.ops[ii];
    if (t < NP)
#pragma unroll
        for (int v = 0; v < 5; ++v) sX[v * NP + t] = A.q[v * KNP + e * NP + t];
    __syncthreads();
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        const double g2 = A.geo[e * 4 + d];
        if (d > 0) __syncthreads();
        central_faces<N>(A.q, KNP, e, rec, A.mort, sX, d, g2 * liftc, 1.0, false,
                         sS, t, NT);
        __syncthreads();
        if (t < NP) {
            const int id = d == 0 ? i : d == 1 ? j : k;
            const int stride = d == 0 ? 1 : d == 1 ? N1 : NF;
            const int side = id == N ? 1 : 0;
            const int fm = d == 0 ? j + N1 * k : d == 1 ? i + N1 * k : i + N1 * j;
            const bool on = id == 0 || id == N;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double* Xp = sX + v * NP + (t - id * stride);
                double acc = 0.0;
#pragma unroll
                for (int mm = 0; mm < N1; ++mm) acc = fma(sD[id * N1 + mm], Xp[mm * stride], acc);
                double s = g2 * acc;
                if (on) s += sS[(side * 5 + v) * NF + fm];
                A.sigma[((int64_t)d * 5 + v) * KNP + e * NP + t] = s;
            }
        }
    }
}

// out += scale R_visc, R_visc = sum_d (2/h_d) D_d (mu sigma_d) + lifted (G* - G-).n
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_visc_div(const ViscArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    __shared__ double sX[5 * NP];
    __shared__ double sS[10 * NF];
    __shared__ double sD[N1 * N1];
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t* const rec = A.srec + e * kStageRec;
    const int t = threadIdx.x;
    const int64_t KNP = A.K * NP;
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;
    const double liftc = 0.5 * N * (N + 1);
    for (int ii = t; ii < N1 * N1; ii += NT) sD[ii] = A.ops[ii];
    double R[5] = {0, 0, 0, 0, 0};
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        const double g2 = A.geo[e * 4 + d];
        const double* const Sd = A.sigma + (int64_t)d * 5 * KNP;
        if (d > 0) __syncthreads();
        if (t < NP)
#pragma unroll
            for (int v = 0; v < 5; ++v) sX[v * NP + t] = Sd[v * KNP + e * NP + t];
        __syncthreads();
        central_faces<N>(Sd, KNP, e, rec, A.mort, sX, d, g2 * liftc, A.mu, true,
                         sS, t, NT);
        __syncthreads();
        if (t < NP) {
            const int id = d == 0 ? i : d == 1 ? j : k;
            const int stride = d == 0 ? 1 : d == 1 ? N1 : NF;
            const int side = id == N ? 1 : 0;
            const int fm = d == 0 ? j + N1 * k : d == 1 ? i + N1 * k : i + N1 * j;
            const bool on = id == 0 || id == N;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double* Xp = sX + v * NP + (t - id * stride);
                double acc = 0.0;
#pragma unroll
                for (int mm = 0; mm < N1; ++mm) acc = fma(sD[id * N1 + mm], Xp[mm * stride], acc);
                R[v] = fma(g2, A.mu * acc, R[v]);
                if (on) R[v] += sS[(side * 5 + v) * NF + fm];
            }
        }
    }
    if (t >= NP) return;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        double* const o = A.out + v * KNP + e * NP + t;
        *o = fma(A.scale, R[v], *o);
    }
}

}  // namespace

#define DG_DISPATCH_N(N_, CALL)                                     \
    switch (N_) {                                                   \
        case 2: { constexpr int NN = 2; CALL; } break;              \
        case 3: { constexpr int NN = 3; CALL; } break;              \
        case 4: { constexpr int NN = 4; CALL; } break;              \
        case 5: { constexpr int NN = 5; CALL; } break;              \
        case 6: { constexpr int NN = 6; CALL; } break;              \
        case 7: { constexpr int NN = 7; CALL; } break;              \
        default: return hipErrorInvalidValue;                        \
    }

hipError_t launch_viscous(int N, const ViscArgs& a, hipStream_t s) {
    if (a.K <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.K);
    // pass 1: central averages of q on the mortars (one table per axis), then sigma
    if (a.n_hang > 0) {
        CentralMortArgs m{a.q, 0, a.mort, a.ops, a.geo, a.hang, a.n_hang, a.K, 1.0};
        DG_DISPATCH_N(N, (k_central_mortar<NN><<<dim3((unsigned)a.n_hang), dim3(Sz<NN>::NT), 0, s>>>(m)));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    DG_DISPATCH_N(N, (k_visc_grad<NN><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // pass 2: central fluxes of mu sigma_d on the mortars, then the divergence
    if (a.n_hang > 0) {
        const int64_t np = (int64_t)(N + 1) * (N + 1) * (N + 1);
        CentralMortArgs m{a.sigma, 5 * a.K * np, a.mort, a.ops, a.geo, a.hang, a.n_hang, a.K, a.mu};
        DG_DISPATCH_N(N, (k_central_mortar<NN><<<dim3((unsigned)a.n_hang), dim3(Sz<NN>::NT), 0, s>>>(m)));
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    DG_DISPATCH_N(N, (k_visc_div<NN><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
    return hipGetLastError();
}

}  // namespace dgamr

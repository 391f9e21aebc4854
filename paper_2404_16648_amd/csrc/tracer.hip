// HIP kernels of the passive tracer (section 2.1: C = rho c obeys
// dC/dt + div(C u) = 0 with u = U / rho from the Euler state) on the same
// meshes, faces and mortars as the Euler operator.
//
// One workgroup per leaf, as for the Euler stage: the leaf's Euler state and
// tracer are staged in LDS, every conforming or wall face node solves the
// tracer part of the Rusanov flux (the Euler system's local maximum wave speed,
// the jump of C) and stores its lifted contribution, hanging faces take theirs
// from a pre-pass (one workgroup per hanging face: mortars, or pointwise
// matching), then the volume term -(2/h_d) D_d (C u_d), the lift and the
// Shu-Osher update.  Each conforming face is evaluated by both leaves with
// mirrored arithmetic (the lifted values are exact negatives of each other), so
// the tracer integral is conserved to round-off with mortars.
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

// The tracer flux along e_D needs three of the five Euler variables: rho', the
// momentum U_D and Theta' (through P').  They are passed as scalars, the momentum
// picked by a select on the axis, so no state array is ever indexed by a run-time
// axis (such an index puts the array in scratch memory).
struct TrState {
    double rho, m, Thp;  // rho', U_D, Theta'
};

// the state's entries for axis d
__device__ __forceinline__ TrState tr_state(double rho, double mx, double my, double mz, double Thp, int d) {
    return TrState{rho, d == 0 ? mx : d == 1 ? my : mz, Thp};
}

// wave speed |u_D| + c of a full state (perturbation about bg) and u_D
__device__ __forceinline__ void speed_u(const TrState& q, const Bg& bg, double Pp, double gamma, double& lam,
                                        double& ud) {
    const double rinv = rcp_pos(bg.rho + q.rho);
    ud = q.m * rinv;
    lam = fabs(ud) + sqrt_pos(gamma * (bg.P + Pp) * rinv);
}

// lifted tracer surface term of the leaf on the L side of a face with outward
// normal sgn e_D: lift (1/2 sgn (C_R u_R - C_L u_L) + 1/2 lambda (C_L - C_R)),
// i.e. lift (F*_C - F_C(L)).n for the Rusanov flux, with the L side's u_D and wave
// speed lL already formed (the stage kernel forms them once per node, with the
// expressions of speed_u)
__device__ __forceinline__ double tracer_lifted(double uL, double lL, double CL, const TrState& qR, double CR,
                                                const Bg& bR, double PpR, double sgn, double gamma, double lift) {
    double lR, uR;
    speed_u(qR, bR, PpR, gamma, lR, uR);
    const double c1 = 0.5 * sgn * lift, c2 = 0.5 * fmax(lL, lR) * lift;
    return fma(c1, CR * uR - CL * uL, c2 * (CL - CR));
}

// F*_C . n for n = sgn e_D (the flux itself, for the mortars) and the L side's own C u.n
__device__ __forceinline__ void tracer_rusanov(const TrState& qL, double CL, const Bg& bL, double PpL,
                                               const TrState& qR, double CR, const Bg& bR, double PpR, double sgn,
                                               double gamma, double& Fs, double& FL) {
    double lL, lR, uL, uR;
    speed_u(qL, bL, PpL, gamma, lL, uL);
    speed_u(qR, bR, PpR, gamma, lR, uR);
    FL = sgn * (CL * uL);
    const double FR = sgn * (CR * uR);
    Fs = 0.5 * (FL + FR) + 0.5 * fmax(lL, lR) * (CL - CR);
}

// Tracer mortar pre-pass (section 3.3's three steps for the tracer flux): the
// coarse trace of the Euler state and of C is interpolated to the four mortars
// (I_a x I_b), the tracer's Rusanov flux is solved at each mortar point from the
// fine side, and the coarse side receives that flux with the sign reversed,
// projected back with R_a x R_b.  PW: the coarse side instead solves at its own
// face nodes against the fine polynomials there (P_a x P_b).  Output per hanging
// face h, lifted: mortC[h][0] the coarse face, mortC[h][1 + quad] the fine
// faces, each [NF].
template <int N, bool PW>
__global__ void __launch_bounds__(Sz<N>::NT) k_tracer_mortar(const TracerMortArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    static_assert(4 * NF <= NT, "one mortar point per thread");
    constexpr int PWOFF = Sz<N>::NOPS;  // P0, P1 after D, I0, I1, R0, R1, w (PW)
    // planes: 0..4 the Euler state, 5 the tracer
    __shared__ double sT[6 * NF], sU[12 * NF], sMq[24 * NF], sG[12 * NF];
    __shared__ double sOps[Sz<N>::NOPS + (PW ? 2 * NF : 0)];
    __shared__ double sBg[3 * N1];
    const int64_t h = xcd_remap(blockIdx.x, gridDim.x);
    const int t = threadIdx.x;
    const int32_t* const row = A.hang + h * 6;
    const int64_t ec = row[0];
    const int f = row[1], fo = f ^ 1;
    const int64_t KNP = A.K * NP, KN1 = A.K * N1;
    const double gamma = A.gamma;
    const double liftc = 0.5 * N * (N + 1);
    const double sgn = (f & 1) ? 1.0 : -1.0;  // the coarse leaf's outward normal
    for (int ii = t; ii < Sz<N>::NOPS; ii += NT) sOps[ii] = A.ops[ii];
    if (PW)
        for (int ii = t; ii < 2 * NF; ii += NT) sOps[PWOFF + ii] = A.ops[Sz<N>::NOPS + 4 * NF + ii];
    if (t < 3 * N1) sBg[t] = A.bg[(t / N1) * KN1 + ec * N1 + (t % N1)];
    for (int it = t; it < 6 * NF; it += NT) {
        const int v = it / NF, m = it % NF;
        const int64_t node = ec * NP + face_node<N>(f, m);
        sT[it] = v < 5 ? A.qs[v * KNP + node] : A.cs[node];
    }
    double qF[5] = {0, 0, 0, 0, 0}, cF = 0.0;
    Bg bF{1.0, 1.0, 1.0, 1.0};
    double lift_f = 0.0;
    const double lift_c = A.geo[ec * 4 + (f >> 1)] * liftc;
    if (t < 4 * NF) {
        const int quad = t / NF, m = t % NF;
        const int64_t ef = row[2 + quad];
        const int nn = face_node<N>(fo, m), kn = face_k<N>(fo, m);
        bF = bg_make(A.bg[ef * N1 + kn], A.bg[KN1 + ef * N1 + kn], A.bg[2 * KN1 + ef * N1 + kn]);
#pragma unroll
        for (int v = 0; v < 5; ++v) qF[v] = A.qs[v * KNP + ef * NP + nn];
        cF = A.cs[ef * NP + nn];
        lift_f = A.geo[ef * 4 + (f >> 1)] * liftc;
    }
    __syncthreads();
    // sU[a][v] = I_a along t1; sMq[quad][v] = I_b along t2 of sU[a]
    apply_t1<N>(sT, sU, 12, [&](int p) { return sOps + (1 + p / 6) * NF; }, [](int p) { return p % 6; }, t, NT);
    __syncthreads();
    apply_t2<N>(sU, sMq, 24, [&](int p) { return sOps + (1 + (p / 6) / 2) * NF; },
                [](int p) { return ((p / 6) & 1) * 6 + p % 6; }, t, NT);
    __syncthreads();
    if (t < 4 * NF) {
        const int quad = t / NF, m = t % NF;
        double qM[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qM[v] = sMq[(quad * 6 + v) * NF + m];
        const double cM = sMq[(quad * 6 + 5) * NF + m];
        const double PpF = pprime(qF[4], bF.rTh, bF.P, gamma, A.binom);
        const double PpM = pprime(qM[4], bF.rTh, bF.P, gamma, A.binom);
        double Fs = 0.0, Fo = 0.0;
        const int d = f >> 1;
        tracer_rusanov(tr_state(qF[0], qF[1], qF[2], qF[3], qF[4], d), cF, bF, PpF,
                       tr_state(qM[0], qM[1], qM[2], qM[3], qM[4], d), cM, bF, PpM, -sgn, gamma, Fs, Fo);
        A.mortC[(h * 5 + 1 + quad) * NF + m] = (Fs - Fo) * lift_f;
        if (PW) {
#pragma unroll
            for (int v = 0; v < 5; ++v) sMq[(quad * 6 + v) * NF + m] = qF[v];
            sMq[(quad * 6 + 5) * NF + m] = cF;
        } else {
            sMq[(quad * 6 + 5) * NF + m] = -Fs;  // the coarse side's flux, in the tracer plane
        }
    }
    __syncthreads();
    // back to the coarse nodes: first along t1 (sum over a), then t2 (sum over b); mortars
    // project the tracer flux with R, pointwise evaluates the fine state and tracer with P
    constexpr int NPL = PW ? 6 : 1;  // planes carried back
    for (int it = t; it < 2 * NPL * NF; it += NT) {
        const int p = it / NF, r = it % NF, bb = r / N1, a2 = r % N1;
        const int qb = p / NPL, v = PW ? p % NPL : 5;
        double acc = 0.0;
#pragma unroll
        for (int qa = 0; qa < 2; ++qa) {
            const double* Op = sOps + (PW ? PWOFF + qa * NF : (3 + qa) * NF) + a2 * N1;
            const double* x = sMq + ((qa + 2 * qb) * 6 + v) * NF + bb * N1;
#pragma unroll
            for (int a = 0; a < N1; ++a) acc = fma(Op[a], x[a], acc);
        }
        sG[it] = acc;
    }
    __syncthreads();
    for (int it = t; it < NPL * NF; it += NT) {
        const int p = it / NF, m = it % NF, b2 = m / N1, a = m % N1;
        double acc = 0.0;
#pragma unroll
        for (int qb = 0; qb < 2; ++qb) {
            const double* Op = sOps + (PW ? PWOFF + qb * NF : (3 + qb) * NF) + b2 * N1;
            const double* x = sG + (qb * NPL + p) * NF + a;
#pragma unroll
            for (int bb = 0; bb < N1; ++bb) acc = fma(Op[bb], x[bb * N1], acc);
        }
        sU[it] = acc;
    }
    __syncthreads();
    if (t < NF) {
        const int m = t, kk = face_k<N>(f, m);
        const Bg b = bg_make(sBg[kk], sBg[N1 + kk], sBg[2 * N1 + kk]);
        double qL[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qL[v] = sT[v * NF + m];
        const double cL = sT[5 * NF + m];
        const double PpL = pprime(qL[4], b.rTh, b.P, gamma, A.binom);
        const int d = f >> 1;
        const TrState sL = tr_state(qL[0], qL[1], qL[2], qL[3], qL[4], d);
        double Fc = 0.0, Fo = 0.0;
        if constexpr (PW) {
            double qR[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) qR[v] = sU[v * NF + m];
            const double cR = sU[5 * NF + m];
            const double PpR = pprime(qR[4], b.rTh, b.P, gamma, A.binom);
            tracer_rusanov(sL, cL, b, PpL, tr_state(qR[0], qR[1], qR[2], qR[3], qR[4], d), cR, b, PpR, sgn, gamma,
                           Fc, Fo);
        } else {
            double lam, ud;
            speed_u(sL, b, PpL, gamma, lam, ud);
            Fo = sgn * (cL * ud);
            Fc = sU[m];
        }
        A.mortC[(h * 5) * NF + m] = (Fc - Fo) * lift_c;
    }
}

// Tracer stage: out = R_C (MODE_RHS) or a c0 + b (cs + dt R_C) (MODE_RK)
template <int N, int MODE>
__global__ void __launch_bounds__(Sz<N>::NT) k_tracer_stage(const TracerArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    __shared__ double sQ[5 * NP];   // the leaf's Euler state
    __shared__ double sC[NP];       // the leaf's tracer
    __shared__ double sF[NP];       // the flux plane of one direction
    __shared__ double sS[6 * NF];   // lifted face contributions [f][m]
    __shared__ double sRinv[NP];    // 1/rho at each node
    __shared__ double sCs[NP];      // the sound speed at each node
    __shared__ double sD[N1 * N1];
    __shared__ double sBg[4 * N1];  // rho, Theta, P, 1/Theta
    __shared__ double sGeo[4];
    const int64_t K = A.K;
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t* const rec = A.srec + e * kStageRec;
    const int t = threadIdx.x;
    const double gamma = A.gamma;
    const int64_t KNP = K * NP, KN1 = K * N1;
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;
    for (int ii = t; ii < N1 * N1; ii += NT) sD[ii] = A.ops[ii];
    if (t < 3 * N1) {
        const double v = A.bg[(t / N1) * KN1 + e * N1 + (t % N1)];
        sBg[t] = v;
        if (t >= N1 && t < 2 * N1) sBg[2 * N1 + t] = 1.0 / v;
    }
    if (t < 4) sGeo[t] = A.geo[e * 4 + t];
    if (t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sQ[v * NP + t] = A.qs[v * KNP + e * NP + t];
        sC[t] = A.cs[e * NP + t];
    }
    // face items grouped by axis, each axis padded to whole waves (a wave never mixes
    // the three axis variants); this thread's items' neighbour states, tracer and
    // mortar terms are loaded with the tile, before the first barrier
    constexpr int PAD = ((2 * NF + 63) / 64) * 64;
    constexpr int ITEMS = (3 * PAD + NT - 1) / NT;
    // (of the neighbour's Euler state only rho', the momentum along the face's axis
    // and Theta' enter the tracer flux)
    double qR_[ITEMS][3], CR_[ITEMS], bR_[ITEMS][3];
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        const int it = t + u * NT;
        CR_[u] = 0.0;
        if (it >= 3 * PAD) continue;
        const int ax = it / PAD, r = it % PAD;
        if (r >= 2 * NF) continue;
        const int f = 2 * ax + r / NF, m = r % NF;
        const int tf = rec[f], type = tf & 0xff;
        if (type == FT_FINE || type == FT_COARSE) {
            const int64_t row = (int64_t)rec[12 + f] * 5 + (type == FT_COARSE ? 0 : 1 + ((tf >> 8) & 0xff));
            sS[f * NF + m] = A.mortC[row * NF + m];
        } else if (type != FT_WALL) {
            const int64_t nb = rec[6 + f];
            const int nn = face_node<N>(f ^ 1, m);
            const int64_t at = nb * NP + nn;
            qR_[u][0] = A.qs[at];
            qR_[u][1] = A.qs[(1 + ax) * KNP + at];
            qR_[u][2] = A.qs[4 * KNP + at];
            CR_[u] = A.cs[at];
            if (tf & FT_BG_NB) {
                const int kn = face_k<N>(f ^ 1, m);
#pragma unroll
                for (int c = 0; c < 3; ++c) bR_[u][c] = A.bg[c * KN1 + nb * N1 + kn];
            }
        }
    }
    __syncthreads();
    // 1/rho and the sound speed once per node (the face items read their own side's
    // here instead of forming them again: the same expressions, the same values)
    double rinv = 0.0;
    if (t < NP) {
        rinv = rcp_pos(sBg[k] + sQ[t]);
        const double Pp = pprime(sQ[4 * NP + t], sBg[3 * N1 + k], sBg[2 * N1 + k], gamma, A.binom);
        sRinv[t] = rinv;
        sCs[t] = sqrt_pos(gamma * (sBg[2 * N1 + k] + Pp) * rinv);
    }
    __syncthreads();
    const double liftc = 0.5 * N * (N + 1);
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        const int it = t + u * NT;
        if (it >= 3 * PAD) continue;
        const int ax = it / PAD, r = it % PAD;
        if (r >= 2 * NF) continue;
        const int f = 2 * ax + r / NF, m = r % NF;
        const int tf = rec[f], type = tf & 0xff;
        if (type == FT_FINE || type == FT_COARSE) continue;
        const int d = ax;
        const double sgn = (f & 1) ? 1.0 : -1.0;
        const int n = face_node<N>(f, m), kk = face_k<N>(f, m);
        const TrState qL{sQ[n], sQ[(1 + d) * NP + n], sQ[4 * NP + n]};
        TrState qR{qL.rho, -qL.m, qL.Thp};  // a wall's mirror state: the normal momentum reversed
        const double CL = sC[n];
        double CR = CL;
        const Bg bL{sBg[kk], sBg[N1 + kk], sBg[2 * N1 + kk], sBg[3 * N1 + kk]};
        Bg bR = bL;
        if (type != FT_WALL) {
            qR = TrState{qR_[u][0], qR_[u][1], qR_[u][2]};
            CR = CR_[u];
            if (tf & FT_BG_NB) bR = bg_make(bR_[u][0], bR_[u][1], bR_[u][2]);
        }
        const double PpR = pprime(qR.Thp, bR.rTh, bR.P, gamma, A.binom);
        const double lift = sGeo[d] * liftc;
        const double uL = qL.m * sRinv[n];
        sS[f * NF + m] = tracer_lifted(uL, fabs(uL) + sCs[n], CL, qR, CR, bR, PpR, sgn, gamma, lift);
    }
    // volume: R = -sum_d (2/h_d) D_d (C u_d), one direction at a time
    double R = 0.0, C = 0.0;
    if (t < NP) C = sC[t];
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        __syncthreads();
        if (t < NP) sF[t] = C * (sQ[(1 + d) * NP + t] * rinv);
        __syncthreads();
        if (t < NP) {
            const int id = d == 0 ? i : d == 1 ? j : k;
            const int stride = d == 0 ? 1 : d == 1 ? N1 : NF;
            const double* Fp = sF + (t - id * stride);
            double acc = 0.0;
#pragma unroll
            for (int mm = 0; mm < N1; ++mm) acc = fma(sD[id * N1 + mm], Fp[mm * stride], acc);
            R = fma(-sGeo[d], acc, R);
        }
    }
    if (t >= NP) return;
    // lift: the faces through this node, x then y then z
    if (i == 0 || i == N) R -= sS[(i == N ? 1 : 0) * NF + j + N1 * k];
    if (j == 0 || j == N) R -= sS[(j == N ? 3 : 2) * NF + i + N1 * k];
    if (k == 0 || k == N) R -= sS[(k == N ? 5 : 4) * NF + i + N1 * j];
    const int64_t at = e * NP + t;
    if (MODE == MODE_RHS) {
        A.out[at] = R;
    } else {
        double o = A.b * fma(A.dt, R, C);
        if (A.a != 0.0) o = fma(A.a, A.c0[at], o);
        A.out[at] = o;
    }
}

// integral of a field [K][Np] with weights J_e W_n, compensated, deterministic
template <int N>
__global__ void __launch_bounds__(256) k_weighted_sum(const double* c, const double* geo, const double* w, int64_t K,
                                                      double* partial) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1, NT = 256;
    __shared__ Comp sh[4 * NT];
    const int t = threadIdx.x;
    Comp acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    const int64_t per = (K + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = blockIdx.x * per, e1 = (e0 + per < K) ? e0 + per : K;
    for (int64_t e = e0; e < e1; ++e) {
        const double J = geo[e * 4 + 3];
        for (int n = t; n < NP; n += NT) {
            const int ii = n % N1, jj = (n / N1) % N1, kk = n / (N1 * N1);
            acc[0] = comp_add(acc[0], J * w[ii] * w[jj] * w[kk] * c[e * NP + n]);
        }
    }
    block_reduce4<NT>(acc, sh);
    if (t == 0) {
        partial[blockIdx.x * 2] = acc[0].s;
        partial[blockIdx.x * 2 + 1] = acc[0].c;
    }
}

__global__ void __launch_bounds__(256) k_weighted_sum_final(const double* partial, int nblk, double* out) {
    constexpr int NT = 256;
    __shared__ Comp sh[4 * NT];
    const int t = threadIdx.x;
    Comp acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int b = t; b < nblk; b += NT) acc[0] = comp_merge(acc[0], Comp{partial[b * 2], partial[b * 2 + 1]});
    block_reduce4<NT>(acc, sh);
    if (t == 0) out[0] = acc[0].s + acc[0].c;
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

hipError_t launch_tracer_mortar(int N, const TracerMortArgs& a, hipStream_t s) {
    if (a.n_hang <= 0) return hipSuccess;
    if (a.pointwise) {
        DG_DISPATCH_N(N, (k_tracer_mortar<NN, true><<<dim3((unsigned)a.n_hang), dim3(Sz<NN>::NT), 0, s>>>(a)));
    } else {
        DG_DISPATCH_N(N, (k_tracer_mortar<NN, false><<<dim3((unsigned)a.n_hang), dim3(Sz<NN>::NT), 0, s>>>(a)));
    }
    return hipGetLastError();
}

hipError_t launch_tracer_stage(int N, int mode, const TracerArgs& a, hipStream_t s) {
    if (a.K <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.K);
    if (mode == MODE_RHS) {
        DG_DISPATCH_N(N, (k_tracer_stage<NN, MODE_RHS><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
    } else {
        DG_DISPATCH_N(N, (k_tracer_stage<NN, MODE_RK><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
    }
    return hipGetLastError();
}

hipError_t launch_weighted_sum(int N, const double* c, const double* geo, const double* w, int64_t K, int nblk,
                               double* partial, double* out_dev, hipStream_t s) {
    DG_DISPATCH_N(N, (k_weighted_sum<NN><<<dim3((unsigned)nblk), dim3(256), 0, s>>>(c, geo, w, K, partial)));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_weighted_sum_final<<<dim3(1), dim3(256), 0, s>>>(partial, nblk, out_dev);
    return hipGetLastError();
}

}  // namespace dgamr

// HIP kernels for gfx950 (MI355X) of the DG-AMR hot path.
//
// One workgroup per leaf ("element-centric"): the fused stage kernel loads the
// leaf's (N+1)^3 tile into LDS, evaluates the pointwise physics and the three
// tensor-product derivative contractions (strong-form volume term, section
// 2.2), then computes the Rusanov flux on each of its six faces against the
// neighbour trace gathered straight from HBM (conforming faces, no-flux walls,
// and L2 mortars on hanging faces, section 3.3), lifts (F* - F).n into the
// face nodes, and writes either R or the Shu-Osher stage a q0 + b (qs + dt R).
// Every face is evaluated by both of its leaves; the Rusanov flux is computed
// so that F*(qL, qR, n) = -F*(qR, qL, -n) bitwise, and both sides of a mortar
// build the mortar state with the same arithmetic, so what one side gains the
// other loses to the last bit (discrete conservation, section 2.1).
//
// The file is compiled with -ffp-contract=off: every fused multiply-add is an
// explicit fma(), so that the rounding of a value does not depend on where the
// compiler inlines it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"

namespace dgamr {
namespace {

using namespace dev;

// sgn * F^D(q) and the wave speed |u_D| + c  (axis D known at compile time, so
// no array is ever indexed by a run-time value)
template <int D>
__device__ __forceinline__ void flux_n(const double q[5], const Bg& bg, double Pp, double sgn, double gamma,
                                       double F[5], double& lam) {
    const double rho = bg.rho + q[0];
    const double rinv = rcp_pos(rho);
    const double ud = q[1 + D] * rinv;
    const double Th = bg.Th + q[4];
    F[0] = sgn * q[1 + D];
    F[1] = sgn * (D == 0 ? q[1] * ud + Pp : q[1] * ud);
    F[2] = sgn * (D == 1 ? q[2] * ud + Pp : q[2] * ud);
    F[3] = sgn * (D == 2 ? q[3] * ud + Pp : q[3] * ud);
    F[4] = sgn * (Th * ud);
    lam = fabs(ud) + sqrt_pos(gamma * (bg.P + Pp) * rinv);
}

// Rusanov flux F*.n, n = sgn e_D:  {F.n} + 1/2 max(|u.n| + c) (q'- - q'+)  (section 2.2);
// also returns FL = F(qL).n
template <int D>
__device__ __forceinline__ void rusanov(const double qL[5], const Bg& bL, double PpL, const double qR[5],
                                        const Bg& bR, double PpR, double sgn, double gamma, double Fs[5],
                                        double FL[5]) {
    double FR[5], lL, lR;
    flux_n<D>(qL, bL, PpL, sgn, gamma, FL, lL);
    flux_n<D>(qR, bR, PpR, sgn, gamma, FR, lR);
    const double hl = 0.5 * fmax(lL, lR);
#pragma unroll
    for (int v = 0; v < 5; ++v) Fs[v] = 0.5 * (FL[v] + FR[v]) + hl * (qL[v] - qR[v]);
}

// lift (F*.n - F(qL).n) for the Rusanov flux, written as
// lift (sgn/2 (F^D(qR) - F^D(qL)) + 1/2 max(|u.n| + c) (q'L - q'R)): the lifted
// surface term of the leaf on the L side, without forming F*.n itself
template <int D>
__device__ __forceinline__ void rusanov_lifted(const double qL[5], const Bg& bL, double PpL, const double qR[5],
                                               const Bg& bR, double PpR, double sgn, double gamma, double lift,
                                               double out[5]) {
    double FL[5], FR[5], lL, lR;
    flux_n<D>(qL, bL, PpL, 1.0, gamma, FL, lL);
    flux_n<D>(qR, bR, PpR, 1.0, gamma, FR, lR);
    const double c1 = 0.5 * sgn * lift, c2 = 0.5 * fmax(lL, lR) * lift;
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v] = fma(c1, FR[v] - FL[v], c2 * (qL[v] - qR[v]));
}

// waves per SIMD the stage kernel is compiled for (bounds its VGPR budget:
// 6 -> 80, 5 -> 96 registers); with the mortars in their own pre-pass the stage
// fits these, and at N = 7 three workgroups of 8 waves then share a CU
template <int N>
struct StageOcc {
    static constexpr int W = N == 7 || N == 4 ? 6 : 5;
    // one batched gather of the tile and the neighbour traces into LDS (pays at low
    // order, where faces carry most of the work), or loads straight into registers
    static constexpr bool GATHER = N <= 5;
};

// LDS plan of the stage kernel: the work area first holds the leaf's float64 tile
// [5][NP], then the flux planes of the volume phase: all 15 at once, or x and y,
// then z (one more barrier), or one direction at a time (five planes; three more
// barriers).  The plan with the most workgroups per CU (160 KB of LDS, W waves per
// SIMD) wins, the one with fewer barriers on a tie.  MIX stores the planes as float
// (flux minus an element-constant reference).
template <int N, bool MIX>
struct StageLds {
    static constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF;
    static constexpr int ESZ = MIX ? 4 : 8;
    static constexpr int work_dbl(int planes) {
        return (planes * NP * ESZ + 7) / 8 > 5 * NP ? (planes * NP * ESZ + 7) / 8 : 5 * NP;
    }
    // bytes of the other LDS arrays of k_stage
    static constexpr int FIXED = 8 * (30 * NF + N1 * N1 + 4 * N1 + 4 + 8 + (MIX ? 15 : 1)) + 4 * (MIX ? 2 * N1 * N1 : 1) + 4 * 18;
    static constexpr int blocks(int planes) {
        const int by_lds = 160 * 1024 / (FIXED + 8 * work_dbl(planes));
        const int by_waves = 4 * StageOcc<N>::W / (Sz<N>::NT / 64);
        return by_lds < by_waves ? by_lds : by_waves;
    }
    static constexpr bool FITS15 = FIXED + 8 * work_dbl(15) <= 64 * 1024;
    static constexpr int PLANES = FITS15 && blocks(15) >= blocks(10) && blocks(15) >= blocks(5) ? 15
                                  : blocks(10) >= blocks(5)                                  ? 10
                                                                                             : 5;
    static constexpr bool ALL3 = PLANES == 15;
    static constexpr int WORK = work_dbl(PLANES);
};

// Mortar pre-pass (section 3.3, the three steps on the mortars of one hanging
// face per workgroup): the coarse trace is interpolated to the four mortars
// (I_a x I_b, two separable passes), the Riemann problem is solved on each
// mortar point from the fine leaf's side, and the coarse side's flux is that
// flux with the sign reversed (the Rusanov flux is antisymmetric bitwise), which
// is projected back with R_a x R_b.  Output per hanging face h, lifted and
// ready for the stage kernel: mort[h][0] the coarse face, mort[h][1 + quad] the
// fine faces, each [5][NF].  The stage kernel copies these into its faces.
// PW (pointwise matching, section 3.3's simpler alternative): the fine faces as
// above; the coarse side instead solves the Riemann problem at each of its own
// face nodes against the fine polynomial evaluated there (sum over quadrants of
// P_a x P_b applied to the fine traces, the same separable passes as the
// projection), so the two sides' fluxes no longer balance.
template <int N, bool PW>
__global__ void __launch_bounds__(Sz<N>::NT) k_mortar(const MortArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    static_assert(4 * NF <= NT, "one mortar point per thread");
    constexpr int PWOFF = Sz<N>::NOPS;       // P0, P1 after D, I0, I1, R0, R1, w (PW)
    __shared__ double sT[5 * NF], sU[10 * NF], sMq[20 * NF], sG[10 * NF];
    __shared__ double sOps[Sz<N>::NOPS + (PW ? 2 * NF : 0)];
    __shared__ double sBg[3 * N1];  // the coarse leaf's background
    const int64_t h = xcd_remap(blockIdx.x, gridDim.x);
    const int t = threadIdx.x;
    const int32_t* const row = A.hang + h * 6;
    const int64_t ec = row[0];
    const int f = row[1], fo = f ^ 1;
    const int KNP = (int)(A.K * NP), KN1 = (int)(A.K * N1);
    const double gamma = A.gamma;
    const double liftc = 0.5 * N * (N + 1);  // 1/w_N
    const double sgn = (f & 1) ? 1.0 : -1.0;  // the coarse leaf's outward normal
    const double* const qs = A.qs;
    for (int ii = t; ii < Sz<N>::NOPS; ii += NT) sOps[ii] = A.ops[ii];
    if (PW)  // the ops table holds 4 transposes (adjoint) before P0, P1
        for (int ii = t; ii < 2 * NF; ii += NT) sOps[PWOFF + ii] = A.ops[Sz<N>::NOPS + 4 * NF + ii];
    if (t < 3 * N1) sBg[t] = A.bg[(t / N1) * KN1 + ec * N1 + (t % N1)];
    for (int it = t; it < 5 * NF; it += NT) {
        const int v = it / NF, m = it % NF;
        sT[it] = qs[v * KNP + ec * NP + face_node<N>(f, m)];
    }
    // this thread's fine-side point and the lift factors, loaded with the trace (every
    // global read of the workgroup is in this one batch): quadrant t / NF
    double qF[5];
    Bg bF{};
    double lift_f = 0.0;
    const double lift_c = A.geo[ec * 4 + (f >> 1)] * liftc;
    if (t < 4 * NF) {
        const int quad = t / NF, m = t % NF;
        const int64_t ef = row[2 + quad];
        const int nn = face_node<N>(fo, m), kn = face_k<N>(fo, m);
        bF = bg_make(A.bg[ef * N1 + kn], A.bg[KN1 + ef * N1 + kn], A.bg[2 * KN1 + ef * N1 + kn]);
#pragma unroll
        for (int v = 0; v < 5; ++v) qF[v] = qs[v * KNP + ef * NP + nn];
        lift_f = A.geo[ef * 4 + (f >> 1)] * liftc;
    }
    __syncthreads();
    // sU[a][v] = I_a along t1; sMq[quad][v] = I_b along t2 of sU[a]  (quad = a + 2b)
    apply_t1<N>(sT, sU, 10, [&](int p) { return sOps + (1 + p / 5) * NF; }, [](int p) { return p % 5; }, t, NT);
    __syncthreads();
    apply_t2<N>(sU, sMq, 20, [&](int p) { return sOps + (1 + (p / 5) / 2) * NF; },
                [](int p) { return ((p / 5) & 1) * 5 + p % 5; }, t, NT);
    __syncthreads();
    if (t < 4 * NF) {
        const int quad = t / NF, m = t % NF;
        double qM[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qM[v] = sMq[(quad * 5 + v) * NF + m];
        const double PpF = pprime(qF[4], bF.rTh, bF.P, gamma, A.binom);
        const double PpM = pprime(qM[4], bF.rTh, bF.P, gamma, A.binom);
        double Fs[5], Fo[5];
        with_axis(f >> 1, [&](auto dc) {
            rusanov<decltype(dc)::value>(qF, bF, PpF, qM, bF, PpM, -sgn, gamma, Fs, Fo);
        });
        double* const out = A.mort + ((h * 5 + 1 + quad) * 5) * NF + m;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            out[v * NF] = (Fs[v] - Fo[v]) * lift_f;
            // in place: the coarse side's flux (mortars) or the fine state (pointwise)
            sMq[(quad * 5 + v) * NF + m] = PW ? qF[v] : -Fs[v];
        }
    }
    __syncthreads();
    // back to the coarse nodes: sG[b][v] = sum_a B_a along t1 of X[a + 2b]; then sum_b
    // B_b along t2, with B = R (mortars: X the flux) or B = P (pointwise: X the fine state)
    for (int it = t; it < 10 * NF; it += NT) {
        const int p = it / NF, r = it % NF, bb = r / N1, a2 = r % N1;
        const int qb = p / 5, v = p % 5;
        double acc = 0.0;
#pragma unroll
        for (int qa = 0; qa < 2; ++qa) {
            const double* Rm = sOps + (PW ? PWOFF + qa * NF : (3 + qa) * NF) + a2 * N1;
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
            const double* Rm = sOps + (PW ? PWOFF + qb * NF : (3 + qb) * NF) + b2 * N1;
            const double* x = sG + (qb * 5 + v) * NF + a;
#pragma unroll
            for (int bb = 0; bb < N1; ++bb) proj = fma(Rm[bb], x[bb * N1], proj);
        }
        sU[it] = proj;
    }
    __syncthreads();
    if (t < NF) {
        const int m = t;
        const int kk = face_k<N>(f, m);
        const Bg b = bg_make(sBg[kk], sBg[N1 + kk], sBg[2 * N1 + kk]);
        double qL[5], Fo[5], Fc[5], lam;
#pragma unroll
        for (int v = 0; v < 5; ++v) qL[v] = sT[v * NF + m];  // the coarse trace at face node m
        const double PpL = pprime(qL[4], b.rTh, b.P, gamma, A.binom);
        if constexpr (PW) {
            // Riemann problem at the coarse node against the fine state there
            double qR[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) qR[v] = sU[v * NF + m];
            const double PpR = pprime(qR[4], b.rTh, b.P, gamma, A.binom);
            with_axis(f >> 1, [&](auto dc) {
                rusanov<decltype(dc)::value>(qL, b, PpL, qR, b, PpR, sgn, gamma, Fc, Fo);
            });
        } else {
            with_axis(f >> 1, [&](auto dc) { flux_n<decltype(dc)::value>(qL, b, PpL, sgn, gamma, Fo, lam); });
#pragma unroll
            for (int v = 0; v < 5; ++v) Fc[v] = sU[v * NF + m];
        }
        double* const out = A.mort + (h * 5 * 5) * NF + m;
#pragma unroll
        for (int v = 0; v < 5; ++v) out[v * NF] = (Fc[v] - Fo[v]) * lift_c;
    }
}

// MIX: the volume contractions in float32 on the flux minus the flux at the
// leaf's first node (exact, since D annihilates constants), with D split into a
// float32 high part and a float32 correction and float32 accumulation; the
// pressure, the fluxes themselves, faces, mortars and the update stay float64.
template <int N, int MODE, bool MIX>
__global__ void __launch_bounds__(Sz<N>::NT) __attribute__((amdgpu_waves_per_eu(StageOcc<N>::W)))
k_stage(const StageArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    constexpr bool ALL3 = StageLds<N, MIX>::ALL3;
    // sS: per face f and variable v the trace slot [f][v][NF]: first the neighbour's
    // trace (conforming faces) or the lifted mortar contribution (hanging faces),
    // then the lifted contribution itself
    __shared__ double sS[30 * NF];
    // sW: first this leaf's tile [5][NP], then the flux planes of the volume phase
    __shared__ double sW[StageLds<N, MIX>::WORK];
    __shared__ float sD32[MIX ? 2 * N1 * N1 : 1];  // MIX: D high and low parts
    __shared__ double sD[N1 * N1];
    __shared__ double sBg[4 * N1];       // rho, Theta, P, 1/Theta of the background
    __shared__ double sGeo[4];
    __shared__ double sBgZ[8];           // far-side background of faces 4, 5 (rho, Theta, P, 1/Theta)
    __shared__ int sType[6];
    __shared__ int sNb[6];               // first neighbour per face
    __shared__ int sHs[6];               // hanging face: row of the mortar pre-pass
    __shared__ double sFr[MIX ? 15 : 1];  // MIX: reference flux [direction][variable]

    const int64_t K = A.K;
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t* const rec = A.srec + e * kStageRec;
    const int t = threadIdx.x;
    const double gamma = A.gamma;
    const double* const D = sD;
    const double* qs = A.qs;
    const int KNP = (int)(K * NP);  // 5 K Np < 2^31 is checked by the host
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;
    // per-variable planes of qs: wave-uniform bases, 32-bit byte offsets within a plane
    // (K Np 8 < 2^32 follows from the 5 K Np < 2^31 the host checks)
    const double* qv[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) qv[v] = qs + (int64_t)v * KNP;
    const uint32_t eoff = (uint32_t)e * NP * 8u;

    constexpr bool GATHER = StageOcc<N>::GATHER;
    // the leaf's face tables: one uniform record, read before any store of the kernel
    // (scalar loads), so the loads that depend on them wait for no LDS round trip
    int tfs[6], nbs[6], hss[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        tfs[f] = rec[f];
        nbs[f] = rec[6 + f];
        hss[f] = rec[12 + f];
    }
    if (t < 6) {
        sType[t] = rec[t];
        sNb[t] = rec[6 + t];
        sHs[t] = rec[12 + t];
    }
    if constexpr (!GATHER) {
        // ---- D and the background profile
        for (int ii = t; ii < N1 * N1; ii += NT) {
            const double dv = A.ops[ii];
            sD[ii] = dv;
            if (MIX) {
                const float hi = (float)dv;
                sD32[ii] = hi;
                sD32[N1 * N1 + ii] = (float)(dv - (double)hi);
            }
        }
        if (t < 3 * N1) {
            const double v = A.bg[(int64_t)(t / N1) * K * N1 + e * N1 + (t % N1)];
            sBg[t] = v;
            if (t >= N1 && t < 2 * N1) sBg[2 * N1 + t] = 1.0 / v;
        }
        if (t < 4) sGeo[t] = A.geo[e * 4 + t];
        __syncthreads();
    } else {
        // ---- gather: every load of the leaf (D, background, geometry, tile, the
        // neighbours' face traces, the mortar contributions) is issued before any of
        // them is written to LDS, so all of them are in flight together: one memory
        // round trip for the leaf, one barrier
        static_assert(NP <= NT && N1 * N1 <= NT && 3 * N1 <= NT, "one thread per node");
        constexpr int NR = (5 * NF + NT - 1) / NT;  // passes over the face slots
        const double dv = t < N1 * N1 ? A.ops[t] : 0.0;
        const double bv = t < 3 * N1 ? A.bg[(int64_t)(t / N1) * K * N1 + e * N1 + (t % N1)] : 0.0;
        const double gv = t < 4 ? A.geo[e * 4 + t] : 0.0;
        double tv[5] = {0, 0, 0, 0, 0};
        if (t < NP)
#pragma unroll
            for (int v = 0; v < 5; ++v) tv[v] = ld_off(qv[v], eoff + (uint32_t)t * 8u);
        // face slots: thread t covers (v, m) of every face, one pass per face; each slot
        // issues one load (a wall face reads its own leaf's entry and drops it)
        int ftype[6], fsrc[6];  // per face: type; neighbour leaf or first mortar row
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int tf = tfs[f], type = tf & 0xff;
            ftype[f] = type;
            fsrc[f] = type == FT_CONF     ? nbs[f]
                      : type == FT_WALL   ? (int)e
                      : type == FT_COARSE ? hss[f] * 5
                                          : hss[f] * 5 + 1 + ((tf >> 8) & 0xff);
        }
        double fv[NR][6];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int vm = (5 * NF % NT == 0 || t + r * NT < 5 * NF) ? t + r * NT : 0;
            const int v = vm / NF, m = vm - v * NF;
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                // conforming: the neighbour's node across the face; wall: this leaf's own
                // face node (the slot becomes the mirror state)
                const int nn = face_node<N>(ftype[f] == FT_CONF ? f ^ 1 : f, m);
                const double* src = ftype[f] == FT_CONF || ftype[f] == FT_WALL
                                        ? qs + (v * KNP + fsrc[f] * NP + nn)
                                        : A.mort + (int64_t)fsrc[f] * 5 * NF + vm;
                fv[r][f] = *src;
            }
        }
        // far side of the z faces (f = 4, 5): this leaf's bottom / top level, or the
        // neighbour's top / bottom level across a periodic wrap along z
        double zb = 0.0;
        const int zc = (t - 32) & 3;
        const bool zt = t >= 32 && t < 40, zhi = t >= 36;
        const bool znb = zt && ((zhi ? tfs[5] : tfs[4]) & FT_BG_NB) != 0;
        if (zt) {
            const int kk = zhi != znb ? N : 0;
            const int64_t src = znb ? (int64_t)(zhi ? nbs[5] : nbs[4]) : e;
            zb = A.bg[(int64_t)(zc == 3 ? 1 : zc) * K * N1 + src * N1 + kk];
        }
        if (t < N1 * N1) {
            sD[t] = dv;
            if (MIX) {
                const float hi = (float)dv;
                sD32[t] = hi;
                sD32[N1 * N1 + t] = (float)(dv - (double)hi);
            }
        }
        if (t < 3 * N1) {
            sBg[t] = bv;
            if (t >= N1 && t < 2 * N1) sBg[2 * N1 + t] = 1.0 / bv;
        }
        if (t < 4) sGeo[t] = gv;
        if (t < NP)
#pragma unroll
            for (int v = 0; v < 5; ++v) sW[v * NP + t] = tv[v];
        if (zt) sBgZ[t - 32] = zc == 3 ? 1.0 / zb : zb;
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (5 * NF % NT == 0 || t + r * NT < 5 * NF)
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    // mirror state of a wall: the normal momentum reversed
                    const bool flip = ftype[f] == FT_WALL && (t + r * NT) / NF == 1 + (f >> 1);
                    sS[f * 5 * NF + t + r * NT] = flip ? -fv[r][f] : fv[r][f];
                }
    }
    if (MIX && t < 3) {
        // element-constant reference flux: the flux at the leaf's first node, one
        // direction per thread (background at the leaf's lowest level, read here)
        double q0n[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) q0n[v] = ld_off(qv[v], eoff);
        const double rho0 = A.bg[e * N1], Th0b = A.bg[K * N1 + e * N1], P0b = A.bg[2 * K * N1 + e * N1];
        const double rinv0 = rcp_pos(rho0 + q0n[0]);
        const double Pp0 = pprime(q0n[4], 1.0 / Th0b, P0b, gamma, A.binom);
        const double Th0 = Th0b + q0n[4];
        const double Ud = t == 0 ? q0n[1] : t == 1 ? q0n[2] : q0n[3];
        const double u0 = Ud * rinv0;
        sFr[t * 5 + 0] = Ud;
        sFr[t * 5 + 1] = t == 0 ? q0n[1] * u0 + Pp0 : q0n[1] * u0;
        sFr[t * 5 + 2] = t == 1 ? q0n[2] * u0 + Pp0 : q0n[2] * u0;
        sFr[t * 5 + 3] = t == 2 ? q0n[3] * u0 + Pp0 : q0n[3] * u0;
        sFr[t * 5 + 4] = Th0 * u0;
    }
    __syncthreads();

    // q0 of the update (stage form, a != 0): requested before the faces when the
    // tile came in one batch, so its latency runs under the face work
    double q0v[5] = {0, 0, 0, 0, 0};
    const bool use_q0 = (MODE == MODE_RK || MODE == MODE_RK_STREAM) && A.a != 0.0;
    auto load_q0 = [&]() {
        if (use_q0 && t < NP)
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double* src = reinterpret_cast<const double*>(
                    reinterpret_cast<const char*>(A.q0 + (int64_t)v * KNP) + (eoff + (uint32_t)t * 8u));
                if constexpr (MODE == MODE_RK_STREAM)
                    q0v[v] = __builtin_nontemporal_load(src);
                else
                    q0v[v] = *src;
            }
    };
    if (GATHER) load_q0();

    // ---- faces, every (face, node) item of a wall or conforming face: Rusanov flux
    // from the own trace (tile) and the neighbour trace (sS), lifted in place;
    // hanging faces already hold the pre-pass contributions
    const double liftc = 0.5 * N * (N + 1);  // 1/w_N
    // items grouped by axis, each axis padded to whole waves, so a wave never
    // mixes the three axis variants of the flux code
    constexpr int PAD = ((2 * NF + 63) / 64) * 64;
#pragma unroll 1
    for (int it = t; it < 3 * PAD; it += NT) {
        // PAD and NT are whole waves: the axis is the same across a wave
        const int ax = it / PAD, r = it % PAD;
        if (r >= 2 * NF) continue;
        const int f = 2 * ax + r / NF, m = r % NF;
        const int tf = sType[f];
        const int type = tf & 0xff;
        if (type == FT_FINE || type == FT_COARSE) {
            if constexpr (!GATHER) {
                const int64_t row = (int64_t)sHs[f] * 5 + (type == FT_COARSE ? 0 : 1 + ((tf >> 8) & 0xff));
#pragma unroll
                for (int v = 0; v < 5; ++v) sS[(f * 5 + v) * NF + m] = A.mort[(row * 5 + v) * NF + m];
            }
            continue;
        }
        const double sgn = (f & 1) ? 1.0 : -1.0;
        const int n = face_node<N>(f, m), kk = face_k<N>(f, m);
        const double lift = sGeo[ax] * liftc;
        double* const slot = sS + f * 5 * NF + m;
        with_axis(ax, [&](auto dc) {
            constexpr int d = decltype(dc)::value;
            double qL[5], qR[5];
            if constexpr (GATHER) {
                // the slot holds the neighbour's trace or a wall's mirror state; the far
                // side's background is this side's except on z faces (sBgZ)
#pragma unroll
                for (int v = 0; v < 5; ++v) qL[v] = sW[v * NP + n];
#pragma unroll
                for (int v = 0; v < 5; ++v) qR[v] = slot[v * NF];
                const Bg bL{sBg[kk], sBg[N1 + kk], sBg[2 * N1 + kk], sBg[3 * N1 + kk]};
                const Bg bR = d == 2 ? Bg{sBgZ[(f & 1) * 4], sBgZ[(f & 1) * 4 + 1], sBgZ[(f & 1) * 4 + 2],
                                          sBgZ[(f & 1) * 4 + 3]}
                                     : bL;
                const double PpL = pprime(qL[4], bL.rTh, bL.P, gamma, A.binom);
                const double PpR = pprime(qR[4], bR.rTh, bR.P, gamma, A.binom);
                double o[5];
                rusanov_lifted<d>(qL, bL, PpL, qR, bR, PpR, sgn, gamma, lift, o);
#pragma unroll
                for (int v = 0; v < 5; ++v) slot[v * NF] = o[v];
                return;
            } else {
                // both traces requested before either is used (a wall face loads its
                // own entry twice and mirrors it below)
                const int nb = type == FT_CONF ? sNb[f] : (int)e;
                const uint32_t nn = (uint32_t)(type == FT_CONF ? face_node<N>(f ^ 1, m) : n);
#pragma unroll
                for (int v = 0; v < 5; ++v) qL[v] = ld_off(qv[v], eoff + (uint32_t)n * 8u);
#pragma unroll
                for (int v = 0; v < 5; ++v) qR[v] = ld_off(qv[v], ((uint32_t)nb * NP + nn) * 8u);
            }
            // the background is a function of z, and the two leaves of a conforming
            // face see bitwise-identical z at its nodes, except across a periodic
            // wrap along z (flagged by the host)
            const Bg bL{sBg[kk], sBg[N1 + kk], sBg[2 * N1 + kk], sBg[3 * N1 + kk]};
            const double PpL = pprime(qL[4], bL.rTh, bL.P, gamma, A.binom);
            Bg bR = bL;
            double PpR = PpL;
            if (type == FT_WALL) {
#pragma unroll
                for (int v = 0; v < 5; ++v) qR[v] = qL[v];
                qR[1 + d] = -qL[1 + d];  // mirror state: reverse the normal momentum
            } else {
                if (tf & FT_BG_NB) {
                    const int nb = sNb[f], kn = face_k<N>(f ^ 1, m);
                    bR = bg_make(A.bg[nb * N1 + kn], A.bg[K * N1 + nb * N1 + kn], A.bg[2 * K * N1 + nb * N1 + kn]);
                }
                PpR = pprime(qR[4], bR.rTh, bR.P, gamma, A.binom);
            }
            double o[5];
            rusanov_lifted<d>(qL, bL, PpL, qR, bR, PpR, sgn, gamma, lift, o);
#pragma unroll
            for (int v = 0; v < 5; ++v) slot[v * NF] = o[v];
        });
    }

    // ---- volume term: R = S - sum_d (2/h_d) D_d F^d, fluxes staged in LDS; q from
    // the tile, q0 of the update (stage form, a != 0) loaded now, used at the end
    double q[5] = {0, 0, 0, 0, 0};
    if (!GATHER) load_q0();
    double rinv = 0.0, Pp = 0.0, Th = 0.0;
    double R[5] = {0, 0, 0, 0, 0};
    if (t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) q[v] = GATHER ? sW[v * NP + t] : ld_off(qv[v], eoff + (uint32_t)t * 8u);
        rinv = rcp_pos(sBg[k] + q[0]);
        Pp = pprime(q[4], sBg[3 * N1 + k], sBg[2 * N1 + k], gamma, A.binom);
        Th = sBg[N1 + k] + q[4];
        R[3] = -q[0] * A.g;  // buoyancy on rho*w
    }
    // GATHER: the faces read other nodes' tile entries, and the flux planes overwrite
    // the tile: every read must be done (otherwise nothing is shared yet: the face
    // results in sS are read after the volume's barriers)
    if constexpr (GATHER) __syncthreads();

    auto put_flux = [&](int d, int plane) {
        const double ud = q[1 + d] * rinv;
        double F[5];
        F[0] = q[1 + d];
        F[1] = d == 0 ? q[1] * ud + Pp : q[1] * ud;
        F[2] = d == 1 ? q[2] * ud + Pp : q[2] * ud;
        F[3] = d == 2 ? q[3] * ud + Pp : q[3] * ud;
        F[4] = Th * ud;
        if (MIX) {
            float* Ff = reinterpret_cast<float*>(sW) + plane * 5 * NP;
#pragma unroll
            for (int v = 0; v < 5; ++v) Ff[v * NP + t] = (float)(F[v] - sFr[d * 5 + v]);
        } else {
            double* Fd = sW + plane * 5 * NP;
#pragma unroll
            for (int v = 0; v < 5; ++v) Fd[v * NP + t] = F[v];
        }
    };
    auto contract = [&](int d, int plane) {
        const int id = d == 0 ? i : d == 1 ? j : k;
        const int stride = d == 0 ? 1 : d == 1 ? N1 : NF;
        const int base = t - id * stride;
        const double g2 = A.geo[e * 4 + d];  // uniform: a scalar load
        if (MIX) {
            const float* Dh = sD32 + id * N1;
            const float* Dl = sD32 + N1 * N1 + id * N1;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const float* F = reinterpret_cast<const float*>(sW) + (plane * 5 + v) * NP + base;
                float ah = 0.0f, al = 0.0f;
#pragma unroll
                for (int m = 0; m < N1; ++m) {
                    const float fv = F[m * stride];
                    ah = fmaf(Dh[m], fv, ah);
                    al = fmaf(Dl[m], fv, al);
                }
                R[v] = fma(-g2, (double)ah + (double)al, R[v]);
            }
        } else {
            const double* Drow = D + id * N1;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double* F = sW + (plane * 5 + v) * NP + base;
                double acc = 0.0;
#pragma unroll
                for (int m = 0; m < N1; ++m) acc = fma(Drow[m], F[m * stride], acc);
                R[v] = fma(-g2, acc, R[v]);
            }
        }
    };
    // float64: the contraction by lines.  One task per (variable, line along d) reads
    // the line's N+1 fluxes once, forms the N+1 sums of D F along it (D from the
    // uniform operator table: scalar operands) and writes them over the line in
    // place (lines are disjoint); after a barrier every node adds -(2/h_d) times its
    // own sum.  The same fma chains as a per-node contraction, with a fifth of its
    // LDS reads and no per-lane reads of D, which sits in scalar registers: for
    // N <= 4 (at higher orders D and the line no longer fit the register budget,
    // and the per-node contraction below is used).
    constexpr bool LINES = !MIX && N <= 4;
    auto lines = [&](int d, int plane) {
        const int stride = d == 0 ? 1 : d == 1 ? N1 : NF;
        for (int task = t; task < 5 * NF; task += NT) {
            const int v = task / NF, l = task - v * NF;
            const int base = d == 0 ? N1 * l : d == 1 ? (l % N1) + NF * (l / N1) : l;
            double* const F = sW + (plane * 5 + v) * NP + base;
            double f[N1];
#pragma unroll
            for (int m = 0; m < N1; ++m) f[m] = F[m * stride];
#pragma unroll
            for (int o = 0; o < N1; ++o) {
                double acc = 0.0;
#pragma unroll
                for (int m = 0; m < N1; ++m) acc = fma(A.ops[o * N1 + m], f[m], acc);
                F[o * stride] = acc;
            }
        }
    };
    auto gather_line_sums = [&](int d, int plane) {
        const double g2 = A.geo[e * 4 + d];  // uniform: a scalar load
        const double* const S = sW + plane * 5 * NP + t;
#pragma unroll
        for (int v = 0; v < 5; ++v) R[v] = fma(-g2, S[v * NP], R[v]);
    };
    if constexpr (LINES) {
        if (ALL3) {
            if (t < NP) {
                put_flux(0, 0);
                put_flux(1, 1);
                put_flux(2, 2);
            }
            __syncthreads();
            lines(0, 0);
            lines(1, 1);
            lines(2, 2);
            __syncthreads();
            if (t < NP) {
                gather_line_sums(0, 0);
                gather_line_sums(1, 1);
                gather_line_sums(2, 2);
            }
        } else if (StageLds<N, MIX>::PLANES == 10) {
            if (t < NP) {
                put_flux(0, 0);
                put_flux(1, 1);
            }
            __syncthreads();
            lines(0, 0);
            lines(1, 1);
            __syncthreads();
            if (t < NP) {
                gather_line_sums(0, 0);
                gather_line_sums(1, 1);
                put_flux(2, 0);  // the node's own entries: read above, then overwritten
            }
            __syncthreads();
            lines(2, 0);
            __syncthreads();
            if (t < NP) gather_line_sums(2, 0);
        } else {
            if (t < NP) put_flux(0, 0);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                __syncthreads();
                lines(d, 0);
                __syncthreads();
                if (t < NP) {
                    gather_line_sums(d, 0);
                    if (d < 2) put_flux(d + 1, 0);
                }
            }
        }
    } else if (ALL3) {
        if (t < NP) {
            put_flux(0, 0);
            put_flux(1, 1);
            put_flux(2, 2);
        }
        __syncthreads();
        if (t < NP) {
            contract(0, 0);
            contract(1, 1);
            contract(2, 2);
        }
    } else if (StageLds<N, MIX>::PLANES == 10) {
        if (t < NP) {
            put_flux(0, 0);
            put_flux(1, 1);
        }
        __syncthreads();
        if (t < NP) {
            contract(0, 0);
            contract(1, 1);
        }
        __syncthreads();
        if (t < NP) put_flux(2, 0);
        __syncthreads();
        if (t < NP) contract(2, 0);
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (d > 0) __syncthreads();
            if (t < NP) put_flux(d, 0);
            __syncthreads();
            if (t < NP) contract(d, 0);
        }
    }

    if (t >= NP) return;
    // ---- lift: subtract the face contributions at the face nodes, x then y then z
    // (a node lies on at most one face per axis; off the faces of an axis it reads a
    // valid slot and subtracts 0, so no branches)
    {
        const double* px = sS + (i == N ? 5 : 0) * NF + j + N1 * k;
        const double* py = sS + (j == N ? 15 : 10) * NF + i + N1 * k;
        const double* pz = sS + (k == N ? 25 : 20) * NF + i + N1 * j;
        // R - w a with w = 1 on a face of the axis and 0 off it: one fma per term
        // (exactly R - a, or R), one select per axis
        const double wx = (i == 0 || i == N) ? -1.0 : -0.0;
        const double wy = (j == 0 || j == N) ? -1.0 : -0.0;
        const double wz = (k == 0 || k == N) ? -1.0 : -0.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) R[v] = fma(wx, px[v * NF], R[v]);
#pragma unroll
        for (int v = 0; v < 5; ++v) R[v] = fma(wy, py[v * NF], R[v]);
#pragma unroll
        for (int v = 0; v < 5; ++v) R[v] = fma(wz, pz[v * NF], R[v]);
    }
    const int64_t base = e * NP + t;
    if (MODE == MODE_RHS) {
#pragma unroll
        for (int v = 0; v < 5; ++v) A.out[v * KNP + base] = R[v];
    } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double o = A.b * fma(A.dt, R[v], q[v]);
            if (use_q0) o = fma(A.a, q0v[v], o);
            if constexpr (MODE == MODE_RK_STREAM)
                __builtin_nontemporal_store(o, A.out + v * KNP + base);
            else
                A.out[v * KNP + base] = o;
        }
    }
}

// ---------------------------------------------------------------- adjoint (transpose of k_stage)

// qbar += J^T a for the flux sgn F^D at a node (a = weights on the 5 flux
// components); rinv = 1/rho, ud = q[1+D] rinv, Th = Thetabar + Theta',
// dPdT = dP'/dTheta' = gamma P / Th
template <int D>
__device__ __forceinline__ void flux_vjp(const double q[5], double rinv, double ud, double Th, double dPdT,
                                         const double a[5], double g[5]) {
    const double ubar = a[1] * q[1] + a[2] * q[2] + a[3] * q[3] + a[4] * Th;
    g[1 + D] += a[0] + ubar * rinv;
    g[1] += a[1] * ud;
    g[2] += a[2] * ud;
    g[3] += a[3] * ud;
    g[4] += a[4] * ud + a[1 + D] * dPdT;
    g[0] -= ubar * ud * rinv;
}

struct NodeState {
    double rinv, ud, Th, dPdT, lam;
    double dlam0, dlamU, dlam4;  // d lam / d q0, d q[1+D], d q4
};

// pointwise state for axis D: u_D, wave speed lam = |u_D| + c and its gradient
// (d|x|/dx = 0 at x = 0)
template <int D>
__device__ __forceinline__ NodeState node_state(const double q[5], const Bg& b, double Pp, double gamma) {
    NodeState s;
    const double rho = b.rho + q[0];
    s.rinv = rcp_pos(rho);
    s.ud = q[1 + D] * s.rinv;
    s.Th = b.Th + q[4];
    const double P = b.P + Pp;
    s.dPdT = gamma * P / s.Th;
    const double c = sqrt_pos(gamma * P * s.rinv);
    const double au = fabs(s.ud);
    const double su = s.ud > 0.0 ? 1.0 : (s.ud < 0.0 ? -1.0 : 0.0);
    s.lam = au + c;
    s.dlam0 = -(au + 0.5 * c) * s.rinv;
    s.dlamU = su * s.rinv;
    s.dlam4 = 0.5 * gamma * c / s.Th;
    return s;
}

// gL (and gR if non-null) = derivative of w . F*(qL, qR, sgn e_D) w.r.t. qL (qR);
// a max tie splits the derivative 1/2, 1/2
template <int D>
__device__ __forceinline__ void rusanov_vjp(const double qL[5], const Bg& bL, double PpL, const double qR[5],
                                            const Bg& bR, double PpR, double sgn, double gamma, const double w[5],
                                            double gL[5], double* gR) {
    const NodeState L = node_state<D>(qL, bL, PpL, gamma);
    const NodeState Rr = node_state<D>(qR, bR, PpR, gamma);
    const double hl = 0.5 * fmax(L.lam, Rr.lam);
    const double tL = L.lam > Rr.lam ? 1.0 : (L.lam < Rr.lam ? 0.0 : 0.5);
    double wj = 0.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) wj += w[v] * (qL[v] - qR[v]);
    double a[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) a[v] = 0.5 * sgn * w[v];
#pragma unroll
    for (int v = 0; v < 5; ++v) gL[v] = hl * w[v];
    flux_vjp<D>(qL, L.rinv, L.ud, L.Th, L.dPdT, a, gL);
    const double cL = 0.5 * wj * tL;
    gL[0] += cL * L.dlam0;
    gL[1 + D] += cL * L.dlamU;
    gL[4] += cL * L.dlam4;
    if (gR) {
#pragma unroll
        for (int v = 0; v < 5; ++v) gR[v] = -hl * w[v];
        flux_vjp<D>(qR, Rr.rinv, Rr.ud, Rr.Th, Rr.dPdT, a, gR);
        const double cR = 0.5 * wj * (1.0 - tL);
        gR[0] += cR * Rr.dlam0;
        gR[1 + D] += cR * Rr.dlamU;
        gR[4] += cR * Rr.dlam4;
    }
}

// g += J^T (lift lam) for the own flux term -(-lift F(q).n) of the lift
template <int D>
__device__ __forceinline__ void own_flux_vjp(const double q[5], const Bg& b, double Pp, double sgn, double gamma,
                                             double lift, const double lam[5], double g[5]) {
    const NodeState S = node_state<D>(q, b, Pp, gamma);
    double a[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) a[v] = lift * sgn * lam[v];
    flux_vjp<D>(q, S.rinv, S.ud, S.Th, S.dPdT, a, g);
}

// Transposed mortar pre-pass (the transpose of k_mortar's three steps, one hanging
// face per workgroup).  With w = -lift_f lam_f + lift_c (R_a^T x R_b^T) lam_c at a
// mortar point, w . F*(q_f, q_m, n_f) is the part of <lam, R> that the point
// carries; its gradient with respect to the fine state goes to the fine face
// (with the fine side's own-flux term), its gradient with respect to the mortar
// state q_m = (I_a x I_b) q_c goes back to the coarse face through I_a^T x I_b^T
// (with the coarse side's own-flux term).  F*(q_m, q_f, n_c) = -F*(q_f, q_m, n_f)
// and the coarse side's weight is -w, so one VJP serves both sides.  Output per
// hanging face h: mort[h][0] the coarse face, mort[h][1 + quad] the fine faces,
// each [5][NF], added to qbar by the adjoint kernel.
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_mortar_adjoint(const MortAdjArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    constexpr int NOPS = Sz<N>::NOPS + 4 * NF;
    static_assert(4 * NF <= NT, "one mortar point per thread");
    // sT [10][NF]: coarse q (0..4) and lam (5..9); sU [20][NF]; sMq [40][NF]: per
    // quadrant q_m (0..4) and R^T lam (5..9), later the mortar-state gradient; sG [10][NF]
    __shared__ double sT[10 * NF], sU[20 * NF], sMq[40 * NF], sG[10 * NF];
    __shared__ double sOps[NOPS];
    __shared__ double sBg[4 * N1];  // the coarse leaf's background, with 1/Theta
    auto IT = [&](int a) { return sOps + 5 * NF + N1 + a * NF; };
    auto RT = [&](int a) { return sOps + 7 * NF + N1 + a * NF; };
    const int64_t h = xcd_remap(blockIdx.x, gridDim.x);
    const int t = threadIdx.x;
    const int32_t* const row = A.hang + h * 6;
    const int64_t ec = row[0];
    const int f = row[1], fo = f ^ 1;
    const int KNP = (int)(A.K * NP), KN1 = (int)(A.K * N1);
    const double gamma = A.gamma;
    const double liftc = 0.5 * N * (N + 1);   // 1/w_N
    const double sgn_c = (f & 1) ? 1.0 : -1.0;  // the coarse leaf's outward normal
    for (int ii = t; ii < NOPS; ii += NT) sOps[ii] = A.ops[ii];
    if (t < 3 * N1) {
        const double v = A.bg[(t / N1) * KN1 + ec * N1 + (t % N1)];
        sBg[t] = v;
        if (t >= N1 && t < 2 * N1) sBg[2 * N1 + t] = 1.0 / v;
    }
    for (int it = t; it < 5 * NF; it += NT) {
        const int v = it / NF, m = it % NF;
        const int off = v * KNP + (int)ec * NP + face_node<N>(f, m);
        sT[it] = A.q[off];
        sT[5 * NF + it] = A.lam[off];
    }
    // this thread's fine-side point and the lift factors, loaded with the coarse trace
    // (every global read of the workgroup is in this one batch): quadrant t / NF
    double qF[5] = {0, 0, 0, 0, 0}, lF[5] = {0, 0, 0, 0, 0};
    Bg bF{1.0, 1.0, 1.0, 1.0};
    double lift_f = 0.0;
    const double lift_c = A.geo[ec * 4 + (f >> 1)] * liftc;
    if (t < 4 * NF) {
        const int quad = t / NF, m = t % NF;
        const int64_t ef = row[2 + quad];
        const int nn = face_node<N>(fo, m), kn = face_k<N>(fo, m);
        bF = bg_make(A.bg[ef * N1 + kn], A.bg[KN1 + ef * N1 + kn], A.bg[2 * KN1 + ef * N1 + kn]);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qF[v] = A.q[v * KNP + ef * NP + nn];
            lF[v] = A.lam[v * KNP + ef * NP + nn];
        }
        lift_f = A.geo[ef * 4 + (f >> 1)] * liftc;
    }
    __syncthreads();
    // sU plane a*10 + c: along t1 with I_a (c < 5, state) or R_a^T (c >= 5, lambda)
    apply_t1<N>(sT, sU, 20, [&](int p) { return (p % 10) < 5 ? sOps + (1 + p / 10) * NF : RT(p / 10); },
                [](int p) { return p % 10; }, t, NT);
    __syncthreads();
    // sMq plane quad*10 + c, quad = a + 2b: along t2 with I_b or R_b^T
    apply_t2<N>(sU, sMq, 40, [&](int p) { return (p % 10) < 5 ? sOps + (1 + (p / 10) / 2) * NF : RT((p / 10) / 2); },
                [](int p) { return ((p / 10) & 1) * 10 + p % 10; }, t, NT);
    __syncthreads();
    if (t < 4 * NF) {
        const int quad = t / NF, m = t % NF;
        double qM[5], w[5], gF[5], gM[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qM[v] = sMq[(quad * 10 + v) * NF + m];
            w[v] = -lift_f * lF[v] + lift_c * sMq[(quad * 10 + 5 + v) * NF + m];
        }
        const double PpF = pprime(qF[4], bF.rTh, bF.P, gamma, A.binom);
        const double PpM = pprime(qM[4], bF.rTh, bF.P, gamma, A.binom);
        with_axis(f >> 1, [&](auto dc) {
            constexpr int d = decltype(dc)::value;
            rusanov_vjp<d>(qF, bF, PpF, qM, bF, PpM, -sgn_c, gamma, w, gF, gM);
            own_flux_vjp<d>(qF, bF, PpF, -sgn_c, gamma, lift_f, lF, gF);
        });
        double* const out = A.mort + ((h * 5 + 1 + quad) * 5) * NF + m;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            out[v * NF] = gF[v];
            sMq[(quad * 10 + v) * NF + m] = gM[v];  // in place: the mortar-state gradient
        }
    }
    __syncthreads();
    // back to the coarse face: sum_ab (I_a^T x I_b^T) gM_ab, first along t1 then t2
    for (int it = t; it < 10 * NF; it += NT) {
        const int p = it / NF, r = it % NF, bb = r / N1, a2 = r % N1;
        const int qb = p / 5, v = p % 5;
        double acc = 0.0;
#pragma unroll
        for (int qa = 0; qa < 2; ++qa) {
            const double* Op = IT(qa) + a2 * N1;
            const double* x = sMq + ((qa + 2 * qb) * 10 + v) * NF + bb * N1;
#pragma unroll
            for (int a = 0; a < N1; ++a) acc = fma(Op[a], x[a], acc);
        }
        sG[it] = acc;
    }
    __syncthreads();
    for (int it = t; it < 5 * NF; it += NT) {
        const int v = it / NF, m = it % NF, b2 = m / N1, a = m % N1;
        double acc = 0.0;
#pragma unroll
        for (int qb = 0; qb < 2; ++qb) {
            const double* Op = IT(qb) + b2 * N1;
            const double* x = sG + (qb * 5 + v) * NF + a;
#pragma unroll
            for (int bb = 0; bb < N1; ++bb) acc = fma(Op[bb], x[bb * N1], acc);
        }
        sU[it] = acc;
    }
    __syncthreads();
    if (t < NF) {
        const int m = t, kk = face_k<N>(f, m);
        const Bg b{sBg[kk], sBg[N1 + kk], sBg[2 * N1 + kk], sBg[3 * N1 + kk]};
        double qL[5], lL[5], g[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qL[v] = sT[v * NF + m];
            lL[v] = sT[(5 + v) * NF + m];
            g[v] = sU[v * NF + m];
        }
        const double PpL = pprime(qL[4], b.rTh, b.P, gamma, A.binom);
        with_axis(f >> 1, [&](auto dc) {
            own_flux_vjp<decltype(dc)::value>(qL, b, PpL, sgn_c, gamma, lift_c, lL, g);
        });
        double* const out = A.mort + (h * 5 * 5) * NF + m;
#pragma unroll
        for (int v = 0; v < 5; ++v) out[v * NF] = g[v];
    }
}

// the adjoint keeps more state per node; bound it less tightly than the forward
// (with the mortars in their own pre-pass, N = 7 fits 4 waves per SIMD: two
// workgroups of 8 waves per CU)
template <int N, bool MIX>
struct AdjOcc {
    static constexpr int W = N >= 6 ? 4 : 3;
};

// MIX: the transposed volume contractions D^T lam in float32 (lambda tile rounded
// to float32, D split into float32 high and low parts, float32 accumulation); the
// faces read lambda from memory in float64, and everything else stays float64.
template <int N, int MODE, bool MIX>
__global__ void __launch_bounds__(Sz<N>::NT) __attribute__((amdgpu_waves_per_eu(AdjOcc<N, MIX>::W)))
k_adjoint(const AdjArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    constexpr int NOPS = N1 * N1;  // D
    __shared__ double sL[MIX ? (5 * NP + 1) / 2 : 5 * NP];  // lambda tile (MIX: float)
    __shared__ float sD32[MIX ? 2 * N1 * N1 : 1];            // MIX: D high and low parts
    float* const sLf = reinterpret_cast<float*>(sL);
    __shared__ double sPp[NP];
    __shared__ double sS[30 * NF];       // face contributions to qbar
    __shared__ double sOps[NOPS];
    __shared__ double sBg[4 * N1];  // rho, Theta, P, 1/Theta of the background
    __shared__ int sType[6];
    __shared__ int sNb[24];
    __shared__ int sHs[6];          // hanging face: row of the transposed mortar pre-pass
    const double* D = sOps;

    const int64_t K = A.K;
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int t = threadIdx.x;
    const double gamma = A.gamma;
    const int KNP = (int)(K * NP);
    const int KN1 = (int)(K * N1);
    const double* const qs = A.q;
    const double* const ls = A.lam;
    const double* const qe = qs + e * NP;
    const double* const le = ls + e * NP;
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;

    for (int ii = t; ii < NOPS; ii += NT) sOps[ii] = A.ops[ii];
    if (MIX)
        for (int ii = t; ii < N1 * N1; ii += NT) {
            const double dv = A.ops[ii];
            const float hi = (float)dv;
            sD32[ii] = hi;
            sD32[N1 * N1 + ii] = (float)(dv - (double)hi);
        }
    if (t < 3 * N1) {
        const double v = A.bg[(t / N1) * KN1 + e * N1 + (t % N1)];
        sBg[t] = v;
        if (t >= N1 && t < 2 * N1) sBg[2 * N1 + t] = 1.0 / v;
    }
    if (t < 6) sType[t] = A.ftype[e * 6 + t];
    if (t < 24) sNb[t] = A.fnb[e * 24 + t];
    if (t < 6) sHs[t] = A.hslot[e * 6 + t];
    double q[5] = {0, 0, 0, 0, 0}, lam[5] = {0, 0, 0, 0, 0};
    if (t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            q[v] = qe[v * KNP + t];
            lam[v] = le[v * KNP + t];
            if (MIX)
                sLf[v * NP + t] = (float)lam[v];
            else
                sL[v * NP + t] = lam[v];
        }
        sPp[t] = pprime(q[4], 1.0 / A.bg[KN1 + e * N1 + k], A.bg[2 * KN1 + e * N1 + k], gamma, A.binom);
    }
    __syncthreads();

    const double liftc = 0.5 * N * (N + 1);
    // ---- conforming faces and walls; items grouped by axis, each axis padded to
    // whole waves (a wave never mixes the three axis variants)
    constexpr int PAD = ((2 * NF + 63) / 64) * 64;
#pragma unroll
    for (int it = t; it < 3 * PAD; it += NT) {
        const int ax = it / PAD, r = it % PAD;
        if (r >= 2 * NF) continue;
        const int f = 2 * ax + r / NF, m = r % NF;
        const int tf = sType[f], type = tf & 0xff;
        if (type == FT_FINE || type == FT_COARSE) {
            // hanging face: the transposed mortar pre-pass holds this side's contribution
            const int64_t row = (int64_t)sHs[f] * 5 + (type == FT_COARSE ? 0 : 1 + ((tf >> 8) & 0xff));
#pragma unroll
            for (int v = 0; v < 5; ++v) sS[(f * 5 + v) * NF + m] = A.mort[(row * 5 + v) * NF + m];
            continue;
        }
        const double sgn = (f & 1) ? 1.0 : -1.0;
        const int n = face_node<N>(f, m), kk = face_k<N>(f, m);
        const double lift = A.geo[e * 4 + ax] * liftc;
        with_axis(ax, [&](auto dc) {
            constexpr int d = decltype(dc)::value;
            double qL[5], lL[5], qR[5], w[5], g[5], gR[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                qL[v] = qe[v * KNP + n];
                lL[v] = MIX ? le[v * KNP + n] : sL[v * NP + n];
            }
            const Bg bL{sBg[kk], sBg[N1 + kk], sBg[2 * N1 + kk], sBg[3 * N1 + kk]};
            const double PpL = sPp[n];
            if (type == FT_WALL) {
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    qR[v] = qL[v];
                    w[v] = -lift * lL[v];
                }
                qR[1 + d] = -qL[1 + d];
                rusanov_vjp<d>(qL, bL, PpL, qR, bL, PpL, sgn, gamma, w, g, gR);
                gR[1 + d] = -gR[1 + d];  // transpose of the mirror map
#pragma unroll
                for (int v = 0; v < 5; ++v) g[v] += gR[v];
            } else {
                const int nb = sNb[f * 4];
                const int nn = face_node<N>(f ^ 1, m), kn = face_k<N>(f ^ 1, m);
                const double liftn = A.geo[nb * 4 + (f >> 1)] * liftc;
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    qR[v] = qs[v * KNP + nb * NP + nn];
                    w[v] = -lift * lL[v] + liftn * ls[v * KNP + nb * NP + nn];
                }
                // same background as this side except across a periodic wrap along z
                const Bg bR = (sType[f] & FT_BG_NB)
                                  ? bg_make(A.bg[nb * N1 + kn], A.bg[KN1 + nb * N1 + kn], A.bg[2 * KN1 + nb * N1 + kn])
                                  : bL;
                const double PpR = pprime(qR[4], bR.rTh, bR.P, gamma, A.binom);
                rusanov_vjp<d>(qL, bL, PpL, qR, bR, PpR, sgn, gamma, w, g, nullptr);
            }
            own_flux_vjp<d>(qL, bL, PpL, sgn, gamma, lift, lL, g);
#pragma unroll
            for (int v = 0; v < 5; ++v) sS[(f * 5 + v) * NF + m] = g[v];
        });
    }

    __syncthreads();

    if (t >= NP) return;
    // ---- volume: a^d = -(2/h_d) D_d^T lam, then the pointwise chain rule
    double g[5] = {0, 0, 0, 0, 0};
    {
        const double rhob = sBg[k], Thb = sBg[N1 + k], Pb = sBg[2 * N1 + k];
        const double rinv = 1.0 / (rhob + q[0]);
        const double Th = Thb + q[4];
        const double dPdT = gamma * (Pb + sPp[t]) / Th;
        const double vel[3] = {q[1] * rinv, q[2] * rinv, q[3] * rinv};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int id = d == 0 ? i : d == 1 ? j : k;
            const int stride = d == 0 ? 1 : d == 1 ? N1 : NF;
            const int base = t - id * stride;
            const double g2 = A.geo[e * 4 + d];
            double a[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                if (MIX) {
                    const float* Lp = sLf + v * NP + base;
                    float ah = 0.0f, al = 0.0f;
#pragma unroll
                    for (int m = 0; m < N1; ++m) {
                        const float lv = Lp[m * stride];
                        ah = fmaf(sD32[m * N1 + id], lv, ah);
                        al = fmaf(sD32[N1 * N1 + m * N1 + id], lv, al);
                    }
                    a[v] = -g2 * ((double)ah + (double)al);
                } else {
                    const double* Lp = sL + v * NP + base;
                    double acc = 0.0;
#pragma unroll
                    for (int m = 0; m < N1; ++m) acc = fma(D[m * N1 + id], Lp[m * stride], acc);
                    a[v] = -g2 * acc;
                }
            }
            if (d == 0) flux_vjp<0>(q, rinv, vel[0], Th, dPdT, a, g);
            if (d == 1) flux_vjp<1>(q, rinv, vel[1], Th, dPdT, a, g);
            if (d == 2) flux_vjp<2>(q, rinv, vel[2], Th, dPdT, a, g);
        }
        g[0] -= A.g * lam[3];  // buoyancy -rho' g on rho*w
    }
    // ---- faces that touch this node, x then y then z (at most one face per axis;
    // off the faces of an axis a valid slot is read and 0 added: no branches)
    {
        const double* px = sS + (i == N ? 5 : 0) * NF + j + N1 * k;
        const double* py = sS + (j == N ? 15 : 10) * NF + i + N1 * k;
        const double* pz = sS + (k == N ? 25 : 20) * NF + i + N1 * j;
        const bool ox = i == 0 || i == N, oy = j == 0 || j == N, oz = k == 0 || k == N;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double a = px[v * NF];
            g[v] += ox ? a : 0.0;
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double a = py[v * NF];
            g[v] += oy ? a : 0.0;
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double a = pz[v * NF];
            g[v] += oz ? a : 0.0;
        }
    }
    const int64_t base = e * NP + t;
    if (MODE == MODE_RHS) {
#pragma unroll
        for (int v = 0; v < 5; ++v) A.out[v * KNP + base] = g[v];
    } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double o = A.b * fma(A.dt, g[v], lam[v]);
            if (A.a1 != 0.0) o = fma(A.a1, A.w1[v * KNP + base], o);
            if (A.a2 != 0.0) o = fma(A.a2, A.w2[v * KNP + base], o);
            A.out[v * KNP + base] = o;
        }
    }
}

// ---------------------------------------------------------------- background, IC, coordinates

__global__ void k_background(int64_t K, int N1, const double* c1d, double* bg, BgParams p) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= K * N1) return;
    const double z = c1d[2 * K * N1 + idx];
    const double R = p.cp - p.cv, gamma = p.cp / p.cv;
    double rho, Th;
    if (p.kind == DG_BG_ISOTHERMAL) {
        // temperature theta0: Pbar = P0 exp(-g z/(R theta0)), Thetabar from the equation of state
        const double Pb = p.P0 * exp(-p.g * z / (R * p.theta0));
        bg[idx] = Pb / (R * p.theta0);
        bg[K * N1 + idx] = (p.P0 / R) * pow(Pb / p.P0, 1.0 / gamma);
        bg[2 * K * N1 + idx] = Pb;
        return;
    }
    if (p.kind == DG_BG_NEUTRAL) {
        const double exner = 1.0 - p.g * z / (p.cp * p.theta0);
        rho = p.P0 * pow(exner, p.cv / R) / (R * p.theta0);
        Th = rho * p.theta0;
    } else {
        rho = p.rho0;
        Th = p.Theta0;
    }
    bg[idx] = rho;
    bg[K * N1 + idx] = Th;
    bg[2 * K * N1 + idx] = p.P0 * pow(R * Th / p.P0, gamma);
}

__global__ void k_init_bell(int64_t K, int N1, const double* c1d, const double* bg, double theta0, dg_bell bell,
                            double* q) {
    const int64_t NP = (int64_t)N1 * N1 * N1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= K * NP) return;
    const int64_t e = idx / NP;
    const int n = (int)(idx % NP);
    const int ii[3] = {n % N1, (n / N1) % N1, n / (N1 * N1)};
    double r2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (bell.radius[d] > 0.0) {
            const double s = (c1d[(int64_t)d * K * N1 + e * N1 + ii[d]] - bell.centre[d]) / bell.radius[d];
            r2 += s * s;
        }
    }
    const double r = sqrt(r2);
    const double thp = r <= 1.0 ? bell.dtheta * 0.5 * (1.0 + cos(M_PI * r)) : 0.0;
    const double rhob = bg[e * N1 + ii[2]];
    q[idx] = -rhob * thp / (theta0 + thp);
    for (int v = 1; v < 5; ++v) q[v * K * NP + idx] = 0.0;
}

__global__ void k_node_coords(int64_t K, int N1, const double* c1d, double* xyz) {
    const int64_t NP = (int64_t)N1 * N1 * N1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= K * NP) return;
    const int64_t e = idx / NP;
    const int n = (int)(idx % NP);
    const int ii[3] = {n % N1, (n / N1) % N1, n / (N1 * N1)};
    for (int d = 0; d < 3; ++d) xyz[d * K * NP + idx] = c1d[d * K * N1 + e * N1 + ii[d]];
}

// ---------------------------------------------------------------- transfer (section 3.3)

// A family is eight consecutive leaves, children 0..7 of one leaf (consecutive in
// Morton order, checked on the host): the targets of a refined leaf, or the
// sources of a merged parent.  Its nodes form one block of (2N+2)^3 points, fine
// index I = a (N+1) + i along each axis, a = the child's bit on that axis.
//
// k_family_reduce: one leaf = (A x A x A) applied to a family block, A an
//   (N+1) x (2N+2) matrix: coarsening, A = [R_0 | R_1]; transpose of refinement,
//   A = [I_0^T | I_1^T].
// Three separable passes; one workgroup per plan entry and field, so a merged
// family's work is spread over as many workgroups as it has fields; kept leaves
// are copied.  The block of a refined family is the one at child 0; the others
// return at once.  The opposite direction (one leaf to its children) is
// k_expand, one child and field per block.

// copy of a kept leaf, fields v0 .. v0 + nf - 1 (nf <= 5, all loads issued before the
// stores): forward q_to[e] = q_from[src]; transpose qbar_from[src] = qbar_to[e]
template <int N, bool ADJ>
__device__ __forceinline__ void xfer_copy(const XferArgs& A, int64_t e, int64_t src, int v0, int nf, int t) {
    constexpr int NP = Sz<N>::NP;
    const int64_t li = ADJ ? e : src, lo = ADJ ? src : e;
    if (t >= NP) return;
    double x[5];
#pragma unroll
    for (int f = 0; f < 5; ++f)
        if (f < nf) x[f] = A.qin[(v0 + f) * A.Kin * NP + li * NP + t];
#pragma unroll
    for (int f = 0; f < 5; ++f)
        if (f < nf) A.qout[(v0 + f) * A.Kout * NP + lo * NP + t] = x[f];
}

// field blockIdx.y of one plan entry per workgroup
template <int N, bool ADJ>
__global__ void __launch_bounds__(Sz<N>::NT) k_family_reduce(const XferArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    constexpr int M = 2 * N1;
    __shared__ double sF[M * M * M];   // family block; reused by the second pass's output
    __shared__ double s1[N1 * M * M];
    __shared__ double sA[N1 * M];      // sA[i M + m]
    double* const s2 = sF;             // [M][N1][N1]
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int v = (int)blockIdx.y;
    const int t = threadIdx.x;
    const int64_t src = A.src[e];
    const int kind = A.kind[e];
    if (kind == DG_KIND_COPY) {  // uniform over the block: every field, by the block of field 0
        if (v == 0) xfer_copy<N, ADJ>(A, e, src, 0, A.nvar, t);
        return;
    }
    if (ADJ && kind != 0) return;  // refined family: handled by the block of child 0
    const int64_t fine0 = ADJ ? e : src, lo = ADJ ? src : e;
    const int64_t KinNP = A.Kin * NP, KoutNP = A.Kout * NP;
    const int ic = t % N1, jc = (t / N1) % N1, kc = t / NF;
    // the eight children's values at this node, requested before the operator is staged
    double pf[8];
    if (t < NP)
#pragma unroll
        for (int c = 0; c < 8; ++c) pf[c] = A.qin[v * KinNP + (fine0 + c) * NP + t];
    for (int x = t; x < N1 * M; x += NT) {
        const int i = x / M, m = x % M, h = m / N1, r = m % N1;
        sA[x] = ADJ ? A.ops[(1 + h) * NF + r * N1 + i]    // I_h^T[i][r]
                    : A.ops[(3 + h) * NF + i * N1 + r];   // R_h[i][r]
    }
    if (t < NP)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int I = (c & 1) * N1 + ic, J = ((c >> 1) & 1) * N1 + jc, Kf = (c >> 2) * N1 + kc;
            sF[(Kf * M + J) * M + I] = pf[c];
        }
    __syncthreads();
    // x: s1[K'][J'][i] = sum_m A[i][m] F[K'][J'][m]
    for (int x = t; x < N1 * M * M; x += NT) {
        const int i = x % N1, row = x / N1;
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < M; ++m) acc = fma(sA[i * M + m], sF[row * M + m], acc);
        s1[x] = acc;
    }
    __syncthreads();
    // y: s2[K'][j][i] = sum_m A[j][m] s1[K'][m][i]
    for (int x = t; x < N1 * N1 * M; x += NT) {
        const int i = x % N1, j = (x / N1) % N1, kk = x / NF;
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < M; ++m) acc = fma(sA[j * M + m], s1[(kk * M + m) * N1 + i], acc);
        s2[x] = acc;
    }
    __syncthreads();
    // z: out[k][j][i] = sum_m A[k][m] s2[m][j][i]
    if (t < NP) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < M; ++m) acc = fma(sA[kc * M + m], s2[m * NF + ic + N1 * jc], acc);
        A.qout[v * KoutNP + lo * NP + t] = acc;
    }
}

// One child of a family per workgroup: child c = (a, b, c') of leaf li gets
// (B_a x B_b x B_c') applied to it, three separable passes: refinement,
// B_h = I_h (grid over the plan's child entries); transpose of coarsening,
// B_h = R_h^T (grid over the plan's entries x 8 children).  Kept leaves are
// copied (by the blocks of child index 0).  FB fields per workgroup (grid z over
// the groups of FB fields), their loads issued together and every pass run over
// all FB at once, so a workgroup has FB times the bytes in flight and the same
// three barriers; the kernel is bound by the bytes in flight per CU (the counters
// show exactly the algorithmic traffic).  (One workgroup per family producing all
// eight children, with the leaf read once, measured slower: 2576 such workgroups
// of the density current against 20608.)
template <int N, bool ADJ, int FB>
__global__ void __launch_bounds__(Sz<N>::NT) k_expand(const XferArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    __shared__ double sIn[FB * NP], s1[FB * NP];  // the second pass writes over sIn
    __shared__ double sM[3 * NF];  // the 1-D operator along x, y, z: sM[d NF + r (N+1) + col]
    double* const s2 = sIn;
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int v0 = (int)blockIdx.z * FB;
    const int nf = A.nvar - v0 < FB ? A.nvar - v0 : FB;
    const int t = threadIdx.x;
    const int64_t src = A.src[e];
    const int kind = A.kind[e];
    if (kind == DG_KIND_COPY) {  // uniform over the block
        if (blockIdx.y == 0) xfer_copy<N, ADJ>(A, e, src, v0, nf, t);
        return;
    }
    int c;
    int64_t li, lo;
    if (!ADJ) {  // refined leaf src: this entry is its child `kind`
        if (kind < 0 || kind > 7) return;
        c = kind;
        li = src;
        lo = e;
    } else {  // merged parent e: its child blockIdx.y is source leaf src + c
        if (kind != DG_KIND_FAMILY) return;
        c = (int)blockIdx.y;
        li = e;
        lo = src + c;
    }
    const int64_t KinNP = A.Kin * NP, KoutNP = A.Kout * NP;
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;
    double p[FB];  // requested before the operator is staged
#pragma unroll
    for (int f = 0; f < FB; ++f) p[f] = (t < NP && f < nf) ? A.qin[(v0 + f) * KinNP + li * NP + t] : 0.0;
    for (int x = t; x < 3 * NF; x += NT) {
        const int d = x / NF, r = (x % NF) / N1, col = x % N1, h = (c >> d) & 1;
        sM[x] = ADJ ? A.ops[(3 + h) * NF + col * N1 + r]    // R_h^T[r][col]
                    : A.ops[(1 + h) * NF + r * N1 + col];   // I_h[r][col]
    }
    if (t < NP)
#pragma unroll
        for (int f = 0; f < FB; ++f) sIn[f * NP + t] = p[f];
    __syncthreads();
    if (t < NP)
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < N1; ++m) acc = fma(sM[i * N1 + m], sIn[f * NP + m + N1 * (j + N1 * k)], acc);
            s1[f * NP + t] = acc;
        }
    __syncthreads();
    if (t < NP)
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < N1; ++m) acc = fma(sM[NF + j * N1 + m], s1[f * NP + i + N1 * (m + N1 * k)], acc);
            s2[f * NP + t] = acc;
        }
    __syncthreads();
    if (t < NP)
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            if (f >= nf) break;
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < N1; ++m) acc = fma(sM[2 * NF + k * N1 + m], s2[f * NP + i + N1 * (j + N1 * m)], acc);
            A.qout[(v0 + f) * KoutNP + lo * NP + t] = acc;
        }
}

// fields per k_expand workgroup: all five (measured: density current refine
// 65 -> 47 us, AMR bubble 41 -> 36 us against one field per workgroup)
template <int N>
constexpr int expand_fields() { return 5; }

// ---------------------------------------------------------------- budgets

template <int N>
__global__ void __launch_bounds__(256) k_budgets(const BudgetArgs A) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1;
    constexpr int NT = 256;
    __shared__ Comp sh[4 * NT];
    const int t = threadIdx.x;
    const int64_t K = A.K;
    const double gamma = A.gamma;
    Comp acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    // each block handles a contiguous range of leaves; thread t covers nodes t, t+NT, ...
    const int64_t per = (K + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = blockIdx.x * per, e1 = (e0 + per < K) ? e0 + per : K;
    for (int64_t e = e0; e < e1; ++e) {
        const double J = A.geo[e * 4 + 3];
        for (int n = t; n < NP; n += NT) {
            const int i = n % N1, j = (n / N1) % N1, k = n / (N1 * N1);
            const double W = (A.Jn ? A.Jn[e * NP + n] : J) * A.w[i] * A.w[j] * A.w[k];
            const double rp = A.q[e * NP + n];
            const double U = A.q[K * NP + e * NP + n], V = A.q[2 * K * NP + e * NP + n],
                         Wm = A.q[3 * K * NP + e * NP + n], Thp = A.q[4 * K * NP + e * NP + n];
            const double rhob = A.bg[e * N1 + k], Thb = A.bg[K * N1 + e * N1 + k], Pb = A.bg[2 * K * N1 + e * N1 + k];
            const double z = A.c1d[2 * K * N1 + e * N1 + k];
            const double rho = rhob + rp;
            const double P = Pb + pprime(Thp, 1.0 / Thb, Pb, gamma, A.binom);
            const double E = P / (gamma - 1.0) + (U * U + V * V + Wm * Wm) / (2.0 * rho) + rho * A.g * z;
            acc[0] = comp_add(acc[0], W * rp);
            acc[1] = comp_add(acc[1], W * rho);
            acc[2] = comp_add(acc[2], W * Thp);
            acc[3] = comp_add(acc[3], W * E);
        }
    }
    block_reduce4<NT>(acc, sh);
    if (t == 0)
        for (int q = 0; q < 4; ++q) {
            A.partial[(blockIdx.x * 4 + q) * 2 + 0] = acc[q].s;
            A.partial[(blockIdx.x * 4 + q) * 2 + 1] = acc[q].c;
        }
}

__global__ void __launch_bounds__(256) k_budgets_final(const double* partial, int nblk, double* out) {
    constexpr int NT = 256;
    __shared__ Comp sh[4 * NT];
    const int t = threadIdx.x;
    Comp acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int b = t; b < nblk; b += NT)
        for (int q = 0; q < 4; ++q)
            acc[q] = comp_merge(acc[q], Comp{partial[(b * 4 + q) * 2], partial[(b * 4 + q) * 2 + 1]});
    block_reduce4<NT>(acc, sh);
    if (t == 0)
        for (int q = 0; q < 4; ++q) out[q] = acc[q].s + acc[q].c;
}

// ---------------------------------------------------------------- indicator

template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_indicator(const IndArgs A) {
    constexpr int N1 = N + 1, NP = Sz<N>::NP, NT = Sz<N>::NT;
    __shared__ double sTh[NP];
    __shared__ double sD[N1 * N1];
    constexpr int P2 = NT <= 64 ? 64 : NT <= 128 ? 128 : NT <= 256 ? 256 : NT <= 512 ? 512 : 1024;
    __shared__ double sMax[P2];
    const int64_t e = blockIdx.x;
    const int64_t K = A.K;
    const int t = threadIdx.x;
    for (int i = t; i < N1 * N1; i += NT) sD[i] = A.ops[i];
    const int i = t % N1, j = (t / N1) % N1, k = t / (N1 * N1);
    double val = 0.0;
    if (t < NP) {
        const double rhob = A.bg[e * N1 + k], Thb = A.bg[K * N1 + e * N1 + k];
        const double rp = A.q[e * NP + t], Thp = A.q[4 * K * NP + e * NP + t];
        const double theta = (Thb + Thp) / (rhob + rp);
        sTh[t] = theta;
        val = fabs(theta - Thb / rhob);
        if (A.kind == DG_IND_PPRIME)
            val = fabs(pprime(Thp, 1.0 / Thb, A.bg[2 * K * N1 + e * N1 + k], A.gamma, A.binom));
    }
    __syncthreads();
    if (A.kind == DG_IND_GRAD_THETA && t < NP) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int m = 0; m < N1; ++m) {
            ax = fma(sD[i * N1 + m], sTh[m + N1 * (j + N1 * k)], ax);
            ay = fma(sD[j * N1 + m], sTh[i + N1 * (m + N1 * k)], ay);
            az = fma(sD[k * N1 + m], sTh[i + N1 * (j + N1 * m)], az);
        }
        ax *= A.geo[e * 4 + 0];
        ay *= A.geo[e * 4 + 1];
        az *= A.geo[e * 4 + 2];
        val = sqrt(ax * ax + ay * ay + az * az);
    }
    sMax[t] = (t < NP) ? val : 0.0;
    if (t + NT < P2) sMax[t + NT] = 0.0;
    __syncthreads();
    for (int w = P2 / 2; w > 0; w >>= 1) {
        if (t < w) {
            const double a = sMax[t], b = sMax[t + w];
            sMax[t] = (a != a || b != b) ? NAN : fmax(a, b);  // a NaN anywhere survives
        }
        __syncthreads();
    }
    if (t == 0) {
        const double eta = sMax[0];
        if (A.eta) A.eta[e] = eta;
        const int lev = A.level[e];
        int8_t fl = 0;
        if (eta > A.thr && lev < A.max_level) fl = 1;
        if (eta <= A.thr && lev > 0) fl = -1;
        A.flags[e] = fl;
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers

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

hipError_t launch_stage(int N, int mode, bool mixed, const StageArgs& a, hipStream_t s) {
    if (a.K <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.K);
    const bool stream = mode == MODE_RK && a.stream_io;
    // a == 0 (the first SSP-RK3 stage): q0 is not read, and the kernel without it
    // keeps the register count of the right-hand side (one more wave per SIMD)
    if (mode == MODE_RK && a.a == 0.0) {
        if (mixed) {
            DG_DISPATCH_N(N, (k_stage<NN, MODE_RK_NOQ0, true><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        } else {
            DG_DISPATCH_N(N, (k_stage<NN, MODE_RK_NOQ0, false><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        }
        return hipGetLastError();
    }
    if (mixed) {
        if (mode == MODE_RHS) {
            DG_DISPATCH_N(N, (k_stage<NN, MODE_RHS, true><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        } else if (stream) {
            DG_DISPATCH_N(N, (k_stage<NN, MODE_RK_STREAM, true><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        } else {
            DG_DISPATCH_N(N, (k_stage<NN, MODE_RK, true><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        }
    } else {
        if (mode == MODE_RHS) {
            DG_DISPATCH_N(N, (k_stage<NN, MODE_RHS, false><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        } else if (stream) {
            DG_DISPATCH_N(N, (k_stage<NN, MODE_RK_STREAM, false><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        } else {
            DG_DISPATCH_N(N, (k_stage<NN, MODE_RK, false><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        }
    }
    return hipGetLastError();
}

// float64 FMA rate calibration: 8 independent dependency chains per thread
__global__ void __launch_bounds__(256) k_fma_burst(int iters, double* sink) {
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double m = 0.9999999, c = 1e-7;
    double x[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = 1e-3 * (double)(threadIdx.x + r);
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = fma(x[r], m, c);
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) acc += x[r];
    sink[gid] = acc;
}

hipError_t launch_fma_burst(int blocks, int iters, double* sink, hipStream_t s) {
    k_fma_burst<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(iters, sink);
    return hipGetLastError();
}

hipError_t launch_mortar_adjoint(int N, const MortAdjArgs& a, hipStream_t s) {
    if (a.n_hang <= 0) return hipSuccess;
    DG_DISPATCH_N(N, (k_mortar_adjoint<NN><<<dim3((unsigned)a.n_hang), dim3(Sz<NN>::NT), 0, s>>>(a)));
    return hipGetLastError();
}

hipError_t launch_mortar(int N, const MortArgs& a, hipStream_t s) {
    if (a.n_hang <= 0) return hipSuccess;
    if (a.pointwise) {
        DG_DISPATCH_N(N, (k_mortar<NN, true><<<dim3((unsigned)a.n_hang), dim3(Sz<NN>::NT), 0, s>>>(a)));
    } else {
        DG_DISPATCH_N(N, (k_mortar<NN, false><<<dim3((unsigned)a.n_hang), dim3(Sz<NN>::NT), 0, s>>>(a)));
    }
    return hipGetLastError();
}

hipError_t launch_adjoint(int N, int mode, bool mixed, const AdjArgs& a, hipStream_t s) {
    if (a.K <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.K);
    if (mixed) {
        if (mode == MODE_RHS) {
            DG_DISPATCH_N(N, (k_adjoint<NN, MODE_RHS, true><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        } else {
            DG_DISPATCH_N(N, (k_adjoint<NN, MODE_RK, true><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        }
    } else {
        if (mode == MODE_RHS) {
            DG_DISPATCH_N(N, (k_adjoint<NN, MODE_RHS, false><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        } else {
            DG_DISPATCH_N(N, (k_adjoint<NN, MODE_RK, false><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        }
    }
    return hipGetLastError();
}

hipError_t launch_background(int64_t K, int N, const double* c1d, double* bg, const BgParams& p, hipStream_t s) {
    const int64_t n = K * (N + 1);
    if (n <= 0) return hipSuccess;
    k_background<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(K, N + 1, c1d, bg, p);
    return hipGetLastError();
}

hipError_t launch_init_bell(int64_t K, int N, const double* c1d, const double* bg, double theta0, const dg_bell& b,
                            double* q, hipStream_t s) {
    const int64_t n = K * (N + 1) * (N + 1) * (N + 1);
    if (n <= 0) return hipSuccess;
    k_init_bell<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(K, N + 1, c1d, bg, theta0, b, q);
    return hipGetLastError();
}

hipError_t launch_node_coords(int64_t K, int N, const double* c1d, double* xyz, hipStream_t s) {
    const int64_t n = K * (N + 1) * (N + 1) * (N + 1);
    if (n <= 0) return hipSuccess;
    k_node_coords<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(K, N + 1, c1d, xyz);
    return hipGetLastError();
}

// one workgroup per plan entry and field (and child, where a family expands)
hipError_t launch_refine(int N, bool adjoint, const XferArgs& a, hipStream_t s) {
    if (a.Kto <= 0) return hipSuccess;
    if (a.nvar < 1 || a.nvar > 5) return hipErrorInvalidValue;
    const unsigned nv = (unsigned)a.nvar;
    if (adjoint) {
        DG_DISPATCH_N(N, (k_family_reduce<NN, true><<<dim3((unsigned)a.Kto, nv), dim3(Sz<NN>::NT), 0, s>>>(a)));
    } else {
        DG_DISPATCH_N(N, (k_expand<NN, false, expand_fields<NN>()><<<dim3((unsigned)a.Kto, 1, (nv + expand_fields<NN>() - 1) / expand_fields<NN>()), dim3(Sz<NN>::NT), 0, s>>>(a)));
    }
    return hipGetLastError();
}

hipError_t launch_coarsen(int N, bool adjoint, const XferArgs& a, hipStream_t s) {
    if (a.Kto <= 0) return hipSuccess;
    if (a.nvar < 1 || a.nvar > 5) return hipErrorInvalidValue;
    const unsigned nv = (unsigned)a.nvar;
    if (adjoint) {
        DG_DISPATCH_N(N, (k_expand<NN, true, expand_fields<NN>()><<<dim3((unsigned)a.Kto, 8, (nv + expand_fields<NN>() - 1) / expand_fields<NN>()), dim3(Sz<NN>::NT), 0, s>>>(a)));
    } else {
        DG_DISPATCH_N(N, (k_family_reduce<NN, false><<<dim3((unsigned)a.Kto, nv), dim3(Sz<NN>::NT), 0, s>>>(a)));
    }
    return hipGetLastError();
}

int budget_blocks(int64_t K) {
    int64_t b = K < kBudgetMaxBlocks ? K : kBudgetMaxBlocks;
    return (int)(b < 1 ? 1 : b);
}

// Partial sums of the allocation-free budgets: one file-scope array per device,
// the most the reduction ever uses (kBudgetMaxBlocks blocks x 4 compensated
// sums), so any mesh fits.  Host code never passes the array's name to a kernel:
// its device address is looked up once per device with hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kBudgetScratchDoubles];

hipError_t budget_scratch(double** out) {
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double*>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_budgets(int N, const BudgetArgs& a, int nblk, double* out_dev, hipStream_t s) {
    DG_DISPATCH_N(N, (k_budgets<NN><<<dim3((unsigned)nblk), dim3(256), 0, s>>>(a)));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_budgets_final<<<dim3(1), dim3(256), 0, s>>>(a.partial, nblk, out_dev);
    return hipGetLastError();
}

hipError_t launch_indicator(int N, const IndArgs& a, hipStream_t s) {
    if (a.K <= 0) return hipSuccess;
    DG_DISPATCH_N(N, (k_indicator<NN><<<dim3((unsigned)a.K), dim3(Sz<NN>::NT), 0, s>>>(a)));
    return hipGetLastError();
}

}  // namespace dgamr

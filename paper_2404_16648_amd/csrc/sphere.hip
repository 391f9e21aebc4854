// HIP kernels of the cubed-sphere shell (section 3.4 spherical geometry, section
// 4.4 global tests): the curvilinear strong-form right-hand side and Shu-Osher
// stage, and the node positions.  One workgroup per element: the tile and the
// contravariant fluxes J a^i . F of the three reference directions are staged in
// LDS, every face node's Rusanov flux along the face's unit normal is lifted with
// the face Jacobian, and the volume divergence is contracted along each
// reference axis and divided by J.  Radial buoyancy -rho' g r_hat.
//
// Compiled with -ffp-contract=off like the box kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device_common.hpp"
#include "kernels.hpp"

namespace dgamr {
namespace {

using namespace dev;

// cube point of panel p at panel coordinates (X, Y)
__device__ __forceinline__ void panel_point(int p, double X, double Y, double c[3]) {
    switch (p) {
        case 0: c[0] = 1.0; c[1] = X; c[2] = Y; break;
        case 1: c[0] = -X; c[1] = 1.0; c[2] = Y; break;
        case 2: c[0] = -1.0; c[1] = -X; c[2] = Y; break;
        case 3: c[0] = X; c[1] = -1.0; c[2] = Y; break;
        case 4: c[0] = -Y; c[1] = X; c[2] = 1.0; break;
        default: c[0] = Y; c[1] = X; c[2] = -1.0; break;
    }
}

// F.n along the unit vector n and the wave speed |u.n| + c
__device__ __forceinline__ void flux_normal(const double q[5], const Bg& b, double Pp, const double n[3],
                                            double gamma, double F[5], double& lam) {
    const double rho = b.rho + q[0];
    const double rinv = rcp_pos(rho);
    const double u0 = q[1] * rinv, u1 = q[2] * rinv, u2 = q[3] * rinv;
    const double un = u0 * n[0] + u1 * n[1] + u2 * n[2];
    const double Th = b.Th + q[4];
    F[0] = q[1] * n[0] + q[2] * n[1] + q[3] * n[2];
    F[1] = q[1] * un + Pp * n[0];
    F[2] = q[2] * un + Pp * n[1];
    F[3] = q[3] * un + Pp * n[2];
    F[4] = Th * un;
    lam = fabs(un) + sqrt_pos(gamma * (b.P + Pp) * rinv);
}

// The shell's stage, one workgroup per element, one thread per node.  (1) One batch
// of loads: the tile into LDS, J, the first metric row, and for the thread's face
// items the face geometry and the neighbour's trace.  (2) Faces: every face node's
// Rusanov flux along the face's unit normal, s F*/(J w_N), for conforming faces and
// walls (both sides of a conforming face sit at the same height: one background);
// hanging faces copy their full lifted term from the mortar pre-pass.  (3) Volume,
// one reference direction d at a time in the LDS the tile used: the contravariant
// flux G_d = J a^d . F at each node (the next direction's metric row in flight),
// the contraction by lines (one task per variable and line reads the line's fluxes
// once and writes the N+1 sums D G along it in place; D from the uniform operator
// table), each node adding -(1/J) times its own sum; a node on a conforming or wall
// face of axis d also adds sgn G_d/(J w_N), the own-flux part of that face's term.
// Radial buoyancy -rho' g r_hat.  MIX (the precision split): the contraction of
// each line in float32, on G_d minus its value at the element's first node (exact:
// D annihilates constants) rounded to float32, with D split into float32 high and
// low parts and float32 accumulation; everything else stays float64.
template <int N, int MODE, bool MIX>
__global__ void __launch_bounds__(Sz<N>::NT) k_stage_sphere(const SphereStageArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    constexpr int ITEMS = (6 * NF + NT - 1) / NT;
    __shared__ double sQ[5 * NP];   // the tile, then the contravariant flux of one direction
    __shared__ double sS[30 * NF];  // [f][v][m]: s F*/(J w_N), or the pre-pass's full term
    __shared__ double sJ[NP];
    __shared__ float sD32[MIX ? 2 * NF : 1];  // MIX: D high and low parts
    __shared__ double sRef[MIX ? 5 : 1];      // MIX: G_d at the element's first node
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t* const rec = A.srec + e * kStageRec;
    const int t = threadIdx.x;
    const int64_t K = A.K, KNP = K * NP, KN1 = K * N1;
    const double gamma = A.gamma;
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;
    const double wN = 2.0 / (N * (N + 1));  // the LGL end weight
    double q[5] = {0, 0, 0, 0, 0}, R[5] = {0, 0, 0, 0, 0};
    // one batch of loads: the tile, J, the first metric row, and for this thread's
    // face items the face geometry and the neighbour's trace
    double jr[3] = {0.0, 0.0, 0.0};
    if (t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sQ[v * NP + t] = A.qs[v * KNP + e * NP + t];
        sJ[t] = A.metric[e * NP + t];
#pragma unroll
        for (int c = 0; c < 3; ++c) jr[c] = A.metric[(1 + c) * KNP + e * NP + t];
    }
    if (MIX)
        for (int x = t; x < NF; x += NT) {
            const double dv = A.ops[x];
            const float hi = (float)dv;
            sD32[x] = hi;
            sD32[NF + x] = (float)(dv - (double)hi);
        }
    const int32_t packed = rec[18];
    int f_[ITEMS], m_[ITEMS];
    double qR_[ITEMS][5], nv_[ITEMS][4];
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        const int it = t + u * NT;
        f_[u] = -1;
        if (it >= 6 * NF) continue;
        const int f = it / NF, m = it - f * NF;
        const int type = rec[f] & 0xff;
        f_[u] = f;
        m_[u] = m;
        if (type == FT_FINE || type == FT_COARSE) continue;
        const double* fg = A.fgeo + ((e * 6 + f) * NF + m) * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) nv_[u][c] = fg[c];
        if (type != FT_WALL) {
            const int64_t e2 = rec[6 + f];
            const int f2 = (packed >> (4 * f)) & 7, flip = (packed >> (4 * f + 3)) & 1;
            const int a = m % N1, bb = m / N1;
            const int n2 = face_node<N>(f2, (flip ? N - a : a) + N1 * bb);
#pragma unroll
            for (int v = 0; v < 5; ++v) qR_[u][v] = A.qs[v * KNP + e2 * NP + n2];
        }
    }
    __syncthreads();

    // ---- faces
    {
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            if (f_[u] < 0) continue;
            const int f = f_[u], m = m_[u];
            const int type = rec[f] & 0xff;
            if (type == FT_FINE || type == FT_COARSE) {
                // hanging face: the full lifted term from the mortar pre-pass
                const int64_t row = (int64_t)rec[12 + f] * 5 + (type == FT_COARSE ? 0 : 1 + ((rec[f] >> 8) & 0xff));
#pragma unroll
                for (int v = 0; v < 5; ++v) sS[(f * 5 + v) * NF + m] = A.mort[(row * 5 + v) * NF + m];
                continue;
            }
            const int n = face_node<N>(f, m), kk = face_k<N>(f, m);
            double qL[5], qR[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) qL[v] = sQ[v * NP + n];
            // both sides of a conforming face sit at the same height: one background
            const Bg b = bg_make(A.bg[e * N1 + kk], A.bg[KN1 + e * N1 + kk], A.bg[2 * KN1 + e * N1 + kk]);
            const double nv[3] = {nv_[u][0], nv_[u][1], nv_[u][2]};
            if (type == FT_WALL) {
                // mirror state: the normal momentum reversed
                const double Un = qL[1] * nv[0] + qL[2] * nv[1] + qL[3] * nv[2];
                qR[0] = qL[0];
#pragma unroll
                for (int c = 0; c < 3; ++c) qR[1 + c] = qL[1 + c] - (2.0 * Un) * nv[c];
                qR[4] = qL[4];
            } else {
#pragma unroll
                for (int v = 0; v < 5; ++v) qR[v] = qR_[u][v];
            }
            const double PpL = pprime(qL[4], b.rTh, b.P, gamma, A.binom);
            const double PpR = pprime(qR[4], b.rTh, b.P, gamma, A.binom);
            double FL[5], FR[5], lL, lR;
            flux_normal(qL, b, PpL, nv, gamma, FL, lL);
            flux_normal(qR, b, PpR, nv, gamma, FR, lR);
            const double lam = fmax(lL, lR);
            const double sface = nv_[u][3] / (sJ[n] * wN);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double Fs = 0.5 * (FL[v] + FR[v]) + 0.5 * lam * (qL[v] - qR[v]);
                sS[(f * 5 + v) * NF + m] = sface * Fs;
            }
        }
    }
    __syncthreads();

    // ---- volume, one direction at a time: G_d in sQ, the contraction by lines in place;
    // G_d = J a^d . F = (U . Ja_d, U (u . Ja_d) + P' Ja_d, Theta u . Ja_d) with the
    // metric row Ja_d read per direction
    double Pp = 0.0, rinv = 0.0, Th = 0.0, Jv = 1.0;
    if (t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) q[v] = sQ[v * NP + t];  // the tile, before the fluxes overwrite it
        Jv = sJ[t];
        const Bg b = bg_make(A.bg[e * N1 + k], A.bg[KN1 + e * N1 + k], A.bg[2 * KN1 + e * N1 + k]);
        Pp = pprime(q[4], b.rTh, b.P, gamma, A.binom);
        rinv = rcp_pos(b.rho + q[0]);
        Th = b.Th + q[4];
    }
    const int ids[3] = {i, j, k};
    double div[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double G[5];
        if (t < NP) {
            const double j0 = jr[0], j1 = jr[1], j2 = jr[2];
            if (d < 2)  // the next direction's metric row, in flight across this direction's passes
#pragma unroll
                for (int c = 0; c < 3; ++c) jr[c] = A.metric[(1 + 3 * (d + 1) + c) * KNP + e * NP + t];
            const double un = (q[1] * rinv) * j0 + (q[2] * rinv) * j1 + (q[3] * rinv) * j2;
            G[0] = q[1] * j0 + q[2] * j1 + q[3] * j2;
            G[1] = q[1] * un + Pp * j0;
            G[2] = q[2] * un + Pp * j1;
            G[3] = q[3] * un + Pp * j2;
            G[4] = Th * un;
#pragma unroll
            for (int v = 0; v < 5; ++v) sQ[v * NP + t] = G[v];
            if (MIX && t == 0)
#pragma unroll
                for (int v = 0; v < 5; ++v) sRef[v] = G[v];
        }
        __syncthreads();
        const int stride = d == 0 ? 1 : d == 1 ? N1 : NF;
        for (int task = t; task < 5 * NF; task += NT) {
            const int v = task / NF, l = task - v * NF;
            const int base = d == 0 ? N1 * l : d == 1 ? (l % N1) + NF * (l / N1) : l;
            double* const Gl = sQ + v * NP + base;
            if constexpr (MIX) {
                const double ref = sRef[v];
                float g[N1];
#pragma unroll
                for (int mm = 0; mm < N1; ++mm) g[mm] = (float)(Gl[mm * stride] - ref);
#pragma unroll
                for (int o = 0; o < N1; ++o) {
                    float ah = 0.0f, al = 0.0f;
#pragma unroll
                    for (int mm = 0; mm < N1; ++mm) {
                        ah = fmaf(sD32[o * N1 + mm], g[mm], ah);
                        al = fmaf(sD32[NF + o * N1 + mm], g[mm], al);
                    }
                    Gl[o * stride] = (double)ah + (double)al;
                }
            } else {
                double g[N1];
#pragma unroll
                for (int mm = 0; mm < N1; ++mm) g[mm] = Gl[mm * stride];
#pragma unroll
                for (int o = 0; o < N1; ++o) {
                    double acc = 0.0;
#pragma unroll
                    for (int mm = 0; mm < N1; ++mm) acc = fma(A.ops[o * N1 + mm], g[mm], acc);
                    Gl[o * stride] = acc;
                }
            }
        }
        __syncthreads();
        if (t < NP) {
#pragma unroll
            for (int v = 0; v < 5; ++v) div[v] = div[v] + sQ[v * NP + t];
            // the own-flux part of a conforming or wall face of axis d at this node
            if (ids[d] == 0 || ids[d] == N) {
                const int f = 2 * d + (ids[d] == N ? 1 : 0);
                const int type = rec[f] & 0xff;
                if (type != FT_FINE && type != FT_COARSE) {
                    const double sg = (f & 1) ? 1.0 : -1.0;
#pragma unroll
                    for (int v = 0; v < 5; ++v) R[v] = R[v] + (sg * G[v]) / (Jv * wN);
                }
            }
        }
        __syncthreads();  // every node has read its sums before the next direction's fluxes
    }
    if (t >= NP) return;
    // radial buoyancy -rho' g r_hat
    {
        double cp[3];
        panel_point(rec[19], A.c1d[e * N1 + i], A.c1d[KN1 + e * N1 + j], cp);
        const double nrm = sqrt(cp[0] * cp[0] + cp[1] * cp[1] + cp[2] * cp[2]);
        const double gb = -q[0] * A.g;
#pragma unroll
        for (int c = 0; c < 3; ++c) R[1 + c] = R[1 + c] + gb * (cp[c] / nrm);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) R[v] = -div[v] / Jv + R[v];
    // a node lies on at most one face per axis
    const int fm[3] = {j + N1 * k, i + N1 * k, i + N1 * j};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (ids[d] == 0 || ids[d] == N) {
            const int f = 2 * d + (ids[d] == N ? 1 : 0);
#pragma unroll
            for (int v = 0; v < 5; ++v) R[v] = R[v] - sS[(f * 5 + v) * NF + fm[d]];
        }
    }
    const int64_t base = e * NP + t;
    if (MODE == MODE_RHS) {
#pragma unroll
        for (int v = 0; v < 5; ++v) A.out[v * KNP + base] = R[v];
    } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double o = A.b * fma(A.dt, R[v], q[v]);
            if (A.a != 0.0) o = fma(A.a, A.q0[v * KNP + base], o);
            A.out[v * KNP + base] = o;
        }
    }
}

// node positions xyz[3][K][Np] = (r_e + h) r_hat
__global__ void k_node_coords_sphere(int64_t K, int N1, const double* c1d, const int32_t* srec, double r_e,
                                     double* xyz) {
    const int64_t NP = (int64_t)N1 * N1 * N1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= K * NP) return;
    const int64_t e = idx / NP;
    const int n = (int)(idx % NP);
    const int i = n % N1, j = (n / N1) % N1, k = n / (N1 * N1);
    double cp[3];
    panel_point(srec[e * kStageRec + 19], c1d[e * N1 + i], c1d[K * N1 + e * N1 + j], cp);
    const double nrm = sqrt(cp[0] * cp[0] + cp[1] * cp[1] + cp[2] * cp[2]);
    const double r = r_e + c1d[2 * K * N1 + e * N1 + k];
#pragma unroll
    for (int c = 0; c < 3; ++c) xyz[c * K * NP + idx] = r * (cp[c] / nrm);
}

// J a^d . F(q) at one node: the Cartesian fluxes contracted with the metric row d
__device__ __forceinline__ void contravariant_flux(const double q[5], const Bg& b, double Pp, const double* metric,
                                                   int64_t KNP, int64_t node, int d, double out[5]) {
    const double rinv = rcp_pos(b.rho + q[0]);
    const double Th = b.Th + q[4];
    double F[3][5];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double uc = q[1 + c] * rinv;
        F[c][0] = q[1 + c];
        F[c][1] = c == 0 ? q[1] * uc + Pp : q[1] * uc;
        F[c][2] = c == 1 ? q[2] * uc + Pp : q[2] * uc;
        F[c][3] = c == 2 ? q[3] * uc + Pp : q[3] * uc;
        F[c][4] = Th * uc;
    }
    const double j0 = metric[(1 + 3 * d + 0) * KNP + node], j1 = metric[(1 + 3 * d + 1) * KNP + node],
                 j2 = metric[(1 + 3 * d + 2) * KNP + node];
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v] = j0 * F[0][v] + j1 * F[1][v] + j2 * F[2][v];
}

template <int N>
struct MortSz {
    static constexpr int NF = (N + 1) * (N + 1);
    static constexpr int NT = ((4 * NF + 63) / 64) * 64;  // one thread per fine face node of the four quadrants
};

// Mortar pre-pass of the shell (section 3.3 on the curved faces of section 3.4), one
// workgroup per hanging row.  On each fine face the coarse trace is interpolated to
// the fine nodes (I_qa x I_qb in the coarse face's axes, read through the
// orientation) and the Riemann problem is solved there along the fine face's own
// normal with the fine nodes' background; the fine face's lifted term is
// (s_f F* - sgn J a^d . F(q_f)) / (J w_N).  The coarse side takes 4 s_f (-F*) (the
// flux per coarse reference area: a fine face covers a quarter of it), projected back
// with R_qa x R_qb and summed over the quadrants, minus its own contravariant flux.
template <int N>
__global__ void __launch_bounds__(MortSz<N>::NT) k_mortar_sphere(const SphereMortArgs A) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1, NF = N1 * N1, NT = MortSz<N>::NT;
    __shared__ double sTc[5 * NF], sG[20 * NF], sI[2 * NF], sR[2 * NF];
    const int t = threadIdx.x;
    const int64_t h = blockIdx.x;
    const int32_t* row = A.hang + h * 6;
    const int64_t ec = row[0];
    const int fc = row[1];
    const int32_t packed = A.srec[ec * kStageRec + 18];
    const int ff = (packed >> (4 * fc)) & 7, flip = (packed >> (4 * fc + 3)) & 1;
    const int64_t K = A.K, KNP = K * NP, KN1 = K * N1;
    const double gamma = A.gamma;
    const double wN = 2.0 / (N * (N + 1));
    for (int x = t; x < 2 * NF; x += NT) {
        sI[x] = A.ops[NF + x];      // I_0, I_1
        sR[x] = A.ops[3 * NF + x];  // R_0, R_1
    }
    if (t < NF) {
        const int n = face_node<N>(fc, t);
#pragma unroll
        for (int v = 0; v < 5; ++v) sTc[v * NF + t] = A.qs[v * KNP + ec * NP + n];
    }
    __syncthreads();
    if (t < 4 * NF) {
        const int quad = t / NF, mf = t - quad * NF;
        const int qa = quad & 1, qb = quad >> 1;
        const int64_t ef = row[2 + quad];
        const int af = mf % N1, bf = mf / N1;
        const int a2 = flip ? N - af : af, b2 = bf;  // the node in the coarse face's axes
        const double* Ia = sI + qa * NF;
        const double* Ib = sI + qb * NF;
        double qm[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double acc = 0.0;
            for (int a = 0; a < N1; ++a) {
                double tb = 0.0;
                for (int b = 0; b < N1; ++b) tb = fma(Ib[b2 * N1 + b], sTc[v * NF + a + N1 * b], tb);
                acc = fma(Ia[a2 * N1 + a], tb, acc);
            }
            qm[v] = acc;
        }
        const int nf = face_node<N>(ff, mf), kf = face_k<N>(ff, mf);
        double qf[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qf[v] = A.qs[v * KNP + ef * NP + nf];
        const Bg b = bg_make(A.bg[ef * N1 + kf], A.bg[KN1 + ef * N1 + kf], A.bg[2 * KN1 + ef * N1 + kf]);
        const double* fg = A.fgeo + ((ef * 6 + ff) * NF + mf) * 4;
        const double nv[3] = {fg[0], fg[1], fg[2]};
        const double sf = fg[3];
        const double PpL = pprime(qf[4], b.rTh, b.P, gamma, A.binom);
        const double PpR = pprime(qm[4], b.rTh, b.P, gamma, A.binom);
        double FL[5], FR[5], lL, lR, Fc[5];
        flux_normal(qf, b, PpL, nv, gamma, FL, lL);
        flux_normal(qm, b, PpR, nv, gamma, FR, lR);
        contravariant_flux(qf, b, PpL, A.metric, KNP, ef * NP + nf, ff >> 1, Fc);
        const double lam = fmax(lL, lR);
        const double sgn = (ff & 1) ? 1.0 : -1.0;
        const double JwN = A.metric[ef * NP + nf] * wN;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double Fs = 0.5 * (FL[v] + FR[v]) + 0.5 * lam * (qf[v] - qm[v]);
            A.mort[((h * 5 + 1 + quad) * 5 + v) * NF + mf] = (sf * Fs - sgn * Fc[v]) / JwN;
            sG[(quad * 5 + v) * NF + a2 + N1 * b2] = (4.0 * sf) * (-Fs);
        }
    }
    __syncthreads();
    if (t < NF) {
        const int a = t % N1, b = t / N1;
        double proj[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        auto add_quadrant = [&](int quad) {
            const double* Ra = sR + (quad & 1) * NF;
            const double* Rb = sR + (quad >> 1) * NF;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                double acc = 0.0;
                for (int a2 = 0; a2 < N1; ++a2) {
                    double tb = 0.0;
                    for (int b2 = 0; b2 < N1; ++b2) tb = fma(Rb[b * N1 + b2], sG[(quad * 5 + v) * NF + a2 + N1 * b2], tb);
                    acc = fma(Ra[a * N1 + a2], tb, acc);
                }
                proj[v] = proj[v] + acc;
            }
        };
        // left to the compiler (unrolled) except at N = 3, where the unrolled form
        // spills to scratch memory
        if constexpr (N == 3) {
#pragma unroll 1
            for (int quad = 0; quad < 4; ++quad) add_quadrant(quad);
        } else {
            for (int quad = 0; quad < 4; ++quad) add_quadrant(quad);
        }
        const int nc = face_node<N>(fc, t), kc = face_k<N>(fc, t);
        double qc[5], Fc[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qc[v] = sTc[v * NF + t];
        const Bg bc = bg_make(A.bg[ec * N1 + kc], A.bg[KN1 + ec * N1 + kc], A.bg[2 * KN1 + ec * N1 + kc]);
        const double Ppc = pprime(qc[4], bc.rTh, bc.P, gamma, A.binom);
        contravariant_flux(qc, bc, Ppc, A.metric, KNP, ec * NP + nc, fc >> 1, Fc);
        const double sgn = (fc & 1) ? 1.0 : -1.0;
        const double JwN = A.metric[ec * NP + nc] * wN;
#pragma unroll
        for (int v = 0; v < 5; ++v) A.mort[((h * 5 + 0) * 5 + v) * NF + t] = (proj[v] - sgn * Fc[v]) / JwN;
    }
}

// ---------------------------------------------------------------- adjoint (transpose of the shell stage)

// g += J^T a for the flux along the vector m at a node, F.m = (U.m, U (u.m) + P' m,
// Theta u.m) with u = U / rho (m a unit normal, or a metric row J a^d); rinv = 1/rho,
// Th = Thetabar + Theta', dPdT = dP'/dTheta' = gamma P / Th
__device__ __forceinline__ void flux_along_vjp(const double q[5], double rinv, double Th, double dPdT,
                                               const double m[3], const double a[5], double g[5]) {
    const double un = (q[1] * m[0] + q[2] * m[1] + q[3] * m[2]) * rinv;
    const double ubar = a[1] * q[1] + a[2] * q[2] + a[3] * q[3] + a[4] * Th;
    const double am = a[1] * m[0] + a[2] * m[1] + a[3] * m[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) g[1 + c] += a[0] * m[c] + a[1 + c] * un + ubar * m[c] * rinv;
    g[0] -= ubar * un * rinv;
    g[4] += a[4] * un + am * dPdT;
}

// pointwise state along a unit normal n: 1/rho, Theta, dP'/dTheta', the wave speed
// lam = |u.n| + c and its gradient (d lam/d U_c = dlamU n_c; d|x|/dx = 0 at x = 0)
struct NormState {
    double rinv, Th, dPdT, lam, dlam0, dlamU, dlam4;
};

__device__ __forceinline__ NormState norm_state(const double q[5], const Bg& b, double Pp, const double n[3],
                                                double gamma) {
    NormState s;
    s.rinv = rcp_pos(b.rho + q[0]);
    const double un = (q[1] * n[0] + q[2] * n[1] + q[3] * n[2]) * s.rinv;
    s.Th = b.Th + q[4];
    const double P = b.P + Pp;
    s.dPdT = gamma * P / s.Th;
    const double c = sqrt_pos(gamma * P * s.rinv);
    const double au = fabs(un);
    s.lam = au + c;
    s.dlam0 = -(au + 0.5 * c) * s.rinv;
    s.dlamU = (un > 0.0 ? 1.0 : (un < 0.0 ? -1.0 : 0.0)) * s.rinv;
    s.dlam4 = 0.5 * gamma * c / s.Th;
    return s;
}

// gL (and gR if non-null) = derivative of w . F*(qL, qR, n) with respect to qL (qR),
// F* the Rusanov flux along the unit normal n with one background on both sides; a
// max tie splits the derivative 1/2, 1/2
__device__ __forceinline__ void rusanov_along_vjp(const double qL[5], double PpL, const double qR[5], double PpR,
                                                  const Bg& b, const double n[3], double gamma, const double w[5],
                                                  double gL[5], double* gR) {
    const NormState L = norm_state(qL, b, PpL, n, gamma);
    const NormState Rr = norm_state(qR, b, PpR, n, gamma);
    const double hl = 0.5 * fmax(L.lam, Rr.lam);
    const double tL = L.lam > Rr.lam ? 1.0 : (L.lam < Rr.lam ? 0.0 : 0.5);
    double wj = 0.0, a[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        wj += w[v] * (qL[v] - qR[v]);
        a[v] = 0.5 * w[v];
        gL[v] = hl * w[v];
    }
    flux_along_vjp(qL, L.rinv, L.Th, L.dPdT, n, a, gL);
    const double cL = 0.5 * wj * tL;
    gL[0] += cL * L.dlam0;
#pragma unroll
    for (int c = 0; c < 3; ++c) gL[1 + c] += cL * L.dlamU * n[c];
    gL[4] += cL * L.dlam4;
    if (gR) {
#pragma unroll
        for (int v = 0; v < 5; ++v) gR[v] = -hl * w[v];
        flux_along_vjp(qR, Rr.rinv, Rr.Th, Rr.dPdT, n, a, gR);
        const double cR = 0.5 * wj * (1.0 - tL);
        gR[0] += cR * Rr.dlam0;
#pragma unroll
        for (int c = 0; c < 3; ++c) gR[1 + c] += cR * Rr.dlamU * n[c];
        gR[4] += cR * Rr.dlam4;
    }
}

// g += the gradient of a . J a^d . F(q) at a node (the own-flux part of a face term)
__device__ __forceinline__ void contravariant_flux_vjp(const double q[5], const Bg& b, double Pp,
                                                       const double* metric, int64_t KNP, int64_t node, int d,
                                                       double gamma, const double a[5], double g[5]) {
    const double rinv = rcp_pos(b.rho + q[0]);
    const double Th = b.Th + q[4];
    const double dPdT = gamma * (b.P + Pp) / Th;
    const double m[3] = {metric[(1 + 3 * d + 0) * KNP + node], metric[(1 + 3 * d + 1) * KNP + node],
                         metric[(1 + 3 * d + 2) * KNP + node]};
    flux_along_vjp(q, rinv, Th, dPdT, m, a, g);
}

// Transposed mortar pre-pass of the shell, one workgroup per hanging row.  With
// mu_c = lam_c / (J w_N) on the coarse face, a mortar point of quadrant (qa, qb)
// carries w . F*(q_f, q_m, n_f) of <lam, R>, w = s_f (4 ((R_qa x R_qb)^T mu_c) -
// lam_f / (J_f w_N)): its gradient with respect to the fine state goes to the fine
// face (slot 1 + quad, with the fine side's own-flux term sgn J a^d . F / (J w_N)),
// its gradient with respect to the mortar state q_m = (I_qa x I_qb) q_c back to the
// coarse face through (I_qa x I_qb)^T (slot 0, with the coarse side's own-flux term).
template <int N>
__global__ void __launch_bounds__(MortSz<N>::NT) k_mortar_sphere_adjoint(const SphereMortAdjArgs A) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1, NF = N1 * N1, NT = MortSz<N>::NT;
    // sTc: the coarse trace; sMu: mu_c; sG: per quadrant, first (R_qa x R_qb)^T mu_c,
    // then the mortar-state gradient, at the fine points in the coarse face's axes
    __shared__ double sTc[5 * NF], sMu[5 * NF], sG[20 * NF], sI[2 * NF], sR[2 * NF];
    const int t = threadIdx.x;
    const int64_t h = blockIdx.x;
    const int32_t* row = A.hang + h * 6;
    const int64_t ec = row[0];
    const int fc = row[1];
    const int32_t packed = A.srec[ec * kStageRec + 18];
    const int ff = (packed >> (4 * fc)) & 7, flip = (packed >> (4 * fc + 3)) & 1;
    const int64_t K = A.K, KNP = K * NP, KN1 = K * N1;
    const double gamma = A.gamma;
    const double wN = 2.0 / (N * (N + 1));
    for (int x = t; x < 2 * NF; x += NT) {
        sI[x] = A.ops[NF + x];      // I_0, I_1
        sR[x] = A.ops[3 * NF + x];  // R_0, R_1
    }
    if (t < NF) {
        const int n = face_node<N>(fc, t);
        const double JwN = A.metric[ec * NP + n] * wN;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            sTc[v * NF + t] = A.q[v * KNP + ec * NP + n];
            sMu[v * NF + t] = A.lam[v * KNP + ec * NP + n] / JwN;
        }
    }
    // this thread's fine point: quadrant t / NF, node mf of the fine face
    const int quad = t / NF, mf = t - quad * NF;
    const int qa = quad & 1, qb = quad >> 1;
    const int af = mf % N1, bf = mf / N1;
    const int a2 = flip ? N - af : af, b2 = bf;  // the node in the coarse face's axes
    double qf[5] = {0, 0, 0, 0, 0}, lf[5] = {0, 0, 0, 0, 0}, fg[4] = {0, 0, 0, 1};
    double JwNf = 1.0;
    int64_t ef = 0;
    int nf = 0, kf = 0;
    if (t < 4 * NF) {
        ef = row[2 + quad];
        nf = face_node<N>(ff, mf);
        kf = face_k<N>(ff, mf);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qf[v] = A.q[v * KNP + ef * NP + nf];
            lf[v] = A.lam[v * KNP + ef * NP + nf];
        }
        const double* g4 = A.fgeo + ((ef * 6 + ff) * NF + mf) * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) fg[c] = g4[c];
        JwNf = A.metric[ef * NP + nf] * wN;
    }
    __syncthreads();
    double qm[5], rm[5];
    if (t < 4 * NF) {
        // q_m = (I_qa x I_qb) q_c and (R_qa x R_qb)^T mu_c at (a2, b2)
        const double* Ia = sI + qa * NF;
        const double* Ib = sI + qb * NF;
        const double* Ra = sR + qa * NF;
        const double* Rb = sR + qb * NF;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double acc = 0.0, accr = 0.0;
            #pragma unroll 1
            for (int a = 0; a < N1; ++a) {
                double tb = 0.0, tr = 0.0;
                for (int b = 0; b < N1; ++b) {
                    tb = fma(Ib[b2 * N1 + b], sTc[v * NF + a + N1 * b], tb);
                    tr = fma(Rb[b * N1 + b2], sMu[v * NF + a + N1 * b], tr);
                }
                acc = fma(Ia[a2 * N1 + a], tb, acc);
                accr = fma(Ra[a * N1 + a2], tr, accr);
            }
            qm[v] = acc;
            rm[v] = accr;
        }
        const Bg b = bg_make(A.bg[ef * N1 + kf], A.bg[KN1 + ef * N1 + kf], A.bg[2 * KN1 + ef * N1 + kf]);
        const double nv[3] = {fg[0], fg[1], fg[2]};
        const double sf = fg[3];
        const double PpF = pprime(qf[4], b.rTh, b.P, gamma, A.binom);
        const double PpM = pprime(qm[4], b.rTh, b.P, gamma, A.binom);
        double w[5], gF[5], gM[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) w[v] = sf * (4.0 * rm[v] - lf[v] / JwNf);
        rusanov_along_vjp(qf, PpF, qm, PpM, b, nv, gamma, w, gF, gM);
        // the fine side's own-flux term +sgn J a^d . F(q_f) / (J w_N)
        const double sgn = (ff & 1) ? 1.0 : -1.0;
        double ao[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) ao[v] = sgn * lf[v] / JwNf;
        contravariant_flux_vjp(qf, b, PpF, A.metric, KNP, ef * NP + nf, ff >> 1, gamma, ao, gF);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            A.mort[((h * 5 + 1 + quad) * 5 + v) * NF + mf] = gF[v];
            sG[(quad * 5 + v) * NF + a2 + N1 * b2] = gM[v];
        }
    }
    __syncthreads();
    if (t < NF) {
        // back to the coarse face: sum over quadrants of (I_qa x I_qb)^T gM
        const int a = t % N1, b = t / N1;
        double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int qd = 0; qd < 4; ++qd) {
            const double* Ia = sI + (qd & 1) * NF;
            const double* Ib = sI + (qd >> 1) * NF;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                double acc = 0.0;
                #pragma unroll 1
                for (int x2 = 0; x2 < N1; ++x2) {
                    double tb = 0.0;
                    for (int y2 = 0; y2 < N1; ++y2) tb = fma(Ib[y2 * N1 + b], sG[(qd * 5 + v) * NF + x2 + N1 * y2], tb);
                    acc = fma(Ia[x2 * N1 + a], tb, acc);
                }
                g[v] = g[v] + acc;
            }
        }
        const int nc = face_node<N>(fc, t), kc = face_k<N>(fc, t);
        double qc[5], ao[5];
        const double sgn = (fc & 1) ? 1.0 : -1.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qc[v] = sTc[v * NF + t];
            ao[v] = sgn * sMu[v * NF + t];
        }
        const Bg bc = bg_make(A.bg[ec * N1 + kc], A.bg[KN1 + ec * N1 + kc], A.bg[2 * KN1 + ec * N1 + kc]);
        const double Ppc = pprime(qc[4], bc.rTh, bc.P, gamma, A.binom);
        contravariant_flux_vjp(qc, bc, Ppc, A.metric, KNP, ec * NP + nc, fc >> 1, gamma, ao, g);
#pragma unroll
        for (int v = 0; v < 5; ++v) A.mort[((h * 5 + 0) * 5 + v) * NF + t] = g[v];
    }
}

// The transposed shell stage, one workgroup per element, one thread per node: with
// mu = -lam / J, (1) faces: at each conforming face node the Rusanov VJP with weight
// w = -s_L lam_L + s_R lam_R (s = face Jacobian / (J w_N) on each side: the
// neighbour's term at its node is +s_R F*(qL, qR, n) by antisymmetry), at a wall the
// VJP through the mirror state, at a hanging face the transposed pre-pass's
// contribution; (2) volume: for each reference direction d the transposed
// contraction Gbar_d = D_d^T mu (plus sgn lam / (J w_N) at the nodes of a conforming
// or wall face of axis d, the own-flux part) and the chain rule through G_d = J a^d.F;
// (3) buoyancy -rho' g r_hat transposed.  MIX: the transposed contractions in
// float32 (mu rounded to float32, D split into float32 high and low parts, float32
// accumulation); faces, mortars, the chain rule and the output stay float64.
template <int N, int MODE, bool MIX>
__global__ void __launch_bounds__(Sz<N>::NT) k_adjoint_sphere(const SphereAdjArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    constexpr int ITEMS = (6 * NF + NT - 1) / NT;
    __shared__ double sQ[5 * NP];   // the tile
    __shared__ double sMu[5 * NP];  // -lam / J
    __shared__ double sS[30 * NF];  // [f][v][m]: the face contributions to qbar
    __shared__ double sJ[NP];
    __shared__ float sMuf[MIX ? 5 * NP : 1];  // MIX: mu in float32
    __shared__ float sD32[MIX ? 2 * NF : 1];  // MIX: D high and low parts
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t* const rec = A.srec + e * kStageRec;
    const int t = threadIdx.x;
    const int64_t K = A.K, KNP = K * NP, KN1 = K * N1;
    const double gamma = A.gamma;
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;
    const double wN = 2.0 / (N * (N + 1));
    double q[5] = {0, 0, 0, 0, 0}, lam[5] = {0, 0, 0, 0, 0};
    if (t < NP) {
        const double Jv = A.metric[e * NP + t];
        sJ[t] = Jv;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            q[v] = A.q[v * KNP + e * NP + t];
            lam[v] = A.lam[v * KNP + e * NP + t];
            sQ[v * NP + t] = q[v];
            const double mu = -lam[v] / Jv;
            sMu[v * NP + t] = mu;
            if (MIX) sMuf[v * NP + t] = (float)mu;
        }
    }
    if (MIX)
        for (int x = t; x < NF; x += NT) {
            const double dv = A.ops[x];
            const float hi = (float)dv;
            sD32[x] = hi;
            sD32[NF + x] = (float)(dv - (double)hi);
        }
    // the face items' loads: face geometry, the neighbour's state, weights, face
    // Jacobian and J at its node
    const int32_t packed = rec[18];
    int f_[ITEMS], m_[ITEMS];
    double qR_[ITEMS][5], lR_[ITEMS][5], nv_[ITEMS][4], sR_[ITEMS];
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        const int it = t + u * NT;
        f_[u] = -1;
        if (it >= 6 * NF) continue;
        const int f = it / NF, m = it - f * NF;
        const int type = rec[f] & 0xff;
        f_[u] = f;
        m_[u] = m;
        if (type == FT_FINE || type == FT_COARSE) continue;
        const double* fg = A.fgeo + ((e * 6 + f) * NF + m) * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) nv_[u][c] = fg[c];
        if (type != FT_WALL) {
            const int64_t e2 = rec[6 + f];
            const int f2 = (packed >> (4 * f)) & 7, flip = (packed >> (4 * f + 3)) & 1;
            const int a = m % N1, bb = m / N1;
            const int m2 = (flip ? N - a : a) + N1 * bb;
            const int n2 = face_node<N>(f2, m2);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                qR_[u][v] = A.q[v * KNP + e2 * NP + n2];
                lR_[u][v] = A.lam[v * KNP + e2 * NP + n2];
            }
            sR_[u] = A.fgeo[((e2 * 6 + f2) * NF + m2) * 4 + 3] / (A.metric[e2 * NP + n2] * wN);
        }
    }
    __syncthreads();

    // ---- faces
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        if (f_[u] < 0) continue;
        const int f = f_[u], m = m_[u];
        const int type = rec[f] & 0xff;
        if (type == FT_FINE || type == FT_COARSE) {
            const int64_t row = (int64_t)rec[12 + f] * 5 + (type == FT_COARSE ? 0 : 1 + ((rec[f] >> 8) & 0xff));
#pragma unroll
            for (int v = 0; v < 5; ++v) sS[(f * 5 + v) * NF + m] = A.mort[(row * 5 + v) * NF + m];
            continue;
        }
        const int n = face_node<N>(f, m), kk = face_k<N>(f, m);
        double qL[5], qR[5], w[5], g[5];
        const double nv[3] = {nv_[u][0], nv_[u][1], nv_[u][2]};
        // -s_L lam_L = face Jacobian * mu_L / w_N
        const double cL = nv_[u][3] / wN;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qL[v] = sQ[v * NP + n];
            w[v] = cL * sMu[v * NP + n];
        }
        const Bg b = bg_make(A.bg[e * N1 + kk], A.bg[KN1 + e * N1 + kk], A.bg[2 * KN1 + e * N1 + kk]);
        const double PpL = pprime(qL[4], b.rTh, b.P, gamma, A.binom);
        if (type == FT_WALL) {
            // qR = M qL, M reverses the normal momentum (symmetric: M^T = M)
            const double Un = qL[1] * nv[0] + qL[2] * nv[1] + qL[3] * nv[2];
            qR[0] = qL[0];
#pragma unroll
            for (int c = 0; c < 3; ++c) qR[1 + c] = qL[1 + c] - (2.0 * Un) * nv[c];
            qR[4] = qL[4];
            double gR[5];
            rusanov_along_vjp(qL, PpL, qR, PpL, b, nv, gamma, w, g, gR);
            const double gn = gR[1] * nv[0] + gR[2] * nv[1] + gR[3] * nv[2];
            g[0] += gR[0];
#pragma unroll
            for (int c = 0; c < 3; ++c) g[1 + c] += gR[1 + c] - (2.0 * gn) * nv[c];
            g[4] += gR[4];
        } else {
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                qR[v] = qR_[u][v];
                w[v] = fma(sR_[u], lR_[u][v], w[v]);
            }
            const double PpR = pprime(qR[4], b.rTh, b.P, gamma, A.binom);
            rusanov_along_vjp(qL, PpL, qR, PpR, b, nv, gamma, w, g, nullptr);
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) sS[(f * 5 + v) * NF + m] = g[v];
    }
    __syncthreads();

    if (t >= NP) return;
    // ---- volume: Gbar_d = D_d^T mu (+ the own-flux part), then the chain rule through
    // G_d = J a^d . F
    double g[5] = {0, 0, 0, 0, 0};
    {
        const Bg b = bg_make(A.bg[e * N1 + k], A.bg[KN1 + e * N1 + k], A.bg[2 * KN1 + e * N1 + k]);
        const double Pp = pprime(q[4], b.rTh, b.P, gamma, A.binom);
        const double rinv = rcp_pos(b.rho + q[0]);
        const double Th = b.Th + q[4];
        const double dPdT = gamma * (b.P + Pp) / Th;
        const double Jv = sJ[t];
        const int ids[3] = {i, j, k};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int id = ids[d];
            const int stride = d == 0 ? 1 : d == 1 ? N1 : NF;
            const int base = t - id * stride;
            double a[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                if constexpr (MIX) {
                    const float* Mu = sMuf + v * NP + base;
                    float ah = 0.0f, al = 0.0f;
#pragma unroll
                    for (int o = 0; o < N1; ++o) {
                        const float mv = Mu[o * stride];
                        ah = fmaf(sD32[o * N1 + id], mv, ah);
                        al = fmaf(sD32[NF + o * N1 + id], mv, al);
                    }
                    a[v] = (double)ah + (double)al;
                } else {
                    const double* Mu = sMu + v * NP + base;
                    double acc = 0.0;
#pragma unroll
                    for (int o = 0; o < N1; ++o) acc = fma(A.ops[o * N1 + id], Mu[o * stride], acc);
                    a[v] = acc;
                }
            }
            if (id == 0 || id == N) {
                const int f = 2 * d + (id == N ? 1 : 0);
                const int type = rec[f] & 0xff;
                if (type != FT_FINE && type != FT_COARSE) {
                    const double sg = (f & 1) ? 1.0 : -1.0;
#pragma unroll
                    for (int v = 0; v < 5; ++v) a[v] += (sg * lam[v]) / (Jv * wN);
                }
            }
            const double m[3] = {A.metric[(1 + 3 * d + 0) * KNP + e * NP + t],
                                 A.metric[(1 + 3 * d + 1) * KNP + e * NP + t],
                                 A.metric[(1 + 3 * d + 2) * KNP + e * NP + t]};
            flux_along_vjp(q, rinv, Th, dPdT, m, a, g);
        }
    }
    // ---- buoyancy -rho' g r_hat on the momentum
    {
        double cp[3];
        panel_point(rec[19], A.c1d[e * N1 + i], A.c1d[KN1 + e * N1 + j], cp);
        const double nrm = sqrt(cp[0] * cp[0] + cp[1] * cp[1] + cp[2] * cp[2]);
        g[0] -= A.g * (lam[1] * (cp[0] / nrm) + lam[2] * (cp[1] / nrm) + lam[3] * (cp[2] / nrm));
    }
    // ---- the faces that touch this node (at most one per axis)
    const int fm[3] = {j + N1 * k, i + N1 * k, i + N1 * j};
    const int ids[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (ids[d] == 0 || ids[d] == N) {
            const int f = 2 * d + (ids[d] == N ? 1 : 0);
#pragma unroll
            for (int v = 0; v < 5; ++v) g[v] += sS[(f * 5 + v) * NF + fm[d]];
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

// ---------------------------------------------------------------- shell transfers
// Between a shell (nc x nc per panel, nzc layers) and the shell with twice the
// elements per edge and twice the layers: child a = ax + 2 ay + 4 az of coarse
// element (p, ia, ib, ir) is fine element (p, 2 ia + ax, 2 ib + ay, 2 ir + az), and
// its reference box is half ax, ay, az of the parent's along the local axes.

// one separable pass over the NFLD fields of a tile in LDS: out[v][node] =
// sum_m M[idx(node, axis)][m] in[v][node with that index replaced by m]
template <int N, int NFLD = 5>
__device__ __forceinline__ void tile_pass(const double* in, double* out, const double* M, int axis, int t) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1, NF = N1 * N1;
    if (t >= NP) return;
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;
    const int id = axis == 0 ? i : axis == 1 ? j : k;
    const int stride = axis == 0 ? 1 : axis == 1 ? N1 : NF;
    const int base = t - id * stride;
#pragma unroll
    for (int v = 0; v < NFLD; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < N1; ++m) acc = fma(M[id * N1 + m], in[v * NP + base + m * stride], acc);
        out[v * NP + t] = acc;
    }
}

// one child: dst[e] = (I_ax x I_ay x I_az) src[parent], ax, ay, az the bits of child
template <int N>
__device__ __forceinline__ void child_of_parent(const double* src, int64_t Ksrc, int64_t parent, double* dst,
                                                int64_t Kdst, int64_t e, int child, const double* ops, double* sT,
                                                double* sU, double* sM, int t) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1, NF = N1 * N1, NT = Sz<N>::NT;
    const int hal[3] = {child & 1, (child >> 1) & 1, child >> 2};
    for (int x = t; x < 3 * NF; x += NT) {
        const int ax = x / NF;
        sM[x] = ops[(1 + hal[ax]) * NF + (x - ax * NF)];  // I_0 or I_1
    }
    if (t < NP)
#pragma unroll
        for (int v = 0; v < 5; ++v) sT[v * NP + t] = src[(v * Ksrc + parent) * NP + t];
    __syncthreads();
    tile_pass<N>(sT, sU, sM, 0, t);
    __syncthreads();
    tile_pass<N>(sU, sT, sM + NF, 1, t);
    __syncthreads();
    if (t < NP) {
        const int k = t / NF, base = t - k * NF;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < N1; ++m) acc = fma(sM[2 * NF + k * N1 + m], sT[v * NP + base + m * NF], acc);
            dst[(v * Kdst + e) * NP + t] = acc;
        }
    }
}

// one family: dst[e] = sum_a (R_ax x R_ay x R_az) src[kid_a] plus, per field, the
// constant c = (sum of the children's J W integrals - the parent's) / the parent's
// J W volume, taken on the conserved fields (rho' and Theta' with their background):
// the family's quadrature of every conserved field is kept.  sRed: [NT][11] doubles.
template <int N>
__device__ __forceinline__ void family_to_parent(const double* src, int64_t Ksrc, const int64_t kids[8], double* dst,
                                                 int64_t Kdst, int64_t e, const double* ops, const double* met_src,
                                                 const double* met_dst, const double* bg_src, const double* bg_dst,
                                                 double* sT, double* sU, double* sR, double* sW, double* sRed,
                                                 int t) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1, NF = N1 * N1, NT = Sz<N>::NT;
    for (int x = t; x < 2 * NF; x += NT) sR[x] = ops[3 * NF + x];  // R_0, R_1
    if (t < N1) sW[t] = ops[5 * NF + t];
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double inside[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int ii = t % N1, jj = (t / N1) % N1, kk = t / NF;
    for (int a = 0; a < 8; ++a) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
        const int64_t ef = kids[a];
        __syncthreads();  // the previous child's last pass has read sT
        if (t < NP)
#pragma unroll
            for (int v = 0; v < 5; ++v) sT[v * NP + t] = src[(v * Ksrc + ef) * NP + t];
        __syncthreads();
        if (t < NP) {
            const double JW = met_src[ef * NP + t] * (sW[ii] * sW[jj] * sW[kk]);
            const double b0 = bg_src[ef * N1 + kk], b4 = bg_src[Ksrc * N1 + ef * N1 + kk];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double full = v == 0 ? b0 + sT[t] : v == 4 ? b4 + sT[4 * NP + t] : sT[v * NP + t];
                inside[v] = fma(JW, full, inside[v]);
            }
        }
        tile_pass<N>(sT, sU, sR + ax * NF, 0, t);
        __syncthreads();
        tile_pass<N>(sU, sT, sR + ay * NF, 1, t);
        __syncthreads();
        if (t < NP) {
            const int k = t / NF, base = t - k * NF;
            const double* Rz = sR + az * NF;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                double s = 0.0;
#pragma unroll
                for (int m = 0; m < N1; ++m) s = fma(Rz[k * N1 + m], sT[v * NP + base + m * NF], s);
                acc[v] += s;
            }
        }
    }
    // the eleven sums: inside[5], the projection's integrals[5], the parent's volume
    double part[11];
#pragma unroll
    for (int x = 0; x < 11; ++x) part[x] = 0.0;
    if (t < NP) {
        const double JW = met_dst[e * NP + t] * (sW[ii] * sW[jj] * sW[kk]);
        const double b0 = bg_dst[e * N1 + kk], b4 = bg_dst[Kdst * N1 + e * N1 + kk];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            part[v] = inside[v];
            part[5 + v] = JW * (v == 0 ? b0 + acc[0] : v == 4 ? b4 + acc[4] : acc[v]);
        }
        part[10] = JW;
    }
    __syncthreads();
#pragma unroll
    for (int x = 0; x < 11; ++x) sRed[x * NT + t] = part[x];
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int x = 0; x < 11; ++x) sRed[x * NT + t] += sRed[x * NT + t + w];
        __syncthreads();
    }
    if (t < NP)
#pragma unroll
        for (int v = 0; v < 5; ++v)
            dst[(v * Kdst + e) * NP + t] = acc[v] + (sRed[v * NT] - sRed[(5 + v) * NT]) / sRed[10 * NT];
}

// refinement between the shell pair: every fine element from its parent
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_shell_refine(const ShellXferArgs A) {
    constexpr int NP = Sz<N>::NP, NF = Sz<N>::NF;
    __shared__ double sT[5 * NP], sU[5 * NP], sM[3 * NF];
    const int64_t ef = blockIdx.x;
    const int nf = 2 * A.nc, nzf = 2 * A.nzc;
    const int iaf = (int)(ef % nf), ibf = (int)((ef / nf) % nf), irf = (int)((ef / ((int64_t)nf * nf)) % nzf);
    const int p = (int)(ef / ((int64_t)nf * nf * nzf));
    const int64_t ec = (((int64_t)p * A.nzc + (irf >> 1)) * A.nc + (ibf >> 1)) * A.nc + (iaf >> 1);
    const int child = (iaf & 1) | ((ibf & 1) << 1) | ((irf & 1) << 2);
    child_of_parent<N>(A.src, A.Ksrc, ec, A.dst, A.Kdst, ef, child, A.ops, sT, sU, sM, threadIdx.x);
}

// coarsening between the shell pair: every coarse element from its eight children
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_shell_coarsen(const ShellXferArgs A) {
    constexpr int N1 = N + 1, NP = Sz<N>::NP, NF = Sz<N>::NF;
    __shared__ double sT[5 * NP], sU[5 * NP], sR[2 * NF], sW[N1], sRed[11 * Sz<N>::NT];
    const int64_t ec = blockIdx.x;
    const int nc = A.nc, nzc = A.nzc, nf = 2 * nc, nzf = 2 * nzc;
    const int ia = (int)(ec % nc), ib = (int)((ec / nc) % nc), ir = (int)((ec / ((int64_t)nc * nc)) % nzc);
    const int p = (int)(ec / ((int64_t)nc * nc * nzc));
    int64_t kids[8];
    for (int a = 0; a < 8; ++a)
        kids[a] = (((int64_t)p * nzf + 2 * ir + (a >> 2)) * nf + 2 * ib + ((a >> 1) & 1)) * nf + 2 * ia + (a & 1);
    family_to_parent<N>(A.src, A.Ksrc, kids, A.dst, A.Kdst, ec, A.ops, A.met_src, A.met_dst, A.bg_src, A.bg_dst, sT,
                        sU, sR, sW, sRed, threadIdx.x);
}

// a refine or coarsen pass of a shell, along the target's plan: kind -1 copies
// leaf src, 0..7 is child kind of leaf src, 8 merges the family src..src+7
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_shell_plan(const ShellPlanArgs A) {
    constexpr int N1 = N + 1, NP = Sz<N>::NP, NF = Sz<N>::NF;
    __shared__ double sT[5 * NP], sU[5 * NP], sM[3 * NF], sW[N1], sRed[11 * Sz<N>::NT];
    const int64_t e = blockIdx.x;
    const int t = threadIdx.x;
    const int kind = A.xkind[e];
    const int64_t src = A.xsrc[e];
    if (kind < 0) {
        if (t < NP)
#pragma unroll
            for (int v = 0; v < 5; ++v) A.dst[(v * A.Kdst + e) * NP + t] = A.src[(v * A.Ksrc + src) * NP + t];
    } else if (kind < 8) {
        child_of_parent<N>(A.src, A.Ksrc, src, A.dst, A.Kdst, e, kind, A.ops, sT, sU, sM, t);
    } else {
        int64_t kids[8];
        for (int a = 0; a < 8; ++a) kids[a] = src + a;
        family_to_parent<N>(A.src, A.Ksrc, kids, A.dst, A.Kdst, e, A.ops, A.met_src, A.met_dst, A.bg_src, A.bg_dst,
                            sT, sU, sM, sW, sRed, t);
    }
}

// J W quadrature of rhobar + rho' over the leaves list[0..n), compensated sums:
// block b takes a contiguous share of the list, partial[b] = (sum, correction)
template <int N>
__global__ void __launch_bounds__(256) k_shell_mass(const double* q, const double* bg, const double* metric,
                                                    const double* w, const int32_t* list, int64_t n, int64_t K,
                                                    double* partial) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1, NT = 256;
    __shared__ Comp sh[4 * NT];
    const int t = threadIdx.x;
    Comp acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = blockIdx.x * per, i1 = (i0 + per < n) ? i0 + per : n;
    for (int64_t i = i0; i < i1; ++i) {
        const int64_t e = list[i];
        for (int nn = t; nn < NP; nn += NT) {
            const int ii = nn % N1, jj = (nn / N1) % N1, k = nn / (N1 * N1);
            const double W = metric[e * NP + nn] * w[ii] * w[jj] * w[k];
            acc[0] = comp_add(acc[0], W * (bg[e * N1 + k] + q[e * NP + nn]));
        }
    }
    block_reduce4<NT>(acc, sh);
    if (t == 0) {
        partial[blockIdx.x * 2 + 0] = acc[0].s;
        partial[blockIdx.x * 2 + 1] = acc[0].c;
    }
}

__global__ void __launch_bounds__(256) k_shell_mass_final(const double* partial, int nblk, double* out) {
    constexpr int NT = 256;
    __shared__ Comp sh[4 * NT];
    const int t = threadIdx.x;
    Comp acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int b = t; b < nblk; b += NT) acc[0] = comp_merge(acc[0], Comp{partial[b * 2], partial[b * 2 + 1]});
    block_reduce4<NT>(acc, sh);
    if (t == 0) out[0] = acc[0].s + acc[0].c;
}

// s = before[0] / after[0] on every conserved field of the leaves list[b]
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_shell_scale_list(double* q, const double* bg, int64_t K,
                                                                const int32_t* list, const double* before,
                                                                const double* after, double* s_out) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1;
    const int t = threadIdx.x;
    const int64_t e = list[blockIdx.x];
    const double s = before[0] / after[0];
    if (blockIdx.x == 0 && t == 0) s_out[0] = s;
    if (t >= NP) return;
    const int k = t / (N1 * N1);
    const int64_t KNP = K * NP, idx = e * NP + t;
    const double rb = bg[e * N1 + k], Tb = bg[K * N1 + e * N1 + k];
    q[idx] = s * q[idx] + (s - 1.0) * rb;
    q[KNP + idx] = s * q[KNP + idx];
    q[2 * KNP + idx] = s * q[2 * KNP + idx];
    q[3 * KNP + idx] = s * q[3 * KNP + idx];
    q[4 * KNP + idx] = s * q[4 * KNP + idx] + (s - 1.0) * Tb;
}

// the refinement's scale factor s = (total mass before) / (total mass after) on
// every conserved field of the fine shell: rho' <- s rho' + (s - 1) rhobar,
// U <- s U, Theta' <- s Theta' + (s - 1) Thetabar
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_shell_scale(double* q, const double* bg, int64_t K,
                                                           const double* tot_before, const double* tot_after,
                                                           double* s_out) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1;
    const int t = threadIdx.x;
    const int64_t e = blockIdx.x;
    const double s = tot_before[1] / tot_after[1];
    if (e == 0 && t == 0) s_out[0] = s;
    if (t >= NP) return;
    const int k = t / (N1 * N1);
    const int64_t KNP = K * NP, idx = e * NP + t;
    const double rb = bg[e * N1 + k], Tb = bg[K * N1 + e * N1 + k];
    q[idx] = s * q[idx] + (s - 1.0) * rb;
    q[KNP + idx] = s * q[KNP + idx];
    q[2 * KNP + idx] = s * q[2 * KNP + idx];
    q[3 * KNP + idx] = s * q[3 * KNP + idx];
    q[4 * KNP + idx] = s * q[4 * KNP + idx] + (s - 1.0) * Tb;
}


// ---------------------------------------------------------------- transposed shell transfers
// The transpose of the derivative of a pass's transfer (dg_sphere_adapt_project) at
// the state it was applied to.  Kept leaves copy qbar.  A refined parent p with
// children a (q_a = s (I_a q_p + B) - B, B the background part of each conserved
// field, s = M_c / M_f the ratio of the parents' mass to the interpolated
// children's): qbar_p = s sum_a I_a^T qbar_a, plus on rho' (dot / M_c) (w_p -
// s sum_a I_a^T w_a), dot = sum over all children of qbar . (q_to + B), w = J W (the
// derivative of s, through both masses).  A merged family (q_p = sum_a R_a q_a + c,
// c per field the constant of the J W integrals): qbar_a = R_a^T qbar_p + (sum of
// qbar_p over the parent's nodes / V_p) (w_a - R_a^T w_p), V_p = sum of w_p.

// sum over the leaves list[0..n) of qbar . (q + B) (B: rhobar on rho', Thetabar on
// Theta'), compensated; block b takes a contiguous share, partial[b] = (sum, correction)
template <int N>
__global__ void __launch_bounds__(256) k_shell_dot(const double* g, const double* q, const double* bg,
                                                   const int32_t* list, int64_t n, int64_t K, double* partial) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1, NT = 256;
    __shared__ Comp sh[4 * NT];
    const int t = threadIdx.x;
    Comp acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = blockIdx.x * per, i1 = (i0 + per < n) ? i0 + per : n;
    const int64_t KNP = K * NP;
    for (int64_t i = i0; i < i1; ++i) {
        const int64_t e = list[i];
        for (int nn = t; nn < NP; nn += NT) {
            const int k = nn / (N1 * N1);
            const int64_t x = e * NP + nn;
            double d = g[x] * (q[x] + bg[e * N1 + k]);
#pragma unroll
            for (int v = 1; v < 4; ++v) d = fma(g[v * KNP + x], q[v * KNP + x], d);
            d = fma(g[4 * KNP + x], q[4 * KNP + x] + bg[K * N1 + e * N1 + k], d);
            acc[0] = comp_add(acc[0], d);
        }
    }
    block_reduce4<NT>(acc, sh);
    if (t == 0) {
        partial[blockIdx.x * 2 + 0] = acc[0].s;
        partial[blockIdx.x * 2 + 1] = acc[0].c;
    }
}

// one workgroup per entry of the target's plan (a refined family is handled by the
// entry of its first child)
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_shell_plan_adjoint(const ShellPlanAdjArgs A) {
    constexpr int N1 = N + 1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    __shared__ double sP[6 * NP], sT[6 * NP], sU[6 * NP], sM[3 * NF], sRed[6 * NT];
    const int64_t e = blockIdx.x;
    const int t = threadIdx.x;
    const int kind = A.xkind[e];
    const int64_t src = A.xsrc[e];
    const int64_t Kf = A.Kfrom, Kt = A.Kto;
    const double* w1 = A.ops + 5 * NF;
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;
    const double Wn = t < NP ? w1[i] * w1[j] * w1[k] : 0.0;
    if (kind < 0) {
        if (t < NP)
#pragma unroll
            for (int v = 0; v < 5; ++v) A.gfrom[(v * Kf + src) * NP + t] = A.gto[(v * Kt + e) * NP + t];
        return;
    }
    if (kind > 0 && kind < 8) return;
    if (kind == 0) {
        // the refined parent src; its children are the entries e .. e + 7
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int a = 0; a < 8; ++a) {
            const int hal[3] = {a & 1, (a >> 1) & 1, a >> 2};
            const int64_t ec = e + a;
            if (t < NP) {
#pragma unroll
                for (int v = 0; v < 5; ++v) sT[v * NP + t] = A.gto[(v * Kt + ec) * NP + t];
                sT[5 * NP + t] = A.met_to[ec * NP + t] * Wn;
            }
            for (int x = t; x < 3 * NF; x += NT) {
                const int ax = x / NF;
                sM[x] = A.ops[5 * NF + N1 + hal[ax] * NF + (x - ax * NF)];  // I_0^T or I_1^T
            }
            __syncthreads();
            tile_pass<N, 6>(sT, sU, sM, 0, t);
            __syncthreads();
            tile_pass<N, 6>(sU, sT, sM + NF, 1, t);
            __syncthreads();
            tile_pass<N, 6>(sT, sU, sM + 2 * NF, 2, t);
            __syncthreads();
            if (t < NP)
#pragma unroll
                for (int f = 0; f < 6; ++f) acc[f] += sU[f * NP + t];
        }
        if (t < NP) {
            const double s = A.s;
            const double coef = A.dot[0] / A.mass[0];
            const double wp = A.met_from[src * NP + t] * Wn;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                double o = s * acc[v];
                if (v == 0) o = fma(coef, wp - s * acc[5], o);
                A.gfrom[(v * Kf + src) * NP + t] = o;
            }
        }
        return;
    }
    // a family src .. src + 7 merged into the target parent e: qbar_p and w_p into sP,
    // the per-field sums over the parent's nodes and its volume by one block reduction
    if (t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sP[v * NP + t] = A.gto[(v * Kt + e) * NP + t];
        sP[5 * NP + t] = A.met_to[e * NP + t] * Wn;
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) sRed[f * NT + t] = t < NP ? sP[f * NP + t] : 0.0;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int f = 0; f < 6; ++f) sRed[f * NT + t] += sRed[f * NT + t + w];
        __syncthreads();
    }
    double cpar[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) cpar[v] = sRed[v * NT] / sRed[5 * NT];
    for (int a = 0; a < 8; ++a) {
        const int hal[3] = {a & 1, (a >> 1) & 1, a >> 2};
        for (int x = t; x < 3 * NF; x += NT) {
            const int ax = x / NF;
            sM[x] = A.ops[7 * NF + N1 + hal[ax] * NF + (x - ax * NF)];  // R_0^T or R_1^T
        }
        __syncthreads();
        tile_pass<N, 6>(sP, sT, sM, 0, t);
        __syncthreads();
        tile_pass<N, 6>(sT, sU, sM + NF, 1, t);
        __syncthreads();
        tile_pass<N, 6>(sU, sT, sM + 2 * NF, 2, t);
        __syncthreads();
        if (t < NP) {
            const int64_t ea = src + a;
            const double wa = A.met_from[ea * NP + t] * Wn;
#pragma unroll
            for (int v = 0; v < 5; ++v)
                A.gfrom[(v * Kf + ea) * NP + t] = fma(cpar[v], wa - sT[5 * NP + t], sT[v * NP + t]);
        }
        __syncthreads();  // sM and sT are rewritten by the next child
    }
}

}  // namespace

// orders 2..5: the tile, the three contravariant flux planes and the face slots
// stay within 64 KB of LDS per workgroup (45 KB at N = 5)
#define DG_DISPATCH_N(N_, CALL)                                     \
    switch (N_) {                                                   \
        case 2: { constexpr int NN = 2; CALL; } break;              \
        case 3: { constexpr int NN = 3; CALL; } break;              \
        case 4: { constexpr int NN = 4; CALL; } break;              \
        case 5: { constexpr int NN = 5; CALL; } break;              \
        default: return hipErrorInvalidValue;                        \
    }

hipError_t launch_stage_sphere(int N, int mode, bool mixed, const SphereStageArgs& a, hipStream_t s) {
    if (a.K <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.K);
    if (mode == MODE_RHS) {
        if (mixed) {
            DG_DISPATCH_N(N, (k_stage_sphere<NN, MODE_RHS, true><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        } else {
            DG_DISPATCH_N(N, (k_stage_sphere<NN, MODE_RHS, false><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        }
    } else {
        if (mixed) {
            DG_DISPATCH_N(N, (k_stage_sphere<NN, MODE_RK, true><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        } else {
            DG_DISPATCH_N(N, (k_stage_sphere<NN, MODE_RK, false><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        }
    }
    return hipGetLastError();
}

hipError_t launch_node_coords_sphere(int64_t K, int N, const double* c1d, const int32_t* srec, double r_e,
                                     double* xyz, hipStream_t s) {
    const int64_t n = K * (N + 1) * (N + 1) * (N + 1);
    if (n <= 0) return hipSuccess;
    k_node_coords_sphere<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(K, N + 1, c1d, srec, r_e, xyz);
    return hipGetLastError();
}

// transfers: orders 2..7 (two tiles and three 1-D operators in LDS)
#define DG_DISPATCH_XFER(N_, CALL)                                  \
    switch (N_) {                                                   \
        case 2: { constexpr int NN = 2; CALL; } break;              \
        case 3: { constexpr int NN = 3; CALL; } break;              \
        case 4: { constexpr int NN = 4; CALL; } break;              \
        case 5: { constexpr int NN = 5; CALL; } break;              \
        case 6: { constexpr int NN = 6; CALL; } break;              \
        case 7: { constexpr int NN = 7; CALL; } break;              \
        default: return hipErrorInvalidValue;                        \
    }

hipError_t launch_shell_refine(int N, const ShellXferArgs& a, hipStream_t s) {
    if (a.Kdst <= 0) return hipSuccess;
    DG_DISPATCH_XFER(N, (k_shell_refine<NN><<<dim3((unsigned)a.Kdst), dim3(Sz<NN>::NT), 0, s>>>(a)));
    return hipGetLastError();
}

hipError_t launch_shell_coarsen(int N, const ShellXferArgs& a, hipStream_t s) {
    if (a.Kdst <= 0) return hipSuccess;
    DG_DISPATCH_XFER(N, (k_shell_coarsen<NN><<<dim3((unsigned)a.Kdst), dim3(Sz<NN>::NT), 0, s>>>(a)));
    return hipGetLastError();
}

hipError_t launch_shell_scale(int N, double* q, const double* bg, int64_t K, const double* tot_before,
                              const double* tot_after, double* s_out, hipStream_t s) {
    if (K <= 0) return hipSuccess;
    DG_DISPATCH_XFER(N, (k_shell_scale<NN><<<dim3((unsigned)K), dim3(Sz<NN>::NT), 0, s>>>(q, bg, K, tot_before,
                                                                                       tot_after, s_out)));
    return hipGetLastError();
}

hipError_t launch_mortar_sphere(int N, const SphereMortArgs& a, hipStream_t s) {
    if (a.n_hang <= 0) return hipSuccess;
    DG_DISPATCH_N(N, (k_mortar_sphere<NN><<<dim3((unsigned)a.n_hang), dim3(MortSz<NN>::NT), 0, s>>>(a)));
    return hipGetLastError();
}

hipError_t launch_mortar_sphere_adjoint(int N, const SphereMortAdjArgs& a, hipStream_t s) {
    if (a.n_hang <= 0) return hipSuccess;
    DG_DISPATCH_N(N, (k_mortar_sphere_adjoint<NN><<<dim3((unsigned)a.n_hang), dim3(MortSz<NN>::NT), 0, s>>>(a)));
    return hipGetLastError();
}

hipError_t launch_adjoint_sphere(int N, int mode, bool mixed, const SphereAdjArgs& a, hipStream_t s) {
    if (a.K <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.K);
    if (mode == MODE_RHS) {
        if (mixed) {
            DG_DISPATCH_N(N, (k_adjoint_sphere<NN, MODE_RHS, true><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        } else {
            DG_DISPATCH_N(N, (k_adjoint_sphere<NN, MODE_RHS, false><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        }
    } else {
        if (mixed) {
            DG_DISPATCH_N(N, (k_adjoint_sphere<NN, MODE_RK, true><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        } else {
            DG_DISPATCH_N(N, (k_adjoint_sphere<NN, MODE_RK, false><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
        }
    }
    return hipGetLastError();
}

hipError_t launch_shell_plan_adjoint(int N, const ShellPlanAdjArgs& a, hipStream_t s) {
    if (a.Kto <= 0) return hipSuccess;
    DG_DISPATCH_N(N, (k_shell_plan_adjoint<NN><<<dim3((unsigned)a.Kto), dim3(Sz<NN>::NT), 0, s>>>(a)));
    return hipGetLastError();
}

hipError_t launch_shell_dot(int N, const double* g, const double* q, const double* bg, const int32_t* list, int64_t n,
                            int64_t K, double* partial, int nblk, double* out, hipStream_t s) {
    if (nblk < 1) return hipErrorInvalidValue;
    if (n > 0) {
        DG_DISPATCH_N(N, (k_shell_dot<NN><<<dim3((unsigned)nblk), dim3(256), 0, s>>>(g, q, bg, list, n, K, partial)));
    }
    k_shell_mass_final<<<dim3(1), dim3(256), 0, s>>>(partial, n > 0 ? nblk : 0, out);
    return hipGetLastError();
}

hipError_t launch_shell_plan(int N, const ShellPlanArgs& a, hipStream_t s) {
    if (a.Kdst <= 0) return hipSuccess;
    DG_DISPATCH_XFER(N, (k_shell_plan<NN><<<dim3((unsigned)a.Kdst), dim3(Sz<NN>::NT), 0, s>>>(a)));
    return hipGetLastError();
}

hipError_t launch_shell_mass(int N, const double* q, const double* bg, const double* metric, const double* w,
                             const int32_t* list, int64_t n, int64_t K, double* partial, int nblk, double* out,
                             hipStream_t s) {
    if (nblk < 1) return hipErrorInvalidValue;
    if (n > 0) {
        DG_DISPATCH_XFER(N, (k_shell_mass<NN><<<dim3((unsigned)nblk), dim3(256), 0, s>>>(q, bg, metric, w, list, n, K,
                                                                                       partial)));
    }
    k_shell_mass_final<<<dim3(1), dim3(256), 0, s>>>(partial, n > 0 ? nblk : 0, out);
    return hipGetLastError();
}

hipError_t launch_shell_scale_list(int N, double* q, const double* bg, int64_t K, const int32_t* list, int64_t n,
                                   const double* tot_before, const double* tot_after, double* s_out,
                                   hipStream_t s) {
    if (n <= 0) return hipSuccess;
    DG_DISPATCH_XFER(N, (k_shell_scale_list<NN><<<dim3((unsigned)n), dim3(Sz<NN>::NT), 0, s>>>(
                            q, bg, K, list, tot_before, tot_after, s_out)));
    return hipGetLastError();
}

}  // namespace dgamr

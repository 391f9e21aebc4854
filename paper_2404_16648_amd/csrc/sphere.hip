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

template <int N, int MODE>
__global__ void __launch_bounds__(Sz<N>::NT) k_stage_sphere(const SphereStageArgs A) {
    constexpr int N1 = Sz<N>::N1, NP = Sz<N>::NP, NF = Sz<N>::NF, NT = Sz<N>::NT;
    __shared__ double sQ[5 * NP];
    __shared__ double sF[15 * NP];  // [i][v][node]: J a^i . F
    __shared__ double sS[30 * NF];  // [f][v][m]: lifted face terms
    __shared__ double sJ[NP];
    __shared__ double sD[N1 * N1];
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t* const rec = A.srec + e * kStageRec;
    const int t = threadIdx.x;
    const int64_t K = A.K, KNP = K * NP, KN1 = K * N1;
    const double gamma = A.gamma;
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;
    for (int ii = t; ii < N1 * N1; ii += NT) sD[ii] = A.ops[ii];
    double q[5] = {0, 0, 0, 0, 0}, R[5] = {0, 0, 0, 0, 0};
    double Jv = 1.0;
    if (t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) q[v] = A.qs[v * KNP + e * NP + t];
        Jv = A.metric[e * NP + t];
        double Ja[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) Ja[c] = A.metric[(1 + c) * KNP + e * NP + t];
        const Bg b = bg_make(A.bg[e * N1 + k], A.bg[KN1 + e * N1 + k], A.bg[2 * KN1 + e * N1 + k]);
        const double Pp = pprime(q[4], b.rTh, b.P, gamma, A.binom);
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
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int v = 0; v < 5; ++v)
                sF[(a * 5 + v) * NP + t] = Ja[a * 3 + 0] * F[0][v] + Ja[a * 3 + 1] * F[1][v] + Ja[a * 3 + 2] * F[2][v];
#pragma unroll
        for (int v = 0; v < 5; ++v) sQ[v * NP + t] = q[v];
        sJ[t] = Jv;
        // radial buoyancy -rho' g r_hat
        double cp[3];
        panel_point(rec[19], A.c1d[e * N1 + i], A.c1d[KN1 + e * N1 + j], cp);
        const double nrm = sqrt(cp[0] * cp[0] + cp[1] * cp[1] + cp[2] * cp[2]);
        const double gb = -q[0] * A.g;
#pragma unroll
        for (int c = 0; c < 3; ++c) R[1 + c] = gb * (cp[c] / nrm);
    }
    __syncthreads();

    // ---- faces: s F*(n) - sgn J a^d . F(q-), divided by J w_N at the face node
    const double wN = 2.0 / (N * (N + 1));  // the LGL end weight
    const int32_t packed = rec[18];
    for (int it = t; it < 6 * NF; it += NT) {
        const int f = it / NF, m = it % NF, d = f >> 1;
        const double sgn = (f & 1) ? 1.0 : -1.0;
        const int n = face_node<N>(f, m), kk = face_k<N>(f, m);
        double qL[5], qR[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qL[v] = sQ[v * NP + n];
        const Bg bL = bg_make(A.bg[e * N1 + kk], A.bg[KN1 + e * N1 + kk], A.bg[2 * KN1 + e * N1 + kk]);
        const double* fg = A.fgeo + ((e * 6 + f) * NF + m) * 4;
        const double nv[3] = {fg[0], fg[1], fg[2]};
        const double sface = fg[3];
        Bg bR = bL;
        if ((rec[f] & 0xff) == FT_WALL) {
            // mirror state: the normal momentum reversed
            const double Un = qL[1] * nv[0] + qL[2] * nv[1] + qL[3] * nv[2];
            qR[0] = qL[0];
#pragma unroll
            for (int c = 0; c < 3; ++c) qR[1 + c] = qL[1 + c] - (2.0 * Un) * nv[c];
            qR[4] = qL[4];
        } else {
            const int64_t e2 = rec[6 + f];
            const int f2 = (packed >> (4 * f)) & 7, flip = (packed >> (4 * f + 3)) & 1;
            const int a = m % N1, bb = m / N1;
            const int m2 = (flip ? N - a : a) + N1 * bb;
            const int n2 = face_node<N>(f2, m2), k2 = face_k<N>(f2, m2);
#pragma unroll
            for (int v = 0; v < 5; ++v) qR[v] = A.qs[v * KNP + e2 * NP + n2];
            bR = bg_make(A.bg[e2 * N1 + k2], A.bg[KN1 + e2 * N1 + k2], A.bg[2 * KN1 + e2 * N1 + k2]);
        }
        const double PpL = pprime(qL[4], bL.rTh, bL.P, gamma, A.binom);
        const double PpR = pprime(qR[4], bR.rTh, bR.P, gamma, A.binom);
        double FL[5], FR[5], lL, lR;
        flux_normal(qL, bL, PpL, nv, gamma, FL, lL);
        flux_normal(qR, bR, PpR, nv, gamma, FR, lR);
        const double lam = fmax(lL, lR);
        const double JwN = sJ[n] * wN;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double Fs = 0.5 * (FL[v] + FR[v]) + 0.5 * lam * (qL[v] - qR[v]);
            const double delta = sface * Fs - sgn * sF[(d * 5 + v) * NP + n];
            sS[(f * 5 + v) * NF + m] = delta / JwN;
        }
    }
    __syncthreads();
    if (t >= NP) return;

    // ---- volume: -(1/J) sum_i D_i (J a^i . F), then the face terms at face nodes
    double div[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int id = d == 0 ? i : d == 1 ? j : k;
        const int stride = d == 0 ? 1 : d == 1 ? N1 : NF;
        const int base = t - id * stride;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double* Fp = sF + (d * 5 + v) * NP + base;
            double acc = 0.0;
#pragma unroll
            for (int mm = 0; mm < N1; ++mm) acc = fma(sD[id * N1 + mm], Fp[mm * stride], acc);
            div[v] = div[v] + acc;
        }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) R[v] = -div[v] / Jv + R[v];
    // a node lies on at most one face per axis
    const int fm[3] = {j + N1 * k, i + N1 * k, i + N1 * j};
    const int ids[3] = {i, j, k};
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

// ---------------------------------------------------------------- shell transfers
// Between a shell (nc x nc per panel, nzc layers) and the shell with twice the
// elements per edge and twice the layers: child a = ax + 2 ay + 4 az of coarse
// element (p, ia, ib, ir) is fine element (p, 2 ia + ax, 2 ib + ay, 2 ir + az), and
// its reference box is half ax, ay, az of the parent's along the local axes.

// one separable pass over the five fields of a tile in LDS: out[v][node] =
// sum_m M[idx(node, axis)][m] in[v][node with that index replaced by m]
template <int N>
__device__ __forceinline__ void tile_pass(const double* in, double* out, const double* M, int axis, int t) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1, NF = N1 * N1;
    if (t >= NP) return;
    const int i = t % N1, j = (t / N1) % N1, k = t / NF;
    const int id = axis == 0 ? i : axis == 1 ? j : k;
    const int stride = axis == 0 ? 1 : axis == 1 ? N1 : NF;
    const int base = t - id * stride;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < N1; ++m) acc = fma(M[id * N1 + m], in[v * NP + base + m * stride], acc);
        out[v * NP + t] = acc;
    }
}

// refinement: every fine element is I_ax x I_ay x I_az of its parent
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_shell_refine(const ShellXferArgs A) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1, NF = N1 * N1, NT = Sz<N>::NT;
    __shared__ double sT[5 * NP], sU[5 * NP], sM[3 * NF];
    const int t = threadIdx.x;
    const int64_t ef = blockIdx.x;
    const int nf = 2 * A.nc, nzf = 2 * A.nzc;
    const int iaf = (int)(ef % nf), ibf = (int)((ef / nf) % nf), irf = (int)((ef / ((int64_t)nf * nf)) % nzf);
    const int p = (int)(ef / ((int64_t)nf * nf * nzf));
    const int64_t ec = (((int64_t)p * A.nzc + (irf >> 1)) * A.nc + (ibf >> 1)) * A.nc + (iaf >> 1);
    const int hal[3] = {iaf & 1, ibf & 1, irf & 1};
    for (int x = t; x < 3 * NF; x += NT) {
        const int ax = x / NF;
        sM[x] = A.ops[(1 + hal[ax]) * NF + (x - ax * NF)];  // I_0 or I_1
    }
    if (t < NP)
#pragma unroll
        for (int v = 0; v < 5; ++v) sT[v * NP + t] = A.src[(v * A.Ksrc + ec) * NP + t];
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
            A.dst[(v * A.Kdst + ef) * NP + t] = acc;
        }
    }
}

// coarsening: the parent is sum_a (R_ax x R_ay x R_az) q_a plus, per field, the
// constant sum_a (w_a - 1/8) m(q_a), w_a the child's volume fraction and m the mean
// over the reference cube, (1/8) sum W q
template <int N>
__global__ void __launch_bounds__(Sz<N>::NT) k_shell_coarsen(const ShellXferArgs A) {
    constexpr int N1 = N + 1, NP = N1 * N1 * N1, NF = N1 * N1, NT = Sz<N>::NT;
    __shared__ double sT[5 * NP], sU[5 * NP], sR[2 * NF], sW[N1], sShift[5];
    const int t = threadIdx.x;
    const int64_t ec = blockIdx.x;
    const int nc = A.nc, nzc = A.nzc, nf = 2 * nc, nzf = 2 * nzc;
    const int ia = (int)(ec % nc), ib = (int)((ec / nc) % nc), ir = (int)((ec / ((int64_t)nc * nc)) % nzc);
    const int p = (int)(ec / ((int64_t)nc * nc * nzc));
    for (int x = t; x < 2 * NF; x += NT) sR[x] = A.ops[3 * NF + x];  // R_0, R_1
    if (t < N1) sW[t] = A.ops[5 * NF + t];
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double shift = 0.0;  // thread v < 5: the constant of field v
    for (int a = 0; a < 8; ++a) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
        const int64_t ef = (((int64_t)p * nzf + 2 * ir + az) * nf + 2 * ib + ay) * nf + 2 * ia + ax;
        __syncthreads();  // the previous child's last pass has read sT
        if (t < NP)
#pragma unroll
            for (int v = 0; v < 5; ++v) sT[v * NP + t] = A.src[(v * A.Ksrc + ef) * NP + t];
        __syncthreads();
        if (t < 5) {
            double m = 0.0;
            for (int nn = 0; nn < NP; ++nn) {
                const int i = nn % N1, j = (nn / N1) % N1, k = nn / NF;
                m = fma(sW[i] * sW[j] * sW[k], sT[t * NP + nn], m);
            }
            shift = fma(A.cw[ef] - 0.125, 0.125 * m, shift);
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
    if (t < 5) sShift[t] = shift;
    __syncthreads();
    if (t < NP)
#pragma unroll
        for (int v = 0; v < 5; ++v) A.dst[(v * A.Kdst + ec) * NP + t] = acc[v] + sShift[v];
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

hipError_t launch_stage_sphere(int N, int mode, const SphereStageArgs& a, hipStream_t s) {
    if (a.K <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.K);
    if (mode == MODE_RHS) {
        DG_DISPATCH_N(N, (k_stage_sphere<NN, MODE_RHS><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
    } else {
        DG_DISPATCH_N(N, (k_stage_sphere<NN, MODE_RK><<<grid, dim3(Sz<NN>::NT), 0, s>>>(a)));
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

}  // namespace dgamr

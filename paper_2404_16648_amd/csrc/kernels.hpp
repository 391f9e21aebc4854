// Kernel argument blocks and launchers (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg.h"
#include "facetypes.hpp"

namespace dgamr {

// C(gamma, k), k = 1..kBinomTerms: binomial series of (1 + x)^gamma - 1 used for P'
// (seven terms: for |x| <= 2^-7 and 1 < gamma < 2 the truncation is below 1e-17
// relative)
constexpr int kBinomTerms = 7;
struct BinomCoef {
    double c[kBinomTerms];
};

constexpr int MODE_RHS = 0;
constexpr int MODE_RK = 1;
constexpr int MODE_RK_STREAM = 2;  // MODE_RK with q0 and the output streamed (non-temporal)
constexpr int MODE_RK_NOQ0 = 3;    // MODE_RK for a == 0: q0 never read (fewer registers)

// per-leaf record of the stage kernel's face tables: per face f its type (f), first
// neighbour (6 + f) and hanging-face row or -1 (12 + f); two ints of padding
constexpr int kStageRec = 20;

struct StageArgs {
    const double* q0;      // [5][K][Np] (read only when a != 0)
    const double* qs;      // [5][K][Np]
    double* out;           // [5][K][Np]
    const double* ops;     // D, I0, I1, R0, R1, w
    const double* geo;     // [K][4]
    const double* bg;      // [3][K][N1]
    const int32_t* ftype;  // [K][6]
    const int32_t* fnb;    // [K][6][4]
    const int32_t* hslot;  // [K][6]: row of the hanging-face table, or -1
    const double* mort;    // [n_hang][5][5][NF]: lifted mortar contributions (k_mortar)
    const int32_t* srec;   // [K][kStageRec]: face tables, one record per leaf
    int64_t K;
    double a, b, dt;
    double gamma, g;
    BinomCoef binom;
    int32_t stream_io;     // stage form: launch MODE_RK_STREAM
};

// adjoint: out = q^T-derivative qbar = (dR/dq)^T(q) lam (MODE_RHS) or
// out = a1 w1 + a2 w2 + b (lam + dt qbar) (MODE_RK)
struct AdjArgs {
    const double* q;
    const double* lam;
    const double* w1;
    const double* w2;
    double* out;
    const double* ops;     // D, I0, I1, R0, R1, w, I0^T, I1^T, R0^T, R1^T
    const double* geo;
    const double* bg;
    const int32_t* ftype;
    const int32_t* fnb;
    const int32_t* hslot;  // [K][6]: row of the hanging-face table, or -1
    const double* mort;    // [n_hang][5][5][NF]: mortar contributions to qbar (k_mortar_adjoint)
    int64_t K;
    double a1, a2, b, dt;
    double gamma, g;
    BinomCoef binom;
};

struct BgParams {
    int32_t kind;
    double cp, cv, P0, g, theta0, rho0, Theta0;
};

// mortar pre-pass of a stage: one workgroup per row of the hanging-face table
struct MortArgs {
    const double* qs;      // [5][K][Np] stage input
    double* mort;          // [n_hang][5][5][NF] output
    const double* ops;
    const double* geo;
    const double* bg;
    const int32_t* hang;   // [n_hang][6]: coarse leaf, its face, the 4 fine leaves by quadrant
    int64_t n_hang, K;
    double gamma;
    BinomCoef binom;
    int32_t pointwise;     // coarse side by pointwise matching instead of the mortar projection
};

// transposed mortar pre-pass: one workgroup per row of the hanging-face table;
// q the state, lam the adjoint weights, mort [n_hang][5][5][NF] the output
struct MortAdjArgs {
    const double* q;
    const double* lam;
    double* mort;
    const double* ops;     // with the transposes I_a^T, R_a^T
    const double* geo;
    const double* bg;
    const int32_t* hang;
    int64_t n_hang, K;
    double gamma;
    BinomCoef binom;
};

// One launch per transfer: the grid runs over the Kto entries of the target
// mesh's transfer plan (src, kind).  Forward: qin = q_from (Kin = K_from
// leaves), qout = q_to.  Transpose: qin = qbar_to (Kin = K_to), qout = qbar_from.
struct XferArgs {
    const double* qin;
    double* qout;
    const double* ops;
    const int32_t* src;
    const int32_t* kind;
    int64_t Kin, Kout, Kto;
    int32_t nvar;          // fields [nvar][K][Np], 1 <= nvar <= 5
};

// passive tracer stage: out = R_C(qs, cs) (MODE_RHS) or a c0 + b (cs + dt R_C) (MODE_RK)
struct TracerArgs {
    const double* qs;      // [5][K][Np] Euler stage input (the velocity and wave speed)
    const double* c0;      // [K][Np] (read only when a != 0)
    const double* cs;      // [K][Np] tracer stage input
    double* out;           // [K][Np]
    const double* ops;
    const double* geo;
    const double* bg;
    const int32_t* srec;   // [K][kStageRec]
    const double* mortC;   // [n_hang][5][NF]: lifted tracer mortar contributions
    int64_t K;
    double a, b, dt;
    double gamma;
    BinomCoef binom;
};

// tracer mortar pre-pass: one workgroup per hanging face
struct TracerMortArgs {
    const double* qs;
    const double* cs;
    double* mortC;         // [n_hang][5][NF] output
    const double* ops;
    const double* geo;
    const double* bg;
    const int32_t* hang;
    int64_t n_hang, K;
    double gamma;
    BinomCoef binom;
    int32_t pointwise;
};

// artificial viscosity, added to a stage's output: out += scale R_visc(q) with
// R_visc = div(mu grad q) in the two-pass central form
struct ViscArgs {
    const double* q;       // [5][K][Np] stage input
    double* sigma;         // [3][5][K][Np] workspace: the gradient, one field per axis
    double* out;           // [5][K][Np], accumulated into
    double* mort;          // [n_hang][5][5][NF] workspace: lifted central mortar terms
    const double* ops;
    const double* geo;
    const int32_t* srec;   // [K][kStageRec]
    const int32_t* hang;   // [n_hang][6]
    int64_t n_hang, K;
    double mu, scale;
};

// central averages on the mortars of the hanging faces: x + d axis_stride is the
// 5-variable field of the face's normal axis d; out as ViscArgs::mort, times mul
struct CentralMortArgs {
    const double* x;
    int64_t axis_stride;
    double* out;
    const double* ops;
    const double* geo;
    const int32_t* hang;
    int64_t n_hang, K;
    double mul;
};

// cubed-sphere shell stage: out = R(qs) (MODE_RHS) or a q0 + b (qs + dt R(qs)) (MODE_RK)
struct SphereStageArgs {
    const double* q0;
    const double* qs;
    double* out;
    const double* ops;     // D first
    const double* bg;      // [3][K][N1] as functions of the height
    const double* c1d;     // [3][K][N1]: tan of the panel angles, height
    const int32_t* srec;   // [K][kStageRec]: 18 = neighbour face | flip << 3 per face (4 bits), 19 = panel
    const double* metric;  // [10][K][Np]
    const double* fgeo;    // [K][6][NF][4]
    const double* mort;    // [n_hang][5][5][NF]: the mortar pre-pass output (hanging faces), or null
    int64_t K;
    double a, b, dt;
    double gamma, g;
    BinomCoef binom;
};

// the shell's mortar pre-pass: per hanging row (coarse leaf, its face, four fine
// leaves by quadrant) the lifted face terms of the coarse face (slot 0) and of the
// four fine faces (slots 1..4), each in its own face's node order
struct SphereMortArgs {
    const double* qs;
    double* mort;
    const double* ops;
    const double* bg;
    const int32_t* srec;
    const int32_t* hang;   // [n_hang][6]
    const double* metric;
    const double* fgeo;
    int64_t n_hang, K;
    double gamma;
    BinomCoef binom;
};
hipError_t launch_mortar_sphere(int N, const SphereMortArgs& a, hipStream_t s);

// transposed shell stage: out = (dR/dq)^T lam (MODE_RHS) or a1 w1 + a2 w2 + b (lam +
// dt (dR/dq)^T lam) (MODE_RK), R the shell's right-hand side at q
struct SphereAdjArgs {
    const double* q;
    const double* lam;
    const double* w1;
    const double* w2;
    double* out;
    const double* ops;     // D first
    const double* bg;
    const double* c1d;
    const int32_t* srec;
    const double* metric;
    const double* fgeo;
    const double* mort;    // [n_hang][5][5][NF]: the transposed mortar pre-pass output, or null
    int64_t K;
    double a1, a2, b, dt;
    double gamma, g;
    BinomCoef binom;
};
hipError_t launch_adjoint_sphere(int N, int mode, bool mixed, const SphereAdjArgs& a, hipStream_t s);

// transposed mortar pre-pass of the shell: per hanging row the contributions of the
// row's mortar terms to qbar at the coarse face (slot 0) and the four fine faces
// (slots 1..4), each in its own face's node order
struct SphereMortAdjArgs {
    const double* q;
    const double* lam;
    double* mort;
    const double* ops;
    const double* bg;
    const int32_t* srec;
    const int32_t* hang;
    const double* metric;
    const double* fgeo;
    int64_t n_hang, K;
    double gamma;
    BinomCoef binom;
};
hipError_t launch_mortar_sphere_adjoint(int N, const SphereMortAdjArgs& a, hipStream_t s);

// transfers of a shell's refine or coarsen pass along the plan (src, kind) of the
// target mesh: copies, children by reference interpolation, families by the
// reference projections plus the constant that keeps their J W integrals
struct ShellPlanArgs {
    const double* src;
    double* dst;
    const double* ops;
    const double* met_src;
    const double* met_dst;
    const double* bg_src;
    const double* bg_dst;
    const int32_t* xsrc;
    const int32_t* xkind;
    int64_t Ksrc, Kdst;
};
hipError_t launch_shell_plan(int N, const ShellPlanArgs& a, hipStream_t s);

// the transpose of a pass's shell transfer at the state it was applied to: qbar on
// the target (gto) to qbar on the source (gfrom); mass = the refined parents' mass
// under q_from, dot = sum over the children of qbar_to . (q_to + background), s the
// transfer's scale factor (device scalars mass, dot; read only with children)
struct ShellPlanAdjArgs {
    const double* gto;
    double* gfrom;
    const double* ops;
    const double* met_from;
    const double* met_to;
    const int32_t* xsrc;
    const int32_t* xkind;
    const double* mass;
    const double* dot;
    double s;
    int64_t Kfrom, Kto;
};
hipError_t launch_shell_plan_adjoint(int N, const ShellPlanAdjArgs& a, hipStream_t s);
hipError_t launch_shell_dot(int N, const double* g, const double* q, const double* bg, const int32_t* list, int64_t n,
                            int64_t K, double* partial, int nblk, double* out, hipStream_t s);
// J W quadrature of rhobar + rho' over the leaves list[0..n) (compensated sums):
// partial [nblk][2], the total to out[0]
hipError_t launch_shell_mass(int N, const double* q, const double* bg, const double* metric, const double* w,
                             const int32_t* list, int64_t n, int64_t K, double* partial, int nblk, double* out,
                             hipStream_t s);

struct BudgetArgs {
    const double* q;
    const double* bg;
    const double* geo;
    const double* Jn;      // [K][Np] per-node Jacobian (shell meshes), or null: geo's constant J
    const double* c1d;
    const double* w;
    double* partial;
    int64_t K;
    double gamma, g;
    BinomCoef binom;
};

struct IndArgs {
    const double* q;
    const double* bg;
    const double* geo;
    const double* ops;
    const int32_t* level;
    double* eta;
    int8_t* flags;
    int64_t K;
    int32_t kind, max_level;
    double thr;
    double gamma;          // DG_IND_PPRIME: P' from Theta'
    BinomCoef binom;
};

hipError_t launch_stage(int N, int mode, bool mixed, const StageArgs& a, hipStream_t s);
hipError_t launch_adjoint(int N, int mode, bool mixed, const AdjArgs& a, hipStream_t s);
hipError_t launch_background(int64_t K, int N, const double* c1d, double* bg, const BgParams& p, hipStream_t s);
hipError_t launch_init_bell(int64_t K, int N, const double* c1d, const double* bg, double theta0, const dg_bell& b,
                            double* q, hipStream_t s);
hipError_t launch_node_coords(int64_t K, int N, const double* c1d, double* xyz, hipStream_t s);
hipError_t launch_mortar(int N, const MortArgs& a, hipStream_t s);
hipError_t launch_mortar_adjoint(int N, const MortAdjArgs& a, hipStream_t s);
hipError_t launch_fma_burst(int blocks, int iters, double* sink, hipStream_t s);
// adjoint = false: the projection; true: its transpose
hipError_t launch_refine(int N, bool adjoint, const XferArgs& a, hipStream_t s);
hipError_t launch_coarsen(int N, bool adjoint, const XferArgs& a, hipStream_t s);
// the budget reduction runs at most kBudgetMaxBlocks blocks, each leaving 4
// compensated sums (8 doubles)
constexpr int kBudgetMaxBlocks = 1024;
constexpr int kBudgetScratchDoubles = 8 * kBudgetMaxBlocks;
constexpr int kMaxDevices = 64;
int budget_blocks(int64_t K);
// device address of the allocation-free budgets' partial sums on the current
// device (looked up once per device)
hipError_t budget_scratch(double** out);
hipError_t launch_budgets(int N, const BudgetArgs& a, int nblk, double* out_dev, hipStream_t s);
hipError_t launch_indicator(int N, const IndArgs& a, hipStream_t s);
hipError_t launch_tracer_mortar(int N, const TracerMortArgs& a, hipStream_t s);
hipError_t launch_tracer_stage(int N, int mode, const TracerArgs& a, hipStream_t s);
// the two viscous passes (mortars, gradient; mortars, divergence) on stream s
hipError_t launch_viscous(int N, const ViscArgs& a, hipStream_t s);
// cubed-sphere shell (N = 2..5): the stage and the node positions
hipError_t launch_stage_sphere(int N, int mode, bool mixed, const SphereStageArgs& a, hipStream_t s);
hipError_t launch_node_coords_sphere(int64_t K, int N, const double* c1d, const int32_t* srec, double r_e,
                                     double* xyz, hipStream_t s);
// transfers between a shell (nc per panel edge, nzc layers) and the shell with twice
// both (N = 2..7): refine reads the coarse src and writes the fine dst, coarsen the
// reverse; the coarsening's constant takes the J of both shells (metric plane 0) and
// their backgrounds
struct ShellXferArgs {
    const double* src;
    double* dst;
    const double* ops;
    const double* met_src;
    const double* met_dst;
    const double* bg_src;
    const double* bg_dst;
    int64_t Ksrc, Kdst;
    int nc, nzc;
};
hipError_t launch_shell_refine(int N, const ShellXferArgs& a, hipStream_t s);
hipError_t launch_shell_coarsen(int N, const ShellXferArgs& a, hipStream_t s);
// s = tot_before[1] / tot_after[1] on every conserved field of q (the fine shell), s to s_out[0]
hipError_t launch_shell_scale(int N, double* q, const double* bg, int64_t K, const double* tot_before,
                              const double* tot_after, double* s_out, hipStream_t s);
// the same with s = tot_before[0] / tot_after[0] on the leaves list[0..n) of q only
hipError_t launch_shell_scale_list(int N, double* q, const double* bg, int64_t K, const int32_t* list, int64_t n,
                                   const double* tot_before, const double* tot_after, double* s_out,
                                   hipStream_t s);
// integral of c [K][Np] with the weights J_e W_n (w the 1-D LGL weights): nblk <= budget_blocks(K)
// blocks leave 2 doubles each in partial, the total goes to out_dev[0]
hipError_t launch_weighted_sum(int N, const double* c, const double* geo, const double* w, int64_t K, int nblk,
                               double* partial, double* out_dev, hipStream_t s);

}  // namespace dgamr

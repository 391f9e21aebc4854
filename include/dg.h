/*
 * dg.h -- C ABI of the MI355X DG-AMR hot path.
 *
 * Nodal discontinuous Galerkin (dGSEM) right-hand side of the compressible Euler
 * equations in hydrostatic-perturbation form on 2:1-balanced oct-tree hexahedral
 * meshes with L2 mortars on hanging faces, the explicit SSP-RK3 stage update,
 * conservative refine/coarsen solution transfer, mass/energy budgets, the
 * adaptation indicator and the discrete adjoint of the right-hand side.
 *
 * Paper: Abdi, Almgren, Giraldo, Jankov, "Comparison of adaptive mesh refinement
 * techniques for numerical weather prediction", arXiv 2404.16648.
 *   equations and equation of state ............ section 2.1
 *   strong-form dGSEM, Rusanov flux ............. section 2.2
 *   forest of trees, leaves only ................ section 3.1
 *   conservative transfer and mortars ........... section 3.3
 *   2:1 balance ................................. section 4.3
 *
 * Conventions shared by every call
 *   - Field arrays are DEVICE pointers to float64, layout q[v][e][n]:
 *     v in {rho', rho*u, rho*v, rho*w, Theta'} (perturbations about the
 *     hydrostatic background for rho and Theta = rho*theta), e = leaf in the
 *     mesh's canonical order, n = i + (N+1)*(j + (N+1)*k) over the LGL nodes of
 *     the leaf (i along x fastest).  Size 5*K*Np doubles, Np = (N+1)^3.
 *   - The caller owns every field buffer; the library owns the mesh handle, its
 *     host tables, its device tables, background profiles and workspaces.
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *     Field calls only enqueue work (asynchronous); dg_budgets and
 *     dg_indicator (flags copied to the host) synchronise the stream.  A mesh's
 *     device tables are uploaded by the first call that uses the mesh on the
 *     GPU (synchronous, on the device that was current at dg_mesh_build); a
 *     mesh that is only inspected on the host costs no device memory.
 *   - Every function returns a dg_status; nothing throws across the ABI.  On an
 *     error the outputs are unspecified, handles stay valid, and
 *     dg_last_error() returns a message (thread-local).  Faults of kernels
 *     already enqueued surface at the next synchronising call as DG_EHIP.
 *   - Aliasing: outputs must not alias inputs unless stated.
 */
#ifndef DGAMR_DG_H
#define DGAMR_DG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dg_status;
#define DG_OK            0
#define DG_EINVAL       -1   /* bad argument, unsupported size, wrong mesh pair */
#define DG_ENOMEM       -2   /* host or device allocation failed */
#define DG_EHIP         -3   /* a HIP runtime call or a kernel failed */
#define DG_EUNSUPPORTED -4   /* valid request the build does not provide */
#define DG_ENONFINITE   -5   /* a budget or indicator saw a non-finite value */

#define DG_PASS_COARSEN 0
#define DG_PASS_REFINE  1

#define DG_BG_NEUTRAL   0    /* constant theta0: exner = 1 - g z/(cp theta0) */
#define DG_BG_CONSTANT  1    /* rhobar = rho0, Thetabar = Theta0 everywhere  */
#define DG_BG_ISOTHERMAL 2   /* temperature theta0 everywhere (section 4.4's
                                shell): Pbar = P0 exp(-g z/(R theta0)),
                                rhobar = Pbar/(R theta0); z = height */

#define DG_FP64         0    /* every operation in float64 */
#define DG_MIXED        1    /* volume flux contractions in float32, rest float64 */

#define DG_NC_MORTAR    0    /* hanging faces: L2 mortars (section 3.3; conservative) */
#define DG_NC_POINTWISE 1    /* hanging faces: pointwise matching (section 3.3's simpler
                                alternative; not conservative, forward calls only) */

#define DG_IND_THETA      0  /* eta_e = max |theta'| over the leaf's nodes   */
#define DG_IND_GRAD_THETA 1  /* eta_e = max |grad theta| over the leaf's nodes */
#define DG_IND_PPRIME     2  /* eta_e = max |P'| over the leaf's nodes (section 4.4 regrids on it) */

#define DG_KIND_COPY   -1    /* transfer: new leaf is old leaf src */
#define DG_KIND_FAMILY  8    /* transfer: new leaf is the parent of old src..src+7 */

typedef struct dg_mesh dg_mesh;   /* opaque */

/* Brick forest: nx*ny*nz root hexes tiling [lo,hi], trees refined up to
 * max_level (<= 12), polynomial order N (2..7).  periodic[d] = 1 joins the two
 * faces normal to axis d, 0 makes them no-flux walls.  host_only = 1 builds the
 * host tables only (no device memory; field calls on such a mesh fail with
 * DG_EINVAL) -- used to check the integer tables on machines without a GPU. */
typedef struct {
    int32_t N, nx, ny, nz, max_level;
    int32_t periodic[3];
    double lo[3], hi[3];
    int32_t host_only;
} dg_forest_desc;

/* A cubed-sphere shell (section 3.4 spherical geometry, section 4.4 global
 * tests): six equiangular panels of n x n elements, nz layers between the radii
 * r_e and r_e + H, order N; elements are isoparametric (the mapping is
 * interpolated at the LGL nodes).  Element e = ((p nz + ir) n + ib) n + ia for
 * panel p, row ib, column ia, layer ir; reference axes: the panel's two angles,
 * then outward.  host_only as for dg_forest_desc. */
typedef struct {
    int32_t N, n, nz;
    double r_e, H;
    int32_t host_only;
    int32_t max_level;   /* refinement levels allowed above the unrefined shell (0: none) */
} dg_sphere_desc;

/* Gas constants (section 2.1: R = cp - cv, gamma = cp/cv, P = P0 (R Theta/P0)^gamma),
 * gravity g and the hydrostatic background (section 2.1 perturbation form;
 * neutral profile of section 4.3).  precision selects DG_FP64 or DG_MIXED;
 * nonconforming selects the hanging-face scheme, DG_NC_MORTAR or
 * DG_NC_POINTWISE (the fine side solves its Riemann problem against the coarse
 * polynomial at its nodes, the coarse side against the fine polynomial at its
 * nodes, averaged over the quadrants on a shared mid-line, with no projection;
 * the adjoint calls return DG_EUNSUPPORTED for it).  mu >= 0 is an artificial
 * viscosity in m^2/s (section 4.3 runs the rising bubble with mu = 1.5): when
 * positive, dg_rhs and dg_rk_stage add div(mu grad q') of every perturbation
 * variable (a reading: the paper gives the coefficient, not the operator),
 * discretised by the two-pass central scheme with mortars on hanging faces and
 * no diffusive flux through walls; the adjoint calls return DG_EUNSUPPORTED for
 * mu > 0, and the passive tracer is not diffused. */
typedef struct {
    double cp, cv, P0, g;
    int32_t background;
    int32_t precision;
    double theta0, rho0, Theta0;
    int32_t nonconforming;
    double mu;
} dg_phys;

typedef struct {
    int64_t K;            /* number of leaves */
    int64_t Np;           /* (N+1)^3 */
    int64_t n_conf;       /* conforming interior faces (incl. periodic wraps) */
    int64_t n_bnd;        /* wall faces */
    int64_t n_hang;       /* hanging faces (each = 1 coarse + 4 fine) */
    int64_t n_refined;    /* old leaves refined by the pass that built this mesh */
    int64_t n_coarsened;  /* families merged by the pass that built this mesh */
    int32_t N;
    int32_t max_level_present;
} dg_mesh_info;

/* Host copies of the integer tables (caller allocates, sizes from dg_mesh_info).
 *   leaf [K][5]       (root, level, ix, iy, iz), root = rx + nx*(ry + ny*rz)
 *   conf [n_conf][3]  (eM, eP, d): plus face of eM meets minus face of eP
 *   bnd  [n_bnd][2]   (e, f), f = 2*d + s (s = 1 plus side)
 *   hang [n_hang][6]  (ec, f, e0, e1, e2, e3): coarse leaf ec's face f is
 *                     covered by fine leaves ordered by quadrant a + 2b over
 *                     the two tangential axes in increasing axis order
 *   xfer_src/kind [K] transfer plan from the previous mesh (DG_KIND_*, or the
 *                     child id 0..7 = a + 2b + 4c of old leaf src)
 * Any pointer may be NULL to skip that table. */
typedef struct {
    int32_t* leaf;
    int32_t* conf;
    int32_t* bnd;
    int32_t* hang;
    int32_t* xfer_src;
    int32_t* xfer_kind;
} dg_mesh_tables;

/* Initial perturbation (row "background + IC"): a cosine bell of potential
 * temperature dtheta * (1 + cos(pi r))/2 for r <= 1, r^2 = sum_d ((x_d - c_d)/r_d)^2
 * over the axes with r_d > 0 (r_d = 0 drops that axis), at unperturbed
 * hydrostatic pressure: Theta' = 0, rho' = -rhobar theta'/(theta0 + theta'),
 * U = 0 (sections 4.2 and 4.3 cosine bell and rising bubble). */
typedef struct {
    double dtheta;
    double centre[3];
    double radius[3];
} dg_bell;

/* Build a mesh (section 3.1: every root hex is a tree and only leaves are kept,
 * flagged leaves replaced by their children or merged into their parent;
 * section 4.3: 2:1 balance; the leaf order, balance algorithm and table formats
 * are not in the paper: leaves follow one Morton curve over the brick, roots in
 * Morton order of their coordinates, then the Morton order inside the root).
 * prev == NULL: uniform level-0 forest from desc (flags, pass ignored).  Otherwise one pass over prev (desc is taken from prev and the
 * argument may be NULL): DG_PASS_REFINE applies the +1 flags of `flags` (host
 * int8[K(prev)]) to leaves below max_level and then refines every leaf that
 * has a face neighbour two or more levels finer, to a fixed point (2:1 face
 * balance, periodic wraps included).  DG_PASS_COARSEN merges every family of 8
 * sibling leaves that are all flagged -1 unless a leaf face-adjacent to the
 * parent is two or more levels finer than the parent (judged on prev).
 * On success *out is a new handle (free with dg_mesh_free) whose transfer
 * plan refers to prev; prev must stay alive while it is used by the
 * projections.  Host work only (the device copy is made at first GPU use). */
dg_status dg_mesh_build(const dg_forest_desc* desc, const dg_mesh* prev, const int8_t* flags,
                        int32_t pass, dg_mesh** out);

/* Build a uniform cubed-sphere shell mesh (sections 3.4, 4.4; the equiangular
 * panels, their orientation and the element order are not in the paper).
 * Walls at the bottom and top (mirror state), every lateral face conforming,
 * across panel edges with the neighbour's face and orientation recorded.  The
 * geometry is made on the host at first GPU use: node positions from the exact
 * mapping, metric terms J a^i in the conservative curl form (so a uniform flow
 * stays uniform up to rounding), the Jacobian, and per face node the unit
 * normal and face Jacobian, taken for a shared face from the (leaf, face) pair
 * that comes first so that both sides use bitwise-opposite normals.  dg_rhs,
 * dg_rk_stage, dg_budgets and dg_node_coords accept such meshes (float64,
 * mu = 0, mortars at hanging faces; background z is the height above r_e), and
 * the dg_sphere_* transfers between a shell and the shell with twice its
 * resolution.  With desc->max_level > 0 the shell is the root level of a forest
 * of oct-trees (section 3.1) and dg_mesh_build(prev = shell, flags, pass) refines
 * or coarsens it with 2:1 balance across faces, also across panel edges; hanging
 * faces take curved mortars (the coarse trace interpolated to the fine face nodes,
 * the Riemann problem along the fine face's normal, the coarse side's flux
 * 4 s_f (-F*) per coarse reference area projected back), and dg_indicator (theta'
 * or P'), dg_pass_changes, dg_flags_after_coarsen, dg_flags_buffer and
 * dg_sphere_adapt_project accept them.  dg_rhs_adjoint and dg_rk_stage_adjoint
 * accept shells: the transpose of the curvilinear right-hand side, with the
 * curved mortars transposed in their own pre-pass.  The precision split
 * (DG_MIXED) runs the stage's line contractions in float32 (G_d minus its value
 * at the element's first node, D in float32 high and low parts, float32
 * accumulation; faces, mortars, metric terms and the update in float64), and the
 * adjoint's transposed contractions D^T (-lam/J) in float32 likewise.  The
 * tracer, viscosity and pointwise matching return DG_EUNSUPPORTED.  N = 2..5.
 * DG_EINVAL on bad sizes. */
dg_status dg_sphere_mesh_build(const dg_sphere_desc* desc, dg_mesh** out);
/* Face connectivity of a shell mesh (not in the paper): nb[K][6][3] (host,
 * caller-owned) = neighbour element (-1 at the walls), its face, and 1 when
 * the neighbour's face-local first axis runs opposite (on a refined shell, see
 * dg_sphere_face_kinds for the hanging faces).  Host only.  DG_EINVAL for a NULL
 * argument or a brick mesh. */
dg_status dg_sphere_faces(const dg_mesh* mesh, int32_t* nb);
/* Geometry of a shell mesh into host arrays (caller-owned): metric[10][K][Np]
 * (J, then J a^i_c at 1 + 3 i + c, c the Cartesian component), fgeo
 * [K][6][(N+1)^2][4] (unit outward normal, face Jacobian |J a^d|), c1d
 * [3][K][N+1] (tan of the two panel angles, height above r_e).  Host only.
 * DG_EINVAL for a NULL argument or a brick mesh. */
dg_status dg_sphere_geometry(const dg_mesh* mesh, double* metric, double* fgeo, double* c1d);
/* Volumes of a shell's elements (section 3.4: areas of the curved elements from
 * the spherical excess of their footprints, and the volume loss of a
 * refinement).  vol (host [K], caller-owned, or NULL): each element's footprint
 * area on the unit sphere (spherical excess of its two great-circle triangles,
 * by the formula of Van Oosterom and Strackee) times (r_top^3 - r_bot^3)/3;
 * these add up exactly across a refinement.  totals (host [2]): the volume the
 * isoparametric elements enclose (J W summed over every node, from the same
 * geometry the kernels use) and the sum of vol; the volume loss of a
 * refinement is the relative change of totals[0] between the two shells.
 * Host work (one evaluation of the geometry).  DG_EINVAL for a NULL totals or a
 * brick mesh. */
dg_status dg_sphere_volumes(const dg_mesh* mesh, double* vol, double* totals);
/* Refinement transfer from a shell to the shell with twice the elements per
 * panel edge and twice the layers (same N, r_e, H), section 3.4 (b) with the
 * reference matrices only: each fine element (p, 2 ia + ax, 2 ib + ay,
 * 2 ir + az) takes I_ax x I_ay x I_az of its parent, then one scale factor
 * s = (total mass of the coarse state) / (total mass of the interpolated
 * state), both the J W quadrature of rhobar + rho' on their own shell,
 * multiplies every conserved field of every fine element, background included
 * (rho' := s rho' + (s - 1) rhobar, U := s U, Theta' := s Theta' + (s - 1)
 * Thetabar; a reading: velocity and potential temperature keep their
 * interpolated values).  q_coarse, q_fine: device [5][K][Np] of their shells,
 * caller-owned, not aliased; phys without viscosity (its background gives
 * rhobar, Thetabar; the transfer runs in float64 for either precision).  If
 * scale (host) is not NULL it receives s and the call waits for the stream;
 * otherwise the call only enqueues.  Uses both meshes' reduction workspaces.
 * DG_EINVAL for shells that are not such a pair; DG_EUNSUPPORTED for mu > 0;
 * DG_ENONFINITE for a non-finite s (only when scale is requested). */
dg_status dg_sphere_refine_project(const dg_mesh* coarse, const dg_mesh* fine, const dg_phys* phys,
                                   const double* q_coarse, double* q_fine, double* scale, void* stream);
/* Coarsening transfer, the reverse pair, section 3.4 (a): each coarse element
 * is the sum over its eight children of R_ax x R_ay x R_az q_a (the reference
 * projection) plus, per conserved field, the constant that makes the element's
 * J W integral the sum of its children's (each child weighs in with its own
 * volume integral, a finite-volume balance on the elements' discrete volumes; rho'
 * and Theta' are balanced with their background, so the total mass and Theta are
 * kept exactly).  A reading: the paper weighs each child by its volume without
 * fixing the measure; this one keeps the quadrature the solver conserves.  phys
 * gives the backgrounds.  Fields as for dg_sphere_refine_project; enqueued on
 * stream.  DG_EINVAL for shells that are not such a pair. */
dg_status dg_sphere_coarsen_project(const dg_mesh* fine, const dg_mesh* coarse, const dg_phys* phys,
                                    const double* q_fine, double* q_coarse, void* stream);
/* The transfer of a refine or coarsen pass of a shell built with max_level > 0
 * (section 3.4's transfer on curved elements, with the reference matrices only):
 * `to` was built by dg_mesh_build(prev = from, ...).  Kept leaves are copied; a
 * child takes I_ax x I_ay x I_az of its parent, and one scale factor s = (mass of
 * the refined parents) / (mass of their interpolated children), both the J W
 * quadrature of rhobar + rho', multiplies every conserved field of every child,
 * background included, as in dg_sphere_refine_project; a merged family becomes the
 * sum of its children's reference projections plus the constant that keeps its
 * J W integrals, as in dg_sphere_coarsen_project: both passes keep the total
 * mass and Theta exactly.  q_from, q_to: device [5][K][Np] of their meshes,
 * caller-owned, not aliased; phys without viscosity (float64 for either
 * precision).  If scale (host) is not NULL it receives s (1 when nothing was
 * refined) and the call waits for the stream; otherwise it only enqueues.  Uses
 * both meshes' reduction workspaces.  DG_EINVAL for meshes that are not such a
 * pair; DG_EUNSUPPORTED for mu > 0. */
dg_status dg_sphere_adapt_project(const dg_mesh* from, const dg_mesh* to, const dg_phys* phys, const double* q_from,
                                  double* q_to, double* scale, void* stream);
/* Not in the paper (the adjoint through a shell's adaptation): the transpose of the
 * derivative of dg_sphere_adapt_project at q_from, qbar_from := (dq_to/dq_from)^T
 * qbar_to in the Euclidean inner product on the DOF vectors.  Kept leaves copy
 * qbar.  A refined parent p gets s sum_a (I_a x I_a x I_a)^T qbar_a over its
 * children, plus on rho' (D / M) (w_p - s sum_a (I_a x I_a x I_a)^T w_a): w = J W,
 * M the refined parents' mass under q_from, D the sum over every child of
 * qbar_to . (q_to + background) (the derivative of the scale factor s through
 * both masses).  A merged family's child a gets (R_a x R_a x R_a)^T qbar_p plus,
 * per field, (the sum of qbar_p over the parent's nodes / the parent's J W volume)
 * (w_a - (R_a x R_a x R_a)^T w_p) (the derivative of the integral constant).
 * q_from, q_to: the forward call's input and output, scale its factor (host);
 * needed, and checked, only when the pass refines (may be NULL otherwise).
 * qbar_to [5][K_to][Np], qbar_from [5][K_from][Np]: device, caller-owned, not
 * aliased; every entry of qbar_from is written.  Uses both meshes' reduction
 * workspaces; enqueued on stream.  DG_EINVAL as dg_sphere_adapt_project, for a
 * non-positive or non-finite scale, or a plan whose refined families are not
 * consecutive; DG_EUNSUPPORTED for mu > 0. */
dg_status dg_sphere_adapt_project_adjoint(const dg_mesh* from, const dg_mesh* to, const dg_phys* phys,
                                          const double* q_from, const double* q_to, double scale,
                                          const double* qbar_to, double* qbar_from, void* stream);
/* Face kinds of a shell (section 3.1's tree on the panels; the encoding is not in
 * the paper): kind[K][6] (host, caller-owned) = 0 wall, 1 conforming, 2 fine side
 * of a hanging face + 4 * its quadrant in the coarse face's axes, 3 coarse side.
 * dg_sphere_faces then gives per face the neighbour, its face and the flip
 * (conforming), the coarse leaf, its face and the flip (fine side), or the row of
 * the hanging-face table of dg_mesh_export, the fine leaves' face and the flip
 * (coarse side).  Host only.  DG_EINVAL for a NULL argument or a brick mesh. */
dg_status dg_sphere_face_kinds(const dg_mesh* mesh, int32_t* kind);
/* Whether dg_mesh_build(prev = mesh, flags, pass) would change a leaf of mesh
 * (section 3.1: a refine pass splits leaves flagged +1 below max_level; a
 * coarsen pass merges complete sibling families flagged -1 that pass the 2:1
 * veto): *changes = 1 if so, else 0.  Host work only, nothing allocated for a
 * result, so a caller can skip building a mesh equal to its input.  flags is
 * host int8[K] as for dg_mesh_build.  DG_EINVAL on a NULL argument or an
 * unknown pass. */
dg_status dg_pass_changes(const dg_mesh* mesh, const int8_t* flags, int32_t pass, int32_t* changes);

/* Release a mesh handle with its host tables and device block (not in the
 * paper; handle management).  NULL is accepted.  Work still enqueued on the
 * mesh must have completed (the device block is freed). */
dg_status dg_mesh_free(dg_mesh* mesh);
/* Sizes of a mesh (not in the paper): leaves, nodes per leaf, face counts and the
 * pass that built it; host only.  DG_EINVAL on a NULL argument. */
dg_status dg_mesh_info_get(const dg_mesh* mesh, dg_mesh_info* info);
/* Host copies of the integer tables into caller-owned arrays sized from
 * dg_mesh_info (the tables of section 3.1's forest, formats not in the paper);
 * host only.  DG_EINVAL on a NULL argument. */
dg_status dg_mesh_export(const dg_mesh* mesh, const dg_mesh_tables* tables);

/* Node coordinates xyz[3][K][Np] (device, float64, caller-owned) of the LGL
 * nodes (section 2.2 nodal dGSEM; the mapping of a brick leaf is not in the
 * paper): x = lo + (hi-lo)/n * (r + (anchor + (1 + xi)/2) / 2^level) per axis,
 * in this association so that two leaves sharing a face give bitwise-identical
 * coordinates there.  Enqueued on stream.  DG_EINVAL on a NULL argument. */
dg_status dg_node_coords(const dg_mesh* mesh, double* xyz, void* stream);

/* q (device [5][K][Np], caller-owned) := the cosine-bell perturbation described
 * by *bell about phys's background (sections 4.2 and 4.3; see dg_bell).
 * Enqueued on stream.  DG_EINVAL on a NULL argument or bad phys. */
dg_status dg_init_bell(const dg_mesh* mesh, const dg_phys* phys, const dg_bell* bell, double* q,
                       void* stream);

/* rhs := R(q), the strong-form dGSEM right-hand side (section 2.2):
 *   R = -sum_d (2/h_d) D_d F^d(q) + S(q) - lift((F* - F(q-)).n)
 * with F the Euler flux carrying the pressure perturbation P', S the buoyancy
 * -rho' g on rho*w, F* the Rusanov flux (local max wave speed, jump of the
 * perturbation variables), mirror states at walls and L2 mortars on hanging
 * faces (section 3.3).  rhs must not alias q.  A mesh periodic along z needs
 * a background constant in z (g = 0 or DG_BG_CONSTANT; a hydrostatic profile
 * cannot be periodic), else DG_EINVAL (also for the stage and adjoint calls).  The mortars are evaluated by a
 * pre-pass into a workspace owned by the mesh, so calls of dg_rhs,
 * dg_rk_stage, dg_rhs_adjoint and dg_rk_stage_adjoint on one mesh must be
 * ordered (one stream, or synchronised); concurrent calls on different meshes
 * are independent. */
dg_status dg_rhs(const dg_mesh* mesh, const dg_phys* phys, const double* q, double* rhs,
                 void* stream);

/* One Shu-Osher stage: qout := a*q0 + b*(qs + dt*R(qs)), with R as in dg_rhs
 * (sections 2.2 and 3.3) fused into the update; the paper integrates with an
 * explicit Runge-Kutta scheme, SSP-RK3 (not named in the paper) uses
 * (a,b) = (0,1), (3/4,1/4), (1/3,2/3).  Device fields [5][K][Np]; qout may
 * alias q0 but not qs; q0 is not read when a == 0.  Enqueued on stream (mortar
 * pre-pass, then the fused kernel).  DG_EINVAL on NULL or aliased fields or bad
 * phys. */
dg_status dg_rk_stage(const dg_mesh* mesh, const dg_phys* phys, double a, double b, double dt,
                      const double* q0, const double* qs, double* qout, void* stream);

/* Conservative transfer (section 3.3): `to` must have been built by a pass over
 * `from`.  Refine: a child (a,b,c) gets (I_a x I_b x I_c) q_parent, I_a the
 * interpolation of the parent polynomial to half-interval a (equal to the L2
 * projection there).  Coarsen: the parent gets sum over the 8 children of
 * (R_a x R_b x R_c) q_child, R_a = 1/2 M^{-1} I_a^T M with the exact mass
 * matrix M (integrals are preserved).  Kept leaves are copied.  q_to must
 * not alias q_from. */
dg_status dg_refine_project(const dg_mesh* from, const dg_mesh* to, const double* q_from,
                            double* q_to, void* stream);
dg_status dg_coarsen_project(const dg_mesh* from, const dg_mesh* to, const double* q_from,
                             double* q_to, void* stream);

/* The same conservative transfer for any set of nvar fields [nvar][K][Np]
 * (1 <= nvar <= 5; e.g. a passive tracer, nvar = 1), in the direction of the
 * pass that built `to` (refine, or coarsen; a pass that changed no leaf copies).
 * Same checks and errors as dg_refine_project; DG_EINVAL for nvar out of range.
 * (Section 3.3: the same projection matrices serve every field.) */
dg_status dg_project_fields(const dg_mesh* from, const dg_mesh* to, int32_t nvar, const double* q_from,
                            double* q_to, void* stream);

/* Transposes of the transfers, for the adjoint through an adaptation: with P
 * the linear map q_from -> q_to of dg_refine_project (resp.
 * dg_coarsen_project) from `from` to `to`, qbar_from := P^T qbar_to in the
 * Euclidean inner product on the DOF vectors.  Refine: a refined leaf gets
 * sum over its 8 children of (I_a x I_b x I_c)^T qbar_child.  Coarsen: each
 * child of a merged parent gets (R_a x R_b x R_c)^T qbar_parent.  Kept leaves
 * are copied.  qbar_to is [5][K_to][Np], qbar_from [5][K_from][Np] (every
 * entry written), device pointers on `to`'s device; they must not alias.
 * Same checks and error codes as the forward transfers. */
dg_status dg_refine_project_adjoint(const dg_mesh* from, const dg_mesh* to, const double* qbar_to,
                                    double* qbar_from, void* stream);
dg_status dg_coarsen_project_adjoint(const dg_mesh* from, const dg_mesh* to, const double* qbar_to,
                                     double* qbar_from, void* stream);

/* Not in the paper (the discrete adjoint of section 2.2's right-hand side):
 * qbar := (dR/dq)^T lam, the exact transpose of the linearised right-hand side
 * in the Euclidean inner product on the DOF vector (d|x|/dx := 0 at 0, a max
 * tie splits the derivative 1/2, 1/2).  qbar must not alias q or lam.  With
 * phys->precision == DG_MIXED the transposed volume contractions D^T lam run in
 * float32 (lam rounded to float32, D split into float32 high and low parts,
 * float32 accumulation); faces, mortars, the chain rule and the output stay
 * float64 (relative error of the order 1e-7 against the float64 transpose).
 * The transposed mortars run as a pre-pass into the mesh's mortar workspace
 * (ordering as for dg_rhs). */
dg_status dg_rhs_adjoint(const dg_mesh* mesh, const dg_phys* phys, const double* q,
                         const double* lam, double* qbar, void* stream);

/* Transposed Shu-Osher stage, the building block of the reverse SSP-RK3 step:
 *   out := a1*w1 + a2*w2 + b*(y + dt*(dR/dq)^T(q) y)
 * with the same transpose as dg_rhs_adjoint evaluated at the stage input q.
 * For the forward stages q1 = q0 + dt R(q0), q2 = 3/4 q0 + 1/4 (q1 + dt R(q1)),
 * q3 = 1/3 q0 + 2/3 (q2 + dt R(q2)) and lam3 = dJ/dq3:
 *   lam2 = (0, -, 0, -, 2/3, dt, q2, lam3),  lam1 = (0, -, 0, -, 1/4, dt, q1, lam2),
 *   dJ/dq0 = (1/3, lam3, 3/4, lam2, 1, dt, q0, lam1).
 * w1 / w2 are not read when a1 / a2 is 0 (may be NULL); out may alias w1 or w2
 * but not q or y.  (Not in the paper: the discrete adjoint of the RK stepping.) */
dg_status dg_rk_stage_adjoint(const dg_mesh* mesh, const dg_phys* phys, double a1, const double* w1, double a2,
                              const double* w2, double b, double dt, const double* q, const double* y, double* out,
                              void* stream);

/* Passive tracer (section 2.1: C = rho c, dC/dt + div(C u) = 0, u = U/rho;
 * section 4.2 compares its loss under mortars and pointwise matching).  c and
 * the outputs are DEVICE float64 [K][Np] (leaf-major like one variable plane of
 * q); q / qs is the Euler state [5][K][Np] that supplies u and the Rusanov wave
 * speed (the same local maximum |u.n| + c as the Euler flux; the tracer jump is
 * C- - C+).  Walls carry no tracer flux; hanging faces use phys->nonconforming
 * (mortars: the tracer's integral is conserved to round-off; pointwise: not),
 * through a pre-pass into the mesh's tracer workspace (tracer calls on one mesh
 * must be ordered among themselves; the workspace is not the one of the Euler
 * calls, and both only read the mesh's tables, so tracer calls may run on another
 * stream beside Euler calls on the same mesh once a call has made its device
 * tables and its background for phys, and has completed or is waited for).
 * dg_tracer_rhs: rhs := R_C(q, c).  dg_tracer_stage:
 * cout := a c0 + b (cs + dt R_C(qs, cs)), the tracer part of the Shu-Osher
 * stage whose Euler part is dg_rk_stage(a, b, dt, q0, qs, ...) (call it before
 * that stage overwrites qs, or with a distinct output); cout may alias c0 but
 * not cs or qs; c0 is not read when a == 0.  Enqueued on stream.  DG_EINVAL on
 * NULL or aliased fields, bad phys or a z-periodic mesh with a z-dependent
 * background. */
dg_status dg_tracer_rhs(const dg_mesh* mesh, const dg_phys* phys, const double* q, const double* c, double* rhs,
                        void* stream);
dg_status dg_tracer_stage(const dg_mesh* mesh, const dg_phys* phys, double a, double b, double dt, const double* qs,
                          const double* c0, const double* cs, double* cout, void* stream);
/* Integral of a tracer field c (device [K][Np]) with the weights of dg_budgets,
 * compensated and deterministic, into out_host[0] (host).  Synchronises the
 * stream; DG_ENONFINITE if not finite. */
dg_status dg_tracer_mass(const dg_mesh* mesh, const double* c, double* out_host, void* stream);

/* Mass and energy budgets (section 2.1: mass is conserved discretely, energy
 * is not; section 4.3 reports both losses; the energy density is not in the
 * paper), over the mesh with weights J_e W_n = (hx hy hz / 8) w_i w_j w_k:
 * out_host[0] = sum rho', [1] = sum (rhobar + rho'), [2] = sum Theta',
 * [3] = sum P/(gamma-1) + |U|^2/(2 rho) + rho g z.  Compensated float64
 * summation in a fixed order (deterministic).  q is device [5][K][Np];
 * out_host is host double[4].  Synchronises the stream; DG_ENONFINITE when a
 * budget is not finite, DG_EINVAL on a NULL argument. */
dg_status dg_budgets(const dg_mesh* mesh, const dg_phys* phys, const double* q, double* out_host,
                     void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the budgets of dg_budgets,
 * written to out_dev (DEVICE double[4], caller-owned) on `stream`, with no
 * allocation, no copy and no synchronisation.  The per-block partial sums go to
 * one file-scope device array per GPU (8 * 1024 doubles = 64 KiB, held until the
 * process ends), whose address is looked up once per device; every entry the
 * reduction reads is written first by the same call, so nothing is cleared.
 * Calls that overlap on one GPU (different streams, no ordering) share that
 * array and race; order them.  The mesh must already have its device tables
 * (made by any earlier field call on it: making them allocates) and its device
 * must be current, else DG_EINVAL; no size of mesh exceeds the array (the
 * reduction uses at most 1024 blocks), the check stays as a guard.  Non-finite
 * budgets are not reported as DG_ENONFINITE (nothing is read back): the caller
 * inspects out_dev. */
dg_status dg_budgets_noalloc(const dg_mesh* mesh, const dg_phys* phys, const double* q, double* out_dev,
                             void* stream);

/* Adaptation indicator (section 3.2: regrid from a criterion every T steps;
 * section 4.3: the potential temperature as the criterion; the two measures and
 * the flag rule are not in the paper): eta_e = max over the leaf's nodes of
 * |theta'| (DG_IND_THETA) or |grad theta| (DG_IND_GRAD_THETA), into eta (device
 * double[K], may be NULL), and flags (host int8[K]): +1 where eta > thr and
 * level < max_level, -1 where eta <= thr and level > 0, else 0.  Synchronises
 * the stream.  DG_EINVAL on a NULL q or flags_host or an unknown kind. */
dg_status dg_indicator(const dg_mesh* mesh, const dg_phys* phys, const double* q, int32_t kind,
                       double thr, double* eta, int8_t* flags_host, void* stream);

/* The same indicator, only enqueued: the flags go to flags_dev (DEVICE int8[K],
 * caller-owned, not aliasing q or eta) and nothing synchronises, for a caller
 * that overlaps the regrid decision (section 3.2: the host-side forest passes)
 * with further GPU work on the stream (copy flags_dev to pinned host memory
 * asynchronously and wait on an event before the passes).  Same errors as
 * dg_indicator; a fault in the kernel surfaces at the next synchronising call. */
dg_status dg_indicator_async(const dg_mesh* mesh, const dg_phys* phys, const double* q, int32_t kind,
                             double thr, double* eta, int8_t* flags_dev, void* stream);

/* Flags of the refine pass of an adaptation cycle whose coarsen pass built
 * `coarsened` from the mesh the flags belong to (section 3.2: one regrid applies
 * the indicator's coarsen and refine decisions): flags_out (host int8[K] of
 * `coarsened`) is +1 where the leaf was kept by the coarsen pass and its flag was
 * +1, else 0 (a parent the coarsen pass made is not refined in the same cycle; -1
 * has no meaning in a refine pass).  flags is host int8[K] of the mesh the
 * coarsen pass started from; a pass that changed no leaf has the identity
 * transfer plan, so the flags carry over unchanged.  Host only.  DG_EINVAL on a
 * NULL argument or a transfer plan out of range. */
dg_status dg_flags_after_coarsen(const dg_mesh* coarsened, const int8_t* flags, int8_t* flags_out);

/* Buffer zone around refinement (section 3.2: a margin of B coarse cells between a
 * feature and the coarse-fine interface, the same B in the tree-based code).
 * Reading: B rounds of face-neighbour dilation of the +1 flags, in place on the
 * host array flags (int8[K], as from dg_indicator): in each round every leaf
 * that shares a face with a leaf flagged +1 (conforming, or either side of a
 * hanging face) becomes +1, whatever its flag was; other flags are kept.  Host
 * only (the mesh's host tables); B >= 0. */
dg_status dg_flags_buffer(const dg_mesh* mesh, int8_t* flags, int32_t B);

/* Message of the last failed call on this thread ("" if none). */
const char* dg_last_error(void);

/* ---- Benchmark calibration export, not part of the method (not in the paper).
 * One launch of `blocks` workgroups of 256 threads, every thread running `iters`
 * rounds of 8 independent float64 fused multiply-adds, so that a benchmark timing
 * it on `stream` can compare the chip's achievable float64 vector rate with its
 * published peak.  sink is a device double[256*blocks] (one value per thread,
 * keeps the work live); *flops_out (host) receives 2*8*iters*256*blocks.
 * blocks, iters > 0, else DG_EINVAL. */
dg_status dg_fma_burst(int32_t blocks, int32_t iters, double* sink, double* flops_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DGAMR_DG_H */

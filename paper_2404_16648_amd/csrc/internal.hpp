// Internal declarations of the DG-AMR library (host side).  Not part of the ABI.
#pragma once

#include <atomic>
#include <cstdint>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "dg.h"
#include "facetypes.hpp"

namespace dgamr {

constexpr int kMaxN = 7;
constexpr int kMinN = 2;
constexpr int kMaxLevel = 12;

struct Leaf {
    int32_t r, l, a[3];
};

// 1-D reference operators for order N, float64 (row-major [N+1][N+1])
struct RefOps {
    int N = 0;
    std::vector<double> x, w, D, I0, I1, R0, R1;
    std::vector<double> P0, P1;  // pointwise matching: half a's polynomial at the parent's nodes
};
RefOps make_refops(int N);

// an allocator under which a vector's new elements of a trivial type are left
// uninitialised (resize without a value): the large tables of a pass are first
// touched by the parallel loops that fill them, not by a serial zero fill
template <class T>
struct NoInit : std::allocator<T> {
    using std::allocator<T>::allocator;
    template <class U>
    struct rebind {
        using other = NoInit<U>;
    };
    template <class U>
    void construct(U* p) noexcept {
        ::new ((void*)p) U;
    }
    template <class U, class... A>
    void construct(U* p, A&&... a) {
        ::new ((void*)p) U(std::forward<A>(a)...);
    }
};
using ivec = std::vector<int32_t, NoInit<int32_t>>;

struct HostMesh {
    dg_forest_desc desc{};
    std::vector<Leaf> leaves;
    ivec conf, bnd, hang;                        // flattened tables (3, 2, 6 per row)
    ivec xfer_src, xfer_kind;
    ivec ftype, fnb;                             // [K][6], [K][6][4]
    int64_t n_refined = 0, n_coarsened = 0;
    bool same_as_prev = false;                   // the pass changed no leaf: tables copied
    // cubed-sphere shell (leaf r = panel, a = (ia, ib, ir)): per face the neighbour
    // leaf (-1: wall), its face and the flip of the face-local first axis
    bool sphere = false;
    dg_sphere_desc sdesc{};
    std::vector<int32_t> snb;                    // [K][6][3]
    std::vector<int8_t> skind, saux;             // [K][6]: SK_* kind; quadrant on a fine side
};

// forest passes (host, integer work); return "" or an error message
std::string forest_uniform(const dg_forest_desc& desc, HostMesh& out);
std::string forest_refine(const HostMesh& prev, const int8_t* flags, HostMesh& out);
std::string forest_coarsen(const HostMesh& prev, const int8_t* flags, HostMesh& out);
void forest_tables(HostMesh& m);
// whether forest_refine (refine) or forest_coarsen (!refine) would change a leaf
bool pass_changes(const HostMesh& prev, const int8_t* flags, bool refine);
// host checks of a new mesh (in parallel): every face has a type and in-range
// neighbours; the transfer plan indexes fields of K_from source leaves (a kept or
// refined source in range, a refined leaf's eight children consecutive with ids
// 0..7 and one source, a merged parent's eight sources in range)
bool tables_consistent(const HostMesh& h);
bool plan_consistent(const HostMesh& h, int64_t K_from);
// per-leaf device arrays of a brick mesh, in parallel: geo [K][4] (2/h per axis,
// volume / 8), c1d [3][K][N+1] node coordinates per axis, level [K]
void box_leaf_arrays(const HostMesh& h, const std::vector<double>& xi, double* geo, double* c1d, int32_t* level);
// the stage kernel's per-leaf face records (rec_len int32 each), in parallel: per
// face the type, the first neighbour and the hanging-face row (hs [K][6]); on a
// shell, entry 18 packs per face the neighbour's face and the flip, entry 19 the panel
void stage_records(const HostMesh& h, const int32_t* hs, int rec_len, int32_t* srec);

// cubed-sphere shell: mesh and tables; geometry into device layouts
// (metric [10][K][Np]: J, then J a^i_c at 1 + 3 i + c; fgeo [K][6][NF][4]: unit
// normal and face Jacobian; c1d [3][K][N+1]: tan of the two panel angles, height)
std::string sphere_build(const dg_sphere_desc& d, HostMesh& out);
void sphere_geometry(const HostMesh& h, const RefOps& ops, double* metric, double* fgeo, double* c1d);
// shell face kinds (skind): wall, conforming, fine side or coarse side of a hanging face
constexpr int8_t SK_WALL = 0, SK_CONF = 1, SK_FINE = 2, SK_COARSE = 3;
// refine and coarsen passes of a shell with max_level > 0 (2:1 across faces, the
// transfer plan as for the brick forest); whether a pass would change a leaf
std::string sphere_refine(const HostMesh& prev, const int8_t* flags, HostMesh& out);
std::string sphere_coarsen(const HostMesh& prev, const int8_t* flags, HostMesh& out);
bool sphere_pass_changes(const HostMesh& prev, const int8_t* flags, bool refine);
void sphere_forest_tables(HostMesh& out);
// spherical-excess volume of every element [K]; of any cell (panel, level, g)
void sphere_volumes(const HostMesh& h, long double* vol);
long double sphere_cell_volume(const dg_sphere_desc& d, const Leaf& c);
// index of element (panel p, column ia, row ib, layer ir)
int64_t sphere_leaf(const dg_sphere_desc& d, int p, int ia, int ib, int ir);

// geometry of leaf e: h[3] and 1-D node coordinates c[3][N+1]
void leaf_geometry(const dg_forest_desc& desc, const Leaf& lf, const std::vector<double>& xi,
                   double h[3], double* c /* [3][N+1] */);

}  // namespace dgamr

struct dg_mesh {
    dgamr::HostMesh h;
    dgamr::RefOps ops;
    const dg_mesh* prev = nullptr;
    uint64_t id = 0, prev_id = 0;
    std::atomic<bool> on_device{false};  // device tables made (at first GPU use)
    int device = 0;
    // the asynchronous upload of the device tables: until its event has completed,
    // a call on another stream than upload_stream waits for it
    void* upload_done = nullptr;    // hipEvent_t
    void* upload_stream = nullptr;  // hipStream_t
    char* d_base = nullptr;       // the one device allocation holding everything below
    // device tables
    double* d_ops = nullptr;      // D, I0, I1, R0, R1 ([N1][N1] each), w [N1]
    double* d_geo = nullptr;      // [K][4]: 2/hx, 2/hy, 2/hz, hx*hy*hz/8
    double* d_c1d = nullptr;      // [3][K][N1] node coordinates per axis
    int32_t* d_ftype = nullptr;   // [K][6]
    int32_t* d_fnb = nullptr;     // [K][6][4]
    int32_t* d_level = nullptr;   // [K]
    int32_t* d_xsrc = nullptr;    // [K]
    int32_t* d_xkind = nullptr;   // [K]
    int32_t* d_hslot = nullptr;   // [K][6]: row of the hanging-face table, or -1
    int32_t* d_hang = nullptr;    // [n_hang][6]: coarse leaf, its face, 4 fine leaves
    int32_t* d_srec = nullptr;    // [K][kStageRec]: face tables of the stage kernel
    double* d_mort = nullptr;     // [n_hang][5][5][NF]: mortar pre-pass output (workspace)
    double* d_mortC = nullptr;    // [n_hang][5][NF]: tracer mortar pre-pass output (workspace)
    int64_t n_hang = 0;
    // background profile [3][K][N1] for bg_phys (computed on first use)
    double* d_bg = nullptr;
    dg_phys bg_phys{};
    bool bg_valid = false;
    // workspaces
    double* d_red = nullptr;      // reduction partials
    int64_t red_len = 0;
    int8_t* d_flags = nullptr;    // [K]
    double* d_eta = nullptr;      // [K]
    double* d_sigma = nullptr;    // [3][5][K][Np]: viscous gradient (own allocation, at first use)
    double* d_metric = nullptr;   // sphere: [10][K][Np] J and metric terms
    double* d_fgeo = nullptr;     // sphere: [K][6][NF][4] face normal and face Jacobian
    int32_t* d_xlist = nullptr;   // sphere: the children of this mesh's plan, then their parents in prev
    int64_t n_xch = 0, n_xpar = 0;
};

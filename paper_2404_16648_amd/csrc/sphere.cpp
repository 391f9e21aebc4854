// Cubed-sphere shell (section 3.4 spherical geometry, section 4.4 global tests):
// the mesh of six equiangular panels of n x n elements and nz radial layers, its
// face connectivity across panel edges (with the orientation of the neighbour's
// face), and the isoparametric geometry: node positions, metric terms in the
// conservative curl form, Jacobian, and the normal and face Jacobian of every
// face node (shared faces take the values of the (leaf, face) pair that comes
// first, the other side the same with the normal reversed).  Host code.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <stdexcept>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace dgamr {
namespace {

using Pt = std::array<int64_t, 3>;

// cube point of panel coordinates (X, Y) with the fixed coordinate c (1 for real
// coordinates, n for the integer lattice of grid lines); every panel frame
// (d/dX, d/dY, outward normal) is right-handed
template <typename T>
std::array<T, 3> panel_point(int p, T X, T Y, T c) {
    switch (p) {
        case 0: return {c, X, Y};
        case 1: return {-X, c, Y};
        case 2: return {-c, -X, Y};
        case 3: return {X, -c, Y};
        case 4: return {-Y, X, c};
        default: return {Y, X, -c};
    }
}

using ld = long double;

// tan of the equiangular angle s pi / (4 n), exactly +-1 on the panel edges
ld tan_grid(ld s, int n) {
    if (s == (ld)n) return 1.0L;
    if (s == -(ld)n) return -1.0L;
    const ld pi = 3.141592653589793238462643383279502884L;
    return std::tan(s * pi / (4.0L * n));
}

}  // namespace

int64_t sphere_leaf(const dg_sphere_desc& d, int p, int ia, int ib, int ir) {
    return (((int64_t)p * d.nz + ir) * d.n + ib) * d.n + ia;
}

std::string sphere_build(const dg_sphere_desc& d, HostMesh& out) {
    if (d.N < kMinN || d.N > kMaxN) return "N out of range";
    if (d.n < 1 || d.nz < 1) return "need n, nz >= 1";
    if (!(d.r_e > 0.0) || !(d.H > 0.0)) return "need r_e, H > 0";
    if (d.max_level < 0 || d.max_level > 10) return "max_level out of range 0..10";
    if (((int64_t)d.n << d.max_level) >= (1LL << 20) || ((int64_t)d.nz << d.max_level) >= (1LL << 14))
        return "n or nz too large for max_level";
    const int n = d.n, nz = d.nz;
    const int64_t K = 6LL * n * n * nz;
    if (K > (1LL << 26)) return "too many elements";
    out = HostMesh{};
    out.sphere = true;
    out.sdesc = d;
    out.desc.N = d.N;
    out.desc.nx = n;
    out.desc.ny = n;
    out.desc.nz = nz;
    out.desc.max_level = d.max_level;
    out.leaves.resize(K);
    for (int p = 0; p < 6; ++p)
        for (int ir = 0; ir < nz; ++ir)
            for (int ib = 0; ib < n; ++ib)
                for (int ia = 0; ia < n; ++ia) out.leaves[sphere_leaf(d, p, ia, ib, ir)] = Leaf{p, 0, {ia, ib, ir}};
    out.snb.assign(K * 18, 0);
    for (int64_t i = 0; i < K * 6; ++i) out.snb[i * 3] = out.snb[i * 3 + 1] = -1;
    // lateral faces: matched by their two horizontal end points on the integer
    // lattice of grid lines and their layer; the end point at the face's a = 0 end
    // decides the orientation
    struct End {
        int64_t e;
        int f;
        Pt p0;
    };
    std::map<std::tuple<Pt, Pt, int>, std::vector<End>> faces;
    for (int64_t e = 0; e < K; ++e) {
        const Leaf& L = out.leaves[e];
        const int p = L.r, ia = L.a[0], ib = L.a[1], ir = L.a[2];
        const int64_t x0 = 2 * ia - n, x1 = 2 * ia + 2 - n, y0 = 2 * ib - n, y1 = 2 * ib + 2 - n;
        const int64_t ends[4][4] = {{x0, y0, x0, y1}, {x1, y0, x1, y1}, {x0, y0, x1, y0}, {x0, y1, x1, y1}};
        for (int f = 0; f < 4; ++f) {
            const Pt P0 = panel_point<int64_t>(p, ends[f][0], ends[f][1], n);
            const Pt P1 = panel_point<int64_t>(p, ends[f][2], ends[f][3], n);
            const auto key = P0 < P1 ? std::make_tuple(P0, P1, ir) : std::make_tuple(P1, P0, ir);
            faces[key].push_back(End{e, f, P0});
        }
        int32_t* nb = &out.snb[e * 18];
        if (ir > 0) {
            nb[4 * 3] = (int32_t)sphere_leaf(d, p, ia, ib, ir - 1);
            nb[4 * 3 + 1] = 5;
        }
        if (ir < nz - 1) {
            nb[5 * 3] = (int32_t)sphere_leaf(d, p, ia, ib, ir + 1);
            nb[5 * 3 + 1] = 4;
        }
    }
    for (const auto& kv : faces) {
        if (kv.second.size() != 2) return "internal: unmatched lateral face";
        const End& A = kv.second[0];
        const End& B = kv.second[1];
        const int flip = A.p0 == B.p0 ? 0 : 1;
        int32_t* na = &out.snb[(A.e * 6 + A.f) * 3];
        int32_t* nbb = &out.snb[(B.e * 6 + B.f) * 3];
        na[0] = (int32_t)B.e;
        na[1] = B.f;
        na[2] = flip;
        nbb[0] = (int32_t)A.e;
        nbb[1] = A.f;
        nbb[2] = flip;
    }
    // element-centric tables shared with the box meshes: types, first neighbour,
    // wall list, the identity transfer plan
    out.ftype.assign(K * 6, FT_WALL);
    out.fnb.assign(K * 24, -1);
    for (int64_t e = 0; e < K; ++e)
        for (int f = 0; f < 6; ++f) {
            const int32_t* nb = &out.snb[(e * 6 + f) * 3];
            if (nb[0] >= 0) {
                out.ftype[e * 6 + f] = FT_CONF;
                out.fnb[(e * 6 + f) * 4] = nb[0];
            } else {
                out.bnd.push_back((int32_t)e);
                out.bnd.push_back(f);
            }
        }
    out.skind.assign(K * 6, SK_WALL);
    out.saux.assign(K * 6, 0);
    for (int64_t i = 0; i < K * 6; ++i)
        if (out.snb[i * 3] >= 0) out.skind[i] = SK_CONF;
    // a shell that may be refined takes its tables from the forest (at level 0 they
    // are the same as above, found another way)
    if (d.max_level > 0) sphere_forest_tables(out);
    out.xfer_src.resize(K);
    out.xfer_kind.assign(K, DG_KIND_COPY);
    for (int64_t e = 0; e < K; ++e) out.xfer_src[e] = (int32_t)e;
    return "";
}

// The geometry of a thin shell is ill-conditioned in float64: the curl-form
// metric terms cancel in proportion to the element aspect ratio (horizontal over
// radial size, several hundred here), so it is evaluated in long double and
// rounded once.
void sphere_geometry(const HostMesh& h, const RefOps& ops, double* metric, double* fgeo, double* c1d) {
    const dg_sphere_desc& d = h.sdesc;
    const int N = d.N, N1 = N + 1, NP = N1 * N1 * N1, NF = N1 * N1, n = d.n;
    const int64_t K = (int64_t)h.leaves.size();
    const std::vector<double>& D = ops.D;
    // own face normals and face Jacobians, [K][6][NF]
    std::vector<ld> own_n((size_t)K * 6 * NF * 3), own_s((size_t)K * 6 * NF);
    std::vector<ld> X(NP * 3), dX(NP * 9), V(NP * 3), Ja(NP * 9), J(NP);
    // d f / d xi_axis at node (f nodal), applied to f minus its value at the line's
    // first node: D annihilates constants, and the shift keeps an offset far larger
    // than the variation along the line (the earth radius in a position) out of the sums
    auto deriv = [&](const ld* f, int axis, int node) {
        const int i = node % N1, j = (node / N1) % N1, k = node / NF;
        const int id = axis == 0 ? i : axis == 1 ? j : k;
        const int stride = axis == 0 ? 1 : axis == 1 ? N1 : NF;
        const int base = node - id * stride;
        ld acc = 0.0L;
        for (int m = 0; m < N1; ++m) acc += (ld)D[id * N1 + m] * (f[base + m * stride] - f[base]);
        return acc;
    };
    for (int64_t e = 0; e < K; ++e) {
        const Leaf& L = h.leaves[e];
        const int p = L.r, ia = L.a[0], ib = L.a[1], ir = L.a[2];
        const int m = n << L.l, mz = d.nz << L.l;  // cells per panel edge and layers at the leaf's level
        ld Xt[8], Yt[8], ht[8];
        for (int a = 0; a < N1; ++a) {
            Xt[a] = tan_grid((ld)(2 * ia - m) + ((ld)ops.x[a] + 1.0L), m);
            Yt[a] = tan_grid((ld)(2 * ib - m) + ((ld)ops.x[a] + 1.0L), m);
            ht[a] = (ld)d.H * ((ld)ir + 0.5L * ((ld)ops.x[a] + 1.0L)) / mz;
            c1d[(0 * K + e) * N1 + a] = (double)Xt[a];
            c1d[(1 * K + e) * N1 + a] = (double)Yt[a];
            c1d[(2 * K + e) * N1 + a] = (double)ht[a];
        }
        for (int node = 0; node < NP; ++node) {
            const int i = node % N1, j = (node / N1) % N1, k = node / NF;
            const auto c = panel_point<ld>(p, Xt[i], Yt[j], 1.0L);
            const ld nrm = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            const ld r = (ld)d.r_e + ht[k];
            for (int q = 0; q < 3; ++q) X[q * NP + node] = r * (c[q] / nrm);
        }
        for (int node = 0; node < NP; ++node)
            for (int q = 0; q < 3; ++q)
                for (int a = 0; a < 3; ++a) dX[(q * 3 + a) * NP + node] = deriv(&X[q * NP], a, node);
        for (int node = 0; node < NP; ++node) {
            const ld* g = &dX[node];
            auto G = [&](int q, int a) { return g[(q * 3 + a) * NP]; };
            J[node] = G(0, 0) * (G(1, 1) * G(2, 2) - G(1, 2) * G(2, 1)) - G(0, 1) * (G(1, 0) * G(2, 2) - G(1, 2) * G(2, 0)) +
                      G(0, 2) * (G(1, 0) * G(2, 1) - G(1, 1) * G(2, 0));
        }
        // curl form: Ja[i][c] = -(curl_xi V)_i, V_a = X_l d_a X_m, (c, m, l) cyclic, X_l
        // relative to the element's first node (the discrete curl of a constant times
        // grad X_m vanishes; the shift only removes cancellation)
        for (int c = 0; c < 3; ++c) {
            const int m = (c + 1) % 3, l = (c + 2) % 3;
            const ld X0 = X[l * NP];
            for (int node = 0; node < NP; ++node)
                for (int a = 0; a < 3; ++a) V[a * NP + node] = (X[l * NP + node] - X0) * dX[(m * 3 + a) * NP + node];
            for (int node = 0; node < NP; ++node) {
                const ld c0 = deriv(&V[2 * NP], 1, node) - deriv(&V[1 * NP], 2, node);
                const ld c1 = deriv(&V[0 * NP], 2, node) - deriv(&V[2 * NP], 0, node);
                const ld c2 = deriv(&V[1 * NP], 0, node) - deriv(&V[0 * NP], 1, node);
                Ja[(0 * 3 + c) * NP + node] = -c0;
                Ja[(1 * 3 + c) * NP + node] = -c1;
                Ja[(2 * 3 + c) * NP + node] = -c2;
            }
        }
        // device layout [10][K][NP]: J, then Ja[i][c] at 1 + 3 i + c
        for (int node = 0; node < NP; ++node) {
            metric[(0 * K + e) * NP + node] = (double)J[node];
            for (int q = 0; q < 9; ++q) metric[((1 + q) * K + e) * NP + node] = (double)Ja[q * NP + node];
        }
        for (int f = 0; f < 6; ++f) {
            const int dd = f >> 1;
            const double sgn = (f & 1) ? 1.0 : -1.0;
            for (int mm = 0; mm < NF; ++mm) {
                const int a = mm % N1, b = mm / N1, idx = (f & 1) ? N : 0;
                const int node = dd == 0 ? idx + N1 * (a + N1 * b) : dd == 1 ? a + N1 * (idx + N1 * b) : a + N1 * (b + N1 * idx);
                ld v[3];
                for (int c = 0; c < 3; ++c) v[c] = (ld)sgn * Ja[(dd * 3 + c) * NP + node];
                const ld s = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                for (int c = 0; c < 3; ++c) own_n[((e * 6 + f) * NF + mm) * 3 + c] = v[c] / s;
                own_s[(e * 6 + f) * NF + mm] = s;
            }
        }
    }
    for (int64_t e = 0; e < K; ++e)
        for (int f = 0; f < 6; ++f) {
            const int32_t* nb = &h.snb[(e * 6 + f) * 3];
            const int64_t e2 = nb[0];
            const int f2 = nb[1], flip = nb[2];
            const bool own = h.skind[e * 6 + f] != SK_CONF || e < e2 || (e == e2 && f < f2);
            for (int mm = 0; mm < NF; ++mm) {
                double* out = fgeo + ((e * 6 + f) * NF + mm) * 4;
                if (own) {
                    for (int c = 0; c < 3; ++c) out[c] = (double)own_n[((e * 6 + f) * NF + mm) * 3 + c];
                    out[3] = (double)own_s[(e * 6 + f) * NF + mm];
                } else {
                    const int a = mm % N1, b = mm / N1;
                    const int m2 = (flip ? N - a : a) + N1 * b;
                    for (int c = 0; c < 3; ++c) out[c] = -(double)own_n[((e2 * 6 + f2) * NF + m2) * 3 + c];
                    out[3] = (double)own_s[(e2 * 6 + f2) * NF + m2];
                }
            }
        }
}

namespace {

using V3 = std::array<ld, 3>;

V3 unit_corner(int p, int sx, int sy, int n) {
    const auto c = panel_point<ld>(p, tan_grid((ld)sx, n), tan_grid((ld)sy, n), 1.0L);
    const ld r = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    return {c[0] / r, c[1] / r, c[2] / r};
}

ld dot3(const V3& a, const V3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// spherical excess (area on the unit sphere) of the triangle abc with great-circle
// edges, by the formula of Van Oosterom and Strackee (1983):
// tan(E/2) = |a . (b x c)| / (1 + a.b + b.c + c.a)
ld tri_excess(const V3& a, const V3& b, const V3& c) {
    const V3 bxc{b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
    const ld num = std::fabs(dot3(a, bxc));
    const ld den = 1.0L + dot3(a, b) + dot3(b, c) + dot3(c, a);
    return 2.0L * std::atan2(num, den);
}

}  // namespace

// Element volumes from the areas of their footprints (section 3.4: spherical
// excess of the curved elements, whose edges are great-circle arcs on an
// equiangular panel): area on the unit sphere (two triangles) times the radial
// integral of r^2, (r1^3 - r0^3)/3 written as (r1 - r0)(r1^2 + r1 r0 + r0^2)/3.
// Long double throughout.
long double sphere_cell_volume(const dg_sphere_desc& d, const Leaf& c) {
    const int p = c.r, ia = c.a[0], ib = c.a[1], ir = c.a[2];
    const int n = d.n << c.l, mz = d.nz << c.l;
    const int x0 = 2 * ia - n, x1 = x0 + 2, y0 = 2 * ib - n, y1 = y0 + 2;
    const V3 c00 = unit_corner(p, x0, y0, n), c10 = unit_corner(p, x1, y0, n);
    const V3 c11 = unit_corner(p, x1, y1, n), c01 = unit_corner(p, x0, y1, n);
    const ld area = tri_excess(c00, c10, c11) + tri_excess(c00, c11, c01);
    const ld r0 = (ld)d.r_e + (ld)d.H * (ld)ir / (ld)mz;
    const ld r1 = (ld)d.r_e + (ld)d.H * (ld)(ir + 1) / (ld)mz;
    return area * (r1 - r0) * (r1 * r1 + r1 * r0 + r0 * r0) / 3.0L;
}

void sphere_volumes(const HostMesh& h, long double* vol) {
    const int64_t K = (int64_t)h.leaves.size();
    for (int64_t e = 0; e < K; ++e) vol[e] = sphere_cell_volume(h.sdesc, h.leaves[e]);
}

// ---------------------------------------------------------------- refinement on the shell
// A leaf is Leaf{p, l, {gx, gy, gz}}: panel, level, and its column, row and layer among
// the (n 2^l) x (n 2^l) x (nz 2^l) cells of its panel at that level.  Order: panel,
// root element (layer, row, column of the unrefined shell), then the Morton key of
// the position inside the root at max_level (x least significant), so the unrefined
// shell keeps its order and the eight children of a leaf are consecutive.
namespace {

struct CellKeyHash {
    size_t operator()(uint64_t k) const { return (size_t)(k * 0x9E3779B97F4A7C15ull); }
};

// gx, gy < 2^21, gz < 2^15 (checked when the shell is built)
uint64_t pack(int p, int l, int64_t gx, int64_t gy, int64_t gz) {
    return (uint64_t)p | ((uint64_t)l << 3) | ((uint64_t)gx << 7) | ((uint64_t)gy << 28) | ((uint64_t)gz << 49);
}
uint64_t pack(const Leaf& c) { return pack(c.r, c.l, c.a[0], c.a[1], c.a[2]); }

struct OrderKey {
    int p;
    int64_t rz, ry, rx;
    uint64_t morton;
    bool operator<(const OrderKey& o) const {
        return std::tie(p, rz, ry, rx, morton) < std::tie(o.p, o.rz, o.ry, o.rx, o.morton);
    }
};

OrderKey order_key(const Leaf& c, int L) {
    const int l = c.l;
    uint64_t lo[3];
    for (int d = 0; d < 3; ++d) lo[d] = ((uint64_t)c.a[d] & ((1ull << l) - 1)) << (L - l);
    uint64_t key = 0;
    for (int b = 0; b < L; ++b)
        for (int d = 0; d < 3; ++d) key |= ((lo[d] >> b) & 1ull) << (3 * b + d);
    return {c.r, (int64_t)c.a[2] >> l, (int64_t)c.a[1] >> l, (int64_t)c.a[0] >> l, key};
}

// (X, Y) of the lattice point P (cube coordinates in units of half a cell at
// resolution m) on panel p, false if P is not on that panel: the inverse of
// panel_point(p, X, Y, m)
bool panel_coords(int p, const Pt& P, int64_t m, int64_t& X, int64_t& Y) {
    switch (p) {
        case 0: if (P[0] != m) return false; X = P[1]; Y = P[2]; return true;
        case 1: if (P[1] != m) return false; X = -P[0]; Y = P[2]; return true;
        case 2: if (P[0] != -m) return false; X = -P[1]; Y = P[2]; return true;
        case 3: if (P[1] != -m) return false; X = P[0]; Y = P[2]; return true;
        case 4: if (P[2] != m) return false; X = P[1]; Y = -P[0]; return true;
        default: if (P[2] != -m) return false; X = P[1]; Y = P[0]; return true;
    }
}

struct Across {
    Leaf c;
    int f2, flip;
};

// same-level neighbour of cell c across face f; false at the bottom and top walls
bool cell_across(const dg_sphere_desc& d, const Leaf& c, int f, Across& out) {
    const int l = c.l;
    const int64_t m = (int64_t)d.n << l, mz = (int64_t)d.nz << l;
    out.c = c;
    out.flip = 0;
    if (f >= 4) {
        const int64_t z2 = c.a[2] + (f == 5 ? 1 : -1);
        if (z2 < 0 || z2 >= mz) return false;
        out.c.a[2] = (int32_t)z2;
        out.f2 = f ^ 1;
        return true;
    }
    const int64_t gx = c.a[0], gy = c.a[1];
    const int64_t sx = f == 0 ? -1 : f == 1 ? 1 : 0, sy = f == 2 ? -1 : f == 3 ? 1 : 0;
    if (gx + sx >= 0 && gx + sx < m && gy + sy >= 0 && gy + sy < m) {
        out.c.a[0] = (int32_t)(gx + sx);
        out.c.a[1] = (int32_t)(gy + sy);
        out.f2 = f ^ 1;
        return true;
    }
    // across a panel edge: the face's two end points on the lattice of grid lines,
    // located on the other panel that holds both
    const int64_t X0 = 2 * gx - m, Y0 = 2 * gy - m, X1 = X0 + 2, Y1 = Y0 + 2;
    const int64_t e[4][4] = {{X0, Y0, X0, Y1}, {X1, Y0, X1, Y1}, {X0, Y0, X1, Y0}, {X0, Y1, X1, Y1}};
    const Pt P0 = panel_point<int64_t>(c.r, e[f][0], e[f][1], m);
    const Pt P1 = panel_point<int64_t>(c.r, e[f][2], e[f][3], m);
    for (int p2 = 0; p2 < 6; ++p2) {
        int64_t a0, b0, a1, b1;
        if (p2 == c.r || !panel_coords(p2, P0, m, a0, b0) || !panel_coords(p2, P1, m, a1, b1)) continue;
        out.c.r = p2;
        if (a0 == a1) {  // an edge of constant X: faces 0 / 1, first axis Y
            out.f2 = a0 == -m ? 0 : 1;
            out.c.a[0] = (int32_t)(out.f2 == 0 ? 0 : m - 1);
            out.c.a[1] = (int32_t)((std::min(b0, b1) + m) / 2);
            out.flip = b0 < b1 ? 0 : 1;
        } else {         // constant Y: faces 2 / 3, first axis X
            out.f2 = b0 == -m ? 2 : 3;
            out.c.a[0] = (int32_t)((std::min(a0, a1) + m) / 2);
            out.c.a[1] = (int32_t)(out.f2 == 2 ? 0 : m - 1);
            out.flip = a0 < a1 ? 0 : 1;
        }
        return true;
    }
    throw std::runtime_error("internal: no panel across a panel edge");
}

Leaf child_of(const Leaf& c, int k) {
    return Leaf{c.r, c.l + 1, {2 * c.a[0] + (k & 1), 2 * c.a[1] + ((k >> 1) & 1), 2 * c.a[2] + (k >> 2)}};
}
Leaf parent_of(const Leaf& c) { return Leaf{c.r, c.l - 1, {c.a[0] >> 1, c.a[1] >> 1, c.a[2] >> 1}}; }
int child_id_of(const Leaf& c) { return (c.a[0] & 1) | ((c.a[1] & 1) << 1) | ((c.a[2] & 1) << 2); }

using LeafMap = std::unordered_map<uint64_t, int64_t, CellKeyHash>;

// the leaf equal to or containing cell c, or -1 (c is refined)
int64_t containing(const LeafMap& idx, const Leaf& c) {
    for (int lv = c.l; lv >= 0; --lv) {
        const int sh = c.l - lv;
        auto it = idx.find(pack(c.r, lv, c.a[0] >> sh, c.a[1] >> sh, c.a[2] >> sh));
        if (it != idx.end()) return it->second;
    }
    return -1;
}

// sorted leaves of a shell and its face tables: per leaf and face the kind (wall,
// conforming, fine or coarse side of a hanging face), snb = (neighbour, its face,
// flip) for conforming faces, (coarse leaf, its face, flip) on a fine side, (row,
// the fine leaves' face, flip) on a coarse side; the hanging rows (coarse leaf, its
// face, the fine leaves by quadrant qa + 2 qb in the coarse face's axes); and the
// element-centric tables the kernels share with the brick meshes
void shell_tables(HostMesh& out) {
    const dg_sphere_desc& d = out.sdesc;
    const int64_t K = (int64_t)out.leaves.size();
    LeafMap idx;
    idx.reserve((size_t)K * 2);
    for (int64_t e = 0; e < K; ++e) idx[pack(out.leaves[e])] = e;
    out.snb.assign(K * 18, 0);
    out.skind.assign(K * 6, SK_WALL);
    out.saux.assign(K * 6, 0);
    out.hang.clear();
    out.bnd.clear();
    out.ftype.assign(K * 6, FT_WALL);
    out.fnb.assign(K * 24, -1);
    for (int64_t e = 0; e < K; ++e) {
        const Leaf& lf = out.leaves[e];
        for (int f = 0; f < 6; ++f) {
            int32_t* nb = &out.snb[(e * 6 + f) * 3];
            nb[0] = nb[1] = -1;
            Across a;
            if (!cell_across(d, lf, f, a)) {
                out.bnd.push_back((int32_t)e);
                out.bnd.push_back(f);
                continue;
            }
            const int64_t x = containing(idx, a.c);
            const int d2 = a.f2 >> 1, s2 = a.f2 & 1;
            const int t1 = d2 == 0 ? 1 : 0, t2 = d2 == 2 ? 1 : 2;
            if (x >= 0 && out.leaves[x].l == lf.l) {
                out.skind[e * 6 + f] = SK_CONF;
                nb[0] = (int32_t)x;
                nb[1] = a.f2;
                nb[2] = a.flip;
                out.ftype[e * 6 + f] = FT_CONF;
                out.fnb[(e * 6 + f) * 4] = (int32_t)x;
            } else if (x >= 0) {
                // fine side: the quadrant of a.c on the coarse leaf's face a.f2
                const int quad = (a.c.a[t1] & 1) + 2 * (a.c.a[t2] & 1);
                out.skind[e * 6 + f] = SK_FINE;
                out.saux[e * 6 + f] = (int8_t)quad;
                nb[0] = (int32_t)x;
                nb[1] = a.f2;
                nb[2] = a.flip;
                out.ftype[e * 6 + f] = FT_FINE | (quad << 8);
                out.fnb[(e * 6 + f) * 4] = (int32_t)x;
            } else {
                // coarse side: the children of a.c on its face a.f2, by their place in
                // this face's axes (the first reversed when the faces' axes run opposite)
                int32_t fine[4] = {-1, -1, -1, -1};
                for (int k = 0; k < 8; ++k) {
                    const Leaf ch = child_of(a.c, k);
                    const int b[3] = {k & 1, (k >> 1) & 1, k >> 2};
                    if (b[d2] != s2) continue;
                    auto it = idx.find(pack(ch));
                    if (it == idx.end()) throw std::runtime_error("internal: unbalanced shell forest");
                    const int qa = a.flip ? 1 - b[t1] : b[t1];
                    fine[qa + 2 * b[t2]] = (int32_t)it->second;
                }
                const int64_t row = (int64_t)out.hang.size() / 6;
                out.skind[e * 6 + f] = SK_COARSE;
                nb[0] = (int32_t)row;
                nb[1] = a.f2;
                nb[2] = a.flip;
                out.hang.push_back((int32_t)e);
                out.hang.push_back(f);
                for (int q = 0; q < 4; ++q) out.hang.push_back(fine[q]);
                out.ftype[e * 6 + f] = FT_COARSE;
                for (int q = 0; q < 4; ++q) out.fnb[(e * 6 + f) * 4 + q] = fine[q];
            }
        }
    }
}

void sort_shell(HostMesh& out) {
    const int L = out.sdesc.max_level;
    std::vector<std::pair<OrderKey, Leaf>> v;
    v.reserve(out.leaves.size());
    for (const Leaf& c : out.leaves) v.push_back({order_key(c, L), c});
    std::sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    for (size_t i = 0; i < v.size(); ++i) out.leaves[i] = v[i].second;
}

// leaves of `leaves` with a face neighbour two or more levels finer
std::vector<Leaf> needs_ripple(const dg_sphere_desc& d, const std::vector<Leaf>& leaves, const LeafMap& idx) {
    std::vector<Leaf> out;
    std::unordered_map<uint64_t, char, CellKeyHash> seen;
    for (const Leaf& lf : leaves)
        for (int f = 0; f < 6; ++f) {
            Across a;
            if (!cell_across(d, lf, f, a)) continue;
            const int64_t x = containing(idx, a.c);
            if (x >= 0 && leaves[x].l <= lf.l - 2 && seen.emplace(pack(leaves[x]), 1).second) out.push_back(leaves[x]);
        }
    return out;
}

}  // namespace

std::string sphere_refine(const HostMesh& prev, const int8_t* flags, HostMesh& out) {
    const dg_sphere_desc& d = prev.sdesc;
    const int64_t Kp = (int64_t)prev.leaves.size();
    std::vector<Leaf> cur;
    cur.reserve((size_t)Kp * 2);
    for (int64_t e = 0; e < Kp; ++e) {
        const Leaf& lf = prev.leaves[e];
        if (flags[e] > 0 && lf.l < d.max_level)
            for (int k = 0; k < 8; ++k) cur.push_back(child_of(lf, k));
        else
            cur.push_back(lf);
    }
    // ripple refinement to a fixed point (2:1 across faces)
    for (;;) {
        LeafMap idx;
        idx.reserve(cur.size() * 2);
        for (size_t i = 0; i < cur.size(); ++i) idx[pack(cur[i])] = (int64_t)i;
        const std::vector<Leaf> todo = needs_ripple(d, cur, idx);
        if (todo.empty()) break;
        std::unordered_map<uint64_t, char, CellKeyHash> split;
        for (const Leaf& x : todo) split[pack(x)] = 1;
        std::vector<Leaf> nxt;
        nxt.reserve(cur.size() + 7 * todo.size());
        for (const Leaf& c : cur) {
            if (split.count(pack(c)))
                for (int k = 0; k < 8; ++k) nxt.push_back(child_of(c, k));
            else
                nxt.push_back(c);
        }
        cur.swap(nxt);
    }
    out = HostMesh{};
    out.sphere = true;
    out.sdesc = d;
    out.desc = prev.desc;
    out.leaves = cur;
    sort_shell(out);
    LeafMap old;
    old.reserve((size_t)Kp * 2);
    for (int64_t e = 0; e < Kp; ++e) old[pack(prev.leaves[e])] = e;
    const int64_t K = (int64_t)out.leaves.size();
    out.xfer_src.resize(K);
    out.xfer_kind.resize(K);
    for (int64_t e = 0; e < K; ++e) {
        const Leaf& lf = out.leaves[e];
        auto it = old.find(pack(lf));
        if (it != old.end()) {
            out.xfer_src[e] = (int32_t)it->second;
            out.xfer_kind[e] = DG_KIND_COPY;
            continue;
        }
        auto ip = old.find(pack(parent_of(lf)));
        if (ip == old.end()) return "a leaf would be refined twice in one pass (max_level allows it)";
        out.xfer_src[e] = (int32_t)ip->second;
        out.xfer_kind[e] = child_id_of(lf);
        ++out.n_refined;
    }
    out.n_refined /= 8;
    shell_tables(out);
    return "";
}

// the parent of a family all flagged -1 is vetoed when a leaf face-adjacent to it
// is two or more levels finer than it
static bool shell_family_vetoed(const dg_sphere_desc& d, const LeafMap& idx, const Leaf& par) {
    for (int f = 0; f < 6; ++f) {
        Across a;
        if (!cell_across(d, par, f, a)) continue;
        if (containing(idx, a.c) >= 0) continue;
        const int d2 = a.f2 >> 1, s2 = a.f2 & 1;
        for (int k = 0; k < 8; ++k) {
            if (((k >> d2) & 1) != s2) continue;
            if (!idx.count(pack(child_of(a.c, k)))) return true;
        }
    }
    return false;
}

std::string sphere_coarsen(const HostMesh& prev, const int8_t* flags, HostMesh& out) {
    const dg_sphere_desc& d = prev.sdesc;
    const int64_t Kp = (int64_t)prev.leaves.size();
    LeafMap idx;
    idx.reserve((size_t)Kp * 2);
    for (int64_t e = 0; e < Kp; ++e) idx[pack(prev.leaves[e])] = e;
    std::unordered_map<uint64_t, char, CellKeyHash> merged;
    std::vector<Leaf> parents;
    for (int64_t e = 0; e < Kp; ++e) {
        const Leaf& lf = prev.leaves[e];
        if (lf.l == 0 || flags[e] >= 0) continue;
        const Leaf par = parent_of(lf);
        if (merged.count(pack(par))) continue;
        bool all = true;
        for (int k = 0; k < 8 && all; ++k) {
            auto it = idx.find(pack(child_of(par, k)));
            all = it != idx.end() && flags[it->second] < 0;
        }
        if (all && !shell_family_vetoed(d, idx, par)) {
            merged[pack(par)] = 1;
            parents.push_back(par);
        }
    }
    out = HostMesh{};
    out.sphere = true;
    out.sdesc = d;
    out.desc = prev.desc;
    for (const Leaf& lf : prev.leaves)
        if (lf.l == 0 || !merged.count(pack(parent_of(lf)))) out.leaves.push_back(lf);
    for (const Leaf& par : parents) out.leaves.push_back(par);
    sort_shell(out);
    const int64_t K = (int64_t)out.leaves.size();
    out.xfer_src.resize(K);
    out.xfer_kind.resize(K);
    for (int64_t e = 0; e < K; ++e) {
        const Leaf& lf = out.leaves[e];
        auto it = idx.find(pack(lf));
        if (it != idx.end()) {
            out.xfer_src[e] = (int32_t)it->second;
            out.xfer_kind[e] = DG_KIND_COPY;
        } else {
            out.xfer_src[e] = (int32_t)idx.at(pack(child_of(lf, 0)));
            out.xfer_kind[e] = DG_KIND_FAMILY;
            ++out.n_coarsened;
        }
    }
    shell_tables(out);
    return "";
}

bool sphere_pass_changes(const HostMesh& prev, const int8_t* flags, bool refine) {
    const int64_t Kp = (int64_t)prev.leaves.size();
    if (refine) {
        for (int64_t e = 0; e < Kp; ++e)
            if (flags[e] > 0 && prev.leaves[e].l < prev.sdesc.max_level) return true;
        return false;
    }
    LeafMap idx;
    idx.reserve((size_t)Kp * 2);
    for (int64_t e = 0; e < Kp; ++e) idx[pack(prev.leaves[e])] = e;
    for (int64_t e = 0; e < Kp; ++e) {
        const Leaf& lf = prev.leaves[e];
        if (lf.l == 0 || flags[e] >= 0 || child_id_of(lf) != 0) continue;
        const Leaf par = parent_of(lf);
        bool all = true;
        for (int k = 0; k < 8 && all; ++k) {
            auto it = idx.find(pack(child_of(par, k)));
            all = it != idx.end() && flags[it->second] < 0;
        }
        if (all && !shell_family_vetoed(prev.sdesc, idx, par)) return true;
    }
    return false;
}

// the shell's tables from the forest (every mesh of a shell with max_level > 0)
void sphere_forest_tables(HostMesh& out) { shell_tables(out); }

}  // namespace dgamr

// Cubed-sphere shell (section 3.4 spherical geometry, section 4.4 global tests):
// the mesh of six equiangular panels of n x n elements and nz radial layers, its
// face connectivity across panel edges (with the orientation of the neighbour's
// face), and the isoparametric geometry: node positions, metric terms in the
// conservative curl form, Jacobian, and the normal and face Jacobian of every
// face node (shared faces take the values of the (leaf, face) pair that comes
// first, the other side the same with the normal reversed).  Host code.
#include <array>
#include <cmath>
#include <map>
#include <string>
#include <tuple>
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
    out.desc.max_level = 0;
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
        ld Xt[8], Yt[8], ht[8];
        for (int a = 0; a < N1; ++a) {
            Xt[a] = tan_grid((ld)(2 * ia - n) + ((ld)ops.x[a] + 1.0L), n);
            Yt[a] = tan_grid((ld)(2 * ib - n) + ((ld)ops.x[a] + 1.0L), n);
            ht[a] = (ld)d.H * ((ld)ir + 0.5L * ((ld)ops.x[a] + 1.0L)) / d.nz;
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
            const bool own = e2 < 0 || e < e2 || (e == e2 && f < f2);
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
void sphere_volumes(const HostMesh& h, long double* vol) {
    const dg_sphere_desc& d = h.sdesc;
    const int n = d.n;
    const int64_t K = (int64_t)h.leaves.size();
    for (int64_t e = 0; e < K; ++e) {
        const Leaf& L = h.leaves[e];
        const int p = L.r, ia = L.a[0], ib = L.a[1], ir = L.a[2];
        const int x0 = 2 * ia - n, x1 = x0 + 2, y0 = 2 * ib - n, y1 = y0 + 2;
        const V3 c00 = unit_corner(p, x0, y0, n), c10 = unit_corner(p, x1, y0, n);
        const V3 c11 = unit_corner(p, x1, y1, n), c01 = unit_corner(p, x0, y1, n);
        const ld area = tri_excess(c00, c10, c11) + tri_excess(c00, c11, c01);
        const ld r0 = (ld)d.r_e + (ld)d.H * (ld)ir / (ld)d.nz;
        const ld r1 = (ld)d.r_e + (ld)d.H * (ld)(ir + 1) / (ld)d.nz;
        vol[e] = area * (r1 - r0) * (r1 * r1 + r1 * r0 + r0 * r0) / 3.0L;
    }
}

}  // namespace dgamr

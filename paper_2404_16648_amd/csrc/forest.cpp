// Brick forest of oct-trees (section 3.1: every coarse cell is the root of a
// tree, only active leaves are kept, flagged cells are replaced by their
// children or their parent), with 2:1 face balance (section 4.3) and the face
// and transfer tables the kernels need.  Host-side integer work.
//
// Ordering and balance rules (the paper fixes none of them):
//   * leaves sorted by (root, Morton key of the anchor scaled to max_level),
//     x the least significant bit; child id c = a + 2b + 4c';
//   * refine pass: +1 flags below max_level, then refine every leaf with a face
//     neighbour two or more levels finer until nothing changes;
//   * coarsen pass: a family of 8 leaves all flagged -1 merges unless a leaf
//     face-adjacent to the parent is two or more levels finer (judged on the
//     mesh before the pass);
//   * face tables enumerated by leaf, then face f = 2d + s; conforming faces
//     from the minus leaf's plus face, hanging faces from the coarse side with
//     fine leaves by quadrant a + 2b over the tangential axes.
#include <algorithm>
#include <cstring>
#include <unordered_map>
#include <unordered_set>

#include "internal.hpp"

namespace dgamr {
namespace {

// packed cell key: root (24 bits) | Morton key at max_level (36 bits) | level (4 bits)
uint64_t morton(int L, int l, const int32_t a[3]) {
    uint64_t X = (uint64_t)a[0] << (L - l), Y = (uint64_t)a[1] << (L - l), Z = (uint64_t)a[2] << (L - l);
    uint64_t k = 0;
    for (int b = 0; b < L; ++b) {
        k |= ((X >> b) & 1ull) << (3 * b);
        k |= ((Y >> b) & 1ull) << (3 * b + 1);
        k |= ((Z >> b) & 1ull) << (3 * b + 2);
    }
    return k;
}

uint64_t cell_key(int L, const Leaf& c) {
    return ((uint64_t)c.r << 40) | (morton(L, c.l, c.a) << 4) | (uint64_t)c.l;
}

Leaf parent_of(const Leaf& c) {
    Leaf p = c;
    p.l = c.l - 1;
    for (int d = 0; d < 3; ++d) p.a[d] = c.a[d] >> 1;
    return p;
}

Leaf child_of(const Leaf& c, int id) {
    Leaf ch = c;
    ch.l = c.l + 1;
    for (int d = 0; d < 3; ++d) ch.a[d] = 2 * c.a[d] + ((id >> d) & 1);
    return ch;
}

int child_id_of(const Leaf& c) { return (c.a[0] & 1) | ((c.a[1] & 1) << 1) | ((c.a[2] & 1) << 2); }

struct Forest {
    const dg_forest_desc& desc;
    int L;
    std::unordered_set<uint64_t> set;
    explicit Forest(const dg_forest_desc& d) : desc(d), L(d.max_level) {}

    bool has(const Leaf& c) const { return set.count(cell_key(L, c)) != 0; }

    // leaf equal to c or containing it; returns false if c is refined / absent
    bool containing(Leaf c, Leaf& out) const {
        for (;;) {
            if (has(c)) { out = c; return true; }
            if (c.l == 0) return false;
            c = parent_of(c);
        }
    }

    // same-level cell across face f = 2d + s; false at a wall
    bool neighbor(const Leaf& c, int f, Leaf& nb) const {
        const int d = f >> 1, s = f & 1;
        const int n[3] = {desc.nx, desc.ny, desc.nz};
        int rc[3] = {c.r % desc.nx, (c.r / desc.nx) % desc.ny, c.r / (desc.nx * desc.ny)};
        nb = c;
        const int span = 1 << c.l;
        nb.a[d] += s ? 1 : -1;
        if (nb.a[d] < 0 || nb.a[d] >= span) {
            nb.a[d] = nb.a[d] < 0 ? span - 1 : 0;
            rc[d] += s ? 1 : -1;
            if (rc[d] < 0 || rc[d] >= n[d]) {
                if (!desc.periodic[d]) return false;
                rc[d] = (rc[d] + n[d]) % n[d];
            }
        }
        nb.r = rc[0] + desc.nx * (rc[1] + desc.ny * rc[2]);
        return true;
    }

    // the 4 children of c touching its face on `side` of axis d, by quadrant
    void face_children(const Leaf& c, int d, int side, Leaf out[4]) const {
        int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        for (int q = 0; q < 4; ++q) {
            int bits[3];
            bits[d] = side;
            bits[t1] = q & 1;
            bits[t2] = q >> 1;
            out[q] = child_of(c, bits[0] | (bits[1] << 1) | (bits[2] << 2));
        }
    }
};

void sort_leaves(int L, std::vector<Leaf>& v) {
    std::sort(v.begin(), v.end(), [L](const Leaf& x, const Leaf& y) { return cell_key(L, x) < cell_key(L, y); });
}

std::string check_desc(const dg_forest_desc& d) {
    if (d.N < kMinN || d.N > kMaxN) return "N must be in [2, 7]";
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return "nx, ny, nz must be >= 1";
    if ((int64_t)d.nx * d.ny * d.nz >= (1 << 24)) return "too many roots";
    if (d.max_level < 0 || d.max_level > kMaxLevel) return "max_level must be in [0, 12]";
    for (int k = 0; k < 3; ++k) {
        if (!(d.hi[k] > d.lo[k])) return "hi must exceed lo on every axis";
        if (d.periodic[k] != 0 && d.periodic[k] != 1) return "periodic must be 0 or 1";
    }
    return "";
}

std::vector<Leaf> to_vector(const Forest& F) {
    std::vector<Leaf> v;
    v.reserve(F.set.size());
    for (uint64_t k : F.set) {
        Leaf c;
        c.l = (int)(k & 15ull);
        c.r = (int)(k >> 40);
        uint64_t mk = (k >> 4) & ((1ull << 36) - 1);
        int X = 0, Y = 0, Z = 0;
        for (int b = 0; b < F.L; ++b) {
            X |= (int)((mk >> (3 * b)) & 1ull) << b;
            Y |= (int)((mk >> (3 * b + 1)) & 1ull) << b;
            Z |= (int)((mk >> (3 * b + 2)) & 1ull) << b;
        }
        int sh = F.L - c.l;
        c.a[0] = X >> sh;
        c.a[1] = Y >> sh;
        c.a[2] = Z >> sh;
        v.push_back(c);
    }
    sort_leaves(F.L, v);
    return v;
}

}  // namespace

std::string forest_uniform(const dg_forest_desc& desc, HostMesh& out) {
    std::string err = check_desc(desc);
    if (!err.empty()) return err;
    out = HostMesh();
    out.desc = desc;
    const int nr = desc.nx * desc.ny * desc.nz;
    out.leaves.resize(nr);
    for (int r = 0; r < nr; ++r) out.leaves[r] = Leaf{r, 0, {0, 0, 0}};
    out.xfer_src.resize(nr);
    out.xfer_kind.assign(nr, DG_KIND_COPY);
    for (int r = 0; r < nr; ++r) out.xfer_src[r] = r;
    forest_tables(out);
    return "";
}

std::string forest_refine(const HostMesh& prev, const int8_t* flags, HostMesh& out) {
    const dg_forest_desc& desc = prev.desc;
    const int L = desc.max_level;
    Forest F(desc);
    std::unordered_map<uint64_t, int32_t> old_index;
    old_index.reserve(prev.leaves.size() * 2);
    for (size_t e = 0; e < prev.leaves.size(); ++e) {
        old_index[cell_key(L, prev.leaves[e])] = (int32_t)e;
        F.set.insert(cell_key(L, prev.leaves[e]));
    }
    for (size_t e = 0; e < prev.leaves.size(); ++e) {
        const Leaf& lf = prev.leaves[e];
        if (flags[e] > 0 && lf.l < L) {
            F.set.erase(cell_key(L, lf));
            for (int c = 0; c < 8; ++c) F.set.insert(cell_key(L, child_of(lf, c)));
        }
    }
    // ripple: refine leaves that have a face neighbour two or more levels finer
    for (;;) {
        std::vector<Leaf> cur = to_vector(F);
        std::unordered_set<uint64_t> todo;
        for (const Leaf& z : cur) {
            if (z.l < 2) continue;
            for (int f = 0; f < 6; ++f) {
                Leaf c, x;
                if (!F.neighbor(z, f, c)) continue;
                if (F.containing(c, x) && x.l <= z.l - 2) todo.insert(cell_key(L, x));
            }
        }
        if (todo.empty()) break;
        for (const Leaf& z : cur) {
            uint64_t k = cell_key(L, z);
            if (!todo.count(k)) continue;
            if (z.l >= L) return "balance would exceed max_level";
            F.set.erase(k);
            for (int c = 0; c < 8; ++c) F.set.insert(cell_key(L, child_of(z, c)));
        }
    }
    out = HostMesh();
    out.desc = desc;
    out.leaves = to_vector(F);
    const size_t K = out.leaves.size();
    out.xfer_src.resize(K);
    out.xfer_kind.resize(K);
    std::unordered_set<int32_t> refined;
    for (size_t e = 0; e < K; ++e) {
        const Leaf& lf = out.leaves[e];
        auto it = old_index.find(cell_key(L, lf));
        if (it != old_index.end()) {
            out.xfer_src[e] = it->second;
            out.xfer_kind[e] = DG_KIND_COPY;
        } else {
            auto ip = old_index.find(cell_key(L, parent_of(lf)));
            if (ip == old_index.end()) return "internal: a leaf was refined twice in one pass";
            out.xfer_src[e] = ip->second;
            out.xfer_kind[e] = child_id_of(lf);
            refined.insert(ip->second);
        }
    }
    out.n_refined = (int64_t)refined.size();
    forest_tables(out);
    return "";
}

std::string forest_coarsen(const HostMesh& prev, const int8_t* flags, HostMesh& out) {
    const dg_forest_desc& desc = prev.desc;
    const int L = desc.max_level;
    Forest F(desc);
    std::unordered_map<uint64_t, int32_t> idx;
    idx.reserve(prev.leaves.size() * 2);
    for (size_t e = 0; e < prev.leaves.size(); ++e) {
        idx[cell_key(L, prev.leaves[e])] = (int32_t)e;
        F.set.insert(cell_key(L, prev.leaves[e]));
    }
    std::unordered_set<uint64_t> parents, tried;
    for (size_t e = 0; e < prev.leaves.size(); ++e) {
        const Leaf& lf = prev.leaves[e];
        if (lf.l == 0 || flags[e] >= 0) continue;
        Leaf p = parent_of(lf);
        uint64_t pk = cell_key(L, p);
        if (!tried.insert(pk).second) continue;
        bool all = true;
        for (int c = 0; c < 8 && all; ++c) {
            auto it = idx.find(cell_key(L, child_of(p, c)));
            all = it != idx.end() && flags[it->second] < 0;
        }
        if (!all) continue;
        bool veto = false;
        for (int f = 0; f < 6 && !veto; ++f) {
            Leaf c, x;
            if (!F.neighbor(p, f, c)) continue;
            if (F.containing(c, x)) continue;  // neighbour leaf no finer than the parent
            Leaf fc[4];
            F.face_children(c, f >> 1, 1 - (f & 1), fc);
            for (int q = 0; q < 4; ++q)
                if (!F.has(fc[q])) veto = true;
        }
        if (!veto) parents.insert(pk);
    }
    // rebuild the set: remove children of merged parents, add the parents
    std::vector<Leaf> newv;
    newv.reserve(prev.leaves.size());
    std::unordered_set<uint64_t> added;
    for (size_t e = 0; e < prev.leaves.size(); ++e) {
        const Leaf& lf = prev.leaves[e];
        if (lf.l > 0) {
            Leaf p = parent_of(lf);
            uint64_t pk = cell_key(L, p);
            if (parents.count(pk)) {
                if (added.insert(pk).second) newv.push_back(p);
                continue;
            }
        }
        newv.push_back(lf);
    }
    sort_leaves(L, newv);
    out = HostMesh();
    out.desc = desc;
    out.leaves = newv;
    const size_t K = newv.size();
    out.xfer_src.resize(K);
    out.xfer_kind.resize(K);
    for (size_t e = 0; e < K; ++e) {
        const Leaf& lf = newv[e];
        auto it = idx.find(cell_key(L, lf));
        if (it != idx.end()) {
            out.xfer_src[e] = it->second;
            out.xfer_kind[e] = DG_KIND_COPY;
        } else {
            out.xfer_src[e] = idx.at(cell_key(L, child_of(lf, 0)));
            out.xfer_kind[e] = DG_KIND_FAMILY;
        }
    }
    out.n_coarsened = (int64_t)parents.size();
    forest_tables(out);
    return "";
}

void forest_tables(HostMesh& m) {
    const dg_forest_desc& desc = m.desc;
    const int L = desc.max_level;
    Forest F(desc);
    std::unordered_map<uint64_t, int32_t> idx;
    idx.reserve(m.leaves.size() * 2);
    for (size_t e = 0; e < m.leaves.size(); ++e) {
        uint64_t k = cell_key(L, m.leaves[e]);
        idx[k] = (int32_t)e;
        F.set.insert(k);
    }
    const size_t K = m.leaves.size();
    m.conf.clear();
    m.bnd.clear();
    m.hang.clear();
    m.ftype.assign(K * 6, -1);
    m.fnb.assign(K * 24, -1);
    for (size_t e = 0; e < K; ++e) {
        const Leaf& lf = m.leaves[e];
        for (int f = 0; f < 6; ++f) {
            const int d = f >> 1, s = f & 1;
            Leaf c, x;
            if (!F.neighbor(lf, f, c)) {
                m.bnd.push_back((int32_t)e);
                m.bnd.push_back(f);
                m.ftype[e * 6 + f] = FT_WALL;
                continue;
            }
            if (F.containing(c, x)) {
                int32_t nb = idx.at(cell_key(L, x));
                if (x.l == lf.l) {
                    if (s == 1) {
                        m.conf.push_back((int32_t)e);
                        m.conf.push_back(nb);
                        m.conf.push_back(d);
                    }
                    m.ftype[e * 6 + f] = FT_CONF;
                    m.fnb[(e * 6 + f) * 4] = nb;
                } else {
                    // this leaf is the fine side: quadrant from its tangential anchor bits
                    int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                    int q = (lf.a[t1] & 1) | ((lf.a[t2] & 1) << 1);
                    m.ftype[e * 6 + f] = FT_FINE | (q << 8);
                    m.fnb[(e * 6 + f) * 4] = nb;
                }
            } else {
                Leaf fc[4];
                F.face_children(c, d, 1 - s, fc);
                m.hang.push_back((int32_t)e);
                m.hang.push_back(f);
                m.ftype[e * 6 + f] = FT_COARSE;
                for (int q = 0; q < 4; ++q) {
                    int32_t ef = idx.at(cell_key(L, fc[q]));
                    m.hang.push_back(ef);
                    m.fnb[(e * 6 + f) * 4 + q] = ef;
                }
            }
        }
    }
}

void leaf_geometry(const dg_forest_desc& desc, const Leaf& lf, const std::vector<double>& xi, double h[3],
                   double* c) {
    const int n[3] = {desc.nx, desc.ny, desc.nz};
    const int rc[3] = {lf.r % desc.nx, (lf.r / desc.nx) % desc.ny, lf.r / (desc.nx * desc.ny)};
    const int N1 = (int)xi.size();
    const double scale = (double)(1 << lf.l);
    for (int d = 0; d < 3; ++d) {
        const double w = (desc.hi[d] - desc.lo[d]) / n[d];
        h[d] = w / scale;
        for (int j = 0; j < N1; ++j)
            c[d * N1 + j] = desc.lo[d] + w * (rc[d] + (lf.a[d] + (1.0 + xi[j]) / 2.0) / scale);
    }
}

}  // namespace dgamr

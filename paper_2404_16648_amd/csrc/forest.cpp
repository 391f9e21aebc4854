// Brick forest of oct-trees (section 3.1: every coarse cell is the root of a
// tree, only active leaves are kept, flagged cells are replaced by their
// children or their parent), with 2:1 face balance (section 4.3) and the face
// and transfer tables the kernels need.  Host-side integer work.
//
// Ordering and balance rules (the paper fixes none of them):
//   * leaves sorted by (rank of the root along a Morton curve over the root
//     coordinates, Morton key of the anchor scaled to max_level), x the least
//     significant bit in both; child id c = a + 2b + 4c' (the whole brick is
//     one space-filling curve, so face neighbours sit close together in memory
//     along every axis);
//   * refine pass: +1 flags below max_level, then refine every leaf with a face
//     neighbour two or more levels finer until nothing changes;
//   * coarsen pass: a family of 8 leaves all flagged -1 merges unless a leaf
//     face-adjacent to the parent is two or more levels finer (judged on the
//     mesh before the pass);
//   * face tables enumerated by leaf, then face f = 2d + s; conforming faces
//     from the minus leaf's plus face, hanging faces from the coarse side with
//     fine leaves by quadrant a + 2b over the tangential axes.
//
// Lookups use the sorted leaf array itself: leaves are disjoint and sorted by
// the key of their lower corner, so the leaf containing a cell (if any) is the
// last leaf whose key does not exceed the cell's key -- a binary search.
#include <omp.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <tuple>

#include "internal.hpp"

namespace dgamr {
namespace {

// rank of every root along the Morton curve over the root coordinates (bits of
// rx, ry, rz interleaved, rx the least significant); cached per brick shape
std::shared_ptr<const std::vector<uint32_t>> root_ranks(const dg_forest_desc& d) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, std::shared_ptr<const std::vector<uint32_t>>> cache;
    const auto shape = std::make_tuple(d.nx, d.ny, d.nz);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(shape);
    if (it != cache.end()) return it->second;
    const int64_t n = (int64_t)d.nx * d.ny * d.nz;
    std::vector<std::pair<uint64_t, uint32_t>> kv((size_t)n);
    for (int64_t r = 0; r < n; ++r) {
        const uint64_t rc[3] = {(uint64_t)(r % d.nx), (uint64_t)((r / d.nx) % d.ny), (uint64_t)(r / ((int64_t)d.nx * d.ny))};
        uint64_t k = 0;
        for (int b = 0; b < 21; ++b)
            for (int a = 0; a < 3; ++a) k |= ((rc[a] >> b) & 1ull) << (3 * b + a);
        kv[(size_t)r] = {k, (uint32_t)r};
    }
    std::sort(kv.begin(), kv.end());
    auto rank = std::make_shared<std::vector<uint32_t>>((size_t)n);
    for (int64_t i = 0; i < n; ++i) (*rank)[kv[(size_t)i].second] = (uint32_t)i;
    cache.emplace(shape, rank);
    return rank;
}

// position key of a cell's lower corner: root rank (24 bits) | Morton key at max_level (36 bits)
uint64_t pos_key(const uint32_t* rank, int L, const Leaf& c) {
    const uint64_t X = (uint64_t)c.a[0] << (L - c.l), Y = (uint64_t)c.a[1] << (L - c.l),
                   Z = (uint64_t)c.a[2] << (L - c.l);
    uint64_t k = 0;
    for (int b = 0; b < L; ++b) {
        k |= ((X >> b) & 1ull) << (3 * b);
        k |= ((Y >> b) & 1ull) << (3 * b + 1);
        k |= ((Z >> b) & 1ull) << (3 * b + 2);
    }
    return ((uint64_t)rank[c.r] << 36) | k;
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

bool same_cell(const Leaf& x, const Leaf& y) {
    return x.r == y.r && x.l == y.l && x.a[0] == y.a[0] && x.a[1] == y.a[1] && x.a[2] == y.a[2];
}

// true if leaf x (level <= c.l) is c or an ancestor of c
bool contains(const Leaf& x, const Leaf& c) {
    if (x.r != c.r || x.l > c.l) return false;
    const int sh = c.l - x.l;
    return (c.a[0] >> sh) == x.a[0] && (c.a[1] >> sh) == x.a[1] && (c.a[2] >> sh) == x.a[2];
}

// sorted leaf array with its keys: the leaves of a mesh are stored in this order
// already and are used in place; any other sequence is sorted into an owned copy
struct Sorted {
    const dg_forest_desc& desc;
    int L;
    std::shared_ptr<const std::vector<uint32_t>> rank_hold;
    const uint32_t* rank;
    std::vector<Leaf> own;
    const std::vector<Leaf>* lv = nullptr;
    std::vector<uint64_t> keys;

    Sorted(const dg_forest_desc& d, const std::vector<Leaf>& v)
        : desc(d), L(d.max_level), rank_hold(root_ranks(d)), rank(rank_hold->data()) {
        if (!key_in_place(v)) sort_copy(v);
    }
    Sorted(const dg_forest_desc& d, std::vector<Leaf>&& v)
        : desc(d), L(d.max_level), rank_hold(root_ranks(d)), rank(rank_hold->data()) {
        own = std::move(v);
        if (!key_in_place(own)) sort_copy(own);
    }
    const std::vector<Leaf>& leaves() const { return *lv; }
    // the sorted leaves, moved out when owned
    std::vector<Leaf> take() {
        if (lv == &own) return std::move(own);
        return *lv;
    }

  private:
    bool key_in_place(const std::vector<Leaf>& v) {
        const int64_t n = (int64_t)v.size();
        keys.resize(n);
#pragma omp parallel for schedule(static) if (n > 4096)
        for (int64_t i = 0; i < n; ++i) keys[i] = pos_key(rank, L, v[i]);
        int unsorted = 0;
#pragma omp parallel for schedule(static) reduction(| : unsorted) if (n > 4096)
        for (int64_t i = 1; i < n; ++i) unsorted |= keys[i - 1] >= keys[i];
        if (!unsorted) lv = &v;
        return !unsorted;
    }
    void sort_copy(const std::vector<Leaf>& v) {
        std::vector<std::pair<uint64_t, Leaf>> kv(v.size());
        for (size_t i = 0; i < v.size(); ++i) kv[i] = {keys[i], v[i]};
        std::sort(kv.begin(), kv.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
        std::vector<Leaf> sorted(kv.size());
        for (size_t i = 0; i < kv.size(); ++i) {
            keys[i] = kv[i].first;
            sorted[i] = kv[i].second;
        }
        own = std::move(sorted);
        lv = &own;
    }

  public:
    // first index in [0, n) whose key exceeds k (upper) or is not below k (!upper),
    // searched by galloping out from `hint`: face neighbours lie close together on
    // the space-filling curve, so the bracket is usually a few entries wide
    size_t gallop(uint64_t k, size_t hint, bool upper) const {
        const size_t n = keys.size();
        auto before = [&](size_t i) { return upper ? keys[i] <= k : keys[i] < k; };
        size_t lo, hi;  // answer in (lo, hi]: before(lo) holds (or lo = npos), before(hi) fails (or hi = n)
        if (hint >= n) hint = n ? n - 1 : 0;
        if (n == 0) return 0;
        if (before(hint)) {
            size_t step = 1;
            lo = hint;
            hi = hint + 1;
            while (hi < n && before(hi)) {
                lo = hi;
                step <<= 1;
                hi = lo + step < n ? lo + step : n;
            }
            ++lo;
        } else {
            size_t step = 1;
            hi = hint;
            size_t cand = hint;
            for (;;) {
                if (cand == 0) {
                    lo = 0;
                    break;
                }
                const size_t nxt = cand >= step ? cand - step : 0;
                if (before(nxt)) {
                    lo = nxt + 1;
                    break;
                }
                hi = nxt;
                cand = nxt;
                step <<= 1;
            }
        }
        // binary search in [lo, hi)
        while (lo < hi) {
            const size_t mid = lo + (hi - lo) / 2;
            if (before(mid))
                lo = mid + 1;
            else
                hi = mid;
        }
        return lo;
    }

    // index of the leaf equal to or containing cell c, or -1 if c is refined
    int containing(const Leaf& c, size_t hint = 0) const {
        const uint64_t k = pos_key(rank, L, c);
        const size_t it = gallop(k, hint, true);
        if (it == 0) return -1;
        const int i = (int)it - 1;
        return contains((*lv)[i], c) ? i : -1;
    }

    // index of the leaf equal to cell c, or -1
    int find(const Leaf& c, size_t hint = 0) const {
        const uint64_t k = pos_key(rank, L, c);
        const size_t i = gallop(k, hint, false);
        if (i == keys.size() || keys[i] != k) return -1;
        return (*lv)[i].l == c.l ? (int)i : -1;
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
};

// the 4 children of c touching its face on `side` of axis d, by quadrant
void face_children(const Leaf& c, int d, int side, Leaf out[4]) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    for (int q = 0; q < 4; ++q) {
        int bits[3];
        bits[d] = side;
        bits[t1] = q & 1;
        bits[t2] = q >> 1;
        out[q] = child_of(c, bits[0] | (bits[1] << 1) | (bits[2] << 2));
    }
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

}  // namespace

std::string forest_uniform(const dg_forest_desc& desc, HostMesh& out) {
    std::string err = check_desc(desc);
    if (!err.empty()) return err;
    out = HostMesh();
    out.desc = desc;
    const int nr = desc.nx * desc.ny * desc.nz;
    out.leaves.resize(nr);
    const auto rank = root_ranks(desc);
    for (int r = 0; r < nr; ++r) out.leaves[(*rank)[r]] = Leaf{r, 0, {0, 0, 0}};
    out.xfer_src.resize(nr);
    out.xfer_kind.assign(nr, DG_KIND_COPY);
    for (int r = 0; r < nr; ++r) out.xfer_src[r] = r;
    forest_tables(out);
    return "";
}

// the result of a pass that changes no leaf: prev's leaves and tables, identity transfer
static void unchanged(const HostMesh& prev, HostMesh& out) {
    out = prev;
    const int64_t K = (int64_t)prev.leaves.size();
    out.xfer_kind.assign(K, DG_KIND_COPY);
    for (int64_t e = 0; e < K; ++e) out.xfer_src[e] = (int32_t)e;
    out.n_refined = out.n_coarsened = 0;
    out.same_as_prev = true;
}

// the face tables of one leaf e of the sorted mesh m (its row of ftype and fnb)
static void leaf_faces(HostMesh& m, const Sorted& S, int64_t e) {
    const dg_forest_desc& desc = m.desc;
    const Leaf& lf = m.leaves[e];
    for (int f = 0; f < 6; ++f) {
        const int d = f >> 1, s = f & 1;
        int32_t* nb = &m.fnb[(e * 6 + f) * 4];
        for (int q = 0; q < 4; ++q) nb[q] = -1;
        Leaf c;
        if (!S.neighbor(lf, f, c)) {
            m.ftype[e * 6 + f] = FT_WALL;
            continue;
        }
        const int x = S.containing(c, (size_t)e);
        if (x >= 0) {
            if (S.leaves()[x].l == lf.l) {
                const int rz = lf.r / (desc.nx * desc.ny);
                const bool wrap_z = d == 2 && (s ? rz == desc.nz - 1 && lf.a[2] == (1 << lf.l) - 1
                                                 : rz == 0 && lf.a[2] == 0);
                m.ftype[e * 6 + f] = FT_CONF | (wrap_z ? FT_BG_NB : 0);
            } else {
                // this leaf is the fine side: quadrant from its tangential anchor bits
                const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                const int q = (lf.a[t1] & 1) | ((lf.a[t2] & 1) << 1);
                m.ftype[e * 6 + f] = FT_FINE | (q << 8);
            }
            nb[0] = x;
        } else {
            Leaf fc[4];
            face_children(c, d, 1 - s, fc);
            m.ftype[e * 6 + f] = FT_COARSE;
            for (int q = 0; q < 4; ++q) nb[q] = S.find(fc[q], (size_t)e);  // leaves, by balance
        }
    }
}

// the global face lists of m from its per-leaf tables, in (leaf, face) order:
// per-leaf counts, their prefix sums, then every leaf writes its own entries
static void face_lists(HostMesh& m) {
    const int64_t K = (int64_t)m.leaves.size();
    std::vector<int64_t, NoInit<int64_t>> oc(K + 1), ob(K + 1), oh(K + 1);
    oc[0] = ob[0] = oh[0] = 0;
#pragma omp parallel for schedule(static) if (K > 4096)
    for (int64_t e = 0; e < K; ++e) {
        int c = 0, b = 0, h = 0;
        for (int f = 0; f < 6; ++f) {
            const int type = m.ftype[e * 6 + f] & 0xff;
            c += type == FT_CONF && (f & 1);
            b += type == FT_WALL;
            h += type == FT_COARSE;
        }
        oc[e + 1] = c;
        ob[e + 1] = b;
        oh[e + 1] = h;
    }
    for (int64_t e = 0; e < K; ++e) {
        oc[e + 1] += oc[e];
        ob[e + 1] += ob[e];
        oh[e + 1] += oh[e];
    }
    m.conf.resize(3 * oc[K]);
    m.bnd.resize(2 * ob[K]);
    m.hang.resize(6 * oh[K]);
#pragma omp parallel for schedule(static) if (K > 4096)
    for (int64_t e = 0; e < K; ++e) {
        int32_t* pc = m.conf.data() + 3 * oc[e];
        int32_t* pb = m.bnd.data() + 2 * ob[e];
        int32_t* ph = m.hang.data() + 6 * oh[e];
        for (int f = 0; f < 6; ++f) {
            const int type = m.ftype[e * 6 + f] & 0xff;
            const int32_t* nb = &m.fnb[(e * 6 + f) * 4];
            if (type == FT_WALL) {
                *pb++ = (int32_t)e;
                *pb++ = f;
            } else if (type == FT_CONF && (f & 1)) {
                *pc++ = (int32_t)e;
                *pc++ = nb[0];
                *pc++ = f >> 1;
            } else if (type == FT_COARSE) {
                *ph++ = (int32_t)e;
                *ph++ = f;
                for (int q = 0; q < 4; ++q) *ph++ = nb[q];
            }
        }
    }
}

// the face tables of m, a pass's result in canonical order with its plan from prev:
// a kept leaf none of whose face neighbours in prev changed has the same faces, so
// its rows are prev's with the neighbour indices renumbered; every other leaf (new,
// or beside a leaf that was refined or merged) is searched as in forest_tables
static void tables_from(HostMesh& m, const HostMesh& prev) {
    const int64_t K = (int64_t)m.leaves.size(), K0 = (int64_t)prev.leaves.size();
    ivec renum(K0);  // the new index of every kept old leaf, else -1
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < K0; ++x) renum[x] = -1;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < K; ++e)
        if (m.xfer_kind[e] == DG_KIND_COPY) renum[m.xfer_src[e]] = (int32_t)e;
    m.ftype.resize(K * 6);  // every row is written below: copied, or searched
    m.fnb.resize(K * 24);
    std::vector<char> dirty(K, 0);
    int64_t ndirty = 0;
#pragma omp parallel for schedule(static) reduction(+ : ndirty)
    for (int64_t e = 0; e < K; ++e) {
        bool d = m.xfer_kind[e] != DG_KIND_COPY;
        const int64_t x = m.xfer_src[e];
        for (int i = 0; i < 24 && !d; ++i) {
            const int32_t y = prev.fnb[x * 24 + i];
            d = y >= 0 && renum[y] < 0;
        }
        if (!d) {
            for (int f = 0; f < 6; ++f) m.ftype[e * 6 + f] = prev.ftype[x * 6 + f];
            for (int i = 0; i < 24; ++i) {
                const int32_t y = prev.fnb[x * 24 + i];
                m.fnb[e * 24 + i] = y >= 0 ? renum[y] : -1;
            }
        }
        dirty[e] = d;
        ndirty += d;
    }
    if (ndirty > 0) {
        Sorted S(m.desc, m.leaves);
        if (S.lv != &m.leaves) throw std::logic_error("internal: a pass left the leaves out of order");
        std::vector<int64_t> list;
        list.reserve(ndirty);
        for (int64_t e = 0; e < K; ++e)
            if (dirty[e]) list.push_back(e);
#pragma omp parallel for schedule(static) if (ndirty > 256)
        for (int64_t i = 0; i < ndirty; ++i) leaf_faces(m, S, list[i]);
    }
    face_lists(m);
}

std::string forest_refine(const HostMesh& prev, const int8_t* flags, HostMesh& out) {
    const dg_forest_desc& desc = prev.desc;
    const int L = desc.max_level;
    bool any_flag = false;
    for (size_t e = 0; e < prev.leaves.size() && !any_flag; ++e) any_flag = flags[e] > 0 && prev.leaves[e].l < L;
    if (!any_flag) {  // prev is balanced, so the ripple has nothing to do either
        unchanged(prev, out);
        return "";
    }
    // the result in canonical order (children take their parent's place, in child
    // order) with its plan: an old leaf kept (COPY, its index) or child id of old
    // leaf src
    const int64_t K0 = (int64_t)prev.leaves.size();
    std::vector<int64_t> at(K0 + 1, 0);  // first position of old leaf e in the result
    for (int64_t e = 0; e < K0; ++e) at[e + 1] = at[e] + ((flags[e] > 0 && prev.leaves[e].l < L) ? 8 : 1);
    std::vector<Leaf> cur(at[K0]);
    ivec src(at[K0]), kind(at[K0]);
#pragma omp parallel for schedule(static) if (K0 > 4096)
    for (int64_t e = 0; e < K0; ++e) {
        const Leaf& lf = prev.leaves[e];
        const int64_t p = at[e];
        if (at[e + 1] - p == 8) {
            for (int c = 0; c < 8; ++c) {
                cur[p + c] = child_of(lf, c);
                src[p + c] = (int32_t)e;
                kind[p + c] = c;
            }
        } else {
            cur[p] = lf;
            src[p] = (int32_t)e;
            kind[p] = DG_KIND_COPY;
        }
    }
    // ripple: refine leaves that have a face neighbour two or more levels finer.
    // prev is balanced, so such a neighbour is always a new leaf: only new leaves
    // are checked
    for (;;) {
        Sorted S(desc, cur);
        if (S.lv != &cur) return "internal: refined leaves out of order";
        std::vector<int64_t> fresh;
        for (int64_t i = 0; i < (int64_t)cur.size(); ++i)
            if (kind[i] != DG_KIND_COPY && cur[i].l >= 2) fresh.push_back(i);
        std::vector<char> todo(cur.size(), 0);
        int any = 0;
        const int64_t nf = (int64_t)fresh.size();
#pragma omp parallel for schedule(static) reduction(| : any) if (nf > 256)
        for (int64_t k = 0; k < nf; ++k) {
            const int64_t zi = fresh[k];
            const Leaf& z = cur[zi];
            for (int f = 0; f < 6; ++f) {
                Leaf c;
                if (!S.neighbor(z, f, c)) continue;
                const int x = S.containing(c, (size_t)zi);
                if (x >= 0 && cur[x].l <= z.l - 2) {
#pragma omp atomic write
                    todo[x] = 1;
                    any = 1;
                }
            }
        }
        if (!any) break;
        std::vector<Leaf> nxt;
        ivec nsrc, nkind;
        nxt.reserve(cur.size() + 64);
        nsrc.reserve(cur.size() + 64);
        nkind.reserve(cur.size() + 64);
        for (size_t i = 0; i < cur.size(); ++i) {
            const Leaf& z = cur[i];
            if (!todo[i]) {
                nxt.push_back(z);
                nsrc.push_back(src[i]);
                nkind.push_back(kind[i]);
                continue;
            }
            if (z.l >= L) return "balance would exceed max_level";
            if (kind[i] != DG_KIND_COPY) return "internal: a leaf was refined twice in one pass";
            for (int c = 0; c < 8; ++c) {
                nxt.push_back(child_of(z, c));
                nsrc.push_back(src[i]);
                nkind.push_back(c);
            }
        }
        cur.swap(nxt);
        src.swap(nsrc);
        kind.swap(nkind);
    }
    out = HostMesh();
    out.desc = desc;
    out.leaves = std::move(cur);
    out.xfer_src = std::move(src);
    out.xfer_kind = std::move(kind);
    int64_t nref = 0;
    for (int32_t k : out.xfer_kind) nref += k == 0;
    out.n_refined = nref;
    tables_from(out, prev);
    return "";
}

// the families the coarsen pass merges: merge[e] = 1 at the first child of each;
// returns their number
static int64_t coarsen_families(const HostMesh& prev, const int8_t* flags, std::vector<char>& merge) {
    const dg_forest_desc& desc = prev.desc;
    Sorted P(desc, prev.leaves);
    const size_t K0 = P.leaves().size();
    // candidate families: 8 consecutive leaves (Morton order keeps a family
    // contiguous) that are the 8 children of one parent, all flagged -1; a family
    // starts at a child 0, so two candidates never overlap and each is judged on
    // its own (in parallel)
    merge.assign(K0, 0);
    const std::vector<Leaf>& lv = P.leaves();
    int64_t nmerged = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : nmerged)
    for (int64_t e = 0; e <= (int64_t)K0 - 8; ++e) {
        const Leaf& lf = lv[e];
        if (lf.l == 0 || child_id_of(lf) != 0 || flags[e] >= 0) continue;
        const Leaf p = parent_of(lf);
        bool fam = true;
        for (int c = 0; c < 8 && fam; ++c) fam = same_cell(lv[e + c], child_of(p, c)) && flags[e + c] < 0;
        if (!fam) continue;
        bool veto = false;
        for (int f = 0; f < 6 && !veto; ++f) {
            Leaf c;
            if (!P.neighbor(p, f, c)) continue;
            if (P.containing(c, (size_t)e) >= 0) continue;  // neighbour leaf no finer than the parent
            Leaf fc[4];
            face_children(c, f >> 1, 1 - (f & 1), fc);
            for (int q = 0; q < 4; ++q)
                if (P.find(fc[q], (size_t)e) < 0) veto = true;
        }
        if (!veto) {
            merge[e] = 1;
            ++nmerged;
        }
    }
    return nmerged;
}

bool pass_changes(const HostMesh& prev, const int8_t* flags, bool refine) {
    if (refine) {
        const int L = prev.desc.max_level;
        for (size_t e = 0; e < prev.leaves.size(); ++e)
            if (flags[e] > 0 && prev.leaves[e].l < L) return true;
        return false;
    }
    std::vector<char> merge;
    return coarsen_families(prev, flags, merge) > 0;
}

std::string forest_coarsen(const HostMesh& prev, const int8_t* flags, HostMesh& out) {
    const dg_forest_desc& desc = prev.desc;
    std::vector<char> merge;  // 1 at the first child of a family that merges
    const int64_t nmerged = coarsen_families(prev, flags, merge);
    if (nmerged == 0) {
        unchanged(prev, out);
        return "";
    }
    // prev's leaves are in canonical (sorted) order, the order the families were found
    // in; an old leaf that stays, or starts a merged family, moves down by 7 for every
    // family merged before it
    const std::vector<Leaf>& src = prev.leaves;
    const int64_t K0 = (int64_t)src.size();
    std::vector<int64_t, NoInit<int64_t>> before(K0 + 1);
    before[0] = 0;
    for (int64_t e = 0; e < K0; ++e) before[e + 1] = before[e] + merge[e];
    std::vector<char> inside(K0, 0);  // the children 1..7 of a merged family
#pragma omp parallel for schedule(static) if (K0 > 4096)
    for (int64_t e = 0; e < K0; ++e)
        if (merge[e])
            for (int c = 1; c < 8; ++c) inside[e + c] = 1;
    out = HostMesh();
    out.desc = desc;
    const int64_t K = K0 - 7 * nmerged;
    out.leaves.resize(K);
    out.xfer_src.resize(K);
    out.xfer_kind.resize(K);
#pragma omp parallel for schedule(static) if (K0 > 4096)
    for (int64_t e = 0; e < K0; ++e) {
        if (inside[e]) continue;
        const int64_t i = e - 7 * before[e];
        out.leaves[i] = merge[e] ? parent_of(src[e]) : src[e];
        out.xfer_src[i] = (int32_t)e;
        out.xfer_kind[i] = merge[e] ? DG_KIND_FAMILY : DG_KIND_COPY;
    }
    out.n_coarsened = nmerged;
    tables_from(out, prev);
    return "";
}

void forest_tables(HostMesh& m) {
    const dg_forest_desc& desc = m.desc;
    std::unique_ptr<Sorted> Sp(new Sorted(desc, m.leaves));
    if (Sp->lv != &m.leaves) {  // into canonical order, then index it in place
        m.leaves = Sp->take();
        Sp.reset(new Sorted(desc, m.leaves));
    }
    const Sorted& S = *Sp;
    const int64_t K = (int64_t)m.leaves.size();
    m.ftype.assign(K * 6, -1);
    m.fnb.assign(K * 24, -1);
    // per leaf and face: type and neighbours (independent, in parallel)
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < K; ++e) leaf_faces(m, S, e);
    face_lists(m);
}

bool tables_consistent(const HostMesh& h) {
    const int64_t K = (int64_t)h.leaves.size();
    if ((int64_t)h.ftype.size() != 6 * K || (int64_t)h.fnb.size() != 24 * K) return false;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad) if (K > 4096)
    for (int64_t i = 0; i < 6 * K; ++i) {
        const int type = h.ftype[i] & 0xff;
        const int nnb = type == FT_WALL ? 0 : type == FT_COARSE ? 4 : 1;
        bad |= type > FT_COARSE || h.ftype[i] < 0;
        for (int q = 0; q < nnb; ++q) bad |= h.fnb[i * 4 + q] < 0 || h.fnb[i * 4 + q] >= K;
    }
    return !bad;
}

bool plan_consistent(const HostMesh& h, int64_t K_from) {
    const int64_t K = (int64_t)h.leaves.size();
    if ((int64_t)h.xfer_src.size() != K || (int64_t)h.xfer_kind.size() != K) return false;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad) if (K > 4096)
    for (int64_t e = 0; e < K; ++e) {
        const int64_t src = h.xfer_src[e];
        const int kind = h.xfer_kind[e];
        if (kind == DG_KIND_COPY) {
            bad |= src < 0 || src >= K_from;
        } else if (kind == DG_KIND_FAMILY) {
            bad |= src < 0 || src + 7 >= K_from;
        } else if (kind >= 0 && kind < 8) {
            const int64_t e0 = e - kind;
            if (src < 0 || src >= K_from || e0 < 0 || e0 + 7 >= K) {
                bad = 1;
            } else {
                for (int c = 0; c < 8; ++c) bad |= h.xfer_kind[e0 + c] != c || h.xfer_src[e0 + c] != src;
            }
        } else {
            bad = 1;
        }
    }
    return !bad;
}

void box_leaf_arrays(const HostMesh& h, const std::vector<double>& xi, double* geo, double* c1d, int32_t* level) {
    const int64_t K = (int64_t)h.leaves.size();
    const int N1 = h.desc.N + 1;
#pragma omp parallel for schedule(static) if (K > 4096)
    for (int64_t e = 0; e < K; ++e) {
        double hh[3], c[3 * 8];  // N + 1 <= 8
        leaf_geometry(h.desc, h.leaves[e], xi, hh, c);
        for (int d = 0; d < 3; ++d) {
            geo[e * 4 + d] = 2.0 / hh[d];
            for (int j = 0; j < N1; ++j) c1d[(d * K + e) * N1 + j] = c[d * N1 + j];
        }
        geo[e * 4 + 3] = hh[0] * hh[1] * hh[2] / 8.0;
        level[e] = h.leaves[e].l;
    }
}

void stage_records(const HostMesh& h, const int32_t* hs, int rec_len, int32_t* srec) {
    const int64_t K = (int64_t)h.leaves.size();
#pragma omp parallel for schedule(static) if (K > 4096)
    for (int64_t e = 0; e < K; ++e) {
        int32_t* rec = srec + e * rec_len;
        for (int f = 0; f < 6; ++f) {
            rec[f] = h.ftype[e * 6 + f];
            rec[6 + f] = h.fnb[e * 24 + f * 4];
            rec[12 + f] = hs[e * 6 + f];
        }
        rec[18] = rec[19] = 0;
        if (h.sphere) {
            for (int f = 0; f < 6; ++f) {
                const int32_t* nb = &h.snb[(e * 6 + f) * 3];
                if (nb[0] >= 0) rec[18] |= (int32_t)((nb[1] & 7) | ((nb[2] & 1) << 3)) << (4 * f);
            }
            rec[19] = h.leaves[e].r;
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

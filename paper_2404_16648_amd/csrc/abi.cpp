// C ABI of the DG-AMR library: argument checks, mesh lifetime, device tables
// and kernel launches.  Declarations and contracts are in include/dg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dg.h"
#include "internal.hpp"
#include "kernels.hpp"

using namespace dgamr;

namespace {

thread_local std::string g_err;
std::atomic<uint64_t> g_next_id{1};

dg_status fail(dg_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

dg_status hip_fail(hipError_t e, const char* where) {
    return fail(DG_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                            \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return hip_fail(e_, #call);        \
    } while (0)

// reference operators per N, computed once per process
RefOps refops_cached(int N) {
    static std::mutex mu;
    static std::map<int, RefOps> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(N);
    if (it == cache.end()) it = cache.emplace(N, make_refops(N)).first;
    return it->second;
}

void free_device(dg_mesh* m) {
    if (m->upload_done) (void)hipEventDestroy((hipEvent_t)m->upload_done);
    m->upload_done = nullptr;
    if (m->d_base) (void)hipFree(m->d_base);
    m->d_base = nullptr;
    m->d_ops = m->d_geo = m->d_c1d = m->d_bg = m->d_red = m->d_eta = nullptr;
    m->d_ftype = m->d_fnb = m->d_level = m->d_xsrc = m->d_xkind = nullptr;
    m->d_hslot = m->d_hang = nullptr;
    m->d_mort = nullptr;
    m->d_mortC = nullptr;
    m->d_flags = nullptr;
    m->d_metric = m->d_fgeo = nullptr;
    m->d_xlist = nullptr;
    if (m->d_sigma) (void)hipFree(m->d_sigma);
    m->d_sigma = nullptr;
}

// byte offsets of the arrays in a mesh's one device block, 256-byte aligned;
// [0, upload) is copied from the host, the rest is device workspace
struct DevLayout {
    size_t ops, geo, c1d, ft, nb, hs, hg, lv, xs, xk, sr, met, fg, xl, upload, bg, red, eta, fl, mort, mortC, total;
};

DevLayout dev_layout(int64_t K, int N, int64_t red_len, int64_t n_hang, bool sphere, int64_t n_xlist) {
    const size_t N1 = (size_t)N + 1, k = (size_t)K;
    size_t end = 0;
    auto take = [&](size_t bytes) {
        const size_t off = (end + 255) & ~(size_t)255;
        end = off + bytes;
        return off;
    };
    DevLayout L{};
    L.ops = take(sizeof(double) * (11 * N1 * N1 + N1));
    L.geo = take(sizeof(double) * 4 * k);
    L.c1d = take(sizeof(double) * 3 * k * N1);
    L.ft = take(sizeof(int32_t) * 6 * k);
    L.nb = take(sizeof(int32_t) * 24 * k);
    L.hs = take(sizeof(int32_t) * 6 * k);
    L.hg = take(sizeof(int32_t) * 6 * (size_t)n_hang);
    L.lv = take(sizeof(int32_t) * k);
    L.xs = take(sizeof(int32_t) * k);
    L.xk = take(sizeof(int32_t) * k);
    L.sr = take(sizeof(int32_t) * kStageRec * k);
    // shell meshes: metric terms and face geometry
    L.met = take(sphere ? sizeof(double) * 10 * k * N1 * N1 * N1 : 0);
    L.fg = take(sphere ? sizeof(double) * 24 * k * N1 * N1 : 0);
    L.xl = take(sphere ? sizeof(int32_t) * (size_t)n_xlist : 0);
    L.upload = end;
    L.bg = take(sizeof(double) * 3 * k * N1);
    L.red = take(sizeof(double) * (size_t)red_len);
    L.eta = take(sizeof(double) * (k > 0 ? k : 1));
    L.fl = take(k > 0 ? k : 1);
    L.mort = take(sizeof(double) * 25 * N1 * N1 * (size_t)n_hang);
    L.mortC = take(sizeof(double) * 5 * N1 * N1 * (size_t)n_hang);
    L.total = end;
    return L;
}

void set_device_pointers(dg_mesh* m, char* base, const DevLayout& L) {
    m->d_base = base;
    m->d_ops = (double*)(base + L.ops);
    m->d_geo = (double*)(base + L.geo);
    m->d_c1d = (double*)(base + L.c1d);
    m->d_ftype = (int32_t*)(base + L.ft);
    m->d_fnb = (int32_t*)(base + L.nb);
    m->d_hslot = (int32_t*)(base + L.hs);
    m->d_hang = (int32_t*)(base + L.hg);
    m->d_mort = (double*)(base + L.mort);
    m->d_mortC = (double*)(base + L.mortC);
    m->d_level = (int32_t*)(base + L.lv);
    m->d_xsrc = (int32_t*)(base + L.xs);
    m->d_xkind = (int32_t*)(base + L.xk);
    m->d_srec = (int32_t*)(base + L.sr);
    m->d_metric = m->h.sphere ? (double*)(base + L.met) : nullptr;
    m->d_fgeo = m->h.sphere ? (double*)(base + L.fg) : nullptr;
    m->d_xlist = m->h.sphere ? (int32_t*)(base + L.xl) : nullptr;
    m->d_bg = (double*)(base + L.bg);
    m->d_red = (double*)(base + L.red);
    m->d_eta = (double*)(base + L.eta);
    m->d_flags = (int8_t*)(base + L.fl);
}

// every face of every leaf has a type and in-range neighbours (the kernels index
// field arrays with them); checked on the host before anything is uploaded
// A pass that changed no leaf leaves every table as it was: the device block is
// cloned from the previous mesh's (and its background, when computed), and only
// the identity transfer plan is uploaded.
// host checks of a new mesh, before any device work: every face has a type and
// in-range neighbours, the transfer plan is sound, the sizes fit the kernels' indexing
dg_status validate_mesh(const dg_mesh* m) {
    const HostMesh& h = m->h;
    const int64_t K = (int64_t)h.leaves.size();
    // a pass that changed no leaf copied the checked tables of prev and holds the
    // identity plan
    if (h.same_as_prev && m->prev && m->prev->h.leaves.size() == h.leaves.size()) return DG_OK;
    if (!tables_consistent(h)) return fail(DG_EINVAL, "internal: inconsistent face tables");
    if (!plan_consistent(h, m->prev ? (int64_t)m->prev->h.leaves.size() : K))
        return fail(DG_EINVAL, "internal: inconsistent transfer plan");
    if (5 * K * (int64_t)(h.desc.N + 1) * (h.desc.N + 1) * (h.desc.N + 1) >= ((int64_t)1 << 31))
        return fail(DG_EINVAL, "mesh too large: 5 K Np must stay below 2^31");
    return DG_OK;
}

// Pinned staging of the device-table uploads, shared by every mesh of the process:
// a mesh's tables are written into it and copied asynchronously on the caller's
// stream, so a new mesh costs no page faults of fresh host memory and no
// synchronisation (a pageable copy of the ~10 MB of tables of a 25k-leaf mesh
// faulted in ~2 ms, the pinned copy takes ~0.2 ms).  The next upload waits for the
// previous copy out of the buffer before overwriting it.
struct UploadStaging {
    std::mutex mu;
    char* buf = nullptr;
    size_t cap = 0;
    hipEvent_t last = nullptr;  // the copy that last read the buffer
};
UploadStaging& upload_staging() {
    static UploadStaging s;
    return s;
}

// one device allocation per mesh, filled from the host tables by one asynchronous
// copy on stream s (on the device the mesh was built on)
dg_status build_device(dg_mesh* m, hipStream_t s) {
    const HostMesh& h = m->h;
    const int64_t K = (int64_t)h.leaves.size();
    const int N = h.desc.N, N1 = N + 1;
    m->red_len = (int64_t)budget_blocks(K) * 8 + 8;
    m->n_hang = (int64_t)h.hang.size() / 6;
    // shells: the children of the plan and their parents (the refinement's scale factor)
    std::vector<int32_t> xlist;
    if (h.sphere) {
        for (int64_t e = 0; e < K; ++e)
            if (h.xfer_kind[e] >= 0 && h.xfer_kind[e] < 8) xlist.push_back((int32_t)e);
        m->n_xch = (int64_t)xlist.size();
        for (int64_t e = 0; e < K; ++e)
            if (h.xfer_kind[e] == 0) xlist.push_back(h.xfer_src[e]);
        m->n_xpar = (int64_t)xlist.size() - m->n_xch;
    }
    const DevLayout L = dev_layout(K, N, m->red_len, m->n_hang, h.sphere, (int64_t)xlist.size());
    // one staging buffer and one copy for every table of the mesh; the background,
    // reduction and flag buffers are carved from the same block
    UploadStaging& stg = upload_staging();
    std::lock_guard<std::mutex> stg_lock(stg.mu);
    if (stg.last) {
        HIP_TRY(hipEventSynchronize(stg.last));
        (void)hipEventDestroy(stg.last);
        stg.last = nullptr;
    }
    if (stg.cap < L.upload) {
        if (stg.buf) (void)hipHostFree(stg.buf);
        stg.buf = nullptr;
        stg.cap = 0;
        const size_t want = std::max(L.upload + L.upload / 4, (size_t)1 << 20);
        HIP_TRY(hipHostMalloc((void**)&stg.buf, want, hipHostMallocDefault));
        stg.cap = want;
    }
    struct View {
        char* p;
        char* data() { return p; }
    } up{stg.buf};
    // D, I0, I1, R0, R1 ([N1][N1] row-major), w [N1], then I0^T, I1^T, R0^T, R1^T (adjoint),
    // then P0, P1 (pointwise matching)
    double* ops = (double*)(up.data() + L.ops);
    for (auto* v : {&m->ops.D, &m->ops.I0, &m->ops.I1, &m->ops.R0, &m->ops.R1, &m->ops.w})
        for (double x : *v) *ops++ = x;
    for (auto* v : {&m->ops.I0, &m->ops.I1, &m->ops.R0, &m->ops.R1})
        for (int c = 0; c < N1; ++c)
            for (int r = 0; r < N1; ++r) *ops++ = (*v)[r * N1 + c];
    for (auto* v : {&m->ops.P0, &m->ops.P1})
        for (double x : *v) *ops++ = x;
    double* geo = (double*)(up.data() + L.geo);
    double* c1d = (double*)(up.data() + L.c1d);
    int32_t* level = (int32_t*)(up.data() + L.lv);
    if (h.sphere) {
        // shell: the curvilinear geometry (geo unused: zeros)
        std::memset(geo, 0, sizeof(double) * 4 * K);
        for (int64_t e = 0; e < K; ++e) level[e] = h.leaves[e].l;
        sphere_geometry(h, m->ops, (double*)(up.data() + L.met), (double*)(up.data() + L.fg), c1d);
        if (!xlist.empty()) std::memcpy(up.data() + L.xl, xlist.data(), sizeof(int32_t) * xlist.size());
    } else {
        box_leaf_arrays(h, m->ops.x, geo, c1d, level);
    }
    std::memcpy(up.data() + L.ft, h.ftype.data(), sizeof(int32_t) * 6 * K);
    std::memcpy(up.data() + L.nb, h.fnb.data(), sizeof(int32_t) * 24 * K);
    // hanging faces: each (leaf, face) on either side of a mortar knows its table row
    int32_t* hs = (int32_t*)(up.data() + L.hs);
    std::fill(hs, hs + 6 * K, -1);
    for (int64_t r = 0; r < m->n_hang; ++r) {
        const int32_t* row = &h.hang[6 * r];
        hs[row[0] * 6 + row[1]] = (int32_t)r;
        // the fine leaves' face: the opposite one in a brick, recorded per row on a shell
        const int ff = h.sphere ? h.snb[(row[0] * 6 + row[1]) * 3 + 1] : (row[1] ^ 1);
        for (int q = 0; q < 4; ++q) hs[row[2 + q] * 6 + ff] = (int32_t)r;
    }
    if (m->n_hang) std::memcpy(up.data() + L.hg, h.hang.data(), sizeof(int32_t) * 6 * m->n_hang);
    std::memcpy(up.data() + L.xs, h.xfer_src.data(), sizeof(int32_t) * K);
    std::memcpy(up.data() + L.xk, h.xfer_kind.data(), sizeof(int32_t) * K);
    // the stage kernel's face tables, one contiguous record per leaf (read with scalar
    // loads): per face type, first neighbour, hanging-face row or -1
    stage_records(h, hs, kStageRec, (int32_t*)(up.data() + L.sr));
    char* base = nullptr;
    HIP_TRY(hipMalloc((void**)&base, L.total));
    set_device_pointers(m, base, L);
    HIP_TRY(hipMemcpyAsync(base, up.data(), L.upload, hipMemcpyHostToDevice, s));
    hipEvent_t ev_stg = nullptr, ev_mesh = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&ev_stg, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ev_stg, s));
    stg.last = ev_stg;
    HIP_TRY(hipEventCreateWithFlags(&ev_mesh, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ev_mesh, s));
    m->upload_done = ev_mesh;
    m->upload_stream = s;
    m->on_device = true;
    return DG_OK;
}

// calls that shell meshes do not provide (no refinement, mortars, adjoint,
// tracer or indicator on the shell)
dg_status no_sphere(const dg_mesh* m) {
    if (m && m->h.sphere) return fail(DG_EUNSUPPORTED, "not provided for cubed-sphere shell meshes");
    return DG_OK;
}

dg_status check_phys(const dg_phys* p) {
    if (!p) return fail(DG_EINVAL, "phys is NULL");
    if (!(p->cv > 0.0) || !(p->cp > p->cv)) return fail(DG_EINVAL, "need cp > cv > 0");
    if (!(p->P0 > 0.0)) return fail(DG_EINVAL, "need P0 > 0");
    if (p->background == DG_BG_NEUTRAL || p->background == DG_BG_ISOTHERMAL) {
        if (!(p->theta0 > 0.0)) return fail(DG_EINVAL, "need theta0 > 0");
    } else if (p->background == DG_BG_CONSTANT) {
        if (!(p->rho0 > 0.0) || !(p->Theta0 > 0.0)) return fail(DG_EINVAL, "need rho0, Theta0 > 0");
    } else {
        return fail(DG_EINVAL, "unknown background");
    }
    if (p->precision != DG_FP64 && p->precision != DG_MIXED) return fail(DG_EINVAL, "unknown precision");
    if (p->nonconforming != DG_NC_MORTAR && p->nonconforming != DG_NC_POINTWISE)
        return fail(DG_EINVAL, "unknown nonconforming-face scheme");
    if (!(p->mu >= 0.0) || !std::isfinite(p->mu)) return fail(DG_EINVAL, "need a finite mu >= 0");
    return DG_OK;
}

// the device tables are made when a call first uses the mesh on the GPU (a mesh that
// is only inspected on the host, such as a pass that changed no leaf and is
// dropped, never costs an allocation or a copy)
// s is the stream of the call: the upload is enqueued on it, and a call on another
// stream waits for the upload until it has completed
dg_status check_dev_mesh(const dg_mesh* mc, hipStream_t s) {
    if (!mc) return fail(DG_EINVAL, "mesh is NULL");
    if (mc->h.desc.host_only) return fail(DG_EINVAL, "mesh was built host_only");
    static std::mutex mu;
    if (mc->on_device) {
        if (!mc->upload_done) return DG_OK;
        std::lock_guard<std::mutex> lock(mu);
        dg_mesh* m = const_cast<dg_mesh*>(mc);
        if (!m->upload_done) return DG_OK;
        if (hipEventQuery((hipEvent_t)m->upload_done) == hipSuccess) {
            (void)hipEventDestroy((hipEvent_t)m->upload_done);
            m->upload_done = nullptr;
        } else if ((void*)s != m->upload_stream) {
            HIP_TRY(hipStreamWaitEvent(s, (hipEvent_t)m->upload_done, 0));
        }
        return DG_OK;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (mc->on_device) return DG_OK;
    dg_mesh* m = const_cast<dg_mesh*>(mc);
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != m->device) HIP_TRY(hipSetDevice(m->device));
    const dg_status st = build_device(m, s);
    if (st != DG_OK) free_device(m);
    if (cur != m->device) (void)hipSetDevice(cur);
    return st;
}

// a background that varies with z (the neutral atmosphere under gravity) cannot be
// periodic in z: the two sides of a z wrap would carry different hydrostatic
// states, and no choice of background at a face across the wrap is consistent
dg_status check_wrap(const dg_mesh* m, const dg_phys* p) {
    if (m->h.desc.periodic[2] && p->background == DG_BG_NEUTRAL && p->g != 0.0)
        return fail(DG_EINVAL, "a periodic z axis needs a background that does not vary with z (g = 0 or DG_BG_CONSTANT)");
    return DG_OK;
}

bool same_bg(const dg_phys& a, const dg_phys& b) {
    return a.cp == b.cp && a.cv == b.cv && a.P0 == b.P0 && a.g == b.g && a.background == b.background &&
           a.theta0 == b.theta0 && a.rho0 == b.rho0 && a.Theta0 == b.Theta0;
}

// background profile [3][K][N+1] for phys, (re)computed on the caller's stream when phys changes
dg_status ensure_bg(dg_mesh* m, const dg_phys* p, hipStream_t s) {
    if (m->bg_valid && same_bg(m->bg_phys, *p)) return DG_OK;
    BgParams bp{p->background, p->cp, p->cv, p->P0, p->g, p->theta0, p->rho0, p->Theta0};
    HIP_TRY(launch_background((int64_t)m->h.leaves.size(), m->h.desc.N, m->d_c1d, m->d_bg, bp, s));
    m->bg_phys = *p;
    m->bg_valid = true;
    return DG_OK;
}

// C(gamma, k), k = 1..kBinomTerms, for the binomial series of (1 + x)^gamma - 1
BinomCoef binom_coef(const dg_phys* p) {
    BinomCoef b{};
    const long double g = (long double)p->cp / (long double)p->cv;
    long double c = 1.0L;
    for (int k = 1; k <= kBinomTerms; ++k) {
        c = c * (g - (k - 1)) / k;
        b.c[k - 1] = (double)c;
    }
    return b;
}

// the viscous gradient workspace [3][5][K][Np], allocated at the first call with
// mu > 0 on this mesh (not while stream s is being captured into a graph)
dg_status ensure_sigma(dg_mesh* m, hipStream_t s) {
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    if (m->d_sigma) return DG_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return fail(DG_EINVAL, "the viscous workspace of this mesh is allocated by the first call with mu > 0, "
                               "which must not be captured into a graph");
    const size_t n1 = (size_t)m->h.desc.N + 1;
    const size_t bytes = 15 * m->h.leaves.size() * n1 * n1 * n1 * sizeof(double);
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != m->device) HIP_TRY(hipSetDevice(m->device));
    const hipError_t e = hipMalloc((void**)&m->d_sigma, bytes ? bytes : 256);
    if (cur != m->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
        m->d_sigma = nullptr;
        return fail(DG_ENOMEM, "viscous workspace: hipMalloc failed");
    }
    return DG_OK;
}

StageArgs stage_args(const dg_mesh* m, const dg_phys* p) {
    StageArgs a{};
    a.ops = m->d_ops;
    a.geo = m->d_geo;
    a.bg = m->d_bg;
    a.ftype = m->d_ftype;
    a.fnb = m->d_fnb;
    a.hslot = m->d_hslot;
    a.mort = m->d_mort;
    a.srec = m->d_srec;
    a.K = (int64_t)m->h.leaves.size();
    a.gamma = p->cp / p->cv;
    a.g = p->g;
    a.binom = binom_coef(p);
    // the update's q0 and its output are touched once per stage: when the three fields
    // of a stage (q0, stage input, output) exceed the 256 MiB last-level cache they are
    // streamed past it, leaving the cache to the stage input, whose face traces are
    // read again by the neighbours (measured: density current, 372 MB, 109 -> 101 us;
    // AMR bubble, 207 MB, whose fields stay cached, 61 -> 67 us if streamed too)
    const double n1 = m->h.desc.N + 1;
    const double field_bytes = 5.0 * (double)a.K * n1 * n1 * n1 * 8.0;
    a.stream_io = 3.0 * field_bytes > 256.0 * 1024 * 1024 ? 1 : 0;
    return a;
}

}  // namespace

extern "C" {

const char* dg_last_error(void) { return g_err.c_str(); }

dg_status dg_mesh_build(const dg_forest_desc* desc, const dg_mesh* prev, const int8_t* flags, int32_t pass,
                        dg_mesh** out) {
    if (!out) return fail(DG_EINVAL, "out is NULL");
    *out = nullptr;
    dg_mesh* m = nullptr;
    try {
        m = new dg_mesh();
        std::string err;
        if (!prev) {
            if (!desc) {
                delete m;
                return fail(DG_EINVAL, "desc is NULL");
            }
            err = forest_uniform(*desc, m->h);
        } else {
            if (prev->h.sphere && prev->h.sdesc.max_level == 0) {
                delete m;
                return fail(DG_EUNSUPPORTED, "the shell was built with max_level = 0 (no refinement)");
            }
            if (!flags && !prev->h.leaves.empty()) {
                delete m;
                return fail(DG_EINVAL, "flags is NULL");
            }
            if (pass != DG_PASS_REFINE && pass != DG_PASS_COARSEN)
                err = "unknown pass";
            else if (prev->h.sphere)
                err = pass == DG_PASS_REFINE ? sphere_refine(prev->h, flags, m->h)
                                             : sphere_coarsen(prev->h, flags, m->h);
            else if (pass == DG_PASS_REFINE)
                err = forest_refine(prev->h, flags, m->h);
            else
                err = forest_coarsen(prev->h, flags, m->h);
            m->prev = prev;
            m->prev_id = prev->id;
        }
        if (!err.empty()) {
            delete m;
            return fail(DG_EINVAL, err);
        }
        m->ops = refops_cached(m->h.desc.N);
        m->id = g_next_id++;
        dg_status st = validate_mesh(m);
        if (st == DG_OK && !m->h.desc.host_only) {
            const hipError_t e = hipGetDevice(&m->device);
            if (e != hipSuccess) st = hip_fail(e, "hipGetDevice");
        }
        if (st != DG_OK) {
            delete m;
            return st;
        }
    } catch (const std::bad_alloc&) {
        if (m) {
            free_device(m);
            delete m;
        }
        return fail(DG_ENOMEM, "host allocation failed");
    } catch (const std::exception& ex) {
        if (m) {
            free_device(m);
            delete m;
        }
        return fail(DG_EINVAL, ex.what());
    }
    *out = m;
    return DG_OK;
}

dg_status dg_sphere_mesh_build(const dg_sphere_desc* desc, dg_mesh** out) {
    if (!out) return fail(DG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!desc) return fail(DG_EINVAL, "desc is NULL");
    if (desc->N > 5) return fail(DG_EINVAL, "shell meshes support N = 2..5");
    dg_mesh* m = nullptr;
    try {
        m = new dg_mesh();
        const std::string err = sphere_build(*desc, m->h);
        if (!err.empty()) {
            delete m;
            return fail(DG_EINVAL, err);
        }
        m->h.desc.host_only = desc->host_only;
        m->ops = refops_cached(desc->N);
        m->id = g_next_id++;
        dg_status st = validate_mesh(m);
        if (st == DG_OK && !desc->host_only) {
            const hipError_t e = hipGetDevice(&m->device);
            if (e != hipSuccess) st = hip_fail(e, "hipGetDevice");
        }
        if (st != DG_OK) {
            delete m;
            return st;
        }
    } catch (const std::bad_alloc&) {
        delete m;
        return fail(DG_ENOMEM, "host allocation failed");
    }
    *out = m;
    return DG_OK;
}

dg_status dg_sphere_faces(const dg_mesh* m, int32_t* nb) {
    if (!m || !nb) return fail(DG_EINVAL, "NULL argument");
    if (!m->h.sphere) return fail(DG_EINVAL, "not a shell mesh");
    std::memcpy(nb, m->h.snb.data(), m->h.snb.size() * sizeof(int32_t));
    return DG_OK;
}

dg_status dg_sphere_geometry(const dg_mesh* m, double* metric, double* fgeo, double* c1d) {
    if (!m || !metric || !fgeo || !c1d) return fail(DG_EINVAL, "NULL argument");
    if (!m->h.sphere) return fail(DG_EINVAL, "not a shell mesh");
    try {
        sphere_geometry(m->h, m->ops, metric, fgeo, c1d);
    } catch (const std::bad_alloc&) {
        return fail(DG_ENOMEM, "host allocation failed");
    }
    return DG_OK;
}

dg_status dg_sphere_volumes(const dg_mesh* m, double* vol, double* totals) {
    if (!m || !totals) return fail(DG_EINVAL, "NULL argument");
    if (!m->h.sphere) return fail(DG_EINVAL, "not a shell mesh");
    try {
        const int64_t K = (int64_t)m->h.leaves.size();
        const int N1 = m->h.desc.N + 1, NP = N1 * N1 * N1;
        std::vector<long double> v(K);
        sphere_volumes(m->h, v.data());
        long double ex = 0.0L;
        for (int64_t e = 0; e < K; ++e) {
            ex += v[e];
            if (vol) vol[e] = (double)v[e];
        }
        // the isoparametric volume: J W summed over every node, J from the geometry
        // the kernels use
        std::vector<double> metric((size_t)10 * K * NP), fgeo((size_t)24 * K * N1 * N1), c1d((size_t)3 * K * N1);
        sphere_geometry(m->h, m->ops, metric.data(), fgeo.data(), c1d.data());
        const std::vector<double>& w = m->ops.w;
        long double disc = 0.0L;
        for (int64_t e = 0; e < K; ++e)
            for (int n = 0; n < NP; ++n)
                disc += (long double)metric[(size_t)e * NP + n] * w[n % N1] * w[(n / N1) % N1] * w[n / (N1 * N1)];
        totals[0] = (double)disc;
        totals[1] = (double)ex;
    } catch (const std::bad_alloc&) {
        return fail(DG_ENOMEM, "host allocation failed");
    }
    return DG_OK;
}

// a shell and the shell with twice the elements per panel edge and twice the layers
static dg_status shell_pair(const dg_mesh* coarse, const dg_mesh* fine) {
    if (!coarse || !fine) return fail(DG_EINVAL, "mesh is NULL");
    if (!coarse->h.sphere || !fine->h.sphere) return fail(DG_EINVAL, "not a shell mesh");
    const dg_sphere_desc &c = coarse->h.sdesc, &f = fine->h.sdesc;
    if (f.N != c.N || f.n != 2 * c.n || f.nz != 2 * c.nz || f.r_e != c.r_e || f.H != c.H)
        return fail(DG_EINVAL, "the fine shell must have the same N, r_e and H and twice the elements per "
                               "panel edge and twice the layers of the coarse one");
    if (coarse->device != fine->device) return fail(DG_EINVAL, "the two shells are on different devices");
    return DG_OK;
}

dg_status dg_sphere_refine_project(const dg_mesh* coarse, const dg_mesh* fine, const dg_phys* phys,
                                   const double* q_coarse, double* q_fine, double* scale, void* stream) {
    dg_status st = shell_pair(coarse, fine);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = check_dev_mesh(coarse, s)) || (st = check_dev_mesh(fine, s))) return st;
    if ((st = check_phys(phys))) return st;
    if (!q_coarse || !q_fine) return fail(DG_EINVAL, "NULL field pointer");
    if (phys->mu != 0.0)  // the transfers run in float64 for either precision of the stage
        return fail(DG_EUNSUPPORTED, "the shell transfer takes physics without viscosity");
    dg_mesh* mc = const_cast<dg_mesh*>(coarse);
    dg_mesh* mf = const_cast<dg_mesh*>(fine);
    if ((st = ensure_bg(mc, phys, s)) || (st = ensure_bg(mf, phys, s))) return st;
    const int N = coarse->h.desc.N;
    const int64_t Kc = (int64_t)coarse->h.leaves.size(), Kf = (int64_t)fine->h.leaves.size();
    ShellXferArgs a{q_coarse, q_fine, fine->d_ops, nullptr, nullptr, nullptr, nullptr, Kc, Kf, coarse->h.sdesc.n,
                    coarse->h.sdesc.nz};
    HIP_TRY(launch_shell_refine(N, a, s));
    // total mass before (coarse) and after (fine, interpolated): the budget reductions
    const double* w = fine->d_ops + 5 * (N + 1) * (N + 1);
    const int nbc = budget_blocks(Kc), nbf = budget_blocks(Kf);
    double* out_c = mc->d_red + (int64_t)nbc * 8;
    double* out_f = mf->d_red + (int64_t)nbf * 8;
    BudgetArgs bc{q_coarse, mc->d_bg, mc->d_geo, mc->d_metric, mc->d_c1d, w, mc->d_red, Kc,
                  phys->cp / phys->cv, phys->g, binom_coef(phys)};
    BudgetArgs bf{q_fine, mf->d_bg, mf->d_geo, mf->d_metric, mf->d_c1d, w, mf->d_red, Kf,
                  phys->cp / phys->cv, phys->g, binom_coef(phys)};
    HIP_TRY(launch_budgets(N, bc, nbc, out_c, s));
    HIP_TRY(launch_budgets(N, bf, nbf, out_f, s));
    HIP_TRY(launch_shell_scale(N, q_fine, mf->d_bg, Kf, out_c, out_f, out_f + 4, s));
    if (scale) {
        HIP_TRY(hipMemcpyAsync(scale, out_f + 4, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (!std::isfinite(*scale)) return fail(DG_ENONFINITE, "non-finite scale factor");
    }
    return DG_OK;
}

dg_status dg_sphere_coarsen_project(const dg_mesh* fine, const dg_mesh* coarse, const dg_phys* phys,
                                    const double* q_fine, double* q_coarse, void* stream) {
    dg_status st = shell_pair(coarse, fine);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = check_dev_mesh(coarse, s)) || (st = check_dev_mesh(fine, s))) return st;
    if ((st = check_phys(phys))) return st;
    if (!q_coarse || !q_fine) return fail(DG_EINVAL, "NULL field pointer");
    dg_mesh* mc = const_cast<dg_mesh*>(coarse);
    dg_mesh* mf = const_cast<dg_mesh*>(fine);
    if ((st = ensure_bg(mc, phys, s)) || (st = ensure_bg(mf, phys, s))) return st;
    const int64_t Kc = (int64_t)coarse->h.leaves.size(), Kf = (int64_t)fine->h.leaves.size();
    ShellXferArgs a{q_fine, q_coarse, fine->d_ops, mf->d_metric, mc->d_metric, mf->d_bg, mc->d_bg, Kf, Kc,
                    coarse->h.sdesc.n, coarse->h.sdesc.nz};
    HIP_TRY(launch_shell_coarsen(coarse->h.desc.N, a, s));
    return DG_OK;
}

dg_status dg_sphere_adapt_project(const dg_mesh* from, const dg_mesh* to, const dg_phys* phys, const double* q_from,
                                  double* q_to, double* scale, void* stream) {
    if (!from || !to) return fail(DG_EINVAL, "mesh is NULL");
    if (!from->h.sphere || !to->h.sphere) return fail(DG_EINVAL, "not a shell mesh");
    if (to->prev_id != from->id) return fail(DG_EINVAL, "`to` was not built from `from`");
    hipStream_t s = (hipStream_t)stream;
    dg_status st = check_dev_mesh(from, s);
    if (st || (st = check_dev_mesh(to, s))) return st;
    if ((st = check_phys(phys))) return st;
    if (phys->mu != 0.0)  // the transfers run in float64 for either precision of the stage
        return fail(DG_EUNSUPPORTED, "the shell transfer takes physics without viscosity");
    if (!q_from || !q_to) return fail(DG_EINVAL, "NULL field pointer");
    if (q_from == q_to) return fail(DG_EINVAL, "input and output fields must not alias");
    dg_mesh* mf = const_cast<dg_mesh*>(from);
    dg_mesh* mt = const_cast<dg_mesh*>(to);
    if ((st = ensure_bg(mf, phys, s)) || (st = ensure_bg(mt, phys, s))) return st;
    const int N = to->h.desc.N;
    const int64_t Kf = (int64_t)from->h.leaves.size(), Kt = (int64_t)to->h.leaves.size();
    ShellPlanArgs a{q_from, q_to, to->d_ops, mf->d_metric, mt->d_metric, mf->d_bg, mt->d_bg, to->d_xsrc,
                    to->d_xkind, Kf, Kt};
    HIP_TRY(launch_shell_plan(N, a, s));
    if (to->n_xch > 0) {
        // the refined parents' mass (source) and their children's (target), then the factor
        const double* w = to->d_ops + 5 * (N + 1) * (N + 1);
        double* out_f = mf->d_red + (int64_t)budget_blocks(Kf) * 8 + 4;
        double* out_t = mt->d_red + (int64_t)budget_blocks(Kt) * 8 + 4;
        HIP_TRY(launch_shell_mass(N, q_from, mf->d_bg, mf->d_metric, w, to->d_xlist + to->n_xch, to->n_xpar, Kf,
                                  mf->d_red, budget_blocks(to->n_xpar), out_f, s));
        HIP_TRY(launch_shell_mass(N, q_to, mt->d_bg, mt->d_metric, w, to->d_xlist, to->n_xch, Kt, mt->d_red,
                                  budget_blocks(to->n_xch), out_t, s));
        HIP_TRY(launch_shell_scale_list(N, q_to, mt->d_bg, Kt, to->d_xlist, to->n_xch, out_f, out_t, out_t + 1, s));
        if (scale) {
            HIP_TRY(hipMemcpyAsync(scale, out_t + 1, sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (!std::isfinite(*scale)) return fail(DG_ENONFINITE, "non-finite scale factor");
        }
    } else if (scale) {
        *scale = 1.0;
    }
    return DG_OK;
}

dg_status dg_sphere_adapt_project_adjoint(const dg_mesh* from, const dg_mesh* to, const dg_phys* phys,
                                          const double* q_from, const double* q_to, double scale,
                                          const double* qbar_to, double* qbar_from, void* stream) {
    if (!from || !to) return fail(DG_EINVAL, "mesh is NULL");
    if (!from->h.sphere || !to->h.sphere) return fail(DG_EINVAL, "not a shell mesh");
    if (to->prev_id != from->id) return fail(DG_EINVAL, "`to` was not built from `from`");
    hipStream_t s = (hipStream_t)stream;
    dg_status st = check_dev_mesh(from, s);
    if (st || (st = check_dev_mesh(to, s))) return st;
    if ((st = check_phys(phys))) return st;
    if (phys->mu != 0.0) return fail(DG_EUNSUPPORTED, "the shell transfer takes physics without viscosity");
    if (!qbar_to || !qbar_from) return fail(DG_EINVAL, "NULL field pointer");
    if (qbar_to == qbar_from) return fail(DG_EINVAL, "input and output fields must not alias");
    if (to->n_xch > 0) {
        if (!q_from || !q_to) return fail(DG_EINVAL, "NULL q_from or q_to for a pass that refines");
        if (!std::isfinite(scale) || scale <= 0.0) return fail(DG_EINVAL, "scale must be the transfer's positive factor");
    }
    // a refined family's children are consecutive entries of the plan, in child order
    const HostMesh& ht = to->h;
    const int64_t Kf = (int64_t)from->h.leaves.size(), Kt = (int64_t)ht.leaves.size();
    for (int64_t e = 0; e < Kt; ++e) {
        if (ht.xfer_kind[e] != 0) continue;
        if (e + 7 >= Kt) return fail(DG_EINVAL, "transfer plan: a refined family runs past the end");
        for (int a = 1; a < 8; ++a)
            if (ht.xfer_kind[e + a] != a || ht.xfer_src[e + a] != ht.xfer_src[e])
                return fail(DG_EINVAL, "transfer plan: a refined family is not consecutive");
    }
    dg_mesh* mf = const_cast<dg_mesh*>(from);
    dg_mesh* mt = const_cast<dg_mesh*>(to);
    if ((st = ensure_bg(mf, phys, s)) || (st = ensure_bg(mt, phys, s))) return st;
    const int N = ht.desc.N;
    double* out_f = mf->d_red + (int64_t)budget_blocks(Kf) * 8 + 4;
    double* out_t = mt->d_red + (int64_t)budget_blocks(Kt) * 8 + 4;
    if (to->n_xch > 0) {
        // the refined parents' mass under q_from, and qbar_to . (q_to + background) over the children
        const double* w = to->d_ops + 5 * (N + 1) * (N + 1);
        HIP_TRY(launch_shell_mass(N, q_from, mf->d_bg, mf->d_metric, w, to->d_xlist + to->n_xch, to->n_xpar, Kf,
                                  mf->d_red, budget_blocks(to->n_xpar), out_f, s));
        HIP_TRY(launch_shell_dot(N, qbar_to, q_to, mt->d_bg, to->d_xlist, to->n_xch, Kt, mt->d_red,
                                 budget_blocks(to->n_xch), out_t, s));
    }
    ShellPlanAdjArgs a{qbar_to, qbar_from, to->d_ops, mf->d_metric, mt->d_metric, to->d_xsrc, to->d_xkind,
                       out_f, out_t, to->n_xch > 0 ? scale : 1.0, Kf, Kt};
    HIP_TRY(launch_shell_plan_adjoint(N, a, s));
    return DG_OK;
}

dg_status dg_sphere_face_kinds(const dg_mesh* m, int32_t* kind) {
    if (!m || !kind) return fail(DG_EINVAL, "NULL argument");
    if (!m->h.sphere) return fail(DG_EINVAL, "not a shell mesh");
    for (size_t i = 0; i < m->h.skind.size(); ++i) kind[i] = m->h.skind[i] + 4 * m->h.saux[i];
    return DG_OK;
}

dg_status dg_pass_changes(const dg_mesh* m, const int8_t* flags, int32_t pass, int32_t* changes) {
    if (!m || !changes) return fail(DG_EINVAL, "NULL argument");
    if (!flags && !m->h.leaves.empty()) return fail(DG_EINVAL, "flags is NULL");
    if (pass != DG_PASS_REFINE && pass != DG_PASS_COARSEN) return fail(DG_EINVAL, "unknown pass");
    try {
        const bool refine = pass == DG_PASS_REFINE;
        if (m->h.sphere)
            *changes = m->h.sdesc.max_level > 0 && sphere_pass_changes(m->h, flags, refine) ? 1 : 0;
        else
            *changes = pass_changes(m->h, flags, refine) ? 1 : 0;
    } catch (const std::bad_alloc&) {
        return fail(DG_ENOMEM, "host allocation failed");
    }
    return DG_OK;
}

dg_status dg_mesh_free(dg_mesh* m) {
    if (!m) return DG_OK;
    free_device(m);
    delete m;
    return DG_OK;
}

dg_status dg_mesh_info_get(const dg_mesh* m, dg_mesh_info* info) {
    if (!m || !info) return fail(DG_EINVAL, "NULL argument");
    const HostMesh& h = m->h;
    info->K = (int64_t)h.leaves.size();
    info->N = h.desc.N;
    info->Np = (int64_t)(h.desc.N + 1) * (h.desc.N + 1) * (h.desc.N + 1);
    info->n_conf = (int64_t)h.conf.size() / 3;
    if (h.sphere) {  // shell: conforming face pairs counted from the connectivity
        int64_t pairs = 0;
        for (size_t i = 0; i < h.skind.size(); ++i) pairs += h.skind[i] == SK_CONF ? 1 : 0;
        info->n_conf = pairs / 2;
    }
    info->n_bnd = (int64_t)h.bnd.size() / 2;
    info->n_hang = (int64_t)h.hang.size() / 6;
    info->n_refined = h.n_refined;
    info->n_coarsened = h.n_coarsened;
    int lmax = 0;
    for (const Leaf& lf : h.leaves) lmax = lf.l > lmax ? lf.l : lmax;
    info->max_level_present = lmax;
    return DG_OK;
}

dg_status dg_mesh_export(const dg_mesh* m, const dg_mesh_tables* t) {
    if (!m || !t) return fail(DG_EINVAL, "NULL argument");
    const HostMesh& h = m->h;
    if (t->leaf)
        for (size_t e = 0; e < h.leaves.size(); ++e) {
            const Leaf& lf = h.leaves[e];
            int32_t* row = t->leaf + 5 * e;
            row[0] = lf.r;
            row[1] = lf.l;
            row[2] = lf.a[0];
            row[3] = lf.a[1];
            row[4] = lf.a[2];
        }
    auto cp = [](int32_t* dst, const ivec& src) {
        if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(int32_t));
    };
    cp(t->conf, h.conf);
    cp(t->bnd, h.bnd);
    cp(t->hang, h.hang);
    cp(t->xfer_src, h.xfer_src);
    cp(t->xfer_kind, h.xfer_kind);
    return DG_OK;
}

dg_status dg_node_coords(const dg_mesh* m, double* xyz, void* stream) {
    dg_status st = check_dev_mesh(m, (hipStream_t)stream);
    if (st) return st;
    if (!xyz) return fail(DG_EINVAL, "xyz is NULL");
    if (m->h.sphere) {
        HIP_TRY(launch_node_coords_sphere((int64_t)m->h.leaves.size(), m->h.desc.N, m->d_c1d, m->d_srec,
                                          m->h.sdesc.r_e, xyz, (hipStream_t)stream));
        return DG_OK;
    }
    HIP_TRY(launch_node_coords((int64_t)m->h.leaves.size(), m->h.desc.N, m->d_c1d, xyz, (hipStream_t)stream));
    return DG_OK;
}

dg_status dg_init_bell(const dg_mesh* mc, const dg_phys* phys, const dg_bell* bell, double* q, void* stream) {
    dg_status st = no_sphere(mc);
    if (st) return st;
    if ((st = check_dev_mesh(mc, (hipStream_t)stream))) return st;
    if ((st = check_phys(phys))) return st;
    if (!bell || !q) return fail(DG_EINVAL, "NULL argument");
    dg_mesh* m = const_cast<dg_mesh*>(mc);
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_bg(m, phys, s))) return st;
    const double th0 = phys->background == DG_BG_NEUTRAL ? phys->theta0 : phys->Theta0 / phys->rho0;
    HIP_TRY(launch_init_bell((int64_t)m->h.leaves.size(), m->h.desc.N, m->d_c1d, m->d_bg, th0, *bell, q, s));
    return DG_OK;
}

static dg_status stage_common(const dg_mesh* mc, const dg_phys* phys, int mode, double a, double b, double dt,
                              const double* q0, const double* qs, double* out, void* stream) {
    dg_status st = check_dev_mesh(mc, (hipStream_t)stream);
    if (st) return st;
    if ((st = check_phys(phys))) return st;
    if ((st = check_wrap(mc, phys))) return st;
    if (!qs || !out) return fail(DG_EINVAL, "NULL field pointer");
    if (out == qs) return fail(DG_EINVAL, "output must not alias the stage input");
    if (mode == MODE_RK && a != 0.0 && !q0) return fail(DG_EINVAL, "q0 is NULL while a != 0");
    dg_mesh* m = const_cast<dg_mesh*>(mc);
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_bg(m, phys, s))) return st;
    if (m->h.sphere) {
        if (phys->mu > 0.0) return fail(DG_EUNSUPPORTED, "no artificial viscosity on shell meshes");
        if (phys->nonconforming != DG_NC_MORTAR)
            return fail(DG_EUNSUPPORTED, "shell meshes take the mortars at hanging faces");
        const int64_t K = (int64_t)m->h.leaves.size();
        if (m->n_hang) {
            SphereMortArgs ma{qs, m->d_mort, m->d_ops, m->d_bg, m->d_srec, m->d_hang, m->d_metric, m->d_fgeo,
                              m->n_hang, K, phys->cp / phys->cv, binom_coef(phys)};
            HIP_TRY(launch_mortar_sphere(m->h.desc.N, ma, s));
        }
        SphereStageArgs sa{q0, qs, out, m->d_ops, m->d_bg, m->d_c1d, m->d_srec, m->d_metric, m->d_fgeo,
                           m->d_mort, K, a, b, dt, phys->cp / phys->cv, phys->g, binom_coef(phys)};
        HIP_TRY(launch_stage_sphere(m->h.desc.N, mode, phys->precision == DG_MIXED, sa, s));
        return DG_OK;
    }
    StageArgs args = stage_args(m, phys);
    args.q0 = q0;
    args.qs = qs;
    args.out = out;
    args.a = a;
    args.b = b;
    args.dt = dt;
    const int N = m->h.desc.N;
    const bool mixed = phys->precision == DG_MIXED;
    if (m->n_hang) {
        MortArgs ma{qs, m->d_mort, m->d_ops, m->d_geo, m->d_bg, m->d_hang, m->n_hang, args.K, args.gamma, args.binom,
                    phys->nonconforming == DG_NC_POINTWISE ? 1 : 0};
        HIP_TRY(launch_mortar(N, ma, s));
    }
    HIP_TRY(launch_stage(N, mode, mixed, args, s));
    if (phys->mu > 0.0) {
        // the stage is linear in R: add b dt R_visc(qs) (R_visc for dg_rhs) to its output
        if ((st = ensure_sigma(m, s))) return st;
        ViscArgs va{qs, m->d_sigma, out, m->d_mort, m->d_ops, m->d_geo, m->d_srec, m->d_hang, m->n_hang, args.K,
                    phys->mu, mode == MODE_RHS ? 1.0 : b * dt};
        HIP_TRY(launch_viscous(m->h.desc.N, va, s));
    }
    return DG_OK;
}

dg_status dg_rhs(const dg_mesh* m, const dg_phys* phys, const double* q, double* rhs, void* stream) {
    return stage_common(m, phys, MODE_RHS, 0.0, 1.0, 0.0, nullptr, q, rhs, stream);
}

dg_status dg_rk_stage(const dg_mesh* m, const dg_phys* phys, double a, double b, double dt, const double* q0,
                      const double* qs, double* qout, void* stream) {
    return stage_common(m, phys, MODE_RK, a, b, dt, q0, qs, qout, stream);
}

static dg_status xfer_common(const dg_mesh* from, const dg_mesh* to, const double* qin, double* qout,
                             void* stream, bool refine, bool adjoint, int32_t nvar = 5) {
    if (dg_status st0 = no_sphere(from)) return st0;
    if (dg_status st0 = no_sphere(to)) return st0;
    dg_status st = check_dev_mesh(from, (hipStream_t)stream);
    if (st) return st;
    if ((st = check_dev_mesh(to, (hipStream_t)stream))) return st;
    if (to->prev_id != from->id) return fail(DG_EINVAL, "`to` was not built from `from`");
    if (!qin || !qout) return fail(DG_EINVAL, "NULL field pointer");
    if (qin == qout) return fail(DG_EINVAL, "input and output fields must not alias");
    if (refine && to->h.n_coarsened) return fail(DG_EINVAL, "`to` was built by a coarsen pass");
    if (!refine && to->h.n_refined) return fail(DG_EINVAL, "`to` was built by a refine pass");
    const int64_t Kf = (int64_t)from->h.leaves.size(), Kt = (int64_t)to->h.leaves.size();
    XferArgs a{qin, qout, to->d_ops, to->d_xsrc, to->d_xkind, adjoint ? Kt : Kf, adjoint ? Kf : Kt, Kt, nvar};
    hipStream_t s = (hipStream_t)stream;
    if (refine)
        HIP_TRY(launch_refine(to->h.desc.N, adjoint, a, s));
    else
        HIP_TRY(launch_coarsen(to->h.desc.N, adjoint, a, s));
    return DG_OK;
}

dg_status dg_refine_project(const dg_mesh* from, const dg_mesh* to, const double* q_from, double* q_to,
                            void* stream) {
    return xfer_common(from, to, q_from, q_to, stream, true, false);
}

dg_status dg_coarsen_project(const dg_mesh* from, const dg_mesh* to, const double* q_from, double* q_to,
                             void* stream) {
    return xfer_common(from, to, q_from, q_to, stream, false, false);
}

dg_status dg_refine_project_adjoint(const dg_mesh* from, const dg_mesh* to, const double* qbar_to, double* qbar_from,
                                    void* stream) {
    return xfer_common(from, to, qbar_to, qbar_from, stream, true, true);
}

dg_status dg_coarsen_project_adjoint(const dg_mesh* from, const dg_mesh* to, const double* qbar_to,
                                     double* qbar_from, void* stream) {
    return xfer_common(from, to, qbar_to, qbar_from, stream, false, true);
}

static dg_status tracer_common(const dg_mesh* mc, const dg_phys* phys, int mode, double a, double b, double dt,
                               const double* qs, const double* c0, const double* cs, double* out, void* stream) {
    dg_status st = no_sphere(mc);
    if (st) return st;
    if ((st = check_dev_mesh(mc, (hipStream_t)stream))) return st;
    if ((st = check_phys(phys))) return st;
    if ((st = check_wrap(mc, phys))) return st;
    if (!qs || !cs || !out) return fail(DG_EINVAL, "NULL field pointer");
    if (out == cs) return fail(DG_EINVAL, "output must not alias the tracer stage input");
    if ((const double*)out == qs) return fail(DG_EINVAL, "output must not alias the Euler state");
    if (mode == MODE_RK && a != 0.0 && !c0) return fail(DG_EINVAL, "c0 is NULL while a != 0");
    dg_mesh* m = const_cast<dg_mesh*>(mc);
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_bg(m, phys, s))) return st;
    const int64_t K = (int64_t)m->h.leaves.size();
    const double gamma = phys->cp / phys->cv;
    const BinomCoef bc = binom_coef(phys);
    if (m->n_hang) {
        TracerMortArgs ma{qs, cs, m->d_mortC, m->d_ops, m->d_geo, m->d_bg, m->d_hang, m->n_hang, K, gamma, bc,
                          phys->nonconforming == DG_NC_POINTWISE ? 1 : 0};
        HIP_TRY(launch_tracer_mortar(m->h.desc.N, ma, s));
    }
    TracerArgs ta{qs, c0, cs, out, m->d_ops, m->d_geo, m->d_bg, m->d_srec, m->d_mortC, K, a, b, dt, gamma, bc};
    HIP_TRY(launch_tracer_stage(m->h.desc.N, mode, ta, s));
    return DG_OK;
}

dg_status dg_tracer_rhs(const dg_mesh* m, const dg_phys* phys, const double* q, const double* c, double* rhs,
                        void* stream) {
    return tracer_common(m, phys, MODE_RHS, 0.0, 1.0, 0.0, q, nullptr, c, rhs, stream);
}

dg_status dg_tracer_stage(const dg_mesh* m, const dg_phys* phys, double a, double b, double dt, const double* qs,
                          const double* c0, const double* cs, double* cout, void* stream) {
    return tracer_common(m, phys, MODE_RK, a, b, dt, qs, c0, cs, cout, stream);
}

dg_status dg_project_fields(const dg_mesh* from, const dg_mesh* to, int32_t nvar, const double* q_from,
                            double* q_to, void* stream) {
    if (nvar < 1 || nvar > 5) return fail(DG_EINVAL, "nvar must be in [1, 5]");
    if (!to) return fail(DG_EINVAL, "to is NULL");
    return xfer_common(from, to, q_from, q_to, stream, to->h.n_coarsened == 0, false, nvar);
}

dg_status dg_tracer_mass(const dg_mesh* mc, const double* c, double* out_host, void* stream) {
    dg_status st = check_dev_mesh(mc, (hipStream_t)stream);
    if (st) return st;
    if (!c || !out_host) return fail(DG_EINVAL, "NULL argument");
    dg_mesh* m = const_cast<dg_mesh*>(mc);
    hipStream_t s = (hipStream_t)stream;
    const int64_t K = (int64_t)m->h.leaves.size();
    const int nblk = budget_blocks(K);
    double* out_dev = m->d_red + (int64_t)nblk * 8;
    HIP_TRY(launch_weighted_sum(m->h.desc.N, c, m->d_geo, m->d_ops + 5 * (m->h.desc.N + 1) * (m->h.desc.N + 1), K,
                                nblk, m->d_red, out_dev, s));
    HIP_TRY(hipMemcpyAsync(out_host, out_dev, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (!std::isfinite(out_host[0])) return fail(DG_ENONFINITE, "non-finite tracer mass");
    return DG_OK;
}

static dg_status adjoint_common(const dg_mesh* mc, const dg_phys* phys, int mode, double a1, const double* w1,
                                double a2, const double* w2, double b, double dt, const double* q, const double* lam,
                                double* out, void* stream) {
    dg_status st = check_dev_mesh(mc, (hipStream_t)stream);
    if (st) return st;
    if ((st = check_phys(phys))) return st;
    if ((st = check_wrap(mc, phys))) return st;
    if (phys->nonconforming != DG_NC_MORTAR)
        return fail(DG_EUNSUPPORTED, "the adjoint is provided for the mortar scheme only");
    if (phys->mu > 0.0) return fail(DG_EUNSUPPORTED, "the adjoint is provided without the artificial viscosity (mu = 0)");
    if (!q || !lam || !out) return fail(DG_EINVAL, "NULL field pointer");
    if (out == q || out == lam) return fail(DG_EINVAL, "output must not alias q or lam");
    if ((a1 != 0.0 && !w1) || (a2 != 0.0 && !w2)) return fail(DG_EINVAL, "NULL w1/w2 with a non-zero weight");
    dg_mesh* m = const_cast<dg_mesh*>(mc);
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_bg(m, phys, s))) return st;
    if (m->h.sphere) {
        const int64_t K = (int64_t)m->h.leaves.size();
        const double gamma = phys->cp / phys->cv;
        if (m->n_hang) {
            SphereMortAdjArgs ma{q, lam, m->d_mort, m->d_ops, m->d_bg, m->d_srec, m->d_hang, m->d_metric, m->d_fgeo,
                                 m->n_hang, K, gamma, binom_coef(phys)};
            HIP_TRY(launch_mortar_sphere_adjoint(m->h.desc.N, ma, s));
        }
        SphereAdjArgs sa{q, lam, w1, w2, out, m->d_ops, m->d_bg, m->d_c1d, m->d_srec, m->d_metric, m->d_fgeo,
                         m->d_mort, K, a1, a2, b, dt, gamma, phys->g, binom_coef(phys)};
        HIP_TRY(launch_adjoint_sphere(m->h.desc.N, mode, phys->precision == DG_MIXED, sa, s));
        return DG_OK;
    }
    AdjArgs a{};
    a.q = q;
    a.lam = lam;
    a.w1 = w1;
    a.w2 = w2;
    a.out = out;
    a.ops = m->d_ops;
    a.geo = m->d_geo;
    a.bg = m->d_bg;
    a.ftype = m->d_ftype;
    a.fnb = m->d_fnb;
    a.hslot = m->d_hslot;
    a.mort = m->d_mort;
    a.K = (int64_t)m->h.leaves.size();
    a.a1 = a1;
    a.a2 = a2;
    a.b = b;
    a.dt = dt;
    a.gamma = phys->cp / phys->cv;
    a.g = phys->g;
    a.binom = binom_coef(phys);
    if (m->n_hang) {
        MortAdjArgs ma{q, lam, m->d_mort, m->d_ops, m->d_geo, m->d_bg, m->d_hang, m->n_hang, a.K, a.gamma, a.binom};
        HIP_TRY(launch_mortar_adjoint(m->h.desc.N, ma, s));
    }
    HIP_TRY(launch_adjoint(m->h.desc.N, mode, phys->precision == DG_MIXED, a, s));
    return DG_OK;
}

dg_status dg_rhs_adjoint(const dg_mesh* m, const dg_phys* phys, const double* q, const double* lam, double* qbar,
                         void* stream) {
    return adjoint_common(m, phys, MODE_RHS, 0.0, nullptr, 0.0, nullptr, 1.0, 1.0, q, lam, qbar, stream);
}

dg_status dg_rk_stage_adjoint(const dg_mesh* m, const dg_phys* phys, double a1, const double* w1, double a2,
                              const double* w2, double b, double dt, const double* q, const double* y, double* out,
                              void* stream) {
    return adjoint_common(m, phys, MODE_RK, a1, w1, a2, w2, b, dt, q, y, out, stream);
}

dg_status dg_flags_after_coarsen(const dg_mesh* mc, const int8_t* flags, int8_t* flags_out) {
    if (!mc || !flags || !flags_out) return fail(DG_EINVAL, "NULL argument");
    const HostMesh& h = mc->h;
    const int64_t K = (int64_t)h.leaves.size();
    const int64_t Kp = mc->prev ? (int64_t)mc->prev->h.leaves.size() : K;
    for (int64_t e = 0; e < K; ++e) {
        const int32_t src = h.xfer_src[e];
        if (src < 0 || src >= Kp) return fail(DG_EINVAL, "transfer plan out of range");
        flags_out[e] = (h.xfer_kind[e] == DG_KIND_COPY && flags[src] > 0) ? 1 : 0;
    }
    return DG_OK;
}

dg_status dg_flags_buffer(const dg_mesh* m, int8_t* flags, int32_t B) {
    if (!m || !flags) return fail(DG_EINVAL, "NULL argument");
    if (B < 0) return fail(DG_EINVAL, "B must be >= 0");
    const HostMesh& h = m->h;
    const int64_t K = (int64_t)h.leaves.size();
    std::vector<int8_t> cur((size_t)K);
    for (int32_t round = 0; round < B; ++round) {
        std::memcpy(cur.data(), flags, (size_t)K);
        for (int64_t e = 0; e < K; ++e) {
            if (cur[(size_t)e] <= 0) continue;
            for (int f = 0; f < 6; ++f) {
                const int type = h.ftype[e * 6 + f] & 0xff;
                const int nnb = type == FT_WALL ? 0 : type == FT_COARSE ? 4 : 1;
                for (int q = 0; q < nnb; ++q) flags[h.fnb[(e * 6 + f) * 4 + q]] = 1;
            }
        }
    }
    return DG_OK;
}

dg_status dg_fma_burst(int32_t blocks, int32_t iters, double* sink, double* flops_out, void* stream) {
    if (blocks <= 0 || iters <= 0 || !sink || !flops_out) return fail(DG_EINVAL, "need blocks, iters > 0 and sink, flops_out");
    HIP_TRY(launch_fma_burst(blocks, iters, sink, (hipStream_t)stream));
    *flops_out = 2.0 * 8.0 * (double)iters * 256.0 * (double)blocks;
    return DG_OK;
}

dg_status dg_budgets(const dg_mesh* mc, const dg_phys* phys, const double* q, double* out_host, void* stream) {
    dg_status st = check_dev_mesh(mc, (hipStream_t)stream);
    if (st) return st;
    if ((st = check_phys(phys))) return st;
    if (!q || !out_host) return fail(DG_EINVAL, "NULL argument");
    dg_mesh* m = const_cast<dg_mesh*>(mc);
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_bg(m, phys, s))) return st;
    const int64_t K = (int64_t)m->h.leaves.size();
    const int nblk = budget_blocks(K);
    BudgetArgs a{q, m->d_bg, m->d_geo, m->h.sphere ? m->d_metric : nullptr, m->d_c1d,
                 m->d_ops + 5 * (m->h.desc.N + 1) * (m->h.desc.N + 1),
                 m->d_red, K, phys->cp / phys->cv, phys->g, binom_coef(phys)};
    double* out_dev = m->d_red + (int64_t)nblk * 8;
    HIP_TRY(launch_budgets(m->h.desc.N, a, nblk, out_dev, s));
    HIP_TRY(hipMemcpyAsync(out_host, out_dev, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(out_host[i])) return fail(DG_ENONFINITE, "non-finite budget");
    return DG_OK;
}

dg_status dg_budgets_noalloc(const dg_mesh* mc, const dg_phys* phys, const double* q, double* out_dev,
                             void* stream) {
    if (!mc) return fail(DG_EINVAL, "mesh is NULL");
    if (mc->h.desc.host_only) return fail(DG_EINVAL, "mesh was built host_only");
    // making the device tables allocates: this entry point only accepts a mesh that
    // already has them
    if (!mc->on_device)
        return fail(DG_EINVAL, "mesh has no device tables yet (any other field call on it makes them)");
    // the tables exist: this only orders the call after their upload (no allocation)
    dg_status st = check_dev_mesh(mc, (hipStream_t)stream);
    if (st) return st;
    st = check_phys(phys);
    if (st) return st;
    if (!q || !out_dev) return fail(DG_EINVAL, "NULL argument");
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != mc->device) return fail(DG_EINVAL, "the mesh's device must be the current device");
    dg_mesh* m = const_cast<dg_mesh*>(mc);
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_bg(m, phys, s))) return st;
    const int64_t K = (int64_t)m->h.leaves.size();
    const int nblk = budget_blocks(K);
    if ((int64_t)nblk * 8 > kBudgetScratchDoubles)
        return fail(DG_EINVAL, "budget partials exceed the static scratch (" +
                                   std::to_string(kBudgetScratchDoubles) + " doubles)");
    double* scr = nullptr;
    HIP_TRY(budget_scratch(&scr));
    BudgetArgs a{q, m->d_bg, m->d_geo, m->h.sphere ? m->d_metric : nullptr, m->d_c1d,
                 m->d_ops + 5 * (m->h.desc.N + 1) * (m->h.desc.N + 1),
                 scr, K, phys->cp / phys->cv, phys->g, binom_coef(phys)};
    HIP_TRY(launch_budgets(m->h.desc.N, a, nblk, out_dev, s));
    return DG_OK;
}

dg_status dg_indicator(const dg_mesh* mc, const dg_phys* phys, const double* q, int32_t kind, double thr,
                       double* eta, int8_t* flags_host, void* stream) {
    dg_status st = check_dev_mesh(mc, (hipStream_t)stream);
    if (st) return st;
    if ((st = check_phys(phys))) return st;
    if (!q || !flags_host) return fail(DG_EINVAL, "NULL argument");
    if (kind != DG_IND_THETA && kind != DG_IND_GRAD_THETA && kind != DG_IND_PPRIME)
        return fail(DG_EINVAL, "unknown indicator kind");
    if (mc->h.sphere && kind == DG_IND_GRAD_THETA)
        return fail(DG_EUNSUPPORTED, "the gradient indicator takes brick meshes");
    dg_mesh* m = const_cast<dg_mesh*>(mc);
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_bg(m, phys, s))) return st;
    const int64_t K = (int64_t)m->h.leaves.size();
    IndArgs a{q, m->d_bg, m->d_geo, m->d_ops, m->d_level, eta ? eta : m->d_eta, m->d_flags, K, kind,
              m->h.desc.max_level, thr, phys->cp / phys->cv, binom_coef(phys)};
    HIP_TRY(launch_indicator(m->h.desc.N, a, s));
    if (K > 0) HIP_TRY(hipMemcpyAsync(flags_host, m->d_flags, K, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return DG_OK;
}

dg_status dg_indicator_async(const dg_mesh* mc, const dg_phys* phys, const double* q, int32_t kind, double thr,
                             double* eta, int8_t* flags_dev, void* stream) {
    dg_status st = check_dev_mesh(mc, (hipStream_t)stream);
    if (st) return st;
    if ((st = check_phys(phys))) return st;
    if (!q || !flags_dev) return fail(DG_EINVAL, "NULL argument");
    if (kind != DG_IND_THETA && kind != DG_IND_GRAD_THETA && kind != DG_IND_PPRIME)
        return fail(DG_EINVAL, "unknown indicator kind");
    if (mc->h.sphere && kind == DG_IND_GRAD_THETA)
        return fail(DG_EUNSUPPORTED, "the gradient indicator takes brick meshes");
    dg_mesh* m = const_cast<dg_mesh*>(mc);
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_bg(m, phys, s))) return st;
    const int64_t K = (int64_t)m->h.leaves.size();
    IndArgs a{q, m->d_bg, m->d_geo, m->d_ops, m->d_level, eta ? eta : m->d_eta, flags_dev, K, kind,
              m->h.desc.max_level, thr, phys->cp / phys->cv, binom_coef(phys)};
    HIP_TRY(launch_indicator(m->h.desc.N, a, s));
    return DG_OK;
}

}  // extern "C"

// C-ABI implementation of the gfx950 D3Q19 + immersed-boundary library.
// Host side: argument checks, context buffers, kernel dispatch by precision.
#include "lbmibm.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ibm_kernels.hpp"
#include "lattice_kernels.hpp"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr uint32_t kMeshMagic = 0x1B3A0C5Du;

uint32_t mesh_tag(const ibm_mesh *m) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        h ^= v;
        h *= 1099511628211ull;
    };
    mix((uint64_t)m->ncells);
    mix((uint64_t)m->nverts);
    mix((uint64_t)m->ntris);
    mix((uint64_t)m->nedges);
    mix((uint64_t)(uintptr_t)m->x);
    mix((uint64_t)(uintptr_t)m->tri);
    mix((uint64_t)(uintptr_t)m->hinge);
    mix((uint64_t)(uintptr_t)m->vert_off);
    mix((uint64_t)(uintptr_t)m->vtri);
    mix((uint64_t)(uintptr_t)m->vedge);
    mix((uint64_t)m->max_cell_verts);
    return kMeshMagic ^ (uint32_t)(h ^ (h >> 32));
}

}  // namespace

struct lbm_ctx {
    lbm_params p;
    hipStream_t s;
    int64_t N, stride;
    int tpr, ntiles;
    size_t rsize;  // sizeof(real)
    uint8_t *cls = nullptr;
    uint32_t *links = nullptr;
    void *fibm = nullptr;        // [N] x 4 real: spread force accumulator
    void *ufield = nullptr;      // [N] x 4 real: fluid velocity of the marked nodes
    uint8_t *need = nullptr;     // [N] 1 = node under some IB stencil this step
    uint8_t *tneed = nullptr;    // [ntiles] 1 = tile holds a marked node
    uint32_t *tlist = nullptr;   // [ntiles] marked tiles, compacted
    uint32_t *tcount = nullptr;  // length of tlist
    // spreading workspace, allocated by the first ibm_rest_shape
    void *srec = nullptr;              // spread records, one per IB point of the largest mesh
    int64_t srec_cap = 0;
    uint32_t *owner = nullptr;         // [N] epoch of the last claim of each base node's slot
    void *cslot = nullptr;             // [N][8] x 4 real: corner contributions per base node
    uint8_t *role = nullptr;           // [N][8] slot flags read by the node gather
    uint32_t epoch = 0;                // ibm_couple calls so far
    bool off32 = false;          // every lattice buffer below 4 GiB
    double *partials = nullptr;
    int64_t nparts = 0;
    double *sums = nullptr;
    double *host_sums = nullptr;
    int cur = 0;  // 0: state in f_a, 1: in f_b
    int64_t steps = 0;
};

#define LBM_API extern "C" __attribute__((visibility("default")))

LBM_API const char *lbm_last_error(void) { return g_err.c_str(); }

LBM_API int64_t lbm_plane_stride(int64_t n, int32_t prec) {
    if (n <= 0) return 0;
    const int64_t es = prec == LBM_F64 ? 8 : 4;
    int64_t s = cdiv(n, 64) * 64;
    // keep consecutive planes off a common 64 KiB alignment
    if ((s * es) % 65536 == 0) s += 192;
    return s;
}

static int check_params(const lbm_params *p) {
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBM_EINVAL, "lattice size must be >= 1 (got %d %d %d)", p->nx, p->ny, p->nz);
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    if (N > (int64_t)INT32_MAX / 2) return fail(LBM_EINVAL, "lattice too large (%lld nodes)", (long long)N);
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_EINVAL, "tau must be finite and > 1/2 (got %g)", p->tau);
    for (int d = 0; d < 3; d++) {
        if (p->periodic[d] != 0 && p->periodic[d] != 1) return fail(LBM_EINVAL, "periodic[%d] must be 0 or 1", d);
        if (!std::isfinite(p->body_force[d])) return fail(LBM_EINVAL, "body_force[%d] is not finite", d);
    }
    if (p->prec != LBM_F64 && p->prec != LBM_F32 && p->prec != LBM_F32_DEV)
        return fail(LBM_EINVAL, "prec must be LBM_F64, LBM_F32 or LBM_F32_DEV (got %d)", p->prec);
    if (p->plane_stride != 0 && (p->plane_stride < N || p->plane_stride % 64 != 0))
        return fail(LBM_EINVAL, "plane_stride must be 0 or a multiple of 64 that is >= N");
    if (!p->solid || !p->f_a || !p->f_b) return fail(LBM_EINVAL, "solid, f_a and f_b must be non-NULL");
    if (p->f_a == p->f_b) return fail(LBM_EINVAL, "f_a and f_b must be distinct buffers");
    const size_t es = p->prec == LBM_F64 ? 8 : 4;
    if ((uintptr_t)p->f_a % 16 || (uintptr_t)p->f_b % 16) return fail(LBM_EINVAL, "f_a/f_b must be 16-byte aligned");
    if (p->gfield && (uintptr_t)p->gfield % es) return fail(LBM_EINVAL, "gfield is misaligned");
    return LBM_OK;
}

LBM_API int64_t lbm_workspace_bytes(const lbm_params *p) {
    if (check_params(p)) return -1;
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const int64_t es = p->prec == LBM_F64 ? 8 : 4;
    const int64_t tiles = cdiv(p->nx, 64) * (int64_t)p->ny * p->nz;
    return N + 4 * N + 8 * N * es + N + cdiv(tiles, 16) * 16 + 4 * tiles + 4 + cdiv(N, 256) * 32 + 32;
}

LBM_API int lbm_init(const lbm_params *p, lbm_ctx **out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (int rc = check_params(p)) return rc;
    lbm_ctx *c = new lbm_ctx();
    c->p = *p;
    c->s = (hipStream_t)p->stream;
    c->N = (int64_t)p->nx * p->ny * p->nz;
    c->stride = p->plane_stride ? p->plane_stride : lbm_plane_stride(c->N, p->prec);
    c->p.plane_stride = c->stride;
    c->tpr = (int)cdiv(p->nx, 64);
    c->ntiles = c->tpr * p->ny * p->nz;
    c->rsize = p->prec == LBM_F64 ? 8 : 4;
    c->nparts = cdiv(c->N, 256);
    c->off32 = 19 * c->stride * (int64_t)c->rsize < (int64_t(1) << 32);
    auto cleanup = [&](int rc) {
        lbm_destroy(c);
        return rc;
    };
    if (hipMalloc(&c->cls, c->N) != hipSuccess || hipMalloc(&c->links, 4 * c->N) != hipSuccess ||
        hipMalloc(&c->fibm, 4 * c->N * c->rsize) != hipSuccess ||
        hipMalloc(&c->ufield, 4 * c->N * c->rsize) != hipSuccess || hipMalloc(&c->need, c->N) != hipSuccess ||
        hipMalloc(&c->tneed, cdiv(c->ntiles, 16) * 16) != hipSuccess ||
        hipMalloc(&c->tlist, 4 * (size_t)c->ntiles) != hipSuccess || hipMalloc(&c->tcount, 4) != hipSuccess ||
        hipMalloc(&c->partials, c->nparts * 4 * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->sums, 4 * sizeof(double)) != hipSuccess ||
        hipHostMalloc(&c->host_sums, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(fail(LBM_ENOMEM, "device allocation of the context work buffers failed"));
    }
    Geometry g{p->nx, p->ny, p->nz, {p->periodic[0], p->periodic[1], p->periodic[2]}};
    const int nb = (int)cdiv(c->N, 256);
    k_classify<<<nb, 256, 0, c->s>>>(g, p->solid, c->cls, c->links);
    if (hipMemsetAsync(c->fibm, 0, 4 * c->N * c->rsize, c->s) != hipSuccess ||
        hipMemsetAsync(c->ufield, 0, 4 * c->N * c->rsize, c->s) != hipSuccess ||
        hipMemsetAsync(c->need, 0, c->N, c->s) != hipSuccess ||
        hipMemsetAsync(c->tneed, 0, cdiv(c->ntiles, 16) * 16, c->s) != hipSuccess ||
        hipMemsetAsync(c->tcount, 0, 4, c->s) != hipSuccess)
        return cleanup(fail(LBM_EHIP, "clearing the force accumulator failed"));
    for (void *f : {p->f_a, p->f_b}) {
        switch (p->prec) {
            case LBM_F64: k_rest<double, false><<<nb, 256, 0, c->s>>>((double *)f, c->stride, c->N); break;
            case LBM_F32: k_rest<float, false><<<nb, 256, 0, c->s>>>((float *)f, c->stride, c->N); break;
            default: k_rest<float, true><<<nb, 256, 0, c->s>>>((float *)f, c->stride, c->N); break;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cleanup(fail(LBM_EHIP, "init kernels: %s", hipGetErrorString(e)));
    *out = c;
    return LBM_OK;
}

LBM_API void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->s);
    if (c->cls) (void)hipFree(c->cls);
    if (c->links) (void)hipFree(c->links);
    if (c->fibm) (void)hipFree(c->fibm);
    if (c->ufield) (void)hipFree(c->ufield);
    if (c->need) (void)hipFree(c->need);
    if (c->tneed) (void)hipFree(c->tneed);
    if (c->tlist) (void)hipFree(c->tlist);
    if (c->tcount) (void)hipFree(c->tcount);
    if (c->srec) (void)hipFree(c->srec);
    if (c->owner) (void)hipFree(c->owner);
    if (c->cslot) (void)hipFree(c->cslot);
    if (c->role) (void)hipFree(c->role);
    if (c->partials) (void)hipFree(c->partials);
    if (c->sums) (void)hipFree(c->sums);
    if (c->host_sums) (void)hipHostFree(c->host_sums);
    delete c;
}

static const void *cur_f(const lbm_ctx *c) { return c->cur ? c->p.f_b : c->p.f_a; }
static void *nxt_f(const lbm_ctx *c) { return c->cur ? c->p.f_a : c->p.f_b; }

template <class S, class R, bool DEV>
static void launch_step(lbm_ctx *c, const StepArgs &a) {
    const int nb = (int)cdiv(c->ntiles, 4);
    if (c->off32) {
        if (c->p.gfield)
            k_collide_stream<S, R, DEV, true, uint32_t><<<nb, 256, 0, c->s>>>(a);
        else
            k_collide_stream<S, R, DEV, false, uint32_t><<<nb, 256, 0, c->s>>>(a);
    } else {
        if (c->p.gfield)
            k_collide_stream<S, R, DEV, true, int64_t><<<nb, 256, 0, c->s>>>(a);
        else
            k_collide_stream<S, R, DEV, false, int64_t><<<nb, 256, 0, c->s>>>(a);
    }
}

LBM_API int lbm_step(lbm_ctx *c, int32_t nsteps) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    StepArgs a{};
    a.stride = c->stride;
    a.cls = c->cls;
    a.links = c->links;
    a.fibm = c->fibm;
    a.need = c->need;
    a.tneed = c->tneed;
    a.gfield = c->p.gfield;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nz = c->p.nz;
    a.tpr = c->tpr;
    a.ntiles = c->ntiles;
    a.N = c->N;
    for (int d = 0; d < 3; d++) a.g[d] = c->p.body_force[d];
    a.omega = 1.0 / c->p.tau;
    a.kf = 1.0 - 0.5 / c->p.tau;
    for (int s = 0; s < nsteps; s++) {
        a.fa = cur_f(c);
        a.fb = nxt_f(c);
        switch (c->p.prec) {
            case LBM_F64: launch_step<double, double, false>(c, a); break;
            case LBM_F32: launch_step<float, float, false>(c, a); break;
            default: launch_step<float, float, true>(c, a); break;
        }
        c->cur ^= 1;
        c->steps++;
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

LBM_API int lbm_current(lbm_ctx *c, void **f_cur, int64_t *steps) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (f_cur) *f_cur = const_cast<void *>(cur_f(c));
    if (steps) *steps = c->steps;
    return LBM_OK;
}

template <class S, class R, bool DEV>
static void launch_moments(lbm_ctx *c, void *rho, void *u) {
    const int nb = (int)c->nparts;
    const R *G = static_cast<const R *>(c->p.gfield);
    const double *g = c->p.body_force;
    if (G)
        k_moments<S, R, DEV, true><<<nb, 256, 0, c->s>>>((const S *)cur_f(c), c->stride, c->cls, G, c->N, g[0], g[1],
                                                          g[2], (R *)rho, (R *)u, c->partials);
    else
        k_moments<S, R, DEV, false><<<nb, 256, 0, c->s>>>((const S *)cur_f(c), c->stride, c->cls, G, c->N, g[0],
                                                           g[1], g[2], (R *)rho, (R *)u, c->partials);
}

LBM_API int lbm_read_fields(lbm_ctx *c, void *rho, void *u, double *host_sums) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    const size_t es = c->rsize;
    if (((uintptr_t)rho % es) || ((uintptr_t)u % es)) return fail(LBM_EINVAL, "rho/u misaligned");
    switch (c->p.prec) {
        case LBM_F64: launch_moments<double, double, false>(c, rho, u); break;
        case LBM_F32: launch_moments<float, float, false>(c, rho, u); break;
        default: launch_moments<float, float, true>(c, rho, u); break;
    }
    HIPCHK(hipGetLastError());
    if (!host_sums) return LBM_OK;
    k_final_sum<<<1, 256, 0, c->s>>>(c->partials, c->nparts, c->sums);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->host_sums, c->sums, 4 * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    for (int k = 0; k < 4; k++) {
        host_sums[k] = c->host_sums[k];
        if (!std::isfinite(host_sums[k])) return fail(LBM_ENONFINITE, "global sum %d is not finite", k);
    }
    return LBM_OK;
}

LBM_API int lbm_store_f64(lbm_ctx *c, double *f64) {
    if (!c || !f64) return fail(LBM_EINVAL, "NULL argument");
    if ((uintptr_t)f64 % 8) return fail(LBM_EINVAL, "f64 misaligned");
    const int nb = (int)cdiv(c->N, 256);
    switch (c->p.prec) {
        case LBM_F64: k_store_f64<double, false><<<nb, 256, 0, c->s>>>((const double *)cur_f(c), c->stride, c->N, f64); break;
        case LBM_F32: k_store_f64<float, false><<<nb, 256, 0, c->s>>>((const float *)cur_f(c), c->stride, c->N, f64); break;
        default: k_store_f64<float, true><<<nb, 256, 0, c->s>>>((const float *)cur_f(c), c->stride, c->N, f64); break;
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

LBM_API int lbm_load_f64(lbm_ctx *c, const double *f64) {
    if (!c || !f64) return fail(LBM_EINVAL, "NULL argument");
    if ((uintptr_t)f64 % 8) return fail(LBM_EINVAL, "f64 misaligned");
    const int nb = (int)cdiv(c->N, 256);
    void *f = const_cast<void *>(cur_f(c));
    switch (c->p.prec) {
        case LBM_F64: k_load_f64<double, false><<<nb, 256, 0, c->s>>>((double *)f, c->stride, c->N, f64); break;
        case LBM_F32: k_load_f64<float, false><<<nb, 256, 0, c->s>>>((float *)f, c->stride, c->N, f64); break;
        default: k_load_f64<float, true><<<nb, 256, 0, c->s>>>((float *)f, c->stride, c->N, f64); break;
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// immersed boundary

static int check_mesh_ptrs(const ibm_mesh *m) {
    if (!m) return fail(LBM_EINVAL, "mesh is NULL");
    if (m->ncells < 1 || m->nverts < 1 || m->ntris < 1 || m->nedges < 1)
        return fail(LBM_EINVAL, "mesh counts must be >= 1");
    if (!m->vert_off || !m->tri_off || !m->edge_off || !m->tri || !m->hinge || !m->anchor || !m->x || !m->v ||
        !m->f_el || !m->moduli || !m->l0 || !m->a0 || !m->th0 || !m->a0c || !m->v0c || !m->avert || !m->vtri_off ||
        !m->vtri || !m->vedge_off || !m->vedge)
        return fail(LBM_EINVAL, "mesh has a NULL array");
    if (!(m->xi > 0) || !(m->mass > 0) || !(m->dt > 0) || !std::isfinite(m->xi) || !std::isfinite(m->mass) ||
        !std::isfinite(m->dt))
        return fail(LBM_EINVAL, "xi, mass and dt must be finite and > 0");
    return LBM_OK;
}

static constexpr size_t kMaxLds = 64 * 1024;

template <class R>
static void launch_membrane(lbm_ctx *c, const ibm_mesh *m, bool rest) {
    MembArgs a{};
    a.tcount = c->tcount;
    a.vtri_off = m->vtri_off;
    a.vtri = m->vtri;
    a.vedge_off = m->vedge_off;
    a.vedge = m->vedge;
    a.maxt = m->max_cell_tris;
    a.maxe = m->max_cell_edges;
    a.vert_off = m->vert_off;
    a.tri_off = m->tri_off;
    a.edge_off = m->edge_off;
    a.tri = m->tri;
    a.hinge = m->hinge;
    a.anchor = m->anchor;
    a.x = static_cast<const double *>(m->x);
    a.f_el = m->f_el;
    a.moduli = m->moduli;
    a.l0 = m->l0;
    a.a0 = m->a0;
    a.th0 = m->th0;
    a.a0c = m->a0c;
    a.v0c = m->v0c;
    a.avert = m->avert;
    a.ncells = m->ncells;
    a.nverts = m->nverts;
    a.ntris = m->ntris;
    a.nedges = m->nedges;
    a.maxv = m->max_cell_verts;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nz = c->p.nz;
    a.tpr = c->tpr;
    a.need = c->need;
    a.tneed = c->tneed;
    const size_t sm = membrane_lds_bytes<R>(m->max_cell_verts, m->max_cell_tris, m->max_cell_edges);
    if (rest)
        k_membrane<R, true><<<m->ncells, kMembThreads, sm, c->s>>>(a);
    else
        k_membrane<R, false><<<m->ncells, kMembThreads, sm, c->s>>>(a);
}

LBM_API int ibm_rest_shape(lbm_ctx *c, ibm_mesh *m) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (int rc = check_mesh_ptrs(m)) return rc;
    // read the topology back and check every index against its cell's range
    std::vector<int32_t> vo(m->ncells + 1), to(m->ncells + 1), eo(m->ncells + 1), tri(3 * (size_t)m->ntris),
        hin(4 * (size_t)m->nedges);
    HIPCHK(hipStreamSynchronize(c->s));
    HIPCHK(hipMemcpy(vo.data(), m->vert_off, vo.size() * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(to.data(), m->tri_off, to.size() * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(eo.data(), m->edge_off, eo.size() * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(tri.data(), m->tri, tri.size() * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hin.data(), m->hinge, hin.size() * 4, hipMemcpyDeviceToHost));
    if (vo[0] != 0 || to[0] != 0 || eo[0] != 0 || vo[m->ncells] != m->nverts || to[m->ncells] != m->ntris ||
        eo[m->ncells] != m->nedges)
        return fail(LBM_EINVAL, "offset arrays must start at 0 and end at the counts");
    int mv = 0, mt = 0, me = 0;
    for (int k = 0; k < m->ncells; k++) {
        const int nv = vo[k + 1] - vo[k], nt = to[k + 1] - to[k], ne = eo[k + 1] - eo[k];
        if (nv < 3 || nt < 1 || ne < 1) return fail(LBM_EINVAL, "cell %d is empty or degenerate", k);
        mv = std::max(mv, nv);
        mt = std::max(mt, nt);
        me = std::max(me, ne);
        for (int t = to[k]; t < to[k + 1]; t++)
            for (int j = 0; j < 3; j++) {
                const int v = tri[(size_t)j * m->ntris + t];
                if (v < vo[k] || v >= vo[k + 1])
                    return fail(LBM_EINVAL, "triangle %d of cell %d uses vertex %d outside the cell", t, k, v);
            }
        for (int e = eo[k]; e < eo[k + 1]; e++)
            for (int j = 0; j < 4; j++) {
                const int v = hin[(size_t)j * m->nedges + e];
                if (v < vo[k] || v >= vo[k + 1])
                    return fail(LBM_EINVAL, "edge %d of cell %d uses vertex %d outside the cell", e, k, v);
            }
    }
    const size_t lds = c->rsize == 8 ? membrane_lds_bytes<double>(mv, mt, me) : membrane_lds_bytes<float>(mv, mt, me);
    if (lds > kMaxLds)
        return fail(LBM_EINVAL, "a cell with %d vertices, %d triangles, %d edges does not fit one workgroup's LDS", mv,
                    mt, me);
    // per-vertex incidence lists, elements in increasing order (the force
    // pass sums over them in this order)
    {
        std::vector<int32_t> toff(m->nverts + 1, 0), eoff(m->nverts + 1, 0), tl(3 * (size_t)m->ntris),
            el(4 * (size_t)m->nedges);
        for (int t = 0; t < m->ntris; t++)
            for (int j = 0; j < 3; j++) toff[tri[(size_t)j * m->ntris + t] + 1]++;
        for (int e = 0; e < m->nedges; e++)
            for (int j = 0; j < 4; j++) eoff[hin[(size_t)j * m->nedges + e] + 1]++;
        for (int v = 0; v < m->nverts; v++) {
            toff[v + 1] += toff[v];
            eoff[v + 1] += eoff[v];
        }
        std::vector<int32_t> tf(toff.begin(), toff.end() - 1), ef(eoff.begin(), eoff.end() - 1);
        for (int t = 0; t < m->ntris; t++)
            for (int j = 0; j < 3; j++) tl[tf[tri[(size_t)j * m->ntris + t]]++] = 4 * t + j;
        for (int e = 0; e < m->nedges; e++)
            for (int j = 0; j < 4; j++) el[ef[hin[(size_t)j * m->nedges + e]]++] = 4 * e + j;
        if ((int64_t)m->ntris * 4 > INT32_MAX || (int64_t)m->nedges * 4 > INT32_MAX)
            return fail(LBM_EINVAL, "mesh too large for 32-bit incidence codes");
        HIPCHK(hipMemcpy(m->vtri_off, toff.data(), toff.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(m->vtri, tl.data(), tl.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(m->vedge_off, eoff.data(), eoff.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(m->vedge, el.data(), el.size() * 4, hipMemcpyHostToDevice));
    }
    m->max_cell_verts = mv;
    m->max_cell_tris = mt;
    m->max_cell_edges = me;
    if (mv > kSpreadMaxPoints) return fail(LBM_EINVAL, "a cell has %d vertices (at most %d)", mv, kSpreadMaxPoints);
    const int64_t need_rec = (int64_t)m->nverts * (c->rsize == 8 ? sizeof(SRec<double>) : sizeof(SRec<float>));
    if (need_rec > c->srec_cap) {
        if (c->srec) HIPCHK(hipFree(c->srec));
        c->srec = nullptr;
        c->srec_cap = 0;
        if (hipMalloc(&c->srec, need_rec) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_ENOMEM, "allocating spread records for %d points failed", m->nverts);
        }
        c->srec_cap = need_rec;
    }
    if (!c->owner) {
        if (hipMalloc(&c->owner, 4 * c->N) != hipSuccess || hipMalloc(&c->cslot, 8 * 4 * c->rsize * c->N) != hipSuccess ||
            hipMalloc(&c->role, 8 * c->N) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_ENOMEM, "allocating the spreading slots (%lld bytes) failed",
                        (long long)((12 + 32 * c->rsize) * c->N));
        }
        HIPCHK(hipMemsetAsync(c->owner, 0, 4 * c->N, c->s));
        HIPCHK(hipMemsetAsync(c->role, 0, 8 * c->N, c->s));
    }
    if (c->p.prec == LBM_F64)
        launch_membrane<double>(c, m, true);
    else
        launch_membrane<float>(c, m, true);
    HIPCHK(hipGetLastError());
    m->checked = mesh_tag(m);
    return LBM_OK;
}

static int waves_grid(const lbm_ctx *c) {
    // one wave per listed tile for lists up to a quarter of the lattice
    return (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(c->ntiles, 4 * 4), 16384));
}

template <class S, class R, bool DEV>
static void launch_node_velocity(lbm_ctx *c) {
    k_compact<<<(int)cdiv(c->ntiles, kCompactThreads * kCompactPerThread), kCompactThreads, 0, c->s>>>(
        c->tneed, c->ntiles, c->tlist, c->tcount);
    NodeVelArgs a{};
    a.f = cur_f(c);
    a.stride = c->stride;
    a.cls = c->cls;
    a.gfield = c->p.gfield;
    a.ufield = c->ufield;
    a.need = c->need;
    a.tlist = c->tlist;
    a.tcount = c->tcount;
    a.nx = c->p.nx;
    a.tpr = c->tpr;
    a.N = c->N;
    for (int d = 0; d < 3; d++) a.g[d] = c->p.body_force[d];
    if (c->p.gfield)
        k_node_velocity<S, R, DEV, true><<<waves_grid(c), 256, 0, c->s>>>(a);
    else
        k_node_velocity<S, R, DEV, false><<<waves_grid(c), 256, 0, c->s>>>(a);
}

template <class R>
static void launch_couple(lbm_ctx *c, const ibm_mesh *m) {
    CoupleArgs a{};
    a.ufield = c->ufield;
    a.srec = c->srec;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nz = c->p.nz;
    a.N = c->N;
    a.vert_off = m->vert_off;
    a.anchor = m->anchor;
    a.x = static_cast<double *>(m->x);
    a.v = m->v;
    a.f_el = m->f_el;
    a.avert = m->avert;
    a.ncells = m->ncells;
    a.nverts = m->nverts;
    a.xi = m->xi;
    a.dt_over_m = m->dt / m->mass;
    a.dt = m->dt;
    dim3 grid((unsigned)cdiv(m->max_cell_verts, 128), (unsigned)m->ncells);
    k_couple<R><<<grid, 128, 0, c->s>>>(a);
    SpreadArgs sp{};
    sp.vert_off = m->vert_off;
    sp.srec = c->srec;
    sp.owner = c->owner;
    sp.cslot = c->cslot;
    sp.role = c->role;
    sp.fibm = c->fibm;
    sp.epoch = c->epoch;
    sp.nx = c->p.nx;
    sp.ny = c->p.ny;
    sp.nz = c->p.nz;
    k_spread_cells<R><<<m->ncells, kSpreadThreads, 0, c->s>>>(sp);
    GatherArgs g{};
    g.tlist = c->tlist;
    g.tcount = c->tcount;
    g.role = c->role;
    g.cslot = c->cslot;
    g.need = c->need;
    g.fibm = c->fibm;
    g.nx = c->p.nx;
    g.ny = c->p.ny;
    g.nz = c->p.nz;
    g.tpr = c->tpr;
    k_gather_nodes<R><<<waves_grid(c), 256, 0, c->s>>>(g);
}

LBM_API int ibm_couple(lbm_ctx *c, const ibm_mesh *m) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (int rc = check_mesh_ptrs(m)) return rc;
    if (m->checked != mesh_tag(m)) return fail(LBM_ESTATE, "call ibm_rest_shape on this mesh first");
    if (++c->epoch == 0) {  // the claim epochs wrapped: forget every old claim
        HIPCHK(hipMemsetAsync(c->owner, 0, 4 * c->N, c->s));
        c->epoch = 1;
    }
    switch (c->p.prec) {
        case LBM_F64:
            launch_membrane<double>(c, m, false);
            launch_node_velocity<double, double, false>(c);
            launch_couple<double>(c, m);
            break;
        case LBM_F32:
            launch_membrane<float>(c, m, false);
            launch_node_velocity<float, float, false>(c);
            launch_couple<float>(c, m);
            break;
        default:
            launch_membrane<float>(c, m, false);
            launch_node_velocity<float, float, true>(c);
            launch_couple<float>(c, m);
            break;
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

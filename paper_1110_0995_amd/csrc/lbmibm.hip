// C-ABI implementation of the gfx950 D3Q19 + immersed-boundary library.
// Host side: argument checks, context buffers, channel tables, kernel
// dispatch by precision, and hipGraph capture of coupled steps.
#include "lbmibm.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "adjoint_kernels.hpp"
#include "contact_kernels.hpp"
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
constexpr int64_t kMaxNodes = (int64_t)INT32_MAX / 2;
constexpr int kMaxChannels = 65535;

struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void mix(uint64_t v) {
        h ^= v;
        h *= 1099511628211ull;
    }
    void mixd(double d) {
        uint64_t v;
        std::memcpy(&v, &d, 8);
        mix(v);
    }
    uint32_t fold() const { return (uint32_t)(h ^ (h >> 32)); }
};

// Identity of a mesh's topology and buffers (set by ibm_rest_shape).
uint32_t mesh_tag(const ibm_mesh *m) {
    Fnv f;
    f.mix((uint64_t)m->ncells);
    f.mix((uint64_t)m->nverts);
    f.mix((uint64_t)m->ntris);
    f.mix((uint64_t)m->nedges);
    f.mix((uint64_t)(uintptr_t)m->x);
    f.mix((uint64_t)(uintptr_t)m->tri);
    f.mix((uint64_t)(uintptr_t)m->hinge);
    f.mix((uint64_t)(uintptr_t)m->vert_off);
    f.mix((uint64_t)(uintptr_t)m->vtri);
    f.mix((uint64_t)(uintptr_t)m->vedge);
    f.mix((uint64_t)(uintptr_t)m->cell_chan);
    f.mix((uint64_t)(uintptr_t)m->contact);
    if (m->contact) {
        f.mix((uint64_t)m->contact->nspheres);
        f.mix((uint64_t)(uintptr_t)m->contact->spheres);
    }
    f.mix((uint64_t)m->max_cell_verts);
    return kMeshMagic ^ f.fold();
}

// Everything a captured coupled step bakes into its kernel arguments.
uint64_t mesh_launch_key(const ibm_mesh *m) {
    if (!m) return 0;
    Fnv f;
    f.mix(mesh_tag(m));
    const void *ptrs[] = {m->tri_off, m->edge_off, m->anchor, m->v,         m->f_el,  m->moduli,
                          m->l0,      m->a0,       m->th0,    m->a0c,       m->v0c,   m->avert,
                          m->vtri_off, m->vedge_off};
    for (const void *p : ptrs) f.mix((uint64_t)(uintptr_t)p);
    f.mixd(m->xi);
    f.mixd(m->mass);
    f.mixd(m->dt);
    f.mix((uint64_t)m->stretch_law);
    if (const ibm_contact *k = m->contact) {
        for (double v : {k->a, k->n, k->rcut, k->roff, k->dmin}) f.mixd(v);
        f.mix((uint64_t)k->cell_cell);
        f.mix((uint64_t)k->nplanes);
        f.mix((uint64_t)k->ncyl);
        for (const void *p : {(const void *)k->planes, (const void *)k->cyl, (const void *)k->cyl_off,
                              (const void *)k->spheres})
            f.mix((uint64_t)(uintptr_t)p);
        f.mix((uint64_t)k->nspheres);
    }
    f.mix((uint64_t)m->max_cell_tris);
    f.mix((uint64_t)m->max_cell_edges);
    return f.h | 1ull;
}

}  // namespace

struct lbm_ctx {
    lbm_params p;
    hipStream_t s = nullptr;
    int nch = 1;
    std::vector<Chan> hchans;
    Chan *chans = nullptr;          // device copy of hchans
    uint16_t *tile_chan = nullptr;  // [ntiles] channel of each tile, null for one channel
    uint32_t *wgtab = nullptr;      // [nwg] collide-stream workgroups: first tile << 3 | (tiles - 1)
    int nwg = 0;
    int64_t N = 0, stride = 0;
    int ntiles = 0;
    size_t rsize = 4;  // sizeof(real)
    uint8_t *cls = nullptr;
    uint4 *tmask = nullptr;      // [ntiles] solid and wall masks of each tile
    uint2 *tnmask = nullptr;     // [ntiles] marks of each marked tile as a mask, from the velocity pass
    uint32_t *links = nullptr;
    void *fibm = nullptr;        // [N] x 4 real: spread force of the step, valid at the nodes marked this step
    void *facc = nullptr;        // [N] x 4 real: accumulator of the atomic fallback spread, zero between steps
    void *ufield = nullptr;      // [N] x 4 real: fluid velocity of the marked nodes
    uint8_t *need = nullptr;     // [N] 1 = node under some IB stencil this step
    uint8_t *tneed = nullptr;    // [ntiles] 1 = tile holds a marked node
    uint32_t *tlist = nullptr;   // [ntiles] marked tiles, compacted
    uint32_t *tcount = nullptr;  // length of tlist
    uint8_t *ftile = nullptr;    // [ntiles] 1 = the spread fell back to atomics in this tile
    uint32_t *epoch = nullptr;   // spreading-claim epoch, advanced on the device by each coupled step
    // spreading workspace, allocated by the first ibm_rest_shape
    void *srec = nullptr;        // spread records, one per IB point of the largest mesh
    int64_t srec_cap = 0;
    uint32_t *owner = nullptr;   // [N] epoch of the last spreading claim of each node
    bool off32 = false;          // every lattice buffer below 4 GiB
    double *partials = nullptr;
    int64_t nparts = 0;
    double *sums = nullptr;
    double *host_sums = nullptr;
    // non-finite populations: the collide-stream pass sets *nf_dev (sticky);
    // lbm_run ends by queueing its copy into pinned *nf_host (ev_nf after
    // the last one), which later lbm_run / lbm_step calls read without
    // waiting: a copy still in flight only delays the report
    uint32_t *nf_dev = nullptr;
    uint32_t *nf_host = nullptr;
    hipEvent_t ev_nf = nullptr;
    bool nf_pending = false;  // a copy may still be in flight
    int cur = 0;  // 0: state in f_a, 1: in f_b
    int64_t steps = 0;
    // launch shape
    int cs_waves = 0;     // tiles (waves) per collide-stream workgroup; 0 = by the lattice (cs_shape)
    int list_blocks = 0;  // workgroups of the tile-list kernels (0: by lattice size)
    // contact work buffers, allocated by ibm_rest_shape for a mesh with cell-cell contact
    double *bounds = nullptr;    // [ncells][4] centroid and radius
    int2 *pairs = nullptr;       // cell pairs in contact range
    uint32_t *npairs = nullptr;  // their number this step
    int bounds_cap = 0, pair_cap = 0;
    int couples = 0;  // membranes coupled since the last collide-stream pass
    int acc = 0;      // the membrane being coupled adds to the force of an earlier one
    // uniform grid of the fixed contact spheres, built by ibm_rest_shape
    int32_t *sph_start = nullptr;  // [cells + 1]
    int32_t *sph_items = nullptr;  // [nspheres] sphere ids, by cell
    int sph_cap_cells = 0, sph_cap_items = 0;
    const double *sph_src = nullptr;  // the spheres the grid was built from
    int sph_n = 0;
    int sph_g[3] = {1, 1, 1};
    double sph_inv[3] = {0.0, 0.0, 0.0};
    // adjoint work buffers, allocated by the first lbm_adjoint_step
    void *lamF = nullptr;  // [N] x 4 real: lambda of the node force at stencil nodes
    void *lamU = nullptr;  // [N] x 4 real: lambda of u_ext at stencil nodes (kept zero between calls)
    int64_t adj_nv = 0;    // IB points the scratch below holds
    double *xs = nullptr;  // [3][nv] positions advanced by the recomputed forward step
    void *vs = nullptr;    // [3][nv] real velocities, likewise
    void *fels = nullptr;  // [3][nv] real elastic forces, likewise
    double *hv = nullptr;  // [3][nv] membrane Jacobian times direction
    // second stream of a coupled step: the membrane forces run on it beside
    // the compaction and velocity passes; ev_fork / ev_join order the two
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // lbm_step_timed: events the next collide-stream launch binds to its own
    // start and end (null otherwise)
    hipEvent_t t_start = nullptr, t_stop = nullptr;
    int ibm_overlap = -1;  // lbm_set_ibm_overlap mode
    // records of the next step's stencil-node populations (see k_next_list):
    // the point update marks the new positions' stencils, the collide-stream
    // pass copies the populations it streams into them, and the next
    // coupling takes the marked nodes' velocities from the copies
    bool rec_capable = false;      // every channel's nx is a multiple of 64
    int rec_mode = 0;              // lbm_set_node_records
    bool rec_valid = false;        // the last pass recorded the nodes marked before it, from the current state
    bool u_from_rec = false;       // this step's velocities already come from the records
    bool last_rec = false;         // the last coupling took its velocities from the records
    int64_t nx_pending = 0;        // IB points whose next stencils were marked since the last pass
    int64_t nx_pts = 0;            // IB points of the meshes given to ibm_rest_shape (sizes the record)
    int64_t nx_cap = 0;            // record slots
    uint8_t *nx_need = nullptr;    // [N] next-step node marks
    uint8_t *nx_tneed = nullptr;   // [ntiles] next-step tile marks
    uint4 *nx_ent = nullptr;       // [ntiles] RecTile: recorded nodes of each tile, first slot
    uint32_t *nx_flags = nullptr;  // [0] slots handed out, [1] a marked node was not recorded
    uint32_t *nx_node = nullptr;   // [nx_cap] node of each slot
    void *nx_rec = nullptr;        // [19][nx_cap] storage type
    // captured graphs: plain coupled steps, recorded steps, reverse sweep
    hipStream_t cap_s = nullptr;
    hipGraphExec_t gx[3] = {nullptr, nullptr, nullptr};
    uint64_t gk[3] = {0, 0, 0};
    bool g_rec_end[3] = {false, false, false};  // rec_valid after each graph
};

enum { G_RUN = 0, G_REC = 1, G_ADJ = 2 };

#define LBM_API extern "C" __attribute__((visibility("default")))

static void drop_graph(lbm_ctx *c) {
    for (int k = 0; k < 3; k++) {
        if (c->gx[k]) (void)hipGraphExecDestroy(c->gx[k]);
        c->gx[k] = nullptr;
        c->gk[k] = 0;
    }
}

LBM_API const char *lbm_last_error(void) { return g_err.c_str(); }

// the error slot shared with the magnetic-stage entry points
namespace lbm {
void set_error(const char *msg) { g_err = msg; }
}  // namespace lbm

LBM_API int64_t lbm_plane_stride(int64_t n, int32_t prec) {
    if (n <= 0) return 0;
    const int64_t es = prec == LBM_F64 ? 8 : 4;
    int64_t s = cdiv(n, 64) * 64;
    // keep consecutive planes off a common 64 KiB alignment
    if ((s * es) % 65536 == 0) s += 192;
    return s;
}

// Checks shared by both init calls; N is the node count of all channels.
static int check_common(const lbm_params *p, int64_t N) {
    if (N > kMaxNodes) return fail(LBM_EINVAL, "lattice too large (%lld nodes)", (long long)N);
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

static int check_params(const lbm_params *p) {
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(LBM_EINVAL, "lattice size must be >= 1 (got %d %d %d)", p->nx, p->ny, p->nz);
    return check_common(p, (int64_t)p->nx * p->ny * p->nz);
}

// Channel table of dims [nch][3]; fails on sizes below 1 or too many nodes.
static int make_channels(int32_t nch, const int32_t *dims, std::vector<Chan> &out, int64_t &N, int64_t &T) {
    out.clear();
    N = 0;
    T = 0;
    for (int k = 0; k < nch; k++) {
        const int nx = dims[3 * k], ny = dims[3 * k + 1], nz = dims[3 * k + 2];
        if (nx < 1 || ny < 1 || nz < 1)
            return fail(LBM_EINVAL, "channel %d size must be >= 1 (got %d %d %d)", k, nx, ny, nz);
        const Chan ch{nx, ny, nz, (int)cdiv(nx, 64), N, (int)T, 0};
        out.push_back(ch);
        N += (int64_t)nx * ny * nz;
        T += (int64_t)ch.tpr * ny * nz;
        if (N > kMaxNodes) return fail(LBM_EINVAL, "lattice too large (more than %lld nodes)", (long long)kMaxNodes);
    }
    return LBM_OK;
}

// Collide-stream workgroups of whole x rows: a channel whose rows are at
// most 8 tiles gets workgroups of floor(8 / tiles per row) rows (the last
// one of the channel may hold fewer); a longer row is cut into pieces of 8
// tiles.  A workgroup never spans two channels.  Entry: first tile << 3 |
// (tiles - 1).
static int64_t row_groups(int tpr, int64_t rows) {
    return tpr <= 8 ? cdiv(rows, 8 / tpr) : rows * cdiv(tpr, 8);
}
static void build_row_groups(const std::vector<Chan> &chs, std::vector<uint32_t> &tab) {
    tab.clear();
    for (const Chan &ch : chs) {
        const int64_t rows = (int64_t)ch.ny * ch.nz;
        if (ch.tpr <= 8) {
            const int rpw = 8 / ch.tpr;
            for (int64_t r0 = 0; r0 < rows; r0 += rpw) {
                const int64_t nr = std::min<int64_t>(rpw, rows - r0);
                tab.push_back((uint32_t)((ch.toff + r0 * ch.tpr) << 3) | (uint32_t)(nr * ch.tpr - 1));
            }
        } else {
            for (int64_t r = 0; r < rows; r++)
                for (int c0 = 0; c0 < ch.tpr; c0 += 8)
                    tab.push_back((uint32_t)((ch.toff + r * ch.tpr + c0) << 3) | (uint32_t)(std::min(8, ch.tpr - c0) - 1));
        }
    }
}

static int64_t workspace(int64_t N, int64_t tiles, int64_t es, int nch, int64_t nwg) {
    // workgroup table, classes, links, three 4-vector fields, node marks, tile
    // marks and fallback tile flags, tile list, solid/wall and stencil-node
    // masks per tile, counters, partial sums, channels
    return 4 * nwg + N + 4 * N + 12 * N * es + N + 2 * cdiv(tiles, 16) * 16 + 4 * tiles + 16 * tiles + 8 * tiles + 4 +
           4 + cdiv(N, 256) * 32 + 32 + (int64_t)nch * (int64_t)sizeof(Chan) + (nch > 1 ? 2 * tiles : 0);
}

LBM_API int64_t lbm_workspace_bytes(const lbm_params *p) {
    if (check_params(p)) return -1;
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const int tpr = (int)cdiv(p->nx, 64);
    return workspace(N, tpr * (int64_t)p->ny * p->nz, p->prec == LBM_F64 ? 8 : 4, 1,
                     row_groups(tpr, (int64_t)p->ny * p->nz));
}

LBM_API int64_t lbm_workspace_bytes_channels(const lbm_params *p, int32_t nch, const int32_t *dims) {
    if (!p || !dims || nch < 1 || nch > kMaxChannels) return -1;
    std::vector<Chan> chs;
    int64_t N, T;
    if (make_channels(nch, dims, chs, N, T) || check_common(p, N)) return -1;
    int64_t nwg = 0;
    for (const Chan &ch : chs) nwg += row_groups(ch.tpr, (int64_t)ch.ny * ch.nz);
    return workspace(N, T, p->prec == LBM_F64 ? 8 : 4, nch, nwg);
}

LBM_API void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->s);
    if (c->cap_s) (void)hipStreamSynchronize(c->cap_s);
    if (c->side) (void)hipStreamSynchronize(c->side);
    drop_graph(c);
    if (c->cap_s) (void)hipStreamDestroy(c->cap_s);
    if (c->side) (void)hipStreamDestroy(c->side);
    for (hipEvent_t e : {c->ev_fork, c->ev_join, c->ev_nf})
        if (e) (void)hipEventDestroy(e);
    void *bufs[] = {c->chans, c->tile_chan, c->cls,  c->tmask, c->tnmask, c->links, c->fibm, c->facc, c->ufield, c->need, c->tneed, c->tlist,
                    c->tcount, c->epoch,    c->srec, c->owner, c->partials, c->sums, c->ftile,
                    c->lamF,  c->lamU,      c->xs,   c->vs,    c->fels,  c->hv, c->bounds, c->pairs, c->npairs,
                    c->sph_start, c->sph_items, c->wgtab, c->nx_need, c->nx_tneed, c->nx_ent,
                    c->nx_flags, c->nx_node, c->nx_rec, c->nf_dev};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (c->host_sums) (void)hipHostFree(c->host_sums);
    if (c->nf_host) (void)hipHostFree(c->nf_host);
    delete c;
}

// Allocate the work buffers for the channels in c->hchans, classify the
// nodes and set both state buffers to rest.
static int init_ctx(lbm_ctx *c) {
    const lbm_params *p = &c->p;
    c->s = (hipStream_t)p->stream;
    c->stride = p->plane_stride ? p->plane_stride : lbm_plane_stride(c->N, p->prec);
    c->p.plane_stride = c->stride;
    c->rsize = p->prec == LBM_F64 ? 8 : 4;
    c->nparts = cdiv(c->N, 256);
    c->off32 = 19 * c->stride * (int64_t)c->rsize < (int64_t(1) << 32);
    c->nch = (int)c->hchans.size();
    c->rec_capable = true;
    for (const Chan &ch : c->hchans) c->rec_capable = c->rec_capable && ch.nx % 64 == 0;
    const size_t tn = (size_t)c->ntiles;
    const size_t tpad = (size_t)cdiv((int64_t)tn, 16) * 16;
    if (hipMalloc(&c->chans, sizeof(Chan) * c->nch) != hipSuccess || hipMalloc(&c->cls, c->N) != hipSuccess ||
        hipMalloc(&c->tmask, sizeof(uint4) * tn) != hipSuccess || hipMalloc(&c->tnmask, sizeof(uint2) * tn) != hipSuccess ||
        hipMalloc(&c->links, 4 * c->N) != hipSuccess || hipMalloc(&c->fibm, 4 * c->N * c->rsize) != hipSuccess ||
        hipMalloc(&c->facc, 4 * c->N * c->rsize) != hipSuccess ||
        hipMalloc(&c->ufield, 4 * c->N * c->rsize) != hipSuccess || hipMalloc(&c->need, c->N) != hipSuccess ||
        hipMalloc(&c->tneed, tpad) != hipSuccess || hipMalloc(&c->tlist, 4 * tn) != hipSuccess ||
        hipMalloc(&c->tcount, 4) != hipSuccess || hipMalloc(&c->epoch, 4) != hipSuccess ||
        hipMalloc(&c->ftile, tpad) != hipSuccess ||
        hipMalloc(&c->partials, c->nparts * 4 * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->sums, 4 * sizeof(double)) != hipSuccess || hipMalloc(&c->nf_dev, 4) != hipSuccess ||
        (c->nch > 1 && hipMalloc(&c->tile_chan, 2 * tn) != hipSuccess) ||
        hipHostMalloc(&c->host_sums, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&c->nf_host, 4, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBM_ENOMEM, "device allocation of the context work buffers failed");
    }
    HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_nf, hipEventDisableTiming));
    *c->nf_host = 0;
    HIPCHK(hipMemcpy(c->chans, c->hchans.data(), sizeof(Chan) * c->nch, hipMemcpyHostToDevice));
    {
        std::vector<uint32_t> tab;
        build_row_groups(c->hchans, tab);
        c->nwg = (int)tab.size();
        if (hipMalloc(&c->wgtab, 4 * tab.size()) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_ENOMEM, "device allocation of the workgroup table failed");
        }
        HIPCHK(hipMemcpy(c->wgtab, tab.data(), 4 * tab.size(), hipMemcpyHostToDevice));
    }
    if (c->nch > 1) {
        std::vector<uint16_t> tc(tn);
        for (int k = 0; k < c->nch; k++) {
            const Chan &ch = c->hchans[k];
            const int nt = ch.tpr * ch.ny * ch.nz;
            std::fill(tc.begin() + ch.toff, tc.begin() + ch.toff + nt, (uint16_t)k);
        }
        HIPCHK(hipMemcpy(c->tile_chan, tc.data(), 2 * tn, hipMemcpyHostToDevice));
    }
    k_classify<<<(int)cdiv(c->ntiles, 4), 256, 0, c->s>>>(c->chans, c->tile_chan, c->ntiles, p->periodic[0],
                                                           p->periodic[1], p->periodic[2], p->solid, c->cls, c->links, c->tmask);
    HIPCHK(hipMemsetAsync(c->fibm, 0, 4 * c->N * c->rsize, c->s));
    HIPCHK(hipMemsetAsync(c->facc, 0, 4 * c->N * c->rsize, c->s));
    HIPCHK(hipMemsetAsync(c->ufield, 0, 4 * c->N * c->rsize, c->s));
    HIPCHK(hipMemsetAsync(c->need, 0, c->N, c->s));
    HIPCHK(hipMemsetAsync(c->tneed, 0, tpad, c->s));
    HIPCHK(hipMemsetAsync(c->tnmask, 0, sizeof(uint2) * tn, c->s));
    HIPCHK(hipMemsetAsync(c->ftile, 0, tpad, c->s));
    HIPCHK(hipMemsetAsync(c->tcount, 0, 4, c->s));
    HIPCHK(hipMemsetAsync(c->epoch, 0, 4, c->s));
    HIPCHK(hipMemsetAsync(c->nf_dev, 0, 4, c->s));
    const int nb = (int)cdiv(c->N, 256);
    for (void *f : {p->f_a, p->f_b}) {
        switch (p->prec) {
            case LBM_F64: k_rest<double, false><<<nb, 256, 0, c->s>>>((double *)f, c->stride, c->N); break;
            case LBM_F32: k_rest<float, false><<<nb, 256, 0, c->s>>>((float *)f, c->stride, c->N); break;
            default: k_rest<float, true><<<nb, 256, 0, c->s>>>((float *)f, c->stride, c->N); break;
        }
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

static int finish_init(lbm_ctx *c, lbm_ctx **out) {
    if (int rc = init_ctx(c)) {
        lbm_destroy(c);
        return rc;
    }
    *out = c;
    return LBM_OK;
}

LBM_API int lbm_init(const lbm_params *p, lbm_ctx **out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (int rc = check_params(p)) return rc;
    lbm_ctx *c = new lbm_ctx();
    c->p = *p;
    const int32_t dims[3] = {p->nx, p->ny, p->nz};
    int64_t T;
    make_channels(1, dims, c->hchans, c->N, T);
    c->ntiles = (int)T;
    return finish_init(c, out);
}

LBM_API int lbm_init_channels(const lbm_params *p, int32_t nch, const int32_t *dims, lbm_ctx **out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (nch < 1 || nch > kMaxChannels) return fail(LBM_EINVAL, "nch must be in [1, %d] (got %d)", kMaxChannels, nch);
    if (!dims) return fail(LBM_EINVAL, "dims is NULL");
    std::vector<Chan> chs;
    int64_t N, T;
    if (int rc = make_channels(nch, dims, chs, N, T)) return rc;
    if (int rc = check_common(p, N)) return rc;
    lbm_ctx *c = new lbm_ctx();
    c->p = *p;
    c->hchans = chs;
    c->N = N;
    c->ntiles = (int)T;
    return finish_init(c, out);
}

LBM_API int lbm_set_launch(lbm_ctx *c, int32_t collide_waves_per_block, int32_t list_blocks) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    const int w = collide_waves_per_block;
    if (w != 0 && w != 1 && w != 2 && w != 4 && w != 8)
        return fail(LBM_EINVAL, "collide_waves_per_block must be 0, 1, 2, 4 or 8 (got %d)", w);
    if (list_blocks < 0 || list_blocks > 65536) return fail(LBM_EINVAL, "list_blocks must be in [0, 65536]");
    c->cs_waves = w;
    c->list_blocks = list_blocks;
    drop_graph(c);  // a captured graph holds the old launch shape
    return LBM_OK;
}

LBM_API int lbm_set_ibm_overlap(lbm_ctx *c, int32_t mode) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (mode < -1 || mode > 1) return fail(LBM_EINVAL, "overlap mode must be -1, 0 or 1 (got %d)", mode);
    if (mode != c->ibm_overlap) drop_graph(c);
    c->ibm_overlap = mode;
    return LBM_OK;
}

LBM_API int lbm_set_node_records(lbm_ctx *c, int32_t mode) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (mode != 0 && mode != 1) return fail(LBM_EINVAL, "node-record mode must be 0 or 1 (got %d)", mode);
    if (mode != c->rec_mode) {
        drop_graph(c);
        c->rec_valid = false;
        c->u_from_rec = false;
    }
    c->rec_mode = mode;
    return LBM_OK;
}

LBM_API int lbm_node_records_used(lbm_ctx *c, int32_t *used, int32_t *missed) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    uint32_t miss = 0;
    if (c->last_rec && c->nx_flags) {
        HIPCHK(hipStreamSynchronize(c->s));
        HIPCHK(hipMemcpy(&miss, c->nx_flags + 1, 4, hipMemcpyDeviceToHost));
    }
    if (used) *used = c->last_rec ? 1 : 0;
    if (missed) *missed = miss ? 1 : 0;
    return LBM_OK;
}

static const void *cur_f(const lbm_ctx *c) { return c->cur ? c->p.f_b : c->p.f_a; }
static void *nxt_f(const lbm_ctx *c) { return c->cur ? c->p.f_a : c->p.f_b; }

// Workgroup shape of the collide-stream passes.  By default (cs_waves = 0)
// workgroups of 8 waves take the row groups of the workgroup table (whole x
// rows of one channel, as many as fit in 8 tiles; pieces of 8 tiles of a
// longer row) in natural order.  An explicit shape (lbm_set_launch) cuts
// the tile range into equal workgroups, renumbered by XCD unless they hold
// whole rows of a one-channel lattice.
struct CsShape {
    int waves, remap, nb;
    const uint32_t *tab;
};
static CsShape cs_shape(const lbm_ctx *c) {
    if (c->cs_waves == 0) return {8, 0, c->nwg, c->wgtab};
    const int tpr = c->nch == 1 ? c->hchans[0].tpr : 0;
    return {c->cs_waves, (tpr >= 1 && c->cs_waves % tpr == 0) ? 0 : 1, (int)cdiv(c->ntiles, c->cs_waves), nullptr};
}

template <class S, class R, bool DEV, bool HAS_G, class IDX, bool EMIT>
static void launch_cs(lbm_ctx *c, const StepArgs &a, int nb, int bs) {
    if (c->t_start)  // the events take the kernel's own start and end
        hipExtLaunchKernelGGL(k_collide_stream<S, R, DEV, HAS_G, IDX, EMIT>, dim3(nb), dim3(bs), 0, c->s, c->t_start,
                              c->t_stop, 0u, a);
    else
        k_collide_stream<S, R, DEV, HAS_G, IDX, EMIT><<<nb, bs, 0, c->s>>>(a);
}

template <class S, class R, bool DEV, bool EMIT>
static void launch_step_as(lbm_ctx *c, const StepArgs &a, int nb, int bs) {
    if (c->off32) {
        if (c->p.gfield)
            launch_cs<S, R, DEV, true, uint32_t, EMIT>(c, a, nb, bs);
        else
            launch_cs<S, R, DEV, false, uint32_t, EMIT>(c, a, nb, bs);
    } else {
        if (c->p.gfield)
            launch_cs<S, R, DEV, true, int64_t, EMIT>(c, a, nb, bs);
        else
            launch_cs<S, R, DEV, false, int64_t, EMIT>(c, a, nb, bs);
    }
}

template <class S, class R, bool DEV>
static void launch_step(lbm_ctx *c, StepArgs a) {
    const CsShape sh = cs_shape(c);
    a.remap = sh.remap;
    a.wgtab = sh.tab;
    a.reverse = (int)(c->steps & 1);  // every other pass walks the table backwards
    if (a.erec)
        launch_step_as<S, R, DEV, true>(c, a, sh.nb, 64 * sh.waves);
    else
        launch_step_as<S, R, DEV, false>(c, a, sh.nb, 64 * sh.waves);
}

static void enqueue_copy(lbm_ctx *c, void *dst, const void *src, size_t bytes) {
    const uintptr_t al = (uintptr_t)dst | (uintptr_t)src | (uintptr_t)bytes;
    auto go = [&](auto tag) {
        using T = decltype(tag);
        const int64_t n = (int64_t)(bytes / sizeof(T));
        const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 16384));
        k_copy<T><<<nb, 256, 0, c->s>>>(static_cast<const T *>(src), static_cast<T *>(dst), n);
    };
    if (al % 16 == 0)
        go(uint4{});
    else if (al % 8 == 0)
        go(uint2{});
    else
        go(uint32_t{});
}

static StepArgs step_args(const lbm_ctx *c) {
    StepArgs a{};
    a.stride = c->stride;
    a.tmask = c->tmask;
    a.links = c->links;
    a.fibm = c->fibm;
    a.facc = c->facc;
    a.ftile = c->ftile;
    a.need = c->need;
    a.tneed = c->tneed;
    a.gfield = c->p.gfield;
    a.chans = c->chans;
    a.tile_chan = c->tile_chan;
    a.ntiles = c->ntiles;
    a.N = c->N;
    for (int d = 0; d < 3; d++) a.g[d] = c->p.body_force[d];
    a.omega = 1.0 / c->p.tau;
    a.kf = 1.0 - 0.5 / c->p.tau;
    for (int d = 0; d < 3; d++) a.per[d] = c->p.periodic[d];
    a.nonfinite = c->nf_dev;
    return a;
}

// LBM_ENONFINITE once a copy of the flag queued by an earlier lbm_run has
// landed with it set; never waits (the flag only goes from 0 to 1 between
// resets, so a stale read just reports later).
static int nonfinite_reported(lbm_ctx *c) {
    if (__atomic_load_n(c->nf_host, __ATOMIC_ACQUIRE))
        return fail(LBM_ENONFINITE, "a collide-stream pass met non-finite populations (state is lost)");
    return LBM_OK;
}

// Queue the copy of the device flag that nonfinite_reported reads later.
static int queue_nonfinite_copy(lbm_ctx *c) {
    HIPCHK(hipMemcpyAsync(c->nf_host, c->nf_dev, 4, hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipEventRecord(c->ev_nf, c->s));
    c->nf_pending = true;
    return LBM_OK;
}

// Clear the flag and its host copy (no copy left in flight to undo it).
static int reset_nonfinite(lbm_ctx *c) {
    if (c->nf_pending) HIPCHK(hipEventSynchronize(c->ev_nf));
    c->nf_pending = false;
    __atomic_store_n(c->nf_host, 0u, __ATOMIC_RELEASE);
    HIPCHK(hipMemsetAsync(c->nf_dev, 0, 4, c->s));
    return LBM_OK;
}

static PopView pop_view(const lbm_ctx *c) {
    PopView v{};
    v.chans = c->chans;
    v.nch = c->nch;
    for (int d = 0; d < 3; d++) v.per[d] = c->p.periodic[d];
    v.cls = c->cls;
    v.links = c->links;
    return v;
}

// One collide-stream pass from fa into fb (the context's parity is untouched).
// With `plain` (a pass of the context's own state, fb becoming the current
// buffer) the populations streamed into nodes marked for the next step are
// recorded, when any were marked since the last pass.
static void enqueue_step_into(lbm_ctx *c, const void *fa, void *fb, bool plain = false) {
    c->couples = 0;  // this pass consumes the spread force
    StepArgs a = step_args(c);
    a.fa = fa;
    a.fb = fb;
    const bool emit = plain && c->nx_pending > 0 && c->nx_rec;
    if (emit) {
        NextListArgs l{};
        l.nx_need = c->nx_need;
        l.nx_tneed = c->nx_tneed;
        l.ent = c->nx_ent;
        l.node = c->nx_node;
        l.count = c->nx_flags;
        l.miss = c->nx_flags + 1;
        l.chans = c->chans;
        l.tile_chan = c->tile_chan;
        l.ntiles = c->ntiles;
        l.cap = c->nx_cap;
        k_next_list<<<(int)cdiv(c->ntiles, kNextListThreads * kNextListPer), kNextListThreads, 0, c->s>>>(l);
        a.etile = c->nx_ent;
        a.erec = c->nx_rec;
        a.ecap = c->nx_cap;
    }
    // the velocity pass left the marks of every marked tile as masks unless
    // a coupling of this step took its velocities from the records
    a.tnmask = c->tnmask;
    a.use_tnmask = c->u_from_rec ? 0 : 1;
    c->rec_valid = emit;
    c->u_from_rec = false;
    c->nx_pending = 0;
    switch (c->p.prec) {
        case LBM_F64: launch_step<double, double, false>(c, a); break;
        case LBM_F32: launch_step<float, float, false>(c, a); break;
        default: launch_step<float, float, true>(c, a); break;
    }
}

static void enqueue_steps(lbm_ctx *c, int32_t nsteps) {
    for (int s = 0; s < nsteps; s++) {
        enqueue_step_into(c, cur_f(c), nxt_f(c), true);
        c->cur ^= 1;
        c->steps++;
    }
}

LBM_API int lbm_step(lbm_ctx *c, int32_t nsteps) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (int rc = nonfinite_reported(c)) return rc;
    enqueue_steps(c, nsteps);
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

LBM_API int lbm_step_timed(lbm_ctx *c, void *start_event, void *stop_event) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (!start_event || !stop_event) return fail(LBM_EINVAL, "start_event and stop_event must be HIP events");
    if (int rc = nonfinite_reported(c)) return rc;
    c->t_start = static_cast<hipEvent_t>(start_event);
    c->t_stop = static_cast<hipEvent_t>(stop_event);
    enqueue_steps(c, 1);
    c->t_start = c->t_stop = nullptr;
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
        k_moments<S, R, DEV, true><<<nb, 256, 0, c->s>>>((const S *)cur_f(c), c->stride, pop_view(c), G, c->N, g[0],
                                                          g[1], g[2], (R *)rho, (R *)u, c->partials);
    else
        k_moments<S, R, DEV, false><<<nb, 256, 0, c->s>>>((const S *)cur_f(c), c->stride, pop_view(c), G, c->N, g[0],
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
        case LBM_F64: k_store_f64<double, false><<<nb, 256, 0, c->s>>>((const double *)cur_f(c), c->stride, c->N, pop_view(c), f64); break;
        case LBM_F32: k_store_f64<float, false><<<nb, 256, 0, c->s>>>((const float *)cur_f(c), c->stride, c->N, pop_view(c), f64); break;
        default: k_store_f64<float, true><<<nb, 256, 0, c->s>>>((const float *)cur_f(c), c->stride, c->N, pop_view(c), f64); break;
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

LBM_API int lbm_load_f64(lbm_ctx *c, const double *f64) {
    if (!c || !f64) return fail(LBM_EINVAL, "NULL argument");
    if ((uintptr_t)f64 % 8) return fail(LBM_EINVAL, "f64 misaligned");
    c->rec_valid = false;  // the records hold the populations this replaces
    c->u_from_rec = false;
    if (int rc = reset_nonfinite(c)) return rc;  // a new state: forget earlier reports
    const int nb = (int)cdiv(c->N, 256);
    void *f = const_cast<void *>(cur_f(c));
    switch (c->p.prec) {
        case LBM_F64: k_load_f64<double, false><<<nb, 256, 0, c->s>>>((double *)f, c->stride, c->N, pop_view(c), f64); break;
        case LBM_F32: k_load_f64<float, false><<<nb, 256, 0, c->s>>>((float *)f, c->stride, c->N, pop_view(c), f64); break;
        default: k_load_f64<float, true><<<nb, 256, 0, c->s>>>((float *)f, c->stride, c->N, pop_view(c), f64); break;
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// immersed boundary

static int check_mesh_ptrs(const lbm_ctx *c, const ibm_mesh *m) {
    if (!m) return fail(LBM_EINVAL, "mesh is NULL");
    if (m->ncells < 1 || m->nverts < 1 || m->ntris < 1 || m->nedges < 1)
        return fail(LBM_EINVAL, "mesh counts must be >= 1");
    if (!m->vert_off || !m->tri_off || !m->edge_off || !m->tri || !m->hinge || !m->anchor || !m->x || !m->v ||
        !m->f_el || !m->moduli || !m->l0 || !m->a0 || !m->th0 || !m->a0c || !m->v0c || !m->avert || !m->vtri_off ||
        !m->vtri || !m->vedge_off || !m->vedge)
        return fail(LBM_EINVAL, "mesh has a NULL array");
    if (c->nch > 1 && !m->cell_chan)
        return fail(LBM_EINVAL, "cell_chan must be given when the context holds several channels");
    if (!(m->xi > 0) || !(m->mass > 0) || !(m->dt > 0) || !std::isfinite(m->xi) || !std::isfinite(m->mass) ||
        !std::isfinite(m->dt))
        return fail(LBM_EINVAL, "xi, mass and dt must be finite and > 0");
    if (m->stretch_law != 0 && m->stretch_law != 1) return fail(LBM_EINVAL, "stretch_law must be 0 or 1");
    if (const ibm_contact *k = m->contact) {
        if (!(k->a > 0) || !(k->n > 0) || !(k->rcut > 0) || !(k->dmin > 0) || !(k->dmin <= k->rcut) ||
            !(k->roff >= 0) || !std::isfinite(k->a) || !std::isfinite(k->n) || !std::isfinite(k->rcut) ||
            !std::isfinite(k->roff))
            return fail(LBM_EINVAL, "contact law needs finite a, n, rcut > 0, 0 < dmin <= rcut and roff >= 0");
        if (k->nplanes < 0 || k->ncyl < 0 || (k->nplanes && !k->planes) || (k->ncyl && !k->cyl))
            return fail(LBM_EINVAL, "contact walls: counts must be >= 0 and arrays given when counts are");
        if (k->cell_cell != 0 && k->cell_cell != 1) return fail(LBM_EINVAL, "contact cell_cell must be 0 or 1");
        if (k->nspheres < 0 || k->nspheres > (1 << 22) || (k->nspheres && !k->spheres))
            return fail(LBM_EINVAL, "contact spheres: 0 <= nspheres <= 2^22, and the array given when nspheres > 0");
        if (k->nspheres && c->nch > 1) return fail(LBM_EINVAL, "contact spheres need a one-channel context");
    }
    return LBM_OK;
}

static constexpr size_t kMaxLds = 64 * 1024;
static constexpr size_t kMaxSpreadLds = 160 * 1024;  // the spread's workgroups may take a compute unit's whole LDS

// Power of two >= a cell's point count (at least 64): the spread's sort size.
static int spread_pmax(int maxv) {
    int p = 64;
    while (p < maxv) p <<= 1;
    return p;
}

// Workgroups of the kernels that walk the compacted tile list.
static int waves_grid(const lbm_ctx *c) {
    if (c->list_blocks) return c->list_blocks;
    // four waves per workgroup, one wave per listed tile for lists up to a
    // quarter of the lattice (the waves stride over longer lists)
    return (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(c->ntiles, 4 * 4), 16384));
}

static MarkArgs mark_args(const lbm_ctx *c, const ibm_mesh *m, bool cover = false) {
    MarkArgs a{};
    if (cover) {  // check the marks against the nodes the last pass recorded
        a.cover = c->nx_ent;
        a.miss = c->nx_flags + 1;
    }
    a.tcount = c->tcount;
    a.epoch = c->epoch;
    a.chans = c->chans;
    a.cell_chan = m->cell_chan;
    a.vert_off = m->vert_off;
    a.anchor = m->anchor;
    a.x = m->x;
    a.ncells = m->ncells;
    a.nverts = m->nverts;
    a.need = c->need;
    a.tneed = c->tneed;
    a.fibm = c->fibm;
    a.accumulate = c->acc;
    return a;
}

// Membrane forces (rest: the rest shape); with `mark` the same kernel sets
// the stencil marks.
template <class R>
static void launch_membrane(lbm_ctx *c, const ibm_mesh *m, bool rest, bool mark = false, bool cover = false) {
    MembArgs a{};
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
    a.x = m->x;
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
    a.stretch_law = m->stretch_law;
    const size_t sm = membrane_lds_bytes<R>(m->max_cell_verts, m->max_cell_tris, m->max_cell_edges);
    if (rest) {
        k_membrane<R, true, false><<<m->ncells, kMembThreads, sm, c->s>>>(a);
    } else if (mark) {
        a.mark = mark_args(c, m, cover);
        k_membrane<R, false, true><<<m->ncells, kMembThreads, sm, c->s>>>(a);
    } else {
        k_membrane<R, false, false><<<m->ncells, kMembThreads, sm, c->s>>>(a);
    }
}

// Stencil marks of this step's positions on their own (with the list length
// and claim epoch reset for the step).
template <class R>
static void launch_mark(lbm_ctx *c, const ibm_mesh *m, bool cover = false) {
    const int nb = (int)cdiv(m->max_cell_verts, 128);
    k_mark<R><<<(unsigned)(nb * cdiv(m->ncells, 8) * 8), 128, 0, c->s>>>(mark_args(c, m, cover), nb);
}

// Sort the fixed contact spheres into a uniform grid over the lattice (one
// channel) whose cells are no smaller than the reach R_max + roff + rcut
// of a sphere, so that the 27 cells around a point hold every sphere that
// can act on it.  Synchronous: reads the spheres back.
static int build_sphere_grid(lbm_ctx *c, const ibm_contact *k) {
    c->sph_src = nullptr;
    c->sph_n = 0;
    if (k->nspheres == 0) return LBM_OK;
    const int ns = k->nspheres;
    std::vector<double> sp(4 * (size_t)ns);
    HIPCHK(hipStreamSynchronize(c->s));
    HIPCHK(hipMemcpy(sp.data(), k->spheres, sp.size() * 8, hipMemcpyDeviceToHost));
    double rmax = 0.0;
    for (int q = 0; q < ns; q++) {
        for (int d = 0; d < 4; d++)
            if (!std::isfinite(sp[4 * q + d])) return fail(LBM_EINVAL, "contact sphere %d is not finite", q);
        if (!(sp[4 * q + 3] > 0)) return fail(LBM_EINVAL, "contact sphere %d needs R > 0", q);
        rmax = std::max(rmax, sp[4 * q + 3]);
    }
    const double reach = (rmax + k->roff + k->rcut) * (1.0 + 1e-9);
    const int dims[3] = {c->p.nx, c->p.ny, c->p.nz};
    int g[3];
    for (int d = 0; d < 3; d++) g[d] = (int)std::max(1.0, std::min(1024.0, std::floor(dims[d] / reach)));
    // at most 2^22 cells (16 MB of offsets): halve the finest axis until it fits
    // (larger cells still hold every sphere in reach)
    while ((int64_t)g[0] * g[1] * g[2] > (int64_t(1) << 22)) {
        const int d = (g[0] >= g[1] && g[0] >= g[2]) ? 0 : (g[1] >= g[2] ? 1 : 2);
        g[d] = std::max(1, g[d] / 2);
    }
    int64_t ncell = 1;
    for (int d = 0; d < 3; d++) {
        c->sph_g[d] = g[d];
        c->sph_inv[d] = g[d] / (double)dims[d];
        ncell *= g[d];
    }
    // the cell of each sphere as the kernel computes it for a point
    std::vector<int32_t> cell(ns), start(ncell + 1, 0), items(ns);
    for (int q = 0; q < ns; q++) {
        int id[3];
        for (int d = 0; d < 3; d++) {
            double v = sp[4 * q + d];
            if (c->p.periodic[d]) v -= dims[d] * std::floor(v / dims[d]);
            const double qd = std::floor(v * c->sph_inv[d]);
            id[d] = qd < 0.0 ? 0 : (qd >= g[d] ? g[d] - 1 : (int)qd);
        }
        cell[q] = id[0] + g[0] * (id[1] + g[1] * id[2]);
        start[cell[q] + 1]++;
    }
    for (int64_t i = 0; i < ncell; i++) start[i + 1] += start[i];
    std::vector<int32_t> fill(start.begin(), start.end() - 1);
    for (int q = 0; q < ns; q++) items[fill[cell[q]]++] = q;  // ascending ids within a cell
    drop_graph(c);  // captured steps hold the grid's shape in their kernel arguments
    if (ncell + 1 > c->sph_cap_cells || ns > c->sph_cap_items) {
        for (void *b : {(void *)c->sph_start, (void *)c->sph_items})
            if (b) HIPCHK(hipFree(b));
        c->sph_start = c->sph_items = nullptr;
        c->sph_cap_cells = c->sph_cap_items = 0;
        if (hipMalloc(&c->sph_start, 4 * (size_t)(ncell + 1)) != hipSuccess ||
            hipMalloc(&c->sph_items, 4 * (size_t)ns) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_ENOMEM, "allocating the contact sphere grid failed");
        }
        c->sph_cap_cells = (int)(ncell + 1);
        c->sph_cap_items = ns;
    }
    HIPCHK(hipMemcpy(c->sph_start, start.data(), 4 * (size_t)(ncell + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->sph_items, items.data(), 4 * (size_t)ns, hipMemcpyHostToDevice));
    c->sph_src = k->spheres;
    c->sph_n = ns;
    return LBM_OK;
}

// Buffers of the next-step records (k_next_list), sized for every IB point
// of the meshes seen so far (at most 8 stencil nodes each, and at most N).
// Called from ibm_rest_shape, which waits on the stream anyway.
static int ensure_records(lbm_ctx *c, int nverts) {
    if (!c->rec_capable) return LBM_OK;
    c->nx_pts += nverts;
    const size_t tn = (size_t)c->ntiles, tpad = (size_t)cdiv((int64_t)tn, 16) * 16;
    if (!c->nx_need) {
        if (hipMalloc(&c->nx_need, c->N) != hipSuccess || hipMalloc(&c->nx_tneed, tpad) != hipSuccess ||
            hipMalloc(&c->nx_ent, 16 * tn) != hipSuccess ||
            hipMalloc(&c->nx_flags, 8) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_ENOMEM, "allocating the next-step marks failed");
        }
        HIPCHK(hipMemsetAsync(c->nx_need, 0, c->N, c->s));
        HIPCHK(hipMemsetAsync(c->nx_tneed, 0, tpad, c->s));
        HIPCHK(hipMemsetAsync(c->nx_ent, 0, 16 * tn, c->s));
        HIPCHK(hipMemsetAsync(c->nx_flags, 0, 8, c->s));
    }
    const int64_t want = std::min<int64_t>(c->N, 8 * c->nx_pts);
    if (want > c->nx_cap) {
        drop_graph(c);  // captured steps name the old record
        for (void *b : {(void *)c->nx_node, c->nx_rec})
            if (b) HIPCHK(hipFree(b));
        c->nx_node = nullptr;
        c->nx_rec = nullptr;
        c->nx_cap = 0;
        c->rec_valid = false;
        if (hipMalloc(&c->nx_node, 4 * (size_t)want) != hipSuccess ||
            hipMalloc(&c->nx_rec, (size_t)Q * want * c->rsize) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_ENOMEM, "allocating the next-step record (%lld slots) failed", (long long)want);
        }
        c->nx_cap = want;
    }
    return LBM_OK;
}

LBM_API int ibm_rest_shape(lbm_ctx *c, ibm_mesh *m) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (int rc = check_mesh_ptrs(c, m)) return rc;
    // read the topology back and check every index against its cell's range
    std::vector<int32_t> vo(m->ncells + 1), to(m->ncells + 1), eo(m->ncells + 1), tri(3 * (size_t)m->ntris),
        hin(4 * (size_t)m->nedges);
    HIPCHK(hipStreamSynchronize(c->s));
    HIPCHK(hipMemcpy(vo.data(), m->vert_off, vo.size() * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(to.data(), m->tri_off, to.size() * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(eo.data(), m->edge_off, eo.size() * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(tri.data(), m->tri, tri.size() * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hin.data(), m->hinge, hin.size() * 4, hipMemcpyDeviceToHost));
    if (m->cell_chan) {
        std::vector<int32_t> cch(m->ncells);
        HIPCHK(hipMemcpy(cch.data(), m->cell_chan, cch.size() * 4, hipMemcpyDeviceToHost));
        for (int k = 0; k < m->ncells; k++)
            if (cch[k] < 0 || cch[k] >= c->nch)
                return fail(LBM_EINVAL, "cell %d names channel %d (the context has %d)", k, cch[k], c->nch);
    }
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
    if (mv > kSpreadMaxPoints) return fail(LBM_EINVAL, "a cell has %d vertices (at most %d)", mv, kSpreadMaxPoints);
    if ((int64_t)m->ntris * 4 > INT32_MAX || (int64_t)m->nedges * 4 > INT32_MAX)
        return fail(LBM_EINVAL, "mesh too large for 32-bit incidence codes");
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
        HIPCHK(hipMemcpy(m->vtri_off, toff.data(), toff.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(m->vtri, tl.data(), tl.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(m->vedge_off, eoff.data(), eoff.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(m->vedge, el.data(), el.size() * 4, hipMemcpyHostToDevice));
    }
    m->max_cell_verts = mv;
    m->max_cell_tris = mt;
    m->max_cell_edges = me;
    const int64_t need_rec = (int64_t)m->nverts * (c->rsize == 8 ? sizeof(SRec<double>) : sizeof(SRec<float>));
    if (need_rec > c->srec_cap) {
        drop_graph(c);  // a captured graph names the old record buffer
        if (c->srec) HIPCHK(hipFree(c->srec));
        c->srec = nullptr;
        c->srec_cap = 0;
        if (hipMalloc(&c->srec, need_rec) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_ENOMEM, "allocating spread records for %d points failed", m->nverts);
        }
        c->srec_cap = need_rec;
    }
    if (int rc = ensure_records(c, m->nverts)) return rc;
    if (!c->owner) {
        if (hipMalloc(&c->owner, 4 * c->N) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_ENOMEM, "allocating the spreading claims (%lld bytes) failed", (long long)(4 * c->N));
        }
        HIPCHK(hipMemsetAsync(c->owner, 0, 4 * c->N, c->s));
    }
    {
        const size_t sl = c->rsize == 8 ? spread_lds_bytes<double>(spread_pmax(mv), mv)
                                        : spread_lds_bytes<float>(spread_pmax(mv), mv);
        if (sl > kMaxSpreadLds) return fail(LBM_EINVAL, "a cell with %d vertices does not fit the spread's LDS", mv);
        const hipError_t e = c->rsize == 8
            ? hipFuncSetAttribute((const void *)k_spread_cells<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sl)
            : hipFuncSetAttribute((const void *)k_spread_cells<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sl);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_EHIP, "the spread's LDS (%zu bytes) was refused: %s", sl, hipGetErrorString(e));
        }
    }
    if (const ibm_contact *k = m->contact) {
        if (int rc = build_sphere_grid(c, k)) return rc;
        if (k->cyl_off && k->ncyl) {
            std::vector<int32_t> co(c->nch + 1);
            HIPCHK(hipMemcpy(co.data(), k->cyl_off, co.size() * 4, hipMemcpyDeviceToHost));
            if (co[0] != 0 || co[c->nch] != k->ncyl) return fail(LBM_EINVAL, "cyl_off must run from 0 to ncyl");
            for (int q = 0; q < c->nch; q++)
                if (co[q + 1] < co[q]) return fail(LBM_EINVAL, "cyl_off must not decrease");
        }
        if (k->cell_cell && m->ncells > 1) {
            const int64_t all = (int64_t)m->ncells * (m->ncells - 1) / 2;
            if (all > (int64_t(1) << 22))
                return fail(LBM_EINVAL, "cell-cell contact supports up to %d cells per mesh", 2897);
            if (3 * (size_t)mv * 8 > kMaxLds)
                return fail(LBM_EINVAL, "a cell with %d vertices is too large for the contact pass", mv);
            if (m->ncells > c->bounds_cap || all > c->pair_cap) {
                drop_graph(c);
                for (void *b : {(void *)c->bounds, (void *)c->pairs, (void *)c->npairs})
                    if (b) HIPCHK(hipFree(b));
                c->bounds = nullptr, c->pairs = nullptr, c->npairs = nullptr;
                c->bounds_cap = c->pair_cap = 0;
                if (hipMalloc(&c->bounds, 32 * (size_t)m->ncells) != hipSuccess ||
                    hipMalloc(&c->pairs, 8 * (size_t)all) != hipSuccess || hipMalloc(&c->npairs, 4) != hipSuccess) {
                    (void)hipGetLastError();
                    return fail(LBM_ENOMEM, "allocating the contact pair list failed");
                }
                c->bounds_cap = m->ncells;
                c->pair_cap = (int)all;
            }
        }
    }
    if (c->p.prec == LBM_F64)
        launch_membrane<double>(c, m, true);
    else
        launch_membrane<float>(c, m, true);
    HIPCHK(hipGetLastError());
    m->checked = mesh_tag(m);
    return LBM_OK;
}

static ContactLaw contact_law(const ibm_contact *k) { return ContactLaw{k->a, k->n, k->rcut, k->roff, k->dmin}; }

// Cell-cell contact forces, added to the membrane force of step n.
template <class R>
static void launch_contact(lbm_ctx *c, const ibm_mesh *m) {
    const ibm_contact *k = m->contact;
    if (!k || !k->cell_cell || m->ncells < 2) return;
    BoundsArgs b{m->vert_off, m->anchor, m->x, c->bounds, c->npairs, m->ncells, m->nverts};
    k_cell_bounds<<<m->ncells, 256, 0, c->s>>>(b);
    PairArgs p{};
    p.bounds = c->bounds;
    p.cell_chan = m->cell_chan;
    p.chans = c->chans;
    p.npairs = c->npairs;
    p.pairs = c->pairs;
    p.ncells = m->ncells;
    p.cap = c->pair_cap;
    for (int d = 0; d < 3; d++) p.per[d] = c->p.periodic[d];
    p.reach = k->roff + k->rcut;
    k_contact_pairs<<<dim3((unsigned)cdiv(m->ncells, 256), (unsigned)m->ncells), 256, 0, c->s>>>(p);
    CellContactArgs a{};
    a.vert_off = m->vert_off;
    a.anchor = m->anchor;
    a.cell_chan = m->cell_chan;
    a.chans = c->chans;
    a.x = m->x;
    a.f_el = m->f_el;
    a.npairs = c->npairs;
    a.pairs = c->pairs;
    a.ncells = m->ncells;
    a.nverts = m->nverts;
    a.cap = c->pair_cap;
    for (int d = 0; d < 3; d++) a.per[d] = c->p.periodic[d];
    a.law = contact_law(k);
    const int grid = (int)std::min<int64_t>(c->pair_cap, 1024);
    k_contact_cells<R><<<grid, kContactThreads, 3 * (size_t)m->max_cell_verts * 8, c->s>>>(a);
}

static void launch_compact(lbm_ctx *c, const uint32_t *gate = nullptr) {
    k_compact<<<(int)cdiv(c->ntiles, kCompactThreads * kCompactPerThread), kCompactThreads, 0, c->s>>>(
        c->tneed, c->ntiles, c->tlist, c->tcount, gate);
}

template <class S, class R, bool DEV>
static void launch_velocity_records(lbm_ctx *c) {
    VelRecArgs a{};
    a.rec = c->nx_rec;
    a.cap = c->nx_cap;
    a.node = c->nx_node;
    a.count = c->nx_flags;
    a.cls = c->cls;
    a.gfield = c->p.gfield;
    a.ufield = c->ufield;
    a.N = c->N;
    for (int d = 0; d < 3; d++) a.g[d] = c->p.body_force[d];
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(c->nx_cap, 256), 16384));
    if (c->p.gfield)
        k_velocity_records<S, R, DEV, true><<<nb, 256, 0, c->s>>>(a);
    else
        k_velocity_records<S, R, DEV, false><<<nb, 256, 0, c->s>>>(a);
}

template <class S, class R, bool DEV>
static void launch_node_velocity(lbm_ctx *c, const void *f) {
    NodeVelArgs a{};
    a.f = f;
    a.stride = c->stride;
    a.links = c->links;
    for (int d = 0; d < 3; d++) a.per[d] = c->p.periodic[d];
    a.gfield = c->p.gfield;
    a.ufield = c->ufield;
    a.need = c->need;
    a.tmask = c->tmask;
    a.tnmask = c->tnmask;
    a.tlist = c->tlist;
    a.tcount = c->tcount;
    a.chans = c->chans;
    a.tile_chan = c->tile_chan;
    a.N = c->N;
    for (int d = 0; d < 3; d++) a.g[d] = c->p.body_force[d];
    if (c->p.gfield)
        k_node_velocity<S, R, DEV, true><<<waves_grid(c), 256, 0, c->s>>>(a);
    else
        k_node_velocity<S, R, DEV, false><<<waves_grid(c), 256, 0, c->s>>>(a);
}

static CoupleArgs couple_args(lbm_ctx *c, const ibm_mesh *m, bool next, bool reset) {
    CoupleArgs a{};
    if (next) {
        a.nx_need = c->nx_need;
        a.nx_tneed = c->nx_tneed;
    }
    if (reset) a.nx_count = c->nx_flags;
    a.ufield = c->ufield;
    a.srec = c->srec;
    a.chans = c->chans;
    a.cell_chan = m->cell_chan;
    a.vert_off = m->vert_off;
    a.anchor = m->anchor;
    a.x = m->x;
    a.v = m->v;
    a.f_el = m->f_el;
    a.avert = m->avert;
    a.ncells = m->ncells;
    a.nverts = m->nverts;
    a.xi = m->xi;
    a.dt_over_m = m->dt / m->mass;
    a.dt = m->dt;
    if (const ibm_contact *k = m->contact) {
        a.wall.planes = k->planes;
        a.wall.cyl = k->cyl;
        a.wall.cyl_off = k->cyl_off;
        a.wall.nplanes = k->nplanes;
        a.wall.ncyl = k->ncyl;
        for (int d = 0; d < 3; d++) a.wall.per[d] = c->p.periodic[d];
        a.wall.law = contact_law(k);
        if (k->nspheres) {  // the grid matches: the mesh tag (checked before) covers the spheres
            a.wall.sph = k->spheres;
            a.wall.sph_start = c->sph_start;
            a.wall.sph_items = c->sph_items;
            a.wall.nsph = k->nspheres;
            for (int d = 0; d < 3; d++) {
                a.wall.sg[d] = c->sph_g[d];
                a.wall.sinv[d] = c->sph_inv[d];
            }
        }
    }
    a.nb = (int)cdiv(m->max_cell_verts, 128);
    return a;
}

// Steps 1-3 of the points: interpolation, coupling force and the spread of
// -F_c, one workgroup per cell (k_spread_cells).
template <class R>
static void launch_couple(lbm_ctx *c, const ibm_mesh *m, bool reset = false) {
    SpreadArgs sp{};
    sp.cp = couple_args(c, m, false, reset);
    sp.vert_off = m->vert_off;
    sp.srec = c->srec;
    sp.owner = c->owner;
    sp.fibm = c->fibm;
    sp.facc = c->facc;
    sp.ftile = c->ftile;
    sp.epoch = c->epoch;
    sp.chans = c->chans;
    sp.cell_chan = m->cell_chan;
    sp.accumulate = c->acc;
    sp.pmax = spread_pmax(m->max_cell_verts);
    sp.maxv = m->max_cell_verts;
    k_spread_cells<R><<<m->ncells, kSpreadThreads, spread_lds_bytes<R>(sp.pmax, sp.maxv), c->s>>>(sp);
}

// Step 4 of the points (needs the membrane force), and the next step's marks.
template <class R>
static void launch_move(lbm_ctx *c, const ibm_mesh *m, bool next) {
    const CoupleArgs a = couple_args(c, m, next, false);
    k_move<R><<<(unsigned)(a.nb * cdiv(m->ncells, 8) * 8), 128, 0, c->s>>>(a);
}

// The immersed-boundary half of a coupled step with the populations f.
// With `overlap`, the membrane (and cell-cell contact) forces run on the
// side stream while the stencil nodes are marked, their velocities
// evaluated, the points' coupling forces computed and spread; the point
// update waits for both.
// The membrane is launched first: its workgroups (a few per compute unit,
// each holding its cell in LDS) then hold their slots before the velocity
// pass fills the chip.  Without it (the adjoint's recomputed steps, small
// and bound by launch latency) the membrane kernel also sets the marks and
// everything runs in order on the caller's stream.  Everything is joined back into the caller's
// stream before the call returns.
//
// `plain` marks a coupling of the context's own current state in a forward
// run.  There, when the last collide-stream pass recorded the nodes marked
// for this step, the stencil nodes' velocities come from those records
// (once per step, for all meshes coupled in it); the marking checks every
// stencil node against the recorded ones, and a node they miss (positions
// changed by the caller, a mesh not marked in the step before) lists the
// marked tiles for the gather pass, which recomputes every marked node from
// the lattice with the same operations, so either way the bits are the same.
// The point update then marks the stencils of the new positions for the
// records of the coming pass, while the record has room for them.
template <class S, class R, bool DEV>
static void enqueue_couple_as(lbm_ctx *c, const ibm_mesh *m, const void *f, bool overlap, bool plain) {
    c->acc = c->couples > 0;  // read by the mark and spread launches below
    c->couples++;
    const bool rec = plain && c->rec_valid;
    const bool next = plain && c->rec_mode && c->rec_capable && c->nx_rec &&
                      (c->nx_pending + m->nverts) * 8 <= c->nx_cap;
    const bool reset = plain && c->nx_rec;
    auto velocities = [&] {
        if (rec && !c->u_from_rec) {
            launch_velocity_records<S, R, DEV>(c);
            c->u_from_rec = true;
        }
        launch_compact(c, rec ? c->nx_flags + 1 : nullptr);
        launch_node_velocity<S, R, DEV>(c, f);
    };
    if (!overlap) {
        launch_membrane<R>(c, m, false, true, rec);
        launch_contact<R>(c, m);
        velocities();
        launch_couple<R>(c, m, reset);
    } else {
        const hipStream_t user = c->s;
        (void)hipEventRecord(c->ev_fork, user);
        (void)hipStreamWaitEvent(c->side, c->ev_fork, 0);
        c->s = c->side;
        launch_membrane<R>(c, m, false);
        launch_contact<R>(c, m);
        (void)hipEventRecord(c->ev_join, c->side);
        c->s = user;
        launch_mark<R>(c, m, rec);
        velocities();
        launch_couple<R>(c, m, reset);
        (void)hipStreamWaitEvent(user, c->ev_join, 0);
    }
    launch_move<R>(c, m, next);
    if (next) c->nx_pending += m->nverts;
    c->last_rec = rec;
}
static void enqueue_couple(lbm_ctx *c, const ibm_mesh *m, const void *f, bool may_overlap = true, bool plain = false) {
    const bool overlap =
        may_overlap && (c->ibm_overlap == 1 || (c->ibm_overlap == -1 && m->nverts >= LBM_OVERLAP_MIN_POINTS));
    switch (c->p.prec) {
        case LBM_F64: enqueue_couple_as<double, double, false>(c, m, f, overlap, plain); break;
        case LBM_F32: enqueue_couple_as<float, float, false>(c, m, f, overlap, plain); break;
        default: enqueue_couple_as<float, float, true>(c, m, f, overlap, plain); break;
    }
}
static void enqueue_couple(lbm_ctx *c, const ibm_mesh *m) { enqueue_couple(c, m, cur_f(c), true, true); }

// A mesh is ready for coupled steps when ibm_rest_shape has seen it in its
// current form and the context's sphere grid is the one of its spheres.
static int check_mesh_ready(const lbm_ctx *c, const ibm_mesh *m) {
    if (m->checked != mesh_tag(m)) return fail(LBM_ESTATE, "call ibm_rest_shape on this mesh first");
    const ibm_contact *k = m->contact;
    if (k && k->nspheres && (c->sph_src != k->spheres || c->sph_n != k->nspheres))
        return fail(LBM_ESTATE, "the context's sphere grid belongs to another mesh: call ibm_rest_shape again");
    return LBM_OK;
}

LBM_API int ibm_couple(lbm_ctx *c, const ibm_mesh *m) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (int rc = check_mesh_ptrs(c, m)) return rc;
    if (int rc = check_mesh_ready(c, m)) return rc;
    enqueue_couple(c, m);
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

// Capture what enqueue() launches into graph slot `slot` unless the slot
// already holds a graph with this key.  The capture runs on a private stream
// so that nothing else the process enqueues is recorded; nothing captured is
// a memset.  The context's state-buffer parity and step count are restored
// afterwards: the caller applies the graph's effect on them at launch.
template <class F>
static int capture_slot(lbm_ctx *c, int slot, uint64_t key, F &&enqueue) {
    if (c->gx[slot] && c->gk[slot] == key) return LBM_OK;
    if (c->gx[slot]) HIPCHK(hipGraphExecDestroy(c->gx[slot]));
    c->gx[slot] = nullptr;
    if (!c->cap_s) HIPCHK(hipStreamCreate(&c->cap_s));
    const hipStream_t user = c->s;
    const int cur0 = c->cur;
    const int64_t steps0 = c->steps;
    c->s = c->cap_s;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->s, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        enqueue();
        e = hipStreamEndCapture(c->s, &g);
    }
    c->s = user;
    c->cur = cur0;
    c->steps = steps0;
    c->g_rec_end[slot] = c->rec_valid;  // every replay ends with the records as the capture left them
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBM_EHIP, "capturing a graph failed: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&c->gx[slot], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->gx[slot] = nullptr;
        (void)hipGetLastError();
        return fail(LBM_EHIP, "instantiating a graph failed: %s", hipGetErrorString(e));
    }
    c->gk[slot] = key;
    return LBM_OK;
}

LBM_API int lbm_run(lbm_ctx *c, const ibm_mesh *m, int32_t nsteps, int32_t steps_per_graph) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (steps_per_graph < 0 || steps_per_graph % 2 || steps_per_graph > 4096)
        return fail(LBM_EINVAL, "steps_per_graph must be 0 or even and at most 4096 (got %d)", steps_per_graph);
    if (m) {
        if (int rc = check_mesh_ptrs(c, m)) return rc;
        if (int rc = check_mesh_ready(c, m)) return rc;
    }
    if (int rc = nonfinite_reported(c)) return rc;
    int32_t left = nsteps;
    // The first step runs as ordinary launches when a mesh coupled before
    // this call left its spread force pending (the first step adds to it;
    // every captured step starts from none), or when the next-step records
    // are not there yet (the captured steps then all find them).
    const bool first_records = m && c->rec_mode && c->rec_capable && c->nx_rec && !c->rec_valid;
    if ((c->couples > 0 || first_records) && left > 0 && steps_per_graph > 0) {
        if (m) enqueue_couple(c, m);
        enqueue_steps(c, 1);
        left--;
    }
    if (steps_per_graph > 0 && left >= steps_per_graph) {
        Fnv key;
        key.mix(G_RUN);
        key.mix((uint64_t)steps_per_graph);
        key.mix((uint64_t)c->cur);
        key.mix((uint64_t)c->rec_valid);
        key.mix((uint64_t)(c->nx_rec != nullptr) | (uint64_t)c->rec_mode << 1);
        key.mix(mesh_launch_key(m));
        if (int rc = capture_slot(c, G_RUN, key.h | 1ull, [&] {
                for (int k = 0; k < steps_per_graph; k++) {
                    if (m) enqueue_couple(c, m);
                    enqueue_steps(c, 1);
                }
            }))
            return rc;
        for (; left >= steps_per_graph; left -= steps_per_graph) {
            HIPCHK(hipGraphLaunch(c->gx[G_RUN], c->s));
            c->steps += steps_per_graph;  // an even number of swaps: the parity is unchanged
        }
        c->rec_valid = c->g_rec_end[G_RUN];
        c->u_from_rec = false;
        c->nx_pending = 0;
    }
    for (int32_t k = 0; k < left; k++) {
        if (m) enqueue_couple(c, m);
        enqueue_steps(c, 1);
    }
    HIPCHK(hipGetLastError());
    return nsteps > 0 ? queue_nonfinite_copy(c) : LBM_OK;
}

LBM_API int lbm_check_finite(lbm_ctx *c, int32_t *nonfinite) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    HIPCHK(hipMemcpyAsync(c->nf_host, c->nf_dev, 4, hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    c->nf_pending = false;
    const uint32_t bad = __atomic_load_n(c->nf_host, __ATOMIC_ACQUIRE);
    if (nonfinite) *nonfinite = bad ? 1 : 0;
    if (bad) return fail(LBM_ENONFINITE, "a collide-stream pass met non-finite populations (state is lost)");
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// adjoint

static int ensure_adjoint(lbm_ctx *c, const ibm_mesh *m) {
    if (!c->lamF) {
        if (hipMalloc(&c->lamF, 4 * c->N * c->rsize) != hipSuccess ||
            hipMalloc(&c->lamU, 4 * c->N * c->rsize) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_ENOMEM, "allocating the adjoint node buffers failed");
        }
        HIPCHK(hipMemsetAsync(c->lamF, 0, 4 * c->N * c->rsize, c->s));
        HIPCHK(hipMemsetAsync(c->lamU, 0, 4 * c->N * c->rsize, c->s));
    }
    if (m && m->nverts > c->adj_nv) {
        for (void *b : {(void *)c->xs, c->vs, c->fels, (void *)c->hv})
            if (b) HIPCHK(hipFree(b));
        c->xs = nullptr, c->vs = nullptr, c->fels = nullptr, c->hv = nullptr;
        c->adj_nv = 0;
        const size_t nv3 = 3 * (size_t)m->nverts;
        if (hipMalloc(&c->xs, nv3 * 8) != hipSuccess || hipMalloc(&c->vs, nv3 * c->rsize) != hipSuccess ||
            hipMalloc(&c->fels, nv3 * c->rsize) != hipSuccess || hipMalloc(&c->hv, nv3 * 8) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_ENOMEM, "allocating the adjoint point buffers failed");
        }
        c->adj_nv = m->nverts;
    }
    return LBM_OK;
}

static int check_jvp_mesh(const lbm_ctx *c, const ibm_mesh *m) {
    if (int rc = check_mesh_ptrs(c, m)) return rc;
    if (m->contact) return fail(LBM_EINVAL, "contact forces are not differentiated; use a mesh without contact");
    if (m->checked != mesh_tag(m)) return fail(LBM_ESTATE, "call ibm_rest_shape on this mesh first");
    if (adj_membrane_lds_bytes(m->max_cell_verts) > kMaxLds)
        return fail(LBM_EINVAL, "a cell with %d vertices is too large for the membrane Jacobian pass",
                    m->max_cell_verts);
    return LBM_OK;
}

template <class R>
static void launch_jvp(lbm_ctx *c, const ibm_mesh *m, const double *x, const double *w, const double *lam_x,
                       const double *lam_v, double *f_out, double *jvp_out) {
    JvpArgs a{};
    a.vert_off = m->vert_off;
    a.tri_off = m->tri_off;
    a.edge_off = m->edge_off;
    a.tri = m->tri;
    a.hinge = m->hinge;
    a.vtri_off = m->vtri_off;
    a.vtri = m->vtri;
    a.vedge_off = m->vedge_off;
    a.vedge = m->vedge;
    a.x = x;
    a.w = w;
    a.lam_x = lam_x;
    a.lam_v = lam_v;
    a.dt = m->dt;
    a.mass = m->mass;
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
    a.stretch_law = m->stretch_law;
    a.f_out = f_out;
    a.jvp_out = jvp_out;
    k_adj_membrane<R><<<m->ncells, kMembThreads, adj_membrane_lds_bytes(m->max_cell_verts), c->s>>>(a);
}

LBM_API int ibm_force_jvp(lbm_ctx *c, const ibm_mesh *m, const double *x, const double *w, double *f_out,
                          double *jvp_out) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (int rc = check_jvp_mesh(c, m)) return rc;
    if (!x || !w || !jvp_out) return fail(LBM_EINVAL, "x, w and jvp_out must be non-NULL");
    if (((uintptr_t)x | (uintptr_t)w | (uintptr_t)jvp_out | (uintptr_t)f_out) % 8)
        return fail(LBM_EINVAL, "x, w, f_out and jvp_out must be 8-byte aligned");
    if (c->p.prec == LBM_F64)
        launch_jvp<double>(c, m, x, w, nullptr, nullptr, f_out, jvp_out);
    else
        launch_jvp<float>(c, m, x, w, nullptr, nullptr, f_out, jvp_out);
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

template <class S, class R, bool DEV>
static void launch_adjoint(lbm_ctx *c, const ibm_mesh *m, const void *f_n, const double *x_n, const void *v_n,
                           const void *lam_next, void *lam, double *lam_x, double *lam_v, void *dgrad) {
    if (m) {
        // the membrane Jacobian-vector product needs only X_n and the
        // incoming adjoints: it runs on the side stream while the forward
        // half is recomputed and the collide-stream pass is transposed, and
        // the point pass waits for it
        const hipStream_t user = c->s;
        (void)hipEventRecord(c->ev_fork, user);
        (void)hipStreamWaitEvent(c->side, c->ev_fork, 0);
        c->s = c->side;
        launch_jvp<R>(c, m, x_n, nullptr, lam_x, lam_v, nullptr, c->hv);
        (void)hipEventRecord(c->ev_join, c->side);
        c->s = user;
        // recompute the forward immersed-boundary half of step n: stencil
        // marks, u_ext and rho at the marked nodes, the spread force
        ibm_mesh mm = *m;
        mm.x = c->xs;
        mm.v = c->vs;
        mm.f_el = c->fels;
        {  // X_n and V_n into the scratch the recomputed step advances (one launch)
            const int64_t n0 = 3 * (int64_t)m->nverts * 2, n1 = 3 * (int64_t)m->nverts * (int64_t)(sizeof(R) / 4);
            k_copy_pair<<<(int)std::max<int64_t>(1, std::min<int64_t>(cdiv(n0 + n1, 256), 4096)), 256, 0, c->s>>>(
                reinterpret_cast<const uint32_t *>(x_n), reinterpret_cast<uint32_t *>(c->xs), n0,
                static_cast<const uint32_t *>(v_n), static_cast<uint32_t *>(c->vs), n1);
        }
        c->couples = 0;
        enqueue_couple(c, &mm, f_n, false);
    }
    c->couples = 0;  // the adjoint pass below consumes the recomputed force
    AdjStepArgs a{};
    a.f = f_n;
    a.lam_next = lam_next;
    a.lam = lam;
    a.stride = c->stride;
    a.links = c->links;
    a.fibm = c->fibm;
    a.facc = c->facc;
    a.ftile = c->ftile;
    a.tneed = c->tneed;
    a.tmask = c->tmask;
    a.tnmask = c->tnmask;
    a.lamF = c->lamF;
    a.dgrad = dgrad;
    a.gfield = c->p.gfield;
    a.chans = c->chans;
    a.tile_chan = c->tile_chan;
    a.ntiles = c->ntiles;
    a.N = c->N;
    for (int d = 0; d < 3; d++) a.g[d] = c->p.body_force[d];
    a.omega = 1.0 / c->p.tau;
    a.kf = 1.0 - 0.5 / c->p.tau;
    for (int d = 0; d < 3; d++) a.per[d] = c->p.periodic[d];
    const CsShape sh = cs_shape(c);
    a.remap = sh.remap;
    a.wgtab = sh.tab;
    const int nb = sh.nb;
    if (c->p.gfield)
        k_adj_collide_stream<S, R, DEV, true><<<nb, 64 * sh.waves, 0, c->s>>>(a);
    else
        k_adj_collide_stream<S, R, DEV, false><<<nb, 64 * sh.waves, 0, c->s>>>(a);
    if (!m) return;
    (void)hipStreamWaitEvent(c->s, c->ev_join, 0);
    AdjPointArgs p{};
    p.ufield = c->ufield;
    p.lamF = c->lamF;
    p.lamU = c->lamU;
    p.chans = c->chans;
    p.cell_chan = m->cell_chan;
    p.vert_off = m->vert_off;
    p.anchor = m->anchor;
    p.x = x_n;
    p.v = v_n;
    p.hv = c->hv;
    p.lam_x = lam_x;
    p.lam_v = lam_v;
    p.avert = m->avert;
    p.ncells = m->ncells;
    p.nverts = m->nverts;
    p.xi = m->xi;
    p.mass = m->mass;
    p.dt = m->dt;
    dim3 grid((unsigned)cdiv(m->max_cell_verts, 128), (unsigned)m->ncells);
    k_adj_points<R><<<grid, 128, 0, c->s>>>(p);
    AdjNodeArgs q{};
    q.tlist = c->tlist;
    q.tcount = c->tcount;
    q.need = c->need;
    q.tneed = c->tneed;
    q.ufield = c->ufield;
    q.lamU = c->lamU;
    q.lam = lam;
    q.dgrad = dgrad;
    q.cls = c->cls;
    q.chans = c->chans;
    q.tile_chan = c->tile_chan;
    q.stride = c->stride;
    q.N = c->N;
    k_adj_nodes<R><<<waves_grid(c), 256, 0, c->s>>>(q);
}

static void enqueue_adjoint(lbm_ctx *c, const ibm_mesh *m, const void *f_n, const double *x_n, const void *v_n,
                            const void *lam_next, void *lam, double *lam_x, double *lam_v, void *dgrad) {
    switch (c->p.prec) {
        case LBM_F64:
            launch_adjoint<double, double, false>(c, m, f_n, x_n, v_n, lam_next, lam, lam_x, lam_v, dgrad);
            break;
        case LBM_F32:
            launch_adjoint<float, float, false>(c, m, f_n, x_n, v_n, lam_next, lam, lam_x, lam_v, dgrad);
            break;
        default:
            launch_adjoint<float, float, true>(c, m, f_n, x_n, v_n, lam_next, lam, lam_x, lam_v, dgrad);
            break;
    }
}

LBM_API int lbm_adjoint_step(lbm_ctx *c, const ibm_mesh *m, const void *f_n, const double *x_n, const void *v_n,
                             const void *lam_next, void *lam, double *lam_x, double *lam_v, void *dgrad) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (!f_n || !lam_next || !lam) return fail(LBM_EINVAL, "f_n, lam_next and lam must be non-NULL");
    if (lam == lam_next || lam == f_n) return fail(LBM_EINVAL, "lam must not alias lam_next or f_n");
    const uintptr_t es = c->rsize;
    if (((uintptr_t)f_n | (uintptr_t)lam_next | (uintptr_t)lam | (uintptr_t)dgrad) % es)
        return fail(LBM_EINVAL, "f_n, lam_next, lam and dgrad must be aligned to their element size");
    if (m) {
        if (int rc = check_jvp_mesh(c, m)) return rc;
        if (!x_n || !v_n || !lam_x || !lam_v) return fail(LBM_EINVAL, "x_n, v_n, lam_x and lam_v must be non-NULL");
        if (((uintptr_t)x_n | (uintptr_t)lam_x | (uintptr_t)lam_v) % 8 || (uintptr_t)v_n % es)
            return fail(LBM_EINVAL, "point arrays misaligned");
        if (!c->owner) return fail(LBM_ESTATE, "call ibm_rest_shape first");
    }
    if (int rc = ensure_adjoint(c, m)) return rc;
    c->rec_valid = false;  // the recomputed step reuses the velocity field and the marks
    c->u_from_rec = false;
    enqueue_adjoint(c, m, f_n, x_n, v_n, lam_next, lam, lam_x, lam_v, dgrad);
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

// Checks shared by the recording run and the reverse sweep.
static int check_record(lbm_ctx *c, const ibm_mesh *m, int32_t nsteps, const void *f_rec, const double *x_rec,
                        const void *v_rec) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (nsteps > 0 && !f_rec) return fail(LBM_EINVAL, "f_rec is NULL");
    if ((uintptr_t)f_rec % 16) return fail(LBM_EINVAL, "f_rec must be 16-byte aligned");
    if (m) {
        if (int rc = check_jvp_mesh(c, m)) return rc;
        if (nsteps > 0 && (!x_rec || !v_rec)) return fail(LBM_EINVAL, "x_rec and v_rec must be non-NULL");
        if ((uintptr_t)x_rec % 8 || (uintptr_t)v_rec % c->rsize) return fail(LBM_EINVAL, "x_rec/v_rec misaligned");
        if (!c->owner) return fail(LBM_ESTATE, "call ibm_rest_shape first");
    }
    return LBM_OK;
}

LBM_API int lbm_run_record(lbm_ctx *c, const ibm_mesh *m, int32_t nsteps, void *f_rec, double *x_rec, void *v_rec,
                           int32_t use_graph) {
    if (int rc = check_record(c, m, nsteps, f_rec, x_rec, v_rec)) return rc;
    if (nsteps == 0) return LBM_OK;
    const size_t fb = 19 * (size_t)c->stride * c->rsize;
    const size_t nv3 = m ? 3 * (size_t)m->nverts : 0;
    char *F = static_cast<char *>(f_rec);
    auto enqueue = [&] {
        // step k reads state k from the record and writes state k+1 into the
        // next record; the last step writes back into the current buffer
        // (its content is record 0 by then), so the parity is unchanged
        enqueue_copy(c, F, cur_f(c), fb);
        for (int k = 0; k < nsteps; k++) {
            const void *fa = F + k * fb;
            if (m) {
                enqueue_copy(c, x_rec + k * nv3, m->x, nv3 * 8);
                enqueue_copy(c, static_cast<char *>(v_rec) + k * nv3 * c->rsize, m->v, nv3 * c->rsize);
                enqueue_couple(c, m, fa);
            }
            enqueue_step_into(c, fa, k + 1 < nsteps ? (void *)(F + (k + 1) * fb) : const_cast<void *>(cur_f(c)));
        }
    };
    if (use_graph) {
        Fnv key;
        key.mix(G_REC);
        key.mix((uint64_t)nsteps);
        key.mix((uint64_t)c->cur);
        key.mix((uint64_t)(c->couples > 0));  // baked into the first step's spread, as in lbm_run
        key.mix(mesh_launch_key(m));
        for (const void *p : {(const void *)f_rec, (const void *)x_rec, (const void *)v_rec}) key.mix((uint64_t)(uintptr_t)p);
        if (int rc = capture_slot(c, G_REC, key.h | 1ull, enqueue)) return rc;
        HIPCHK(hipGraphLaunch(c->gx[G_REC], c->s));
    } else {
        enqueue();
    }
    c->couples = 0;  // the last recorded step consumed every spread force
    c->rec_valid = false;  // its passes record nothing
    c->u_from_rec = false;
    c->nx_pending = 0;
    c->steps += nsteps;
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

LBM_API int lbm_adjoint_run(lbm_ctx *c, const ibm_mesh *m, int32_t nsteps, const void *f_rec, const double *x_rec,
                            const void *v_rec, void *lam_a, void *lam_b, double *lam_x, double *lam_v, void *dgrad,
                            int32_t use_graph) {
    if (int rc = check_record(c, m, nsteps, f_rec, x_rec, v_rec)) return rc;
    if (!lam_a || !lam_b || lam_a == lam_b) return fail(LBM_EINVAL, "lam_a and lam_b must be distinct and non-NULL");
    if (((uintptr_t)lam_a | (uintptr_t)lam_b) % 16 || (uintptr_t)dgrad % c->rsize)
        return fail(LBM_EINVAL, "lam_a/lam_b must be 16-byte aligned and dgrad aligned to its element");
    if (m && (!lam_x || !lam_v || ((uintptr_t)lam_x | (uintptr_t)lam_v) % 8))
        return fail(LBM_EINVAL, "lam_x and lam_v must be non-NULL and 8-byte aligned");
    if (nsteps == 0) return LBM_OK;
    if (int rc = ensure_adjoint(c, m)) return rc;
    c->rec_valid = false;  // the recomputed steps reuse the velocity field and the marks
    c->u_from_rec = false;
    const size_t fb = 19 * (size_t)c->stride * c->rsize;
    const size_t nv3 = m ? 3 * (size_t)m->nverts : 0;
    const char *F = static_cast<const char *>(f_rec);
    auto enqueue = [&] {
        void *lam[2] = {lam_a, lam_b};
        for (int k = nsteps - 1, j = 0; k >= 0; k--, j ^= 1)
            enqueue_adjoint(c, m, F + k * fb, m ? x_rec + k * nv3 : nullptr,
                            m ? static_cast<const char *>(v_rec) + k * nv3 * c->rsize : nullptr, lam[j], lam[j ^ 1],
                            lam_x, lam_v, dgrad);
        if (nsteps % 2) enqueue_copy(c, lam_a, lam_b, fb);
    };
    if (use_graph) {
        Fnv key;
        key.mix(G_ADJ);
        key.mix((uint64_t)nsteps);
        key.mix(mesh_launch_key(m));
        for (const void *p : {(const void *)f_rec, (const void *)x_rec, (const void *)v_rec, (const void *)lam_a,
                              (const void *)lam_b, (const void *)lam_x, (const void *)lam_v, (const void *)dgrad,
                              (const void *)c->xs, (const void *)c->hv, (const void *)c->lamF})
            key.mix((uint64_t)(uintptr_t)p);
        if (int rc = capture_slot(c, G_ADJ, key.h | 1ull, enqueue)) return rc;
        HIPCHK(hipGraphLaunch(c->gx[G_ADJ], c->s));
    } else {
        enqueue();
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

// Immersed-boundary kernels (Sec. 2.2) and membrane forces (Sec. 2.3).
//
// One coupled step runs these kernels before the collide-stream pass:
//
// k_mark (one thread per IB point) marks, with plain byte stores, every
//   lattice node of every point's 2x2x2 stencil and the 64-node tile
//   holding it.
//
// k_membrane (one workgroup per cell; on a second stream, beside the
//   compaction and velocity passes, which do not need its forces): the
//   cell's vertex positions are staged in LDS; the cell's total area and
//   volume (the global constraints
//   that need every vertex of the cell, Sec. 2.3.3) are reduced first, then
//   each triangle and each edge/hinge stores its scalar force coefficient in
//   LDS, and each vertex sums its incident elements' gradients in a fixed
//   order and writes its force once.
//   Lengths, areas, angles and volumes are evaluated in FP64 from the FP64
//   positions, so their small departures from the (FP64) rest shape keep
//   full accuracy in every storage precision.
//
// k_compact: the marked tiles become a dense list.
//
// k_node_velocity (one wave per listed tile): u_ext = (j + F_ext/2)/rho of
//   the marked nodes only, from their current populations, into an AoS
//   field (one 16-byte record per node: u_ext and rho); each node is
//   evaluated once however many IB points use it.
//
// k_couple (one thread per IB point): trilinear interpolation of that field
//   (Sec. 2.2 step 1), coupling force (step 2), and the point update (step
//   4).  The point also writes a spread record: its stencil's base node,
//   fractional offsets and the force it exerts on the fluid (-F_c).
//
// Spreading (step 3) avoids per-contribution float atomics, which run at a
// small fraction of store throughput on this GPU:
// k_spread_cells (one workgroup per cell) sorts the cell's records by base
//   node in LDS, sums each base node's points into its 8 corner
//   contributions, and writes them to that base node's slot after claiming
//   it with one compare-and-swap of the call's epoch (a base node already
//   claimed by another cell in this call falls back to float atomics into
//   a separate accumulator, kept zero between steps; that needs two
//   membranes inside one lattice cell).  The owner also sets, at each of the 8 corner nodes, the byte
//   that says "base node in role q has a slot for you".
// k_gather_nodes (one wave per listed tile) reads its node's 8 role bytes
//   with one load, adds the flagged slots in a fixed order, clears the
//   bytes and writes the node's spread force at every marked node; the
//   fallback path flags its tiles so that only those read the accumulated
//   atomics back (and clear them).
// All sums except the fallback are in a fixed order, so the spread is
// bit-reproducible.
//
// The node and tile marks stay set until the collide-stream pass: they are
// exactly the nodes whose spread force the gather wrote this step, so that
// pass reads the force record of marked nodes only (a record elsewhere may
// hold an earlier step's force) and clears the marks.
#pragma once

#include "d3q19.hpp"
#include "lattice_kernels.hpp"

namespace lbm {

// 4-wide AoS record of the force accumulator and the velocity field
template <class R>
struct Vec4;
template <>
struct Vec4<float> {
    using T = float4;
};
template <>
struct Vec4<double> {
    using T = double4;
};

struct V3 {
    double x, y, z;
};
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 crs(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 scl(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }

// Signed angle between the outward normals of (p1,p2,qa) and (p2,p1,qb):
// zero when flat, positive for a convex fold.  Also returns the unnormalised
// normals and the edge vector.
__device__ __forceinline__ double hinge_angle(V3 p1, V3 p2, V3 qa, V3 qb, V3 &na, V3 &nb, V3 &e) {
    e = sub(p2, p1);
    na = crs(e, sub(qa, p1));
    nb = crs(sub(p1, p2), sub(qb, p2));
    return atan2(dot(crs(na, nb), e) / sqrt(dot(e, e)), dot(na, nb));
}

__device__ __forceinline__ int cell_channel(const int32_t *cell_chan, int c) { return cell_chan ? cell_chan[c] : 0; }

struct MarkArgs {
    uint32_t *tcount;  // tile-list length, reset here for this step
    uint32_t *epoch;   // spreading-claim epoch, advanced here for this step
    const Chan *chans;
    const int32_t *cell_chan;  // [ncells] channel of each cell, null for a single channel
    const int32_t *vert_off, *anchor;
    const double *x;  // [3][nverts] offsets
    int ncells, nverts;
    uint8_t *need;   // [N] stencil-node marks
    uint8_t *tneed;  // [ntiles] tile marks
    void *fibm;      // [N] Vec4 spread force: zeroed at newly marked nodes when `accumulate`
    int accumulate;  // 1: another membrane was coupled earlier in this step (its force stays)
};

// Mark the 2x2x2 stencil of a point at offset (px, py, pz) from anchor
// (ax, ay, az) in channel ch: every node, and the 64-node tile holding it,
// with plain byte stores.
template <class R>
__device__ __forceinline__ void mark_stencil(const MarkArgs &a, const Chan &ch, int ax, int ay, int az, double px,
                                             double py, double pz) {
    const int x0 = pmod(ax + (int)floor(px), ch.nx);
    const int y0 = pmod(ay + (int)floor(py), ch.ny);
    const int z0 = pmod(az + (int)floor(pz), ch.nz);
    const int xs[2] = {x0, x0 + 1 == ch.nx ? 0 : x0 + 1};
    const int ys[2] = {y0, y0 + 1 == ch.ny ? 0 : y0 + 1};
    const int zs[2] = {z0, z0 + 1 == ch.nz ? 0 : z0 + 1};
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int row = ys[q & 1] + ch.ny * zs[q >> 1];
#pragma unroll
        for (int e = 0; e < 2; e++) {
            const int64_t nn = ch.noff + (int64_t)row * ch.nx + xs[e];
            if (a.accumulate) {
                // a node first marked now starts from zero force; one
                // marked by an earlier membrane of the step keeps its force
                if (!a.need[nn]) {
                    a.need[nn] = 1;
                    static_cast<typename Vec4<R>::T *>(a.fibm)[nn] = typename Vec4<R>::T{R(0), R(0), R(0), R(0)};
                }
            } else {
                a.need[nn] = 1;
            }
            // the two x of a row share a tile unless the pair crosses a tile edge
            if (e == 0 || (xs[1] >> 6) != (xs[0] >> 6)) a.tneed[ch.toff + (int64_t)row * ch.tpr + (xs[e] >> 6)] = 1;
        }
    }
}

// Reset of the tile-list length and advance of the claim epoch for a step.
__device__ __forceinline__ void start_marks(const MarkArgs &a) {
    *a.tcount = 0;
    *a.epoch += 1u;
}

// The stencil marks of every point (positions of this step) on their own:
// one thread per point, blockIdx.y = cell.  Independent of the membrane
// forces, so the velocity pass that reads the marks can run beside the
// membrane kernel.
template <class R>
__global__ __launch_bounds__(128) void k_mark(MarkArgs a) {
    const int c = blockIdx.y;
    if (c == 0 && blockIdx.x == 0 && threadIdx.x == 0) start_marks(a);
    const int v0 = a.vert_off[c], k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.vert_off[c + 1] - v0) return;
    const int NV = a.nverts;
    mark_stencil<R>(a, a.chans[cell_channel(a.cell_chan, c)], a.anchor[c], a.anchor[a.ncells + c],
                    a.anchor[2 * a.ncells + c], a.x[v0 + k], a.x[NV + v0 + k], a.x[2 * NV + v0 + k]);
}

struct MembArgs {
    const int32_t *vert_off, *tri_off, *edge_off, *tri, *hinge;
    // per-vertex incidence (global vertex ids; entries are element*4 + role)
    const int32_t *vtri_off, *vtri, *vedge_off, *vedge;
    const double *x;  // [3][nverts] offsets
    void *f_el;       // [3][nverts]
    const void *moduli;
    double *l0, *a0, *th0, *a0c, *v0c, *avert;
    int ncells, nverts, ntris, nedges, maxv, maxt, maxe;
    int stretch_law;  // 0: linear edge springs, 1: neo-Hookean edge springs
    MarkArgs mark;    // the stencil marks, when the kernel also sets them (MARK)
};

constexpr int kMembThreads = 512;
constexpr int kInc = 4;  // incident elements whose indices a vertex loads together


// LDS layout: reduction scratch (2 doubles per wave), x, y, z positions
// (double), then one coefficient per triangle and two per edge (R).
template <class R>
__host__ __device__ inline size_t membrane_lds_bytes(int maxv, int maxt, int maxe) {
    return 2 * (kMembThreads / 64) * sizeof(double) + 3 * (size_t)maxv * sizeof(double) +
           ((size_t)maxt + 2 * (size_t)maxe) * sizeof(R);
}

// Force on a vertex in role r of triangle (A, B, C) with area coefficient h
// and volume coefficient cv6: grad of area ~ (next - prev) x n, of volume
// (next x prev)/6.
__device__ __forceinline__ void tri_term(const V3 &A, const V3 &B, const V3 &C, int r, double h, double cv6,
                                         double &fx, double &fy, double &fz) {
    const V3 n = crs(sub(B, A), sub(C, A));
    const V3 nx_ = r == 0 ? B : (r == 1 ? C : A), pv = r == 0 ? C : (r == 1 ? A : B);
    const V3 g = crs(sub(nx_, pv), n), vg3 = crs(nx_, pv);
    fx += h * g.x - cv6 * vg3.x;
    fy += h * g.y - cv6 * vg3.y;
    fz += h * g.z - cv6 * vg3.z;
}

// Force on a vertex in role r (0: p1, 1: p2, 2: qa, 3: qb) of hinge
// (p1, p2, qa, qb) with stretch coefficient cs and bend coefficient cb.
// d theta/d qa = -|e| na/|na|^2, d theta/d qb = -|e| nb/|nb|^2; the edge ends
// take the combinations that keep net force and torque zero.
__device__ __forceinline__ void edge_term(const V3 &p1, const V3 &p2, const V3 &qa, const V3 &qb, int r, double cs,
                                          double cb, double &fx, double &fy, double &fz) {
    const V3 ev = sub(p2, p1);
    const V3 na = crs(ev, sub(qa, p1)), nb = crs(sub(p1, p2), sub(qb, p2));
    const double l2 = dot(ev, ev), l = sqrt(l2);
    const V3 ga = scl(-l / dot(na, na), na), gb = scl(-l / dot(nb, nb), nb);
    V3 g;
    double s = 0.0;
    if (r == 2) {
        g = ga;
    } else if (r == 3) {
        g = gb;
    } else {
        const double sa = dot(sub(qa, p1), ev) / l2, sb = dot(sub(qb, p1), ev) / l2;
        const double ca_ = r == 0 ? -(1.0 - sa) : -sa, cb_ = r == 0 ? -(1.0 - sb) : -sb;
        g = V3{ca_ * ga.x + cb_ * gb.x, ca_ * ga.y + cb_ * gb.y, ca_ * ga.z + cb_ * gb.z};
        s = r == 0 ? cs : -cs;
    }
    fx += s * ev.x - cb * g.x;
    fy += s * ev.y - cb * g.y;
    fz += s * ev.z - cb * g.z;
}

// REST = true: write the rest shape; false: elastic forces, and with MARK
// the stencil marks of the cell's points as well (the coupled step that does
// not run the membrane beside the velocity pass).
//
// Forces are the exact gradients of the energies written element by
// element.  A first pass computes each element's scalar coefficient (a
// triangle's area factor, an edge's stretch and bend factors; after the
// cell's area and volume are reduced).  A second pass gives each vertex the
// sum over its incident elements, walked in a fixed order from the
// incidence lists, of coefficient times the element's gradient with respect
// to that vertex.  No atomics, so the forces are bit-reproducible.
template <class R, bool REST, bool MARK>
__global__ __launch_bounds__(kMembThreads) void k_membrane(MembArgs a) {
    extern __shared__ double smem_d[];
    const int c = blockIdx.x;
    const int v0 = a.vert_off[c], nv = a.vert_off[c + 1] - v0;
    const int t0 = a.tri_off[c], nt = a.tri_off[c + 1] - t0;
    const int e0 = a.edge_off[c], ne = a.edge_off[c + 1] - e0;
    double *red = smem_d;  // 2 per wave
    double *px = smem_d + 2 * (kMembThreads / 64), *py = px + a.maxv, *pz = py + a.maxv;
    R *tco = reinterpret_cast<R *>(pz + a.maxv);  // [maxt]
    R *eco = tco + a.maxt;                        // [2*maxe]
    const double *X = a.x;
    const int NV = a.nverts;
    for (int k = threadIdx.x; k < nv; k += blockDim.x) {
        px[k] = X[v0 + k];
        py[k] = X[NV + v0 + k];
        pz[k] = X[2 * NV + v0 + k];
    }
    __syncthreads();
    auto P = [&](int k) { return V3{px[k], py[k], pz[k]}; };
    const int NT = a.ntris, NE = a.nedges;
    if (MARK) {
        const MarkArgs &mk = a.mark;
        if (c == 0 && threadIdx.x == 0) start_marks(mk);
        const Chan ch = mk.chans[cell_channel(mk.cell_chan, c)];
        const int ax = mk.anchor[c], ay = mk.anchor[mk.ncells + c], az = mk.anchor[2 * mk.ncells + c];
        for (int k = threadIdx.x; k < nv; k += blockDim.x) mark_stencil<R>(mk, ch, ax, ay, az, px[k], py[k], pz[k]);
    }

    // cell area and volume (FP64 sums of FP64 per-triangle values, fixed order)
    double acc[2] = {0.0, 0.0};
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
        const V3 A = P(a.tri[t0 + t] - v0), B = P(a.tri[NT + t0 + t] - v0), C = P(a.tri[2 * NT + t0 + t] - v0);
        const V3 n = crs(sub(B, A), sub(C, A));
        acc[0] += 0.5 * sqrt(dot(n, n));
        acc[1] += dot(A, crs(B, C)) / 6.0;
    }
    block_sum<2>(acc, red);
    const R *mod = static_cast<const R *>(a.moduli);
    const int NC = a.ncells;
    const double ks = mod[c], kb = mod[NC + c], kal = mod[2 * NC + c], kag = mod[3 * NC + c],
                 kv = mod[4 * NC + c];
    if (REST) {
        if (threadIdx.x == 0) {
            a.a0c[c] = acc[0];
            a.v0c[c] = acc[1];
        }
    }
    const double cag = REST ? 0.0 : kag * (acc[0] - a.a0c[c]) / a.a0c[c];
    const double cv6 = REST ? 0.0 : kv * (acc[1] - a.v0c[c]) / a.v0c[c] / 6.0;

    // element pass: one coefficient per triangle, two per edge
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
        const V3 A = P(a.tri[t0 + t] - v0), B = P(a.tri[NT + t0 + t] - v0), C = P(a.tri[2 * NT + t0 + t] - v0);
        const V3 n = crs(sub(B, A), sub(C, A));
        const double nn = sqrt(dot(n, n));
        const double area = 0.5 * nn;
        if (REST) {
            a.a0[t0 + t] = area;
            tco[t] = R(area);
            continue;
        }
        const double ref = a.a0[t0 + t];
        // -dE/dA * grad A with grad_a A = (b - c) x n / (2|n|)
        tco[t] = R(-0.5 * (kal * (area - ref) / ref + cag) / nn);
    }
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        const V3 p1 = P(a.hinge[e0 + e] - v0), p2 = P(a.hinge[NE + e0 + e] - v0);
        const V3 qa = P(a.hinge[2 * NE + e0 + e] - v0), qb = P(a.hinge[3 * NE + e0 + e] - v0);
        V3 na, nb, ev;
        const double th = hinge_angle(p1, p2, qa, qb, na, nb, ev);
        const double l = sqrt(dot(ev, ev));
        if (REST) {
            a.l0[e0 + e] = l;
            a.th0[e0 + e] = th;
            continue;
        }
        const double ref = a.l0[e0 + e];
        // dE/dl / l; neo-Hookean: E = (k_s/6) l0 (lam^2 + 2/lam - 3), lam = l/l0
        const double lam = l / ref;
        const double dEdl = a.stretch_law ? ks / 3.0 * (lam - 1.0 / (lam * lam)) : ks * (l - ref) / ref;
        eco[2 * e] = R(dEdl / l);                      // force on p1 = cs (p2 - p1)
        eco[2 * e + 1] = R(kb * (th - a.th0[e0 + e]));  // force = -cb grad theta
    }
    __syncthreads();

    // vertex pass
    R *FE = static_cast<R *>(a.f_el);
    for (int k = threadIdx.x; k < nv; k += blockDim.x) {
        const int vg = v0 + k;
        if (REST) {  // each vertex carries a third of its triangles' rest area
            double s = 0.0;
            for (int i = a.vtri_off[vg]; i < a.vtri_off[vg + 1]; i++) s += a.a0[a.vtri[i] >> 2] / 3.0;
            a.avert[vg] = s;
            continue;
        }
        double fx = 0.0, fy = 0.0, fz = 0.0;
        // The incident elements are taken kInc at a time: their codes and
        // vertex indices are loaded first (independent loads in flight
        // together), then the terms are added in list order.
        const int ti0 = a.vtri_off[vg], ti1 = a.vtri_off[vg + 1];
        for (int base = ti0; base < ti1; base += kInc) {
            int tv[kInc][3], tt[kInc], tr[kInc];
#pragma unroll
            for (int j = 0; j < kInc; j++) {
                const int code = base + j < ti1 ? a.vtri[base + j] : a.vtri[ti0];
                tt[j] = (code >> 2) - t0;
                tr[j] = code & 3;
            }
#pragma unroll
            for (int j = 0; j < kInc; j++)
#pragma unroll
                for (int q = 0; q < 3; q++) tv[j][q] = a.tri[q * NT + t0 + tt[j]] - v0;
#pragma unroll
            for (int j = 0; j < kInc; j++) {
                if (base + j >= ti1) break;
                tri_term(P(tv[j][0]), P(tv[j][1]), P(tv[j][2]), tr[j], (double)tco[tt[j]], cv6, fx, fy, fz);
            }
        }
        const int ei0 = a.vedge_off[vg], ei1 = a.vedge_off[vg + 1];
        for (int base = ei0; base < ei1; base += kInc) {
            int ev4[kInc][4], ee[kInc], er[kInc];
#pragma unroll
            for (int j = 0; j < kInc; j++) {
                const int code = base + j < ei1 ? a.vedge[base + j] : a.vedge[ei0];
                ee[j] = (code >> 2) - e0;
                er[j] = code & 3;
            }
#pragma unroll
            for (int j = 0; j < kInc; j++)
#pragma unroll
                for (int q = 0; q < 4; q++) ev4[j][q] = a.hinge[q * NE + e0 + ee[j]] - v0;
#pragma unroll
            for (int j = 0; j < kInc; j++) {
                if (base + j >= ei1) break;
                const int e = ee[j];
                edge_term(P(ev4[j][0]), P(ev4[j][1]), P(ev4[j][2]), P(ev4[j][3]), er[j], (double)eco[2 * e],
                          (double)eco[2 * e + 1], fx, fy, fz);
            }
        }
        FE[vg] = R(fx);
        FE[NV + vg] = R(fy);
        FE[2 * NV + vg] = R(fz);
    }
}

// Marked tiles -> dense list.  Each thread reads the flags of 16 tiles with
// one 16-byte load; the block scans its counts and reserves its slots with a
// single atomic, so the list length costs one atomic per 4096 tiles.
constexpr int kCompactThreads = 256, kCompactPerThread = 16;
__global__ __launch_bounds__(kCompactThreads) void k_compact(const uint8_t *__restrict__ tneed, int ntiles,
                                                             uint32_t *__restrict__ tlist, uint32_t *tcount) {
    __shared__ uint32_t wsum[kCompactThreads / 64];
    __shared__ uint32_t base_s;
    const int t0 = (blockIdx.x * kCompactThreads + threadIdx.x) * kCompactPerThread;
    uint32_t bits = 0;  // bit j: tile t0 + j is marked
    if (t0 + kCompactPerThread <= ntiles) {
        const uint4 v = *reinterpret_cast<const uint4 *>(tneed + t0);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int k = 0; k < 4; k++)
                if ((w[i] >> (8 * k)) & 0xffu) bits |= 1u << (4 * i + k);
    } else {
        for (int j = 0; j < kCompactPerThread; j++)
            if (t0 + j < ntiles && tneed[t0 + j]) bits |= 1u << j;
    }
    const uint32_t cnt = __popc(bits);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(inc, o, 64);
        if (lane >= o) inc += v;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < kCompactThreads / 64; w++) tot += wsum[w];
        base_s = tot ? atomicAdd(tcount, tot) : 0u;
    }
    __syncthreads();
    uint32_t pos = base_s + inc - cnt;
    for (int w = 0; w < wave; w++) pos += wsum[w];
    while (bits) {
        const int j = __ffs(bits) - 1;
        bits &= bits - 1;
        tlist[pos++] = (uint32_t)(t0 + j);
    }
}

struct NodeVelArgs {
    const void *f;
    int64_t stride;
    const uint8_t *cls;
    const void *gfield;
    void *ufield;  // [N] Vec4
    const uint8_t *need;
    const uint32_t *tlist;
    const uint32_t *tcount;
    const Chan *chans;
    const uint16_t *tile_chan;
    int64_t N;
    double g[3];
};

// u_ext of the marked nodes of every listed tile.  A fixed grid of waves
// strides over the list (its length is only known on the device).
template <class S, class R, bool DEV, bool HAS_G>
__global__ __launch_bounds__(256) void k_node_velocity(NodeVelArgs a) {
    using R4 = typename Vec4<R>::T;
    const int lane = threadIdx.x & 63;
    const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
    const uint32_t count = *a.tcount;
    const S *f = static_cast<const S *>(a.f);
    R4 *U = static_cast<R4 *>(a.ufield);
    for (uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < count; w += nwaves) {
        const int tile = __builtin_amdgcn_readfirstlane((int)a.tlist[w]);
        const Chan ch = a.chans[tile_channel(a.tile_chan, tile)];
        const int lt = tile - ch.toff, row = lt / ch.tpr;
        const int x = (lt - row * ch.tpr) * 64 + lane;
        if (x >= ch.nx) continue;
        const int64_t n = ch.noff + (int64_t)row * ch.nx + x;
        if (!a.need[n]) continue;
        R ux = R(0), uy = R(0), uz = R(0), rho = R(0);
        if (a.cls[n] != CLS_SOLID) {
            R v[Q];
#pragma unroll
            for (int i = 0; i < Q; i++) v[i] = R(f[i * a.stride + n]);
            R s = R(0);
#pragma unroll
            for (int i = 0; i < Q; i++) s += v[i];
            const R jx = (v[1] - v[2]) + (v[7] - v[8]) + (v[9] - v[10]) + (v[11] - v[12]) + (v[13] - v[14]);
            const R jy = (v[3] - v[4]) + (v[7] - v[8]) + (v[10] - v[9]) + (v[15] - v[16]) + (v[17] - v[18]);
            const R jz = (v[5] - v[6]) + (v[11] - v[12]) + (v[14] - v[13]) + (v[15] - v[16]) + (v[18] - v[17]);
            R Fx = R(a.g[0]), Fy = R(a.g[1]), Fz = R(a.g[2]);
            if (HAS_G) {
                const R *G = static_cast<const R *>(a.gfield);
                Fx += G[n];
                Fy += G[a.N + n];
                Fz += G[2 * a.N + n];
            }
            rho = DEV ? R(1) + s : s;
            const R ir = R(1) / rho;
            ux = (jx + R(0.5) * Fx) * ir;
            uy = (jy + R(0.5) * Fy) * ir;
            uz = (jz + R(0.5) * Fz) * ir;
        }
        U[n] = R4{ux, uy, uz, rho};
    }
}

// Contact law of the collisions (Sec. 2.4; a reading, the paper names the
// potential only): U(d) = a d^-n for d = r - roff in (0, rcut), 0 beyond,
// continued linearly below dmin.
struct ContactLaw {
    double a, n, rcut, roff, dmin;
};

// -dU/dd at surface distance d (0 beyond the cut-off)
__device__ __forceinline__ double contact_force(const ContactLaw &P, double d) {
    if (d >= P.rcut) return 0.0;
    return P.n * P.a * pow(d < P.dmin ? P.dmin : d, -P.n - 1.0);
}

__device__ __forceinline__ double min_image(double d, int L, int periodic) {
    return periodic ? d - L * floor(d / L + 0.5) : d;
}

// Walls for the contact law: planes n.x = offset (unit normal into the
// fluid) and z-axis cylinders (fluid outside), those of channel k being
// [cyl_off[k], cyl_off[k+1]) (all when cyl_off is null).
struct WallContact {
    const double *planes;    // [nplanes][4]
    const double *cyl;       // [ncyl][3] = xc, yc, R
    const int32_t *cyl_off;  // [nch+1] or null
    const double *sph;       // [nsph][4] = xc, yc, zc, R
    const int32_t *sph_start, *sph_items;  // uniform grid of the spheres: cell c holds items [start[c], start[c+1])
    int nplanes, ncyl, nsph;
    int sg[3];               // grid cells per axis
    double sinv[3];          // 1 / grid cell size per axis
    int per[3];
    ContactLaw law;
};

// Grid cell of coordinate v along an axis of length L: wrapped into
// [0, L) along a periodic axis, clamped to the grid at the faces of a
// non-periodic one (so a cell's neighbours still hold every sphere within
// one cell size).
__device__ __forceinline__ int grid_cell(double v, double L, int per, double inv, int g) {
    if (per) v -= L * floor(v / L);
    const double q = floor(v * inv);
    return q < 0.0 ? 0 : (q >= (double)g ? g - 1 : (int)q);
}

// Wall contact force on a point at absolute position (px, py, pz) of
// channel `chan` (distances with the minimum image across periodic axes).
__device__ __forceinline__ void wall_force(const WallContact &w, int chan, const Chan &ch, double px, double py,
                                           double pz, double &fx, double &fy, double &fz) {
    fx = fy = fz = 0.0;
    for (int p = 0; p < w.nplanes; p++) {
        const double *pl = w.planes + 4 * p;
        const double f = contact_force(w.law, pl[0] * px + pl[1] * py + pl[2] * pz - pl[3] - w.law.roff);
        fx += f * pl[0];
        fy += f * pl[1];
        fz += f * pl[2];
    }
    const int c0 = w.cyl_off ? w.cyl_off[chan] : 0, c1 = w.cyl_off ? w.cyl_off[chan + 1] : w.ncyl;
    for (int q = c0; q < c1; q++) {
        const double *cy = w.cyl + 3 * q;
        const double dx = min_image(px - cy[0], ch.nx, w.per[0]), dy = min_image(py - cy[1], ch.ny, w.per[1]);
        const double rho = sqrt(dx * dx + dy * dy);
        if (rho == 0.0) continue;
        const double f = contact_force(w.law, rho - cy[2] - w.law.roff) / rho;
        fx += f * dx;
        fy += f * dy;
    }
    if (w.nsph == 0) return;
    // spheres in the 3 x 3 x 3 grid cells around the point (every cell once
    // along an axis of fewer than 3 cells)
    const double Ld[3] = {(double)ch.nx, (double)ch.ny, (double)ch.nz};
    const double pv[3] = {px, py, pz};
    int lo[3], cnt[3], ci[3];
    for (int d = 0; d < 3; d++) {
        ci[d] = grid_cell(pv[d], Ld[d], w.per[d], w.sinv[d], w.sg[d]);
        if (w.sg[d] < 3) {
            lo[d] = 0;
            cnt[d] = w.sg[d];
        } else if (w.per[d]) {
            lo[d] = ci[d] - 1;
            cnt[d] = 3;
        } else {
            lo[d] = ci[d] > 0 ? ci[d] - 1 : 0;
            cnt[d] = min(ci[d] + 1, w.sg[d] - 1) - lo[d] + 1;
        }
    }
    for (int a = 0; a < cnt[2]; a++) {
        const int cz = (lo[2] + a + w.sg[2]) % w.sg[2];
        for (int b = 0; b < cnt[1]; b++) {
            const int cyy = (lo[1] + b + w.sg[1]) % w.sg[1];
            for (int e = 0; e < cnt[0]; e++) {
                const int cx = (lo[0] + e + w.sg[0]) % w.sg[0];
                const int cell = cx + w.sg[0] * (cyy + w.sg[1] * cz);
                for (int it = w.sph_start[cell]; it < w.sph_start[cell + 1]; it++) {
                    const double *sp = w.sph + 4 * w.sph_items[it];
                    const double dx = min_image(px - sp[0], ch.nx, w.per[0]);
                    const double dy = min_image(py - sp[1], ch.ny, w.per[1]);
                    const double dz = min_image(pz - sp[2], ch.nz, w.per[2]);
                    const double r = sqrt(dx * dx + dy * dy + dz * dz);
                    if (r == 0.0) continue;
                    const double f = contact_force(w.law, r - sp[3] - w.law.roff) / r;
                    fx += f * dx;
                    fy += f * dy;
                    fz += f * dz;
                }
            }
        }
    }
}

// Spread record of one IB point: its stencil's base node, fractional
// offsets, and the force it exerts on the fluid (-F_c).
template <class R>
struct SRec {
    uint32_t base;
    R dx, dy, dz, fx, fy, fz;
};

struct CoupleArgs {
    const void *ufield;  // [N] Vec4
    void *srec;          // [nverts] SRec
    const Chan *chans;
    const int32_t *cell_chan;
    const int32_t *vert_off, *anchor;
    double *x;
    void *v;
    const void *f_el;
    const double *avert;
    int ncells, nverts;
    double xi, dt_over_m, dt;
    WallContact wall;  // nplanes = ncyl = 0: no wall contact forces
};

template <class R>
__global__ __launch_bounds__(128) void k_couple(CoupleArgs a) {
    using R4 = typename Vec4<R>::T;
    const int c = blockIdx.y;
    const int vb = a.vert_off[c], ve = a.vert_off[c + 1];
    const int k = vb + blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ve) return;
    const int NV = a.nverts;
    double *X = a.x;
    R *Vv = static_cast<R *>(a.v);
    const R *FE = static_cast<const R *>(a.f_el);
    const R4 *U = static_cast<const R4 *>(a.ufield);
    const double ox = X[k], oy = X[NV + k], oz = X[2 * NV + k];
    const double flx = floor(ox), fly = floor(oy), flz = floor(oz);
    const R dx = R(ox - flx), dy = R(oy - fly), dz = R(oz - flz);
    const Chan ch = a.chans[cell_channel(a.cell_chan, c)];
    const int x0 = pmod(a.anchor[c] + (int)flx, ch.nx);
    const int y0 = pmod(a.anchor[a.ncells + c] + (int)fly, ch.ny);
    const int z0 = pmod(a.anchor[2 * a.ncells + c] + (int)flz, ch.nz);
    const int xs[2] = {x0, x0 + 1 == ch.nx ? 0 : x0 + 1};
    const int ys[2] = {y0, y0 + 1 == ch.ny ? 0 : y0 + 1};
    const int zs[2] = {z0, z0 + 1 == ch.nz ? 0 : z0 + 1};
    const R wx[2] = {R(1) - dx, dx}, wy[2] = {R(1) - dy, dy}, wz[2] = {R(1) - dz, dz};

    // step 1: interpolate u_ext
    R ux = R(0), uy = R(0), uz = R(0);
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int bx = q & 1, by = (q >> 1) & 1, bz = q >> 2;
        const int64_t n = ch.noff + xs[bx] + (int64_t)ch.nx * (ys[by] + (int64_t)ch.ny * zs[bz]);
        const R wt = wx[bx] * wy[by] * wz[bz];
        const R4 u = U[n];
        ux += wt * u.x;
        uy += wt * u.y;
        uz += wt * u.z;
    }
    // step 2: coupling force, friction per unit area times the vertex's area
    const double ak = a.avert[k];
    const R vx = Vv[k], vy = Vv[NV + k], vz = Vv[2 * NV + k];
    const R xi = R(a.xi * ak);
    const R fcx = xi * (ux - vx), fcy = xi * (uy - vy), fcz = xi * (uz - vz);
    // step 3 input: the spread record
    SRec<R> *SR = static_cast<SRec<R> *>(a.srec);
    SR[k] = SRec<R>{(uint32_t)(ch.noff + x0 + (int64_t)ch.nx * (y0 + (int64_t)ch.ny * z0)), dx, dy, dz, -fcx, -fcy, -fcz};
    // step 4 (points): semi-implicit Euler with the vertex's mass; the
    // membrane force carries the wall contact force when walls are given
    R fex = FE[k], fey = FE[NV + k], fez = FE[2 * NV + k];
    if (a.wall.nplanes + a.wall.ncyl + a.wall.nsph > 0) {
        double wx_, wy_, wz_;
        wall_force(a.wall, cell_channel(a.cell_chan, c), ch, a.anchor[c] + ox, a.anchor[a.ncells + c] + oy,
                   a.anchor[2 * a.ncells + c] + oz, wx_, wy_, wz_);
        fex += R(wx_);
        fey += R(wy_);
        fez += R(wz_);
    }
    const R h = R(a.dt_over_m / ak);
    const R nvx = vx + h * (fex + fcx), nvy = vy + h * (fey + fcy), nvz = vz + h * (fez + fcz);
    Vv[k] = nvx;
    Vv[NV + k] = nvy;
    Vv[2 * NV + k] = nvz;
    X[k] = ox + a.dt * (double)nvx;
    X[NV + k] = oy + a.dt * (double)nvy;
    X[2 * NV + k] = oz + a.dt * (double)nvz;
}

constexpr int kSpreadThreads = 512;
constexpr int kSpreadMaxPoints = 2048;  // per cell (bounded by the membrane pass's LDS anyway)

struct SpreadArgs {
    const int32_t *vert_off;
    const void *srec;
    uint32_t *owner;   // [N] epoch of the call that last claimed the base node's slot
    void *cslot;       // [N][8] Vec4: corner contributions of a base node
    uint8_t *role;     // [N][8] role[n][q] = 1: base node of n in role q holds a slot
    void *facc;        // [N] Vec4: accumulator of the fallback (zero between steps)
    uint8_t *ftile;    // [ntiles] 1: a node of the tile got fallback atomics this call
    const uint32_t *epoch;
    const Chan *chans;
    const int32_t *cell_chan;
};

template <class R>
__global__ __launch_bounds__(kSpreadThreads) void k_spread_cells(SpreadArgs a) {
    using R4 = typename Vec4<R>::T;
    __shared__ unsigned long long key[kSpreadMaxPoints];
    const int c = blockIdx.x;
    const int v0 = a.vert_off[c], nv = a.vert_off[c + 1] - v0;
    int P = 64;
    while (P < nv) P <<= 1;
    const SRec<R> *SR = static_cast<const SRec<R> *>(a.srec) + v0;
    for (int i = threadIdx.x; i < P; i += blockDim.x)
        key[i] = i < nv ? ((unsigned long long)SR[i].base << 32) | (unsigned)i : ~0ull;
    __syncthreads();
    // bitonic sort of (base node, point) keys
    for (int kk = 2; kk <= P; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long ki = key[i], kl = key[l];
                    const bool up = (i & kk) == 0;
                    if ((ki > kl) == up) {
                        key[i] = kl;
                        key[l] = ki;
                    }
                }
            }
            __syncthreads();
        }
    // one thread per run of equal base nodes
    R4 *CS = static_cast<R4 *>(a.cslot);
    const uint32_t epoch = *a.epoch;
    const Chan ch = a.chans[cell_channel(a.cell_chan, c)];
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        const uint32_t b = (uint32_t)(key[i] >> 32);
        if (i > 0 && (uint32_t)(key[i - 1] >> 32) == b) continue;
        R F[8][3];
#pragma unroll
        for (int q = 0; q < 8; q++) F[q][0] = F[q][1] = F[q][2] = R(0);
        for (int j = i; j < nv && (uint32_t)(key[j] >> 32) == b; j++) {
            const SRec<R> r = SR[(uint32_t)key[j]];
            const R wx[2] = {R(1) - r.dx, r.dx}, wy[2] = {R(1) - r.dy, r.dy}, wz[2] = {R(1) - r.dz, r.dz};
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const R wt = wx[q & 1] * wy[(q >> 1) & 1] * wz[q >> 2];
                F[q][0] += wt * r.fx;
                F[q][1] += wt * r.fy;
                F[q][2] += wt * r.fz;
            }
        }
        // claim the base node's slot for this call
        uint32_t old = a.owner[b];
        bool won = false;
        while (old != epoch) {
            const uint32_t seen = atomicCAS(&a.owner[b], old, epoch);
            if (seen == old) {
                won = true;
                break;
            }
            old = seen;
        }
        const int64_t lb = (int64_t)b - ch.noff;
        const int bx = (int)(lb % ch.nx), by = (int)((lb / ch.nx) % ch.ny), bz = (int)(lb / ((int64_t)ch.nx * ch.ny));
        const int xs[2] = {bx, bx + 1 == ch.nx ? 0 : bx + 1};
        const int ys[2] = {by, by + 1 == ch.ny ? 0 : by + 1};
        const int zs[2] = {bz, bz + 1 == ch.nz ? 0 : bz + 1};
        if (won) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                CS[(size_t)b * 8 + q] = R4{F[q][0], F[q][1], F[q][2], R(0)};
                const int64_t n = ch.noff + xs[q & 1] + (int64_t)ch.nx * (ys[(q >> 1) & 1] + (int64_t)ch.ny * zs[q >> 2]);
                a.role[n * 8 + q] = 1;
            }
        } else {
            R4 *FI = static_cast<R4 *>(a.facc);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int ys_ = ys[(q >> 1) & 1], zs_ = zs[q >> 2];
                const int64_t n = ch.noff + xs[q & 1] + (int64_t)ch.nx * (ys_ + (int64_t)ch.ny * zs_);
                R *rec = reinterpret_cast<R *>(&FI[n]);
                atomicAdd(rec + 0, F[q][0]);
                atomicAdd(rec + 1, F[q][1]);
                atomicAdd(rec + 2, F[q][2]);
                a.ftile[ch.toff + (int64_t)(ys_ + ch.ny * zs_) * ch.tpr + (xs[q & 1] >> 6)] = 1;
            }
        }
    }
}

struct GatherArgs {
    const uint32_t *tlist, *tcount;
    uint8_t *role;   // [N][8], cleared here
    const void *cslot;
    const uint8_t *need;
    uint8_t *ftile;  // [ntiles] fallback flags, cleared here
    void *fibm;      // [N] Vec4: spread force, written (or, with `accumulate`, added) at the nodes this call spreads to
    void *facc;      // [N] Vec4: fallback accumulator, read and cleared in flagged tiles
    int accumulate;  // as in MembArgs
    const Chan *chans;
    const uint16_t *tile_chan;
};

// Each listed tile: every lane reads its node's 8 role bytes with one load
// (zero away from the stencils), adds the flagged slots in a fixed order and
// stores the sum as the node's spread force.  Every node marked by the
// call's membrane gets a slot role or sits in a tile the fallback path
// flagged, so the force is written at every marked node and the
// collide-stream pass never needs the record cleared.  Only in a flagged tile
// does the sum go on top of the accumulated atomics, which are read and
// cleared; with `accumulate` (a second membrane coupled in the same step)
// it is added to the force already there.  The common chain is list -> role
// word -> slots -> store.
template <class R>
__global__ __launch_bounds__(256) void k_gather_nodes(GatherArgs a) {
    using R4 = typename Vec4<R>::T;
    const int lane = threadIdx.x & 63;
    const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
    const uint32_t count = *a.tcount;
    const R4 *CS = static_cast<const R4 *>(a.cslot);
    R4 *FI = static_cast<R4 *>(a.fibm);
    for (uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < count; w += nwaves) {
        const int tile = __builtin_amdgcn_readfirstlane((int)a.tlist[w]);
        const Chan ch = a.chans[tile_channel(a.tile_chan, tile)];
        const bool fallback = __builtin_amdgcn_readfirstlane((int)a.ftile[tile]) != 0;
        const int lt = tile - ch.toff, row = lt / ch.tpr;
        const int x = (lt - row * ch.tpr) * 64 + lane;
        if (fallback && lane == 0) a.ftile[tile] = 0;
        if (x >= ch.nx) continue;
        const int64_t n = ch.noff + (int64_t)row * ch.nx + x;
        unsigned long long *rp = reinterpret_cast<unsigned long long *>(a.role) + n;
        const unsigned long long roles = *rp;
        R Fx = R(0), Fy = R(0), Fz = R(0);
        if (roles) {
            *rp = 0ull;
            const int y = row % ch.ny, z = row / ch.ny;
            const int xb[2] = {x, x == 0 ? ch.nx - 1 : x - 1};
            const int yb[2] = {y, y == 0 ? ch.ny - 1 : y - 1};
            const int zb[2] = {z, z == 0 ? ch.nz - 1 : z - 1};
            // node n is corner q of base node (x - qx, y - qy, z - qz)
#pragma unroll
            for (int q = 0; q < 8; q++) {
                if (!((roles >> (8 * q)) & 0xffull)) continue;
                const int64_t b =
                    ch.noff + xb[q & 1] + (int64_t)ch.nx * (yb[(q >> 1) & 1] + (int64_t)ch.ny * zb[q >> 2]);
                const R4 f = CS[b * 8 + q];
                Fx += f.x;
                Fy += f.y;
                Fz += f.z;
            }
        }
        if (fallback) {
            if (!a.need[n]) continue;
            R4 *FA = static_cast<R4 *>(a.facc);
            const R4 f = FA[n];
            FA[n] = R4{R(0), R(0), R(0), R(0)};
            Fx += f.x;
            Fy += f.y;
            Fz += f.z;
        } else if (!roles) {
            continue;
        }
        if (a.accumulate) {
            const R4 f = FI[n];
            Fx = f.x + Fx;
            Fy = f.y + Fy;
            Fz = f.z + Fz;
        }
        FI[n] = R4{Fx, Fy, Fz, R(0)};
    }
}

}  // namespace lbm

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
// couple_record (per IB point, inside the spread's workgroup of its cell):
//   trilinear interpolation of that field (Sec. 2.2 step 1) and the
//   coupling force (step 2), as a spread record: the stencil's base node,
//   fractional offsets and the force the point exerts on the fluid (-F_c).
//
// k_move (one thread per IB point, after the spread and the membrane
//   kernel): the point update (step 4) with the membrane force and F_c.
//
// Spreading (step 3) avoids per-contribution float atomics, which run at a
// small fraction of store throughput on this GPU:
// k_spread_cells (one workgroup per cell) computes each point's record
//   (interpolated velocity, coupling force: couple_record, also written out
//   for the point update), sorts the records by base
//   node in LDS, finds the cell's stencil nodes in a bitmap over the box of
//   its base nodes and, one thread per node, sums the node's contributions
//   in a fixed order, claims the node with one atomic exchange of the
//   call's epoch and writes the sum as the node's spread force.  A node
//   already claimed by another cell in this call (two membranes within a
//   lattice spacing) falls back to float atomics into a separate
//   accumulator, kept zero between steps, and flags its tile; the
//   collide-stream pass adds that accumulator at the flagged tiles' marked
//   nodes and clears it.
// All sums except the fallback's are in a fixed order, so the spread is
// bit-reproducible.
//
// The node and tile marks stay set until the collide-stream pass: they are
// exactly the nodes whose spread force the call wrote this step, so that
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
    // stencil nodes whose populations the last collide-stream pass recorded
    // (bit x & 63 of word tile); a marked node outside them sets *miss.
    // Null when the step does not use the records.
    const uint4 *cover;  // RecTile entries (mask in x, y)
    uint32_t *miss;
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
            const int64_t tile = ch.toff + (int64_t)row * ch.tpr + (xs[e] >> 6);
            if (a.cover) {
                const uint4 ce = a.cover[tile];
                if (!((((uint64_t)ce.y << 32 | ce.x) >> (xs[e] & 63)) & 1ull)) *a.miss = 1u;
            }
            // the two x of a row share a tile unless the pair crosses a tile edge
            if (e == 0 || (xs[1] >> 6) != (xs[0] >> 6)) a.tneed[tile] = 1;
        }
    }
}

// Reset of the tile-list length and advance of the claim epoch for a step.
__device__ __forceinline__ void start_marks(const MarkArgs &a) {
    *a.tcount = 0;
    *a.epoch += 1u;
}

// The stencil marks of every point (positions of this step) on their own:
// one thread per point (cell and chunk from the workgroup index as below).  Independent of the membrane
// forces, so the velocity pass that reads the marks can run beside the
// membrane kernel.
// Workgroups go to the 8 XCDs round-robin by index.  For the per-point
// kernels this mapping keeps all nb chunks of a cell on one XCD, so that
// the lines the cell's points share (partially written marks, gathered
// velocities) live in one L2: workgroup L takes cell 8 (L / 8nb) + L % 8
// and chunk (L / 8) % nb (grid: nb * ncells rounded up to 8).
__device__ __forceinline__ void xcd_cell_chunk(int L, int nb, int &c, int &chunk) {
    c = (L / (8 * nb)) * 8 + (L & 7);
    chunk = (L >> 3) % nb;
}

template <class R>
__global__ __launch_bounds__(128) void k_mark(MarkArgs a, int nb) {
    const int L = blockIdx.x;
    int c, chunk;
    xcd_cell_chunk(L, nb, c, chunk);
    if (L == 0 && threadIdx.x == 0) start_marks(a);
    if (c >= a.ncells) return;
    const int v0 = a.vert_off[c], k = chunk * blockDim.x + threadIdx.x;
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
// With `gate`, nothing is listed unless *gate is non-zero (a step whose
// velocities come from records lists tiles only when a node was missed).
__global__ __launch_bounds__(kCompactThreads) void k_compact(const uint8_t *__restrict__ tneed, int ntiles,
                                                             uint32_t *__restrict__ tlist, uint32_t *tcount,
                                                             const uint32_t *gate) {
    __shared__ uint32_t wsum[kCompactThreads / 64];
    __shared__ uint32_t base_s;
    if (gate && *gate == 0u) return;
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
    const uint32_t *links;
    int per[3];
    const void *gfield;
    void *ufield;  // [N] Vec4
    const uint8_t *need;  // [N] node marks (0 or 1)
    const uint4 *tmask;   // [ntiles] solid and wall masks of each tile
    uint2 *tnmask;        // [ntiles] written for every listed tile: its node marks as a 64-bit mask
    const uint32_t *tlist;
    const uint32_t *tcount;
    const Chan *chans;
    const uint16_t *tile_chan;
    int64_t N;
    double g[3];
};

// u_ext = (j + F_ext/2)/rho and rho of a fluid node from its 19
// populations v (deviations in DEV), F_ext = g + G(n).  Both velocity passes
// use this one sequence of operations, so they give the same bits.
template <class R, bool DEV, bool HAS_G>
__device__ __forceinline__ typename Vec4<R>::T node_u(const R (&v)[Q], const double (&g)[3], const void *gfield,
                                                      int64_t N, int64_t n) {
    R s = R(0);
#pragma unroll
    for (int i = 0; i < Q; i++) s += v[i];
    const R jx = (v[1] - v[2]) + (v[7] - v[8]) + (v[9] - v[10]) + (v[11] - v[12]) + (v[13] - v[14]);
    const R jy = (v[3] - v[4]) + (v[7] - v[8]) + (v[10] - v[9]) + (v[15] - v[16]) + (v[17] - v[18]);
    const R jz = (v[5] - v[6]) + (v[11] - v[12]) + (v[14] - v[13]) + (v[15] - v[16]) + (v[18] - v[17]);
    R Fx = R(g[0]), Fy = R(g[1]), Fz = R(g[2]);
    if (HAS_G) {
        const R *G = static_cast<const R *>(gfield);
        Fx += G[n];
        Fy += G[N + n];
        Fz += G[2 * N + n];
    }
    const R rho = DEV ? R(1) + s : s;
    const R ir = R(1) / rho;
    return typename Vec4<R>::T{(jx + R(0.5) * Fx) * ir, (jy + R(0.5) * Fy) * ir, (jz + R(0.5) * Fz) * ir, rho};
}

// Four mark bytes (each 0 or 1) -> four bits.
__device__ __forceinline__ uint32_t mark_nibble(uint32_t w) { return (w | w >> 7 | w >> 14 | w >> 21) & 0xfu; }

// u_ext of the marked nodes of every listed tile, and the tile's marks as a
// 64-bit mask (bit x & 63) for the collide-stream pass.  What a wave needs to
// know of its tile comes in scalar loads (the list entry, the channel, the
// solid and wall masks, and the 64 mark bytes of a whole tile that starts on
// a 4-byte boundary; a vector load and a ballot otherwise), so the 19 loads
// of its marked nodes are issued at once.  A fixed grid of waves strides
// over the list (its length is only known on the device).
template <class S, class R, bool DEV, bool HAS_G>
__global__ __launch_bounds__(256) void k_node_velocity(NodeVelArgs a) {
    using R4 = typename Vec4<R>::T;
    struct Marks {
        uint32_t w[16];
    };
    const int lane = threadIdx.x & 63;
    const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
    const uint32_t count = *a.tcount;
    const S *f = static_cast<const S *>(a.f);
    R4 *U = static_cast<R4 *>(a.ufield);
    for (uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < count; w += nwaves) {
        const int tile = (int)uniform_load(a.tlist, __builtin_amdgcn_readfirstlane((int)w));
        const Chan ch = uniform_load(a.chans, tile_channel(a.tile_chan, tile));
        const uint4 tm = uniform_load(a.tmask, tile);
        const int lt = tile - ch.toff, row = lt / ch.tpr, x0 = (lt - row * ch.tpr) * 64;
        const int x = x0 + lane;
        const int64_t n0 = ch.noff + (int64_t)row * ch.nx + x0, n = n0 + lane;
        uint64_t mk;
        if (x0 + 64 <= ch.nx && (n0 & 3) == 0) {
            const Marks b = uniform_load(reinterpret_cast<const Marks *>(a.need + n0), 0);
            mk = 0;
#pragma unroll
            for (int k = 0; k < 16; k++) mk |= (uint64_t)mark_nibble(b.w[k]) << (4 * k);
        } else {
            mk = __builtin_amdgcn_ballot_w64(x < ch.nx && a.need[n]);
        }
        if (lane == 0) a.tnmask[tile] = uint2{(uint32_t)mk, (uint32_t)(mk >> 32)};
        if (!((mk >> lane) & 1u)) continue;  // unmarked (or past the row's end)
        R4 u = R4{R(0), R(0), R(0), R(0)};
        if (!((((uint64_t)tm.y << 32 | tm.x) >> lane) & 1u)) {  // fluid
            const bool wall = (((uint64_t)tm.w << 32 | tm.z) >> lane) & 1u;
            const uint32_t lk = wall ? a.links[n] : 0u;
            R v[Q];
#pragma unroll
            for (int i = 0; i < Q; i++) v[i] = R(f[i * a.stride + n]);
            if (lk) {  // populations bounced back from solid neighbours lie in their slots
                const int y = row % ch.ny, z = row / ch.ny;
#pragma unroll
                for (int i = 0; i < Q; i++)
                    if ((lk >> opp(i)) & 1u) v[i] = R(f[pop_slot<int64_t>(i, n, lk, x, y, z, ch, a.stride, a.per)]);
            }
            u = node_u<R, DEV, HAS_G>(v, a.g, a.gfield, a.N, n);
        }
        U[n] = u;
    }
}

// Records of the next step's stencil nodes.  The point update marks the
// stencil of every point's new position (nx_need, nx_tneed); before the
// collide-stream pass, k_next_list turns the marks into one entry per tile
// (RecTile: a 64-bit mask, bit x & 63 set for a marked node, and the first
// slot of the tile's range; slots are numbered in bit order)
// and lists each slot's node; the pass then writes, beside every
// population it streams into a marked node, a copy into the record
// rec[i * cap + slot].  The next step's velocity pass reads a marked node's
// 19 populations there, 64 consecutive slots per wave, instead of the 19
// planes of the lattice (whole lines of every plane for the few marked
// nodes of a tile).  Requires every channel's nx to be a multiple of 64.
struct NextListArgs {
    uint8_t *nx_need;     // [N] next-step marks, cleared here
    uint8_t *nx_tneed;    // [ntiles] tile marks, cleared here
    uint4 *ent;           // [ntiles] RecTile, written for every tile (mask 0 when unmarked or beyond the capacity)
    uint32_t *node;       // [cap] node of each slot
    uint32_t *count;      // slots handed out (zeroed by the point update before)
    uint32_t *miss;       // zeroed here: set by the next step's marking when a marked node is not recorded
    const Chan *chans;
    const uint16_t *tile_chan;
    int ntiles;
    int64_t cap;
};

constexpr int kNextListThreads = 256, kNextListPer = 4;  // tiles per thread
__global__ __launch_bounds__(kNextListThreads) void k_next_list(NextListArgs a) {
    __shared__ uint32_t wsum[kNextListThreads / 64];
    __shared__ uint32_t base_s;
    const int t0 = (blockIdx.x * kNextListThreads + threadIdx.x) * kNextListPer;
    if (t0 == 0) *a.miss = 0u;
    uint64_t m[kNextListPer];
    int64_t node0[kNextListPer];
    uint32_t cnt = 0;
#pragma unroll
    for (int j = 0; j < kNextListPer; j++) {
        const int t = t0 + j;
        m[j] = 0;
        node0[j] = 0;
        if (t < a.ntiles && a.nx_tneed[t]) {
            const Chan ch = a.chans[a.tile_chan ? (int)a.tile_chan[t] : 0];
            const int lt = t - ch.toff, row = lt / ch.tpr;
            node0[j] = ch.noff + (int64_t)row * ch.nx + (int64_t)(lt - row * ch.tpr) * 64;
            uint4 *b = reinterpret_cast<uint4 *>(a.nx_need + node0[j]);  // 64 bytes, 64-byte aligned (nx % 64 == 0)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const uint4 v = b[q];
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int k = 0; k < 4; k++)
                        if ((w[i] >> (8 * k)) & 0xffu) m[j] |= 1ull << (16 * q + 4 * i + k);
                b[q] = uint4{0u, 0u, 0u, 0u};
            }
            a.nx_tneed[t] = 0;
        }
        cnt += (uint32_t)__popcll(m[j]);
    }
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
        for (int w = 0; w < kNextListThreads / 64; w++) tot += wsum[w];
        base_s = tot ? atomicAdd(a.count, tot) : 0u;
    }
    __syncthreads();
    uint32_t pos = base_s + inc - cnt;
    for (int w = 0; w < wave; w++) pos += wsum[w];
#pragma unroll
    for (int j = 0; j < kNextListPer; j++) {
        const int t = t0 + j;
        if (t >= a.ntiles) break;
        uint64_t mj = m[j];
        const uint32_t cj = (uint32_t)__popcll(mj);
        // a tile whose range would pass the capacity is left out (its nodes
        // are not recorded; the next step finds them uncovered and gathers them)
        if ((int64_t)pos + cj > a.cap) mj = 0;
        a.ent[t] = uint4{(uint32_t)mj, (uint32_t)(mj >> 32), pos, 0u};
        uint32_t p = pos;
        while (mj) {
            const int b = __ffsll((unsigned long long)mj) - 1;
            mj &= mj - 1;
            a.node[p++] = (uint32_t)(node0[j] + b);
        }
        pos += cj;
    }
}

struct VelRecArgs {
    const void *rec;       // [19][cap] storage type
    int64_t cap;
    const uint32_t *node;  // [cap]
    const uint32_t *count;
    const uint8_t *cls;
    const void *gfield;
    void *ufield;          // [N] Vec4
    int64_t N;
    double g[3];
};

// u_ext of every recorded node from its record, one thread per slot (a
// fixed grid strides over the slots, whose number is known on the device).
// The 19 record loads of a slot go out together with its node's, before
// the node's class is known (a solid node's record is never written and its
// velocity is 0 whatever the loads return).
template <class S, class R, bool DEV, bool HAS_G>
__global__ __launch_bounds__(256) void k_velocity_records(VelRecArgs a) {
    using R4 = typename Vec4<R>::T;
    const uint32_t count = *a.count;
    const __amdgpu_buffer_rsrc_t rr = buf_rsrc(a.rec, (uint64_t)Q * (uint64_t)a.cap * sizeof(S));
    R4 *U = static_cast<R4 *>(a.ufield);
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < count; s += gridDim.x * blockDim.x) {
        R v[Q];
#pragma unroll
        for (int i = 0; i < Q; i++)
            v[i] = R(buf_load<S>(rr, s * (uint32_t)sizeof(S), (uint32_t)i * (uint32_t)a.cap * (uint32_t)sizeof(S)));
        const uint32_t n = a.node[s];
        R4 u = node_u<R, DEV, HAS_G>(v, a.g, a.gfield, a.N, n);
        if (a.cls[n] == CLS_SOLID) u = R4{R(0), R(0), R(0), R(0)};
        U[n] = u;
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
    int nb;            // point chunks of 128 per cell (workgroup mapping as for k_mark)
    // marks of the next step's stencils (the new positions), or null
    uint8_t *nx_need, *nx_tneed;
    uint32_t *nx_count;  // zeroed here (read before by this step's velocity pass, counted next by k_next_list)
};

// Steps 1-2 of point k of cell c and the input of step 3: the interpolated
// velocity, the coupling force F_c = xi A_k (u_k - V_k), and the spread
// record (base node, fractional offsets, -F_c).  The membrane force is not
// needed here, so this runs while the membrane kernel is still at work.
template <class R>
__device__ __forceinline__ SRec<R> couple_record(const CoupleArgs &a, int c, int k, const Chan &ch) {
    using R4 = typename Vec4<R>::T;
    const int NV = a.nverts;
    const double *X = a.x;
    const R *Vv = static_cast<const R *>(a.v);
    const R4 *U = static_cast<const R4 *>(a.ufield);
    const double ox = X[k], oy = X[NV + k], oz = X[2 * NV + k];
    const double flx = floor(ox), fly = floor(oy), flz = floor(oz);
    const R dx = R(ox - flx), dy = R(oy - fly), dz = R(oz - flz);
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
    return SRec<R>{(uint32_t)(ch.noff + x0 + (int64_t)ch.nx * (y0 + (int64_t)ch.ny * z0)), dx, dy, dz, -fcx, -fcy, -fcz};
}

// Step 4 of a point (semi-implicit Euler with the vertex's mass), once the
// membrane force is there: the coupling force is read back from the spread
// record (negated, exactly), the wall contact force added when walls are
// given; then, with next-step marks, the stencil of the new position is
// marked.  Workgroup index -> (cell, chunk) as for k_mark.
template <class R>
__global__ __launch_bounds__(128) void k_move(CoupleArgs a) {
    int c, chunk;
    xcd_cell_chunk(blockIdx.x, a.nb, c, chunk);
    if (c >= a.ncells) return;
    const int vb = a.vert_off[c], ve = a.vert_off[c + 1];
    const int k = vb + chunk * blockDim.x + threadIdx.x;
    if (k >= ve) return;
    const int NV = a.nverts;
    double *X = a.x;
    R *Vv = static_cast<R *>(a.v);
    const R *FE = static_cast<const R *>(a.f_el);
    const SRec<R> r = static_cast<const SRec<R> *>(a.srec)[k];
    const R fcx = -r.fx, fcy = -r.fy, fcz = -r.fz;
    const double ox = X[k], oy = X[NV + k], oz = X[2 * NV + k];
    const double ak = a.avert[k];
    const R vx = Vv[k], vy = Vv[NV + k], vz = Vv[2 * NV + k];
    const Chan ch = a.chans[cell_channel(a.cell_chan, c)];
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
    const double qx = ox + a.dt * (double)nvx, qy = oy + a.dt * (double)nvy, qz = oz + a.dt * (double)nvz;
    X[k] = qx;
    X[NV + k] = qy;
    X[2 * NV + k] = qz;
    if (a.nx_need) {  // the next step's stencil of the new position
        const int x1 = pmod(a.anchor[c] + (int)floor(qx), ch.nx);
        const int y1 = pmod(a.anchor[a.ncells + c] + (int)floor(qy), ch.ny);
        const int z1 = pmod(a.anchor[2 * a.ncells + c] + (int)floor(qz), ch.nz);
        const int xn[2] = {x1, x1 + 1 == ch.nx ? 0 : x1 + 1};
        const int yn[2] = {y1, y1 + 1 == ch.ny ? 0 : y1 + 1};
        const int zn[2] = {z1, z1 + 1 == ch.nz ? 0 : z1 + 1};
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int row = yn[q & 1] + ch.ny * zn[q >> 1];
#pragma unroll
            for (int e = 0; e < 2; e++) {
                a.nx_need[ch.noff + (int64_t)row * ch.nx + xn[e]] = 1;
                if (e == 0 || (xn[1] >> 6) != (xn[0] >> 6)) a.nx_tneed[ch.toff + (int64_t)row * ch.tpr + (xn[e] >> 6)] = 1;
            }
        }
    }
}

constexpr int kSpreadThreads = 512;
constexpr int kSpreadMaxPoints = 2048;  // per cell (bounded by the membrane pass's LDS anyway)
constexpr int kSpreadBox = 16384;       // nodes of the largest per-cell box of base nodes kept in LDS
static_assert(kSpreadBox / 32 <= kSpreadThreads, "the spread scans one bitmap word per thread");

struct SpreadArgs {
    const int32_t *vert_off;
    void *srec;        // [nverts] SRec, written here for the point update
    uint32_t *owner;   // [N] epoch of the call that last claimed the node
    void *fibm;        // [N] Vec4: spread force, written (with `accumulate`, added) at the nodes a cell claims
    void *facc;        // [N] Vec4: accumulator of the fallback (zero between steps)
    uint8_t *ftile;    // [ntiles] 1: a node of the tile got fallback atomics (cleared by the collide-stream pass)
    const uint32_t *epoch;
    const Chan *chans;
    const int32_t *cell_chan;
    int accumulate;    // as in MarkArgs
    int pmax;          // power of two >= the largest cell's point count (>= 64)
    int maxv;          // the largest cell's point count
    CoupleArgs cp;     // inputs of the points' interpolation and coupling force (couple_record)
};

// A point's offsets and force, staged in LDS by the spread.
template <class R>
struct SPoint {
    R dx, dy, dz, fx, fy, fz;
};

// q = a / b and r = a % b (a >= 0, b >= 1, a < 2^50) from the reciprocal rb
// = 1/b: the estimate is within one of q, and one correction step makes both
// exact.
__device__ __forceinline__ void divmod_est(int64_t a, int b, double rb, int64_t &q, int64_t &r) {
    q = (int64_t)((double)a * rb);
    r = a - q * b;
    if (r < 0) {
        q--;
        r += b;
    } else if (r >= b) {
        q++;
        r -= b;
    }
}
// The same for a, b below 2^24 with a float reciprocal.
__device__ __forceinline__ void divmod_est(int a, int b, float rb, int &q, int &r) {
    q = (int)((float)a * rb);
    r = a - q * b;
    if (r < 0) {
        q--;
        r += b;
    } else if (r >= b) {
        q++;
        r -= b;
    }
}
// Box index li = lx + bx (ly + by lz) -> (lx, ly, lz).
__device__ __forceinline__ void box_coords(int li, int bx, int by, float rbx, float rby, int &lx, int &ly, int &lz) {
    int row;
    divmod_est(li, bx, rbx, row, lx);
    divmod_est(row, by, rby, lz, ly);
}
// v mod n for any v (one step in the usual case of v in [-n, 2n)).
__device__ __forceinline__ int wrap_to(int v, int n) {
    while (v >= n) v -= n;
    while (v < 0) v += n;
    return v;
}

// LDS of k_spread_cells: sort keys [pmax] (u32), staged points [maxv],
// their base nodes [maxv] (u32), base-node and stencil-node bitmaps over the
// box [kSpreadBox/32] (u32 each), prefix counts of the base bitmap's words
// [kSpreadBox/32] (u16), run starts [maxv] and node list [8 maxv] (u16), and
// a few scalars.
template <class R>
__host__ __device__ inline size_t spread_lds_bytes(int pmax, int maxv) {
    return 4 * (size_t)pmax + sizeof(SPoint<R>) * (size_t)maxv + 4 * (size_t)maxv + 2 * (kSpreadBox / 32) * 4 +
           (kSpreadBox / 32) * 2 + 18 * (size_t)maxv + 256;
}

// Block-wide exclusive prefix sum of one int per thread (blockDim.x <= 1024);
// `wsum` holds one int per wave.  Returns the prefix; `total` gets the sum.
__device__ __forceinline__ int block_exclusive_scan(int v, int *wsum, int &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int before = 0;
    total = 0;
    for (int w = 0; w < nw; w++) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    __syncthreads();
    return before + inc - v;
}

// Spreading, one workgroup per cell (Sec. 2.2 step 3: every point exerts
// -F_c on its 2x2x2 stencil with the trilinear weights).  The cell's base
// nodes, unwrapped around its first point, span a small box; the points
// are sorted by (base node in the box, point) in LDS; a bitmap of the base
// nodes over the box with per-word prefix counts gives each base node's
// run of points.  The stencil nodes are the set bits of a second bitmap
// over the box; each is summed by one thread, corner by
// corner and within a corner in sorted point order, claimed for this call
// with one atomic exchange of the call's epoch, and its sum written as the
// node's spread force.  A node already claimed by another cell in this
// call (membranes within a lattice spacing of each other) takes the sum as
// float atomics into a separate accumulator, kept zero between steps, and
// flags its tile for the collide-stream pass, which adds the accumulator
// at the flagged tiles' marked nodes and clears it; so does every node of a cell whose box
// exceeds kSpreadBox nodes (point by point, after its claim has set the
// node's force to zero, or kept it with `accumulate`).  Every stencil node of
// the call is written, so the collide-stream pass reads the force at the
// marked nodes without clearing.
template <class R>
__global__ __launch_bounds__(kSpreadThreads) void k_spread_cells(SpreadArgs a) {
    using R4 = typename Vec4<R>::T;
    constexpr int kWords = kSpreadBox / 32;
    extern __shared__ uint32_t smem_u32[];
    uint32_t *key = smem_u32;                                          // [pmax]
    SPoint<R> *pts = reinterpret_cast<SPoint<R> *>(key + a.pmax);     // [maxv]
    uint32_t *pbase = reinterpret_cast<uint32_t *>(pts + a.maxv);     // [maxv] the points' base nodes
    uint32_t *bbits = pbase + a.maxv;                                  // [kWords] base nodes of the cell
    uint32_t *bits = bbits + kWords;                                   // [kWords] stencil nodes
    uint16_t *wpre = reinterpret_cast<uint16_t *>(bits + kWords);     // [kWords] base bits in earlier words
    uint16_t *rstart = wpre + kWords;                                  // [maxv] first sorted index of each run
    uint16_t *nodes = rstart + a.maxv;                                 // [8 maxv]
    int *sc = reinterpret_cast<int *>(nodes + 8 * a.maxv + (a.maxv & 1));  // scalars and scan scratch
    const int c = blockIdx.x;
    const int v0 = a.vert_off[c], nv = a.vert_off[c + 1] - v0;
    if (nv <= 0) return;
    const Chan ch = a.chans[cell_channel(a.cell_chan, c)];
    SRec<R> *SR = static_cast<SRec<R> *>(a.srec) + v0;
    const uint32_t epoch = *a.epoch;
    if (a.cp.nx_count && c == 0 && threadIdx.x == 0) *a.cp.nx_count = 0u;
    R4 *FI = static_cast<R4 *>(a.fibm);
    R4 *FA = static_cast<R4 *>(a.facc);
    // node index -> coordinates in the channel (quotients from a reciprocal,
    // corrected to the exact integer ones)
    const double rnx = 1.0 / ch.nx, rny = 1.0 / ch.ny;
    auto decode = [&](uint32_t b, int &x, int &y, int &z) {
        int64_t row;
        int64_t r;
        divmod_est((int64_t)b - ch.noff, ch.nx, rnx, row, r);
        x = (int)r;
        int64_t zz;
        divmod_est(row, ch.ny, rny, zz, r);
        y = (int)r;
        z = (int)zz;
    };
    auto unwrap = [](int d, int L) {  // d mod L in (-L/2, L/2], for d in (-L, L)
        if (d < 0) d += L;
        return 2 * d > L ? d - L : d;
    };
    auto fallback_add = [&](uint32_t y, int gx, int gy, int gz, R fx, R fy, R fz) {
        R *rec = reinterpret_cast<R *>(&FA[y]);
        atomicAdd(rec + 0, fx);
        atomicAdd(rec + 1, fy);
        atomicAdd(rec + 2, fz);
        a.ftile[ch.toff + (int64_t)(gy + ch.ny * gz) * ch.tpr + (gx >> 6)] = 1;
    };
    // steps 1-2 of every point of the cell (its record kept for the point
    // update), staged in LDS
    // two points per thread at a time (the second clamped to the last point
    // and kept only when it exists), so that both points' loads are in flight
    // together
    for (int i = threadIdx.x; i < nv; i += 2 * blockDim.x) {
        const int i2 = i + blockDim.x;
        const SRec<R> r = couple_record<R>(a.cp, c, v0 + i, ch);
        const SRec<R> r2 = couple_record<R>(a.cp, c, v0 + min(i2, nv - 1), ch);
        SR[i] = r;
        pbase[i] = r.base;
        pts[i] = SPoint<R>{r.dx, r.dy, r.dz, r.fx, r.fy, r.fz};
        if (i2 < nv) {
            SR[i2] = r2;
            pbase[i2] = r2.base;
            pts[i2] = SPoint<R>{r2.dx, r2.dy, r2.dz, r2.fx, r2.fy, r2.fz};
        }
    }
    __syncthreads();
    // base nodes unwrapped around the first point's; their bounding box
    int rx, ry, rz;
    decode(pbase[0], rx, ry, rz);
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        int x, y, z;
        decode(pbase[i], x, y, z);
        const int u[3] = {unwrap(x - rx, ch.nx), unwrap(y - ry, ch.ny), unwrap(z - rz, ch.nz)};
        for (int d = 0; d < 3; d++) {
            lo[d] = min(lo[d], u[d]);
            hi[d] = max(hi[d], u[d]);
        }
    }
    for (int d = 0; d < 3; d++) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo[d] = min(lo[d], __shfl_xor(lo[d], o, 64));
            hi[d] = max(hi[d], __shfl_xor(hi[d], o, 64));
        }
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 6; d++) sc[d] = d < 3 ? INT32_MAX : INT32_MIN;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        for (int d = 0; d < 3; d++) {
            atomicMin(&sc[d], lo[d]);
            atomicMax(&sc[3 + d], hi[d]);
        }
    __syncthreads();
    const int mx = sc[0], my = sc[1], mz = sc[2];
    const int64_t Bx = (int64_t)sc[3] - mx + 2, By = (int64_t)sc[4] - my + 2, Bz = (int64_t)sc[5] - mz + 2;
    const bool boxed = Bx * By * Bz <= kSpreadBox;
    if (!boxed) {
        // a cell too large for the box: point by point through the fallback
        for (int t = threadIdx.x; t < 8 * nv; t += blockDim.x) {
            const int i = t >> 3, q = t & 7;
            const SPoint<R> r = pts[i];
            int x, y, z;
            decode(pbase[i], x, y, z);
            const int gx = (q & 1) ? (x + 1 == ch.nx ? 0 : x + 1) : x;
            const int gy = ((q >> 1) & 1) ? (y + 1 == ch.ny ? 0 : y + 1) : y;
            const int gz = (q >> 2) ? (z + 1 == ch.nz ? 0 : z + 1) : z;
            const uint32_t n = (uint32_t)(ch.noff + gx + (int64_t)ch.nx * (gy + (int64_t)ch.ny * gz));
            if (atomicExch(&a.owner[n], epoch) != epoch && !a.accumulate) FI[n] = R4{R(0), R(0), R(0), R(0)};
            const R wx = (q & 1) ? r.dx : R(1) - r.dx, wy = ((q >> 1) & 1) ? r.dy : R(1) - r.dy;
            const R wz = (q >> 2) ? r.dz : R(1) - r.dz;
            const R wt = wx * wy * wz;
            fallback_add(n, gx, gy, gz, wt * r.fx, wt * r.fy, wt * r.fz);
        }
        return;
    }
    const int bx_ = (int)Bx, by_ = (int)By, V = (int)(Bx * By * Bz);
    const float rbx = 1.0f / (float)bx_, rby = 1.0f / (float)by_;
    const int nwords = (V + 31) / 32;
    // Counting sort of the points by (box index of the base node, point).  A
    // run of points with one base node is numbered by that node's rank among
    // the set base bits; a point's place is its run's start plus the number
    // of the run's points with a smaller index.
    constexpr int kPer = kSpreadMaxPoints / kSpreadThreads;  // points per thread at most
    int *cnt = reinterpret_cast<int *>(nodes + (a.maxv & 1));     // [maxv] points per run (the node list comes later)
    uint16_t *memb = reinterpret_cast<uint16_t *>(cnt + a.maxv);  // [maxv] the runs' points, unordered
    uint32_t lis[kPer];
#pragma unroll
    for (int m = 0; m < kPer; m++) {
        const int i = threadIdx.x + m * kSpreadThreads;
        lis[m] = 0;
        if (i < nv) {
            int x, y, z;
            decode(pbase[i], x, y, z);
            lis[m] = (uint32_t)((unwrap(x - rx, ch.nx) - mx) +
                                bx_ * ((unwrap(y - ry, ch.ny) - my) + by_ * (unwrap(z - rz, ch.nz) - mz)));
        }
        if (i < a.maxv) cnt[i] = 0;
    }
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) bbits[i] = bits[i] = 0;
    __syncthreads();
    // base-node and stencil-node bitmaps
#pragma unroll
    for (int m = 0; m < kPer; m++) {
        if (threadIdx.x + m * kSpreadThreads >= nv) continue;
        const uint32_t li = lis[m];
        atomicOr(&bbits[li >> 5], 1u << (li & 31));
        int lx, ly, lz;
        box_coords((int)li, bx_, by_, rbx, rby, lx, ly, lz);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int nn = (lx + (q & 1)) + bx_ * ((ly + ((q >> 1) & 1)) + by_ * (lz + (q >> 2)));
            atomicOr(&bits[nn >> 5], 1u << (nn & 31));
        }
    }
    __syncthreads();
    int nruns;
    {
        const int w = threadIdx.x;  // nwords <= kWords = blockDim.x
        const int pre = block_exclusive_scan(w < nwords ? __popc(bbits[w]) : 0, sc + 8, nruns);
        if (w < nwords) wpre[w] = (uint16_t)pre;
    }
    __syncthreads();
    int run[kPer];
#pragma unroll
    for (int m = 0; m < kPer; m++) {
        run[m] = -1;
        if (threadIdx.x + m * kSpreadThreads < nv) {
            const uint32_t li = lis[m];
            run[m] = wpre[li >> 5] + __popc(bbits[li >> 5] & ((1u << (li & 31)) - 1u));
            atomicAdd(&cnt[run[m]], 1);
        }
    }
    __syncthreads();
    {
        // run starts: exclusive scan of the counts, kPer consecutive runs per thread
        const int r0 = threadIdx.x * kPer;
        int c4[kPer], sum = 0;
#pragma unroll
        for (int m = 0; m < kPer; m++) {
            c4[m] = r0 + m < nruns ? cnt[r0 + m] : 0;
            sum += c4[m];
        }
        int tot;
        int pre = block_exclusive_scan(sum, sc + 8, tot);
#pragma unroll
        for (int m = 0; m < kPer; m++) {
            if (r0 + m < nruns) rstart[r0 + m] = (uint16_t)pre;
            pre += c4[m];
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kPer; m++)
        if (run[m] >= 0) memb[rstart[run[m]] + atomicSub(&cnt[run[m]], 1) - 1] = (uint16_t)(threadIdx.x + m * kSpreadThreads);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kPer; m++)
        if (run[m] >= 0) {
            const int i = threadIdx.x + m * kSpreadThreads, r = run[m];
            const int s0 = rstart[r], s1 = r + 1 < nruns ? (int)rstart[r + 1] : nv;
            int rank = 0;
            for (int j = s0; j < s1; j++) rank += memb[j] < i;
            key[s0 + rank] = (lis[m] << 11) | (uint32_t)i;
        }
    __syncthreads();
    // node list (box indices, ascending)
    int total = 0;
    for (int w0 = 0; w0 < nwords; w0 += blockDim.x) {
        const int w = w0 + threadIdx.x;
        uint32_t m = w < nwords ? bits[w] : 0u;
        int tot;
        int off = total + block_exclusive_scan(__popc(m), sc + 8, tot);
        while (m) {
            const int b = __builtin_ctz(m);
            m &= m - 1;
            nodes[off++] = (uint16_t)(w * 32 + b);
        }
        total += tot;
    }
    __syncthreads();
    // one thread per stencil node
    for (int k = threadIdx.x; k < total; k += blockDim.x) {
        const int li = nodes[k];
        int lx, ly, lz;
        box_coords(li, bx_, by_, rbx, rby, lx, ly, lz);
        const int gx = wrap_to(rx + mx + lx, ch.nx), gy = wrap_to(ry + my + ly, ch.ny), gz = wrap_to(rz + mz + lz, ch.nz);
        const uint32_t n = (uint32_t)(ch.noff + gx + (int64_t)ch.nx * (gy + (int64_t)ch.ny * gz));
        // the claim goes out first, so that its round trip overlaps the sum
        const uint32_t prev = atomicExch(&a.owner[n], epoch);
        // The eight base nodes whose stencils could hold this node (q: its
        // offset from them).  Their LDS lookups (base bit, word prefix, run
        // start, the run's first key) are independent across the eight, so
        // each level goes out for all eight before any is used; the sums
        // then take the runs in the order of a plain loop over q.
        uint32_t bq[8], mq[8], kq[8];
        bool in[8];
        int sq[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int ex = lx - (q & 1), ey = ly - ((q >> 1) & 1), ez = lz - (q >> 2);
            in[q] = ex >= 0 && ey >= 0 && ez >= 0;
            bq[q] = in[q] ? (uint32_t)(ex + bx_ * (ey + by_ * ez)) : 0u;
            mq[q] = bbits[bq[q] >> 5];
        }
        // (every read is made, at index 0 where the corner is out, and masked
        // arithmetically, so none waits behind a branch)
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const uint32_t bit = 1u << (bq[q] & 31);
            in[q] = in[q] && (mq[q] & bit);
            sq[q] = ((int)wpre[bq[q] >> 5] + __popc(mq[q] & (bit - 1u))) * (int)in[q];
        }
#pragma unroll
        for (int q = 0; q < 8; q++) sq[q] = (int)rstart[sq[q]] * (int)in[q];
#pragma unroll
        for (int q = 0; q < 8; q++) kq[q] = key[sq[q]];  // the run's first point (a set base bit has one)
        R Fx = R(0), Fy = R(0), Fz = R(0);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            if (!in[q]) continue;
            R Sx = R(0), Sy = R(0), Sz = R(0);
            uint32_t kk = kq[q];
            int j = sq[q];
            do {
                const SPoint<R> r = pts[kk & 0x7ffu];
                const R wx = (q & 1) ? r.dx : R(1) - r.dx, wy = ((q >> 1) & 1) ? r.dy : R(1) - r.dy;
                const R wz = (q >> 2) ? r.dz : R(1) - r.dz;
                const R wt = wx * wy * wz;
                Sx += wt * r.fx;
                Sy += wt * r.fy;
                Sz += wt * r.fz;
                ++j;
                kk = j < nv ? key[j] : ~0u;
            } while ((kk >> 11) == bq[q]);
            Fx += Sx;
            Fy += Sy;
            Fz += Sz;
        }
        if (prev != epoch) {
            if (a.accumulate) {
                const R4 f = FI[n];
                Fx = f.x + Fx;
                Fy = f.y + Fy;
                Fz = f.z + Fz;
            }
            FI[n] = R4{Fx, Fy, Fz, R(0)};
        } else {
            fallback_add(n, gx, gy, gz, Fx, Fy, Fz);
        }
    }
}

}  // namespace lbm

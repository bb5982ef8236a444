// Contact forces (Sec. 2.4, collisions): a soft-sphere repulsion between IB
// points of different cells and between IB points and the walls, cut at an
// interaction range so that only close neighbours interact.
//
// Law (a reading; the paper names the potential only): U(d) = a d^-n for
// d = r - roff in (0, rcut), 0 beyond, continued linearly below dmin, so the
// force magnitude is n a d^-(n+1) clamped at d = dmin.
//
// Cell-cell part, per coupled step:
//   k_cell_bounds (one workgroup per cell): vertex centroid and radius;
//   k_contact_pairs (one thread per cell pair of one channel): pairs whose
//     bounding spheres come within roff + rcut are appended to a list;
//   k_contact_cells (workgroups stride over the list): each side of a pair in
//     turn stages the other cell's points in LDS and every point sums the
//     repulsion of all of them, then adds it to its membrane force with
//     three float atomics (only points in range do, so the order of these
//     few adds is the one part of a step that is not fixed).
// The wall part is evaluated per point inside the point update, k_move (wall_force).
#pragma once

#include "ibm_kernels.hpp"

namespace lbm {

struct BoundsArgs {
    const int32_t *vert_off, *anchor;
    const double *x;   // [3][nverts] offsets
    double *bounds;    // [ncells][4]: centroid (absolute, channel coordinates), radius
    uint32_t *npairs;  // reset here
    int ncells, nverts;
};

__global__ __launch_bounds__(256) void k_cell_bounds(BoundsArgs a) {
    __shared__ double red[4 * 3];
    const int c = blockIdx.x;
    const int v0 = a.vert_off[c], nv = a.vert_off[c + 1] - v0, NV = a.nverts;
    if (c == 0 && threadIdx.x == 0) *a.npairs = 0;
    double s[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nv; k += blockDim.x) {
        s[0] += a.x[v0 + k];
        s[1] += a.x[NV + v0 + k];
        s[2] += a.x[2 * NV + v0 + k];
    }
    block_sum<3>(s, red);
    const double cx = s[0] / nv, cy = s[1] / nv, cz = s[2] / nv;
    double r2[1] = {0.0};
    for (int k = threadIdx.x; k < nv; k += blockDim.x) {
        const double dx = a.x[v0 + k] - cx, dy = a.x[NV + v0 + k] - cy, dz = a.x[2 * NV + v0 + k] - cz;
        r2[0] = fmax(r2[0], dx * dx + dy * dy + dz * dz);
    }
    // max over the block (fixed order like block_sum)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) r2[0] = fmax(r2[0], __shfl_xor(r2[0], o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r2[0];
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) m = fmax(m, red[w]);
        a.bounds[4 * c + 0] = a.anchor[c] + cx;
        a.bounds[4 * c + 1] = a.anchor[a.ncells + c] + cy;
        a.bounds[4 * c + 2] = a.anchor[2 * a.ncells + c] + cz;
        a.bounds[4 * c + 3] = sqrt(m);
    }
}

struct PairArgs {
    const double *bounds;
    const int32_t *cell_chan;
    const Chan *chans;
    uint32_t *npairs;
    int2 *pairs;
    int ncells, cap;
    int per[3];
    double reach;  // roff + rcut
};

__global__ __launch_bounds__(256) void k_contact_pairs(PairArgs a) {
    const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j <= i || j >= a.ncells) return;
    const int ci = cell_channel(a.cell_chan, i);
    if (cell_channel(a.cell_chan, j) != ci) return;
    const Chan ch = a.chans[ci];
    const double *bi = a.bounds + 4 * i, *bj = a.bounds + 4 * j;
    const double dx = min_image(bi[0] - bj[0], ch.nx, a.per[0]);
    const double dy = min_image(bi[1] - bj[1], ch.ny, a.per[1]);
    const double dz = min_image(bi[2] - bj[2], ch.nz, a.per[2]);
    const double lim = bi[3] + bj[3] + a.reach;
    if (dx * dx + dy * dy + dz * dz >= lim * lim) return;
    const uint32_t k = atomicAdd(a.npairs, 1u);
    if (k < (uint32_t)a.cap) a.pairs[k] = make_int2(i, j);
}

struct CellContactArgs {
    const int32_t *vert_off, *anchor, *cell_chan;
    const Chan *chans;
    const double *x;  // [3][nverts] offsets
    void *f_el;       // [3][nverts] real, contact forces added
    const uint32_t *npairs;
    const int2 *pairs;
    int ncells, nverts, cap;
    int per[3];
    ContactLaw law;
};

constexpr int kContactThreads = 256;

template <class R>
__global__ __launch_bounds__(kContactThreads) void k_contact_cells(CellContactArgs a) {
    extern __shared__ double lds[];  // 3 x maxv positions of the other cell
    const int NV = a.nverts, NC = a.ncells;
    const uint32_t np = min(*a.npairs, (uint32_t)a.cap);
    R *FE = static_cast<R *>(a.f_el);
    for (uint32_t p = blockIdx.x; p < np; p += gridDim.x) {
        const int2 pr = a.pairs[p];
        const Chan ch = a.chans[cell_channel(a.cell_chan, pr.x)];
        for (int side = 0; side < 2; side++) {
            const int me = side ? pr.y : pr.x, other = side ? pr.x : pr.y;
            const int o0 = a.vert_off[other], no = a.vert_off[other + 1] - o0;
            double *ox = lds, *oy = lds + no, *oz = lds + 2 * no;
            const double ax = a.anchor[other], ay = a.anchor[NC + other], az = a.anchor[2 * NC + other];
            __syncthreads();
            for (int k = threadIdx.x; k < no; k += blockDim.x) {
                ox[k] = ax + a.x[o0 + k];
                oy[k] = ay + a.x[NV + o0 + k];
                oz[k] = az + a.x[2 * NV + o0 + k];
            }
            __syncthreads();
            const int m0 = a.vert_off[me], nm = a.vert_off[me + 1] - m0;
            const double mx = a.anchor[me], my = a.anchor[NC + me], mz = a.anchor[2 * NC + me];
            for (int k = threadIdx.x; k < nm; k += blockDim.x) {
                const double px = mx + a.x[m0 + k], py = my + a.x[NV + m0 + k], pz = mz + a.x[2 * NV + m0 + k];
                double fx = 0.0, fy = 0.0, fz = 0.0;
                for (int q = 0; q < no; q++) {
                    const double dx = min_image(px - ox[q], ch.nx, a.per[0]);
                    const double dy = min_image(py - oy[q], ch.ny, a.per[1]);
                    const double dz = min_image(pz - oz[q], ch.nz, a.per[2]);
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const double reach = a.law.roff + a.law.rcut;
                    if (r2 >= reach * reach || r2 == 0.0) continue;
                    const double r = sqrt(r2);
                    const double f = contact_force(a.law, r - a.law.roff) / r;
                    fx += f * dx;
                    fy += f * dy;
                    fz += f * dz;
                }
                if (fx != 0.0 || fy != 0.0 || fz != 0.0) {
                    atomicAdd(&FE[m0 + k], R(fx));
                    atomicAdd(&FE[NV + m0 + k], R(fy));
                    atomicAdd(&FE[2 * NV + m0 + k], R(fz));
                }
            }
        }
    }
}

}  // namespace lbm

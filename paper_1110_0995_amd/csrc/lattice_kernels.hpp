// Lattice kernels: node classification, rest state, the fused
// collide-and-stream step (LBM equation of Sec. 2.1 with halfway
// bounce-back of Sec. 2.4), and the moments / FP64 global sums.
#pragma once

#include "d3q19.hpp"

namespace lbm {

// Node classes.  The collide-stream kernel takes the plain streaming path
// for CLS_BULK nodes and consults the per-node link mask only for CLS_WALL.
enum : uint8_t { CLS_BULK = 0, CLS_WALL = 1, CLS_SOLID = 2 };

// A context holds one or more independent lattices ("channels") in one
// concatenated node index space (channel c owns nodes [noff, noff + N_c))
// and one concatenated tile space (tiles [toff, toff + ntiles_c)).  A tile
// is 64 consecutive x of one (y, z) row of one channel.
struct Chan {
    int nx, ny, nz, tpr;  // size; tpr = 64-node tiles per x-row
    int64_t noff;         // first node
    int toff, pad;        // first tile
};

// Channel of a global tile, uniform across the wave.
__device__ __forceinline__ int tile_channel(const uint16_t *tile_chan, int tile) {
    return tile_chan ? __builtin_amdgcn_readfirstlane((int)tile_chan[tile]) : 0;
}

// cls[n] and links[n] (bit i set = the link along c_i ends on a solid node
// or leaves a non-periodic axis, so population i bounces back).  One wave
// per tile.
__global__ __launch_bounds__(256) void k_classify(const Chan *__restrict__ chans, const uint16_t *__restrict__ tile_chan,
                                                  int ntiles, int px, int py, int pz,
                                                  const uint8_t *__restrict__ solid, uint8_t *__restrict__ cls,
                                                  uint32_t *__restrict__ links) {
    const int tile = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const Chan ch = chans[tile_channel(tile_chan, tile)];
    const int lt = tile - ch.toff, row = lt / ch.tpr;
    const int x = (lt - row * ch.tpr) * 64 + (threadIdx.x & 63);
    if (x >= ch.nx) return;
    const int y = row % ch.ny, z = row / ch.ny;
    const int64_t n = ch.noff + (int64_t)row * ch.nx + x;
    if (solid[n]) {
        cls[n] = CLS_SOLID;
        links[n] = 0;
        return;
    }
    const int per[3] = {px, py, pz}, d[3] = {ch.nx, ch.ny, ch.nz};
    uint32_t m = 0;
    for (int i = 1; i < Q; i++) {
        int p[3] = {x + cx(i), y + cy(i), z + cz(i)};
        bool out = false;
        for (int k = 0; k < 3; k++) {
            if (p[k] < 0 || p[k] >= d[k]) {
                if (per[k]) p[k] = pmod(p[k], d[k]);
                else out = true;
            }
        }
        if (out || solid[ch.noff + p[0] + (int64_t)ch.nx * (p[1] + (int64_t)ch.ny * p[2])]) m |= 1u << i;
    }
    cls[n] = m ? CLS_WALL : CLS_BULK;
    links[n] = m;
}

// Fluid at rest: f_i = w_i (or h_i = 0 for the deviation storage).
template <class S, bool DEV>
__global__ void k_rest(S *__restrict__ f, int64_t stride, int64_t N) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
#pragma unroll
    for (int i = 0; i < Q; i++) f[i * stride + n] = DEV ? S(0) : wgt<S>(i);
}

// BGK relaxation with Guo's source for one node, in place on f[19].
// rho = sum f (DEV: 1 + sum h), j = sum f c, u = (j + F/2)/rho,
// f_eq = w rho (1 + 3cu + 9/2 (cu)^2 - 3/2 u.u) (DEV: minus w),
// S_i = (1 - 1/(2 tau)) w_i (3 (c_i - u).F + 9 (c_i.u)(c_i.F)),
// f_i <- f_i - (f_i - f_eq_i)/tau + S_i.
template <class R, bool DEV>
__device__ __forceinline__ void collide(R (&f)[Q], R Fx, R Fy, R Fz, R omega, R kf) {
    R s = R(0);
#pragma unroll
    for (int i = 0; i < Q; i++) s += f[i];
    const R jx = (f[1] - f[2]) + (f[7] - f[8]) + (f[9] - f[10]) + (f[11] - f[12]) + (f[13] - f[14]);
    const R jy = (f[3] - f[4]) + (f[7] - f[8]) + (f[10] - f[9]) + (f[15] - f[16]) + (f[17] - f[18]);
    const R jz = (f[5] - f[6]) + (f[11] - f[12]) + (f[14] - f[13]) + (f[15] - f[16]) + (f[18] - f[17]);
    const R rho = DEV ? R(1) + s : s;
    const R ir = R(1) / rho;
    const R ux = (jx + R(0.5) * Fx) * ir;
    const R uy = (jy + R(0.5) * Fy) * ir;
    const R uz = (jz + R(0.5) * Fz) * ir;
    const R usq = R(1.5) * (ux * ux + uy * uy + uz * uz);
    const R uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const R cu = R(cx(i)) * ux + R(cy(i)) * uy + R(cz(i)) * uz;
        const R cF = R(cx(i)) * Fx + R(cy(i)) * Fy + R(cz(i)) * Fz;
        const R e = R(3) * cu + R(4.5) * cu * cu - usq;
        const R w = wgt<R>(i);
        const R feq = DEV ? w * (s + rho * e) : w * rho * (R(1) + e);
        const R src = kf * w * (R(3) * (cF - uF) + R(9) * cu * cF);
        f[i] = f[i] - omega * (f[i] - feq) + src;
    }
}

// Element i of an array addressed from its base: with a 32-bit IDX the byte
// offset is formed in 32 bits (the host only picks IDX = uint32_t when every
// buffer the kernel touches is below 4 GiB), so loads and stores use a
// uniform 64-bit base plus a 32-bit per-lane offset.
template <class T, class IDX>
__device__ __forceinline__ T &at(T *base, IDX i) {
    if constexpr (sizeof(IDX) == 4)
        return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (uint32_t)(i * (uint32_t)sizeof(T)));
    else
        return base[i];
}
template <class T, class IDX>
__device__ __forceinline__ const T &at(const T *base, IDX i) {
    if constexpr (sizeof(IDX) == 4)
        return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (uint32_t)(i * (uint32_t)sizeof(T)));
    else
        return base[i];
}

struct StepArgs {
    const void *fa;
    void *fb;
    int64_t stride;
    const uint8_t *cls;
    const uint32_t *links;
    const void *fibm;     // [N] x 4 immersed-boundary force (x, y, z, unused), valid at marked nodes
    void *facc;           // [N] x 4 the spread's fallback accumulator: added and cleared in flagged tiles
    uint8_t *ftile;       // [ntiles] 1: the tile holds fallback sums (cleared here)
    uint8_t *need;        // [N] 1: the node received spread force this step
    uint8_t *tneed;       // [ntiles] 1: the tile holds such a node
    const void *gfield;   // [3][N] or null
    const Chan *chans;
    const uint16_t *tile_chan;  // null for a single channel
    int ntiles;
    int remap;            // 1: renumber workgroups so each XCD walks one contiguous tile range
    const uint32_t *wgtab; // [gridDim.x] workgroup table (first tile << 3 | tiles - 1), or null
    int reverse;          // 1: take the table's entries in reverse order
    int64_t N;
    double g[3];
    double omega, kf;
};

// One fused collide-and-stream pass (push): each wave owns one tile of 64
// consecutive x of one (y,z) row, reads the 19 planes of its nodes
// coalesced, collides in registers and writes every post-collision value
// straight to its destination slot (neighbour along c_i, or the opposite
// slot of the same node when that link is a wall link).  The spread force is
// read only at nodes marked as stencil nodes of this step (where the spread
// wrote it; in a tile the spread flagged, plus its fallback accumulator,
// which is cleared), and the marks are cleared.
// A workgroup is blockDim/64 consecutive tiles (the tile shape is a launch
// parameter); when it holds whole x rows, the partial cache lines of the
// x-shifted stores of a row meet in one L2 whatever XCD runs it and the
// workgroups keep their natural order (the chip then streams through one
// compact address range), otherwise they are renumbered by XCD (`remap`) so
// that neighbouring tiles share an L2.  Every other pass takes the table in
// reverse order, so that it starts on the rows the previous pass wrote last
// (still held by the memory-side cache).  IDX is the index type of element offsets from the buffer
// base: uint32_t when 19 planes fit in 4 GiB (single 64-bit base + 32-bit
// lane offsets), int64_t otherwise.
template <class S, class R, bool DEV, bool HAS_G, class IDX>
__global__ __launch_bounds__(512) void k_collide_stream(StepArgs a) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int tile;
    if (a.wgtab) {
        const uint32_t e = a.wgtab[a.reverse ? gridDim.x - 1 - blockIdx.x : blockIdx.x];
        if (wave > (int)(e & 7u)) return;
        tile = (int)(e >> 3) + wave;
    } else {
        const int blk = a.remap ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
        tile = blk * (blockDim.x >> 6) + wave;
    }
    if (tile >= a.ntiles) return;
    const Chan ch = a.chans[tile_channel(a.tile_chan, tile)];
    const int lt = tile - ch.toff;
    const int row = lt / ch.tpr;
    const int x = (lt - row * ch.tpr) * 64 + lane;
    if (x >= ch.nx) return;
    const IDX base = (IDX)ch.noff;
    const IDX n = base + (IDX)row * (IDX)ch.nx + (IDX)x;
    const IDX N = (IDX)a.N;
    const IDX stride = (IDX)a.stride;

    R Fx = R(a.g[0]), Fy = R(a.g[1]), Fz = R(a.g[2]);
    if (HAS_G) {
        const R *G = static_cast<const R *>(a.gfield);
        Fx += at(G, n);
        Fy += at(G, N + n);
        Fz += at(G, 2 * N + n);
    }
    if (a.tneed[tile]) {
        const bool fl = a.ftile[tile] != 0;
        if (at(a.need, n)) {
            const R *fi = static_cast<const R *>(a.fibm);
            R fx = at(fi, 4 * n), fy = at(fi, 4 * n + 1), fz = at(fi, 4 * n + 2);
            if (fl) {  // the spread's fallback sums, taken once
                R *fa = static_cast<R *>(a.facc);
                fx = fx + at(fa, 4 * n);
                fy = fy + at(fa, 4 * n + 1);
                fz = fz + at(fa, 4 * n + 2);
                at(fa, 4 * n) = R(0);
                at(fa, 4 * n + 1) = R(0);
                at(fa, 4 * n + 2) = R(0);
            }
            Fx += fx;
            Fy += fy;
            Fz += fz;
            at(a.need, n) = 0;
        }
        if (lane == 0) {
            a.tneed[tile] = 0;
            if (fl) a.ftile[tile] = 0;
        }
    }
    const uint8_t cl = at(a.cls, n);
    if (cl == CLS_SOLID) return;

    const S *__restrict__ fa = static_cast<const S *>(a.fa);
    S *__restrict__ fb = static_cast<S *>(a.fb);
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) f[i] = R(at(fa, (IDX)i * stride + n));

    collide<R, DEV>(f, Fx, Fy, Fz, R(a.omega), R(a.kf));

    const int y = row % ch.ny, z = row / ch.ny;
    const int xp = (x + 1 == ch.nx) ? 0 : x + 1;
    const int xm = (x == 0) ? ch.nx - 1 : x - 1;
    const int yp = (y + 1 == ch.ny) ? 0 : y + 1;
    const int ym = (y == 0) ? ch.ny - 1 : y - 1;
    const int zp = (z + 1 == ch.nz) ? 0 : z + 1;
    const int zm = (z == 0) ? ch.nz - 1 : z - 1;
    const uint32_t links = (cl == CLS_WALL) ? at(a.links, n) : 0u;
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const int xq = cx(i) > 0 ? xp : (cx(i) < 0 ? xm : x);
        const int yq = cy(i) > 0 ? yp : (cy(i) < 0 ? ym : y);
        const int zq = cz(i) > 0 ? zp : (cz(i) < 0 ? zm : z);
        const IDX dst = ((links >> i) & 1u)
                            ? (IDX)opp(i) * stride + n
                            : (IDX)i * stride + base + (IDX)xq + (IDX)ch.nx * ((IDX)yq + (IDX)ch.ny * (IDX)zq);
        at(fb, dst) = S(f[i]);
    }
}

// rho and u = (j + F_ext/2)/rho per node (solid: 0), plus per-block FP64
// partial sums of rho and j over fluid nodes.
template <class S, class R, bool DEV, bool HAS_G>
__global__ __launch_bounds__(256) void k_moments(const S *__restrict__ f, int64_t stride,
                                                 const uint8_t *__restrict__ cls, const R *__restrict__ G,
                                                 int64_t N, double gx, double gy, double gz, R *rho_out,
                                                 R *u_out, double *partials) {
    __shared__ double red[4 * 4];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (n < N) {
        if (cls[n] != CLS_SOLID) {
            double r = DEV ? 1.0 : 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const double v = (double)f[i * stride + n];
                r += v;
                j[0] += cx(i) * v;
                j[1] += cy(i) * v;
                j[2] += cz(i) * v;
            }
            acc[0] = r;
            acc[1] = j[0];
            acc[2] = j[1];
            acc[3] = j[2];
            const double F[3] = {gx + (HAS_G ? (double)G[n] : 0.0), gy + (HAS_G ? (double)G[N + n] : 0.0),
                                 gz + (HAS_G ? (double)G[2 * N + n] : 0.0)};
            if (rho_out) rho_out[n] = R(r);
            if (u_out)
                for (int d = 0; d < 3; d++) u_out[d * N + n] = R((j[d] + 0.5 * F[d]) / r);
        } else {
            if (rho_out) rho_out[n] = R(0);
            if (u_out)
                for (int d = 0; d < 3; d++) u_out[d * N + n] = R(0);
        }
    }
    block_sum<4>(acc, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; k++) partials[4 * (int64_t)blockIdx.x + k] = acc[k];
}

__global__ __launch_bounds__(256) void k_final_sum(const double *__restrict__ partials, int64_t nparts,
                                                   double *out) {
    __shared__ double red[4 * 4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t p = threadIdx.x; p < nparts; p += blockDim.x)
        for (int k = 0; k < 4; k++) acc[k] += partials[4 * p + k];
    block_sum<4>(acc, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; k++) out[k] = acc[k];
}

// Plain device copy (snapshots taken inside captured graphs, where a
// memcpy node is avoided).
template <class T>
__global__ __launch_bounds__(256) void k_copy(const T *__restrict__ src, T *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

template <class S, bool DEV>
__global__ void k_store_f64(const S *__restrict__ f, int64_t stride, int64_t N, double *__restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
#pragma unroll
    for (int i = 0; i < Q; i++) out[i * N + n] = (double)f[i * stride + n] + (DEV ? wgt<double>(i) : 0.0);
}

template <class S, bool DEV>
__global__ void k_load_f64(S *__restrict__ f, int64_t stride, int64_t N, const double *__restrict__ in) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
#pragma unroll
    for (int i = 0; i < Q; i++) f[i * stride + n] = S(in[i * N + n] - (DEV ? wgt<double>(i) : 0.0));
}

}  // namespace lbm

// Lattice kernels: node classification, rest state, the fused
// collide-and-stream step (LBM equation of Sec. 2.1 with halfway
// bounce-back of Sec. 2.4), and the moments / FP64 global sums.
#pragma once

#include <type_traits>

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

// Where a state buffer keeps the populations.  Every pass writes each slot
// (plane i, node m) exactly once, from the node m - c_i that streams into
// it, so that every cache line is written whole:
//  - a population streamed into a fluid node lies in that node's slot;
//  - a population a fluid node sends towards a solid neighbour (halfway
//    bounce-back: it returns to the node along the opposite direction) is
//    streamed into the solid node's slot like any other, and the node reads
//    it back from there: population i of fluid node n whose link opp(i)
//    ends on a solid node s = n - c_i lies in slot opp(i) of s;
//  - a solid node streams its rest value into its destinations, slots whose
//    content nobody reads;
//  - a population bounced at a non-periodic face of the lattice (no node
//    beyond it) is written into the node's own slot opp(i), as the
//    population i of the next step.
// So population i of fluid node n is in slot (i, n) unless link opp(i) of n
// ends on a solid node inside the lattice.

// The link of (x, y, z) along c_i leaves the channel through a non-periodic face.
__device__ __forceinline__ bool leaves_lattice(int i, int x, int y, int z, const Chan &ch, const int (&per)[3]) {
    return (!per[0] && ((cx(i) > 0 && x + 1 == ch.nx) || (cx(i) < 0 && x == 0))) ||
           (!per[1] && ((cy(i) > 0 && y + 1 == ch.ny) || (cy(i) < 0 && y == 0))) ||
           (!per[2] && ((cz(i) > 0 && z + 1 == ch.nz) || (cz(i) < 0 && z == 0)));
}

// Element index of population i of fluid node n = (x, y, z) of channel ch
// (links: its link mask).
template <class IDX>
__device__ __forceinline__ IDX pop_slot(int i, IDX n, uint32_t links, int x, int y, int z, const Chan &ch, IDX stride,
                                        const int (&per)[3]) {
    if (!((links >> opp(i)) & 1u) || leaves_lattice(opp(i), x, y, z, ch, per)) return (IDX)i * stride + n;
    const int xs = x - cx(i) < 0 ? ch.nx - 1 : (x - cx(i) == ch.nx ? 0 : x - cx(i));
    const int ys = y - cy(i) < 0 ? ch.ny - 1 : (y - cy(i) == ch.ny ? 0 : y - cy(i));
    const int zs = z - cz(i) < 0 ? ch.nz - 1 : (z - cz(i) == ch.nz ? 0 : z - cz(i));
    return (IDX)opp(i) * stride + (IDX)ch.noff + (IDX)xs + (IDX)ch.nx * ((IDX)ys + (IDX)ch.ny * (IDX)zs);
}

// Coordinates of node n (concatenated index) in its channel (nch channels,
// ascending node offsets).
__device__ __forceinline__ void node_coords(const Chan *chans, int nch, int64_t n, Chan &ch, int &x, int &y, int &z) {
    int lo = 0, hi = nch - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chans[mid].noff <= n) lo = mid;
        else hi = mid - 1;
    }
    ch = chans[lo];
    const int64_t l = n - ch.noff;
    x = (int)(l % ch.nx);
    y = (int)((l / ch.nx) % ch.ny);
    z = (int)(l / ((int64_t)ch.nx * ch.ny));
}

// Population i of node n as a per-node kernel reads it (a bulk node's own
// slot; a wall node's through pop_slot).
struct PopView {
    const Chan *chans;
    int nch;
    int per[3];
    const uint8_t *cls;
    const uint32_t *links;
};
template <class S>
__device__ __forceinline__ void load_node(const S *f, int64_t stride, int64_t n, const PopView &pv, S (&v)[Q]) {
#pragma unroll
    for (int i = 0; i < Q; i++) v[i] = f[i * stride + n];
    if (pv.cls[n] != CLS_WALL) return;
    const uint32_t lk = pv.links[n];
    Chan ch;
    int x, y, z;
    node_coords(pv.chans, pv.nch, n, ch, x, y, z);
#pragma unroll
    for (int i = 0; i < Q; i++)
        if ((lk >> opp(i)) & 1u) v[i] = f[pop_slot<int64_t>(i, n, lk, x, y, z, ch, stride, pv.per)];
}

// cls[n] and links[n] (bit i set = the link along c_i ends on a solid node
// or leaves a non-periodic axis, so population i bounces back), and per
// tile the 64-bit masks of its solid and of its wall nodes (bit x & 63;
// tmask[t] = {solid lo, solid hi, wall lo, wall hi}), which the
// collide-stream pass reads with one scalar load per wave.  One wave per
// tile.
__global__ __launch_bounds__(256) void k_classify(const Chan *__restrict__ chans, const uint16_t *__restrict__ tile_chan,
                                                  int ntiles, int px, int py, int pz,
                                                  const uint8_t *__restrict__ solid, uint8_t *__restrict__ cls,
                                                  uint32_t *__restrict__ links, uint4 *__restrict__ tmask) {
    const int tile = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const Chan ch = chans[tile_channel(tile_chan, tile)];
    const int lt = tile - ch.toff, row = lt / ch.tpr;
    const int x = (lt - row * ch.tpr) * 64 + (threadIdx.x & 63);
    uint8_t c = CLS_BULK;
    if (x < ch.nx) {
        const int y = row % ch.ny, z = row / ch.ny;
        const int64_t n = ch.noff + (int64_t)row * ch.nx + x;
        uint32_t m = 0;
        if (solid[n]) {
            c = CLS_SOLID;
        } else {
            const int per[3] = {px, py, pz}, d[3] = {ch.nx, ch.ny, ch.nz};
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
            c = m ? CLS_WALL : CLS_BULK;
        }
        cls[n] = c;
        links[n] = m;
    }
    const uint64_t sm = __builtin_amdgcn_ballot_w64(c == CLS_SOLID), wm = __builtin_amdgcn_ballot_w64(c == CLS_WALL);
    if ((threadIdx.x & 63) == 0) tmask[tile] = uint4{(uint32_t)sm, (uint32_t)(sm >> 32), (uint32_t)wm, (uint32_t)(wm >> 32)};
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
// Returns the sum of the populations before the collision (of the
// deviations, with DEV): not finite iff some population is not.
template <class R, bool DEV>
__device__ __forceinline__ R collide(R (&f)[Q], R Fx, R Fy, R Fz, R omega, R kf) {
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
    return s;
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

// Raw buffer access (32-bit byte offsets from a resource descriptor, range
// checked against the buffer's size: an access beyond it reads 0 and writes
// nothing).  The plane offset of a population goes in the scalar offset, so
// the 19 loads of a node share one per-lane offset register.
constexpr int kBufFlags = 0x00020000;  // descriptor word 3: raw 32-bit data
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, uint64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0,
                                             (int)(bytes > 0xffffffffull ? 0xffffffffu : (uint32_t)bytes), kBufFlags);
}
template <class T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    } else {
        static_assert(sizeof(T) == 8, "4- or 8-byte elements");
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    }
}
template <class T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 0);
    } else {
        static_assert(sizeof(T) == 8, "4- or 8-byte elements");
        using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, (int)voff, (int)soff, 0);
    }
}

struct StepArgs {
    const void *fa;
    void *fb;
    int64_t stride;
    const uint4 *tmask;   // [ntiles] solid and wall masks of each tile (k_classify)
    const uint32_t *links;
    const void *fibm;     // [N] x 4 immersed-boundary force (x, y, z, unused), valid at marked nodes
    void *facc;           // [N] x 4 the spread's fallback accumulator: added and cleared in flagged tiles
    uint8_t *ftile;       // [ntiles] 1: the tile holds fallback sums (cleared here)
    uint8_t *need;        // [N] 1: the node received spread force this step
    uint8_t *tneed;       // [ntiles] 1: the tile holds such a node
    const uint2 *tnmask;  // [ntiles] the marks of each marked tile as a 64-bit mask (bit x & 63), written by
                          // the velocity pass of the step
    int use_tnmask;       // 0: the masks are not all current (velocities from records); read the node marks
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
    // records of the next step's stencil nodes (EMIT): per-tile entries
    // (RecTile), the record [19][cap]
    const uint4 *etile;
    void *erec;
    int64_t ecap;
    int per[3];  // periodic axes (a link leaving a non-periodic face bounces in place)
    uint32_t *nonfinite;  // set to 1 by a node whose populations are not all finite (never cleared here)
};

// Byte t of a byte array allocated in whole 16-byte units, for a
// wave-uniform t: one scalar load of the aligned word that holds it.
__device__ __forceinline__ uint32_t uniform_byte(const uint8_t *p, int t) {
    const uint32_t w = *reinterpret_cast<const uint32_t *>(p + (t & ~3));
    return (w >> (8 * (t & 3))) & 0xffu;
}

// Element i of an array that nothing writes while the kernel runs, read at a
// wave-uniform index through the constant address space, so that it is one
// scalar load even where the compiler cannot prove that no store of the
// kernel reaches it.
template <class T>
__device__ __forceinline__ T uniform_load(const T *p, int64_t i) {
    static_assert(sizeof(T) % 4 == 0, "whole dwords");
    using CU = const __attribute__((address_space(4))) uint32_t;
    CU *q = (CU *)(p + i);
    struct W {
        uint32_t w[sizeof(T) / 4];
    } v;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); k++) v.w[k] = q[k];
    return __builtin_bit_cast(T, v);
}

// Number of set bits of m below this lane.
__device__ __forceinline__ uint32_t bits_below_lane(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Per-tile entry of the next-step records (written by k_next_list): the
// tile's marked nodes (bit x & 63) and the first slot of their range.
struct RecTile {
    uint32_t mlo, mhi, tbase, pad;
};

// The 27 tiles around a wave's tile, (dc, dy, dz) in {-1, 0, 1}^3 (tile
// column, row y, row z; wrapped like the streaming), entry L = (dc + 1) +
// 3 (dy + 1) + 9 (dz + 1) loaded by lane L into the wave's LDS slots `rt`
// at the start of the pass (while every lane of the wave is active), so that
// the entries arrive with the populations; the emission reads them back as
// wave-uniform LDS loads.
constexpr int kRecTiles = 27;
__device__ __forceinline__ void stage_rec_tiles(const uint4 *ent, const Chan &ch, int col, int y, int z, int lane,
                                                uint4 *rt) {
    if (lane < kRecTiles) {
        const int dc = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
        const int c2 = col + dc < 0 ? ch.tpr - 1 : (col + dc == ch.tpr ? 0 : col + dc);
        const int y2 = y + dy < 0 ? ch.ny - 1 : (y + dy == ch.ny ? 0 : y + dy);
        const int z2 = z + dz < 0 ? ch.nz - 1 : (z + dz == ch.nz ? 0 : z + dz);
        rt[lane] = ent[ch.toff + (int64_t)(y2 + ch.ny * z2) * ch.tpr + c2];
    }
    // the other lanes of the wave read these slots later
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Entry L of the wave's staged tiles as wave-uniform values: mask, first slot.
// (readfirstlane returns a signed int: each word goes through uint32_t before
// widening, or a mask with bit 31 set would sign-extend into the high word)
__device__ __forceinline__ uint64_t rt_mask(const uint4 *rt, int L) {
    const uint4 e = rt[L];
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane(e.x), hi = (uint32_t)__builtin_amdgcn_readfirstlane(e.y);
    return (uint64_t)lo | (uint64_t)hi << 32;
}
__device__ __forceinline__ uint32_t rt_base(const uint4 *rt, int L) {
    return (uint32_t)__builtin_amdgcn_readfirstlane(rt[L].z);
}

// Record of population i, just streamed, when it lands on a node marked for
// the next step (see k_next_list): lane l's value goes to node (x + cx,
// y + cy, z + cz) in tile column col + (l + cx) / 64, or, on a bounced link,
// to slot opp(i) of its own node.  m0/b0: mask and first slot of the tile
// of the destination row in the wave's own column; ms/bs: of the column
// col + cx (cx != 0); mown/bown: of the wave's own tile.  The lane's bit and
// slot come from the mask shifted by cx: for cx = +1 lane 63 lands on bit 0
// of the next column, for cx = -1 lane 0 on bit 63 of the previous one.
// Requires nx % 64 == 0, so tiles are whole.
template <int I, class S>
__device__ __forceinline__ void emit_record(const StepArgs &a, __amdgpu_buffer_rsrc_t rrec, int lane, uint32_t links,
                                            uint64_t m0, uint32_t b0, uint64_t ms, uint32_t bs, uint64_t mown,
                                            uint32_t bown, S val) {
    constexpr int CX = cx(I);
    if (!(m0 | ms | mown)) return;
    const bool bounce = (links >> I) & 1u;
    bool hit;
    uint32_t slot;
    if (bounce) {
        hit = (mown >> lane) & 1ull;
        slot = bown + bits_below_lane(mown);
    } else if (CX == 0) {
        hit = (m0 >> lane) & 1ull;
        slot = b0 + bits_below_lane(m0);
    } else if (CX > 0) {
        if (lane == 63) {
            hit = ms & 1ull;
            slot = bs;
        } else {
            hit = (m0 >> (lane + 1)) & 1ull;
            slot = b0 + (uint32_t)(m0 & 1ull) + bits_below_lane(m0 >> 1);
        }
    } else {
        if (lane == 0) {
            hit = ms >> 63;
            slot = bs + (uint32_t)__popcll(ms) - 1u;
        } else {
            hit = (m0 >> (lane - 1)) & 1ull;
            slot = b0 + bits_below_lane(m0 << 1);
        }
    }
    if (hit) buf_store(val, rrec, (uint32_t)(((bounce ? opp(I) : I) * (uint32_t)a.ecap + slot) * sizeof(S)), 0u);
}

// The streaming order of the pass: by destination row (cy, cz), the
// direction with cx = 0 first, then cx = +1, then cx = -1, so that the
// record entries of a row are read once for its directions.
constexpr int kRowDirs[9][3] = {{0, 1, 2},  {3, 7, 10},  {4, 9, 8},  {5, 11, 14}, {6, 13, 12},
                                {15, -1, -1}, {16, -1, -1}, {17, -1, -1}, {18, -1, -1}};

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
template <class S, class R, bool DEV, bool HAS_G, class IDX, bool EMIT = false>
__global__ __launch_bounds__(512, sizeof(S) == 4 ? 8 : 1) void k_collide_stream(StepArgs a) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // A wave without a tile (a shorter table entry, the end of the tile
    // range) ends at once: the barrier below waits only for the waves of the
    // workgroup that have not ended.  Every other wave reaches it, the lanes
    // past the end of a row only skipping the work.
    int tile;
    bool wlive = true;  // wave-uniform: the wave owns a tile
    if (a.wgtab) {
        const uint32_t e = a.wgtab[a.reverse ? gridDim.x - 1 - blockIdx.x : blockIdx.x];
        tile = (int)(e >> 3) + wave;
        wlive = wave <= (int)(e & 7u);
    } else {
        const int blk = a.remap ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
        tile = blk * (blockDim.x >> 6) + wave;
    }
    if (!wlive || tile >= a.ntiles) return;
    const Chan ch = a.chans[tile_channel(a.tile_chan, tile)];
    const int lt = tile - ch.toff;
    const int row = lt / ch.tpr;
    const int x = (lt - row * ch.tpr) * 64 + lane;
    __shared__ uint4 rec_tiles[EMIT ? 8 * kRecTiles : 1];
    uint4 *rt = rec_tiles + (EMIT ? wave * kRecTiles : 0);
    if constexpr (EMIT)  // every lane of the wave is active here
        stage_rec_tiles(a.etile, ch, lt - row * ch.tpr, row % ch.ny, row / ch.ny, lane, rt);
    const bool live = x < ch.nx;
    const IDX base = (IDX)ch.noff;
    const IDX n = base + (IDX)row * (IDX)ch.nx + (IDX)x;
    const IDX N = (IDX)a.N;
    const IDX stride = (IDX)a.stride;
    const int y = row % ch.ny, z = row / ch.ny;

    const S *__restrict__ fa = static_cast<const S *>(a.fa);
    S *__restrict__ fb = static_cast<S *>(a.fb);
    constexpr bool BUF = sizeof(IDX) == 4;  // every buffer below 4 GiB: raw buffer access
    const uint64_t fbytes = (uint64_t)Q * (uint64_t)a.stride * sizeof(S);
    __amdgpu_buffer_rsrc_t ra, rb;
    if constexpr (BUF) {
        ra = buf_rsrc(fa, fbytes);
        rb = buf_rsrc(fb, fbytes);
    }
    R f[Q];
    bool solid = false;  // streams its rest value (see pop_slot)
    uint32_t links = 0u;
    R sum = R(0);  // population sum before the collision (0 for solid nodes)
    if (live) {
        // What the wave needs to know about its tile comes in scalar loads:
        // the tile's solid and wall masks, its stencil and fallback marks and
        // the mask of its stencil nodes.  So every vector load of the node
        // (its links, its immersed-boundary force, its 19 slots) is issued
        // before any has to be waited for, the populations last: waiting for
        // the links then does not wait for the populations.
        const int utile = __builtin_amdgcn_readfirstlane(tile);
        const uint4 tm = a.tmask[utile];
        const uint32_t tmark = uniform_byte(a.tneed, utile), tfall = uniform_byte(a.ftile, utile);
        const uint2 nm = a.tnmask[utile];  // meaningful only where tmark and use_tnmask are set
        solid = (((uint64_t)tm.y << 32 | tm.x) >> lane) & 1u;
        const bool wall = (((uint64_t)tm.w << 32 | tm.z) >> lane) & 1u;
        bool nmark = false;
        if (tmark) {
            if (a.use_tnmask)
                nmark = (((uint64_t)nm.y << 32 | nm.x) >> lane) & 1u;
            else
                nmark = at(a.need, n) != 0;
        }
        links = wall ? at(a.links, n) : 0u;
        // the spread force (and its fallback sums), used once the populations are requested
        R ibx = R(0), iby = R(0), ibz = R(0), acx = R(0), acy = R(0), acz = R(0);
        if (nmark) {
            const R *fi = static_cast<const R *>(a.fibm);
            ibx = at(fi, 4 * n);
            iby = at(fi, 4 * n + 1);
            ibz = at(fi, 4 * n + 2);
            if (tfall) {
                const R *acc = static_cast<const R *>(a.facc);
                acx = at(acc, 4 * n);
                acy = at(acc, 4 * n + 1);
                acz = at(acc, 4 * n + 2);
            }
        }
        if (!solid) {
#pragma unroll
            for (int i = 0; i < Q; i++) {
                if constexpr (BUF)
                    f[i] = R(buf_load<S>(ra, (uint32_t)n * (uint32_t)sizeof(S), (uint32_t)i * (uint32_t)a.stride * (uint32_t)sizeof(S)));
                else
                    f[i] = R(at(fa, (IDX)i * stride + n));
            }
        }

        R Fx = R(a.g[0]), Fy = R(a.g[1]), Fz = R(a.g[2]);
        if (HAS_G) {
            const R *G = static_cast<const R *>(a.gfield);
            Fx += at(G, n);
            Fy += at(G, N + n);
            Fz += at(G, 2 * N + n);
        }
        if (nmark) {
            if (tfall) {  // the spread's fallback sums, taken once
                ibx = ibx + acx;
                iby = iby + acy;
                ibz = ibz + acz;
                R *acc = static_cast<R *>(a.facc);
                at(acc, 4 * n) = R(0);
                at(acc, 4 * n + 1) = R(0);
                at(acc, 4 * n + 2) = R(0);
            }
            Fx += ibx;
            Fy += iby;
            Fz += ibz;
        }
        // the marks are cleared for the next step: every lane of a marked
        // tile stores, so the tile's 64 mark bytes go out as one whole write
        if (tmark) at(a.need, n) = 0;
        if (tmark && lane == 0) {
            a.tneed[tile] = 0;
            if (tfall) a.ftile[tile] = 0;
        }
        if (!solid) {
            if (links) {  // populations bounced back from solid neighbours lie in their slots
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    if (!((links >> opp(i)) & 1u)) continue;
                    const IDX src = pop_slot<IDX>(i, n, links, x, y, z, ch, stride, a.per);
                    if constexpr (BUF)
                        f[i] = R(buf_load<S>(ra, (uint32_t)src * (uint32_t)sizeof(S), 0u));
                    else
                        f[i] = R(at(fa, src));
                }
            }
            sum = collide<R, DEV>(f, Fx, Fy, Fz, R(a.omega), R(a.kf));
        } else {
#pragma unroll
            for (int i = 0; i < Q; i++) f[i] = DEV ? R(0) : wgt<R>(i);
        }
    }
    // The workgroup's waves store together.  Most slots of a line are written
    // by one wave, but an x-shifted store also covers the first or last
    // element of the neighbouring tile's line, which the neighbouring wave
    // (the same workgroup when it holds whole rows) completes: issued at the
    // same time, the two halves meet in L2 and the line goes to HBM once,
    // whole.  Waves left free to drift apart (one waiting on the spread
    // force, a neighbour not) leave the partial lines in L2 long enough to be
    // written back in pieces.
    __syncthreads();
    if (!live) return;
    // failure detection: a wave with a non-finite node raises the flag (a
    // wave-uniform branch; the active lanes store the same value)
    if (__builtin_amdgcn_ballot_w64(!__builtin_isfinite(sum))) *a.nonfinite = 1u;

    const int xp = (x + 1 == ch.nx) ? 0 : x + 1;
    const int xm = (x == 0) ? ch.nx - 1 : x - 1;
    const int yp = (y + 1 == ch.ny) ? 0 : y + 1;
    const int ym = (y == 0) ? ch.ny - 1 : y - 1;
    const int zp = (z + 1 == ch.nz) ? 0 : z + 1;
    const int zm = (z == 0) ? ch.nz - 1 : z - 1;
    __amdgpu_buffer_rsrc_t rrec;
    uint64_t mown = 0;
    uint32_t bown = 0;
    if constexpr (EMIT) {
        rrec = buf_rsrc(a.erec, (uint64_t)Q * (uint64_t)a.ecap * sizeof(S));
        mown = rt_mask(rt, 13);
        bown = rt_base(rt, 13);
    }
    auto stream = [&](auto ic, uint64_t m0, uint32_t b0, uint64_t ms, uint32_t bs) {
        constexpr int i = decltype(ic)::value;
        const int xq = cx(i) > 0 ? xp : (cx(i) < 0 ? xm : x);
        const int yq = cy(i) > 0 ? yp : (cy(i) < 0 ? ym : y);
        const int zq = cz(i) > 0 ? zp : (cz(i) < 0 ? zm : z);
        // streamed (into a solid node too: a bounced population waits there),
        // except across a non-periodic face, where it bounces in place
        const bool out = leaves_lattice(i, x, y, z, ch, a.per);
        if (!(solid && out)) {
            const IDX dst = out ? (IDX)opp(i) * stride + n
                                : (IDX)i * stride + base + (IDX)xq + (IDX)ch.nx * ((IDX)yq + (IDX)ch.ny * (IDX)zq);
            if constexpr (BUF)
                buf_store(S(f[i]), rb, (uint32_t)dst * (uint32_t)sizeof(S), 0u);
            else
                at(fb, dst) = S(f[i]);
        }
        if constexpr (EMIT)
            if (!solid) emit_record<i, S>(a, rrec, lane, links, m0, b0, ms, bs, mown, bown, S(f[i]));
    };
    auto stream_row = [&](auto rc) {
        constexpr int r = decltype(rc)::value;
        constexpr int i0 = kRowDirs[r][0], ip = kRowDirs[r][1], im = kRowDirs[r][2];
        constexpr int L0 = 1 + 3 * (cy(i0) + 1) + 9 * (cz(i0) + 1);  // entry of the row's tile in this column
        uint64_t m0 = 0, mp = 0, mm = 0;
        uint32_t b0 = 0, bp = 0, bm = 0;
        if constexpr (EMIT) {
            m0 = r == 0 ? mown : rt_mask(rt, L0);
            b0 = r == 0 ? bown : rt_base(rt, L0);
            if constexpr (ip >= 0) {
                mp = rt_mask(rt, L0 + 1);
                bp = rt_base(rt, L0 + 1);
                mm = rt_mask(rt, L0 - 1);
                bm = rt_base(rt, L0 - 1);
            }
        }
        stream(std::integral_constant<int, i0>{}, m0, b0, 0ull, 0u);
        if constexpr (ip >= 0) {
            stream(std::integral_constant<int, ip>{}, m0, b0, mp, bp);
            stream(std::integral_constant<int, im>{}, m0, b0, mm, bm);
        }
    };
    stream_row(std::integral_constant<int, 0>{});
    stream_row(std::integral_constant<int, 1>{});
    stream_row(std::integral_constant<int, 2>{});
    stream_row(std::integral_constant<int, 3>{});
    stream_row(std::integral_constant<int, 4>{});
    stream_row(std::integral_constant<int, 5>{});
    stream_row(std::integral_constant<int, 6>{});
    stream_row(std::integral_constant<int, 7>{});
    stream_row(std::integral_constant<int, 8>{});
}

// rho and u = (j + F_ext/2)/rho per node (solid: 0), plus per-block FP64
// partial sums of rho and j over fluid nodes.
template <class S, class R, bool DEV, bool HAS_G>
__global__ __launch_bounds__(256) void k_moments(const S *__restrict__ f, int64_t stride, PopView pv,
                                                 const R *__restrict__ G, int64_t N, double gx, double gy, double gz,
                                                 R *rho_out, R *u_out, double *partials) {
    __shared__ double red[4 * 4];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (n < N) {
        if (pv.cls[n] != CLS_SOLID) {
            double r = DEV ? 1.0 : 0.0, j[3] = {0.0, 0.0, 0.0};
            S fv[Q];
            load_node(f, stride, n, pv, fv);
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const double v = (double)fv[i];
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

// Full populations of every node (solid nodes carry none: their rest
// weights are reported).
template <class S, bool DEV>
__global__ void k_store_f64(const S *__restrict__ f, int64_t stride, int64_t N, PopView pv, double *__restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    if (pv.cls[n] == CLS_SOLID) {
#pragma unroll
        for (int i = 0; i < Q; i++) out[i * N + n] = wgt<double>(i);
        return;
    }
    S v[Q];
    load_node(f, stride, n, pv, v);
#pragma unroll
    for (int i = 0; i < Q; i++) out[i * N + n] = (double)v[i] + (DEV ? wgt<double>(i) : 0.0);
}

// Fluid nodes' populations into the slots that hold them (solid nodes'
// values are ignored: those slots may hold a neighbour's population).
template <class S, bool DEV>
__global__ void k_load_f64(S *__restrict__ f, int64_t stride, int64_t N, PopView pv, const double *__restrict__ in) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint8_t cl = pv.cls[n];
    if (cl == CLS_SOLID) return;
    const uint32_t lk = cl == CLS_WALL ? pv.links[n] : 0u;
    Chan ch{};
    int x = 0, y = 0, z = 0;
    if (lk) node_coords(pv.chans, pv.nch, n, ch, x, y, z);
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const int64_t slot = lk ? pop_slot<int64_t>(i, n, lk, x, y, z, ch, stride, pv.per) : i * stride + n;
        f[slot] = S(in[i * N + n] - (DEV ? wgt<double>(i) : 0.0));
    }
}

}  // namespace lbm

// Reverse-mode (adjoint) kernels of one coupled step.
//
// The forward step n maps (f_n, X_n, V_n; G) to (f_{n+1}, X_{n+1}, V_{n+1}):
//   u_ext = (j + F_ext/2)/rho at the stencil nodes (F_ext = g + G),
//   u_k = sum_q W_q(X_k) u_ext(x_q)                      (Sec. 2.2 step 1)
//   F_c,k = xi A_k (u_k - V_k), F_el = -grad E(X)        (step 2, Sec. 2.3)
//   F(x) = F_ext(x) + sum_k W(x - X_k)(-F_c,k)           (step 3)
//   f* = f - omega (f - f_eq(rho, u)) + S(u, F), u = (j + F/2)/rho,
//   f_{n+1} = stream(f*) with halfway bounce-back        (Sec. 2.1, 2.4)
//   V_{n+1} = V + dt/m_k (F_el + F_c), X_{n+1} = X + dt V_{n+1}   (step 4)
// Given the adjoints of the outputs (lambda_f', lambda_X', lambda_V') these
// kernels produce the adjoints of the inputs and add dJ/dG of this step:
//
// k_adj_collide_stream (one wave per tile): pull lambda* from the nodes the
//   forward pushed to, then the transposed local Jacobian of the collision,
//     lambda_f_i = (1 - omega) lambda*_i + dPhi/drho + (c_i - u).dPhi/du / rho,
//     lambda_F   = dPhi/dF + dPhi/du / (2 rho),
//   with Phi = sum_i lambda*_i (omega f_eq_i + S_i).  lambda_F is added to
//   dJ/dG and kept at the stencil nodes for the points.
// k_adj_membrane (one workgroup per cell): the membrane part of
//   lambda_X, (dF_el/dX)^T w = (dF_el/dX) w (F_el = -grad E, so its Jacobian
//   is minus the symmetric Hessian), by forward-mode dual numbers through
//   the exact energy gradient; w_k = dt/m_k (lambda_V' + dt lambda_X').
// k_adj_points (one thread per IB point): transposes of the coupling,
//   interpolation and spreading, including the derivative of the trilinear
//   weights with respect to X; lambda_u of every point is spread to the
//   stencil nodes (float atomics: the order of these adds is not fixed).
// k_adj_nodes (one wave per listed tile): the u_ext part of lambda_f and of
//   dJ/dG at the stencil nodes, lambda_f_i += (c_i - u_ext).lambda_u/rho,
//   dJ/dG += lambda_u/(2 rho).
#pragma once

#include "ibm_kernels.hpp"

namespace lbm {

// Two plain copies in one launch (4-byte words): elements [0, n0) of the
// first pair, then [0, n1) of the second.
__global__ __launch_bounds__(256) void k_copy_pair(const uint32_t *__restrict__ s0, uint32_t *__restrict__ d0,
                                                   int64_t n0, const uint32_t *__restrict__ s1,
                                                   uint32_t *__restrict__ d1, int64_t n1) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n0 + n1; i += (int64_t)gridDim.x * 256) {
        if (i < n0)
            d0[i] = s0[i];
        else
            d1[i - n0] = s1[i - n0];
    }
}

// ---------------------------------------------------------------------------
// forward-mode dual numbers (value, directional derivative)

struct Dual {
    double v, d;
};
__device__ __forceinline__ Dual mk(double v) { return {v, 0.0}; }
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.v * b.d + a.d * b.v}; }
__device__ __forceinline__ Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual operator/(Dual a, double s) { return {a.v / s, a.d / s}; }
__device__ __forceinline__ Dual dsqrt(Dual a) {
    const double r = sqrt(a.v);
    return {r, a.d / (2.0 * r)};
}
__device__ __forceinline__ Dual datan2(Dual y, Dual x) {
    return {atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / (x.v * x.v + y.v * y.v)};
}

struct DV3 {
    Dual x, y, z;
};
__device__ __forceinline__ DV3 operator-(DV3 a, DV3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ DV3 operator+(DV3 a, DV3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ DV3 operator*(Dual s, DV3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ DV3 cross(DV3 a, DV3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ Dual dotd(DV3 a, DV3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// ---------------------------------------------------------------------------
// adjoint of the fused collide-stream pass

struct AdjStepArgs {
    const void *f;         // f_n [19][stride], storage type
    const void *lam_next;  // lambda of f_{n+1} [19][stride], real
    void *lam;             // lambda of f_n [19][stride], real (written)
    int64_t stride;
    const uint32_t *links;
    const void *fibm;      // spread force of step n, valid at the marked nodes
    void *facc;            // the spread's fallback accumulator: added and cleared in flagged tiles
    uint8_t *ftile;        // tiles holding fallback sums (cleared here)
    const uint8_t *tneed;  // tile marks (the node marks stay set for k_adj_nodes)
    const uint4 *tmask;    // [ntiles] solid and wall masks of each tile
    const uint2 *tnmask;   // [ntiles] node marks of each marked tile (the recomputed velocity pass)
    void *lamF;            // [N] Vec4: lambda_F at marked nodes (written)
    void *dgrad;           // [3][N] real, dJ/dG accumulated, or null
    const void *gfield;    // [3][N] real, or null
    const Chan *chans;
    const uint16_t *tile_chan;
    int ntiles;
    int remap;             // as in StepArgs
    const uint32_t *wgtab; // [gridDim.x] workgroup table (first tile << 3 | tiles - 1), or null
    int64_t N;
    double g[3];
    double omega, kf;
    int per[3];  // periodic axes (where f_n keeps its bounced populations, see pop_slot)
};

template <class S, class R, bool DEV, bool HAS_G>
__global__ __launch_bounds__(512) void k_adj_collide_stream(AdjStepArgs a) {
    using R4 = typename Vec4<R>::T;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int tile;
    if (a.wgtab) {
        const uint32_t e = a.wgtab[blockIdx.x];
        if (wave > (int)(e & 7u)) return;
        tile = (int)(e >> 3) + wave;
    } else {
        const int blk = a.remap ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
        tile = blk * (blockDim.x >> 6) + wave;
    }
    if (tile >= a.ntiles) return;
    const Chan ch = a.chans[tile_channel(a.tile_chan, tile)];
    const int lt = tile - ch.toff, row = lt / ch.tpr;
    const int x = (lt - row * ch.tpr) * 64 + lane;
    if (x >= ch.nx) return;
    const int64_t n = ch.noff + (int64_t)row * ch.nx + x;
    const int64_t N = a.N, st = a.stride;
    // What the wave needs to know about its tile comes in scalar loads (solid
    // and wall masks, marks, fallback flag), so that the loads of f_n and of
    // lambda* go out before any vector load has to be waited for; a wall
    // node's bounced entries are loaded again once its links are in.
    const int utile = __builtin_amdgcn_readfirstlane(tile);
    const uint4 tm = uniform_load(a.tmask, utile);
    const uint2 nm = uniform_load(a.tnmask, utile);
    const uint32_t tmark = uniform_byte(a.tneed, utile), tfall = uniform_byte(a.ftile, utile);
    const bool solid = (((uint64_t)tm.y << 32 | tm.x) >> lane) & 1u;
    const bool wall = (((uint64_t)tm.w << 32 | tm.z) >> lane) & 1u;
    const bool marked = tmark && ((((uint64_t)nm.y << 32 | nm.x) >> lane) & 1u);
    const bool fl = tmark && tfall;
    R *L = static_cast<R *>(a.lam);
    R4 *LF = static_cast<R4 *>(a.lamF);
    if (fl && lane == 0) a.ftile[tile] = 0;
    if (solid) {
        if (fl && marked) {  // the fallback sums are taken (and cleared) at every marked node
            R4 *FA = static_cast<R4 *>(a.facc);
            FA[n] = R4{R(0), R(0), R(0), R(0)};
        }
#pragma unroll
        for (int i = 0; i < Q; i++) L[i * st + n] = R(0);
        if (marked) LF[n] = R4{R(0), R(0), R(0), R(0)};
        return;
    }
    const S *f = static_cast<const S *>(a.f);
    const int y = row % ch.ny, z = row / ch.ny;
    const uint32_t links = wall ? a.links[n] : 0u;
    // lambda* pulled from where population i goes (lambda is kept per node
    // and direction: a bounced population is population opp(i) of the node)
    const int xp = (x + 1 == ch.nx) ? 0 : x + 1, xm = (x == 0) ? ch.nx - 1 : x - 1;
    const int yp = (y + 1 == ch.ny) ? 0 : y + 1, ym = (y == 0) ? ch.ny - 1 : y - 1;
    const int zp = (z + 1 == ch.nz) ? 0 : z + 1, zm = (z == 0) ? ch.nz - 1 : z - 1;
    const R *LN = static_cast<const R *>(a.lam_next);
    R ls[Q], v[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const int xq = cx(i) > 0 ? xp : (cx(i) < 0 ? xm : x);
        const int yq = cy(i) > 0 ? yp : (cy(i) < 0 ? ym : y);
        const int zq = cz(i) > 0 ? zp : (cz(i) < 0 ? zm : z);
        ls[i] = LN[i * st + ch.noff + xq + (int64_t)ch.nx * (yq + (int64_t)ch.ny * zq)];
    }
#pragma unroll
    for (int i = 0; i < Q; i++) v[i] = R(f[i * st + n]);
    R Fx = R(a.g[0]), Fy = R(a.g[1]), Fz = R(a.g[2]);
    if (HAS_G) {
        const R *G = static_cast<const R *>(a.gfield);
        Fx += G[n];
        Fy += G[N + n];
        Fz += G[2 * N + n];
    }
    const R4 *FI = static_cast<const R4 *>(a.fibm);
    if (marked) {
        R4 fi = FI[n];
        if (fl) {  // the spread's fallback sums, taken once
            R4 *FA = static_cast<R4 *>(a.facc);
            const R4 fa = FA[n];
            fi = R4{fi.x + fa.x, fi.y + fa.y, fi.z + fa.z, R(0)};
            FA[n] = R4{R(0), R(0), R(0), R(0)};
        }
        Fx += fi.x;
        Fy += fi.y;
        Fz += fi.z;
    }
    if (links) {  // bounced entries: f_n in the solid neighbour's slot, lambda* in the node's own opposite slot
#pragma unroll
        for (int i = 0; i < Q; i++) {
            if ((links >> opp(i)) & 1u) v[i] = R(f[pop_slot<int64_t>(i, n, links, x, y, z, ch, st, a.per)]);
            if ((links >> i) & 1u) ls[i] = LN[opp(i) * st + n];
        }
    }
    R s = R(0);
#pragma unroll
    for (int i = 0; i < Q; i++) s += v[i];
    const R jx = (v[1] - v[2]) + (v[7] - v[8]) + (v[9] - v[10]) + (v[11] - v[12]) + (v[13] - v[14]);
    const R jy = (v[3] - v[4]) + (v[7] - v[8]) + (v[10] - v[9]) + (v[15] - v[16]) + (v[17] - v[18]);
    const R jz = (v[5] - v[6]) + (v[11] - v[12]) + (v[14] - v[13]) + (v[15] - v[16]) + (v[18] - v[17]);
    const R rho = DEV ? R(1) + s : s;
    const R ir = R(1) / rho;
    const R ux = (jx + R(0.5) * Fx) * ir, uy = (jy + R(0.5) * Fy) * ir, uz = (jz + R(0.5) * Fz) * ir;
    const R usq = R(1.5) * (ux * ux + uy * uy + uz * uz);


    // derivatives of Phi = sum_i ls_i (omega f_eq_i(rho, u) + S_i(u, F))
    const R omega = R(a.omega), kf = R(a.kf);
    R drho = R(0), dux = R(0), duy = R(0), duz = R(0), dFx = R(0), dFy = R(0), dFz = R(0);
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const R cu = R(cx(i)) * ux + R(cy(i)) * uy + R(cz(i)) * uz;
        const R cF = R(cx(i)) * Fx + R(cy(i)) * Fy + R(cz(i)) * Fz;
        const R lw = ls[i] * wgt<R>(i);
        drho += lw * (R(1) + R(3) * cu + R(4.5) * cu * cu - usq);
        // d f_eq/du = w rho (3c + 9 (c.u) c - 3u);  dS/du = kf w (9 (c.F) c - 3F)
        const R a1 = omega * rho * lw, a2 = kf * lw;
        const R cc = a1 * (R(3) + R(9) * cu) + a2 * R(9) * cF;  // coefficient of c
        const R cuu = -(a1 * R(3));                              // coefficient of u
        dux += cc * R(cx(i)) + cuu * ux - a2 * R(3) * Fx;
        duy += cc * R(cy(i)) + cuu * uy - a2 * R(3) * Fy;
        duz += cc * R(cz(i)) + cuu * uz - a2 * R(3) * Fz;
        // dS/dF = kf w (3 (c - u) + 9 (c.u) c)
        const R cf = a2 * (R(3) + R(9) * cu);
        dFx += cf * R(cx(i)) - a2 * R(3) * ux;
        dFy += cf * R(cy(i)) - a2 * R(3) * uy;
        dFz += cf * R(cz(i)) - a2 * R(3) * uz;
    }
    drho *= omega;
    const R one_m = R(1) - omega;
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const R cdu = (R(cx(i)) - ux) * dux + (R(cy(i)) - uy) * duy + (R(cz(i)) - uz) * duz;
        L[i * st + n] = one_m * ls[i] + drho + cdu * ir;
    }
    const R h = R(0.5) * ir;
    const R lFx = dFx + h * dux, lFy = dFy + h * duy, lFz = dFz + h * duz;
    if (a.dgrad) {
        R *DG = static_cast<R *>(a.dgrad);
        DG[n] += lFx;
        DG[N + n] += lFy;
        DG[2 * N + n] += lFz;
    }
    if (marked) LF[n] = R4{lFx, lFy, lFz, R(0)};
}

// ---------------------------------------------------------------------------
// membrane force Jacobian times a direction, by dual numbers

struct JvpArgs {
    const int32_t *vert_off, *tri_off, *edge_off, *tri, *hinge;
    const int32_t *vtri_off, *vtri, *vedge_off, *vedge;
    const double *x;  // [3][nverts] positions (offsets from the anchors)
    // direction: w given, or w_k = dt/m_k (lam_v + dt lam_x) when lam_x is set
    const double *w;
    const double *lam_x, *lam_v;
    double dt, mass;
    const void *moduli;
    const double *l0, *a0, *th0, *a0c, *v0c, *avert;
    int ncells, nverts, ntris, nedges, maxv;
    int stretch_law;
    double *f_out;    // [3][nverts] F_el(X) in FP64, or null
    double *jvp_out;  // [3][nverts] (dF_el/dX) w
};

template <class R>
__global__ __launch_bounds__(kMembThreads) void k_adj_membrane(JvpArgs a) {
    extern __shared__ double smem_d[];
    const int c = blockIdx.x;
    const int v0 = a.vert_off[c], nv = a.vert_off[c + 1] - v0;
    const int t0 = a.tri_off[c], nt = a.tri_off[c + 1] - t0;
    const int e0 = a.edge_off[c];
    const int NV = a.nverts, NT = a.ntris, NE = a.nedges, NC = a.ncells;
    double *red = smem_d;
    double *px = smem_d + 4 * (kMembThreads / 64), *py = px + a.maxv, *pz = py + a.maxv;
    double *wx = pz + a.maxv, *wy = wx + a.maxv, *wz = wy + a.maxv;
    for (int k = threadIdx.x; k < nv; k += blockDim.x) {
        const int g = v0 + k;
        px[k] = a.x[g];
        py[k] = a.x[NV + g];
        pz[k] = a.x[2 * NV + g];
        if (a.lam_x) {
            const double h = a.dt / (a.mass * a.avert[g]);
            wx[k] = h * (a.lam_v[g] + a.dt * a.lam_x[g]);
            wy[k] = h * (a.lam_v[NV + g] + a.dt * a.lam_x[NV + g]);
            wz[k] = h * (a.lam_v[2 * NV + g] + a.dt * a.lam_x[2 * NV + g]);
        } else {
            wx[k] = a.w[g];
            wy[k] = a.w[NV + g];
            wz[k] = a.w[2 * NV + g];
        }
    }
    __syncthreads();
    auto P = [&](int gvert) {
        const int k = gvert - v0;
        return DV3{{px[k], wx[k]}, {py[k], wy[k]}, {pz[k], wz[k]}};
    };

    // cell area and volume with their directional derivatives
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
        const DV3 A = P(a.tri[t0 + t]), B = P(a.tri[NT + t0 + t]), C = P(a.tri[2 * NT + t0 + t]);
        const DV3 n = cross(B - A, C - A);
        const Dual ar = 0.5 * dsqrt(dotd(n, n));
        const Dual vo = dotd(A, cross(B, C)) / 6.0;
        acc[0] += ar.v;
        acc[1] += ar.d;
        acc[2] += vo.v;
        acc[3] += vo.d;
    }
    block_sum<4>(acc, red);
    const R *mod = static_cast<const R *>(a.moduli);
    const double ks = mod[c], kb = mod[NC + c], kal = mod[2 * NC + c], kag = mod[3 * NC + c], kv = mod[4 * NC + c];
    const Dual Ac{acc[0], acc[1]}, Vc{acc[2], acc[3]};
    const Dual cag = (kag / a.a0c[c]) * (Ac - mk(a.a0c[c]));
    const Dual cv6 = (kv / a.v0c[c] / 6.0) * (Vc - mk(a.v0c[c]));

    for (int k = threadIdx.x; k < nv; k += blockDim.x) {
        const int vg = v0 + k;
        DV3 F{mk(0.0), mk(0.0), mk(0.0)};
        for (int i = a.vtri_off[vg]; i < a.vtri_off[vg + 1]; i++) {
            const int code = a.vtri[i], t = code >> 2, r = code & 3;
            const DV3 A = P(a.tri[t]), B = P(a.tri[NT + t]), C = P(a.tri[2 * NT + t]);
            const DV3 n = cross(B - A, C - A);
            const Dual nn = dsqrt(dotd(n, n));
            const double ref = a.a0[t];
            const Dual h = (-0.5) * ((kal / ref) * (0.5 * nn - mk(ref)) + cag) / nn;
            const DV3 nx_ = r == 0 ? B : (r == 1 ? C : A), pv = r == 0 ? C : (r == 1 ? A : B);
            F = F + h * cross(nx_ - pv, n) - cv6 * cross(nx_, pv);
        }
        for (int i = a.vedge_off[vg]; i < a.vedge_off[vg + 1]; i++) {
            const int code = a.vedge[i], e = code >> 2, r = code & 3;
            const DV3 p1 = P(a.hinge[e]), p2 = P(a.hinge[NE + e]);
            const DV3 qa = P(a.hinge[2 * NE + e]), qb = P(a.hinge[3 * NE + e]);
            const DV3 ev = p2 - p1;
            const DV3 na = cross(ev, qa - p1), nb = cross(p1 - p2, qb - p2);
            const Dual l2 = dotd(ev, ev), l = dsqrt(l2);
            const Dual th = datan2(dotd(cross(na, nb), ev) / l, dotd(na, nb));
            const double ref = a.l0[e];
            const Dual lam = l / ref;
            const Dual cs = (a.stretch_law ? (ks / 3.0) * (lam - mk(1.0) / (lam * lam)) : (ks / ref) * (l - mk(ref))) / l;
            const Dual cb = kb * (th - mk(a.th0[e]));
            const DV3 ga = (-(l / dotd(na, na))) * na, gb = (-(l / dotd(nb, nb))) * nb;
            DV3 gth;
            Dual sc = mk(0.0);
            if (r == 2) {
                gth = ga;
            } else if (r == 3) {
                gth = gb;
            } else {
                const Dual sa = dotd(qa - p1, ev) / l2, sb = dotd(qb - p1, ev) / l2;
                const Dual ca_ = r == 0 ? (sa - mk(1.0)) : -sa, cb_ = r == 0 ? (sb - mk(1.0)) : -sb;
                gth = ca_ * ga + cb_ * gb;
                sc = r == 0 ? cs : -cs;
            }
            F = F + sc * ev - cb * gth;
        }
        if (a.f_out) {
            a.f_out[vg] = F.x.v;
            a.f_out[NV + vg] = F.y.v;
            a.f_out[2 * NV + vg] = F.z.v;
        }
        a.jvp_out[vg] = F.x.d;
        a.jvp_out[NV + vg] = F.y.d;
        a.jvp_out[2 * NV + vg] = F.z.d;
    }
}

__host__ __device__ inline size_t adj_membrane_lds_bytes(int maxv) {
    return 4 * (kMembThreads / 64) * sizeof(double) + 6 * (size_t)maxv * sizeof(double);
}

// ---------------------------------------------------------------------------
// adjoint of the point half: coupling, interpolation, spreading, update

struct AdjPointArgs {
    const void *ufield;  // [N] Vec4 (u_ext of step n at the stencil nodes)
    const void *lamF;    // [N] Vec4 lambda_F at the stencil nodes
    void *lamU;          // [N] Vec4 lambda of u_ext (accumulated here)
    const Chan *chans;
    const int32_t *cell_chan;
    const int32_t *vert_off, *anchor;
    const double *x;     // X_n offsets [3][nverts]
    const void *v;       // V_n [3][nverts] real
    const double *hv;    // membrane part (dF_el/dX) w
    double *lam_x;       // in: lambda of X_{n+1}; out: of X_n
    double *lam_v;       // in: lambda of V_{n+1}; out: of V_n
    const double *avert;
    int ncells, nverts;
    double xi, mass, dt;
};

template <class R>
__global__ __launch_bounds__(128) void k_adj_points(AdjPointArgs a) {
    using R4 = typename Vec4<R>::T;
    const int c = blockIdx.y;
    const int vb = a.vert_off[c], ve = a.vert_off[c + 1];
    const int k = vb + blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ve) return;
    const int NV = a.nverts;
    const double ox = a.x[k], oy = a.x[NV + k], oz = a.x[2 * NV + k];
    const double flx = floor(ox), fly = floor(oy), flz = floor(oz);
    const double dx = ox - flx, dy = oy - fly, dz = oz - flz;
    const Chan ch = a.chans[cell_channel(a.cell_chan, c)];
    const int x0 = pmod(a.anchor[c] + (int)flx, ch.nx);
    const int y0 = pmod(a.anchor[a.ncells + c] + (int)fly, ch.ny);
    const int z0 = pmod(a.anchor[2 * a.ncells + c] + (int)flz, ch.nz);
    const int xs[2] = {x0, x0 + 1 == ch.nx ? 0 : x0 + 1};
    const int ys[2] = {y0, y0 + 1 == ch.ny ? 0 : y0 + 1};
    const int zs[2] = {z0, z0 + 1 == ch.nz ? 0 : z0 + 1};
    const double wx[2] = {1.0 - dx, dx}, wy[2] = {1.0 - dy, dy}, wz[2] = {1.0 - dz, dz};
    const double sg[2] = {-1.0, 1.0};
    const R4 *U = static_cast<const R4 *>(a.ufield);
    const R4 *LF = static_cast<const R4 *>(a.lamF);
    int64_t nq[8];
    double uq[8][3], lq[8][3];
    double ux = 0.0, uy = 0.0, uz = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int bx = q & 1, by = (q >> 1) & 1, bz = q >> 2;
        nq[q] = ch.noff + xs[bx] + (int64_t)ch.nx * (ys[by] + (int64_t)ch.ny * zs[bz]);
        const R4 u = U[nq[q]], l = LF[nq[q]];
        uq[q][0] = u.x, uq[q][1] = u.y, uq[q][2] = u.z;
        lq[q][0] = l.x, lq[q][1] = l.y, lq[q][2] = l.z;
        const double wt = wx[bx] * wy[by] * wz[bz];
        ux += wt * uq[q][0];
        uy += wt * uq[q][1];
        uz += wt * uq[q][2];
        sx += wt * lq[q][0];
        sy += wt * lq[q][1];
        sz += wt * lq[q][2];
    }
    const R *Vv = static_cast<const R *>(a.v);
    const double ak = a.avert[k], xia = a.xi * ak, h = a.dt / (a.mass * ak);
    const double fcx = xia * (ux - (double)Vv[k]), fcy = xia * (uy - (double)Vv[NV + k]),
                 fcz = xia * (uz - (double)Vv[2 * NV + k]);
    double *LX = a.lam_x, *LV = a.lam_v;
    const double mx = LV[k] + a.dt * LX[k], my = LV[NV + k] + a.dt * LX[NV + k],
                 mz = LV[2 * NV + k] + a.dt * LX[2 * NV + k];
    // lambda of F_c: from the spread force (-F_c) and from the velocity update
    const double lcx = -sx + h * mx, lcy = -sy + h * my, lcz = -sz + h * mz;
    const double lux = xia * lcx, luy = xia * lcy, luz = xia * lcz;
    double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int bx = q & 1, by = (q >> 1) & 1, bz = q >> 2;
        const double s = -(fcx * lq[q][0] + fcy * lq[q][1] + fcz * lq[q][2]) +
                         (uq[q][0] * lux + uq[q][1] * luy + uq[q][2] * luz);
        gx += s * sg[bx] * wy[by] * wz[bz];
        gy += s * wx[bx] * sg[by] * wz[bz];
        gz += s * wx[bx] * wy[by] * sg[bz];
    }
    LX[k] += a.hv[k] + gx;
    LX[NV + k] += a.hv[NV + k] + gy;
    LX[2 * NV + k] += a.hv[2 * NV + k] + gz;
    LV[k] = mx - xia * lcx;
    LV[NV + k] = my - xia * lcy;
    LV[2 * NV + k] = mz - xia * lcz;
    R4 *LU = static_cast<R4 *>(a.lamU);
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int bx = q & 1, by = (q >> 1) & 1, bz = q >> 2;
        const double wt = wx[bx] * wy[by] * wz[bz];
        R *rec = reinterpret_cast<R *>(&LU[nq[q]]);
        atomicAdd(rec + 0, R(wt * lux));
        atomicAdd(rec + 1, R(wt * luy));
        atomicAdd(rec + 2, R(wt * luz));
    }
}

// ---------------------------------------------------------------------------
// u_ext part at the stencil nodes; clears lambda_u and the marks

struct AdjNodeArgs {
    const uint32_t *tlist, *tcount;
    uint8_t *need, *tneed;
    const void *ufield;  // [N] Vec4 (u_ext, rho)
    void *lamU;          // [N] Vec4 (read and cleared)
    void *lam;           // [19][stride] real
    void *dgrad;         // [3][N] real or null
    const uint8_t *cls;
    const Chan *chans;
    const uint16_t *tile_chan;
    int64_t stride, N;
};

template <class R>
__global__ __launch_bounds__(256) void k_adj_nodes(AdjNodeArgs a) {
    using R4 = typename Vec4<R>::T;
    const int lane = threadIdx.x & 63;
    const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
    const uint32_t count = *a.tcount;
    R4 *LU = static_cast<R4 *>(a.lamU);
    const R4 *U = static_cast<const R4 *>(a.ufield);
    R *L = static_cast<R *>(a.lam);
    for (uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < count; w += nwaves) {
        const int tile = __builtin_amdgcn_readfirstlane((int)a.tlist[w]);
        const Chan ch = a.chans[tile_channel(a.tile_chan, tile)];
        const int lt = tile - ch.toff, row = lt / ch.tpr;
        const int x = (lt - row * ch.tpr) * 64 + lane;
        if (lane == 0) a.tneed[tile] = 0;
        if (x >= ch.nx) continue;
        const int64_t n = ch.noff + (int64_t)row * ch.nx + x;
        if (!a.need[n]) continue;
        a.need[n] = 0;
        const R4 lu = LU[n];
        LU[n] = R4{R(0), R(0), R(0), R(0)};
        if (a.cls[n] == CLS_SOLID) continue;  // u_ext is fixed at 0 there
        const R4 u = U[n];
        const R ir = R(1) / u.w;
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const R cdu = (R(cx(i)) - u.x) * lu.x + (R(cy(i)) - u.y) * lu.y + (R(cz(i)) - u.z) * lu.z;
            L[i * a.stride + n] += cdu * ir;
        }
        if (a.dgrad) {
            R *DG = static_cast<R *>(a.dgrad);
            const R h = R(0.5) * ir;
            DG[n] += h * lu.x;
            DG[a.N + n] += h * lu.y;
            DG[2 * a.N + n] += h * lu.z;
        }
    }
}

}  // namespace lbm

// Immersed-boundary kernels (Sec. 2.2) and membrane forces (Sec. 2.3).
//
// k_membrane: one workgroup per cell.  The cell's vertex offsets are staged
// in LDS; the cell's total area and volume (the global constraints that need
// every vertex of the cell, Sec. 2.3.3) are reduced in FP64 first, then each
// triangle and each edge/hinge adds its energy gradient to its vertices with
// LDS atomics, and the result is written out once.
//
// k_couple: one thread per IB point: trilinear interpolation of the fluid
// velocity from the 8 surrounding nodes, coupling force, spreading of its
// reaction onto the same 8 nodes (global atomics into the force
// accumulator, tile flags for the collide kernel), then the point update.
#pragma once

#include "d3q19.hpp"
#include "lattice_kernels.hpp"

namespace lbm {

// ---- geometry helpers --------------------------------------------------
// Contraction is switched off here so that the rest shape and the later
// force evaluations compute bit-identical lengths, areas and angles from the
// same positions (undeformed cells then feel exactly zero force).

template <class R>
struct V3 {
    R x, y, z;
};
template <class R>
__device__ __forceinline__ V3<R> sub(V3<R> a, V3<R> b) {
#pragma clang fp contract(off)
    return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <class R>
__device__ __forceinline__ V3<R> crs(V3<R> a, V3<R> b) {
#pragma clang fp contract(off)
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class R>
__device__ __forceinline__ R dot(V3<R> a, V3<R> b) {
#pragma clang fp contract(off)
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <class R>
__device__ __forceinline__ V3<R> scl(R s, V3<R> a) {
    return {s * a.x, s * a.y, s * a.z};
}

// Unnormalised outward normal (b-a)x(c-a); area = |n|/2.
template <class R>
__device__ __forceinline__ V3<R> tri_normal(V3<R> a, V3<R> b, V3<R> c) {
    return crs(sub(b, a), sub(c, a));
}
template <class R>
__device__ __forceinline__ R tri_area(V3<R> n) {
#pragma clang fp contract(off)
    return R(0.5) * sqrt(dot(n, n));
}
// a.(b x c)/6: volume of the tetrahedron (anchor, a, b, c).
template <class R>
__device__ __forceinline__ R tri_vol(V3<R> a, V3<R> b, V3<R> c) {
#pragma clang fp contract(off)
    return dot(a, crs(b, c)) / R(6);
}
// Signed angle between the outward normals of (p1,p2,qa) and (p2,p1,qb):
// zero when flat, positive for a convex fold.
template <class R>
__device__ __forceinline__ R hinge_angle(V3<R> p1, V3<R> p2, V3<R> qa, V3<R> qb, V3<R> &na, V3<R> &nb, V3<R> &e) {
#pragma clang fp contract(off)
    e = sub(p2, p1);
    na = crs(e, sub(qa, p1));
    nb = crs(sub(p1, p2), sub(qb, p2));
    const R s = dot(crs(na, nb), e) / sqrt(dot(e, e));
    const R c = dot(na, nb);
    return atan2(s, c);
}

struct MembArgs {
    const int32_t *vert_off, *tri_off, *edge_off, *tri, *hinge;
    const void *x;  // [3][nverts] offsets
    void *f_el;     // [3][nverts]
    const void *moduli;
    void *l0, *a0, *th0;
    double *a0c, *v0c;
    int ncells, nverts, ntris, nedges, maxv;
};

// REST = true: write the rest shape; false: elastic forces.
template <class R, bool REST>
__global__ __launch_bounds__(256) void k_membrane(MembArgs a) {
    extern __shared__ double smem_d[];
    const int c = blockIdx.x;
    const int v0 = a.vert_off[c], nv = a.vert_off[c + 1] - v0;
    const int t0 = a.tri_off[c], nt = a.tri_off[c + 1] - t0;
    const int e0 = a.edge_off[c], ne = a.edge_off[c + 1] - e0;
    double *red = smem_d;  // 4 waves x 2
    R *px = reinterpret_cast<R *>(smem_d + 8);
    R *py = px + a.maxv, *pz = py + a.maxv;
    R *fx = pz + a.maxv, *fy = fx + a.maxv, *fz = fy + a.maxv;
    const R *X = static_cast<const R *>(a.x);
    const int NV = a.nverts;
    for (int k = threadIdx.x; k < nv; k += blockDim.x) {
        px[k] = X[v0 + k];
        py[k] = X[NV + v0 + k];
        pz[k] = X[2 * NV + v0 + k];
        if (!REST) fx[k] = fy[k] = fz[k] = R(0);
    }
    __syncthreads();
    auto P = [&](int k) { return V3<R>{px[k], py[k], pz[k]}; };
    const int NT = a.ntris, NE = a.nedges;

    // cell area and volume (FP64 sums of per-triangle values)
    double acc[2] = {0.0, 0.0};
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
        const V3<R> A = P(a.tri[t0 + t] - v0), B = P(a.tri[NT + t0 + t] - v0), C = P(a.tri[2 * NT + t0 + t] - v0);
        acc[0] += (double)tri_area(tri_normal(A, B, C));
        acc[1] += (double)tri_vol(A, B, C);
    }
    block_sum<2>(acc, red);
    if (REST) {
        if (threadIdx.x == 0) {
            a.a0c[c] = acc[0];
            a.v0c[c] = acc[1];
        }
    }
    const R *mod = static_cast<const R *>(a.moduli);
    const int NC = a.ncells;
    const R ks = mod[c], kb = mod[NC + c], kal = mod[2 * NC + c];
    const double kag = (double)mod[3 * NC + c], kv = (double)mod[4 * NC + c];
    const R cag = REST ? R(0) : R(kag * (acc[0] - a.a0c[c]) / a.a0c[c]);
    const R cv6 = REST ? R(0) : R(kv * (acc[1] - a.v0c[c]) / a.v0c[c] / 6.0);
    R *A0 = static_cast<R *>(a.a0), *L0 = static_cast<R *>(a.l0), *TH0 = static_cast<R *>(a.th0);

    // triangles: local + global area, volume
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
        const int ia = a.tri[t0 + t] - v0, ib = a.tri[NT + t0 + t] - v0, ic = a.tri[2 * NT + t0 + t] - v0;
        const V3<R> A = P(ia), B = P(ib), C = P(ic);
        const V3<R> n = tri_normal(A, B, C);
        const R area = tri_area(n);
        if (REST) {
            A0[t0 + t] = area;
            continue;
        }
        const R ref = A0[t0 + t];
        const R ca = kal * (area - ref) / ref + cag;
        const R h = -R(0.5) * ca / (R(2) * area);  // -ca/2 * (1/|n|), |n| = 2 area
        // -ca * grad_a A = -ca/2 (b - c) x n_hat, cyclic
        const V3<R> ga = crs(sub(B, C), n), gb = crs(sub(C, A), n), gc = crs(sub(A, B), n);
        const V3<R> va = crs(B, C), vb = crs(C, A), vc = crs(A, B);
        atomicAdd(&fx[ia], h * ga.x - cv6 * va.x);
        atomicAdd(&fy[ia], h * ga.y - cv6 * va.y);
        atomicAdd(&fz[ia], h * ga.z - cv6 * va.z);
        atomicAdd(&fx[ib], h * gb.x - cv6 * vb.x);
        atomicAdd(&fy[ib], h * gb.y - cv6 * vb.y);
        atomicAdd(&fz[ib], h * gb.z - cv6 * vb.z);
        atomicAdd(&fx[ic], h * gc.x - cv6 * vc.x);
        atomicAdd(&fy[ic], h * gc.y - cv6 * vc.y);
        atomicAdd(&fz[ic], h * gc.z - cv6 * vc.z);
    }
    // edges: stretching and bending
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        const int i1 = a.hinge[e0 + e] - v0, i2 = a.hinge[NE + e0 + e] - v0;
        const int ia = a.hinge[2 * NE + e0 + e] - v0, ib = a.hinge[3 * NE + e0 + e] - v0;
        const V3<R> p1 = P(i1), p2 = P(i2), qa = P(ia), qb = P(ib);
        V3<R> na, nb, ev;
        const R th = hinge_angle(p1, p2, qa, qb, na, nb, ev);
        const R l = sqrt(dot(ev, ev));
        if (REST) {
            L0[e0 + e] = l;
            TH0[e0 + e] = th;
            continue;
        }
        const R ref = L0[e0 + e];
        const R cs = ks * (l - ref) / ref / l;  // force on p1 = cs (p2 - p1)
        const R cb = kb * (th - TH0[e0 + e]);
        // d theta/d qa = -|e| na/|na|^2, d theta/d qb = -|e| nb/|nb|^2; the edge ends
        // take the combinations that keep net force and torque zero.
        const V3<R> ga = scl(-l / dot(na, na), na), gb = scl(-l / dot(nb, nb), nb);
        const R il2 = R(1) / (l * l);
        const R sa = dot(sub(qa, p1), ev) * il2, sb = dot(sub(qb, p1), ev) * il2;
        const V3<R> g1 = {-(R(1) - sa) * ga.x - (R(1) - sb) * gb.x, -(R(1) - sa) * ga.y - (R(1) - sb) * gb.y,
                          -(R(1) - sa) * ga.z - (R(1) - sb) * gb.z};
        const V3<R> g2 = {-sa * ga.x - sb * gb.x, -sa * ga.y - sb * gb.y, -sa * ga.z - sb * gb.z};
        atomicAdd(&fx[i1], cs * ev.x - cb * g1.x);
        atomicAdd(&fy[i1], cs * ev.y - cb * g1.y);
        atomicAdd(&fz[i1], cs * ev.z - cb * g1.z);
        atomicAdd(&fx[i2], -cs * ev.x - cb * g2.x);
        atomicAdd(&fy[i2], -cs * ev.y - cb * g2.y);
        atomicAdd(&fz[i2], -cs * ev.z - cb * g2.z);
        atomicAdd(&fx[ia], -cb * ga.x);
        atomicAdd(&fy[ia], -cb * ga.y);
        atomicAdd(&fz[ia], -cb * ga.z);
        atomicAdd(&fx[ib], -cb * gb.x);
        atomicAdd(&fy[ib], -cb * gb.y);
        atomicAdd(&fz[ib], -cb * gb.z);
    }
    if (REST) return;
    __syncthreads();
    R *FE = static_cast<R *>(a.f_el);
    for (int k = threadIdx.x; k < nv; k += blockDim.x) {
        FE[v0 + k] = fx[k];
        FE[NV + v0 + k] = fy[k];
        FE[2 * NV + v0 + k] = fz[k];
    }
}

struct CoupleArgs {
    const void *f;  // current populations
    int64_t stride;
    const uint8_t *cls;
    const void *gfield;
    void *fibm;
    uint8_t *tflag;
    int nx, ny, nz, tpr;
    int64_t N;
    double g[3];
    const int32_t *vert_off, *anchor;
    void *x, *v;
    const void *f_el;
    int ncells, nverts;
    double xi, dt_over_m, dt;
};

// u_ext = (j + F_ext/2)/rho at node n from its current populations.
template <class S, class R, bool DEV, bool HAS_G>
__device__ __forceinline__ void node_velocity(const CoupleArgs &a, int64_t n, R &ux, R &uy, R &uz) {
    const S *f = static_cast<const S *>(a.f);
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
    const R ir = R(1) / (DEV ? R(1) + s : s);
    ux = (jx + R(0.5) * Fx) * ir;
    uy = (jy + R(0.5) * Fy) * ir;
    uz = (jz + R(0.5) * Fz) * ir;
}

template <class S, class R, bool DEV, bool HAS_G>
__global__ __launch_bounds__(128) void k_couple(CoupleArgs a) {
    const int c = blockIdx.y;
    const int vb = a.vert_off[c], ve = a.vert_off[c + 1];
    const int k = vb + blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ve) return;
    const int NV = a.nverts;
    R *X = static_cast<R *>(a.x);
    R *Vv = static_cast<R *>(a.v);
    const R *FE = static_cast<const R *>(a.f_el);
    const R ox = X[k], oy = X[NV + k], oz = X[2 * NV + k];
    const R flx = floor(ox), fly = floor(oy), flz = floor(oz);
    const R dx = ox - flx, dy = oy - fly, dz = oz - flz;
    const int x0 = pmod(a.anchor[c] + (int)flx, a.nx);
    const int y0 = pmod(a.anchor[a.ncells + c] + (int)fly, a.ny);
    const int z0 = pmod(a.anchor[2 * a.ncells + c] + (int)flz, a.nz);
    const int xs[2] = {x0, x0 + 1 == a.nx ? 0 : x0 + 1};
    const int ys[2] = {y0, y0 + 1 == a.ny ? 0 : y0 + 1};
    const int zs[2] = {z0, z0 + 1 == a.nz ? 0 : z0 + 1};
    const R wx[2] = {R(1) - dx, dx}, wy[2] = {R(1) - dy, dy}, wz[2] = {R(1) - dz, dz};

    // step 1: interpolate u_ext
    R ux = R(0), uy = R(0), uz = R(0);
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int bx = q & 1, by = (q >> 1) & 1, bz = q >> 2;
        const int64_t n = xs[bx] + (int64_t)a.nx * (ys[by] + (int64_t)a.ny * zs[bz]);
        if (a.cls[n] == CLS_SOLID) continue;
        R u, v, w;
        node_velocity<S, R, DEV, HAS_G>(a, n, u, v, w);
        const R wt = wx[bx] * wy[by] * wz[bz];
        ux += wt * u;
        uy += wt * v;
        uz += wt * w;
    }
    // step 2: coupling force
    const R vx = Vv[k], vy = Vv[NV + k], vz = Vv[2 * NV + k];
    const R xi = R(a.xi);
    const R fcx = xi * (ux - vx), fcy = xi * (uy - vy), fcz = xi * (uz - vz);
    // step 3: spread -F_c
    R *FI = static_cast<R *>(a.fibm);
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int bx = q & 1, by = (q >> 1) & 1, bz = q >> 2;
        const int row = ys[by] + a.ny * zs[bz];
        const int64_t n = xs[bx] + (int64_t)a.nx * row;
        const R wt = wx[bx] * wy[by] * wz[bz];
        atomicAdd(&FI[n], -wt * fcx);
        atomicAdd(&FI[a.N + n], -wt * fcy);
        atomicAdd(&FI[2 * a.N + n], -wt * fcz);
        a.tflag[(int64_t)row * a.tpr + (xs[bx] >> 6)] = 1;
    }
    // step 4 (points): semi-implicit Euler
    const R h = R(a.dt_over_m), dt = R(a.dt);
    const R nvx = vx + h * (FE[k] + fcx), nvy = vy + h * (FE[NV + k] + fcy), nvz = vz + h * (FE[2 * NV + k] + fcz);
    Vv[k] = nvx;
    Vv[NV + k] = nvy;
    Vv[2 * NV + k] = nvz;
    X[k] = ox + dt * nvx;
    X[NV + k] = oy + dt * nvy;
    X[2 * NV + k] = oz + dt * nvz;
}

}  // namespace lbm

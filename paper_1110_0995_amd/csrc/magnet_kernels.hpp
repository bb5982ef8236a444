// Kernels of the magnetic bead stage (Sec. 2.5): sheet field in closed
// form, induced moments and gradient force, all-pairs dipole interaction and
// repulsion, the overdamped update, and fixing the beads into the solid mask.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mag {

constexpr int kMaxSheets = 8;
constexpr int kPairThreads = 256;  // targets per pair block = sources per LDS tile
constexpr double kPi = 3.14159265358979323846;

enum { M_APPLY = 1, M_MOMENTS = 2, M_TOTAL = 4 };

struct MagArgs {
    double sheet[kMaxSheets][6];  // (zs, x0, x1, y0, y1, sigma)
    double bias[3];
    double alpha;      // 4 pi a^3 chi/(chi + 3)
    double mob;        // dt/(6 pi eta a)
    double a;
    double rep_a, rep_n, rep_cut, rep_dmin;
    int rep_pow;       // n + 1 when that is an integer in [1, 16] (the force by products), else 0
    double L[3];       // periodic lengths
    double ztop;       // nz - 3/2
    int per[3];
    int nsheets;
    int walls;
    int n;
    int nslice;        // source slices of the pair kernel
    int slice_len;     // sources per slice (multiple of kPairThreads)
    double *x;         // [3][n]
    double *m;         // [3][n]
    double *fs;        // [3][n] gradient + wall force
    double *part;      // [nslice][3][n] pair forces per source slice
    double *fout;      // [3][n] total force (M_TOTAL)
};

// ln(Y + R) with R = sqrt(X^2 + Y^2 + w^2), without cancellation for Y < 0
__device__ __forceinline__ double log_yr(double Y, double R, double q) {
    return Y >= 0.0 ? log(Y + R) : log(q / (R - Y));  // q = X^2 + w^2 = (R + Y)(R - Y)
}
// 1/(Y + R), likewise
__device__ __forceinline__ double inv_yr(double Y, double R, double q) { return Y >= 0.0 ? 1.0 / (Y + R) : (R - Y) / q; }

// Field of one charged rectangle at p and its gradient (upper triangle
// xx, yy, xy, xz, yz; zz = -xx - yy), added into B and J: the Coulomb
// kernel integrated over the rectangle has, at each corner (X, Y) relative
// to p (w = pz - zs, R = |(X, Y, w)|), the antiderivatives ln(Y + R),
// ln(X + R) and atan(XY/(wR)), combined with signs (+ - - +).
__device__ __forceinline__ void sheet_field(const double *S, double px, double py, double pz, double B[3],
                                            double J[5]) {
    const double w = pz - S[0], w2 = w * w;
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, jxx = 0.0, jyy = 0.0, jxy = 0.0, jxz = 0.0, jyz = 0.0;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const int i = c & 1, j = c >> 1;
        const double s = (i == j) ? 1.0 : -1.0;
        const double X = (i ? S[2] : S[1]) - px, Y = (j ? S[4] : S[3]) - py;
        const double qx = X * X + w2, qy = Y * Y + w2;  // qx pairs with Y, qy with X
        const double R = sqrt(qx + Y * Y), iR = 1.0 / R;
        const double iy = inv_yr(Y, R, qx), ix = inv_yr(X, R, qy);
        b0 += s * log_yr(Y, R, qx);
        b1 += s * log_yr(X, R, qy);
        b2 += s * atan(X * Y / (w * R));
        jxx -= s * X * iR * iy;
        jyy -= s * Y * iR * ix;
        jxy -= s * iR;
        jxz += s * w * iR * iy;
        jyz += s * w * iR * ix;
    }
    const double k = S[5] / (4.0 * kPi);
    B[0] += k * b0;
    B[1] += k * b1;
    B[2] += k * b2;
    J[0] += k * jxx;
    J[1] += k * jyy;
    J[2] += k * jxy;
    J[3] += k * jxz;
    J[4] += k * jyz;
}

__device__ __forceinline__ double rep_force(const MagArgs &A, double g) {
    if (g >= A.rep_cut) return 0.0;
    return A.rep_n * A.rep_a * pow(g < A.rep_dmin ? A.rep_dmin : g, -A.rep_n - 1.0);
}

__device__ __forceinline__ double min_image(double d, double L, int per) {
    return per ? d - L * floor(d / L + 0.5) : d;
}

// Field (and gradient) at points: one thread per point.
struct FieldArgs {
    double sheet[kMaxSheets][6];
    double bias[3];
    int nsheets, npts;
    const double *p;
    double *B, *J;  // J may be null
};

__global__ void k_mag_field(FieldArgs A) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.npts) return;
    const int n = A.npts;
    const double px = A.p[k], py = A.p[n + k], pz = A.p[2 * n + k];
    double B[3] = {A.bias[0], A.bias[1], A.bias[2]}, J[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < A.nsheets; s++) sheet_field(A.sheet[s], px, py, pz, B, J);
    for (int d = 0; d < 3; d++) A.B[d * n + k] = B[d];
    if (A.J) {
        const double full[9] = {J[0], J[2], J[3], J[2], J[1], J[4], J[3], J[4], -J[0] - J[1]};
        for (int d = 0; d < 9; d++) A.J[d * n + k] = full[d];
    }
}

// One thread per bead.  M_APPLY / M_TOTAL: total force f = fs + the pair
// partials (slices in order); M_TOTAL writes it to fout, M_APPLY moves the
// bead by mob f.  M_MOMENTS: moment and gradient + wall force at the
// (moved) position.
__global__ void k_mag_self(MagArgs A, int mode) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.n) return;
    const int n = A.n;
    double p[3] = {A.x[k], A.x[n + k], A.x[2 * n + k]};
    if (mode & (M_APPLY | M_TOTAL)) {
        double f[3];
        for (int d = 0; d < 3; d++) {
            double s = 0.0;
            for (int q = 0; q < A.nslice; q++) s += A.part[((int64_t)q * 3 + d) * n + k];
            f[d] = A.fs[d * n + k] + s;
        }
        if (mode & M_TOTAL)
            for (int d = 0; d < 3; d++) A.fout[d * n + k] = f[d];
        if (mode & M_APPLY)
            for (int d = 0; d < 3; d++) {
                p[d] += A.mob * f[d];
                A.x[d * n + k] = p[d];
            }
    }
    if (mode & M_MOMENTS) {
        double B[3] = {A.bias[0], A.bias[1], A.bias[2]}, J[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int s = 0; s < A.nsheets; s++) sheet_field(A.sheet[s], p[0], p[1], p[2], B, J);
        const double m0 = A.alpha * B[0], m1 = A.alpha * B[1], m2 = A.alpha * B[2];
        // F_j = sum_i m_i dB_i/dx_j, J symmetric
        double f0 = m0 * J[0] + m1 * J[2] + m2 * J[3];
        double f1 = m0 * J[2] + m1 * J[1] + m2 * J[4];
        double f2 = m0 * J[3] + m1 * J[4] + m2 * (-J[0] - J[1]);
        if (A.walls) f2 += rep_force(A, p[2] - 0.5 - A.a) - rep_force(A, A.ztop - p[2] - A.a);
        A.m[k] = m0;
        A.m[n + k] = m1;
        A.m[2 * n + k] = m2;
        A.fs[k] = f0;
        A.fs[n + k] = f1;
        A.fs[2 * n + k] = f2;
    }
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton-Raphson
// steps y <- y (3 - x y^2)/2, each of which squares the relative error
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - (0.5 * x * y) * y);
    y = y * (1.5 - (0.5 * x * y) * y);
    return y;
}

// repulsion magnitude over |r| for g < cut; an integer power n + 1 is taken
// by repeated products (within a few roundings of pow), any other by pow
template <bool kIntPow>
__device__ __forceinline__ double rep_over_r(const MagArgs &A, double g, double rn) {
    if (!kIntPow) return rep_force(A, g) / rn;
    const double ig = 1.0 / (g < A.rep_dmin ? A.rep_dmin : g);
    double p = ig;
    for (int e = 1; e < A.rep_pow; e++) p *= ig;
    return A.rep_n * A.rep_a * p / rn;
}

// All pairs: block (bx, q) takes targets [bx*256, +256) against the sources
// of slice q, staged through LDS a tile of 256 at a time as three 16-byte
// records per bead (every lane reads the same record: broadcast).  Writes
// the slice's force on each target.  kPer is the mask of periodic axes
// (bit d = axis d).  The minimum image rounds r/L to nearest by a product
// with 1/L, which can differ from d - L floor(d/L + 1/2) only at
// separations of half a period.  A lane's own bead gets |r|^2 = 1e300,
// whose force underflows to exactly zero.
template <bool kIntPow, int kPer>
__global__ __launch_bounds__(kPairThreads) void k_mag_pairs(MagArgs A) {
    __shared__ double2 sa[kPairThreads], sb[kPairThreads], sc[kPairThreads];  // (x0,x1) (x2,m0) (m1,m2)
    const int n = A.n, t = threadIdx.x;
    const int k = blockIdx.x * kPairThreads + t;
    const bool valid = k < n;
    const int kk = valid ? k : 0;
    const double xk0 = A.x[kk], xk1 = A.x[n + kk], xk2 = A.x[2 * n + kk];
    const double mk0 = A.m[kk], mk1 = A.m[n + kk], mk2 = A.m[2 * n + kk];
    const int l0 = blockIdx.y * A.slice_len;
    const int l1 = min(n, l0 + A.slice_len);
    const double twoa = 2.0 * A.a, c0 = 3.0 / (4.0 * kPi);
    const double L0 = A.L[0], L1 = A.L[1], L2 = A.L[2];
    const double i0 = 1.0 / L0, i1 = 1.0 / L1, i2 = 1.0 / L2;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int base = l0; base < l1; base += kPairThreads) {
        const int l = base + t;
        if (l < l1) {
            sa[t] = make_double2(A.x[l], A.x[n + l]);
            sb[t] = make_double2(A.x[2 * n + l], A.m[l]);
            sc[t] = make_double2(A.m[n + l], A.m[2 * n + l]);
        }
        __syncthreads();
        const int cnt = min(kPairThreads, l1 - base);
        const int self = k - base;  // this lane's own index in the tile, if there
        for (int j = 0; j < cnt; j++) {
            const double2 pa = sa[j], pb = sb[j], pc = sc[j];
            double r0 = xk0 - pa.x, r1 = xk1 - pa.y, r2 = xk2 - pb.x;
            if (kPer & 1) r0 -= L0 * rint(r0 * i0);
            if (kPer & 2) r1 -= L1 * rint(r1 * i1);
            if (kPer & 4) r2 -= L2 * rint(r2 * i2);
            const double ml0 = pb.y, ml1 = pc.x, ml2 = pc.y;
            double rr = r0 * r0 + r1 * r1 + r2 * r2;
            rr = j == self ? 1e300 : rr;
            const double ir = rsqrt_nr(rr), ir2 = ir * ir;
            const double c = c0 * ir2 * ir2 * ir;
            const double m1r = ml0 * r0 + ml1 * r1 + ml2 * r2;  // source moment . r
            const double m2r = mk0 * r0 + mk1 * r1 + mk2 * r2;  // target moment . r
            const double mm = ml0 * mk0 + ml1 * mk1 + ml2 * mk2;
            const double q = mm - 5.0 * m1r * m2r * ir2;
            a0 += c * (m1r * mk0 + m2r * ml0 + q * r0);
            a1 += c * (m1r * mk1 + m2r * ml1 + q * r1);
            a2 += c * (m1r * mk2 + m2r * ml2 + q * r2);
            const double rn = rr * ir;
            const double g = rn - twoa;
            if (g < A.rep_cut) {
                const double fr = rep_over_r<kIntPow>(A, g, rn);
                a0 += fr * r0;
                a1 += fr * r1;
                a2 += fr * r2;
            }
        }
        __syncthreads();
    }
    if (valid) {
        double *P = A.part + (int64_t)blockIdx.y * 3 * n;
        P[k] = a0;
        P[n + k] = a1;
        P[2 * n + k] = a2;
    }
}

// Fixing the beads: one thread per (bead, node of a cube of side 2h+1
// around it).  The decision |d|^2 <= a^2 is taken in FP64 exactly as
// written (d by minimum image, no fused multiply-add), so it is the same
// wherever it is evaluated in that form.
struct FreezeArgs {
    const double *x;
    int n;
    int h, side;  // cube half-width and side
    int dims[3];
    int per[3];
    double a2;
    uint8_t *solid;
};

__global__ void k_mag_freeze(FreezeArgs A) {
#pragma clang fp contract(off)
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cube = (int64_t)A.side * A.side * A.side;
    if (gid >= cube * A.n) return;
    const int k = (int)(gid / cube);
    int rem = (int)(gid - (int64_t)k * cube);
    const int o[3] = {rem % A.side - A.h, (rem / A.side) % A.side - A.h, rem / (A.side * A.side) - A.h};
    double r2 = 0.0;
    int64_t idx = 0, stride = 1;
    for (int d = 0; d < 3; d++) {
        const double xb = A.x[(int64_t)d * A.n + k];
        const double fc = floor(xb) + o[d];
        const int L = A.dims[d];
        // node coordinate, wrapped into [0, L) along a periodic axis; any
        // other value (outside the lattice, or from a non-finite bead) is
        // no node
        const double cw = A.per[d] ? fc - (double)L * floor(fc / (double)L) : fc;
        if (!(cw >= 0.0 && cw <= (double)(L - 1))) return;
        double dd = cw - xb;
        if (A.per[d]) dd = dd - (double)L * floor(dd / (double)L + 0.5);
        r2 = r2 + dd * dd;
        idx += (int64_t)cw * stride;
        stride *= L;
    }
    if (r2 <= A.a2) A.solid[idx] = 1;
}

}  // namespace mag

// Kernels of the magnetic bead stage (Sec. 2.5): sheet field in closed
// form, induced moments and gradient force, all-pairs dipole interaction and
// repulsion, the overdamped update, and fixing the beads into the solid mask.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mag {

constexpr int kMaxSheets = 8;
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
    int nslice;        // bead blocks of the pair kernel (its partial sums per bead)
    double *x;         // [3][n]
    double *m;         // [3][n]
    double *fs;        // [3][n] gradient + wall force
    double *part;      // [nslice][3][n]: part[r][.][k] = force on bead k from the beads of block r
    double *fout;      // [3][n] total force (M_TOTAL)
};

// ln(Y + R) with R = sqrt(X^2 + Y^2 + w^2), without cancellation for Y < 0
__device__ __forceinline__ double log_yr(double Y, double R, double q) {
    return Y >= 0.0 ? log(Y + R) : log(q / (R - Y));  // q = X^2 + w^2 = (R + Y)(R - Y)
}
// 1/(Y + R), likewise
__device__ __forceinline__ double inv_yr(double Y, double R, double q) { return Y >= 0.0 ? 1.0 / (Y + R) : (R - Y) / q; }

// Field of one charged rectangle at p and its gradient (upper triangle
// xx, yy, xy, xz, yz; zz = -xx - yy): the Coulomb kernel integrated over
// the rectangle has, at each corner (X, Y) relative to p (w = pz - zs,
// R = |(X, Y, w)|), the antiderivatives ln(Y + R), ln(X + R) and
// atan(XY/(wR)), combined with signs (+ - - +).  sheet_corner adds one
// corner's terms (scaled by sigma/(4 pi)) into B and J.
__device__ __forceinline__ void sheet_corner(const double *S, int c, double px, double py, double pz, double B[3],
                                             double J[5]) {
    const double w = pz - S[0], w2 = w * w;
    const int i = c & 1, j = c >> 1;
    const double k = ((i == j) ? 1.0 : -1.0) * S[5] / (4.0 * kPi);
    const double X = (i ? S[2] : S[1]) - px, Y = (j ? S[4] : S[3]) - py;
    const double qx = X * X + w2, qy = Y * Y + w2;  // qx pairs with Y, qy with X
    const double R = sqrt(qx + Y * Y), iR = 1.0 / R;
    const double iy = inv_yr(Y, R, qx), ix = inv_yr(X, R, qy);
    B[0] += k * log_yr(Y, R, qx);
    B[1] += k * log_yr(X, R, qy);
    B[2] += k * atan(X * Y / (w * R));
    J[0] -= k * X * iR * iy;
    J[1] -= k * Y * iR * ix;
    J[2] -= k * iR;
    J[3] += k * w * iR * iy;
    J[4] += k * w * iR * ix;
}

__device__ __forceinline__ void sheet_field(const double *S, double px, double py, double pz, double B[3],
                                            double J[5]) {
    for (int c = 0; c < 4; c++) sheet_corner(S, c, px, py, pz, B, J);
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

constexpr int kLanesPerBead = 8;  // lanes sharing one bead's sheet corners in k_mag_self

// Eight consecutive lanes per bead (a group inside one wave).  M_APPLY /
// M_TOTAL: total force f = the pair partials of all blocks + fs; M_TOTAL
// writes it to fout, M_APPLY moves the bead by mob f.  M_MOMENTS: field and
// gradient at the (moved) position -- the lanes split the sheets' corners
// and add their terms with a butterfly over the group -- then the moment
// and the gradient + wall force.
__global__ __launch_bounds__(256) void k_mag_self(MagArgs A, int mode) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = gid / kLanesPerBead, sub = gid % kLanesPerBead;
    if (k >= A.n) return;  // whole groups leave together
    const int n = A.n;
    double p[3] = {A.x[k], A.x[n + k], A.x[2 * n + k]};
    if (mode & (M_APPLY | M_TOTAL)) {
        // the partial sums of the blocks, split over the group's lanes and
        // added with a butterfly (every lane ends with the total)
        double f[3] = {0.0, 0.0, 0.0};
        for (int q = sub; q < A.nslice; q += kLanesPerBead)
            for (int d = 0; d < 3; d++) f[d] += A.part[((int64_t)q * 3 + d) * n + k];
        for (int off = kLanesPerBead / 2; off > 0; off >>= 1)
            for (int d = 0; d < 3; d++) f[d] += __shfl_xor(f[d], off, kLanesPerBead);
        for (int d = 0; d < 3; d++) f[d] += A.fs[d * n + k];
        if ((mode & M_TOTAL) && sub == 0)
            for (int d = 0; d < 3; d++) A.fout[d * n + k] = f[d];
        if (mode & M_APPLY)
            for (int d = 0; d < 3; d++) {
                p[d] += A.mob * f[d];
                if (sub == 0) A.x[d * n + k] = p[d];
            }
    }
    if (mode & M_MOMENTS) {
        double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // B (3), J xx yy xy xz yz
        for (int c = sub; c < 4 * A.nsheets; c += kLanesPerBead) {
            double B[3] = {0.0, 0.0, 0.0}, J[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            sheet_corner(A.sheet[c >> 2], c & 3, p[0], p[1], p[2], B, J);
            for (int i = 0; i < 3; i++) acc[i] += B[i];
            for (int i = 0; i < 5; i++) acc[3 + i] += J[i];
        }
        for (int off = kLanesPerBead / 2; off > 0; off >>= 1)
            for (int i = 0; i < 8; i++) acc[i] += __shfl_xor(acc[i], off, kLanesPerBead);
        if (sub != 0) return;
        const double B0 = A.bias[0] + acc[0], B1 = A.bias[1] + acc[1], B2 = A.bias[2] + acc[2];
        const double *J = acc + 3;
        const double m0 = A.alpha * B0, m1 = A.alpha * B1, m2 = A.alpha * B2;
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

// Rotate a value one lane along the whole 64-lane wave (DPP wave_ror:1).
__device__ __forceinline__ int ror1(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x13C, 0xF, 0xF, false); }
__device__ __forceinline__ double ror1(double v) {
    return __hiloint2double(ror1(__double2hiint(v)), ror1(__double2loint(v)));
}

// Force on a bead at xk with moment mk from one at xl with moment ml
// (Eq. interaction plus the repulsion), r = xk - xl by minimum image; `off`
// replaces |r|^2 by 1e300, whose force underflows to exactly zero (the
// bead itself, or a lane without a bead).
template <bool kIntPow, int kPer>
__device__ __forceinline__ void pair_force(const MagArgs &A, const double iL[3], double xk0, double xk1, double xk2,
                                           double mk0, double mk1, double mk2, double xl0, double xl1, double xl2,
                                           double ml0, double ml1, double ml2, bool off, double &f0, double &f1,
                                           double &f2) {
    const double c0 = 3.0 / (4.0 * kPi);
    double r0 = xk0 - xl0, r1 = xk1 - xl1, r2 = xk2 - xl2;
    if (kPer & 1) r0 -= A.L[0] * rint(r0 * iL[0]);
    if (kPer & 2) r1 -= A.L[1] * rint(r1 * iL[1]);
    if (kPer & 4) r2 -= A.L[2] * rint(r2 * iL[2]);
    double rr = r0 * r0 + r1 * r1 + r2 * r2;
    rr = off ? 1e300 : rr;
    const double ir = rsqrt_nr(rr), ir2 = ir * ir;
    const double c = c0 * ir2 * ir2 * ir;
    const double m1r = ml0 * r0 + ml1 * r1 + ml2 * r2;  // source moment . r
    const double m2r = mk0 * r0 + mk1 * r1 + mk2 * r2;  // target moment . r
    const double mm = ml0 * mk0 + ml1 * mk1 + ml2 * mk2;
    const double q = mm - 5.0 * m1r * m2r * ir2;
    f0 = c * (m1r * mk0 + m2r * ml0 + q * r0);
    f1 = c * (m1r * mk1 + m2r * ml1 + q * r1);
    f2 = c * (m1r * mk2 + m2r * ml2 + q * r2);
    const double rn = rr * ir;
    const double g = rn - 2.0 * A.a;
    if (g < A.rep_cut) {
        const double fr = rep_over_r<kIntPow>(A, g, rn);
        f0 += fr * r0;
        f1 += fr * r1;
        f2 += fr * r2;
    }
}

// All pairs, each unordered pair once (the interaction is antisymmetric:
// the force on bead 1 from bead 2 is minus the force on 2 from 1).  The
// beads form blocks of 64 kW (kW waves per workgroup); workgroup p takes the
// block pair (I, J), I <= J, of the p-th upper-triangle entry.  I < J: wave
// w holds 64 beads of I (one per lane) and, in phase s, the 64 beads of J's
// part (w + s) mod kW, one per lane; 64 rotations of the J beads along the
// wave (DPP) meet every I bead with every J bead once, the J beads carrying
// the sums of their reactions along; after the phase these are added into
// LDS (the waves take different parts in a phase, so each part gets its kW
// adds in a fixed order).  I = J: every bead of the block sums all others
// (broadcast from LDS).  Results: part[J][.][k] for k in I, part[I][.][l]
// for l in J, each slot written by exactly one workgroup.  kPer is the mask
// of periodic axes; the minimum image rounds r/L to nearest by a product
// with 1/L, which can differ from d - L floor(d/L + 1/2) only at
// separations of half a period.
template <bool kIntPow, int kPer, int kW>
__global__ __launch_bounds__(64 * kW) void k_mag_pairs(MagArgs A) {
    constexpr int kB = 64 * kW;  // beads per block
    __shared__ double2 sa[kB], sb[kB], sc[kB];  // (x0,x1) (x2,m0) (m1,m2)
    __shared__ double sacc[3][kB];
    const int n = A.n, t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int64_t NB = A.nslice;
    // block pair of this workgroup: row I has NB - I entries, starting at I NB - I (I - 1)/2
    const int64_t p = blockIdx.x;
    const double a2 = 2.0 * NB + 1.0;
    int64_t I = (int64_t)floor((a2 - sqrt(a2 * a2 - 8.0 * (double)p)) * 0.5);
    auto row0 = [NB](int64_t r) { return r * NB - r * (r - 1) / 2; };
    while (I > 0 && row0(I) > p) I--;
    while (I + 1 < NB && row0(I + 1) <= p) I++;
    const int64_t J = I + (p - row0(I));
    const double iL[3] = {1.0 / A.L[0], 1.0 / A.L[1], 1.0 / A.L[2]};

    const int k = (int)(I * kB) + t;
    const bool kval = k < n;
    const int kk = kval ? k : n - 1;
    const double xk0 = A.x[kk], xk1 = A.x[n + kk], xk2 = A.x[2 * n + kk];
    const double mk0 = A.m[kk], mk1 = A.m[n + kk], mk2 = A.m[2 * n + kk];
    double a0 = 0.0, a1 = 0.0, a2s = 0.0;

    if (I == J) {
        if (kval) {
            sa[t] = make_double2(xk0, xk1);
            sb[t] = make_double2(xk2, mk0);
            sc[t] = make_double2(mk1, mk2);
        }
        __syncthreads();
        const int cnt = min(kB, n - (int)(I * kB));
        for (int j = 0; j < cnt; j++) {
            const double2 pa = sa[j], pb = sb[j], pc = sc[j];
            double f0, f1, f2;
            pair_force<kIntPow, kPer>(A, iL, xk0, xk1, xk2, mk0, mk1, mk2, pa.x, pa.y, pb.x, pb.y, pc.x, pc.y,
                                      j == t, f0, f1, f2);
            a0 += f0;
            a1 += f1;
            a2s += f2;
        }
        if (kval) {
            double *P = A.part + I * 3 * n;
            P[k] = a0;
            P[n + k] = a1;
            P[2 * n + k] = a2s;
        }
        return;
    }

    for (int d = 0; d < 3; d++) sacc[d][t] = 0.0;
    __syncthreads();
    for (int s = 0; s < kW; s++) {
        const int q = (w + s) % kW;
        const int l = (int)(J * kB) + q * 64 + lane;
        const bool lval = l < n;
        const int ll = lval ? l : n - 1;
        double xl0 = A.x[ll], xl1 = A.x[n + ll], xl2 = A.x[2 * n + ll];
        double ml0 = A.m[ll], ml1 = A.m[n + ll], ml2 = A.m[2 * n + ll];
        int lv = lval ? 1 : 0;
        double b0 = 0.0, b1 = 0.0, b2 = 0.0;  // reaction sums carried with the J bead
        for (int step = 0; step < 64; step++) {
            double f0, f1, f2;
            pair_force<kIntPow, kPer>(A, iL, xk0, xk1, xk2, mk0, mk1, mk2, xl0, xl1, xl2, ml0, ml1, ml2,
                                      !(kval && lv), f0, f1, f2);
            a0 += f0;
            a1 += f1;
            a2s += f2;
            b0 -= f0;
            b1 -= f1;
            b2 -= f2;
            xl0 = ror1(xl0);
            xl1 = ror1(xl1);
            xl2 = ror1(xl2);
            ml0 = ror1(ml0);
            ml1 = ror1(ml1);
            ml2 = ror1(ml2);
            b0 = ror1(b0);
            b1 = ror1(b1);
            b2 = ror1(b2);
            lv = ror1(lv);
        }
        // 64 rotations: every J bead is back in its own lane
        sacc[0][q * 64 + lane] += b0;
        sacc[1][q * 64 + lane] += b1;
        sacc[2][q * 64 + lane] += b2;
        __syncthreads();
    }
    if (kval) {
        double *P = A.part + J * 3 * n;
        P[k] = a0;
        P[n + k] = a1;
        P[2 * n + k] = a2s;
    }
    const int l = (int)(J * kB) + t;
    if (l < n) {
        double *P = A.part + I * 3 * n;
        P[l] = sacc[0][t];
        P[n + l] = sacc[1][t];
        P[2 * n + l] = sacc[2][t];
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

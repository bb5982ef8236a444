// C-ABI of the magnetic bead stage (Sec. 2.5): argument checks, the
// work-buffer layout and kernel dispatch.  Shares the error slot of the
// lattice library (lbm_last_error).
#include "magnet.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "lbmibm.h"
#include "magnet_kernels.hpp"

namespace lbm {
void set_error(const char *msg);  // defined with the lattice library's C-ABI
}

namespace {

using namespace mag;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    lbm::set_error(buf);
    return code;
}

#define MAGCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool finite_all(const double *v, int k) {
    for (int i = 0; i < k; i++)
        if (!std::isfinite(v[i])) return false;
    return true;
}

bool aligned8(const void *q) { return ((uintptr_t)q & 7) == 0; }

int check_params(const mag_params *p) {
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->n < 1 || p->n > MAG_MAX_BEADS) return fail(LBM_EINVAL, "n must be in [1, %d] (got %d)", MAG_MAX_BEADS, p->n);
    if (p->nsheets < 0 || p->nsheets > MAG_MAX_SHEETS)
        return fail(LBM_EINVAL, "nsheets must be in [0, %d] (got %d)", MAG_MAX_SHEETS, p->nsheets);
    for (int s = 0; s < p->nsheets; s++) {
        const double *S = p->sheets[s];
        if (!finite_all(S, 6)) return fail(LBM_EINVAL, "sheet %d has a non-finite value", s);
        if (!(S[1] < S[2]) || !(S[3] < S[4])) return fail(LBM_EINVAL, "sheet %d needs x0 < x1 and y0 < y1", s);
    }
    if (!finite_all(p->bias, 3)) return fail(LBM_EINVAL, "bias is not finite");
    if (!(p->a > 0) || !std::isfinite(p->a)) return fail(LBM_EINVAL, "a must be finite and > 0");
    if (!(p->chi >= 0) || !std::isfinite(p->chi)) return fail(LBM_EINVAL, "chi must be finite and >= 0");
    if (!(p->eta > 0) || !std::isfinite(p->eta)) return fail(LBM_EINVAL, "eta must be finite and > 0");
    if (!(p->dt > 0) || !std::isfinite(p->dt)) return fail(LBM_EINVAL, "dt must be finite and > 0");
    if (!(p->rep_a >= 0) || !std::isfinite(p->rep_a)) return fail(LBM_EINVAL, "rep_a must be finite and >= 0");
    if (!(p->rep_n > 0) || !std::isfinite(p->rep_n)) return fail(LBM_EINVAL, "rep_n must be finite and > 0");
    if (!(p->rep_cut > 0) || !std::isfinite(p->rep_cut)) return fail(LBM_EINVAL, "rep_cut must be finite and > 0");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBM_EINVAL, "nx, ny, nz must be >= 1");
    if ((int64_t)p->nx * p->ny * p->nz > (int64_t)INT32_MAX) return fail(LBM_EINVAL, "lattice too large");
    for (int d = 0; d < 3; d++)
        if (p->periodic[d] != 0 && p->periodic[d] != 1) return fail(LBM_EINVAL, "periodic[%d] must be 0 or 1", d);
    if (p->walls_z != 0 && p->walls_z != 1) return fail(LBM_EINVAL, "walls_z must be 0 or 1");
    return LBM_OK;
}

// Waves per workgroup of the pair kernel (blocks of 64 of them beads): the
// largest of 4, 2, 1 that still gives about 2048 workgroups (block pairs),
// so that small bead counts fill the chip too.  Its partial sums hold one
// [3][n] array per block.
int pair_waves(int n) {
    for (int w : {4, 2}) {
        const int64_t nb = cdiv(n, 64 * w);
        if (nb * (nb + 1) / 2 >= 2048) return w;
    }
    return 1;
}
int blocks(int n) { return (int)cdiv(n, 64 * pair_waves(n)); }

int64_t work_bytes(int n) {
    const int64_t plane = cdiv((int64_t)3 * n * 8, 256) * 256;  // one [3][n] double array, 256-aligned
    return plane * (2 + blocks(n));
}

void fill_common(const mag_params *p, double sheet[kMaxSheets][6], double bias[3], int *nsheets) {
    std::memset(sheet, 0, sizeof(double) * kMaxSheets * 6);
    std::memcpy(sheet, p->sheets, sizeof(double) * 6 * p->nsheets);
    for (int d = 0; d < 3; d++) bias[d] = p->bias[d];
    *nsheets = p->nsheets;
}

MagArgs make_args(const mag_params *p, double *x, void *work) {
    MagArgs A;
    std::memset(&A, 0, sizeof A);
    fill_common(p, A.sheet, A.bias, &A.nsheets);
    A.alpha = 4.0 * kPi * p->a * p->a * p->a * p->chi / (p->chi + 3.0);
    A.mob = p->dt / (6.0 * kPi * p->eta * p->a);
    A.a = p->a;
    A.rep_a = p->rep_a;
    A.rep_n = p->rep_n;
    A.rep_cut = p->rep_cut;
    A.rep_dmin = p->rep_cut / 100.0;
    const double e = p->rep_n + 1.0;
    A.rep_pow = (e == std::floor(e) && e >= 1.0 && e <= 16.0) ? (int)e : 0;
    A.L[0] = p->nx;
    A.L[1] = p->ny;
    A.L[2] = p->nz;
    A.ztop = p->nz - 1.5;
    for (int d = 0; d < 3; d++) A.per[d] = p->periodic[d];
    A.walls = p->walls_z;
    A.n = p->n;
    A.nslice = blocks(p->n);
    const int64_t plane = cdiv((int64_t)3 * p->n * 8, 256) * 256;
    char *w = (char *)work;
    A.x = x;
    A.m = (double *)w;
    A.fs = (double *)(w + plane);
    A.part = (double *)(w + 2 * plane);
    A.fout = nullptr;
    return A;
}

int launch_self(const MagArgs &A, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_mag_self, dim3((unsigned)cdiv((int64_t)A.n * kLanesPerBead, 256)), dim3(256), 0, s, A, mode);
    MAGCHK(hipGetLastError());
    return LBM_OK;
}

int launch_pairs(const MagArgs &A, hipStream_t s) {
    const int64_t nb = A.nslice;
    const int waves = pair_waves(A.n);
    const dim3 grid((unsigned)(nb * (nb + 1) / 2)), block(64 * waves);
    const int per = A.per[0] | (A.per[1] << 1) | (A.per[2] << 2);
#define MAG_PAIRS_W(P, W)                                                                        \
    if (waves == W) {                                                                            \
        if (A.rep_pow)                                                                           \
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mag_pairs<true, P, W>), grid, block, 0, s, A);  \
        else                                                                                     \
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mag_pairs<false, P, W>), grid, block, 0, s, A); \
    }
#define MAG_PAIRS(P)        \
    case P:                 \
        MAG_PAIRS_W(P, 1)   \
        MAG_PAIRS_W(P, 2)   \
        MAG_PAIRS_W(P, 4)   \
        break;
    switch (per) {
        MAG_PAIRS(0)
        MAG_PAIRS(1)
        MAG_PAIRS(2)
        MAG_PAIRS(3)
        MAG_PAIRS(4)
        MAG_PAIRS(5)
        MAG_PAIRS(6)
        MAG_PAIRS(7)
    }
#undef MAG_PAIRS_W
#undef MAG_PAIRS
    MAGCHK(hipGetLastError());
    return LBM_OK;
}

int check_work(const mag_params *p, const void *work) {
    if (!work) return fail(LBM_EINVAL, "work is NULL");
    if (((uintptr_t)work & 255) != 0) return fail(LBM_EINVAL, "work must be 256-byte aligned");
    return LBM_OK;
}

// step t: forces at x_t (moments, pairs), then x_(t+1) = x_t + mob F;
// the move of step t is fused with the moments of step t + 1
int run_steps(const mag_params *p, double *x, int32_t nsteps, void *work) {
    const hipStream_t s = (hipStream_t)p->stream;
    const MagArgs A = make_args(p, x, work);
    if (int rc = launch_self(A, M_MOMENTS, s)) return rc;
    for (int t = 0; t < nsteps; t++) {
        if (int rc = launch_pairs(A, s)) return rc;
        if (int rc = launch_self(A, t + 1 < nsteps ? (M_APPLY | M_MOMENTS) : M_APPLY, s)) return rc;
    }
    return LBM_OK;
}

// Work memory of mag_run_static: one array per GPU, in the code object's
// device globals, reserved when the library is loaded on that GPU and held
// until the process ends.  Host code reaches it only through the address
// hipGetSymbolAddress gives for the current device (static_work); the
// array's name is a host-side stand-in, not a device address.
constexpr int64_t kStaticWorkBytes = int64_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWorkBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};

// Device address of the current device's array (looked up once per device).
int static_work(void **out) {
    int dev = -1;
    MAGCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EINVAL, "device %d is beyond the %d this library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        MAGCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr & 255) != 0) return fail(LBM_EHIP, "the static work array has no usable device address");
        g_static_ptr[dev] = ptr;
    }
    *out = g_static_ptr[dev];
    return LBM_OK;
}

}  // namespace

#define MAG_API extern "C" __attribute__((visibility("default")))

MAG_API int64_t mag_workspace_bytes(const mag_params *p) {
    if (check_params(p) != LBM_OK) return 0;
    return work_bytes(p->n);
}

MAG_API int mag_field(const mag_params *p, const double *pts, int32_t npts, double *B, double *J) {
    // only the field description of p is used: n may be anything here
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    mag_params q = *p;
    q.n = 1;
    if (int rc = check_params(&q)) return rc;
    if (npts < 0) return fail(LBM_EINVAL, "npts must be >= 0");
    if (npts == 0) return LBM_OK;
    if (!pts || !B) return fail(LBM_EINVAL, "pts and B must be non-NULL");
    if (!aligned8(pts) || !aligned8(B) || (J && !aligned8(J))) return fail(LBM_EINVAL, "arrays must be 8-byte aligned");
    FieldArgs A;
    std::memset(&A, 0, sizeof A);
    fill_common(p, A.sheet, A.bias, &A.nsheets);
    A.npts = npts;
    A.p = pts;
    A.B = B;
    A.J = J;
    hipLaunchKernelGGL(k_mag_field, dim3((unsigned)cdiv(npts, 256)), dim3(256), 0, (hipStream_t)p->stream, A);
    MAGCHK(hipGetLastError());
    return LBM_OK;
}

MAG_API int mag_forces(const mag_params *p, const double *x, double *m, double *F, void *work) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_work(p, work)) return rc;
    if (!x || !m || !F) return fail(LBM_EINVAL, "x, m and F must be non-NULL");
    if (!aligned8(x) || !aligned8(m) || !aligned8(F)) return fail(LBM_EINVAL, "arrays must be 8-byte aligned");
    const hipStream_t s = (hipStream_t)p->stream;
    MagArgs A = make_args(p, const_cast<double *>(x), work);  // x is only read without M_APPLY
    A.fout = F;
    if (int rc = launch_self(A, M_MOMENTS, s)) return rc;
    if (int rc = launch_pairs(A, s)) return rc;
    if (int rc = launch_self(A, M_TOTAL, s)) return rc;
    MAGCHK(hipMemcpyAsync(m, A.m, sizeof(double) * 3 * p->n, hipMemcpyDeviceToDevice, s));
    return LBM_OK;
}

MAG_API int mag_run(const mag_params *p, double *x, int32_t nsteps, void *work) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_work(p, work)) return rc;
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (!x || !aligned8(x)) return fail(LBM_EINVAL, "x must be non-NULL and 8-byte aligned");
    if (nsteps == 0) return LBM_OK;
    return run_steps(p, x, nsteps, work);
}

MAG_API int mag_run_static(const mag_params *p, double *x, int32_t nsteps) {
    if (int rc = check_params(p)) return rc;
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (!x || !aligned8(x)) return fail(LBM_EINVAL, "x must be non-NULL and 8-byte aligned");
    const int64_t need = work_bytes(p->n);
    if (need > kStaticWorkBytes)
        return fail(LBM_EINVAL, "%d beads need %lld bytes of work, more than the %lld of mag_run_static; use mag_run",
                    p->n, (long long)need, (long long)kStaticWorkBytes);
    void *work = nullptr;
    if (int rc = static_work(&work)) return rc;
    if (nsteps == 0) return LBM_OK;
    return run_steps(p, x, nsteps, work);
}

MAG_API int mag_freeze(const mag_params *p, const double *x, uint8_t *solid) {
    if (int rc = check_params(p)) return rc;
    if (!x || !solid) return fail(LBM_EINVAL, "x and solid must be non-NULL");
    if (!aligned8(x)) return fail(LBM_EINVAL, "x must be 8-byte aligned");
    FreezeArgs A;
    A.x = x;
    A.n = p->n;
    A.h = (int)std::floor(p->a) + 2;
    A.side = 2 * A.h + 1;
    if ((int64_t)A.side * A.side * A.side > (int64_t)1 << 24) return fail(LBM_EINVAL, "bead radius too large to fix");
    A.dims[0] = p->nx;
    A.dims[1] = p->ny;
    A.dims[2] = p->nz;
    for (int d = 0; d < 3; d++) A.per[d] = p->periodic[d];
    A.a2 = p->a * p->a;
    A.solid = solid;
    const int64_t total = (int64_t)A.side * A.side * A.side * p->n;
    const int64_t blocks = cdiv(total, 256);
    if (blocks > INT32_MAX) return fail(LBM_EINVAL, "too many beads for this radius");
    hipLaunchKernelGGL(k_mag_freeze, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)p->stream, A);
    MAGCHK(hipGetLastError());
    return LBM_OK;
}

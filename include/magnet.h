/*
 * magnet.h -- C ABI of the magnetic bead stage of the gfx950 library
 * (liblbmibm.so; the same error codes and lbm_last_error() as lbmibm.h).
 *
 * The stage (paper: Gusenbauer et al., Sec. 2.5, Eqs. (Fstart) and
 * (interaction), and the staged run that follows it): soft-magnetic beads in
 * the field of magnetic charge sheets and a homogeneous bias field move under
 * the gradient force, their mutual dipole forces, friction and collisions,
 * and form chains; the chains are then fixed in space and become solid
 * obstacles of the lattice-Boltzmann run.
 *
 * Where the paper leaves the form open (it defers to a companion paper), the
 * library implements, in units with mu0 = 1 (so B = H outside the magnets):
 *   - sheet field: a sheet is a rectangle [x0,x1] x [y0,y1] in the plane
 *     z = zs carrying uniform magnetic surface charge sigma; its field is
 *     sigma/(4 pi) times the integral of the Coulomb kernel (p - r')/|p - r'|^3
 *     over the rectangle, evaluated in closed form (log and arctangent sums
 *     over the four corners), with the gradient dB_i/dx_j likewise; the bias
 *     field is added.  A point must not lie in the plane of a sheet.
 *   - induced moment: m = 4 pi a^3 chi/(chi + 3) B(x) (a sphere of radius a
 *     and susceptibility chi in a uniform field; the beads' own fields are
 *     not fed back into the moments);
 *   - gradient force F_g = grad(m . B) at fixed m (Eq. Fstart):
 *     F_g,j = sum_i m_i dB_i/dx_j;
 *   - dipole interaction (Eq. interaction) on bead 2 from bead 1,
 *     r = x2 - x1: 3/(4 pi |r|^5) [(m1.r) m2 + (m2.r) m1 + (m1.m2) r -
 *     5 (m1.r)(m2.r) r/|r|^2], summed over all other beads (minimum image
 *     along periodic axes);
 *   - collisions: a soft-sphere repulsion n A g^-(n+1) along the line of
 *     centres for surface distance g = |r| - 2a in (0, cut), evaluated at
 *     max(g, cut/100) below cut/100; with walls_z, the same law pushes a bead
 *     off the walls z = 1/2 and z = nz - 3/2 (g = z - 1/2 - a, resp.
 *     nz - 3/2 - z - a);
 *   - friction: overdamped motion against Stokes drag,
 *     x <- x + dt F / (6 pi eta a), all forces taken at the step's start.
 *   - fixing the chains: lattice node (i, j, k) becomes solid when its
 *     centre lies within a of a bead centre (minimum image along periodic
 *     axes); node index i + nx (j + ny k) as in lbmibm.h.
 *
 * Conventions: bead arrays are device memory, [3][n] doubles (component
 * planes).  The caller owns every buffer; `work` is device memory of at
 * least mag_workspace_bytes(p) bytes, 256-byte aligned, owned by the caller
 * and used only while a call's work runs on p->stream.  Calls enqueue on
 * p->stream and return without waiting.  Errors: LBM_OK or a negative code
 * (LBM_EINVAL for a bad argument, LBM_EHIP for a runtime or launch error);
 * argument checks run on the host before anything is enqueued.
 */
#ifndef MAGNET_H
#define MAGNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MAG_MAX_SHEETS 8
#define MAG_MAX_BEADS (1 << 17)

typedef struct {
    int32_t n;                           /* beads, 1 .. MAG_MAX_BEADS */
    int32_t nsheets;                     /* 0 .. MAG_MAX_SHEETS */
    double sheets[MAG_MAX_SHEETS][6];    /* (zs, x0, x1, y0, y1, sigma), x0 < x1, y0 < y1 */
    double bias[3];                      /* homogeneous bias field */
    double a;                            /* bead radius, > 0 */
    double chi;                          /* susceptibility, >= 0 */
    double eta;                          /* fluid viscosity, > 0 */
    double dt;                           /* time step, > 0 */
    double rep_a, rep_n, rep_cut;        /* repulsion strength >= 0, exponent > 0, range > 0 */
    int32_t nx, ny, nz;                  /* lattice size (periodic lengths, walls, fixing), each >= 1 */
    int32_t periodic[3];                 /* 1 = periodic axis (minimum image), else 0 */
    int32_t walls_z;                     /* 1 = repulsive walls at z = 1/2 and nz - 3/2 */
    void *stream;                        /* hipStream_t (NULL = null stream) */
} mag_params;

/* Bytes of device workspace mag_forces and mag_run need for p->n beads:
 * moments, one-bead forces and the pair forces from each block of b beads,
 * (2 + ceil(n/b)) arrays of 3n doubles, each rounded up to 256 bytes; b is
 * the largest of 256, 128, 64 for which the ceil(n/b) blocks form at least
 * 2048 block pairs (counting a block with itself), else 64 (1.6 GB at the
 * largest n); 0 if p is invalid (lbm_last_error() says why). */
int64_t mag_workspace_bytes(const mag_params *p);

/* Field of the sheets plus the bias (Sec. 2.5 set-up) at npts points:
 * pts [3][npts] in, B [3][npts] out, and, if J is not NULL, the gradient
 * J [9][npts], J[3 i + j] = dB_i/dx_j (symmetric, traceless).  npts >= 0. */
int mag_field(const mag_params *p, const double *pts, int32_t npts, double *B, double *J);

/* Moments m [3][n] and total forces F [3][n] (gradient + dipole
 * interaction + bead and wall repulsion) on beads at x [3][n]
 * (Eqs. Fstart and interaction). */
int mag_forces(const mag_params *p, const double *x, double *m, double *F, void *work);

/* nsteps >= 0 overdamped steps of the beads, x [3][n] advanced in place. */
int mag_run(const mag_params *p, double *x, int32_t nsteps, void *work);

/* mag_run without the work argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc): the same kernels, on the same inputs, give the
 * same results, with their work in an array of 32 MiB that the library
 * holds on each GPU it runs on (reserved when the library is loaded there,
 * kept until the process ends).  The call allocates nothing.  The work of p
 * (mag_workspace_bytes) must fit in 32 MiB -- every n up to 13184 does, and
 * so does 16384 -- else LBM_EINVAL, before anything is enqueued.  Runs on
 * the current device, whose stream p->stream must be.  Every call on one
 * GPU shares its array: calls that overlap there (on two streams, or from
 * two host threads) race and give wrong results; one call's contents
 * survive into the next, and no part of the array needs to start at zero. */
int mag_run_static(const mag_params *p, double *x, int32_t nsteps);

/* Fix the chains: OR the bead spheres into solid [nx*ny*nz] (uint8, 1 =
 * solid); x [3][n].  Nodes are only set, never cleared. */
int mag_freeze(const mag_params *p, const double *x, uint8_t *solid);

#ifdef __cplusplus
}
#endif

#endif

/*
 * lbmibm.h -- C ABI of the MI355X (gfx950) D3Q19 lattice-Boltzmann +
 * immersed-boundary cell-flow library.
 *
 * The method (paper: Gusenbauer et al., "A tunable cancer cell filter using
 * magnetic beads: cellular and fluid dynamic simulations"):
 *   - Sec. 2.1, LBM equation: one BGK collide-and-stream step of the D3Q19
 *     populations f_i with an external force term F_i;
 *   - Sec. 2.2, the four immersed-boundary steps: lattice velocity is
 *     interpolated to the membrane (IB) points, forces are computed at the
 *     points, spread back to the lattice with a discrete delta, and fluid
 *     and points are advanced;
 *   - Sec. 2.3, the membrane forces from the moduli K^S, K^B, K^A_l, K^A_g,
 *     K^V of Table 1 (the global terms need the whole cell, Sec. 2.3.3);
 *   - Sec. 2.4, halfway bounce-back at solid nodes.
 * Where the paper leaves the form open, the library implements: second-order
 * polynomial equilibrium, Guo's forcing with u = (j + F/2)/rho, trilinear
 * delta, frictional coupling F_c = xi A_k (u(X_k) - V_k) with friction and
 * point mass taken per unit membrane area (A_k = rest area of vertex k),
 * linear-spring/area/volume/angle energies, and the step order interpolate
 * -> forces -> spread -> collide/stream -> move points.
 *
 * Conventions
 *   - Lattice node n = x + nx*(y + ny*z), N = nx*ny*nz, x fastest.  A
 *     context made by lbm_init_channels holds several independent lattices
 *     ("channels") back to back: channel k owns nodes [noff_k, noff_k + N_k)
 *     with noff_k = N_0 + ... + N_(k-1), N = the sum of all N_k, and every
 *     per-node array below uses that concatenated index.
 *   - Populations: 19 planes, plane i at element offset i*plane_stride.
 *     D3Q19 order: 0 rest; 1,2 = +-x; 3,4 = +-y; 5,6 = +-z; 7,8 = (1,1,0),
 *     (-1,-1,0); 9,10 = (1,-1,0),(-1,1,0); 11,12 = (1,0,1),(-1,0,-1);
 *     13,14 = (1,0,-1),(-1,0,1); 15,16 = (0,1,1),(0,-1,-1);
 *     17,18 = (0,1,-1),(0,-1,1).  Odd i and i+1 are opposite.
 *     Population i of a fluid node n lies in slot (i, n), except when the
 *     neighbour n - c_i is a solid node: then the population (the one n
 *     sent towards that neighbour in the step before, returned by halfway
 *     bounce-back) lies in slot (opp(i), n - c_i) of the solid node, where
 *     the streaming put it.  Solid nodes hold no populations of their own
 *     (their other slots carry rest values).  lbm_store_f64 / lbm_load_f64
 *     convert to and from plain per-node populations.
 *   - Precision LBM_F64: double populations and arithmetic.  LBM_F32: float
 *     f_i.  LBM_F32_DEV: float deviations h_i = f_i - w_i from the rest
 *     weights, float arithmetic.  Global mass/momentum sums are double in
 *     every mode.  "real" below means double for LBM_F64, float otherwise.
 *   - Vector fields are [3][N] (component planes), point arrays [3][nverts].
 *   - Ownership: the caller allocates every buffer passed in (device
 *     memory unless stated) and keeps it alive until lbm_destroy; the
 *     library only borrows them.  The context owns its own work buffers
 *     (node classes, immersed-boundary spread force and fallback
 *     accumulator, reduction partials, collide-stream workgroup table),
 *     allocated in lbm_init and freed in lbm_destroy.
 *   - Streams: every call enqueues on params.stream and returns without
 *     waiting, except lbm_read_fields with a non-NULL host_sums,
 *     ibm_rest_shape (reads the mesh topology back to check it) and
 *     lbm_init/lbm_destroy.
 *   - Errors: functions return LBM_OK (0) or a negative code; nothing is
 *     thrown across the ABI.  lbm_last_error() gives the message of the last
 *     failure on the calling thread.  Argument checks run on the host before
 *     any device work is enqueued, so a rejected call changes nothing.
 *   - One context must not be used from two host threads at once.
 */
#ifndef LBMIBM_H
#define LBMIBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)     /* bad argument (sizes, tau <= 1/2, null/misaligned pointer, bad mesh) */
#define LBM_ENOMEM (-2)     /* device allocation failed */
#define LBM_EHIP (-3)       /* HIP runtime or launch error */
#define LBM_ENONFINITE (-4) /* a global sum, or a node's populations, came out NaN or Inf */
#define LBM_ESTATE (-5)     /* call out of order (e.g. ibm_couple before ibm_rest_shape) */

#define LBM_F64 0
#define LBM_F32 1
#define LBM_F32_DEV 2

typedef struct lbm_ctx lbm_ctx;

/* Lattice description for lbm_init (Sec. 2.1, 2.4). */
typedef struct {
    int32_t nx, ny, nz;      /* lattice size, each >= 1 */
    int32_t periodic[3];     /* 1 = periodic axis; a link leaving a non-periodic axis bounces back */
    double tau;              /* BGK relaxation time, > 1/2 (viscosity (tau - 1/2)/3) */
    double body_force[3];    /* uniform force density g (lattice units) */
    int32_t prec;            /* LBM_F64, LBM_F32 or LBM_F32_DEV */
    int64_t plane_stride;    /* elements between population planes: 0 = lbm_plane_stride(), else >= N and a multiple of 64 */
    const uint8_t *solid;    /* [N] uint8, 1 = solid node, 0 = fluid */
    void *f_a;               /* [19*plane_stride] populations (storage type of prec); state buffer A */
    void *f_b;               /* same size; state buffer B */
    const void *gfield;      /* [3][N] real external forcing field G added to g, or NULL */
    void *stream;            /* hipStream_t to enqueue on (NULL = null stream) */
} lbm_params;

/* Contact forces between cells and with the walls (Sec. 2.4, collisions: a
 * soft-sphere potential between IB points of different cells and between
 * IB points and the walls, cut at an interaction range).  The law is a
 * reading: U(d) = a d^-n for d = r - roff in (0, rcut), 0 beyond, continued
 * linearly below dmin (force magnitude n a max(d, dmin)^-(n+1)); r is the
 * distance between two points (minimum image across periodic axes) or from a
 * point to a wall surface on the fluid side (planes, z-axis cylinders and
 * fixed spheres).  Cell-cell forces are added to the membrane force of the
 * step (m->f_el then holds elastic + contact); the wall forces act in the
 * point update of the same step. */
typedef struct {
    double a, n;            /* strength and exponent, > 0 */
    double rcut;            /* interaction range beyond roff, > 0 */
    double roff;            /* offset, >= 0 */
    double dmin;            /* 0 < dmin <= rcut */
    int32_t cell_cell;      /* 1: IB points of different cells of one channel repel each other */
    int32_t nplanes;        /* wall planes */
    const double *planes;   /* device [nplanes][4]: unit normal into the fluid, offset (surface n.x = offset) */
    int32_t ncyl;           /* z-axis cylinders (posts) */
    const double *cyl;      /* device [ncyl][3]: xc, yc, radius R; fluid outside */
    const int32_t *cyl_off; /* device [nch+1]: channel k's cylinders are [cyl_off[k], cyl_off[k+1]); NULL: all in every channel */
    int32_t nspheres;       /* fixed spheres (Sec. 2.5: the beads of the chains fixed in space), 0 .. 2^22;
                               only in a one-channel context */
    const double *spheres;  /* device [nspheres][4]: xc, yc, zc, R > 0; fluid outside.  Read by ibm_rest_shape,
                               which sorts them into a uniform grid of cells no smaller than R_max + roff + rcut;
                               after changing them call ibm_rest_shape again */
} ibm_contact;

/* Membrane population (Sec. 2.2, 2.3).  All pointers are device memory.
 * Topology arrays use global vertex ids; each cell's triangles and edges may
 * only reference that cell's vertices [vert_off[c], vert_off[c+1]). */
typedef struct {
    int32_t ncells, nverts, ntris, nedges;
    const int32_t *vert_off; /* [ncells+1] first vertex of each cell */
    const int32_t *tri_off;  /* [ncells+1] first triangle of each cell */
    const int32_t *edge_off; /* [ncells+1] first edge of each cell */
    const int32_t *tri;      /* [3][ntris] vertices (a,b,c), counter-clockwise seen from outside */
    const int32_t *hinge;    /* [4][nedges] (p1,p2,qa,qb): triangles (p1,p2,qa) and (p2,p1,qb) share edge p1-p2 */
    const int32_t *anchor;   /* [3][ncells] integer anchor of each cell */
    const int32_t *cell_chan;/* [ncells] channel holding each cell (see lbm_init_channels); NULL = channel 0,
                                allowed only when the context has one channel */
    double *x;               /* [3][nverts] position minus the cell's anchor, FP64 in every precision (updated by ibm_couple) */
    void *v;                 /* [3][nverts] real: velocity (updated by ibm_couple) */
    void *f_el;              /* [3][nverts] real: written with the elastic force of the last ibm_couple */
    const void *moduli;      /* [5][ncells] real: k_s, k_b, k_al, k_ag, k_v per cell (Table 1 order K^S, K^B, K^A_l, K^A_g, K^V) */
    double *l0;              /* [nedges] rest edge lengths           (written by ibm_rest_shape) */
    double *a0;              /* [ntris]  rest triangle areas         (written by ibm_rest_shape) */
    double *th0;             /* [nedges] rest hinge angles           (written by ibm_rest_shape) */
    double *a0c;             /* [ncells] rest cell areas             (written by ibm_rest_shape) */
    double *v0c;             /* [ncells] rest cell volumes           (written by ibm_rest_shape) */
    double *avert;           /* [nverts] rest area carried by each vertex, a third of its triangles' (written by ibm_rest_shape) */
    int32_t *vtri_off;       /* [nverts+1] incident-triangle list offsets     (written by ibm_rest_shape) */
    int32_t *vtri;           /* [3*ntris]  triangle*4 + corner, per vertex    (written by ibm_rest_shape) */
    int32_t *vedge_off;      /* [nverts+1] incident-edge list offsets         (written by ibm_rest_shape) */
    int32_t *vedge;          /* [4*nedges] edge*4 + role (p1,p2,qa,qb)        (written by ibm_rest_shape) */
    double xi;               /* coupling friction per unit membrane area: vertex k feels F_c = xi*avert[k]*(u(X_k) - V_k); > 0 */
    double mass;             /* membrane mass per unit area: vertex k has mass mass*avert[k] (Newton equation of Sec. 2.2); > 0 */
    double dt;               /* IB time step, > 0 */
    const ibm_contact *contact; /* host struct (its arrays on the device) of contact forces, or NULL for none;
                                   ibm_rest_shape sizes the pair list for it, so it must not change afterwards */
    int32_t stretch_law;     /* edge stretching (Sec. 2.3.1): 0 = linear springs (k_s/2)(l - l0)^2/l0;
                                1 = neo-Hookean (k_s/6) l0 (lam^2 + 2/lam - 3), lam = l/l0 (same small-strain limit) */
    /* filled by ibm_rest_shape; the caller must not edit them */
    int32_t max_cell_verts, max_cell_tris, max_cell_edges;
    uint32_t checked;
} ibm_mesh;

/* Suggested population plane stride (elements) for an N-node lattice:
 * N rounded up to 64 plus a pad that keeps the 19 plane starts off a common
 * large power-of-two alignment. */
int64_t lbm_plane_stride(int64_t n_nodes, int32_t prec);

/* Bytes lbm_init allocates on the device for this lattice (the first
 * ibm_rest_shape adds 4*N bytes of spreading claims, plus one spread record
 * per IB point). */
int64_t lbm_workspace_bytes(const lbm_params *p);

/* Validate p, create a context and set both state buffers to the fluid at
 * rest (f_i = w_i; h_i = 0 in LBM_F32_DEV).  The LBM equation of Sec. 2.1
 * starts from this state.  On failure *out is NULL. */
int lbm_init(const lbm_params *p, lbm_ctx **out);

/* Batched form: one context over nch >= 1 independent channels, dims
 * (host memory) = [nch][3] sizes (nx, ny, nz) of each, stepped together by
 * every call below, one launch per kernel for the whole batch.  Each
 * channel is its own lattice of Sec. 2.1/2.4 (its own periodic wrap, no
 * link between channels); p->nx, ny, nz are ignored; periodic, tau,
 * body_force and prec apply to all channels; solid, f_a, f_b, gfield and
 * plane_stride refer to the concatenated node index.  A channel alone and
 * the same channel inside a batch give bitwise equal results. */
int lbm_init_channels(const lbm_params *p, int32_t nch, const int32_t *dims, lbm_ctx **out);

/* lbm_workspace_bytes for lbm_init_channels (-1 on invalid arguments). */
int64_t lbm_workspace_bytes_channels(const lbm_params *p, int32_t nch, const int32_t *dims);

/* Launch shape, results unchanged: collide_waves_per_block = 64-node tiles
 * per collide-stream workgroup (1, 2, 4 or 8; 0 = by the channels: each
 * workgroup takes whole x rows of one channel, as many as fit in 8 tiles,
 * or a piece of 8 tiles of a longer row), list_blocks = workgroups of the
 * kernels that walk the list of tiles under a membrane stencil (0 = by
 * lattice size, at most 65536).  Drops a captured graph. */
int lbm_set_launch(lbm_ctx *c, int32_t collide_waves_per_block, int32_t list_blocks);

/* Schedule of a coupled step's immersed-boundary kernels, results unchanged
 * (bitwise): with overlap, the membrane forces (Sec. 2.3) run on a second
 * stream owned by the context while the velocities at the stencil nodes
 * (Sec. 2.2 step 1) are evaluated on p->stream, and both are joined into
 * p->stream before the point update; without it they run in order.  Either
 * way every call's work is on p->stream when it returns.  mode = 1: always,
 * 0: never, -1 (the default): when the mesh has at least
 * LBM_OVERLAP_MIN_POINTS IB points (below that the join costs more than the
 * overlap saves).  The adjoint's recomputed steps never overlap.  Drops a
 * captured graph; LBM_EINVAL for another mode. */
#define LBM_OVERLAP_MIN_POINTS 16384
int lbm_set_ibm_overlap(lbm_ctx *c, int32_t mode);

/* Where a coupled step takes the fluid velocity at the stencil nodes from
 * (Sec. 2.2 step 1; results unchanged, bitwise).  mode = 1: every
 * ibm_couple marks the stencils of the points' new positions, and the next
 * collide-stream pass (lbm_step) copies the populations it streams into
 * those nodes into a record, from which the next ibm_couple reads them; a
 * stencil node the record lacks (for instance after the caller moved the
 * points) sends that step through the lattice gather.  mode = 0 (the
 * default): always the gather.  The records need every channel's nx to be a multiple of 64
 * (otherwise the gather is always used); they take 19 reals and 4 bytes per
 * slot, min(N, 8 x the IB points of the meshes given to ibm_rest_shape)
 * slots, allocated by ibm_rest_shape.  Drops a captured graph; LBM_EINVAL
 * for another mode. */
int lbm_set_node_records(lbm_ctx *c, int32_t mode);

/* How the last ibm_couple on c found the stencil velocities: *used = 1 if it
 * read the records of the pass before it, *missed = 1 if a stencil node
 * was not among them (that step then gathered from the lattice).  Valid
 * until the next lbm_step; waits on the stream.  Either pointer may be
 * NULL. */
int lbm_node_records_used(lbm_ctx *c, int32_t *used, int32_t *missed);

/* nsteps >= 0 coupled steps: for each, ibm_couple(c, m) (skipped when m is
 * NULL) then lbm_step(c, 1).  With steps_per_graph > 0 (even, at most
 * 4096) the steps are taken in groups of steps_per_graph, captured once into
 * a HIP graph and replayed with one graph launch per group on
 * params.stream; the remainder runs as ordinary launches.  The graph is
 * captured again when the mesh (its buffers, xi, mass or dt), the group
 * length, the launch shape or the parity of the state buffer changes.
 * Graph and ordinary launches run the same kernels on the same data, so
 * the results are bitwise those of the eager loop.  When a mesh was
 * coupled (ibm_couple) before the call, its spread force is still pending:
 * the first step then runs as ordinary launches, adding m's force to it as
 * the eager loop does, and the graph groups follow.
 *
 * Failure detection: every collide-stream pass flags, on the device, a node
 * whose populations are not all finite; the flag stays set until
 * lbm_load_f64.  lbm_run ends by queueing a copy of it to the host, and a
 * later lbm_run or lbm_step call that finds the copy landed and set returns
 * LBM_ENONFINITE without doing anything.  Nothing waits for that copy, so the
 * report comes one or more calls after the pass that met the values; call
 * lbm_check_finite to wait for it. */
int lbm_run(lbm_ctx *c, const ibm_mesh *m, int32_t nsteps, int32_t steps_per_graph);

/* Wait for the stream, then *nonfinite (host, may be NULL) = 1 if a
 * collide-stream pass since the context was made (or since the last
 * lbm_load_f64) met non-finite populations, else 0; returns LBM_ENONFINITE
 * in the first case.  The state is then lost: reload it (lbm_load_f64) or
 * destroy the context. */
int lbm_check_finite(lbm_ctx *c, int32_t *nonfinite);

/* Advance the lattice nsteps >= 0 times: fused BGK collision with Guo
 * forcing (force = g + G + the immersed-boundary force spread by the last
 * ibm_couple, which this call consumes and clears), then streaming with
 * halfway bounce-back (Sec. 2.1 LBM equation, Sec. 2.4).  With cells present
 * call ibm_couple before each single step.  Returns LBM_ENONFINITE, without
 * stepping, once an earlier pass is known to have met non-finite
 * populations (see lbm_run). */
int lbm_step(lbm_ctx *c, int32_t nsteps);

/* lbm_step(c, 1) (the same step: Sec. 2.1 LBM equation, Sec. 2.4) whose
 * collide-stream kernel is launched with two HIP events (hipEvent_t, created
 * by the caller with timing enabled and not recorded on another stream
 * meanwhile): the runtime sets them to that
 * kernel's own start and end, so hipEventElapsedTime(start, stop) is the
 * kernel's duration, without the dispatch gaps that events recorded around
 * the call include.  For measurement; not for graph capture.  LBM_EINVAL if
 * either event is NULL. */
int lbm_step_timed(lbm_ctx *c, void *start_event, void *stop_event);

/* Compute the rest shape (edge lengths, triangle areas, hinge angles, cell
 * area and volume, vertex areas; all in FP64) of the mesh at its current
 * positions into m->l0, a0, th0, a0c, v0c, avert, and the per-vertex
 * incidence lists into m->vtri_off, vtri, vedge_off, vedge, after checking the topology (read back to the host; this
 * call waits on the stream).  Must be called once per mesh before
 * ibm_couple; fills the trailing fields of *m. */
int ibm_rest_shape(lbm_ctx *c, ibm_mesh *m);

/* The immersed-boundary part of one step (Sec. 2.2 steps 1-3 and the point
 * half of step 4): per cell, area/volume then elastic forces (written to
 * m->f_el); per point, interpolated velocity u_k from the current
 * populations, F_c = xi A_k (u_k - V), spreading of -F_c to the 8
 * surrounding nodes for the next lbm_step, then V += dt/m_k (F_el + F_c),
 * X += dt V.  Lengths, areas, angles, cell area and volume are evaluated in
 * FP64 from the stored positions in every precision, so their small
 * departures from the rest shape are not lost to rounding.  Several meshes
 * may be coupled before one lbm_step: their spread forces add up (the
 * next lbm_step consumes the sum). */
int ibm_couple(lbm_ctx *c, const ibm_mesh *m);

/* rho [N] and u [3][N] (real, device, either may be NULL) of the current
 * state: u = (j + (g + G)/2)/rho on fluid nodes, 0 on solid nodes (rho 0).
 * host_sums (host memory, may be NULL): double [4] = sum over fluid nodes of
 * rho, j_x, j_y, j_z; when given, the call waits and returns
 * LBM_ENONFINITE if any sum is not finite. */
int lbm_read_fields(lbm_ctx *c, void *rho, void *u, double *host_sums);

/* Device pointer of the state buffer that holds the current populations
 * (f_a or f_b) and the number of steps taken so far. */
int lbm_current(lbm_ctx *c, void **f_cur, int64_t *steps);

/* Copy the current state to / from full FP64 populations f_i ([19][N]
 * double, device, plain per-node layout) -- adds / subtracts w_i in
 * LBM_F32_DEV.  Solid nodes read as their rest weights w_i and are ignored
 * when loading. */
int lbm_store_f64(lbm_ctx *c, double *f64);
int lbm_load_f64(lbm_ctx *c, const double *f64);

/* Membrane force and its directional derivative (Sec. 2.3 energies,
 * Sec. 2.3.3 global terms), in FP64 at any positions: f_out = F_el(x)
 * (may be NULL) and jvp_out = (dF_el/dx) w, with x and w device [3][nverts]
 * doubles (x as offsets from the anchors, like m->x).  F_el = -grad E, so
 * the Jacobian is minus the energy Hessian and is symmetric: jvp_out is
 * also the transposed product the adjoint needs.  Exact to rounding
 * (forward-mode dual numbers through the energy gradient).  The mesh must
 * have had ibm_rest_shape. */
int ibm_force_jvp(lbm_ctx *c, const ibm_mesh *m, const double *x, const double *w, double *f_out, double *jvp_out);

/* One reverse step of the coupled map: the adjoint (transposed derivative)
 * of the step (f_n, X_n, V_n; G) -> (f_{n+1}, X_{n+1}, V_{n+1}) that
 * ibm_couple + lbm_step(c, 1) take (Sec. 2.1 LBM equation with forcing, the
 * four immersed-boundary steps of Sec. 2.2, the membrane forces of Sec.
 * 2.3, bounce-back of Sec. 2.4), for the differentiation of an objective J
 * of a run with respect to its inputs.
 *   f_n       [19*plane_stride] storage type: the populations at step n
 *             (the layout of f_a / f_b); read only.
 *   x_n, v_n  [3][nverts] FP64 offsets and real velocities at step n.
 *   lam_next  [19*plane_stride] real: dJ/df_{n+1}; read only.
 *   lam       [19*plane_stride] real, written with dJ/df_n (0 at solid nodes);
 *             must not alias lam_next or f_n.
 *   lam_x, lam_v  [3][nverts] FP64: on entry dJ/dX_{n+1}, dJ/dV_{n+1}; on
 *             exit dJ/dX_n, dJ/dV_n (updated in place).
 *   dgrad     [3][N] real or NULL: dJ/dG of this step is ADDED (G = the
 *             forcing field of lbm_params, whether or not one was given).
 * m may be NULL for a run without cells (then the point arguments are
 * ignored).  The call recomputes the immersed-boundary half of step n from
 * (f_n, x_n, v_n) in its own scratch (the context's lattice state and the
 * mesh's x, v, f_el are not touched) and then runs the reverse kernels.
 * Arithmetic is in the context's real type; the points' adjoints are FP64.
 * The order of the float additions that spread lambda_u to the lattice is
 * not fixed, so repeated calls may differ in the last bits. */
int lbm_adjoint_step(lbm_ctx *c, const ibm_mesh *m, const void *f_n, const double *x_n, const void *v_n,
                     const void *lam_next, void *lam, double *lam_x, double *lam_v, void *dgrad);

/* nsteps coupled steps (as lbm_run) that also record the state at the start
 * of every step, for a later reverse sweep: f_rec [nsteps][19*plane_stride]
 * storage type (16-byte aligned), x_rec [nsteps][3][nverts] FP64 offsets,
 * v_rec [nsteps][3][nverts] real (ignored when m is NULL).  Step k reads its
 * populations from record k and writes record k+1 (the last step writes the
 * context's current state buffer, so lbm_current does not change), so
 * recording costs one copy of the state per call, not per step.  use_graph != 0 captures the
 * whole call into a HIP graph (reused while the arguments, the mesh and the
 * state-buffer parity are the same) and replays it. */
int lbm_run_record(lbm_ctx *c, const ibm_mesh *m, int32_t nsteps, void *f_rec, double *x_rec, void *v_rec,
                   int32_t use_graph);

/* Reverse sweep over steps recorded by lbm_run_record: lbm_adjoint_step for
 * k = nsteps-1 down to 0.  lam_a [19*plane_stride] real holds dJ/df at the
 * end of the recorded steps on entry and dJ/df at their start on exit; lam_b
 * is scratch of the same size; lam_x, lam_v (FP64 [3][nverts]) are updated
 * in place; dJ/dG of every step is added to dgrad ([3][N] real, or NULL).
 * use_graph as for lbm_run_record. */
int lbm_adjoint_run(lbm_ctx *c, const ibm_mesh *m, int32_t nsteps, const void *f_rec, const double *x_rec,
                    const void *v_rec, void *lam_a, void *lam_b, double *lam_x, double *lam_v, void *dgrad,
                    int32_t use_graph);

/* Free the context's own buffers (waits for its stream). NULL is a no-op. */
void lbm_destroy(lbm_ctx *c);

/* Message of the last failed call on this thread ("" if none). */
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBMIBM_H */

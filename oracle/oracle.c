/*
 * FP64 CPU oracle for the D3Q19 BGK + immersed-boundary cell-flow step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or helper with the GPU library (which has its own D3Q19
 * table, kernels and host code); the two meet only in the seeded input
 * arrays.
 *
 * What it computes, step n -> n+1 (one call of orc_step), following the
 * paper's four-step immersed-boundary procedure (Sec. 2.2) around the
 * forced LBM update (Sec. 2.1, eq. for f_i):
 *   1. rho = sum_i f_i, j = sum_i f_i c_i on fluid nodes; F_ext = g + G(x);
 *      u_ext = (j + F_ext/2)/rho (fluid), 0 on solid nodes.
 *   2. IB points: u_k = sum over the 2x2x2 stencil of W(x - X_k) u_ext(x)
 *      (trilinear discrete delta, periodic wrap)        [Sec. 2.2 step 1]
 *   3. per cell: total area A_c and enclosed volume V_c, then the elastic
 *      force F_el = -grad(E_s + E_b + E_al + E_ag + E_v)  [Sec. 2.3.1, 2.3.3]
 *      and the coupling force F_c = xi A_k (u_k - V_k)    [Sec. 2.2 step 2]
 *   4. F(x) = F_ext(x) + sum_k W(x - X_k) (-F_c,k)         [Sec. 2.2 step 3]
 *   5. BGK collision with the Guo source on fluid nodes, u = (j + F/2)/rho,
 *      then streaming to x + c_i, or halfway bounce-back into the opposite
 *      slot when x + c_i is a solid node                   [Sec. 2.1, 2.4]
 *   6. V_k += dt/m_k (F_el + F_c), X_k += dt V_k            [Sec. 2.2 step 4]
 *      (with contact forces enabled, F_el also carries the soft-sphere
 *      repulsion between cells and from the walls, Sec. 2.4)
 *      Reading: friction xi and point mass are densities per unit membrane
 *      area, so vertex k, carrying the rest area A_k (a third of its
 *      triangles' areas), has friction xi A_k and mass m_k = mass A_k.
 * The points where the paper is silent (form of f_eq, of the source term, of
 * the delta function, of the membrane energies, the ordering above) are the
 * readings listed in the design notes; each is marked "reading" below.
 *
 * Layouts: lattice node n = x + nx*(y + ny*z); populations f[i*N + n];
 * vector fields v[d*N + n]; IB points X[k*3 + d] (absolute, unwrapped).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19
#define PI_ 3.14159265358979323846

/* D3Q19 velocities: rest, 6 faces, 12 edges; the opposite of odd i is i+1. */
static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

static double weight(int i) {
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static int opposite(int i) {
    if (i == 0) return 0;
    return (i % 2 == 1) ? i + 1 : i - 1;
}

typedef struct {
    int nx, ny, nz;
    int periodic[3];
    double tau;
    double g[3];
    const uint8_t *solid; /* [N], 1 = solid */
    const double *G;      /* [3][N] external forcing field, or NULL */
} orc_lattice;

/* Contact forces (Sec. 2.4, collisions): a soft-sphere potential between IB
 * points of different cells and between IB points and the walls, cut at an
 * interaction range.  Reading: U(d) = a d^-n for d = r - roff in (0, rcut),
 * zero beyond; below dmin the potential continues linearly with the slope
 * it has at dmin (a finite force for overlapping points).  Walls are
 * analytic surfaces: planes n.x = offset (unit normal n into the fluid),
 * z-axis cylinders of radius R and fixed spheres of radius R (the beads of
 * the frozen chains; fluid outside both); r is then the distance to the
 * surface on the fluid side (minimum image across periodic axes). */
typedef struct {
    double a, n, rcut, roff, dmin;
    int cell_cell;          /* 1: points of different cells repel each other */
    int nplanes;
    const double *planes;   /* [nplanes][4] = (nx, ny, nz, offset) */
    int ncyl;
    const double *cyl;      /* [ncyl][3] = (xc, yc, R) */
    int nsph;
    const double *sph;      /* [nsph][4] = (xc, yc, zc, R): fixed spheres (the beads of frozen chains), fluid outside */
} orc_contact;

typedef struct {
    int ncells, nverts, ntris, nedges;
    const int *vert_off; /* [ncells+1] */
    const int *tri_off;  /* [ncells+1] */
    const int *edge_off; /* [ncells+1] */
    const int *tri;      /* [ntris][3], outward counter-clockwise */
    const int *hinge;    /* [nedges][4] = (p1, p2, qa, qb) */
    const double *moduli;/* [ncells][5] = (k_s, k_b, k_al, k_ag, k_v) */
    double xi, mass, dt; /* friction and mass per unit membrane area, time step */
    int stretch_law;     /* 0: linear springs, 1: neo-Hookean springs (see membrane_energy) */
    /* rest shape, filled by orc_rest_shape */
    double *l0;  /* [nedges] */
    double *A0;  /* [ntris]  */
    double *th0; /* [nedges] */
    double *A0c; /* [ncells] */
    double *V0c; /* [ncells] */
    double *Av;  /* [nverts] rest area carried by each vertex */
    const orc_contact *contact; /* contact forces, or NULL */
} orc_mesh;

/* Threads the OpenMP loops below will use. */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* tables (exported so the tests can check the lattice identities)          */
/* ------------------------------------------------------------------------ */

void orc_d3q19(int *c /* [19][3] */, double *w /* [19] */, int *opp /* [19] */) {
    for (int i = 0; i < Q; i++) {
        c[3 * i + 0] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}

/* ------------------------------------------------------------------------ */
/* local collision pieces (Sec. 2.1)                                         */
/* ------------------------------------------------------------------------ */

/* Reading: the second-order polynomial equilibrium of D3Q19,
 * f_eq_i = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u). */
void orc_equilibrium(double rho, const double u[3], double feq[Q]) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; i++) {
        double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        feq[i] = weight(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Reading: the forcing term F_i of the LBM equation is Guo's source,
 * F_i = (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F,
 * used together with the half-force velocity u = (j + F/2)/rho. */
void orc_forcing(double tau, const double u[3], const double F[3], double S[Q]) {
    for (int i = 0; i < Q; i++) {
        double c[3] = {CX[i], CY[i], CZ[i]};
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        double s = 0.0;
        for (int d = 0; d < 3; d++) s += (3.0 * (c[d] - u[d]) + 9.0 * cu * c[d]) * F[d];
        S[i] = (1.0 - 0.5 / tau) * weight(i) * s;
    }
}

/* One BGK relaxation with source, for a single node. */
void orc_collide_node(double tau, const double f[Q], const double F[3], double fout[Q]) {
    double rho = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; i++) {
        rho += f[i];
        j[0] += f[i] * CX[i];
        j[1] += f[i] * CY[i];
        j[2] += f[i] * CZ[i];
    }
    double u[3];
    for (int d = 0; d < 3; d++) u[d] = (j[d] + 0.5 * F[d]) / rho;
    double feq[Q], S[Q];
    orc_equilibrium(rho, u, feq);
    orc_forcing(tau, u, F, S);
    for (int i = 0; i < Q; i++) fout[i] = f[i] - (f[i] - feq[i]) / tau + S[i];
}

/* ------------------------------------------------------------------------ */
/* lattice helpers                                                           */
/* ------------------------------------------------------------------------ */

static long nnodes(const orc_lattice *L) { return (long)L->nx * L->ny * L->nz; }

static int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* Neighbour of (x,y,z) along c_i; -1 if it leaves a non-periodic axis. */
static long neighbour(const orc_lattice *L, int x, int y, int z, int i) {
    int p[3] = {x + CX[i], y + CY[i], z + CZ[i]};
    int n[3] = {L->nx, L->ny, L->nz};
    for (int d = 0; d < 3; d++) {
        if (p[d] < 0 || p[d] >= n[d]) {
            if (!L->periodic[d]) return -1;
            p[d] = wrap(p[d], n[d]);
        }
    }
    return p[0] + (long)L->nx * (p[1] + (long)L->ny * p[2]);
}

/* rho and u_ext = (j + F_ext/2)/rho per node; solid nodes get rho = 0, u = 0
 * (reading: the interpolated velocity excludes the not-yet-known IB force). */
void orc_fluid_velocity(const orc_lattice *L, const double *f, double *rho, double *uext) {
    long N = nnodes(L);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
        if (L->solid[n]) {
            if (rho) rho[n] = 0.0;
            for (int d = 0; d < 3; d++) uext[d * N + n] = 0.0;
            continue;
        }
        double r = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < Q; i++) {
            double v = f[i * N + n];
            r += v;
            j[0] += v * CX[i];
            j[1] += v * CY[i];
            j[2] += v * CZ[i];
        }
        for (int d = 0; d < 3; d++) {
            double Fe = L->g[d] + (L->G ? L->G[d * N + n] : 0.0);
            uext[d * N + n] = (j[d] + 0.5 * Fe) / r;
        }
        if (rho) rho[n] = r;
    }
}

/* Compensated (Neumaier) running sum, so that the global sums below do not
 * lose the conservation signal to the rounding of large partial sums. */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double v) {
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}

/* Sum of rho and j over fluid nodes: out = (M, Px, Py, Pz). */
void orc_mass_momentum(const orc_lattice *L, const double *f, double out[4]) {
    long N = nnodes(L);
    ksum acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (long n = 0; n < N; n++) {
        if (L->solid[n]) continue;
        double r = 0, jx = 0, jy = 0, jz = 0;
        for (int i = 0; i < Q; i++) {
            double v = f[i * N + n];
            r += v;
            jx += v * CX[i];
            jy += v * CY[i];
            jz += v * CZ[i];
        }
        kadd(&acc[0], r);
        kadd(&acc[1], jx);
        kadd(&acc[2], jy);
        kadd(&acc[3], jz);
    }
    for (int d = 0; d < 4; d++) out[d] = acc[d].s + acc[d].c;
}

/* Collide every fluid node with total force F[3][N] and stream into fnew.
 * A population heading into a solid node (or out through a non-periodic
 * face) is reflected into the opposite slot of its own node (halfway
 * bounce-back).  Solid-node slots of fnew are left untouched. */
void orc_collide_stream(const orc_lattice *L, const double *f, const double *F, double *fnew) {
    long N = nnodes(L);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < L->nz; z++) {
        for (int y = 0; y < L->ny; y++) {
            for (int x = 0; x < L->nx; x++) {
                long n = x + (long)L->nx * (y + (long)L->ny * z);
                if (L->solid[n]) continue;
                double fl[Q], fo[Q], Fn[3];
                for (int i = 0; i < Q; i++) fl[i] = f[i * N + n];
                for (int d = 0; d < 3; d++) Fn[d] = F[d * N + n];
                orc_collide_node(L->tau, fl, Fn, fo);
                for (int i = 0; i < Q; i++) {
                    long m = neighbour(L, x, y, z, i);
                    if (m < 0 || L->solid[m])
                        fnew[opposite(i) * N + n] = fo[i];
                    else
                        fnew[i * N + m] = fo[i];
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* discrete delta (Sec. 2.2 steps 1 and 3)                                   */
/* ------------------------------------------------------------------------ */

/* Reading: the discrete delta is the trilinear kernel over the 8 nodes
 * around X; node indices wrap periodically on every axis. */
static void stencil(const orc_lattice *L, const double X[3], long idx[8], double w[8]) {
    int i0[3];
    double fr[3];
    int n[3] = {L->nx, L->ny, L->nz};
    for (int d = 0; d < 3; d++) {
        double fl = floor(X[d]);
        i0[d] = (int)fl;
        fr[d] = X[d] - fl;
    }
    int k = 0;
    for (int bz = 0; bz < 2; bz++)
        for (int by = 0; by < 2; by++)
            for (int bx = 0; bx < 2; bx++) {
                int x = wrap(i0[0] + bx, n[0]);
                int y = wrap(i0[1] + by, n[1]);
                int z = wrap(i0[2] + bz, n[2]);
                idx[k] = x + (long)n[0] * (y + (long)n[1] * z);
                w[k] = (bx ? fr[0] : 1.0 - fr[0]) * (by ? fr[1] : 1.0 - fr[1]) * (bz ? fr[2] : 1.0 - fr[2]);
                k++;
            }
}

/* out[k] = sum_x W(x - X_k) field(x) for a vector field [3][N]. */
void orc_interpolate(const orc_lattice *L, const double *field, int nv, const double *X, double *out) {
    long N = nnodes(L);
    for (int k = 0; k < nv; k++) {
        long idx[8];
        double w[8];
        stencil(L, X + 3 * k, idx, w);
        for (int d = 0; d < 3; d++) {
            double s = 0.0;
            for (int c = 0; c < 8; c++) s += w[c] * field[d * N + idx[c]];
            out[3 * k + d] = s;
        }
    }
}

/* field(x) += sum_k W(x - X_k) Fk[k] */
void orc_spread(const orc_lattice *L, int nv, const double *X, const double *Fk, double *field) {
    long N = nnodes(L);
    for (int k = 0; k < nv; k++) {
        long idx[8];
        double w[8];
        stencil(L, X + 3 * k, idx, w);
        for (int c = 0; c < 8; c++)
            for (int d = 0; d < 3; d++) field[d * N + idx[c]] += w[c] * Fk[3 * k + d];
    }
}

/* ------------------------------------------------------------------------ */
/* membrane geometry and elastic forces (Sec. 2.3.1, Table 1)                */
/* ------------------------------------------------------------------------ */

static void sub3(const double *a, const double *b, double *r) {
    r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static void cross3(const double *a, const double *b, double *r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* Triangle area, half the norm of (b-a) x (c-a). */
static double tri_area(const double *a, const double *b, const double *c) {
    double e1[3], e2[3], n[3];
    sub3(b, a, e1);
    sub3(c, a, e2);
    cross3(e1, e2, n);
    return 0.5 * norm3(n);
}

/* Signed volume of the tetrahedron (origin, a, b, c): a.(b x c)/6. */
static double tri_volume(const double *a, const double *b, const double *c) {
    double n[3];
    cross3(b, c, n);
    return dot3(a, n) / 6.0;
}

/* Angle between the outward normals of triangles (p1,p2,qa) and (p2,p1,qb),
 * signed so that a convex fold is positive and a flat hinge is zero. */
static double dihedral(const double *p1, const double *p2, const double *qa, const double *qb) {
    double e[3], t1[3], t2[3], na[3], nb[3], m[3];
    sub3(p2, p1, e);
    sub3(qa, p1, t1);
    cross3(e, t1, na);           /* (p2-p1) x (qa-p1) */
    double me[3] = {-e[0], -e[1], -e[2]};
    sub3(qb, p2, t2);
    cross3(me, t2, nb);          /* (p1-p2) x (qb-p2) */
    cross3(na, nb, m);
    double s = dot3(m, e) / norm3(e);
    double c = dot3(na, nb);
    return atan2(s, c);
}

static const double *vtx(const double *X, int k) { return X + 3 * k; }

/* Per-cell total area and volume (divergence theorem on absolute positions). */
void orc_cell_area_volume(const orc_mesh *M, const double *X, double *A, double *V) {
    for (int c = 0; c < M->ncells; c++) {
        double a = 0.0, v = 0.0;
        for (int t = M->tri_off[c]; t < M->tri_off[c + 1]; t++) {
            const int *T = M->tri + 3 * t;
            a += tri_area(vtx(X, T[0]), vtx(X, T[1]), vtx(X, T[2]));
            v += tri_volume(vtx(X, T[0]), vtx(X, T[1]), vtx(X, T[2]));
        }
        A[c] = a;
        V[c] = v;
    }
}

/* Edge lengths, triangle areas and dihedral angles of the mesh at X. */
void orc_mesh_geometry(const orc_mesh *M, const double *X, double *l, double *A, double *th) {
    for (int e = 0; e < M->nedges; e++) {
        const int *h = M->hinge + 4 * e;
        double d[3];
        sub3(vtx(X, h[1]), vtx(X, h[0]), d);
        if (l) l[e] = norm3(d);
        if (th) th[e] = dihedral(vtx(X, h[0]), vtx(X, h[1]), vtx(X, h[2]), vtx(X, h[3]));
    }
    if (A)
        for (int t = 0; t < M->ntris; t++) {
            const int *T = M->tri + 3 * t;
            A[t] = tri_area(vtx(X, T[0]), vtx(X, T[1]), vtx(X, T[2]));
        }
}

/* Reading: the rest shape is the mesh as given (the initial icosphere), so
 * the elastic forces vanish initially. */
void orc_rest_shape(orc_mesh *M, const double *X) {
    orc_mesh_geometry(M, X, M->l0, M->A0, M->th0);
    orc_cell_area_volume(M, X, M->A0c, M->V0c);
    /* each vertex carries one third of the rest area of its triangles */
    for (int k = 0; k < M->nverts; k++) M->Av[k] = 0.0;
    for (int t = 0; t < M->ntris; t++)
        for (int j = 0; j < 3; j++) M->Av[M->tri[3 * t + j]] += M->A0[t] / 3.0;
}

/* Stretching energy of one edge and -dE/dl.  Reading: linear springs, or
 * (Sec. 2.3.1: nonlinear, neo-Hookean-like) the uniaxial incompressible
 * neo-Hookean energy W(lambda) = lambda^2 + 2/lambda - 3 of the stretch
 * lambda = l/l0, scaled so that both laws agree for small strain:
 * E = (k_s/6) l0 W(lambda) ~ (k_s/2) (l - l0)^2 / l0.                     */
static double stretch_energy(int law, double ks, double l, double l0) {
    if (law == 0) return 0.5 * ks * (l - l0) * (l - l0) / l0;
    double lam = l / l0;
    return ks * l0 / 6.0 * (lam * lam + 2.0 / lam - 3.0);
}
static double stretch_force(int law, double ks, double l, double l0) {
    if (law == 0) return -ks * (l - l0) / l0;
    double lam = l / l0;
    return -ks / 3.0 * (lam - 1.0 / (lam * lam));
}

/* Reading of the four moduli as energies (all values from Table 1):
 *   E_s  = sum_edges (k_s/2) (l - l0)^2 / l0          (linear stretching,
 *          or the neo-Hookean edge energy above)
 *   E_b  = sum_hinges (k_b/2) (theta - theta0)^2      (preferred angle)
 *   E_al = sum_tris (k_al/2) (A - A0)^2 / A0          (local area)
 *   E_ag = (k_ag/2) (A_c - A0_c)^2 / A0_c             (global area)
 *   E_v  = (k_v/2) (V_c - V0_c)^2 / V0_c              (volume)            */
double orc_membrane_energy(const orc_mesh *M, const double *X) {
    double E = 0.0;
    for (int c = 0; c < M->ncells; c++) {
        const double *k = M->moduli + 5 * c;
        double Ac = 0.0, Vc = 0.0;
        for (int t = M->tri_off[c]; t < M->tri_off[c + 1]; t++) {
            const int *T = M->tri + 3 * t;
            double A = tri_area(vtx(X, T[0]), vtx(X, T[1]), vtx(X, T[2]));
            Ac += A;
            Vc += tri_volume(vtx(X, T[0]), vtx(X, T[1]), vtx(X, T[2]));
            E += 0.5 * k[2] * (A - M->A0[t]) * (A - M->A0[t]) / M->A0[t];
        }
        E += 0.5 * k[3] * (Ac - M->A0c[c]) * (Ac - M->A0c[c]) / M->A0c[c];
        E += 0.5 * k[4] * (Vc - M->V0c[c]) * (Vc - M->V0c[c]) / M->V0c[c];
        for (int e = M->edge_off[c]; e < M->edge_off[c + 1]; e++) {
            const int *h = M->hinge + 4 * e;
            double d[3];
            sub3(vtx(X, h[1]), vtx(X, h[0]), d);
            double l = norm3(d);
            E += stretch_energy(M->stretch_law, k[0], l, M->l0[e]);
            double th = dihedral(vtx(X, h[0]), vtx(X, h[1]), vtx(X, h[2]), vtx(X, h[3]));
            E += 0.5 * k[1] * (th - M->th0[e]) * (th - M->th0[e]);
        }
    }
    return E;
}

static void addv(double *F, int k, double s, const double *v) {
    F[3 * k + 0] += s * v[0];
    F[3 * k + 1] += s * v[1];
    F[3 * k + 2] += s * v[2];
}

/* F = -grad E (membrane_energy), written out term by term.
 *   grad_a A   = (b - c) x n_hat / 2 (cyclic in a, b, c)
 *   grad_a V_t = (b x c) / 6        (cyclic)
 *   grad l     = +-(p2 - p1)/l
 *   grad theta: wings qa, qb get -|e| n_a/|n_a|^2, -|e| n_b/|n_b|^2; the edge
 *   ends get the combinations that keep the sum and the torque zero,
 *   grad_p1 = -(1-s_a) g_qa - (1-s_b) g_qb, grad_p2 = -s_a g_qa - s_b g_qb,
 *   with s_q = (q - p1).e/|e|^2.                                           */
void orc_membrane_forces(const orc_mesh *M, const double *X, double *F) {
    memset(F, 0, sizeof(double) * 3 * M->nverts);
    for (int c = 0; c < M->ncells; c++) {
        const double *k = M->moduli + 5 * c;
        /* global constraints first: they need the whole cell (Sec. 2.3.3) */
        double Ac = 0.0, Vc = 0.0;
        for (int t = M->tri_off[c]; t < M->tri_off[c + 1]; t++) {
            const int *T = M->tri + 3 * t;
            Ac += tri_area(vtx(X, T[0]), vtx(X, T[1]), vtx(X, T[2]));
            Vc += tri_volume(vtx(X, T[0]), vtx(X, T[1]), vtx(X, T[2]));
        }
        double cag = k[3] * (Ac - M->A0c[c]) / M->A0c[c];
        double cv = k[4] * (Vc - M->V0c[c]) / M->V0c[c];
        for (int t = M->tri_off[c]; t < M->tri_off[c + 1]; t++) {
            const int *T = M->tri + 3 * t;
            const double *a = vtx(X, T[0]), *b = vtx(X, T[1]), *cc = vtx(X, T[2]);
            double e1[3], e2[3], n[3];
            sub3(b, a, e1);
            sub3(cc, a, e2);
            cross3(e1, e2, n);
            double nn = norm3(n);
            double A = 0.5 * nn;
            double nh[3] = {n[0] / nn, n[1] / nn, n[2] / nn};
            double cal = k[2] * (A - M->A0[t]) / M->A0[t];
            double ca = cal + cag; /* both area terms share grad A_t */
            double d[3], gA[3];
            sub3(b, cc, d); cross3(d, nh, gA); addv(F, T[0], -0.5 * ca, gA);
            sub3(cc, a, d); cross3(d, nh, gA); addv(F, T[1], -0.5 * ca, gA);
            sub3(a, b, d); cross3(d, nh, gA); addv(F, T[2], -0.5 * ca, gA);
            double gV[3];
            cross3(b, cc, gV); addv(F, T[0], -cv / 6.0, gV);
            cross3(cc, a, gV); addv(F, T[1], -cv / 6.0, gV);
            cross3(a, b, gV); addv(F, T[2], -cv / 6.0, gV);
        }
        for (int e = M->edge_off[c]; e < M->edge_off[c + 1]; e++) {
            const int *h = M->hinge + 4 * e;
            const double *p1 = vtx(X, h[0]), *p2 = vtx(X, h[1]), *qa = vtx(X, h[2]), *qb = vtx(X, h[3]);
            /* stretching */
            double ev[3];
            sub3(p2, p1, ev);
            double l = norm3(ev);
            double cs = -stretch_force(M->stretch_law, k[0], l, M->l0[e]); /* dE/dl */
            addv(F, h[0], cs / l, ev);  /* -dE/dp1 = +dE/dl (p2-p1)/l */
            addv(F, h[1], -cs / l, ev);
            /* bending */
            double th = dihedral(p1, p2, qa, qb);
            double cb = k[1] * (th - M->th0[e]);
            double t1[3], t2[3], na[3], nb[3], me[3] = {-ev[0], -ev[1], -ev[2]};
            sub3(qa, p1, t1);
            cross3(ev, t1, na);
            sub3(qb, p2, t2);
            cross3(me, t2, nb);
            double na2 = dot3(na, na), nb2 = dot3(nb, nb);
            double ga[3] = {-l * na[0] / na2, -l * na[1] / na2, -l * na[2] / na2};
            double gb[3] = {-l * nb[0] / nb2, -l * nb[1] / nb2, -l * nb[2] / nb2};
            double sa = dot3(t1, ev) / (l * l);
            double qb1[3];
            sub3(qb, p1, qb1);
            double sb = dot3(qb1, ev) / (l * l);
            addv(F, h[2], -cb, ga);
            addv(F, h[3], -cb, gb);
            double g1[3], g2[3];
            for (int d = 0; d < 3; d++) {
                g1[d] = -(1.0 - sa) * ga[d] - (1.0 - sb) * gb[d];
                g2[d] = -sa * ga[d] - sb * gb[d];
            }
            addv(F, h[0], -cb, g1);
            addv(F, h[1], -cb, g2);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* contact forces                                                            */
/* ------------------------------------------------------------------------ */

/* potential and -dU/dd of the contact law at surface distance d */
static void soft_sphere(const orc_contact *P, double d, double *U, double *f) {
    *U = 0.0;
    *f = 0.0;
    if (d >= P->rcut) return;
    if (d >= P->dmin) {
        *U = P->a * pow(d, -P->n);
        *f = P->n * P->a * pow(d, -P->n - 1.0);
    } else {
        double fm = P->n * P->a * pow(P->dmin, -P->n - 1.0);
        *U = P->a * pow(P->dmin, -P->n) + fm * (P->dmin - d);
        *f = fm;
    }
}

/* minimum-image difference along a periodic axis of length L */
static double min_image(double d, int L, int periodic) {
    if (!periodic) return d;
    return d - L * floor(d / L + 0.5);
}

static int cell_of(const orc_mesh *M, int k) {
    int c = 0;
    while (M->vert_off[c + 1] <= k) c++;
    return c;
}

/* Energy of the contact potential and forces F = -grad (F [nv][3], overwritten). */
static double contact(const orc_lattice *L, const orc_mesh *M, const double *X, double *F) {
    const orc_contact *P = M->contact;
    const int dims[3] = {L->nx, L->ny, L->nz};
    double E = 0.0;
    if (F) memset(F, 0, sizeof(double) * 3 * M->nverts);
    if (!P) return 0.0;
    if (P->cell_cell) {
        for (int i = 0; i < M->nverts; i++) {
            int ci = cell_of(M, i);
            for (int j = M->vert_off[ci + 1]; j < M->nverts; j++) {
                double d[3];
                for (int a = 0; a < 3; a++) d[a] = min_image(X[3 * i + a] - X[3 * j + a], dims[a], L->periodic[a]);
                double r = norm3(d);
                if (r == 0.0) continue; /* coincident points: no direction */
                double U, f;
                soft_sphere(P, r - P->roff, &U, &f);
                E += U;
                if (F && f != 0.0) {
                    addv(F, i, f / r, d);
                    addv(F, j, -f / r, d);
                }
            }
        }
    }
    for (int k = 0; k < M->nverts; k++) {
        const double *x = X + 3 * k;
        for (int p = 0; p < P->nplanes; p++) {
            const double *pl = P->planes + 4 * p;
            double U, f;
            soft_sphere(P, dot3(pl, x) - pl[3] - P->roff, &U, &f);
            E += U;
            if (F) addv(F, k, f, pl);
        }
        for (int q = 0; q < P->ncyl; q++) {
            const double *cy = P->cyl + 3 * q;
            double d[3] = {min_image(x[0] - cy[0], L->nx, L->periodic[0]),
                           min_image(x[1] - cy[1], L->ny, L->periodic[1]), 0.0};
            double rho = norm3(d);
            if (rho == 0.0) continue; /* on the axis: no direction */
            double U, f;
            soft_sphere(P, rho - cy[2] - P->roff, &U, &f);
            E += U;
            if (F && f != 0.0) addv(F, k, f / rho, d);
        }
        for (int q = 0; q < P->nsph; q++) {
            const double *sp = P->sph + 4 * q;
            double d[3];
            for (int a = 0; a < 3; a++) d[a] = min_image(x[a] - sp[a], dims[a], L->periodic[a]);
            double r = norm3(d);
            if (r == 0.0) continue; /* at the centre: no direction */
            double U, f;
            soft_sphere(P, r - sp[3] - P->roff, &U, &f);
            E += U;
            if (F && f != 0.0) addv(F, k, f / r, d);
        }
    }
    return E;
}

double orc_contact_energy(const orc_lattice *L, const orc_mesh *M, const double *X) {
    return contact(L, M, X, NULL);
}

void orc_contact_forces(const orc_lattice *L, const orc_mesh *M, const double *X, double *F) {
    contact(L, M, X, F);
}

/* ------------------------------------------------------------------------ */
/* the coupled step                                                          */
/* ------------------------------------------------------------------------ */

/* Optional per-step diagnostics written by orc_step (NULL to skip). */
typedef struct {
    double *uk;   /* [nv][3] interpolated velocity */
    double *Fel;  /* [nv][3] elastic force (plus contact forces when enabled) */
    double *Fc;   /* [nv][3] coupling force */
    double *F;    /* [3][N]  total force seen by the collision */
} orc_trace;

/* One step n -> n+1.  f (in) and fnew (out) are distinct [19][N] arrays;
 * solid-node slots of fnew are copied from f.  M may be NULL (no cells);
 * otherwise X, V [nv][3] are advanced in place. */
int orc_step(const orc_lattice *L, const orc_mesh *M, const double *f, double *fnew, double *X, double *V,
             const orc_trace *tr) {
    long N = nnodes(L);
    double *uext = malloc(sizeof(double) * 3 * N);
    double *F = malloc(sizeof(double) * 3 * N);
    if (!uext || !F) { free(uext); free(F); return -1; }
    orc_fluid_velocity(L, f, NULL, uext);
    for (int d = 0; d < 3; d++)
        for (long n = 0; n < N; n++) F[d * N + n] = L->g[d] + (L->G ? L->G[d * N + n] : 0.0);
    double *uk = NULL, *Fel = NULL, *Fc = NULL;
    int nv = M ? M->nverts : 0;
    if (nv) {
        uk = malloc(sizeof(double) * 3 * nv);
        Fel = malloc(sizeof(double) * 3 * nv);
        Fc = malloc(sizeof(double) * 3 * nv);
        double *mFc = malloc(sizeof(double) * 3 * nv);
        orc_interpolate(L, uext, nv, X, uk);                 /* step 1 */
        orc_membrane_forces(M, X, Fel);                      /* step 2 */
        if (M->contact) {                                    /* collisions, Sec. 2.4 */
            double *Fk = malloc(sizeof(double) * 3 * nv);
            contact(L, M, X, Fk);
            for (int i = 0; i < 3 * nv; i++) Fel[i] += Fk[i];
            free(Fk);
        }
        for (int i = 0; i < 3 * nv; i++) {
            Fc[i] = M->xi * M->Av[i / 3] * (uk[i] - V[i]);
            mFc[i] = -Fc[i];
        }
        orc_spread(L, nv, X, mFc, F);                        /* step 3 */
        free(mFc);
    }
    for (int i = 0; i < Q; i++)
        for (long n = 0; n < N; n++)
            if (L->solid[n]) fnew[i * N + n] = f[i * N + n];
    orc_collide_stream(L, f, F, fnew);                      /* step 4, fluid */
    for (int i = 0; i < 3 * nv; i++) {                      /* step 4, points */
        V[i] += M->dt / (M->mass * M->Av[i / 3]) * (Fel[i] + Fc[i]);
        X[i] += M->dt * V[i];
    }
    if (tr) {
        if (tr->uk && nv) memcpy(tr->uk, uk, sizeof(double) * 3 * nv);
        if (tr->Fel && nv) memcpy(tr->Fel, Fel, sizeof(double) * 3 * nv);
        if (tr->Fc && nv) memcpy(tr->Fc, Fc, sizeof(double) * 3 * nv);
        if (tr->F) memcpy(tr->F, F, sizeof(double) * 3 * N);
    }
    free(uk); free(Fel); free(Fc);
    free(uext); free(F);
    return 0;
}

/* nsteps steps; the result is left in f (two-buffer swap internally). */
int orc_run(const orc_lattice *L, const orc_mesh *M, double *f, double *X, double *V, int nsteps) {
    long N = nnodes(L);
    double *g = malloc(sizeof(double) * Q * N);
    if (!g) return -1;
    double *a = f, *b = g;
    for (int s = 0; s < nsteps; s++) {
        if (orc_step(L, M, a, b, X, V, NULL)) { free(g); return -1; }
        double *t = a; a = b; b = t;
    }
    if (a != f) memcpy(f, a, sizeof(double) * Q * N);
    free(g);
    return 0;
}

/* Objective of the differentiation workload (the paper has none; reading):
 * the outflow through the last x plane, sum over its fluid nodes of
 * j_x + (g_x + G_x)/2 (the x-momentum carried by the populations f, with
 * the half-force shift of the velocity), plus for every cell of M the
 * squared distance between the vertex centroid of X and that of X0 (both
 * [nv][3] absolute positions).  M may be NULL (no cell term). */
double orc_objective(const orc_lattice *L, const orc_mesh *M, const double *f, const double *X, const double *X0) {
    long N = nnodes(L);
    ksum J = {0, 0};
    for (int z = 0; z < L->nz; z++)
        for (int y = 0; y < L->ny; y++) {
            long n = (L->nx - 1) + (long)L->nx * (y + (long)L->ny * z);
            if (L->solid[n]) continue;
            double jx = 0.0;
            for (int i = 0; i < Q; i++) jx += f[i * N + n] * CX[i];
            kadd(&J, jx + 0.5 * (L->g[0] + (L->G ? L->G[n] : 0.0)));
        }
    if (M)
        for (int c = 0; c < M->ncells; c++) {
            int a = M->vert_off[c], b = M->vert_off[c + 1];
            double d2 = 0.0;
            for (int d = 0; d < 3; d++) {
                double s1 = 0.0, s0 = 0.0;
                for (int k = a; k < b; k++) {
                    s1 += X[3 * k + d];
                    s0 += X0[3 * k + d];
                }
                double dd = (s1 - s0) / (b - a);
                d2 += dd * dd;
            }
            kadd(&J, d2);
        }
    return J.s + J.c;
}

/* ------------------------------------------------------------------------ */
/* magnetic bead stage (the chain-forming part of the filter, Sec. 2.5)      */
/* ------------------------------------------------------------------------ */

/* Units: lattice lengths and steps, magnetic constant mu0 = 1, so B = H
 * outside the magnets.  Readings: the magnets are planar sheets of uniform
 * magnetic surface charge sigma (z = const, rectangle [x0,x1] x [y0,y1]),
 * whose field is H(r) = sigma/(4 pi) * integral (r - r')/|r - r'|^3 dA';
 * plus a uniform bias field.  A soft-magnetic bead of radius a and
 * susceptibility chi takes the induced moment m = 4 pi a^3 chi/(chi + 3) B
 * (a sphere in a uniform field; the beads' fields on each other are not fed
 * back into the moments).  Forces: the gradient force F_g = grad(m.B) at
 * fixed m; the dipole interaction of two beads (the paper's interaction
 * equation); a soft-sphere repulsion between beads (surface distance
 * r - 2a) and from the walls z = 1/2, nz - 3/2 (distance z - 1/2 - a);
 * overdamped motion against Stokes drag, x += dt F / (6 pi eta a). */
typedef struct {
    int nsheets;
    const double *sheets; /* [nsheets][6] = (z, x0, x1, y0, y1, sigma) */
    double bias[3];
    double a, chi, eta, dt;
    double rep_a, rep_n, rep_cut; /* repulsion U(d) = rep_a d^-rep_n for d in (0, rep_cut), linear below rep_cut/100 */
    int nx, ny, nz;
    int periodic[3];
    int walls_z;                  /* 1: walls at z = 1/2 and nz - 3/2 */
    int quad;                     /* Gauss-Legendre panels per side of a sheet (8 points per panel) */
} orc_mag;

/* 8-point Gauss-Legendre nodes and weights on [-1, 1] */
static const double GLX[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290, -0.1834346424956498,
                              0.1834346424956498,  0.5255324099163290,  0.7966664774136267,  0.9602898564975363};
static const double GLW[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873, 0.3626837833783620,
                              0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};

/* field of the sheets and the bias at p, and (if J is not NULL) its
 * gradient J[i][j] = dB_i/dx_j, by composite Gauss-Legendre quadrature of
 * the Coulomb kernel r/|r|^3 and of its gradient delta_ij/|r|^3 -
 * 3 r_i r_j/|r|^5 (differentiation under the integral sign) */
static void mag_field_at(const orc_mag *G, const double p[3], double B[3], double J[9]) {
    for (int d = 0; d < 3; d++) B[d] = G->bias[d];
    if (J)
        for (int d = 0; d < 9; d++) J[d] = 0.0;
    for (int s = 0; s < G->nsheets; s++) {
        const double *S = G->sheets + 6 * s;
        /* panels no wider than a third of the point's distance from the sheet plane */
        double L = fmax(S[2] - S[1], S[4] - S[3]), dz = fabs(p[2] - S[0]);
        int np = G->quad > 0 ? G->quad : 16;
        double need = dz > 0 ? ceil(3.0 * L / dz) : 1024.0;
        if (need > np) np = need > 1024.0 ? 1024 : (int)need;
        double hx = (S[2] - S[1]) / np, hy = (S[4] - S[3]) / np;
        double acc[3] = {0.0, 0.0, 0.0}, jac[9] = {0.0};
        for (int i = 0; i < np; i++)
            for (int j = 0; j < np; j++)
                for (int a = 0; a < 8; a++)
                    for (int b = 0; b < 8; b++) {
                        double xq = S[1] + hx * (i + 0.5 + 0.5 * GLX[a]);
                        double yq = S[3] + hy * (j + 0.5 + 0.5 * GLX[b]);
                        double r[3] = {p[0] - xq, p[1] - yq, p[2] - S[0]};
                        double R2 = dot3(r, r), R = sqrt(R2);
                        double w = GLW[a] * GLW[b] * 0.25 * hx * hy / (R2 * R);
                        for (int d = 0; d < 3; d++) acc[d] += w * r[d];
                        if (J)
                            for (int d = 0; d < 3; d++)
                                for (int e = 0; e < 3; e++)
                                    jac[3 * d + e] += w * ((d == e ? 1.0 : 0.0) - 3.0 * r[d] * r[e] / R2);
                    }
        for (int d = 0; d < 3; d++) B[d] += S[5] / (4.0 * PI_) * acc[d];
        if (J)
            for (int d = 0; d < 9; d++) J[d] += S[5] / (4.0 * PI_) * jac[d];
    }
}

void orc_mag_field(const orc_mag *G, const double *p, int n, double *B, double *J) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; k++) mag_field_at(G, p + 3 * k, B + 3 * k, J ? J + 9 * k : NULL);
}

/* dipole-dipole force on bead 2 from bead 1, r = x2 - x1 (the paper's
 * interaction equation with mu0 = 1) */
static void dipole_force(const double *m1, const double *m2, const double *r, double *F) {
    double r2 = dot3(r, r), rn = sqrt(r2);
    double m1r = dot3(m1, r), m2r = dot3(m2, r), mm = dot3(m1, m2);
    double c = 3.0 / (4.0 * PI_ * r2 * r2 * rn);
    for (int d = 0; d < 3; d++) F[d] = c * (m1r * m2[d] + m2r * m1[d] + mm * r[d] - 5.0 * m1r * m2r * r[d] / r2);
}

/* dipole-dipole energy, for the gradient pin: U = (m1.m2 - 3 (m1.rh)(m2.rh)) / (4 pi r^3) */
double orc_dipole_energy(const double *m1, const double *m2, const double *r) {
    double r2 = dot3(r, r), rn = sqrt(r2);
    return (dot3(m1, m2) - 3.0 * dot3(m1, r) * dot3(m2, r) / r2) / (4.0 * PI_ * r2 * rn);
}

void orc_dipole_force(const double *m1, const double *m2, const double *r, double *F) { dipole_force(m1, m2, r, F); }

static double rep_force(const orc_mag *G, double d) {
    if (d >= G->rep_cut) return 0.0;
    double dmin = G->rep_cut / 100.0;
    return G->rep_n * G->rep_a * pow(d < dmin ? dmin : d, -G->rep_n - 1.0);
}

/* induced moments m [n][3] of beads at x [n][3] */
void orc_mag_moments(const orc_mag *G, const double *x, int n, double *m) {
    const double alpha = 4.0 * PI_ * G->a * G->a * G->a * G->chi / (G->chi + 3.0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < n; k++) {
        double B[3];
        mag_field_at(G, x + 3 * k, B, NULL);
        for (int d = 0; d < 3; d++) m[3 * k + d] = alpha * B[d];
    }
}

/* total force on bead k given every bead's moment: gradient force
 * F_j = sum_i m_i dB_i/dx_j, then the dipole force and repulsion of every
 * other bead (minimum image), then the walls */
static void force_on(const orc_mag *G, const double *x, int n, const double *m, int k, double F[3]) {
    const int dims[3] = {G->nx, G->ny, G->nz};
    double B[3], J[9];
    mag_field_at(G, x + 3 * k, B, J);
    for (int j = 0; j < 3; j++) {
        double s = 0.0;
        for (int i = 0; i < 3; i++) s += m[3 * k + i] * J[3 * i + j];
        F[j] = s;
    }
    for (int l = 0; l < n; l++) {
        if (l == k) continue;
        double r[3];
        for (int d = 0; d < 3; d++) r[d] = min_image(x[3 * k + d] - x[3 * l + d], dims[d], G->periodic[d]);
        double Fd[3];
        dipole_force(m + 3 * l, m + 3 * k, r, Fd); /* on k from l */
        double rn = norm3(r);
        double fr = rep_force(G, rn - 2.0 * G->a) / rn;
        for (int d = 0; d < 3; d++) F[d] += Fd[d] + fr * r[d];
    }
    if (G->walls_z) {
        double z = x[3 * k + 2];
        F[2] += rep_force(G, z - 0.5 - G->a) - rep_force(G, (G->nz - 1.5) - z - G->a);
    }
}

/* moments m [n][3] and total forces F [n][3] on beads at x [n][3] */
void orc_mag_forces(const orc_mag *G, const double *x, int n, double *m, double *F) {
    orc_mag_moments(G, x, n, m);
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < n; k++) force_on(G, x, n, m, k, F + 3 * k);
}

/* total forces F [nidx][3] on the beads idx [nidx] only (every bead's
 * moment is still needed); returns -1 on a bad index or no memory */
int orc_mag_forces_sample(const orc_mag *G, const double *x, int n, const int *idx, int nidx, double *F) {
    for (int i = 0; i < nidx; i++)
        if (idx[i] < 0 || idx[i] >= n) return -1;
    double *m = malloc(sizeof(double) * 3 * (size_t)n);
    if (!m) return -1;
    orc_mag_moments(G, x, n, m);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < nidx; i++) force_on(G, x, n, m, idx[i], F + 3 * i);
    free(m);
    return 0;
}

/* nsteps overdamped steps of the beads, x [n][3] in place */
int orc_mag_run(const orc_mag *G, double *x, int n, int nsteps) {
    double *m = malloc(sizeof(double) * 3 * n), *F = malloc(sizeof(double) * 3 * n);
    if (!m || !F) { free(m); free(F); return -1; }
    const double mob = G->dt / (6.0 * PI_ * G->eta * G->a);
    for (int s = 0; s < nsteps; s++) {
        orc_mag_forces(G, x, n, m, F);
        for (int i = 0; i < 3 * n; i++) x[i] += mob * F[i];
    }
    free(m);
    free(F);
    return 0;
}

/* the chains fixed in space: node (x, y, z) is solid if its centre lies
 * within a of a bead centre (minimum image); solid is OR-ed in */
void orc_mag_freeze(const orc_mag *G, const double *x, int n, uint8_t *solid) {
    const int dims[3] = {G->nx, G->ny, G->nz};
    for (int z = 0; z < G->nz; z++)
        for (int y = 0; y < G->ny; y++)
            for (int xx = 0; xx < G->nx; xx++) {
                const double p[3] = {xx, y, z};
                for (int k = 0; k < n; k++) {
                    double r2 = 0.0;
                    for (int d = 0; d < 3; d++) {
                        double dd = min_image(p[d] - x[3 * k + d], dims[d], G->periodic[d]);
                        r2 += dd * dd;
                    }
                    if (r2 <= G->a * G->a) {
                        solid[xx + (long)G->nx * (y + (long)G->ny * z)] = 1;
                        break;
                    }
                }
            }
}

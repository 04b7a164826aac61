/*
 * CPU oracle for the well-balanced WCSPH hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * FP64 statement of what the GPU path computes.  Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header or constant with the HIP library and never calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (contraction off so that a*b+c is two roundings, the same as written).
 *
 * Paper passages followed (section / equation / algorithm):
 *   kernel          Sec. 2.1, Eq. (c2kernel); 3D normalisation 21/(16 pi h^3)
 *   potential       Sec. 2.2.1, rho = rho0 exp(phi / C0^2), Eq. (newEqns)
 *   gradient        Sec. 2.2.2, Eqs. (parGrad), (renorm), (lfsover)
 *   stabilisers     Sec. 2.3: delta-SPH term, particle shifting, TIC switch
 *   final system    Sec. 2.3, Eq. (sph)
 *   integrator      Sec. 2.3, SSP-RK2 stages and the three-way time step rule
 *   walls           Sec. 2.4, Eq. (phiBn) and the slip mirror
 *   moving walls    Sec. 4 (aircraft ditching): a body moving along a
 *                   prescribed velocity history U(T) given piecewise
 *   free body       Sec. 4 (cylinder water entry): a rigid body falling
 *                   under gravity and the water's force and torque
 *   neighbours      Sec. 3, Eqs. (hashid), (ixyz), Algorithm 1
 *   eigenvalues     Sec. 3 (minimum eigenvalue of L), by Jacobi rotations
 * Readings of passages that are silent or garbled are noted where they are
 * used below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EDOMAIN (-4)
#define ORC_ENONFINITE (-5)
#define ORC_ECAP (-8)
#define ORC_ENOMEM (-9)

/* flags */
#define ORC_DELTA 1u          /* delta-SPH potential diffusion            */
#define ORC_PST 2u            /* particle shifting                        */
#define ORC_TIC 4u            /* tensile-instability switch               */
#define ORC_FS_PROJECT 8u     /* remove the normal part of dU at the FS   */
#define ORC_CONT_UNCORR 16u   /* uncorrected continuity where TIC is on   */

#define ORC_FS_NONE 0
#define ORC_FS_EXACT 1

#define NFEAT 16

typedef struct {
    int32_t dim, fs_mode;
    uint32_t flags, pad_;
    double dx, h, c0, rho0, nu, delta, cfl, pst_R, pst_n;
    double lambda_tic, lambda_fs_lo, lambda_fs_hi, lambda_singular;
    double gravity[3], forcing_amp[3], forcing_omega;
    double domain_lo[3], domain_hi[3], cell_size;
    /* prescribed body motion: U(t) = a_k + b_k t on piece k, T_k <= t <=
     * T_{k+1} (k = 0..body_pieces-1, the lower piece at a shared breakpoint),
     * zero outside [T_0, T_K]; body_a / body_b hold 3 components per piece */
    int32_t body_pieces, pad2_;
    double body_t[5], body_a[12], body_b[12];
    /* a rigid body of kind-2 dummies moving under G(t) and the water's force
     * and torque (body_free != 0; the prescribed motion is then unused):
     * mass, inertia tensor about the centre in the body frame (xx yy zz xy
     * xz yz), and the centre of the pose the dummies are given in */
    int32_t body_free, pad3_;
    double body_mass, body_inertia[6], body_c0[3];
} orc_params;

/* State of the free body: centre, unit quaternion (w, x, y, z) of the
 * rotation from the reference pose, velocity, angular velocity (world
 * frame). */
typedef struct {
    double c[3], q[4], v[3], w[3];
} orc_body;

/* Outputs of one right-hand-side evaluation, one row per particle in the
 * caller's order.  Rows of dummy particles hold the mirrored phi / U and the
 * source fluid index; their rate rows are zero. */
typedef struct {
    double *acc;       /* n*dim  DU/Dt                                   */
    double *dphi;      /* n      Dphi/Dt                                 */
    double *dushift;   /* n*dim  delta U (clamped, projected)            */
    double *lam;       /* n*3    eigenvalues of sym(L), ascending        */
    double *normal;    /* n*dim  unit free-surface normal (0 if none)    */
    int32_t *fs;       /* n      1 = free surface                        */
    int32_t *tic;      /* n      1 = conservative branch used            */
    int32_t *nnb;      /* n      |N(i)|                                  */
    double *feat;      /* n*16   classifier features                     */
    double *fs_margin; /* n      distance of the scan decision to a tie  */
    double *mir_phi;   /* n      dummies: mirrored phi                   */
    double *mir_u;     /* n*dim  dummies: mirrored U                     */
    int32_t *mir_src;  /* n      dummies: source fluid index or -1       */
    double *scal;      /* 10     U_max, |G(t)|, t, singular count, force
                                   (3) and torque (3) of the water on the
                                   free body                             */
} orc_rates;

static const double ORC_PI = 3.14159265358979323846;

/* ---------------------------------------------------------------- kernel */

/* Wendland C2 normalisation: 2D value printed with Eq. (c2kernel); the 3D
 * value is the one that makes the kernel integrate to one over R^3. */
static double kern_alpha(int dim, double h) {
    if (dim == 2) return 7.0 / (4.0 * ORC_PI * h * h);
    return 21.0 / (16.0 * ORC_PI * h * h * h);
}

/* W(q), Eq. (c2kernel). */
double orc_W(int dim, double h, double q) {
    if (q > 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return kern_alpha(dim, h) * t * t * t * t * (2.0 * q + 1.0);
}

/* K(q) such that grad_i W_ij = K(q) * (x_j - x_i).  From dW/dq = -5 alpha q
 * (1-q/2)^3 and dq/dx_i = -(x_j - x_i)/(q h^2). */
double orc_K(int dim, double h, double q) {
    if (q > 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return 5.0 * kern_alpha(dim, h) / (h * h) * t * t * t;
}

/* Body force G(t): gravity plus the tank-frame forcing A w^2 sin(w t). */
static void body_force(const orc_params *p, double t, double G[3]) {
    double s = sin(p->forcing_omega * t);
    for (int a = 0; a < 3; ++a)
        G[a] = p->gravity[a] + p->forcing_amp[a] * p->forcing_omega * p->forcing_omega * s;
}

/* Prescribed motion of the body (kind 2 dummies).  The ditching case of
 * Sec. 4 gives the body's velocity as a piecewise function of time; here a
 * piece is affine in t.  U is the velocity at t; D the displacement since
 * T_0, the integral of U from T_0 to t, piece by piece:
 *   int_{T_k}^{tau} (a + b s) ds = a (tau - T_k) + b (tau^2 - T_k^2) / 2.
 * Reading: the body is given at its position of time T_0 (D = 0), and it
 * only translates. */
void orc_body_motion(const orc_params *p, double t, double D[3], double U[3]) {
    for (int a = 0; a < 3; ++a) D[a] = U[a] = 0.0;
    int found = 0;
    for (int k = 0; k < p->body_pieces; ++k) {
        double t0 = p->body_t[k], t1 = p->body_t[k + 1];
        if (!found && t >= t0 && t <= t1) {
            for (int a = 0; a < 3; ++a) U[a] = p->body_a[3 * k + a] + p->body_b[3 * k + a] * t;
            found = 1;
        }
        if (t > t0) {
            double tau = t < t1 ? t : t1;
            for (int a = 0; a < 3; ++a)
                D[a] += p->body_a[3 * k + a] * (tau - t0) + p->body_b[3 * k + a] * (tau * tau - t0 * t0) / 2.0;
        }
    }
}

static double body_force_max(const orc_params *p) {
    /* max over t of |G(t)|: the forcing is a single sinusoid, so the maximum
     * is reached at sin = +1 or -1. */
    double best = 0.0;
    for (int sgn = -1; sgn <= 1; sgn += 2) {
        double s2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double g = p->gravity[a] + sgn * p->forcing_amp[a] * p->forcing_omega * p->forcing_omega;
            s2 += g * g;
        }
        if (sqrt(s2) > best) best = sqrt(s2);
    }
    return best;
}

/* Rotation matrix (row-major) of the unit quaternion q = (w, x, y, z). */
static void quat_matrix(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Pose of a free-body dummy: x = c + R (x_ref - c0), n = R n_ref, and the
 * wall velocity there, U_w = v + w x (x - c).  dim-component rows. */
static void free_body_place(const orc_params *p, const orc_body *b, const double *xr, const double *nr, double *x,
                            double *n, double *uw) {
    int dim = p->dim;
    double R[9], d0[3] = {0, 0, 0}, n0[3] = {0, 0, 0}, d[3], r[3], wr[3];
    quat_matrix(b->q, R);
    for (int a = 0; a < dim; ++a) {
        d0[a] = xr[a] - p->body_c0[a];
        n0[a] = nr[a];
    }
    for (int a = 0; a < 3; ++a) {
        d[a] = R[3 * a] * d0[0] + R[3 * a + 1] * d0[1] + R[3 * a + 2] * d0[2];
        r[a] = R[3 * a] * n0[0] + R[3 * a + 1] * n0[1] + R[3 * a + 2] * n0[2];
    }
    cross3(b->w, d, wr);
    for (int a = 0; a < dim; ++a) {
        x[a] = b->c[a] + d[a];
        n[a] = r[a];
        uw[a] = b->v[a] + wr[a];
    }
}

/* ---------------------------------------------------------- neighbours */

static double cell_R(const orc_params *p) { return p->cell_size > 0.0 ? p->cell_size : 2.0 * p->h; }

/* Number of background cells along each axis.  Eq. (ixyz) prints
 * floor((max-min)/R); one is added so that the last partial cell exists. */
static void grid_dims(const orc_params *p, int64_t N[3]) {
    double R = cell_R(p);
    for (int a = 0; a < 3; ++a) {
        if (a < p->dim) N[a] = (int64_t)floor((p->domain_hi[a] - p->domain_lo[a]) / R) + 1;
        else N[a] = 1;
    }
}

/* Cell coordinates, Eq. (ixyz), and HashID, Eq. (hashid). */
int orc_cells(const orc_params *p, int64_t n, const double *x, int32_t *cell3, int64_t *hash) {
    int64_t N[3];
    grid_dims(p, N);
    double R = cell_R(p);
    int dim = p->dim;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) {
            double xa = x[i * dim + a];
            if (!isfinite(xa)) return ORC_ENONFINITE;
            if (xa < p->domain_lo[a] || xa > p->domain_hi[a]) return ORC_EDOMAIN;
            c[a] = (int64_t)floor((xa - p->domain_lo[a]) / R);
            if (c[a] < 0 || c[a] >= N[a]) return ORC_EDOMAIN;
        }
        if (cell3) for (int a = 0; a < 3; ++a) cell3[i * 3 + a] = (int32_t)c[a];
        if (hash) hash[i] = c[0] + c[1] * N[0] + c[2] * N[0] * N[1];
    }
    return ORC_OK;
}

/* |x_j - x_i|^2, summed in axis order. */
static double dist2(int dim, const double *xi, const double *xj) {
    double s = 0.0;
    for (int a = 0; a < dim; ++a) {
        double d = xj[a] - xi[a];
        s += d * d;
    }
    return s;
}

/* Neighbour relation: j != i and |x_j - x_i| <= 2h (Algorithm 1's test),
 * compared on squares. */
static int in_range(double r2, double two_h) { return r2 <= two_h * two_h; }

/* Brute-force O(n^2) neighbour lists in CSR form, j ascending. */
int orc_neighbors_brute(const orc_params *p, int64_t n, const double *x, int64_t *off,
                        int32_t *ids, int64_t cap, int64_t *needed) {
    int dim = p->dim;
    double two_h = 2.0 * p->h;
    int64_t k = 0;
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r2 = dist2(dim, x + i * dim, x + j * dim);
            if (in_range(r2, two_h)) {
                if (r2 == 0.0) return ORC_ENONFINITE;
                if (ids && k < cap) ids[k] = (int32_t)j;
                ++k;
            }
        }
        off[i + 1] = k;
    }
    if (needed) *needed = k;
    return k > cap ? ORC_ECAP : ORC_OK;
}

/* Cell-list neighbour lists (Sec. 3): HashID, a stable counting sort of the
 * particles by HashID (within a cell: ascending index), begin/end per cell,
 * then Algorithm 1's 3^d-cell loop (z outermost, x innermost). */
typedef struct {
    int64_t N[3];
    int64_t ncell;
    int64_t *begin;   /* ncell+1 */
    int64_t *sorted;  /* n       */
    int32_t *cell3;   /* n*3     */
} cell_list;

static void cell_list_free(cell_list *cl) {
    free(cl->begin);
    free(cl->sorted);
    free(cl->cell3);
    memset(cl, 0, sizeof(*cl));
}

static int cell_list_build(const orc_params *p, int64_t n, const double *x, cell_list *cl) {
    memset(cl, 0, sizeof(*cl));
    grid_dims(p, cl->N);
    cl->ncell = cl->N[0] * cl->N[1] * cl->N[2];
    int64_t *hash = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    cl->cell3 = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(n > 0 ? n : 1));
    cl->begin = (int64_t *)calloc((size_t)cl->ncell + 1, sizeof(int64_t));
    cl->sorted = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!hash || !cl->cell3 || !cl->begin || !cl->sorted) {
        free(hash);
        cell_list_free(cl);
        return ORC_ENOMEM;
    }
    int st = orc_cells(p, n, x, cl->cell3, hash);
    if (st != ORC_OK) {
        free(hash);
        cell_list_free(cl);
        return st;
    }
    for (int64_t i = 0; i < n; ++i) cl->begin[hash[i] + 1]++;
    for (int64_t c = 0; c < cl->ncell; ++c) cl->begin[c + 1] += cl->begin[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cl->ncell > 0 ? cl->ncell : 1));
    if (!fill) {
        free(hash);
        cell_list_free(cl);
        return ORC_ENOMEM;
    }
    memcpy(fill, cl->begin, sizeof(int64_t) * (size_t)cl->ncell);
    for (int64_t i = 0; i < n; ++i) cl->sorted[fill[hash[i]]++] = i;
    free(fill);
    free(hash);
    return ORC_OK;
}

/* Visit the candidates of particle i in Algorithm 1's order (z outermost, x
 * innermost); emit j in range.  With R = 2h the stencil is Algorithm 1's
 * 3^d cells; a smaller R widens it to ceil(2h / R) cells on each side so that
 * the same neighbour set is found.  Returns the number found (writes at most
 * cap ids). */
static int64_t cell_list_query(const orc_params *p, const cell_list *cl, const double *x, int64_t i,
                               int32_t *ids, int64_t cap, int *zero_dist) {
    int dim = p->dim;
    double two_h = 2.0 * p->h;
    const int32_t *ci = cl->cell3 + i * 3;
    int64_t k = 0;
    int reach = (int)ceil(two_h / cell_R(p));
    int zr = dim == 3 ? reach : 0;
    for (int dz = -zr; dz <= zr; ++dz) {
        int64_t cz = ci[2] + dz;
        if (cz < 0 || cz >= cl->N[2]) continue;
        for (int dy = -reach; dy <= reach; ++dy) {
            int64_t cy = ci[1] + dy;
            if (cy < 0 || cy >= cl->N[1]) continue;
            for (int dxc = -reach; dxc <= reach; ++dxc) {
                int64_t cx = ci[0] + dxc;
                if (cx < 0 || cx >= cl->N[0]) continue;
                int64_t c = cx + cy * cl->N[0] + cz * cl->N[0] * cl->N[1];
                for (int64_t s = cl->begin[c]; s < cl->begin[c + 1]; ++s) {
                    int64_t j = cl->sorted[s];
                    if (j == i) continue;
                    double r2 = dist2(dim, x + i * dim, x + j * dim);
                    if (in_range(r2, two_h)) {
                        if (r2 == 0.0) *zero_dist = 1;
                        if (ids && k < cap) ids[k] = (int32_t)j;
                        ++k;
                    }
                }
            }
        }
    }
    return k;
}

int orc_neighbors_cells(const orc_params *p, int64_t n, const double *x, int64_t *off,
                        int32_t *ids, int64_t cap, int64_t *needed) {
    cell_list cl;
    int st = cell_list_build(p, n, x, &cl);
    if (st != ORC_OK) return st;
    int zero = 0;
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + cell_list_query(p, &cl, x, i, NULL, 0, &zero);
    if (needed) *needed = off[n];
    if (zero) {
        cell_list_free(&cl);
        return ORC_ENONFINITE;
    }
    if (off[n] > cap) {
        cell_list_free(&cl);
        return ORC_ECAP;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int z = 0;
        cell_list_query(p, &cl, x, i, ids + off[i], off[i + 1] - off[i], &z);
    }
    cell_list_free(&cl);
    return ORC_OK;
}

/* Builds the CSR of every particle with the chosen mode (0 brute, 1 cells). */
static int build_csr(const orc_params *p, int64_t n, const double *x, int mode, int64_t **off_out,
                     int32_t **ids_out) {
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!off) return ORC_ENOMEM;
    int64_t need = 0;
    int st = mode == 0 ? orc_neighbors_brute(p, n, x, off, NULL, 0, &need)
                       : orc_neighbors_cells(p, n, x, off, NULL, 0, &need);
    if (st != ORC_OK && st != ORC_ECAP) {
        free(off);
        return st;
    }
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(need > 0 ? need : 1));
    if (!ids) {
        free(off);
        return ORC_ENOMEM;
    }
    st = mode == 0 ? orc_neighbors_brute(p, n, x, off, ids, need, &need)
                   : orc_neighbors_cells(p, n, x, off, ids, need, &need);
    if (st != ORC_OK) {
        free(off);
        free(ids);
        return st;
    }
    *off_out = off;
    *ids_out = ids;
    return ORC_OK;
}

/* The same CSR (cells mode) restricted to the rows with rows[i] != 0; the
 * other rows are empty.  Lets a large case be checked on a sample of
 * particles without the neighbour lists of all of them. */
static int build_csr_rows(const orc_params *p, int64_t n, const double *x, const uint8_t *rows,
                          int64_t **off_out, int32_t **ids_out) {
    cell_list cl;
    int st = cell_list_build(p, n, x, &cl);
    if (st != ORC_OK) return st;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!off) {
        cell_list_free(&cl);
        return ORC_ENOMEM;
    }
    int zero = 0;
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i)
        off[i + 1] = off[i] + (rows[i] ? cell_list_query(p, &cl, x, i, NULL, 0, &zero) : 0);
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(off[n] > 0 ? off[n] : 1));
    if (!ids) {
        free(off);
        cell_list_free(&cl);
        return ORC_ENOMEM;
    }
    if (zero) {
        free(off);
        free(ids);
        cell_list_free(&cl);
        return ORC_ENONFINITE;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        if (!rows[i]) continue;
        int z = 0;
        cell_list_query(p, &cl, x, i, ids + off[i], off[i + 1] - off[i], &z);
    }
    cell_list_free(&cl);
    *off_out = off;
    *ids_out = ids;
    return ORC_OK;
}

/* -------------------------------------------------------- small algebra */

/* Eigenvalues of the symmetric part of a 2x2 / 3x3 matrix, ascending
 * (Sec. 3 uses the minimum eigenvalue of the correction matrix).  The method
 * evaluates them in closed form; the oracle takes their definition instead
 * and diagonalises by cyclic Jacobi rotations (Golub & Van Loan, Matrix
 * Computations, Sec. 8.5) until the off-diagonal part is below 1e-18 of the
 * matrix norm, which is accurate to a few ulps of |S| also where two
 * eigenvalues nearly coincide (the trigonometric closed form there loses half
 * the digits).  S is row-major d x d. */
void orc_eigvals(int dim, const double *S, double *lam) {
    double A[3][3] = {{0}};
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) A[a][b] = 0.5 * (S[a * dim + b] + S[b * dim + a]);
    double norm2 = 0.0;
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) norm2 += A[a][b] * A[a][b];
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off2 = 0.0;
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b)
                if (a != b) off2 += A[a][b] * A[a][b];
        if (off2 <= 1e-36 * norm2) break;
        for (int p = 0; p < dim; ++p)
            for (int q = p + 1; q < dim; ++q) {
                if (A[p][q] == 0.0) continue;
                /* rotation J (J_pp = J_qq = c, J_pq = s, J_qp = -s) with
                 * (J^T A J)_pq = 0 */
                double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = tau >= 0.0 ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                      : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                double J[3][3] = {{0}};
                for (int k = 0; k < dim; ++k) J[k][k] = 1.0;
                J[p][p] = c;
                J[q][q] = c;
                J[p][q] = s;
                J[q][p] = -s;
                double AJ[3][3] = {{0}}, B[3][3] = {{0}};
                for (int a = 0; a < dim; ++a)
                    for (int b = 0; b < dim; ++b)
                        for (int k = 0; k < dim; ++k) AJ[a][b] += A[a][k] * J[k][b];
                for (int a = 0; a < dim; ++a)
                    for (int b = 0; b < dim; ++b)
                        for (int k = 0; k < dim; ++k) B[a][b] += J[k][a] * AJ[k][b];
                B[p][q] = B[q][p] = 0.0;
                for (int a = 0; a < dim; ++a)
                    for (int b = 0; b < dim; ++b) A[a][b] = 0.5 * (B[a][b] + B[b][a]);
            }
    }
    double e[3] = {A[0][0], A[1][1], dim == 3 ? A[2][2] : 0.0};
    for (int i = 0; i < dim; ++i)
        for (int j = i + 1; j < dim; ++j)
            if (e[j] < e[i]) {
                double tmp = e[i];
                e[i] = e[j];
                e[j] = tmp;
            }
    lam[0] = e[0];
    lam[1] = e[1];
    lam[2] = dim == 3 ? e[2] : 0.0;
}

static double det_d(int dim, const double *M) {
    if (dim == 2) return M[0] * M[3] - M[1] * M[2];
    return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
           M[2] * (M[3] * M[7] - M[4] * M[6]);
}

/* Solves L^T y = v by the adjugate of L^T (Sec. 3: the correction moved
 * outside the sum leaves one small linear system per particle). */
static void solve_LT(int dim, const double *L, const double *v, double *y) {
    double M[9] = {0};
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) M[a * dim + b] = L[b * dim + a];
    double det = det_d(dim, M);
    if (dim == 2) {
        y[0] = (M[3] * v[0] - M[1] * v[1]) / det;
        y[1] = (-M[2] * v[0] + M[0] * v[1]) / det;
        return;
    }
    double inv[9];
    inv[0] = M[4] * M[8] - M[5] * M[7];
    inv[1] = M[2] * M[7] - M[1] * M[8];
    inv[2] = M[1] * M[5] - M[2] * M[4];
    inv[3] = M[5] * M[6] - M[3] * M[8];
    inv[4] = M[0] * M[8] - M[2] * M[6];
    inv[5] = M[2] * M[3] - M[0] * M[5];
    inv[6] = M[3] * M[7] - M[4] * M[6];
    inv[7] = M[1] * M[6] - M[0] * M[7];
    inv[8] = M[0] * M[4] - M[1] * M[3];
    for (int a = 0; a < 3; ++a) y[a] = (inv[a * 3 + 0] * v[0] + inv[a * 3 + 1] * v[1] + inv[a * 3 + 2] * v[2]) / det;
}

/* L^{-1} in full (for the corrected divergence tr(L^{-1} N)). */
static void inverse_d(int dim, const double *L, double *Li) {
    double det = det_d(dim, L);
    if (dim == 2) {
        Li[0] = L[3] / det;
        Li[1] = -L[1] / det;
        Li[2] = -L[2] / det;
        Li[3] = L[0] / det;
        return;
    }
    Li[0] = (L[4] * L[8] - L[5] * L[7]) / det;
    Li[1] = (L[2] * L[7] - L[1] * L[8]) / det;
    Li[2] = (L[1] * L[5] - L[2] * L[4]) / det;
    Li[3] = (L[5] * L[6] - L[3] * L[8]) / det;
    Li[4] = (L[0] * L[8] - L[2] * L[6]) / det;
    Li[5] = (L[2] * L[3] - L[0] * L[5]) / det;
    Li[6] = (L[3] * L[7] - L[4] * L[6]) / det;
    Li[7] = (L[1] * L[6] - L[0] * L[7]) / det;
    Li[8] = (L[0] * L[4] - L[1] * L[3]) / det;
}

/* ------------------------------------------------------------ one RHS */

/* rho = rho0 exp(phi / C0^2) (Sec. 2.2.1); V = m / rho. */
static double volume_of(const orc_params *p, double m, double phi) {
    return m / (p->rho0 * exp(phi / (p->c0 * p->c0)));
}

/* Mirror for the dummy wall particles (Sec. 2.4): nearest fluid particle f
 * within 2h (ties -> lower index); phi_d = phi_f + G.(x_d - x_f) (Eq. phiBn);
 * slip velocity U_d = U_f - (U_f.n_d) n_d.  No fluid within 2h -> inactive.
 * Reading for a moving body (kind 2, wall velocity Uw): the slip condition
 * holds relative to the wall, U_d = U_f - ((U_f - Uw).n_d) n_d, so that the
 * dummy carries the wall's normal velocity and the fluid's tangential one
 * (Sec. 2.4 gives the no-slip form 2 Uw - U_f with the wall velocity, and
 * the slip form for fixed walls); Eq. (phiBn) is kept as printed. */
static void mirror_dummies(const orc_params *p, int64_t n, const double *x, const double *u,
                           const double *phi, const uint8_t *kind, const double *nd, const double *G,
                           const double *Uw, const int64_t *off, const int32_t *ids, double *mphi,
                           double *mu, int32_t *msrc) {
    /* nd: unit normals of every row; Uw: wall velocity of every row (used
     * for kind 2) */
    int dim = p->dim;
#pragma omp parallel for schedule(static)
    for (int64_t d = 0; d < n; ++d) {
        if (kind[d] == 0) continue;
        int64_t best = -1;
        double bestr2 = 0.0;
        for (int64_t k = off[d]; k < off[d + 1]; ++k) {
            int64_t f = ids[k];
            if (kind[f] != 0) continue;
            double r2 = dist2(dim, x + d * dim, x + f * dim);
            if (best < 0 || r2 < bestr2 || (r2 == bestr2 && f < best)) {
                best = f;
                bestr2 = r2;
            }
        }
        msrc[d] = (int32_t)best;
        if (best < 0) {
            mphi[d] = phi[d];
            for (int a = 0; a < dim; ++a) mu[d * dim + a] = 0.0;
            continue;
        }
        double gp = 0.0;
        for (int a = 0; a < dim; ++a) gp += G[a] * (x[d * dim + a] - x[best * dim + a]);
        mphi[d] = phi[best] + gp;
        double un = 0.0;
        for (int a = 0; a < dim; ++a) {
            double rel = u[best * dim + a] - (kind[d] == 2 ? Uw[d * dim + a] : 0.0);
            un += rel * nd[d * dim + a];
        }
        for (int a = 0; a < dim; ++a) mu[d * dim + a] = u[best * dim + a] - un * nd[d * dim + a];
    }
}

/* Scan-region free-surface test for a candidate (lambda in (lo, hi]): i is
 * NOT on the free surface iff a neighbour j lies in the umbrella-shaped scan
 * region around T = x_i + h n.  Returns 1 for free surface; *margin receives
 * the smallest distance of any tested quantity to its threshold. */
static int scan_region(const orc_params *p, int64_t i, const double *x, const double *nrm,
                       const int64_t *off, const int32_t *ids, double *margin) {
    int dim = p->dim;
    double h = p->h;
    double T[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) T[a] = x[i * dim + a] + h * nrm[a];
    double mg = INFINITY;
    for (int64_t k = off[i]; k < off[i + 1]; ++k) {
        int64_t j = ids[k];
        double s2 = dist2(dim, x + i * dim, x + j * dim);
        double dT[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) dT[a] = x[j * dim + a] - T[a];
        double m1 = fabs(s2 - 2.0 * h * h);
        if (m1 < mg) mg = m1;
        if (s2 >= 2.0 * h * h) {
            double d2 = 0.0;
            for (int a = 0; a < dim; ++a) d2 += dT[a] * dT[a];
            double m2 = fabs(d2 - h * h);
            if (m2 < mg) mg = m2;
            if (d2 < h * h) {
                *margin = mg;
                return 0;
            }
        } else {
            double dn = 0.0;
            for (int a = 0; a < dim; ++a) dn += nrm[a] * dT[a];
            double tt = 0.0;
            for (int a = 0; a < dim; ++a) {
                double c = dT[a] - dn * nrm[a];
                tt += c * c;
            }
            double val = fabs(dn) + sqrt(tt);
            double m2 = fabs(val - h) * h;
            if (m2 < mg) mg = m2;
            if (val < h) {
                *margin = mg;
                return 0;
            }
        }
    }
    *margin = mg;
    return 1;
}

/* One evaluation of the semi-discrete system, Eq. (sph), at time t.  With
 * only != NULL the rates are computed for the fluid particles with only[i]
 * != 0 alone (the others are left zero), from neighbour lists of those
 * particles, of the dummies among their neighbours and, with a free body, of
 * all of its dummies (cells mode).  Rows of kind 2 (the moving body) hold the
 * body at T_0 (prescribed motion; they take part at x + D(t)) or in its
 * reference pose (free body; placed from its state). */
int orc_eval_rates(const orc_params *p, int64_t n, const double *x_in, const double *u,
                   const double *phi, const double *mass, const uint8_t *kind, const double *nd_in,
                   double t, int nbr_mode, const uint8_t *only, orc_rates *out, const orc_body *body) {
    int dim = p->dim;
    if (dim != 2 && dim != 3) return ORC_EINVAL;
    if (only && nbr_mode == 0) return ORC_EINVAL;
    if (p->body_free && (!body || !(p->body_mass > 0.0))) return ORC_EINVAL;
    /* kind-2 rows at the time t: the prescribed motion's translation, or
     * the free body's pose (positions, rotated normals, wall velocities) */
    double Db[3], Ub[3];
    orc_body_motion(p, t, Db, Ub);
    size_t nn_ = (size_t)(n > 0 ? n : 1);
    double *xw = (double *)malloc(sizeof(double) * nn_ * dim);
    double *ndw = (double *)malloc(sizeof(double) * nn_ * dim);
    double *uww = (double *)malloc(sizeof(double) * nn_ * dim);
    if (!xw || !ndw || !uww) {
        free(xw); free(ndw); free(uww);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (kind[i] == 2 && p->body_free) {
            free_body_place(p, body, x_in + i * dim, nd_in + i * dim, xw + i * dim, ndw + i * dim, uww + i * dim);
            continue;
        }
        for (int a = 0; a < dim; ++a) {
            xw[i * dim + a] = x_in[i * dim + a] + (kind[i] == 2 ? Db[a] : 0.0);
            ndw[i * dim + a] = nd_in[i * dim + a];
            uww[i * dim + a] = kind[i] == 2 ? Ub[a] : 0.0;
        }
    }
    const double *x = xw;
    const double *nd = ndw;
    int64_t *off = NULL;
    int32_t *ids = NULL;
    int st;
    if (!only) {
        st = build_csr(p, n, x, nbr_mode, &off, &ids);
    } else {
        /* rows: the sampled fluid particles, then also the dummies in their
         * neighbour lists (the wall mirror needs their lists) */
        uint8_t *rows = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
        if (!rows) {
            free(xw); free(ndw); free(uww);
            return ORC_ENOMEM;
        }
        for (int64_t i = 0; i < n; ++i) rows[i] = (uint8_t)(only[i] && kind[i] == 0);
        st = build_csr_rows(p, n, x, rows, &off, &ids);
        if (st == ORC_OK) {
            for (int64_t i = 0; i < n; ++i) {
                if (!(only[i] && kind[i] == 0)) continue;
                for (int64_t k = off[i]; k < off[i + 1]; ++k)
                    if (kind[ids[k]] != 0) rows[ids[k]] = 1;
            }
            /* the free body's force and torque sum over all of its dummies:
             * each needs its own list (mirror source and fluid neighbours) */
            if (p->body_free)
                for (int64_t i = 0; i < n; ++i)
                    if (kind[i] == 2) rows[i] = 1;
            free(off);
            free(ids);
            off = NULL;
            ids = NULL;
            st = build_csr_rows(p, n, x, rows, &off, &ids);
        }
        free(rows);
    }
    if (st != ORC_OK) {
        free(xw); free(ndw); free(uww);
        return st;
    }

    double G[3];
    body_force(p, t, G);
    const double h = p->h, c0 = p->c0;

    /* walls: mirrored potential and velocity */
    double *phiv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *uv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * dim);
    double *V = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!phiv || !uv || !V || !src) {
        free(off); free(ids); free(phiv); free(uv); free(V); free(src); free(xw); free(ndw); free(uww);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) src[i] = -1;
    memcpy(phiv, phi, sizeof(double) * (size_t)n);
    memcpy(uv, u, sizeof(double) * (size_t)n * dim);
    mirror_dummies(p, n, x, u, phi, kind, nd, G, uww, off, ids, phiv, uv, src);
    for (int64_t i = 0; i < n; ++i) {
        if (kind[i] != 0 && src[i] < 0) V[i] = 0.0;
        else V[i] = volume_of(p, mass[i], phiv[i]);
    }

    /* U_max over fluid, used by the shifting velocity scale */
    double umax2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (kind[i] != 0) continue;
        double s = 0.0;
        for (int a = 0; a < dim; ++a) s += u[i * dim + a] * u[i * dim + a];
        if (s > umax2) umax2 = s;
    }
    const double umax = sqrt(umax2);
    const double W0 = orc_W(dim, h, p->dx / h); /* W(dx) for the PST weight */
    double nsing = 0.0;

#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nsing)
    for (int64_t i = 0; i < n; ++i) {
        double *acc = out->acc + i * dim;
        double *dus = out->dushift + i * dim;
        double *nrm = out->normal + i * dim;
        double *lam = out->lam + i * 3;
        double *ft = out->feat + i * NFEAT;
        for (int a = 0; a < dim; ++a) acc[a] = dus[a] = nrm[a] = 0.0;
        lam[0] = lam[1] = lam[2] = 0.0;
        for (int f = 0; f < NFEAT; ++f) ft[f] = 0.0;
        out->dphi[i] = 0.0;
        out->fs[i] = 0;
        out->tic[i] = 0;
        out->fs_margin[i] = INFINITY;
        out->nnb[i] = (int32_t)(off[i + 1] - off[i]);
        out->mir_phi[i] = phiv[i];
        for (int a = 0; a < dim; ++a) out->mir_u[i * dim + a] = uv[i * dim + a];
        out->mir_src[i] = src[i];
        if (kind[i] != 0 || (only && !only[i])) continue;

        /* pair sums over N(i), Algorithm 1 / Eq. (sph) */
        double L[9] = {0}, g[3] = {0}, SR[3] = {0}, SC[3] = {0}, Nm[9] = {0}, P[3] = {0};
        double Dsum = 0.0;
        const double *xi = x + i * dim, *ui = uv + i * dim;
        const double phii = phiv[i];
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            int64_t j = ids[k];
            const double *xj = x + j * dim, *uj = uv + j * dim;
            double r[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) r[a] = xj[a] - xi[a];
            double s = sqrt(dist2(dim, xi, xj));
            double q = s / h;
            double Kq = orc_K(dim, h, q);
            double Wq = orc_W(dim, h, q);
            double Vj = V[j];
            double gw[3] = {0, 0, 0}; /* grad_i W_ij */
            for (int a = 0; a < dim; ++a) gw[a] = Kq * r[a];
            /* renormalisation matrix, Eq. (renorm): L_ab += r_a (grad W)_b V_j */
            for (int a = 0; a < dim; ++a)
                for (int b = 0; b < dim; ++b) L[a * dim + b] += r[a] * gw[b] * Vj;
            for (int a = 0; a < dim; ++a) g[a] += gw[a] * Vj;
            /* Lax-Friedrichs interface potential, Eq. (lfsover):
             * 2(phi*_ij - phi_i) = (phi_j - phi_i) - C0 (U_j,n - U_i,n) */
            double du[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) du[a] = uj[a] - ui[a];
            double dun = 0.0;
            for (int a = 0; a < dim; ++a) dun += du[a] * r[a];
            dun = dun / s;
            double twophi = (phiv[j] - phii) - c0 * dun;
            for (int a = 0; a < dim; ++a) SR[a] += twophi * gw[a] * Vj;
            /* conservative form used by the tensile-instability switch */
            for (int a = 0; a < dim; ++a) SC[a] += (phiv[j] + phii) * gw[a] * Vj;
            /* velocity-gradient tensor for the continuity equation */
            for (int a = 0; a < dim; ++a)
                for (int b = 0; b < dim; ++b) Nm[a * dim + b] += du[a] * gw[b] * Vj;
            /* delta-SPH: Phi_ij . grad W = 2 (phi_j - phi_i) (r . grad W) / |r|^2 */
            double rg = 0.0;
            for (int a = 0; a < dim; ++a) rg += r[a] * gw[a];
            Dsum += 2.0 * (phiv[j] - phii) * rg / (s * s) * Vj;
            /* particle shifting weight [1 + R (W / W(dx))^n] */
            double wr = Wq / W0;
            double pw = 1.0 + p->pst_R * pow(wr, p->pst_n);
            for (int a = 0; a < dim; ++a) P[a] += pw * gw[a] * Vj;
        }

        /* eigenvalues of the (symmetric) correction matrix */
        orc_eigvals(dim, L, lam);
        const double lmin = lam[0];
        int singular = lmin <= p->lambda_singular;
        int tic_on = (p->flags & ORC_TIC) && lmin < p->lambda_tic;
        int cons = singular || tic_on;
        out->tic[i] = cons;
        if (singular) nsing += 1.0;

        /* momentum, Eq. (sph): a = -L^{-T} S_R + G, or -S_C + G (TIC branch) */
        double grad[3] = {0, 0, 0};
        if (cons) {
            for (int a = 0; a < dim; ++a) grad[a] = SC[a];
        } else {
            solve_LT(dim, L, SR, grad);
        }
        for (int a = 0; a < dim; ++a) acc[a] = -grad[a] + G[a];

        /* continuity, Eq. (sph): -C0^2 sum (U_j-U_i).L^{-T} grad W V_j
         * = -C0^2 tr(L^{-1} N) */
        double div = 0.0;
        int uncorr = singular || (tic_on && (p->flags & ORC_CONT_UNCORR));
        if (uncorr) {
            for (int a = 0; a < dim; ++a) div += Nm[a * dim + a];
        } else {
            double Li[9];
            inverse_d(dim, L, Li);
            for (int a = 0; a < dim; ++a)
                for (int b = 0; b < dim; ++b) div += Li[a * dim + b] * Nm[b * dim + a];
        }
        double dphi = -c0 * c0 * div;
        if (p->flags & ORC_DELTA) dphi += p->delta * h * c0 * Dsum;
        out->dphi[i] = dphi;

        /* free-surface normal n = -L^{-T} g / |.|  (-g / |g| if L singular) */
        double ng[3] = {0, 0, 0};
        if (singular) {
            for (int a = 0; a < dim; ++a) ng[a] = -g[a];
        } else {
            solve_LT(dim, L, g, ng);
            for (int a = 0; a < dim; ++a) ng[a] = -ng[a];
        }
        double nn = 0.0;
        for (int a = 0; a < dim; ++a) nn += ng[a] * ng[a];
        nn = sqrt(nn);
        if (nn > 0.0)
            for (int a = 0; a < dim; ++a) nrm[a] = ng[a] / nn;

        /* particle shifting: dU* = -2 h U_max P, clamped to U_max / 2 */
        if (p->flags & ORC_PST) {
            double dstar[3] = {0, 0, 0}, dn2 = 0.0;
            for (int a = 0; a < dim; ++a) {
                dstar[a] = -2.0 * h * umax * P[a];
                dn2 += dstar[a] * dstar[a];
            }
            double dnrm = sqrt(dn2);
            if (dnrm > 0.0) {
                double mag = dnrm < 0.5 * umax ? dnrm : 0.5 * umax;
                for (int a = 0; a < dim; ++a) dus[a] = mag * dstar[a] / dnrm;
            }
        }

        /* features (16), all from the sums above: eigenvalues of L, det L,
         * the shifting sum P along the normal n, neighbour count, |g| h, the
         * moments of the kernel-gradient sum g and of L along n and across
         * it, |L^-T g| h, n against gravity, P across n, the cosine between
         * P and n, |P| h */
        {
            double ng = 0.0, gn2 = 0.0, nLn = 0.0, trL = 0.0, Pn2 = 0.0, ngrav = 0.0, gg2 = 0.0, nP = 0.0;
            for (int a = 0; a < dim; ++a) {
                ng += nrm[a] * g[a];
                gn2 += g[a] * g[a];
                trL += L[a * dim + a];
                Pn2 += P[a] * P[a];
                nP += nrm[a] * P[a];
                ngrav += nrm[a] * G[a];
                gg2 += G[a] * G[a];
                for (int b = 0; b < dim; ++b) nLn += nrm[a] * L[a * dim + b] * nrm[b];
            }
            double gt2 = 0.0, Pt2 = 0.0; /* tangential parts by components */
            for (int a = 0; a < dim; ++a) {
                double tg = g[a] - ng * nrm[a], tp = P[a] - nP * nrm[a];
                gt2 += tg * tg;
                Pt2 += tp * tp;
            }
            int cnt = (int)(off[i + 1] - off[i]);
            double Pm = sqrt(Pn2);
            ft[0] = lam[0];
            ft[1] = lam[1];
            ft[2] = dim == 3 ? lam[2] : lam[1];
            ft[3] = det_d(dim, L);
            ft[4] = nP * h;
            ft[5] = (double)cnt;
            ft[6] = sqrt(gn2) * h;
            ft[7] = ng * h;
            ft[8] = sqrt(gt2) * h;
            ft[9] = nLn;
            ft[10] = trL - nLn;
            ft[11] = nn * h;
            ft[12] = gg2 > 0.0 ? ngrav / sqrt(gg2) : 0.0;
            ft[13] = sqrt(Pt2) * h;
            ft[14] = Pm > 0.0 ? nP / Pm : 0.0;
            ft[15] = Pm * h;
        }
    }

    /* free-surface detection: lambda <= lo -> surface; lambda > hi -> not;
     * otherwise the scan-region test around x_i + h n. */
    if (p->fs_mode == ORC_FS_EXACT) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            if (kind[i] != 0 || (only && !only[i])) continue;
            double lmin = out->lam[i * 3];
            double nn = 0.0;
            for (int a = 0; a < dim; ++a) nn += out->normal[i * dim + a] * out->normal[i * dim + a];
            int fs;
            if (lmin <= p->lambda_fs_lo) fs = 1;
            else if (lmin > p->lambda_fs_hi) fs = 0;
            else if (nn == 0.0) fs = 1;
            else fs = scan_region(p, i, x, out->normal + i * dim, off, ids, &out->fs_margin[i]);
            out->fs[i] = fs;
            /* shifting at the surface: keep only the tangential part */
            if (fs && (p->flags & ORC_FS_PROJECT) && (p->flags & ORC_PST)) {
                double *dus = out->dushift + i * dim;
                const double *nr = out->normal + i * dim;
                double dn = 0.0;
                for (int a = 0; a < dim; ++a) dn += dus[a] * nr[a];
                for (int a = 0; a < dim; ++a) dus[a] -= dn * nr[a];
            }
        }
    }

    if (out->scal) {
        out->scal[0] = umax;
        out->scal[1] = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
        out->scal[2] = t;
        out->scal[3] = nsing;
        for (int a = 4; a < 10; ++a) out->scal[a] = 0.0;
    }

    /* Force and torque of the water on the free body.  Reading (the paper
     * says the cylinder falls under gravity and the interaction force with
     * the water, not how that force is formed): each dummy of the body gets
     * the acceleration Eq. (sph) gives a particle with a truncated support,
     * the conservative form (Sec. 2.3, the branch for lambda_min < 0.75),
     * from its fluid neighbours, a_d = -sum_i (phi_i + phi_d) grad_d W_di V_i,
     * with its mirrored potential; the body's force is sum_d m_d a_d and its
     * torque about the centre sum_d (x_d - c) x m_d a_d.  The dummies' forces
     * on one another are internal to the rigid body; fixed walls do not act
     * on it.  Summed in ascending row order. */
    if (p->body_free && out->scal) {
        double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
        for (int64_t d = 0; d < n; ++d) {
            if (kind[d] != 2 || src[d] < 0) continue;
            double ad[3] = {0, 0, 0};
            for (int64_t k = off[d]; k < off[d + 1]; ++k) {
                int64_t i = ids[k];
                if (kind[i] != 0) continue;
                double r[3] = {0, 0, 0};
                for (int a = 0; a < dim; ++a) r[a] = x[i * dim + a] - x[d * dim + a];
                double q = sqrt(dist2(dim, x + d * dim, x + i * dim)) / h;
                double Kq = orc_K(dim, h, q); /* grad_d W_di = K (x_i - x_d) */
                for (int a = 0; a < dim; ++a) ad[a] -= (phiv[i] + phiv[d]) * Kq * r[a] * V[i];
            }
            double fd[3] = {0, 0, 0}, arm[3] = {0, 0, 0}, td[3];
            for (int a = 0; a < dim; ++a) {
                fd[a] = mass[d] * ad[a];
                arm[a] = x[d * dim + a] - body->c[a];
                F[a] += fd[a];
            }
            cross3(arm, fd, td);
            for (int a = 0; a < 3; ++a) T[a] += td[a];
        }
        for (int a = 0; a < 3; ++a) {
            out->scal[4 + a] = F[a];
            out->scal[7 + a] = T[a];
        }
    }
    free(off); free(ids); free(phiv); free(uv); free(V); free(src); free(xw); free(ndw); free(uww);
    return ORC_OK;
}

/* ------------------------------------------------------------ stepping */

/* Time step rule (Sec. 2.3): CFL * min(dx/(C0+|U|max), dx^2/(2 nu),
 * sqrt(2 dx / |G|)); a zero viscosity or force drops its term. */
double orc_dt(const orc_params *p, int64_t n, const double *u, const uint8_t *kind) {
    int dim = p->dim;
    double umax2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (kind[i] != 0) continue;
        double s = 0.0;
        for (int a = 0; a < dim; ++a) s += u[i * dim + a] * u[i * dim + a];
        if (s > umax2) umax2 = s;
    }
    double dt = p->dx / (p->c0 + sqrt(umax2));
    if (p->nu > 0.0) {
        double dd = p->dx * p->dx / (2.0 * p->nu);
        if (dd < dt) dt = dd;
    }
    double gm = body_force_max(p);
    if (gm > 0.0) {
        double dg = sqrt(2.0 * p->dx / gm);
        if (dg < dt) dt = dg;
    }
    return p->cfl * dt;
}

static int alloc_rates(orc_rates *r, int64_t n, int dim) {
    size_t nn = (size_t)(n > 0 ? n : 1);
    memset(r, 0, sizeof(*r));
    r->acc = (double *)malloc(sizeof(double) * nn * dim);
    r->dphi = (double *)malloc(sizeof(double) * nn);
    r->dushift = (double *)malloc(sizeof(double) * nn * dim);
    r->lam = (double *)malloc(sizeof(double) * nn * 3);
    r->normal = (double *)malloc(sizeof(double) * nn * dim);
    r->fs = (int32_t *)malloc(sizeof(int32_t) * nn);
    r->tic = (int32_t *)malloc(sizeof(int32_t) * nn);
    r->nnb = (int32_t *)malloc(sizeof(int32_t) * nn);
    r->feat = (double *)malloc(sizeof(double) * nn * NFEAT);
    r->fs_margin = (double *)malloc(sizeof(double) * nn);
    r->mir_phi = (double *)malloc(sizeof(double) * nn);
    r->mir_u = (double *)malloc(sizeof(double) * nn * dim);
    r->mir_src = (int32_t *)malloc(sizeof(int32_t) * nn);
    r->scal = NULL;
    if (!r->acc || !r->dphi || !r->dushift || !r->lam || !r->normal || !r->fs || !r->tic || !r->nnb ||
        !r->feat || !r->fs_margin || !r->mir_phi || !r->mir_u || !r->mir_src)
        return ORC_ENOMEM;
    return ORC_OK;
}

static void free_rates(orc_rates *r) {
    free(r->acc); free(r->dphi); free(r->dushift); free(r->lam); free(r->normal);
    free(r->fs); free(r->tic); free(r->nnb); free(r->feat); free(r->fs_margin);
    free(r->mir_phi); free(r->mir_u); free(r->mir_src);
    memset(r, 0, sizeof(*r));
}

/* Rates of the free body's state: dc/dt = v; dv/dt = F/M + G; dq/dt =
 * (0, w) q / 2; dw/dt = I_w^-1 (T - w x I_w w) with I_w = R I_b R^T, the
 * inertia tensor in the world frame (Euler's equations).  In 2D the body
 * moves in the plane and turns about z only. */
static void free_body_rates(const orc_params *p, const orc_body *b, const double F[3], const double T[3],
                            const double G[3], orc_body *rate) {
    int dim = p->dim;
    const double *Ib = p->body_inertia;
    double Bm[9] = {Ib[0], Ib[3], Ib[4], Ib[3], Ib[1], Ib[5], Ib[4], Ib[5], Ib[2]};
    double R[9], RB[9], Iw[9];
    quat_matrix(b->q, R);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += R[3 * i + k] * Bm[3 * k + j];
            RB[3 * i + j] = acc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += RB[3 * i + k] * R[3 * j + k];
            Iw[3 * i + j] = acc;
        }
    double Lw[3], gyro[3], rhs[3];
    for (int a = 0; a < 3; ++a) Lw[a] = Iw[3 * a] * b->w[0] + Iw[3 * a + 1] * b->w[1] + Iw[3 * a + 2] * b->w[2];
    cross3(b->w, Lw, gyro);
    for (int a = 0; a < 3; ++a) rhs[a] = T[a] - gyro[a];
    for (int a = 0; a < 3; ++a) {
        rate->c[a] = b->v[a];
        rate->v[a] = F[a] / p->body_mass + G[a];
    }
    if (dim == 2) {
        rate->c[2] = rate->v[2] = rate->w[0] = rate->w[1] = 0.0;
        rate->w[2] = rhs[2] / Iw[8];
    } else {
        double Ii[9];
        inverse_d(3, Iw, Ii);
        for (int a = 0; a < 3; ++a) rate->w[a] = Ii[3 * a] * rhs[0] + Ii[3 * a + 1] * rhs[1] + Ii[3 * a + 2] * rhs[2];
    }
    /* (0, w) * q, Hamilton product */
    const double *q = b->q, *w = b->w;
    rate->q[0] = 0.5 * (-w[0] * q[1] - w[1] * q[2] - w[2] * q[3]);
    rate->q[1] = 0.5 * (w[0] * q[0] + w[1] * q[3] - w[2] * q[2]);
    rate->q[2] = 0.5 * (-w[0] * q[3] + w[1] * q[0] + w[2] * q[1]);
    rate->q[3] = 0.5 * (w[0] * q[2] - w[1] * q[1] + w[2] * q[0]);
}

static void quat_normalise(double q[4]) {
    double s = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int a = 0; a < 4; ++a) q[a] /= s;
}

/* SSP-RK2 (Sec. 2.3).  dt from U at t^n (dt_override > 0 replaces the
 * rule).  Stage 1 at t^n, stage 2 at t^n + dt (the body, kind 2, at its
 * positions of those times).  On return x, u, phi hold t^{n+nsteps} (dummy
 * rows untouched); *t advanced; *dt_last set.  A free body (body_free)
 * advances with the same two stages, its force and torque taken at each
 * right-hand side; its quaternion is renormalised after each stage. */
int orc_step(const orc_params *p, int64_t n, double *x, double *u, double *phi, const double *mass,
             const uint8_t *kind, const double *nd, double *t, int32_t nsteps, double dt_override,
             int nbr_mode, double *dt_last, orc_body *body) {
    int dim = p->dim;
    if (p->body_free && !body) return ORC_EINVAL;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *x0 = (double *)malloc(sizeof(double) * nn * dim);
    double *u0 = (double *)malloc(sizeof(double) * nn * dim);
    double *p0 = (double *)malloc(sizeof(double) * nn);
    double scal[10];
    orc_rates r;
    int st = alloc_rates(&r, n, dim);
    r.scal = scal;
    if (!x0 || !u0 || !p0 || st != ORC_OK) {
        free(x0); free(u0); free(p0); r.scal = NULL; free_rates(&r);
        return ORC_ENOMEM;
    }
    orc_body b0, b1, rt;
    for (int32_t s = 0; s < nsteps && st == ORC_OK; ++s) {
        double dt = dt_override > 0.0 ? dt_override : orc_dt(p, n, u, kind);
        memcpy(x0, x, sizeof(double) * nn * dim);
        memcpy(u0, u, sizeof(double) * nn * dim);
        memcpy(p0, phi, sizeof(double) * n);
        double G[3];
        /* first stage */
        st = orc_eval_rates(p, n, x, u, phi, mass, kind, nd, *t, nbr_mode, NULL, &r, body);
        if (st != ORC_OK) break;
        for (int64_t i = 0; i < n; ++i) {
            if (kind[i] != 0) continue;
            phi[i] = p0[i] + dt * r.dphi[i];
            for (int a = 0; a < dim; ++a) {
                u[i * dim + a] = u0[i * dim + a] + dt * r.acc[i * dim + a];
                x[i * dim + a] = x0[i * dim + a] + dt * (u0[i * dim + a] + r.dushift[i * dim + a]);
            }
        }
        if (p->body_free) {
            b0 = *body;
            body_force(p, *t, G);
            free_body_rates(p, &b0, scal + 4, scal + 7, G, &rt);
            for (int a = 0; a < 3; ++a) {
                b1.c[a] = b0.c[a] + dt * rt.c[a];
                b1.v[a] = b0.v[a] + dt * rt.v[a];
                b1.w[a] = b0.w[a] + dt * rt.w[a];
            }
            for (int a = 0; a < 4; ++a) b1.q[a] = b0.q[a] + dt * rt.q[a];
            quat_normalise(b1.q);
            *body = b1;
        }
        /* second stage */
        st = orc_eval_rates(p, n, x, u, phi, mass, kind, nd, *t + dt, nbr_mode, NULL, &r, body);
        if (st != ORC_OK) break;
        for (int64_t i = 0; i < n; ++i) {
            if (kind[i] != 0) continue;
            phi[i] = 0.5 * p0[i] + 0.5 * (phi[i] + dt * r.dphi[i]);
            for (int a = 0; a < dim; ++a) {
                double u1 = u[i * dim + a];
                u[i * dim + a] = 0.5 * u0[i * dim + a] + 0.5 * (u1 + dt * r.acc[i * dim + a]);
                x[i * dim + a] = 0.5 * x0[i * dim + a] +
                                 0.5 * (x[i * dim + a] + dt * (u1 + r.dushift[i * dim + a]));
            }
        }
        if (p->body_free) {
            body_force(p, *t + dt, G);
            free_body_rates(p, &b1, scal + 4, scal + 7, G, &rt);
            for (int a = 0; a < 3; ++a) {
                body->c[a] = 0.5 * b0.c[a] + 0.5 * (b1.c[a] + dt * rt.c[a]);
                body->v[a] = 0.5 * b0.v[a] + 0.5 * (b1.v[a] + dt * rt.v[a]);
                body->w[a] = 0.5 * b0.w[a] + 0.5 * (b1.w[a] + dt * rt.w[a]);
            }
            for (int a = 0; a < 4; ++a) body->q[a] = 0.5 * b0.q[a] + 0.5 * (b1.q[a] + dt * rt.q[a]);
            quat_normalise(body->q);
        }
        *t = *t + dt;
        if (dt_last) *dt_last = dt;
    }
    free(x0); free(u0); free(p0); r.scal = NULL; free_rates(&r);
    return st;
}

/* Threads OpenMP would use (reported by the CPU baseline). */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int k) {
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

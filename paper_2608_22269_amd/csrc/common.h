// Internal declarations of the gfx950 WCSPH library: device-side parameter
// blocks, the particle layout in HBM, small device math shared by the kernels
// (kernel function, cell geometry, the cell-row walker of Algorithm 1, the
// closed-form symmetric eigenvalues and the small linear solves).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "wbsph.h"

namespace wb {

constexpr int kBlock = 256;   // threads per block for streaming kernels
// padding records after the FP64 neighbour records: candidate loads are
// issued in batches and may run this many records past a run's end
constexpr int kRecPad = 8;
constexpr int kNFeat = 16;    // classifier features per particle
constexpr int kMaxReach = 3;  // cells searched each side: ceil(2h / R) <= 3
// Tag bit of a candidate-list entry kept for the second stage of a step that
// is not a neighbour at the first (record indices stay below 2^31).
constexpr uint32_t kSkinTag = 0x80000000u;
// LDS list entries per lane of the pair passes; candidate lists kept from the
// first stage to the second: chunks (one LDS list fill) per lane.
constexpr int kPairList = 32;
constexpr int kKeepChunks = 8;
static_assert(kPairList % 8 == 0 && kPairList <= 255, "kept chunks are staged eight entries at a time");

// error bits accumulated on the device
enum : uint32_t {
  kErrDomain = 1u,
  kErrNonFinite = 2u,
  kErrCapacity = 4u,
};

// per-particle flag bits (fluid, sorted order)
enum : uint32_t {
  kFlagCons = 1u,       // conservative (TIC / singular) branch used
  kFlagFS = 2u,         // free surface
  kFlagCand = 4u,       // 0.2 < lambda <= 0.75: decided by scan or MLP
  kFlagSingular = 8u,   // lambda_min <= lambda_singular
  kFlagByScan = 16u,    // decided by the scan-region pass
  kFlagByMLP = 32u,     // decided by the classifier
};

// Background grid (Sec. 3): N_a = floor((hi - lo) / R) + 1 cells per axis.
//
// Storage order of the cells.  The paper orders particles by HashID = i_x +
// i_y N_x + i_z N_x N_y; a particle's z-neighbours then sit a whole cell layer
// away.  The sort key used here groups the x-rows into tiles of B_y x B_z rows
// (whole x-rows, so every row stays one contiguous run) and ranks the tiles
// along a Morton curve:
//   key = rank(y / B_y, z / B_z) * N_x B_y B_z + x + (y mod B_y) N_x
//         + (z mod B_z) N_x B_y.
// B_y = B_z = 0 is the paper's linear order.  Cell coordinates, HashID and the
// neighbour sets do not depend on it; only the storage and visiting order do.
#ifndef WB_TILE_Y
#define WB_TILE_Y 8
#endif
#ifndef WB_TILE_Z
#define WB_TILE_Z 8
#endif
#ifndef WB_XCD_REMAP
#define WB_XCD_REMAP 1
#endif
constexpr int kTileY = WB_TILE_Y, kTileZ = WB_TILE_Z;  // powers of two (or 0)
constexpr bool kLinearOrder = (WB_TILE_Y == 0 || WB_TILE_Z == 0);
static_assert(kLinearOrder || ((kTileY & (kTileY - 1)) == 0 && (kTileZ & (kTileZ - 1)) == 0),
              "tile sizes are powers of two");

struct Grid {
  double lo[3];
  double hi[3];
  double R;
  double invR;   // not used for cell indices (IEEE division is), only for pruning
  int32_t N[3];
  int32_t reach; // cells searched on each side, ceil(2h / R)
  int64_t ncell;
  int32_t NT[2];     // tiles along y and z
  int64_t nkey;      // number of sort keys (>= ncell)
  const uint32_t *trank;  // Morton rank of every (y, z) tile (NT0 NT1 entries)
};

// Sort key of cell (x, y, z).
__device__ __forceinline__ uint32_t cell_key(const Grid &g, int x, int y, int z) {
  if (kLinearOrder) return (uint32_t)(x + (int64_t)y * g.N[0] + (int64_t)z * g.N[0] * g.N[1]);
  const int ty = y / kTileY, tz = z / kTileZ;  // constant powers of two: shifts
  const uint32_t r = g.trank[ty + tz * g.NT[0]];
  return r * (uint32_t)(g.N[0] * kTileY * kTileZ) +
         (uint32_t)(x + (y - ty * kTileY) * g.N[0] + (z - tz * kTileZ) * g.N[0] * kTileY);
}

// Physical / numerical constants as the kernels need them.
struct Phys {
  int32_t dim;
  uint32_t flags;
  int32_t fs_mode;
  int32_t pad_;
  double h, inv_h, two_h, two_h2;  // two_h2 = (2h)*(2h)
  double c0, rho0, inv_c02, dx;
  double alpha;    // Wendland normalisation 7/(4 pi h^2) or 21/(16 pi h^3)
  double kfac;     // 5 alpha / h^2:  grad_i W_ij = kfac t^3 (x_j - x_i)
  double w0inv;    // 1 / W(dx / h)
  double wself;    // W(0)
  double m_half_inv_h;  // -1 / (2h):  t = 1 - q/2 = 1 + s m_half_inv_h
  double two_inv_h;     // 2 / h:      2q + 1 = 1 + s two_inv_h
  double aw0;           // alpha / W(dx):  W / W(dx) = aw0 t^4 (2q + 1)
  double delta, pst_R, pst_n;
  double lambda_tic, lambda_lo, lambda_hi, lambda_sing;
  double grav[3], famp[3], fomega;
  double cfl, nu, gmax;   // gmax = max_t |G(t)|
  double skin_max;        // skin of kept lists: the cells' room reach R - 2h (0: none)
  double skin_pad;        // part of the skin reserved for the rounding of positions
  double win;             // window radius of the mirror and scan cell searches:
                          // 2h, wider over the cells of a kept-list build
};

// Device-resident scalars (one instance in the workspace).
struct Scalars {
  double t;          // time at the start of the current step
  double dt;         // current step
  double t_rhs;      // time of the right-hand side being evaluated
  double umax;       // sqrt of umax2 for the current right-hand side
  unsigned long long umax2_bits;  // atomic max of |U|^2 (non-negative double bits)
  unsigned long long pairs;       // sum of fluid neighbour counts of the last RHS
  unsigned long long tests;       // candidate distance tests of the last pair pass
  uint32_t err;
  uint32_t n_cand;   // candidates listed by the pair pass
  uint32_t n_scan;   // candidates sent to the scan pass
  uint32_t n_fs, n_cons, n_sing, n_mlp;
  uint32_t pad_;
  double steps;
  double disp;       // bound on any particle's move since the kept lists were built
  double umax1;      // U_max of the current step's first stage
  uint32_t vovf;     // a lane's candidates exceeded the kept chunks at the last build
  uint32_t mode;     // pair-pass mode of the last right-hand side (kPairSearch...)
  // pairs and tests of the last right-hand side that searched (s) and of the
  // last one that ran from kept lists (k), before the current one
  unsigned long long pairs_s, tests_s, pairs_k, tests_k;
  double body_x[3], body_u[3];  // moving body: displacement and velocity at t_rhs
  // free body: on/off, centre of its reference pose, state (c, q, v, omega)
  // at the current right-hand side, its copy of t^n (second stage), and the
  // water's force and torque of the last right-hand side
  uint32_t fb_on, fb_pad_;
  double fb_c0[3];
  double fb[13], fb0[13], fbF[6];
};

// Fluid state, FP64 path, sorted by (cell, original index).
struct FluidF64 {
  double *x[3], *u[3], *phi, *m;
  double *x0[3], *u0[3], *phi0;  // stage-0 copies (SSP-RK2 second stage)
  uint32_t *id;                  // original index
};

// Fluid state, mixed path: int cell (packed) + FP32 offset in [0, R),
// FP32 velocity, FP64 potential; Kahan compensations and the stage-1
// increments used by the incremental form of the second stage.
struct FluidMixed {
  uint32_t *cell;      // ix | iy << 11 | iz << 22
  float *o[3], *oc[3]; // offset and its Kahan compensation
  float *u[3], *uc[3];
  double *phi;
  float *m;
  float *dx1[3], *du1[3];  // stage-1 increments dt*(U+dU), dt*a
  double *dphi1;
  uint32_t *id;
};

// Per-fluid outputs of one right-hand side (sorted order).
struct Rates {
  double *acc[3], *dphi, *dus[3], *lam[3], *nrm[3];
  uint32_t *flags;
  uint32_t *nnb;
  float *feat;    // nf * 16 (all particles, SPH_F_FEATURES) or candidate rows
  float *logit;   // nf
};

// ------------------------------------------------------------ device math

__device__ __forceinline__ void body_force(const Phys &P, double t, double G[3]) {
  double s = sin(P.fomega * t);
  double w2 = P.fomega * P.fomega;
#pragma unroll
  for (int a = 0; a < 3; ++a) G[a] = P.grav[a] + P.famp[a] * w2 * s;
}

// Rotation matrix (row-major) of the unit quaternion q = (w, x, y, z).
// Rounded as written (no contraction): the free body's dummy positions then
// do not depend on the compiler's choice of fused operations.
__device__ __forceinline__ void quat_rotation(const double q[4], double R[9]) {
#pragma clang fp contract(off)
  const double w = q[0], x = q[1], y = q[2], z = q[3];
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

// R v for a row-major 3x3 R, rounded as written.
__device__ __forceinline__ void mat3_apply(const double R[9], const double v[3], double out[3]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a] = R[3 * a] * v[0] + R[3 * a + 1] * v[1] + R[3 * a + 2] * v[2];
}

// Velocity of the free body's material point at offset d from its centre,
// v + omega x d (state layout c[3] q[4] v[3] omega[3]), rounded as written.
__device__ __forceinline__ void free_body_point_velocity(const double fb[13], const double d[3], double U[3]) {
#pragma clang fp contract(off)
  const double *v = fb + 7, *w = fb + 10;
  U[0] = v[0] + (w[1] * d[2] - w[2] * d[1]);
  U[1] = v[1] + (w[2] * d[0] - w[0] * d[2]);
  U[2] = v[2] + (w[0] * d[1] - w[1] * d[0]);
}

// Cell coordinate along one axis, Eq. (ixyz): floor((x - lo) / R) with an
// IEEE subtraction and division (no contraction), as the cell index must be
// reproducible bit for bit.
__device__ __forceinline__ int cell_coord(double x, double lo, double R) {
  return (int)floor((x - lo) / R);
}

// |r|^2 summed in axis order without contraction (the neighbour test of
// Algorithm 1 decides set membership, so it is evaluated exactly as written).
template <int DIM>
__device__ __forceinline__ double dist2_exact(double rx, double ry, double rz) {
#pragma clang fp contract(off)
  double s = rx * rx;
  s = s + ry * ry;
  if (DIM == 3) s = s + rz * rz;
  return s;
}

// 1 / sqrt(x) for a finite, normal x > 0: the hardware estimate (relative
// error below 2^-22) refined by one third-order step, y (1 + e/2 + 3e^2/8)
// with e = 1 - x y^2, which leaves an error of order e^3 (below FP64
// rounding).  Zero, infinite and denormal arguments are not handled.
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

// Closed-form eigenvalues of a symmetric 2x2 / 3x3 matrix (Sec. 3),
// ascending.  S = (xx, yy, zz, xy, xz, yz).
//
// 3x3: the trigonometric solution of the characteristic cubic loses half the
// digits for the two eigenvalues of a nearly repeated pair (acos is steep at
// +-1), which lattice rows next to a wall or the surface hit (L = diag(a, a,
// b) up to round-off).  So only the isolated eigenvalue is taken from it --
// the largest when det((S - qI)/p)/2 >= 0, else the smallest; its distance to
// the other two is at least 1.5 p there and its value depends smoothly on the
// cosine argument -- and the other two come from the 2x2 compression of S onto
// the plane orthogonal to that eigenvalue's eigenvector (the largest cross
// product of two rows of S - e I), whose eigenvalues m +- sqrt(d^2 + b^2)
// involve no cancellation (Eberly, "A Robust Eigensolver for 3x3 Symmetric
// Matrices", Geometric Tools, 2014).  Accurate to a few ulps of |S|.
template <int DIM>
__device__ __forceinline__ void eig_sym(const double S[6], double lam[3]) {
  if (DIM == 2) {
    double m = 0.5 * (S[0] + S[1]), d = 0.5 * (S[0] - S[1]);
    double r = sqrt(d * d + S[3] * S[3]);
    lam[0] = m - r;
    lam[1] = m + r;
    lam[2] = 0.0;
    return;
  }
  const double a00 = S[0], a11 = S[1], a22 = S[2], a01 = S[3], a02 = S[4], a12 = S[5];
  double p1 = a01 * a01 + a02 * a02 + a12 * a12;
  if (p1 == 0.0) {
    double e0 = fmin(a00, fmin(a11, a22)), e2 = fmax(a00, fmax(a11, a22));
    lam[0] = e0;
    lam[2] = e2;
    lam[1] = a00 + a11 + a22 - e0 - e2;
    return;
  }
  double q = (a00 + a11 + a22) * (1.0 / 3.0);
  double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
  double p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * p1;
  double p = sqrt(p2 * (1.0 / 6.0));
  double ip = 1.0 / p;
  double B00 = b00 * ip, B11 = b11 * ip, B22 = b22 * ip, B01 = a01 * ip, B02 = a02 * ip, B12 = a12 * ip;
  double det = B00 * (B11 * B22 - B12 * B12) - B01 * (B01 * B22 - B12 * B02) + B02 * (B01 * B12 - B11 * B02);
  double r = fmin(1.0, fmax(-1.0, 0.5 * det));
  double ang = acos(r) * (1.0 / 3.0);
  // isolated eigenvalue: q + 2p cos(ang) (largest) or q + 2p cos(ang + 2 pi/3)
  const double e1 = q + 2.0 * p * cos(r >= 0.0 ? ang : ang + 2.0943951023931954923);
  // its eigenvector: rows of S - e1 I span the orthogonal plane
  const double r0x = a00 - e1, r1y = a11 - e1, r2z = a22 - e1;
  const double c0x = a01 * a12 - a02 * r1y, c0y = a02 * a01 - r0x * a12, c0z = r0x * r1y - a01 * a01;
  const double c1x = a01 * r2z - a02 * a12, c1y = a02 * a02 - r0x * r2z, c1z = r0x * a12 - a01 * a02;
  const double c2x = r1y * r2z - a12 * a12, c2y = a12 * a02 - a01 * r2z, c2z = a01 * a12 - r1y * a02;
  const double n0 = c0x * c0x + c0y * c0y + c0z * c0z;
  const double n1 = c1x * c1x + c1y * c1y + c1z * c1z;
  const double n2 = c2x * c2x + c2y * c2y + c2z * c2z;
  double vx = c0x, vy = c0y, vz = c0z, nv = n0;
  if (n1 > nv) { vx = c1x; vy = c1y; vz = c1z; nv = n1; }
  if (n2 > nv) { vx = c2x; vy = c2y; vz = c2z; nv = n2; }
  double e2, e3;
  if (nv > 0.0) {
    const double iv = 1.0 / sqrt(nv);
    vx *= iv; vy *= iv; vz *= iv;
    // orthonormal u, w spanning v's orthogonal plane
    double ux, uy, uz;
    if (fabs(vx) > fabs(vy)) {
      const double s = 1.0 / sqrt(vx * vx + vz * vz);
      ux = -vz * s; uy = 0.0; uz = vx * s;
    } else {
      const double s = 1.0 / sqrt(vy * vy + vz * vz);
      ux = 0.0; uy = vz * s; uz = -vy * s;
    }
    const double wx = vy * uz - vz * uy, wy = vz * ux - vx * uz, wz = vx * uy - vy * ux;
    const double aux = a00 * ux + a01 * uy + a02 * uz, auy = a01 * ux + a11 * uy + a12 * uz,
                 auz = a02 * ux + a12 * uy + a22 * uz;
    const double awx = a00 * wx + a01 * wy + a02 * wz, awy = a01 * wx + a11 * wy + a12 * wz,
                 awz = a02 * wx + a12 * wy + a22 * wz;
    const double m00 = ux * aux + uy * auy + uz * auz;
    const double m01 = wx * aux + wy * auy + wz * auz;
    const double m11 = wx * awx + wy * awy + wz * awz;
    const double m = 0.5 * (m00 + m11), d = 0.5 * (m00 - m11);
    const double rr = sqrt(d * d + m01 * m01);
    e2 = m - rr;
    e3 = m + rr;
  } else {  // p at the bottom of the FP64 range: the cubic's roots as they are
    const double hi = q + 2.0 * p * cos(ang), lo = q + 2.0 * p * cos(ang + 2.0943951023931954923);
    lam[0] = lo;
    lam[2] = hi;
    lam[1] = 3.0 * q - hi - lo;
    return;
  }
  const double lo = fmin(e1, fmin(e2, e3)), hi = fmax(e1, fmax(e2, e3));
  lam[0] = lo;
  lam[2] = hi;
  lam[1] = e1 + e2 + e3 - lo - hi;
}

// Inverse of a symmetric matrix S = (xx, yy, zz, xy, xz, yz) as the same
// packed form; returns the determinant.
template <int DIM>
__device__ __forceinline__ double inv_sym(const double S[6], double I[6]) {
  if (DIM == 2) {
    double det = S[0] * S[1] - S[3] * S[3];
    double id = 1.0 / det;
    I[0] = S[1] * id;
    I[1] = S[0] * id;
    I[3] = -S[3] * id;
    I[2] = I[4] = I[5] = 0.0;
    return det;
  }
  double c00 = S[1] * S[2] - S[5] * S[5];
  double c11 = S[0] * S[2] - S[4] * S[4];
  double c22 = S[0] * S[1] - S[3] * S[3];
  double c01 = S[4] * S[5] - S[3] * S[2];
  double c02 = S[3] * S[5] - S[4] * S[1];
  double c12 = S[3] * S[4] - S[0] * S[5];
  double det = S[0] * c00 + S[3] * c01 + S[4] * c02;
  double id = 1.0 / det;
  I[0] = c00 * id;
  I[1] = c11 * id;
  I[2] = c22 * id;
  I[3] = c01 * id;
  I[4] = c02 * id;
  I[5] = c12 * id;
  return det;
}

template <int DIM>
__device__ __forceinline__ void sym_mul(const double I[6], const double v[3], double y[3]) {
  if (DIM == 2) {
    y[0] = I[0] * v[0] + I[3] * v[1];
    y[1] = I[3] * v[0] + I[1] * v[1];
    y[2] = 0.0;
  } else {
    y[0] = I[0] * v[0] + I[3] * v[1] + I[4] * v[2];
    y[1] = I[3] * v[0] + I[1] * v[1] + I[5] * v[2];
    y[2] = I[4] * v[0] + I[5] * v[1] + I[2] * v[2];
  }
}

// ------------------------------------------------------- cell-row walker
//
// Algorithm 1 visits the 3^d cells around the particle's cell.  Cells along x
// are consecutive in storage, so each (y, z) offset is one contiguous run of
// particles: one "row".  With cells smaller than 2h the walker visits
// (2 reach + 1)^(d-1) rows; a row whose (y, z) slab is farther than 2h from
// the particle is skipped and the x span is cut to the particle's reach.  The
// cuts only bound the search, so they are evaluated in FP32 in cell units
// from the particle's position inside its own cell and widened by 1e-5 cell
// (far above the FP32 rounding of numbers below 2 reach + 1); set membership
// is decided per pair by the exact test.  Each row yields up to two runs:
// its fluid and its dummy records.
struct RowWalker {
  int32_t row;        // next row index in [0, nrows)
  int32_t nrows;
  int32_t seg;        // 0: fluid part of the current row emitted, 1: row done
  uint32_t cur, end;  // current run [cur, end) in record index space
  uint32_t dlo, dhi;  // dummy run of the current row (absolute record index)
  int32_t cx, cy, cz;
  float ux, uy, uz;   // position inside the own cell, in cells ([0, 1) up to rounding)
  float rr2;          // (2h / R)^2, widened
  int32_t tkey;       // tile of the cached rank (-1: none)
  uint32_t tbase;     // first sort key of that tile
};

constexpr float kWalkSlack = 1e-5f;

// From an FP64 position: the own cell is the exact cell index of Eq. (ixyz).
template <int DIM>
__device__ __forceinline__ void walker_init(RowWalker &w, const Grid &g, double x, double y, double z,
                                            double two_h) {
  w.cx = cell_coord(x, g.lo[0], g.R);
  w.cy = cell_coord(y, g.lo[1], g.R);
  w.cz = DIM == 3 ? cell_coord(z, g.lo[2], g.R) : 0;
  w.ux = (float)((x - (g.lo[0] + (double)w.cx * g.R)) * g.invR);
  w.uy = (float)((y - (g.lo[1] + (double)w.cy * g.R)) * g.invR);
  w.uz = DIM == 3 ? (float)((z - (g.lo[2] + (double)w.cz * g.R)) * g.invR) : 0.0f;
  const float rr = (float)(two_h * g.invR);
  w.rr2 = rr * rr * (1.0f + 4.0f * kWalkSlack);
  w.nrows = DIM == 3 ? (2 * g.reach + 1) * (2 * g.reach + 1) : 2 * g.reach + 1;
  w.row = 0;
  w.seg = 1;
  w.cur = w.end = 0;
  w.dlo = w.dhi = 0;
  w.tkey = -1;
  w.tbase = 0;
}

// From a stored cell and the offset inside it (mixed path; offsets in metres).
template <int DIM>
__device__ __forceinline__ void walker_init_cell(RowWalker &w, const Grid &g, int cx, int cy, int cz, float ox,
                                                 float oy, float oz, double two_h) {
  w.cx = cx;
  w.cy = cy;
  w.cz = DIM == 3 ? cz : 0;
  const float invR = (float)g.invR;
  w.ux = ox * invR;
  w.uy = oy * invR;
  w.uz = DIM == 3 ? oz * invR : 0.0f;
  const float rr = (float)(two_h * g.invR);
  w.rr2 = rr * rr * (1.0f + 4.0f * kWalkSlack);
  w.nrows = DIM == 3 ? (2 * g.reach + 1) * (2 * g.reach + 1) : 2 * g.reach + 1;
  w.row = 0;
  w.seg = 1;
  w.cur = w.end = 0;
  w.dlo = w.dhi = 0;
  w.tkey = -1;
  w.tbase = 0;
}

// Sort key of cell (x, y, z), reusing the walker's cached tile rank.
__device__ __forceinline__ uint32_t walker_key(RowWalker &w, const Grid &g, int x, int y, int z) {
  if (kLinearOrder) return cell_key(g, x, y, z);
  const int ty = y / kTileY, tz = z / kTileZ;
  const int t = ty + tz * g.NT[0];
  if (t != w.tkey) {
    w.tkey = t;
    w.tbase = g.trank[t] * (uint32_t)(g.N[0] * kTileY * kTileZ);
  }
  return w.tbase + (uint32_t)(x + (y - ty * kTileY) * g.N[0] + (z - tz * kTileZ) * g.N[0] * kTileY);
}

// Window of row r of the walk (raster order): the sort keys [k0, k1) of the
// row's cells within the walk's reach, and the row's (y, z) cell; false if
// the row lies outside the grid or beyond the reach.
template <int DIM>
__device__ __forceinline__ bool walker_row(RowWalker &w, const Grid &g, int r, uint32_t &k0, uint32_t &k1, int &iy,
                                           int &iz) {
  const int side = 2 * g.reach + 1;
  const int dy = (DIM == 3 ? r % side : r) - g.reach;
  const int dz = DIM == 3 ? r / side - g.reach : 0;
  iy = w.cy + dy;
  iz = w.cz + dz;
  if (iy < 0 || iy >= g.N[1]) return false;
  if (DIM == 3 && (iz < 0 || iz >= g.N[2])) return false;
  // distance (cells) from the particle to the row's (y, z) slab, shortened
  float ey = dy > 0 ? (float)dy - w.uy : (dy < 0 ? w.uy - (float)(dy + 1) : 0.0f);
  float ez = DIM == 3 ? (dz > 0 ? (float)dz - w.uz : (dz < 0 ? w.uz - (float)(dz + 1) : 0.0f)) : 0.0f;
  ey = fmaxf(0.0f, ey - kWalkSlack);
  ez = fmaxf(0.0f, ez - kWalkSlack);
  const float rem = w.rr2 - ey * ey - ez * ez;
  if (rem < 0.0f) return false;
  const float reach = __builtin_amdgcn_sqrtf(rem) + kWalkSlack;  // hardware sqrt (~1 ulp), covered by the slack
  int x0 = w.cx + (int)floorf(w.ux - reach);
  int x1 = w.cx + (int)floorf(w.ux + reach);
  x0 = max(x0, max(w.cx - g.reach, 0));
  x1 = min(x1, min(w.cx + g.reach, g.N[0] - 1));
  if (x0 > x1) return false;
  k0 = walker_key(w, g, x0, iy, iz);
  k1 = k0 + (uint32_t)(x1 - x0) + 1u;  // x-row cells are consecutive keys
  return true;
}

// Fluid runs [lo[r], hi[r]) of all NR rows of the walk (NR = (2 reach +
// 1)^(d-1)), the cell-start loads of every row issued together rather than
// one row after the other (empty runs for rows out of reach).
template <int DIM, int NR>
__device__ __forceinline__ void walker_fluid_runs(RowWalker &w, const Grid &g, const uint32_t *__restrict__ cs_f,
                                                  uint32_t (&lo)[NR], uint32_t (&hi)[NR]) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    uint32_t k0 = 0u, k1 = 0u;
    int iy, iz;
    const bool ok = walker_row<DIM>(w, g, r, k0, k1, iy, iz);
    lo[r] = ok ? cs_f[k0] : 0u;
    hi[r] = ok ? cs_f[k1] : 0u;
  }
}

// Advances to the next non-empty run; returns false when the walk is over.
// cs_f / cs_d: start index (per sort key, nkey + 1 entries) of the fluid and
// dummy records; dummy records live at index nf + k.
template <int DIM>
__device__ __forceinline__ bool walker_next(RowWalker &w, const Grid &g, const uint32_t *__restrict__ cs_f,
                                            const uint32_t *__restrict__ cs_d, uint32_t nf) {
  for (;;) {
    if (w.seg == 0) {  // fluid part done: emit the dummy part of the same row
      w.seg = 1;
      if (w.dlo < w.dhi) {
        w.cur = w.dlo;
        w.end = w.dhi;
        return true;
      }
      continue;
    }
    if (w.row >= w.nrows) return false;
    const int r = w.row++;
    uint32_t k0, k1;
    int iy, iz;
    if (!walker_row<DIM>(w, g, r, k0, k1, iy, iz)) continue;
    const uint32_t flo = cs_f[k0], fhi = cs_f[k1];
    w.dlo = nf + cs_d[k0];
    w.dhi = nf + cs_d[k1];
    w.seg = 0;
    if (flo < fhi) {
      w.cur = flo;
      w.end = fhi;
      return true;
    }
  }
}

// Logical block index with consecutive logical blocks on the same XCD: the
// hardware deals blocks round-robin over the 8 XCDs (each with its own L2),
// so block b runs on XCD b % 8; XCD x is given the x-th contiguous share of
// the logical range, which keeps a neighbourhood's records in one L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nblocks) {
  if (!WB_XCD_REMAP) return b;
  const uint32_t q = nblocks / 8, rm = nblocks % 8;
  const uint32_t x = b % 8, k = b / 8;
  return x * q + min(x, rm) + k;
}

// ---------------------------------------------------------- launch helpers

inline unsigned grid_for(int64_t n, int block = kBlock) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Grid of the passes with one wave per free-surface candidate: the count is
// on the device, so the grid is sized from the fluid count, up to 2,048
// blocks, and the waves stride over the list (16,384 blocks measured 3.4x
// slower on the 17.5M-particle tank's 125,000 candidates).
inline unsigned candidate_grid(int64_t nf) {
  const unsigned b = grid_for(nf);
  return b > 2048u ? 2048u : b;
}

// Host launchers implemented in the kernel translation units.  All take the
// stream to enqueue on and return hipSuccess or the launch error.
struct Ctx;  // host context (api.hip)

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s);
// exclusive scan of n u32 values into out (out may alias in); total written
// to out[n]; tmp needs scan_tmp_words(n) words.
size_t scan_tmp_words(int64_t n);
hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s);

}  // namespace wb

// Neighbour-grid build (Sec. 3): cell index and HashID per particle
// (Eqs. ixyz, hashid), ordering of the particles by HashID, begin/end index
// of every cell, and the reorder of the particle arrays.
//
// The ordering is a counting sort on the dense HashID key -- a radix sort with
// a single digit of log2(ncell) bits: one histogram pass (atomic slot per
// particle), one exclusive scan over the cells (which *is* the begin/end
// table), one scatter.  The scatter order inside a cell depends on atomic
// arrival, so a per-cell pass then sorts each cell's short run by original
// index: the final order is (HashID, original index), identical to a stable
// radix sort of the particles in original order, and deterministic.
#include "common.h"
#include "kernels.h"

namespace wb {

// ------------------------------------------------------------------ fills

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------- scan
// Exclusive scan of u32 in three passes: per-tile sums (tile = 1024), a
// single-block scan of the tile sums, a per-tile scan that adds the offset.

constexpr int kScanTile = 1024;  // 256 threads x 4 items

size_t scan_tmp_words(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
  // 256 threads, wave64: inclusive scan inside each wave, then across waves
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  uint32_t wbase = 0;
  for (int k = 0; k < wid; ++k) wbase += sh[k];
  total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return wbase + x - v;
}

__global__ void __launch_bounds__(256) k_scan_tiles(const uint32_t *__restrict__ in, uint32_t *__restrict__ sums,
                                                    int64_t n) {
  __shared__ uint32_t sh[4];
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
  uint32_t v = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (base + k < n) v += in[base + k];
  uint32_t tot;
  block_exclusive_scan(v, sh, tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_scan_sums(uint32_t *sums, int64_t m) {
  // exclusive scan of m tile sums in place by one block; sums[m] = total
  __shared__ uint32_t sh[4];
  uint32_t carry = 0;
  for (int64_t base = 0; base < m; base += 256) {
    int64_t i = base + threadIdx.x;
    uint32_t v = i < m ? sums[i] : 0;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(v, sh, tot);
    if (i < m) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) sums[m] = carry;
}

__global__ void __launch_bounds__(256) k_scan_apply(const uint32_t *__restrict__ in, uint32_t *out,
                                                    const uint32_t *__restrict__ sums, int64_t n) {
  __shared__ uint32_t sh[4];
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
  uint32_t v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = base + k < n ? in[base + k] : 0;
  uint32_t tot;
  uint32_t ex = block_exclusive_scan(v[0] + v[1] + v[2] + v[3], sh, tot) + sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    // grand total
    int64_t m = gridDim.x;
    out[n] = sums[m];
  }
}

hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s) {
  int64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles < 1) tiles = 1;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(256), 0, s, in, tmp, n);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, tmp, tiles);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(256), 0, s, in, out, tmp, n);
  return hipGetLastError();
}

// ------------------------------------------------------------ hash + count

// Slots inside the cells: lanes of a wave with the same key in a contiguous
// run (particles arrive nearly sorted) reserve their slots with one atomic
// add by the run's first lane.  Every lane must call it (valid lanes form a
// prefix of the wave); returns this lane's slot.
__device__ __forceinline__ uint32_t reserve_slot(uint32_t *count, uint32_t k, bool valid) {
  const int lane = (int)(threadIdx.x & 63);
  const uint32_t prev = __shfl_up(k, 1, 64);
  const unsigned long long vmask = __ballot(valid);
  const unsigned long long heads = __ballot(valid && (lane == 0 || prev != k));
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);  // bits 0 .. lane
  const int h = 63 - __clzll((long long)(heads & upto));                      // this lane's run head
  uint32_t base = 0;
  if (valid && h == lane) {
    const unsigned long long later = heads & ~upto;
    const int end = later ? __ffsll((long long)later) - 1 : __popcll(vmask);
    base = atomicAdd(&count[k], (uint32_t)(end - lane));
  }
  base = __shfl(base, valid ? h : lane, 64);
  return base + (uint32_t)(lane - h);
}

// Cell of particle i, Eq. (ixyz), its sort key (the cell in the storage
// order of cell_key), plus its slot inside the cell (arrival order).
// Out-of-domain or non-finite positions set an error bit and are parked in
// cell 0 so that every later index stays valid.
template <int DIM>
__global__ void __launch_bounds__(256) k_hash_f64(Grid g, const double *__restrict__ x,
                                                  const double *__restrict__ y, const double *__restrict__ z,
                                                  int64_t n, uint32_t *__restrict__ key, uint32_t *__restrict__ slot,
                                                  uint32_t *__restrict__ count, Scalars *sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  double p[3] = {0.0, 0.0, 0.0};
  if (valid) {
    p[0] = x[i];
    p[1] = y[i];
    if (DIM == 3) p[2] = z[i];
  }
  int c[3] = {0, 0, 0};
  bool bad = !valid;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (!valid) {
    } else if (!isfinite(p[a])) {
      atomicOr(&sc->err, kErrNonFinite);
      bad = true;
    } else if (p[a] < g.lo[a] || p[a] > g.hi[a]) {
      atomicOr(&sc->err, kErrDomain);
      bad = true;
    } else {
      c[a] = cell_coord(p[a], g.lo[a], g.R);
      if (c[a] < 0 || c[a] >= g.N[a]) {
        atomicOr(&sc->err, kErrDomain);
        bad = true;
      }
    }
  }
  uint32_t k = 0;
  if (valid && !bad) k = cell_key(g, c[0], c[1], c[2]);
  const uint32_t sl = reserve_slot(count, k, valid);
  if (valid) {
    key[i] = k;
    slot[i] = sl;
  }
}

// Mixed path: the cell is stored; the key is computed from it directly.
__global__ void __launch_bounds__(256) k_hash_packed(Grid g, const uint32_t *__restrict__ cell, int64_t n,
                                                     uint32_t *__restrict__ key, uint32_t *__restrict__ slot,
                                                     uint32_t *__restrict__ count, Scalars *sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  const uint32_t c = valid ? cell[i] : 0u;
  const int cx = c & 2047u, cy = (c >> 11) & 2047u, cz = c >> 22;
  uint32_t k = 0;
  if (valid && (cx >= g.N[0] || cy >= g.N[1] || cz >= g.N[2])) {
    atomicOr(&sc->err, kErrDomain);
  } else if (valid) {
    k = cell_key(g, cx, cy, cz);
  }
  const uint32_t sl = reserve_slot(count, k, valid);
  if (valid) {
    key[i] = k;
    slot[i] = sl;
  }
}

__global__ void __launch_bounds__(256) k_scatter(const uint32_t *__restrict__ key, const uint32_t *__restrict__ slot,
                                                 const uint32_t *__restrict__ start, int64_t n,
                                                 uint32_t *__restrict__ perm) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  perm[start[key[i]] + slot[i]] = (uint32_t)i;
}

// Sorts each cell's run of perm by original index (insertion sort; runs are
// a few dozen long).  One thread per cell.
__global__ void __launch_bounds__(256) k_canon(const uint32_t *__restrict__ start, int64_t ncell,
                                               const uint32_t *__restrict__ id, uint32_t *__restrict__ perm) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  uint32_t b = start[c], e = start[c + 1];
  // a cell this full only occurs with particles parked after a domain error;
  // keep arrival order there rather than spend quadratic time
  if (e - b > 1024u) return;
  for (uint32_t k = b + 1; k < e; ++k) {
    uint32_t v = perm[k];
    uint32_t vid = id[v];
    uint32_t m = k;
    while (m > b && id[perm[m - 1]] > vid) {
      perm[m] = perm[m - 1];
      --m;
    }
    perm[m] = v;
  }
}

hipError_t launch_sort_keys(const Grid &g, int dim, const double *x, const double *y, const double *z,
                            const uint32_t *packed_cell, int64_t n, const uint32_t *id, SortScratch &ss,
                            uint32_t *start, uint32_t *perm, Scalars *sc, hipStream_t s) {
  hipError_t e = launch_fill_u32(ss.count, 0u, g.nkey + 1, s);
  if (e != hipSuccess) return e;
  if (n > 0) {
    if (packed_cell)
      hipLaunchKernelGGL(k_hash_packed, dim3(grid_for(n)), dim3(kBlock), 0, s, g, packed_cell, n, ss.key, ss.slot,
                         ss.count, sc);
    else if (dim == 2)
      hipLaunchKernelGGL(k_hash_f64<2>, dim3(grid_for(n)), dim3(kBlock), 0, s, g, x, y, z, n, ss.key, ss.slot,
                         ss.count, sc);
    else
      hipLaunchKernelGGL(k_hash_f64<3>, dim3(grid_for(n)), dim3(kBlock), 0, s, g, x, y, z, n, ss.key, ss.slot,
                         ss.count, sc);
  }
  e = launch_exclusive_scan(ss.count, start, g.nkey, ss.scan_tmp, s);
  if (e != hipSuccess) return e;
  if (n > 0) {
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(n)), dim3(kBlock), 0, s, ss.key, ss.slot, start, n, perm);
    hipLaunchKernelGGL(k_canon, dim3(grid_for(g.nkey)), dim3(kBlock), 0, s, start, g.nkey, id, perm);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------- reorder

// Gathers the FP64 fluid state into sorted order (src -> dst) and writes the
// neighbour-facing records rec0 = (x, y, z, phi), rec1 = (u, v, w, V) with
// V = m / (rho0 exp(phi / C0^2)).  with_stage0 also carries the stage-0
// copies (second stage of SSP-RK2).
template <int DIM>
__global__ void __launch_bounds__(256) k_reorder_f64(Phys P, const uint32_t *__restrict__ perm, int64_t n,
                                                     FluidF64 src, FluidF64 dst, double4 *__restrict__ rec0,
                                                     double4 *__restrict__ rec1, int with_stage0) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  uint32_t o = perm[k];
  double xs[3], us[3];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    xs[a] = src.x[a][o];
    us[a] = src.u[a][o];
    dst.x[a][k] = xs[a];
    dst.u[a][k] = us[a];
  }
  if (DIM == 2) xs[2] = us[2] = 0.0;
  double ph = src.phi[o], m = src.m[o];
  dst.phi[k] = ph;
  dst.m[k] = m;
  dst.id[k] = src.id[o];
  if (with_stage0) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      dst.x0[a][k] = src.x0[a][o];
      dst.u0[a][k] = src.u0[a][o];
    }
    dst.phi0[k] = src.phi0[o];
  }
  double V = m / (P.rho0 * exp(ph * P.inv_c02));
  rec0[k] = make_double4(xs[0], xs[1], xs[2], ph);
  rec1[k] = make_double4(us[0], us[1], us[2], V);
}

hipError_t launch_reorder_f64(const Phys &P, const uint32_t *perm, int64_t n, const FluidF64 &src,
                              const FluidF64 &dst, double4 *rec0, double4 *rec1, int with_stage0, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_reorder_f64<2>, dim3(grid_for(n)), dim3(kBlock), 0, s, P, perm, n, src, dst, rec0, rec1,
                       with_stage0);
  else
    hipLaunchKernelGGL(k_reorder_f64<3>, dim3(grid_for(n)), dim3(kBlock), 0, s, P, perm, n, src, dst, rec0, rec1,
                       with_stage0);
  return hipGetLastError();
}

// Neighbour-facing records of the FP64 state in its current order, without a
// sort (second stage of a step that keeps the first stage's candidates).
template <int DIM>
__global__ void __launch_bounds__(256) k_refresh_f64(Phys P, FluidF64 f, int64_t n, double4 *__restrict__ rec0,
                                                     double4 *__restrict__ rec1) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double x = f.x[0][k], y = f.x[1][k], z = DIM == 3 ? f.x[2][k] : 0.0;
  const double u = f.u[0][k], v = f.u[1][k], w = DIM == 3 ? f.u[2][k] : 0.0;
  const double ph = f.phi[k];
  const double V = f.m[k] / (P.rho0 * exp(ph * P.inv_c02));
  rec0[k] = make_double4(x, y, z, ph);
  rec1[k] = make_double4(u, v, w, V);
}

hipError_t launch_refresh_f64(const Phys &P, const FluidF64 &f, int64_t n, double4 *rec0, double4 *rec1,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_refresh_f64<2>, dim3(grid_for(n)), dim3(kBlock), 0, s, P, f, n, rec0, rec1);
  else
    hipLaunchKernelGGL(k_refresh_f64<3>, dim3(grid_for(n)), dim3(kBlock), 0, s, P, f, n, rec0, rec1);
  return hipGetLastError();
}

}  // namespace wb

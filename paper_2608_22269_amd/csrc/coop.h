// Candidate search of the pair passes (FP64 and mixed) with the rows walked
// in lockstep by the wave (Algorithm 1).
//
// The lanes of a wave hold consecutive particles in storage order, so they
// sit in one x-row of cells or in two adjacent ones, and they visit the same
// (y, z) neighbour rows.  The search therefore runs per group of lanes that
// share (y, z) and lie within a bounded x span: for every neighbour row the
// wave reads the cell-start entries of the group's union span with one
// coalesced load (fluid and dummy tables), each lane takes the bounds of its
// own window (the cells within its reach, cut as the per-lane row walker of
// common.h cuts them) from those entries by a cross-lane read, and then loads
// and tests its window's records, a batch at a time.  Walking the rows in
// lockstep keeps the lanes converged, where per-lane walkers drift apart and
// the wave runs the union of their row changes.
//
// The candidate set and its order (rows in walk order, each row's fluid run
// before its dummy run, ascending storage index) equal the per-lane walker's,
// so the neighbour lists and the summation order are the same.
//
// In-range candidates are appended to the lane's column of an LDS list.  The
// search is a resumable state machine: it returns to the caller as soon as
// one lane's list might overflow; the caller consumes every lane's list (the
// dense pair body) and resumes it.  Keeping the pair body out of the search's
// loops keeps the search state that lives across it to a few registers.
#pragma once

#include "common.h"

namespace wb {

// Orders the LDS writes of a wave before its later reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

// Position of a particle in its own cell, in cell units (walker conventions).
struct CellPos {
  int cx, cy, cz;
  float ux, uy, uz;
};

// A particle outside the grid (an error the hash reports) keeps a cell a few
// cells outside it, so that its windows are empty and the group arithmetic
// cannot overflow.
template <int DIM>
__device__ __forceinline__ CellPos cellpos_of(const Grid &g, double x, double y, double z) {
  CellPos c;
  c.cx = cell_coord(x, g.lo[0], g.R);
  c.cy = cell_coord(y, g.lo[1], g.R);
  c.cz = DIM == 3 ? cell_coord(z, g.lo[2], g.R) : 0;
  c.ux = (float)((x - (g.lo[0] + (double)c.cx * g.R)) * g.invR);
  c.uy = (float)((y - (g.lo[1] + (double)c.cy * g.R)) * g.invR);
  c.uz = DIM == 3 ? (float)((z - (g.lo[2] + (double)c.cz * g.R)) * g.invR) : 0.0f;
  c.cx = min(max(c.cx, -8), g.N[0] + 8);
  c.cy = min(max(c.cy, -8), g.N[1] + 8);
  c.cz = min(max(c.cz, -8), g.N[2] + 8);
  return c;
}

// Search state of one wave.  Group, row and segment are the same in every
// lane; the windows and the cursor are per lane.
struct CoopWalk {
  unsigned long long todo;  // lanes not yet searched
  int gcy, gcz;             // group: first lane's (y, z) cell
  int U0, ncs;              // union span [U0, U0 + ncs - 2] of the group
  int dy, dz;               // next row (offsets from the group's row)
  int seg;                  // 1: fluid window of the row, 2: its dummy window
  int tkey;                 // tile of the cached rank
  uint32_t tbase;
  bool mem;                 // lane in the group
  int c, ce;                // lane's cursor and end in the current window (record index)
  uint32_t dlo, dhi;        // lane's dummy window of the current row
  float rr2;
};

__device__ __forceinline__ void coop_init(CoopWalk &w, const Grid &g, bool active, float two_h, int dim) {
  w.todo = __ballot(active);
  w.dy = 0;
  w.dz = g.reach + 1;  // past the last row: the first call forms a group
  const float rr = two_h * (float)g.invR;
  w.rr2 = rr * rr * (1.0f + 4.0f * kWalkSlack);
  w.tkey = -1;
  w.tbase = 0;
  w.mem = false;
  w.c = w.ce = 0;  // no window yet
  w.dlo = w.dhi = 0;
  w.seg = 2;
}

// Advances the walk to the next row in which some lane of the group has a
// window and sets every lane's windows; false when every lane is done.
template <int DIM>
__device__ __forceinline__ bool coop_next_row(CoopWalk &w, const Grid &g, const uint32_t *__restrict__ cs_f,
                                              const uint32_t *__restrict__ cs_d, uint32_t nf, const CellPos &p) {
  const int lane = (int)(threadIdx.x & 63);
  for (;;) {
    int dy = __builtin_amdgcn_readfirstlane(w.dy), dz = __builtin_amdgcn_readfirstlane(w.dz);
    if (dz > (DIM == 3 ? g.reach : 0)) {
      // next group: the first remaining lane and the lanes that share its
      // (y, z) row within the x span
      if (w.todo == 0ull) return false;
      const int f = __ffsll((long long)w.todo) - 1;
      const int gcx = __builtin_amdgcn_readlane(p.cx, f);
      w.gcy = __builtin_amdgcn_readlane(p.cy, f);
      w.gcz = __builtin_amdgcn_readlane(p.cz, f);
      const int wmax = 62 - 2 * g.reach;  // group x span, so that ncs <= 64
      // lane f always joins, so every group removes at least one lane
      w.mem = lane == f ||
              (((w.todo >> lane) & 1ull) && p.cy == w.gcy && p.cz == w.gcz && p.cx >= gcx && p.cx <= gcx + wmax);
      w.todo &= ~__ballot(w.mem);
      const int ghi = wave_max_int(w.mem ? p.cx : gcx);
      w.U0 = max(gcx - g.reach, 0);
      const int U1 = min(ghi + g.reach, g.N[0] - 1);
      w.ncs = U1 - w.U0 + 2;  // cell starts of U0 .. U1 + 1
      dy = -g.reach;
      dz = DIM == 3 ? -g.reach : 0;
    }
    // rows in walk order: dy fastest, then dz (one sweep of dy in 2D)
    if (dy < g.reach) {
      w.dy = dy + 1;
      w.dz = dz;
    } else {
      w.dy = -g.reach;
      w.dz = dz + 1;
    }
    const int iy = w.gcy + dy, iz = w.gcz + dz;
    if (iy < 0 || iy >= g.N[1]) continue;
    if (DIM == 3 && (iz < 0 || iz >= g.N[2])) continue;
    // this lane's window of cells in the row (the walker's cut)
    float ey = dy > 0 ? (float)dy - p.uy : (dy < 0 ? p.uy - (float)(dy + 1) : 0.0f);
    float ez = DIM == 3 ? (dz > 0 ? (float)dz - p.uz : (dz < 0 ? p.uz - (float)(dz + 1) : 0.0f)) : 0.0f;
    ey = fmaxf(0.0f, ey - kWalkSlack);
    ez = fmaxf(0.0f, ez - kWalkSlack);
    const float rem = w.rr2 - ey * ey - ez * ez;
    // the hardware square root (about 1 ulp): the slack covers it
    const float reach = __builtin_amdgcn_sqrtf(fmaxf(rem, 0.0f)) + kWalkSlack;
    int x0 = p.cx + (int)floorf(p.ux - reach);
    int x1 = p.cx + (int)floorf(p.ux + reach);
    x0 = max(x0, max(p.cx - g.reach, 0));
    x1 = min(x1, min(p.cx + g.reach, g.N[0] - 1));
    const bool has = w.mem && rem >= 0.0f && x0 <= x1;
    if (__ballot(has) == 0ull) continue;
    // first sort key of the union span (x-row cells are consecutive keys)
    uint32_t key0;
    if (kLinearOrder) {
      key0 = cell_key(g, w.U0, iy, iz);
    } else {
      const int ty = iy / kTileY, tz = iz / kTileZ;
      const int t = ty + tz * g.NT[0];
      if (t != w.tkey) {
        w.tkey = t;
        w.tbase = g.trank[t] * (uint32_t)(g.N[0] * kTileY * kTileZ);
      }
      key0 = w.tbase + (uint32_t)(w.U0 + (iy - ty * kTileY) * g.N[0] + (iz - tz * kTileZ) * g.N[0] * kTileY);
    }
    // cell starts of the union span, fluid and dummy, one coalesced load each
    const bool ld = lane < w.ncs;
    const uint32_t sf = ld ? cs_f[key0 + (uint32_t)lane] : 0u;
    const uint32_t sd = ld ? cs_d[key0 + (uint32_t)lane] : 0u;
    const int i0 = has ? x0 - w.U0 : 0, i1 = has ? x1 - w.U0 + 1 : 0;
    const uint32_t flo = __shfl(sf, i0, 64), fhi = __shfl(sf, i1, 64);
    const uint32_t dlo = __shfl(sd, i0, 64), dhi = __shfl(sd, i1, 64);
    w.c = (int)flo;
    w.ce = has ? (int)fhi : (int)flo;
    w.dlo = nf + dlo;
    w.dhi = has ? nf + dhi : nf + dlo;
    w.seg = 1;
    return true;
  }
}

// Fills this wave's lists until one lane might overflow (returns false: the
// caller consumes the lists and calls again) or the search ends (true).
// load(j) returns record j's position; near(pos, j) classifies the candidate:
// 0 rejected, 1 taken, 2 taken with kSkinTag set on its list entry (a
// candidate kept for later that is not a neighbour now).
// list_col points at this lane's column (entry k at list_col[k * stride]).
// Loads run up to BATCH - 1 records past a window's end: the record arrays
// carry that many padding records.  Requires 2 reach + 2 <= 64 (the union
// span's cell starts fit one load).
template <int DIM, int LIST, int BATCH, class LoadFn, class NearFn>
__device__ __forceinline__ bool coop_fill(CoopWalk &w, const Grid &g, const uint32_t *__restrict__ cs_f,
                                          const uint32_t *__restrict__ cs_d, uint32_t nf, const CellPos &p,
                                          uint32_t *list_col, int stride, int &cnt, uint32_t &ntest,
                                          LoadFn load, NearFn near) {
  for (;;) {
    // batches of the current windows (the hot loop: only the cursor and the
    // list count change here)
    int c = w.c;
    const int ce = w.ce;
    while (__ballot(c < ce)) {
      if (__ballot(cnt > LIST - BATCH)) {
        w.c = c;
        return false;
      }
      // idle lanes load record 0 (always present)
      const bool busy = c < ce;
      const uint32_t c0 = busy ? (uint32_t)c : 0u;
      decltype(load(0u)) b[BATCH];
#pragma unroll
      for (int k = 0; k < BATCH; ++k) b[k] = load(c0 + (uint32_t)k);
      const int n = busy ? min(BATCH, ce - c) : 0;
#pragma unroll
      for (int k = 0; k < BATCH; ++k) {
        const uint32_t j = c0 + (uint32_t)k;
        const uint32_t code = k < n ? near(b[k], j) : 0u;
        list_col[cnt * stride] = j | ((code >> 1) * kSkinTag);  // branch-free append (cnt <= LIST - BATCH)
        cnt += code != 0u ? 1 : 0;
      }
      ntest += (uint32_t)n;
      c += n;
    }
    w.c = c;
    if (w.seg == 1) {  // then the dummy windows of the row
      w.seg = 2;
      w.c = (int)w.dlo;
      w.ce = (int)w.dhi;
      continue;
    }
    if (!coop_next_row<DIM>(w, g, cs_f, cs_d, nf, p)) return true;
  }
}

// ------------------------------------------------ one wave per particle

// The fluid and dummy windows of row r of particle p's search (the walker's
// cut), for a wave that spreads one particle's rows over its lanes.  Empty
// when the row is outside the grid or pruned.
template <int DIM>
__device__ __forceinline__ void row_windows(const Grid &g, const CellPos &p, float rr2, int r,
                                            const uint32_t *__restrict__ cs_f, const uint32_t *__restrict__ cs_d,
                                            uint32_t nf, uint32_t &fb, uint32_t &fl, uint32_t &db, uint32_t &dl) {
  fb = fl = db = dl = 0;
  const int side = 2 * g.reach + 1;
  const int dy = (DIM == 3 ? r % side : r) - g.reach;
  const int dz = DIM == 3 ? r / side - g.reach : 0;
  const int iy = p.cy + dy, iz = p.cz + dz;
  if (iy < 0 || iy >= g.N[1]) return;
  if (DIM == 3 && (iz < 0 || iz >= g.N[2])) return;
  float ey = dy > 0 ? (float)dy - p.uy : (dy < 0 ? p.uy - (float)(dy + 1) : 0.0f);
  float ez = DIM == 3 ? (dz > 0 ? (float)dz - p.uz : (dz < 0 ? p.uz - (float)(dz + 1) : 0.0f)) : 0.0f;
  ey = fmaxf(0.0f, ey - kWalkSlack);
  ez = fmaxf(0.0f, ez - kWalkSlack);
  const float rem = rr2 - ey * ey - ez * ez;
  if (rem < 0.0f) return;
  const float reach = __builtin_amdgcn_sqrtf(rem) + kWalkSlack;
  int x0 = p.cx + (int)floorf(p.ux - reach);
  int x1 = p.cx + (int)floorf(p.ux + reach);
  x0 = max(x0, max(p.cx - g.reach, 0));
  x1 = min(x1, min(p.cx + g.reach, g.N[0] - 1));
  if (x0 > x1) return;
  const uint32_t k0 = cell_key(g, x0, iy, iz);
  const uint32_t k1 = k0 + (uint32_t)(x1 - x0) + 1u;
  fb = cs_f[k0];
  fl = cs_f[k1] - fb;
  db = nf + cs_d[k0];
  dl = nf + cs_d[k1] - db;
}

// Per-wave tables of one particle's row windows (LDS), for kBlock-thread blocks.
struct RowTables {
  uint32_t pre[kBlock / 64][64], fb[kBlock / 64][64], fl[kBlock / 64][64], db[kBlock / 64][64];
};

// Lays one particle's row windows out as one index range [0, M) (rows in
// walk order, each row's fluid window before its dummy window) and returns
// M; record_of() then maps an index to its record.  Called by the whole wave.
template <int DIM>
__device__ __forceinline__ uint32_t rows_layout(RowTables &t, const Grid &g, const CellPos &p, float two_h,
                                                const uint32_t *__restrict__ cs_f,
                                                const uint32_t *__restrict__ cs_d, uint32_t nf, int &nrows) {
  const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
  const int side = 2 * g.reach + 1;
  nrows = DIM == 3 ? side * side : side;
  const float rr = two_h * (float)g.invR;
  const float rr2 = rr * rr * (1.0f + 4.0f * kWalkSlack);
  uint32_t fb = 0, fl = 0, db = 0, dl = 0;
  if (lane < nrows) row_windows<DIM>(g, p, rr2, lane, cs_f, cs_d, nf, fb, fl, db, dl);
  const uint32_t len = fl + dl;
  uint32_t incl = len;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  t.pre[wv][lane] = incl - len;
  t.fb[wv][lane] = fb;
  t.fl[wv][lane] = fl;
  t.db[wv][lane] = db;
  wave_lds_sync();
  return __shfl(incl, 63, 64);
}

// Record of index idx < M of the layout (the row is the last one whose
// prefix does not exceed idx; it is never an empty row).
__device__ __forceinline__ uint32_t record_of(const RowTables &t, int nrows, uint32_t idx) {
  const int wv = (int)(threadIdx.x >> 6);
  int lo = 0, hi = nrows - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t.pre[wv][mid] <= idx) lo = mid;
    else hi = mid - 1;
  }
  const uint32_t off = idx - t.pre[wv][lo];
  return off < t.fl[wv][lo] ? t.fb[wv][lo] + off : t.db[wv][lo] + (off - t.fl[wv][lo]);
}

}  // namespace wb

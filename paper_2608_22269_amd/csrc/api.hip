// Host runtime and C ABI (declared in include/wbsph.h): parameter checks,
// workspace carving, set-up, the per-step launch sequence on the caller's
// stream, field export in the caller's particle order, and the neighbour-list
// export used by parity checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "mixed.h"
#include "mlp.h"

using namespace wb;

namespace {

constexpr size_t kAlign = 256;

// Bump allocator over the caller's workspace; with base == 0 it only sizes.
struct Carver {
  uintptr_t base, off, cap;
  bool dry;
  template <typename T>
  T *take(int64_t count) {
    off = (off + kAlign - 1) & ~(uintptr_t)(kAlign - 1);
    T *p = dry ? nullptr : reinterpret_cast<T *>(base + off);
    off += (uintptr_t)(count > 0 ? count : 1) * sizeof(T);
    return p;
  }
};

const double kPi = 3.14159265358979323846;

bool finite_pos(double v) { return std::isfinite(v); }

}  // namespace

struct sph_ctx {
  sph_params p;
  Phys P;
  Grid g;
  int dim;
  int64_t n, nf, nd;
  hipStream_t s;

  // FP64 fluid state (double buffered for the reorder) and records
  FluidF64 cur, alt;
  // mixed fluid state
  FluidMixed mcur, malt;
  MixedRec mrec;
  double4 *rec0, *rec1;  // nf + nd (FP64 path; dummies at nf.. in both paths)
  uint32_t *cs_f, *cs_d;
  uint32_t *perm;
  SortScratch ss;
  Dummies dm;
  Dummies dm2;  // moving body: the dummies' second buffer for their re-sort
  bool has_body;   // a prescribed or a free body
  bool free_body;  // body_free
  Body body;
  FreeBody fbody;
  double *body_ft;  // free body: force and torque partials (6 per block of dummies)
  // SPH_F_GRAPH: two steps captured on a stream of the library's own and
  // replayed on the caller's; valid while the buffers a step swaps are where
  // they were at the capture (they return there every two steps)
  hipStream_t cap_s;
  hipGraphExec_t gexec;
  bool g_ok;
  double g_dt;
  FluidF64 g_cur, g_alt;
  FluidMixed g_mcur, g_malt;
  Dummies g_dm, g_dm2;
  Rates r;
  uint32_t *cand, *fallback;
  float *cand_logit;
  // candidate lists kept from a step's first stage (SPH_F_KEEP_LISTS)
  uint32_t *kent;
  unsigned long long *kcnt;
  double n_kept, n_rebuilt;  // second stages run from them / rebuilt instead
  Scalars *sc;
  unsigned char *stage;
  size_t stage_bytes;
  // classifier (learned mode)
  Classifier clf;
  bool has_clf;

  // per-kernel timing (sph_profile)
  bool profiling;
  std::vector<hipEvent_t> ev_a, ev_b;
  std::vector<int> ev_kind;
  size_t ev_used;
  double prof_ms[8], prof_cnt[8];

  sph_status status;
  std::string err;
  bool cells_current;  // grid/order match the current positions
  bool rates_current;  // rates align with the current order
  bool lists_valid;    // kept lists match the current order (no sort since their build)
  bool umax_fresh;     // sc->umax2_bits holds max |U|^2 of the current state
  bool recs_fresh;     // the neighbour records hold the current state
  bool mixed;
};

namespace {

sph_status fail(sph_ctx *c, sph_status st, const std::string &msg) {
  if (c) c->err = msg;
  return st;
}

sph_status hip_check(sph_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return SPH_OK;
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (c) {
    c->status = SPH_EHIP;
    c->err = m;
  }
  return SPH_EHIP;
}

double kernel_alpha(int dim, double h) {
  return dim == 2 ? 7.0 / (4.0 * kPi * h * h) : 21.0 / (16.0 * kPi * h * h * h);
}

double wendland(int dim, double h, double q) {
  if (q > 2.0) return 0.0;
  double t = 1.0 - 0.5 * q;
  return kernel_alpha(dim, h) * t * t * t * t * (2.0 * q + 1.0);
}

bool params_ok(const sph_params *p, std::string *why) {
  auto bad = [&](const char *m) {
    if (why) *why = m;
    return false;
  };
  if (!p) return bad("params is NULL");
  if (p->dim != 2 && p->dim != 3) return bad("dim must be 2 or 3");
  if (p->precision != SPH_FP64 && p->precision != SPH_MIXED && p->precision != SPH_FP32)
    return bad("unknown precision");
  if (p->fs_mode < SPH_FS_NONE || p->fs_mode > SPH_FS_LEARNED) return bad("unknown fs_mode");
  if (!(p->dx > 0) || !(p->h > 0) || !(p->c0 > 0) || !(p->rho0 > 0)) return bad("dx, h, c0, rho0 must be > 0");
  if (!(p->cfl > 0) || !(p->nu >= 0)) return bad("cfl must be > 0 and nu >= 0");
  if (!(p->pst_n > 0)) return bad("pst_n must be > 0");
  double R = p->cell_size > 0 ? p->cell_size : 2.0 * p->h;
  if (std::ceil(2.0 * p->h / R) > kMaxReach) return bad("cell_size must be >= 2h/3");
  for (int a = 0; a < p->dim; ++a) {
    if (!(p->domain_hi[a] > p->domain_lo[a])) return bad("domain_hi must exceed domain_lo");
    double N = std::floor((p->domain_hi[a] - p->domain_lo[a]) / R) + 1;
    if (N > (a == 2 ? 1023 : 2047)) return bad("too many cells along an axis (max 2047, 2047, 1023)");
  }
  double ncell = 1;
  for (int a = 0; a < p->dim; ++a) ncell *= std::floor((p->domain_hi[a] - p->domain_lo[a]) / R) + 1 + 16;
  if (ncell > 2.0e9) return bad("too many cells");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->gravity[a]) || !std::isfinite(p->forcing_amp[a])) return bad("non-finite body force");
  if (p->flags & ~511u) return bad("unknown flag bits");
  if ((p->flags & SPH_F_GRAPH) && (p->flags & SPH_F_KEEP_LISTS))
    return bad("SPH_F_GRAPH excludes SPH_F_KEEP_LISTS");
  if ((p->flags & SPH_F_KEEP_ACROSS_STEPS) && !(p->flags & SPH_F_KEEP_LISTS))
    return bad("SPH_F_KEEP_ACROSS_STEPS needs SPH_F_KEEP_LISTS");
  if (p->body_pieces < 0 || p->body_pieces > 4) return bad("body_pieces must be 0..4");
  for (int k = 0; k < p->body_pieces; ++k) {
    if (!std::isfinite(p->body_t[k]) || !std::isfinite(p->body_t[k + 1]) || !(p->body_t[k + 1] > p->body_t[k]))
      return bad("body breakpoints must be finite and strictly increasing");
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(p->body_a[k][a]) || !std::isfinite(p->body_b[k][a])) return bad("non-finite body motion");
  }
  if (p->body_free) {
    if (p->body_pieces != 0) return bad("a free body excludes a prescribed motion (body_pieces must be 0)");
    if (!(p->body_mass > 0.0) || !std::isfinite(p->body_mass)) return bad("body_mass must be finite and > 0");
    for (int k = 0; k < 6; ++k)
      if (!std::isfinite(p->body_inertia[k])) return bad("non-finite body_inertia");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(p->body_c0[k])) return bad("non-finite body_c0");
    for (int k = 0; k < 13; ++k)
      if (!std::isfinite(p->body_state0[k])) return bad("non-finite body_state0");
    const double *q = p->body_state0 + 3;
    if (std::fabs(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3] - 1.0) > 1e-12)
      return bad("body_state0: the quaternion must have unit norm");
    const double *I = p->body_inertia;
    if (p->dim == 2) {
      if (!(I[2] > 0.0)) return bad("body_inertia: zz must be > 0");
      if (q[1] != 0.0 || q[2] != 0.0 || p->body_state0[9] != 0.0 || p->body_state0[10] != 0.0 ||
          p->body_state0[11] != 0.0)
        return bad("2D free body: q = (cos, 0, 0, sin), v_z = 0, omega = (0, 0, wz)");
    } else {
      // Sylvester's criterion on the packed xx yy zz xy xz yz tensor
      const double m2 = I[0] * I[1] - I[3] * I[3];
      const double m3 = I[0] * (I[1] * I[2] - I[5] * I[5]) - I[3] * (I[3] * I[2] - I[5] * I[4]) +
                        I[4] * (I[3] * I[5] - I[1] * I[4]);
      if (!(I[0] > 0.0) || !(m2 > 0.0) || !(m3 > 0.0)) return bad("body_inertia must be positive definite");
    }
  }
  return true;
}

void derive(const sph_params *p, Phys &P, Grid &g) {
  std::memset(&P, 0, sizeof(P));
  std::memset(&g, 0, sizeof(g));
  P.dim = p->dim;
  P.flags = p->flags;
  P.fs_mode = p->fs_mode;
  P.h = p->h;
  P.inv_h = 1.0 / p->h;
  P.two_h = 2.0 * p->h;
  P.two_h2 = P.two_h * P.two_h;
  P.c0 = p->c0;
  P.rho0 = p->rho0;
  P.inv_c02 = 1.0 / (p->c0 * p->c0);
  P.dx = p->dx;
  P.alpha = kernel_alpha(p->dim, p->h);
  P.kfac = 5.0 * P.alpha / (p->h * p->h);
  P.w0inv = 1.0 / wendland(p->dim, p->h, p->dx / p->h);
  P.wself = wendland(p->dim, p->h, 0.0);
  P.m_half_inv_h = -0.5 / p->h;
  P.two_inv_h = 2.0 / p->h;
  P.aw0 = P.alpha * P.w0inv;
  P.delta = p->delta;
  P.pst_R = p->pst_R;
  P.pst_n = p->pst_n;
  P.lambda_tic = p->lambda_tic;
  P.lambda_lo = p->lambda_fs_lo;
  P.lambda_hi = p->lambda_fs_hi;
  P.lambda_sing = p->lambda_singular;
  for (int a = 0; a < 3; ++a) {
    P.grav[a] = p->gravity[a];
    P.famp[a] = p->forcing_amp[a];
  }
  P.fomega = p->forcing_omega;
  P.cfl = p->cfl;
  P.nu = p->nu;
  double gm = 0.0;
  for (int sgn = -1; sgn <= 1; sgn += 2) {
    double s2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      double v = p->gravity[a] + sgn * p->forcing_amp[a] * p->forcing_omega * p->forcing_omega;
      s2 += v * v;
    }
    gm = std::max(gm, std::sqrt(s2));
  }
  P.gmax = gm;
  g.R = p->cell_size > 0 ? p->cell_size : 2.0 * p->h;
  g.invR = 1.0 / g.R;
  g.reach = (int32_t)std::ceil(2.0 * p->h / g.R);
  P.win = P.two_h;
  // cells of reach R cover a ball of radius reach R around any point; the
  // kept lists need 2h + skin inside it (a small margin keeps the cut away
  // from the rounding of cell indices)
  // (a moving body re-sorts the dummies at every right-hand side: no lists)
  const bool keep = (p->flags & SPH_F_KEEP_LISTS) != 0u && p->body_pieces == 0 && !p->body_free;
  P.skin_max = keep ? std::max(0.0, (double)g.reach * g.R - P.two_h - 1e-6 * g.R) : 0.0;
  // absolute part of the skin: far above the rounding of FP64 positions; on
  // the mixed path, above twice the rounding of the FP32 absolute positions
  // and of the FP32 distance test
  double xmax = 0.0;
  for (int a = 0; a < p->dim; ++a) xmax = std::max(xmax, std::max(std::fabs(p->domain_lo[a]), std::fabs(p->domain_hi[a])));
  P.skin_pad = p->precision != SPH_FP64 ? 1e-6 * xmax + 1e-5 * p->h : 1e-9 * p->h;
  g.ncell = 1;
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = p->domain_lo[a];
    g.hi[a] = p->domain_hi[a];
    g.N[a] = a < p->dim ? (int32_t)std::floor((p->domain_hi[a] - p->domain_lo[a]) / g.R) + 1 : 1;
    g.ncell *= g.N[a];
  }
  g.NT[0] = kLinearOrder ? 1 : (g.N[1] + kTileY - 1) / kTileY;
  g.NT[1] = kLinearOrder ? 1 : (g.N[2] + kTileZ - 1) / kTileZ;
  const int64_t nb = (int64_t)g.NT[0] * g.NT[1];
  g.nkey = kLinearOrder ? g.ncell : nb * (int64_t)g.N[0] * kTileY * kTileZ;
  g.trank = nullptr;
}

// Morton rank of every (y, z) tile (tiles sorted by interleaved coordinates).
std::vector<uint32_t> tile_ranks(const Grid &g) {
  auto spread = [](uint64_t v) {
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
  };
  const int64_t nb = (int64_t)g.NT[0] * g.NT[1];
  std::vector<std::pair<uint64_t, uint32_t>> code((size_t)nb);
  for (int64_t tz = 0, k = 0; tz < g.NT[1]; ++tz)
    for (int64_t ty = 0; ty < g.NT[0]; ++ty, ++k) code[(size_t)k] = {spread((uint64_t)ty) | (spread((uint64_t)tz) << 1), (uint32_t)k};
  std::sort(code.begin(), code.end());
  std::vector<uint32_t> rank((size_t)nb);
  for (size_t r = 0; r < code.size(); ++r) rank[code[r].second] = (uint32_t)r;
  return rank;
}

// Carves every device array of a context.  Returns the bytes used.
size_t carve(sph_ctx *c, uintptr_t base, size_t cap) {
  Carver cv{base, 0, cap, base == 0};
  const int64_t nf = c->nf, nd = c->nd, n = c->n, nmax = std::max(nf, nd);
  const int dim = c->dim;
  const bool mixed = c->mixed;
  auto f64 = [&](int64_t k) { return cv.take<double>(k); };
  if (!mixed) {
    for (FluidF64 *f : {&c->cur, &c->alt}) {
      for (int a = 0; a < 3; ++a) {
        f->x[a] = a < dim ? f64(nf) : nullptr;
        f->u[a] = a < dim ? f64(nf) : nullptr;
        f->x0[a] = a < dim ? f64(nf) : nullptr;
        f->u0[a] = a < dim ? f64(nf) : nullptr;
      }
      f->phi = f64(nf);
      f->m = f64(nf);
      f->phi0 = f64(nf);
      f->id = cv.take<uint32_t>(nf);
    }
  } else {
    for (FluidMixed *f : {&c->mcur, &c->malt}) {
      f->cell = cv.take<uint32_t>(nf);
      for (int a = 0; a < 3; ++a) {
        bool on = a < dim;
        f->o[a] = on ? cv.take<float>(nf) : nullptr;
        f->oc[a] = on ? cv.take<float>(nf) : nullptr;
        f->u[a] = on ? cv.take<float>(nf) : nullptr;
        f->uc[a] = on ? cv.take<float>(nf) : nullptr;
        f->dx1[a] = on ? cv.take<float>(nf) : nullptr;
        f->du1[a] = on ? cv.take<float>(nf) : nullptr;
      }
      f->phi = f64(nf);
      f->m = cv.take<float>(nf);
      f->dphi1 = f64(nf);
      f->id = cv.take<uint32_t>(nf);
    }
    c->mrec.r0 = cv.take<float4>(nf + nd);
    c->mrec.r1 = cv.take<float4>(nf + nd);
    c->mrec.xa = cv.take<float4>(nf + nd + kRecPad);
    c->mrec.phi = f64(nf + nd);
  }
  c->rec0 = mixed ? nullptr : cv.take<double4>(nf + nd + kRecPad);
  c->rec1 = mixed ? nullptr : cv.take<double4>(nf + nd);
  c->cs_f = cv.take<uint32_t>(c->g.nkey + 1);
  c->cs_d = cv.take<uint32_t>(c->g.nkey + 1);
  c->g.trank = cv.take<uint32_t>((int64_t)c->g.NT[0] * c->g.NT[1]);
  c->perm = cv.take<uint32_t>(nmax);
  c->ss.key = cv.take<uint32_t>(nmax);
  c->ss.slot = cv.take<uint32_t>(nmax);
  c->ss.count = cv.take<uint32_t>(c->g.nkey + 1);
  c->ss.scan_tmp = cv.take<uint32_t>((int64_t)scan_tmp_words(std::max<int64_t>(c->g.nkey, n + 1)) + 1);
  const bool body = c->p.body_pieces > 0 || c->p.body_free;
  const bool fbody = c->p.body_free != 0;
  for (Dummies *d : {&c->dm, &c->dm2}) {
    const bool on = d == &c->dm || body;
    for (int a = 0; a < 3; ++a) {
      d->x[a] = on && a < dim ? f64(nd) : nullptr;
      d->n[a] = on && a < dim ? f64(nd) : nullptr;
      d->x0[a] = body && a < dim ? f64(nd) : nullptr;
      d->n0[a] = fbody && a < dim ? f64(nd) : nullptr;
    }
    d->m = on ? f64(nd) : nullptr;
    d->phi_in = on ? f64(nd) : nullptr;
    d->id = on ? cv.take<uint32_t>(nd) : nullptr;
    d->src = on ? cv.take<int32_t>(nd) : nullptr;
    d->mov = body ? cv.take<uint8_t>(nd) : nullptr;
  }
  c->body_ft = fbody ? f64(6 * (int64_t)grid_for(nd)) : nullptr;
  for (int a = 0; a < 3; ++a) {
    c->r.acc[a] = a < dim ? f64(nf) : nullptr;
    c->r.dus[a] = a < dim ? f64(nf) : nullptr;
    c->r.nrm[a] = a < dim ? f64(nf) : nullptr;
    c->r.lam[a] = f64(nf);
  }
  c->r.dphi = f64(nf);
  c->r.flags = cv.take<uint32_t>(nf);
  c->r.nnb = cv.take<uint32_t>(nf);
  const bool want_feat = (c->p.flags & SPH_F_FEATURES) || c->p.fs_mode == SPH_FS_LEARNED;
  c->r.feat = want_feat ? cv.take<float>(nf * kNFeat) : nullptr;
  c->r.logit = cv.take<float>(nf);
  c->cand = cv.take<uint32_t>(nf);
  c->fallback = cv.take<uint32_t>(nf);
  if (c->P.skin_max > 0.0) {
    const int64_t np = (int64_t)grid_for(std::max<int64_t>(nf, 1)) * kBlock;
    c->kent = cv.take<uint32_t>((int64_t)kKeepChunks * kPairList * np);
    c->kcnt = cv.take<unsigned long long>(np);
  } else {
    c->kent = nullptr;
    c->kcnt = nullptr;
  }
  c->cand_logit = c->p.fs_mode == SPH_FS_LEARNED ? cv.take<float>(nf) : nullptr;
  c->clf.w = cv.take<float>(kMlpParams);
  c->clf.mean = cv.take<float>(kNFeat);
  c->clf.std = cv.take<float>(kNFeat);
  c->sc = cv.take<Scalars>(1);
  // staging: init copies of the inputs, dummy staging, field export, rank scans
  int64_t per = 8 * (3 * dim + 2) + 1 + 8 * (2 * dim + 2) + 8 + (body ? 8 * dim + 1 : 0) + (fbody ? 8 * dim : 0);
  c->stage_bytes = (size_t)n * (size_t)std::max<int64_t>(per + 16, 64 + 8) + ((size_t)16 << 20);
  c->stage = cv.take<unsigned char>((int64_t)c->stage_bytes);
  return cv.off + kAlign;
}

// ----------------------------------------------------------- profiling

constexpr size_t kProfSlots = 512;

void prof_drain(sph_ctx *c) {
  if (c->ev_used == 0) return;
  (void)hipStreamSynchronize(c->s);
  for (size_t k = 0; k < c->ev_used; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_a[k], c->ev_b[k]) == hipSuccess) {
      c->prof_ms[c->ev_kind[k]] += ms;
      c->prof_cnt[c->ev_kind[k]] += 1.0;
    }
  }
  c->ev_used = 0;
}

// RAII bracket: records a start event now and a stop event at scope end.
struct ProfScope {
  sph_ctx *c;
  size_t slot;
  bool on;
  ProfScope(sph_ctx *ctx, int kind) : c(ctx), slot(0), on(ctx->profiling) {
    if (!on) return;
    if (c->ev_used == c->ev_a.size()) prof_drain(c);
    slot = c->ev_used++;
    c->ev_kind[slot] = kind;
    (void)hipEventRecord(c->ev_a[slot], c->s);
  }
  ~ProfScope() {
    if (on) (void)hipEventRecord(c->ev_b[slot], c->s);
  }
};

// ------------------------------------------------------------ rebuilds

sph_status rebuild(sph_ctx *c, int with_stage0) {
  ProfScope ps(c, 2);
  hipError_t e;
  if (!c->mixed) {
    e = launch_sort_keys(c->g, c->dim, c->cur.x[0], c->cur.x[1], c->cur.x[2], nullptr, c->nf, c->cur.id, c->ss,
                         c->cs_f, c->perm, c->sc, c->s);
    if (e == hipSuccess) e = launch_reorder_f64(c->P, c->perm, c->nf, c->cur, c->alt, c->rec0, c->rec1, with_stage0, c->s);
    std::swap(c->cur, c->alt);
  } else {
    e = launch_sort_keys(c->g, c->dim, nullptr, nullptr, nullptr, c->mcur.cell, c->nf, c->mcur.id, c->ss, c->cs_f,
                         c->perm, c->sc, c->s);
    if (e == hipSuccess)
      e = launch_reorder_mixed(c->P, c->g, c->perm, c->nf, c->mcur, c->malt, c->mrec, with_stage0, c->s);
    std::swap(c->mcur, c->malt);
  }
  c->cells_current = true;
  c->rates_current = false;
  c->lists_valid = false;  // indices of the kept lists refer to the old order
  c->recs_fresh = true;    // the reorder wrote them
  return hip_check(c, e, "grid rebuild");
}

// Records of the current state in the current order (a right-hand side from
// kept lists: the cells and the order stay those of their build).
sph_status refresh(sph_ctx *c) {
  if (c->recs_fresh) return SPH_OK;  // the stage update wrote them
  c->recs_fresh = true;
  ProfScope ps(c, 2);
  hipError_t e = c->mixed ? launch_refresh_mixed(c->P, c->g, c->mcur, c->nf, c->mrec, c->s)
                          : launch_refresh_f64(c->P, c->cur, c->nf, c->rec0, c->rec1, c->s);
  return hip_check(c, e, "record refresh");
}

// The moving body at the right-hand side's time: its dummies moved to x0 +
// D(t_rhs) (prescribed motion) or to the pose of the free body's current
// state, then all dummies re-sorted by (cell, original index) into the
// second buffer (the cell-start table of the dummies is rebuilt).
sph_status move_body(sph_ctx *c) {
  if (c->nd == 0) return SPH_OK;
  ProfScope ps(c, 2);
  hipError_t e = c->free_body ? launch_free_body_place(c->dm, c->nd, c->dim, c->sc, c->s)
                              : launch_body_move(c->body, c->dm, c->nd, c->dim, c->sc, c->s);
  if (e == hipSuccess)
    e = launch_sort_keys(c->g, c->dim, c->dm.x[0], c->dm.x[1], c->dm.x[2], nullptr, c->nd, c->dm.id, c->ss, c->cs_d,
                         c->perm, c->sc, c->s);
  if (e == hipSuccess) e = launch_gather_dummies(c->perm, c->nd, c->dm, c->dm2, c->dim, c->s);
  std::swap(c->dm, c->dm2);
  return hip_check(c, e, "body motion");
}

// One right-hand side.  mode: the pair pass's kPairSearch / kPairSearchKeep /
// kPairKept; win_extra widens the cell searches of the mirror and scan passes
// (over the cells of the kept lists' build: the bound on any particle's move
// since).
sph_status rhs(sph_ctx *c, int stage, int mode = kPairSearch, double win_extra = 0.0) {
  hipError_t e = launch_stage_time(c->sc, stage, c->s, mode);
  if (e == hipSuccess && c->has_body) {
    sph_status sb = move_body(c);
    if (sb != SPH_OK) return sb;
  }
  // classifier features: every row when exported, else the candidates' in
  // the learned mode (all sixteen from the pair pass's own sums)
  const bool feat = (c->p.flags & SPH_F_FEATURES) != 0;
  const bool learned = c->p.fs_mode == SPH_FS_LEARNED && c->has_clf;
  Phys Pw = c->P;
  Pw.win = c->P.two_h + win_extra;
  if (!c->mixed) {
    if (e == hipSuccess) {
      ProfScope ps(c, 1);
      e = launch_mirror_f64(Pw, c->g, c->dm, c->nd, c->rec0, c->rec1, c->rec0 + c->nf, c->rec1 + c->nf, c->cs_f,
                            (uint32_t)c->nf, c->sc, c->s, c->cur.id);
      // the water's force and torque on the free body at this right-hand side
      if (e == hipSuccess && c->free_body && c->nd > 0)
        e = launch_body_force_f64(Pw, c->g, c->dm, c->nd, c->rec0, c->rec1, c->rec0 + c->nf, c->cs_f,
                                  (uint32_t)c->nf, c->sc, c->body_ft, c->s);
      if (e == hipSuccess && c->free_body)
        e = launch_free_body_sum(c->body_ft, c->nd > 0 ? (int64_t)grid_for(c->nd) : 0, c->sc, c->s);
    }
    if (e == hipSuccess) {
      ProfScope ps(c, mode == kPairKept ? 5 : 0);
      e = launch_pair_f64(c->P, c->g, c->rec0, c->rec1, c->cs_f, c->cs_d, (uint32_t)c->nf, c->sc, c->r, c->cand, mode,
                          c->kent, c->kcnt, c->s);
    }
  } else {
    if (e == hipSuccess) {
      ProfScope ps(c, 1);
      e = launch_mirror_mixed(Pw, c->g, c->dm, c->nd, c->mrec, c->cs_f, (uint32_t)c->nf, c->sc, c->s, c->mcur.id);
      if (e == hipSuccess && c->free_body && c->nd > 0)
        e = launch_body_force_mixed(Pw, c->g, c->dm, c->nd, c->mrec, c->cs_f, (uint32_t)c->nf, c->sc, c->body_ft,
                                    c->s);
      if (e == hipSuccess && c->free_body)
        e = launch_free_body_sum(c->body_ft, c->nd > 0 ? (int64_t)grid_for(c->nd) : 0, c->sc, c->s);
    }
    if (e == hipSuccess) {
      ProfScope ps(c, mode == kPairKept ? 5 : 0);
      e = launch_pair_mixed(c->P, c->g, c->mrec, c->cs_f, c->cs_d, (uint32_t)c->nf, c->sc, c->r, c->cand, mode,
                            c->kent, c->kcnt, c->s, c->p.precision == SPH_FP32);
    }
  }
  ProfScope ps_fs(c, 3);
  // classifier features: every fluid row when exported, else the candidates'
  if (e == hipSuccess && feat) {
    e = launch_features(c->P, c->r, nullptr, nullptr, (uint32_t)c->nf, c->sc, c->s);
  } else if (e == hipSuccess && learned) {
    e = launch_features(c->P, c->r, c->cand, &c->sc->n_cand, (uint32_t)c->nf, c->sc, c->s);
  }
  if (e == hipSuccess && c->p.fs_mode != SPH_FS_NONE) {
    const uint32_t *list = c->cand;
    const uint32_t *count = &c->sc->n_cand;
    if (c->p.fs_mode == SPH_FS_LEARNED && c->has_clf) {
      e = launch_classify(c->clf, c->r, c->cand, &c->sc->n_cand, c->fallback, c->sc, c->P, (uint32_t)c->nf,
                          c->cand_logit, c->s);
      list = c->fallback;
      count = &c->sc->n_scan;
    }
    if (e == hipSuccess) {
      if (!c->mixed)
        e = launch_scan_f64(Pw, c->g, c->rec0, c->cs_f, c->cs_d, (uint32_t)c->nf, list, count, c->r, c->sc, c->s);
      else
        e = launch_scan_mixed(Pw, c->g, c->mrec, c->cs_f, c->cs_d, (uint32_t)c->nf, list, count, c->r, c->sc, c->s);
    }
  }
  c->rates_current = true;
  return hip_check(c, e, "right-hand side");
}

sph_status umax_of_current(sph_ctx *c) {
  if (c->umax_fresh) return SPH_OK;  // the stage update computed it
  c->umax_fresh = true;
  ProfScope ps(c, 4);
  hipError_t e;
  if (!c->mixed) {
    const double *u[3] = {c->cur.u[0], c->cur.u[1], c->cur.u[2]};
    e = launch_umax(c->dim, u, nullptr, c->nf, c->sc, c->s);
  } else {
    const float *u[3] = {c->mcur.u[0], c->mcur.u[1], c->mcur.u[2]};
    e = launch_umax(c->dim, nullptr, u, c->nf, c->sc, c->s);
  }
  return hip_check(c, e, "max |U|");
}

sph_status read_scalars(sph_ctx *c, Scalars *h) {
  hipError_t e = hipMemcpyAsync(h, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  return hip_check(c, e, "read scalars");
}

sph_status sync_errors(sph_ctx *c) {
  Scalars h;
  sph_status st = read_scalars(c, &h);
  if (st != SPH_OK) return st;
  if (h.err) {
    sph_status es = (h.err & kErrDomain) ? SPH_EDOMAIN : (h.err & kErrNonFinite) ? SPH_ENONFINITE : SPH_ECAPACITY;
    c->status = es;
    c->err = (h.err & kErrDomain)      ? "a particle left the hashed domain"
             : (h.err & kErrNonFinite) ? "non-finite state or coincident particles"
                                       : "capacity exceeded";
    return es;
  }
  return SPH_OK;
}

sph_status usable(sph_ctx *c) {
  if (!c) return SPH_EINVAL;
  if (c->status != SPH_OK) return fail(c, SPH_ESTATE, "context is in an error state: " + c->err);
  return SPH_OK;
}

}  // namespace

// ======================================================================= ABI

extern "C" {

const char *sph_status_string(sph_status s) {
  switch (s) {
    case SPH_OK: return "ok";
    case SPH_EINVAL: return "invalid argument";
    case SPH_EWORKSPACE: return "workspace too small or misaligned";
    case SPH_EHIP: return "HIP runtime error";
    case SPH_EDOMAIN: return "particle outside the hashed domain";
    case SPH_ENONFINITE: return "non-finite state";
    case SPH_ESTATE: return "call not allowed in this state";
    case SPH_EUNSUPPORTED: return "unsupported";
    case SPH_ECAPACITY: return "capacity exceeded";
    default: return "unknown status";
  }
}

sph_status sph_validate(const sph_params *p) { return params_ok(p, nullptr) ? SPH_OK : SPH_EINVAL; }

size_t sph_workspace_bytes(const sph_params *p, int64_t n_fluid, int64_t n_dummy) {
  if (!params_ok(p, nullptr) || n_fluid < 0 || n_dummy < 0) return 0;
  if (n_fluid + n_dummy >= (int64_t)1 << 31) return 0;
  sph_ctx c;
  c.p = *p;
  c.dim = p->dim;
  c.nf = n_fluid;
  c.nd = n_dummy;
  c.n = n_fluid + n_dummy;
  c.mixed = p->precision != SPH_FP64;
  derive(p, c.P, c.g);
  return carve(&c, 0, 0);
}

const char *sph_last_error(const sph_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void sph_destroy(sph_ctx *ctx) {
  if (!ctx) return;
  if (ctx->g_ok) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->cap_s) (void)hipStreamDestroy(ctx->cap_s);
  for (auto ev : ctx->ev_a) (void)hipEventDestroy(ev);
  for (auto ev : ctx->ev_b) (void)hipEventDestroy(ev);
  delete ctx;
}

sph_status sph_init(const sph_params *p, int64_t n, const double *x, const double *u, const double *phi,
                    const double *mass, const uint8_t *kind, const double *normal, int32_t inputs_on_device,
                    void *workspace, size_t ws_bytes, void *hip_stream, sph_ctx **out) {
  if (!out) return SPH_EINVAL;
  *out = nullptr;
  std::string why;
  if (!params_ok(p, &why)) return SPH_EINVAL;
  if (n < 0 || n >= ((int64_t)1 << 31)) return SPH_EINVAL;
  if (n > 0 && (!x || !u || !phi || !kind)) return SPH_EINVAL;
  const int dim = p->dim;
  int64_t nf = 0, nd = 0;
  if (!inputs_on_device) {
    // host-side validation before any launch
    for (int64_t i = 0; i < n; ++i) {
      if (kind[i] > 2) return SPH_EINVAL;
      (kind[i] == 0 ? nf : nd)++;
      for (int a = 0; a < dim; ++a) {
        double v = x[i * dim + a];
        if (!finite_pos(v) || !std::isfinite(u[i * dim + a])) return SPH_ENONFINITE;
        if (v < p->domain_lo[a] || v > p->domain_hi[a]) return SPH_EDOMAIN;
      }
      if (!std::isfinite(phi[i])) return SPH_ENONFINITE;
      if (mass && !(mass[i] > 0.0)) return SPH_EINVAL;
      if (kind[i] != 0) {
        if (!normal) return SPH_EINVAL;
        double s = 0;
        for (int a = 0; a < dim; ++a) s += normal[i * dim + a] * normal[i * dim + a];
        if (std::fabs(s - 1.0) > 1e-6) return SPH_EINVAL;
      }
    }
  }
  hipStream_t s = (hipStream_t)hip_stream;
  // device inputs: count the kinds on the device first
  sph_ctx *c = new sph_ctx();
  c->p = *p;
  c->dim = dim;
  c->n = n;
  c->s = s;
  c->mixed = p->precision != SPH_FP64;
  c->status = SPH_OK;
  c->has_clf = false;
  c->cap_s = nullptr;
  c->g_ok = false;
  c->g_dt = 0.0;
  c->has_body = p->body_pieces > 0 || p->body_free;
  c->free_body = p->body_free != 0;
  c->fbody.mass = p->body_mass;
  for (int k = 0; k < 6; ++k) c->fbody.I[k] = p->body_inertia[k];
  std::memset(&c->body, 0, sizeof(c->body));
  c->body.pieces = p->body_pieces;
  for (int k = 0; k <= p->body_pieces; ++k) c->body.T[k] = p->body_t[k];
  for (int k = 0; k < p->body_pieces; ++k)
    for (int a = 0; a < 3; ++a) {
      c->body.a[k][a] = p->body_a[k][a];
      c->body.b[k][a] = p->body_b[k][a];
    }
  c->n_kept = c->n_rebuilt = 0.0;
  c->lists_valid = false;
  c->umax_fresh = c->recs_fresh = false;
  c->profiling = false;
  c->ev_used = 0;
  for (int k = 0; k < 8; ++k) c->prof_ms[k] = c->prof_cnt[k] = 0.0;
  derive(p, c->P, c->g);
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) {
    delete c;
    return SPH_EWORKSPACE;
  }
  // kind counting for device inputs uses the start of the workspace as scratch
  if (inputs_on_device && n > 0) {
    uint32_t *isf = reinterpret_cast<uint32_t *>(workspace);
    uint32_t *isd = isf + (n + 1);
    uint32_t *tmp = isd + (n + 1);
    size_t need = sizeof(uint32_t) * (size_t)(2 * (n + 1) + scan_tmp_words(n + 1) + 1);
    if (need > ws_bytes) {
      delete c;
      return SPH_EWORKSPACE;
    }
    hipError_t e = launch_kind_flags(kind, n, isf, isd, s);
    if (e == hipSuccess) e = launch_exclusive_scan(isf, isf, n, tmp, s);
    uint32_t tot = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&tot, isf + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      delete c;
      return SPH_EHIP;
    }
    nf = tot;
    nd = n - nf;
  }
  c->nf = nf;
  c->nd = nd;
  size_t need = carve(c, 0, 0);
  if (need > ws_bytes) {
    delete c;
    return SPH_EWORKSPACE;
  }
  carve(c, (uintptr_t)workspace, ws_bytes);

  // inputs into device staging
  unsigned char *st = c->stage;
  auto take = [&](size_t bytes) {
    unsigned char *q = st;
    st += (bytes + kAlign - 1) & ~(kAlign - 1);
    return q;
  };
  const double *dx_ = x, *du_ = u, *dphi_ = phi, *dm_ = mass, *dn_ = normal;
  const uint8_t *dk_ = kind;
  const bool copy_in = !inputs_on_device && n > 0;
  double *sx = nullptr, *su = nullptr, *sph = nullptr, *sm = nullptr, *sn = nullptr;
  uint8_t *sk = nullptr;
  if (copy_in) {
    sx = (double *)take(sizeof(double) * n * dim);
    su = (double *)take(sizeof(double) * n * dim);
    sph = (double *)take(sizeof(double) * n);
    sk = (uint8_t *)take((size_t)n);
    if (mass) sm = (double *)take(sizeof(double) * n);
    if (normal) sn = (double *)take(sizeof(double) * n * dim);
  }
  // kind ranks
  uint32_t *frank = (uint32_t *)take(sizeof(uint32_t) * (n + 1));
  uint32_t *drank = (uint32_t *)take(sizeof(uint32_t) * (n + 1));
  // unsorted fluid goes to `alt` (FP64) / a staging FluidF64 (mixed); dummies to staging
  Dummies dst;
  for (int a = 0; a < 3; ++a) {
    dst.x[a] = a < dim ? (double *)take(sizeof(double) * nd) : nullptr;
    dst.n[a] = a < dim ? (double *)take(sizeof(double) * nd) : nullptr;
  }
  dst.m = (double *)take(sizeof(double) * nd);
  dst.phi_in = (double *)take(sizeof(double) * nd);
  dst.id = (uint32_t *)take(sizeof(uint32_t) * nd);
  dst.src = nullptr;
  for (int a = 0; a < 3; ++a) dst.x0[a] = c->has_body && a < dim ? (double *)take(sizeof(double) * nd) : nullptr;
  for (int a = 0; a < 3; ++a) dst.n0[a] = c->free_body && a < dim ? (double *)take(sizeof(double) * nd) : nullptr;
  dst.mov = c->has_body ? (uint8_t *)take((size_t)nd) : nullptr;
  FluidF64 f0;
  std::memset(&f0, 0, sizeof(f0));
  if (!c->mixed) {
    f0 = c->cur;  // the first rebuild sorts cur into alt and swaps
  } else {
    for (int a = 0; a < dim; ++a) {
      f0.x[a] = (double *)take(sizeof(double) * nf);
      f0.u[a] = (double *)take(sizeof(double) * nf);
    }
    f0.phi = (double *)take(sizeof(double) * nf);
    f0.m = (double *)take(sizeof(double) * nf);
    f0.id = (uint32_t *)take(sizeof(uint32_t) * nf);
  }
  if ((size_t)(st - c->stage) > c->stage_bytes) {
    delete c;
    return SPH_EWORKSPACE;
  }
  hipError_t e = hipSuccess;
  if (copy_in) {
    e = hipMemcpyAsync(sx, x, sizeof(double) * n * dim, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(su, u, sizeof(double) * n * dim, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sph, phi, sizeof(double) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sk, kind, (size_t)n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && mass) e = hipMemcpyAsync(sm, mass, sizeof(double) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && normal) e = hipMemcpyAsync(sn, normal, sizeof(double) * n * dim, hipMemcpyHostToDevice, s);
    dx_ = sx;
    du_ = su;
    dphi_ = sph;
    dk_ = sk;
    dm_ = mass ? sm : nullptr;
    dn_ = normal ? sn : nullptr;
  }
  if (e == hipSuccess) e = launch_kind_flags(dk_, n, frank, drank, s);
  if (e == hipSuccess) e = launch_exclusive_scan(frank, frank, n, c->ss.scan_tmp, s);
  if (e == hipSuccess) e = launch_exclusive_scan(drank, drank, n, c->ss.scan_tmp, s);
  if (e == hipSuccess) e = launch_split(c->P, n, dx_, du_, dphi_, dm_, dk_, dn_, frank, drank, f0, dst, s);
  // scalars and the brick order of the sort keys
  Scalars h;
  std::memset(&h, 0, sizeof(h));
  if (c->free_body) {
    h.fb_on = 1u;
    for (int a = 0; a < 3; ++a) h.fb_c0[a] = p->body_c0[a];
    for (int k = 0; k < 13; ++k) h.fb[k] = h.fb0[k] = p->body_state0[k];
  }
  if (e == hipSuccess) e = hipMemcpyAsync(c->sc, &h, sizeof(Scalars), hipMemcpyHostToDevice, s);
  const std::vector<uint32_t> ranks = tile_ranks(c->g);
  if (e == hipSuccess)
    e = hipMemcpyAsync((void *)c->g.trank, ranks.data(), sizeof(uint32_t) * ranks.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  // dummies: sort once by (cell, original index)
  if (e == hipSuccess && nd > 0) {
    e = launch_sort_keys(c->g, dim, dst.x[0], dst.x[1], dst.x[2], nullptr, nd, dst.id, c->ss, c->cs_d, c->perm, c->sc,
                         s);
    if (e == hipSuccess) e = launch_gather_dummies(c->perm, nd, dst, c->dm, dim, s);
  } else if (e == hipSuccess) {
    e = launch_fill_u32(c->cs_d, 0u, c->g.nkey + 1, s);
  }
  // padding records after the FP64 neighbour records (read by batched
  // candidate loads, never used)
  if (e == hipSuccess && !c->mixed)
    e = launch_fill_u32(reinterpret_cast<uint32_t *>(c->rec0 + c->n), 0u, (int64_t)kRecPad * 8, s);
  if (e == hipSuccess && c->mixed)
    e = launch_fill_u32(reinterpret_cast<uint32_t *>(c->mrec.xa + c->n), 0u, (int64_t)kRecPad * 4, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete c;
    return SPH_EHIP;
  }
  sph_status rs;
  if (!c->mixed) {
    rs = rebuild(c, 0);
  } else {
    hipError_t e2 = launch_to_mixed(c->P, c->g, f0, nf, c->mcur, c->sc, s);
    rs = hip_check(c, e2, "mixed conversion");
    if (rs == SPH_OK) rs = rebuild(c, 0);
  }
  if (rs == SPH_OK) {
    // mirrored wall values at t = 0, so that fields are defined before any step
    hipError_t e3 = launch_stage_time(c->sc, 1, s);
    if (e3 == hipSuccess && c->has_body) {
      rs = move_body(c);
      if (rs != SPH_OK) e3 = hipErrorUnknown;
    }
    if (e3 == hipSuccess) {
      if (!c->mixed)
        e3 = launch_mirror_f64(c->P, c->g, c->dm, nd, c->rec0, c->rec1, c->rec0 + nf, c->rec1 + nf, c->cs_f,
                               (uint32_t)nf, c->sc, s, c->cur.id);
      else
        e3 = launch_mirror_mixed(c->P, c->g, c->dm, nd, c->mrec, c->cs_f, (uint32_t)nf, c->sc, s, c->mcur.id);
    }
    rs = hip_check(c, e3, "initial mirror");
  }
  if (rs == SPH_OK) rs = sync_errors(c);
  if (rs != SPH_OK) {
    delete c;
    return rs;
  }
  *out = c;
  return SPH_OK;
}

sph_status sph_build_cells(sph_ctx *c) {
  sph_status st = usable(c);
  if (st != SPH_OK) return st;
  return rebuild(c, 0);
}

sph_status sph_eval_rates(sph_ctx *c) {
  sph_status st = usable(c);
  if (st != SPH_OK) return st;
  st = umax_of_current(c);
  if (st == SPH_OK && !c->cells_current) st = rebuild(c, 0);
  if (st == SPH_OK) st = rhs(c, 1);
  return st;
}

// The right-hand side of one stage of a step.  With SPH_F_KEEP_LISTS the
// kept lists serve the second stage (and with SPH_F_KEEP_ACROSS_STEPS any
// stage) while they are valid (no sort since their build, no overflow) and
// twice the bound on any particle's move since their build, plus the
// rounding pad, fits their skin: a pair within 2h now was within 2h + skin
// at the build.  The bound lives on the device; reading it costs one
// synchronisation.  Otherwise the stage sorts, searches and builds new lists.
sph_status stage_rhs(sph_ctx *c, int stage) {
  if (!c->kent) {
    sph_status st = rebuild(c, stage == 2);
    return st == SPH_OK ? rhs(c, stage) : st;
  }
  bool reuse = false;
  double disp = 0.0;
  if (c->lists_valid && (stage == 2 || (c->p.flags & SPH_F_KEEP_ACROSS_STEPS))) {
    Scalars h;
    sph_status st = read_scalars(c, &h);
    if (st != SPH_OK) return st;
    disp = h.disp;
    reuse = h.vovf == 0u && h.err == 0u && 2.0 * disp + c->P.skin_pad <= c->P.skin_max;
  }
  if (reuse) {
    c->n_kept += 1.0;
    sph_status st = refresh(c);
    return st == SPH_OK ? rhs(c, stage, kPairKept, disp) : st;
  }
  c->n_rebuilt += 1.0;
  sph_status st = rebuild(c, stage == 2);
  if (st == SPH_OK) st = rhs(c, stage, kPairSearchKeep);
  if (st == SPH_OK) c->lists_valid = true;
  return st;
}

// The stage update of SSP-RK2.  It also computes max |U| of the new state
// (for the next right-hand side or step), writes the neighbour records when
// the next right-hand side may run from kept lists (it then needs no
// refresh), and on the FP64 path checks the state for finiteness after the
// second stage.
sph_status stage_update(sph_ctx *c, int stage) {
  ProfScope ps(c, 4);
  hipError_t e;
  const bool recs = c->kent && c->lists_valid && (stage == 1 || (c->p.flags & SPH_F_KEEP_ACROSS_STEPS));
  if (c->mixed)
    e = launch_stage_mixed(c->P, c->g, c->mcur, c->r, c->nf, c->sc, stage, c->s, recs ? &c->mrec : nullptr);
  else {
    // stage 1 writes the new state into the stage-0 arrays and the roles
    // swap: the state of t^n becomes the stage-0 copy without a copy
    if (stage == 1) {
      for (int a = 0; a < 3; ++a) {
        std::swap(c->cur.x[a], c->cur.x0[a]);
        std::swap(c->cur.u[a], c->cur.u0[a]);
      }
      std::swap(c->cur.phi, c->cur.phi0);
    }
    e = launch_stage_f64(c->P, c->cur, c->r, c->nf, c->sc, stage, c->s, recs ? c->rec0 : nullptr,
                         recs ? c->rec1 : nullptr, stage == 2 ? 1 : 0);
  }
  c->umax_fresh = true;
  c->recs_fresh = recs;
  if (e == hipSuccess && c->free_body) e = launch_free_body_stage(c->fbody, c->P, c->sc, stage, c->s);
  if (e == hipSuccess && c->kent) e = launch_disp_add(c->sc, stage, c->s);
  if (e == hipSuccess && stage == 2) e = launch_advance_time(c->sc, c->s);
  return hip_check(c, e, stage == 1 ? "stage 1" : "stage 2");
}

// One SSP-RK2 step, launched on c->s.
sph_status one_step(sph_ctx *c, double dt_override) {
  sph_status st = umax_of_current(c);
  if (st == SPH_OK) st = hip_check(c, launch_dt(c->P, c->sc, dt_override, c->s), "time step");
  if (st == SPH_OK) st = stage_rhs(c, 1);
  if (st == SPH_OK) st = stage_update(c, 1);
  if (st == SPH_OK) st = umax_of_current(c);
  if (st == SPH_OK) st = stage_rhs(c, 2);
  if (st == SPH_OK) st = stage_update(c, 2);
  c->cells_current = false;
  return st;
}

bool same_bytes(const void *a, const void *b, size_t n) { return std::memcmp(a, b, n) == 0; }

// The buffers a step swaps sit where they sat at the capture.
bool graph_matches(const sph_ctx *c, double dt_override) {
  return c->g_ok && c->g_dt == dt_override && same_bytes(&c->cur, &c->g_cur, sizeof(FluidF64)) &&
         same_bytes(&c->alt, &c->g_alt, sizeof(FluidF64)) && same_bytes(&c->mcur, &c->g_mcur, sizeof(FluidMixed)) &&
         same_bytes(&c->malt, &c->g_malt, sizeof(FluidMixed)) && same_bytes(&c->dm, &c->g_dm, sizeof(Dummies)) &&
         same_bytes(&c->dm2, &c->g_dm2, sizeof(Dummies));
}

void graph_drop(sph_ctx *c) {
  if (c->g_ok) (void)hipGraphExecDestroy(c->gexec);
  c->g_ok = false;
}

// Captures two steps on the library's own stream (nothing runs during the
// capture; the host-side buffer swaps of the two steps bring every buffer
// back to where it was).  The first step of a capture recomputes max |U|.
sph_status graph_capture(sph_ctx *c, double dt_override) {
  graph_drop(c);
  if (!c->cap_s) {
    if (hipStreamCreateWithFlags(&c->cap_s, hipStreamNonBlocking) != hipSuccess) {
      c->cap_s = nullptr;
      return fail(c, SPH_EHIP, "graph: stream creation failed");
    }
  }
  c->umax_fresh = false;
  c->g_cur = c->cur;
  c->g_alt = c->alt;
  c->g_mcur = c->mcur;
  c->g_malt = c->malt;
  c->g_dm = c->dm;
  c->g_dm2 = c->dm2;
  hipStream_t user = c->s;
  hipError_t e = hipStreamBeginCapture(c->cap_s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_check(c, e, "graph: begin capture");
  c->s = c->cap_s;
  sph_status st = one_step(c, dt_override);
  if (st == SPH_OK) st = one_step(c, dt_override);
  c->s = user;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(c->cap_s, &graph);
  if (st != SPH_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_check(c, e, "graph: capture");
  if (!same_bytes(&c->cur, &c->g_cur, sizeof(FluidF64)) || !same_bytes(&c->dm, &c->g_dm, sizeof(Dummies))) {
    (void)hipGraphExecDestroy(c->gexec);
    return fail(c, SPH_EHIP, "graph: two steps did not bring the buffers back");
  }
  c->g_ok = true;
  c->g_dt = dt_override;
  return SPH_OK;
}

sph_status sph_step(sph_ctx *c, int32_t nsteps, double dt_override) {
  sph_status st = usable(c);
  if (st != SPH_OK) return st;
  if (nsteps < 0 || !std::isfinite(dt_override)) return fail(c, SPH_EINVAL, "bad nsteps or dt_override");
  if ((c->p.flags & SPH_F_GRAPH) && !c->profiling && nsteps >= 2) {
    if (!graph_matches(c, dt_override)) st = graph_capture(c, dt_override);
    for (; nsteps >= 2 && st == SPH_OK; nsteps -= 2)
      st = hip_check(c, hipGraphLaunch(c->gexec, c->s), "graph launch");
  }
  for (int32_t k = 0; k < nsteps && st == SPH_OK; ++k) st = one_step(c, dt_override);
  return st;
}

sph_status sph_set_time(sph_ctx *c, double t) {
  sph_status st = usable(c);
  if (st != SPH_OK) return st;
  if (!std::isfinite(t)) return fail(c, SPH_EINVAL, "non-finite time");
  return hip_check(c, launch_set_time(c->sc, t, c->s), "set time");
}

sph_status sph_sync(sph_ctx *c) {
  if (!c) return SPH_EINVAL;
  if (c->status != SPH_OK) return c->status;
  return sync_errors(c);
}

sph_status sph_stats(sph_ctx *c, double out[20]) {
  if (!c || !out) return SPH_EINVAL;
  Scalars h;
  sph_status st = read_scalars(c, &h);
  if (st != SPH_OK) return st;
  for (int k = 0; k < 20; ++k) out[k] = 0.0;
  out[0] = h.t;
  out[1] = h.dt;
  out[2] = h.steps;
  out[3] = h.umax;
  out[4] = (double)c->nf;
  out[5] = (double)c->nd;
  out[6] = h.n_fs;
  out[7] = h.n_cons;
  out[8] = c->p.fs_mode == SPH_FS_LEARNED && c->has_clf ? h.n_scan : h.n_cand;
  out[9] = h.n_mlp;
  out[10] = h.n_sing;
  out[11] = (double)h.pairs;
  out[12] = h.n_cand;
  out[13] = (double)h.tests;
  out[14] = c->n_kept;
  out[15] = c->n_rebuilt;
  const bool last_kept = h.mode == (uint32_t)kPairKept;
  out[16] = (double)(last_kept ? h.pairs_s : h.pairs);
  out[17] = (double)(last_kept ? h.tests_s : h.tests);
  out[18] = (double)(last_kept ? h.pairs : h.pairs_k);
  out[19] = (double)(last_kept ? h.tests : h.tests_k);
  return c->status != SPH_OK ? c->status : SPH_OK;
}

sph_status sph_body_state(sph_ctx *c, double out[19]) {
  if (!c || !out) return SPH_EINVAL;
  if (!c->free_body) return fail(c, SPH_ESTATE, "no free body");
  Scalars h;
  sph_status st = read_scalars(c, &h);
  if (st != SPH_OK) return st;
  for (int k = 0; k < 13; ++k) out[k] = h.fb[k];
  for (int k = 0; k < 6; ++k) out[13 + k] = h.fbF[k];
  return c->status != SPH_OK ? c->status : SPH_OK;
}

sph_status sph_set_classifier(sph_ctx *c, const float *params, int64_t nparams, const float *mean, const float *std,
                              float margin) {
  sph_status st = usable(c);
  if (st != SPH_OK) return st;
  if (!params || !mean || !std || nparams != kMlpParams || !(margin >= 0.0f))
    return fail(c, SPH_EINVAL, "classifier: bad parameters");
  if (c->p.fs_mode != SPH_FS_LEARNED) return fail(c, SPH_ESTATE, "classifier needs fs_mode SPH_FS_LEARNED");
  graph_drop(c);  // the margin and the classifier's presence are launch arguments
  for (int k = 0; k < kNFeat; ++k)
    if (!(std[k] > 0.0f) || !std::isfinite(mean[k])) return fail(c, SPH_EINVAL, "classifier: bad mean/std");
  for (int64_t k = 0; k < nparams; ++k)
    if (!std::isfinite(params[k])) return fail(c, SPH_EINVAL, "classifier: non-finite weight");
  hipError_t e = hipMemcpyAsync(c->clf.w, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->clf.mean, mean, sizeof(float) * kNFeat, hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->clf.std, std, sizeof(float) * kNFeat, hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  st = hip_check(c, e, "classifier upload");
  if (st != SPH_OK) return st;
  c->clf.margin = margin;
  c->has_clf = true;
  return SPH_OK;
}

sph_status sph_profile(sph_ctx *c, int32_t enable) {
  if (!c) return SPH_EINVAL;
  if (enable && c->ev_a.empty()) {
    c->ev_a.resize(kProfSlots);
    c->ev_b.resize(kProfSlots);
    c->ev_kind.resize(kProfSlots);
    for (size_t k = 0; k < kProfSlots; ++k) {
      if (hipEventCreate(&c->ev_a[k]) != hipSuccess || hipEventCreate(&c->ev_b[k]) != hipSuccess)
        return fail(c, SPH_EHIP, "event creation failed");
    }
  }
  if (!enable) prof_drain(c);
  c->profiling = enable != 0;
  return SPH_OK;
}

sph_status sph_profile_read(sph_ctx *c, double out[16]) {
  if (!c || !out) return SPH_EINVAL;
  prof_drain(c);
  for (int k = 0; k < 8; ++k) {
    out[2 * k] = c->prof_ms[k];
    out[2 * k + 1] = c->prof_cnt[k];
    c->prof_ms[k] = c->prof_cnt[k] = 0.0;
  }
  return SPH_OK;
}

}  // extern "C"

// ----------------------------------------------------------------- fields

namespace {

__global__ void k_mirror_src_ids(const int32_t *__restrict__ src, const uint32_t *__restrict__ did,
                                 const uint32_t *__restrict__ fid, int64_t nd, int32_t *__restrict__ dst,
                                 uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nd) return;
  int32_t s = src[k];
  if (did[k] < nout) dst[did[k]] = s >= 0 ? (int32_t)fid[s] : -1;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_path_of(const uint32_t *__restrict__ flags, const uint32_t *__restrict__ id, int64_t n,
                          int32_t *__restrict__ dst, uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || id[k] >= nout) return;
  uint32_t f = flags[k];
  dst[id[k]] = (f & kFlagByMLP) ? 2 : (f & kFlagByScan) ? 1 : 0;
}

struct FieldShape {
  int width;
  size_t elem;
};

FieldShape shape_of(int field, int dim) {
  switch (field) {
    case SPH_FIELD_X: case SPH_FIELD_U: case SPH_FIELD_DUDT: case SPH_FIELD_DELTA_U: case SPH_FIELD_NORMAL:
      return {dim, 8};
    case SPH_FIELD_PHI: case SPH_FIELD_RHO: case SPH_FIELD_P: case SPH_FIELD_DPHIDT: case SPH_FIELD_MASS:
      return {1, 8};
    case SPH_FIELD_LAMBDA: return {3, 8};
    case SPH_FIELD_CELL: return {3, 4};
    case SPH_FIELD_FEATURES: return {kNFeat, 4};
    case SPH_FIELD_FS: case SPH_FIELD_TIC: case SPH_FIELD_NNB: case SPH_FIELD_MIRROR_SRC: case SPH_FIELD_FS_PATH:
    case SPH_FIELD_LOGIT:
      return {1, 4};
    default: return {0, 0};
  }
}

}  // namespace

extern "C" sph_status sph_fields(sph_ctx *c, int32_t field, void *out, int32_t out_on_device) {
  if (!c || !out) return SPH_EINVAL;
  FieldShape fs = shape_of(field, c->dim);
  if (fs.width == 0) return fail(c, SPH_EINVAL, "unknown field");
  const bool rate_field = field == SPH_FIELD_DUDT || field == SPH_FIELD_DPHIDT || field == SPH_FIELD_DELTA_U ||
                          field == SPH_FIELD_LAMBDA || field == SPH_FIELD_NORMAL || field == SPH_FIELD_FS ||
                          field == SPH_FIELD_TIC || field == SPH_FIELD_NNB || field == SPH_FIELD_FEATURES ||
                          field == SPH_FIELD_LOGIT || field == SPH_FIELD_FS_PATH;
  if (rate_field && !c->rates_current)
    return fail(c, SPH_ESTATE, "no right-hand side has been evaluated at the current ordering");
  if (field == SPH_FIELD_FEATURES && !c->r.feat) return fail(c, SPH_EUNSUPPORTED, "features not enabled");
  const size_t bytes = (size_t)c->n * fs.width * fs.elem;
  if (!out_on_device && bytes > c->stage_bytes) return fail(c, SPH_EWORKSPACE, "staging too small");
  void *dst = out_on_device ? out : (void *)c->stage;
  hipStream_t s = c->s;
  const int dim = c->dim;
  const int64_t nf = c->nf, nd = c->nd;
  hipError_t e = hipSuccess;
  double *dd = (double *)dst;
  int32_t *di = (int32_t *)dst;
  const uint32_t *fid = c->mixed ? c->mcur.id : c->cur.id;
  // zero first for fields that only fluid rows define
  if (rate_field || field == SPH_FIELD_MIRROR_SRC) {
    if (fs.elem == 8) e = launch_fill_f64(dd, 0.0, c->n * fs.width, s);
    else hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(c->n * fs.width)), dim3(kBlock), 0, s, di,
                            field == SPH_FIELD_MIRROR_SRC ? -1 : 0, c->n * fs.width);
  }
  if (c->mixed && (field == SPH_FIELD_X || field == SPH_FIELD_U || field == SPH_FIELD_PHI || field == SPH_FIELD_RHO ||
                   field == SPH_FIELD_P || field == SPH_FIELD_MASS || field == SPH_FIELD_CELL)) {
    e = launch_fields_mixed(c->P, c->g, c->mcur, nf, field, dst, s, (uint32_t)c->n);
  } else {
    switch (field) {
      case SPH_FIELD_X:
        for (int a = 0; a < dim && e == hipSuccess; ++a) e = launch_gather_f64(c->cur.x[a], fid, nf, dd, dim, a, s, (uint32_t)c->n);
        break;
      case SPH_FIELD_U:
        for (int a = 0; a < dim && e == hipSuccess; ++a) e = launch_gather_f64(c->cur.u[a], fid, nf, dd, dim, a, s, (uint32_t)c->n);
        break;
      case SPH_FIELD_PHI: e = launch_gather_f64(c->cur.phi, fid, nf, dd, 1, 0, s, (uint32_t)c->n); break;
      case SPH_FIELD_MASS: e = launch_gather_f64(c->cur.m, fid, nf, dd, 1, 0, s, (uint32_t)c->n); break;
      case SPH_FIELD_RHO: case SPH_FIELD_P:
        e = launch_rho_p(c->P, c->cur.phi, fid, nf, dd, field == SPH_FIELD_RHO ? 0 : 1, s, (uint32_t)c->n);
        break;
      case SPH_FIELD_CELL: {
        const double *xx[3] = {c->cur.x[0], c->cur.x[1], c->cur.x[2]};
        e = launch_cells_of(c->g, dim, xx, fid, nf, di, s, (uint32_t)c->n);
        break;
      }
      default: break;
    }
  }
  // dummy rows of state fields
  if (e == hipSuccess) {
    switch (field) {
      case SPH_FIELD_X:
        for (int a = 0; a < dim && e == hipSuccess; ++a) e = launch_gather_f64(c->dm.x[a], c->dm.id, nd, dd, dim, a, s, (uint32_t)c->n);
        break;
      case SPH_FIELD_MASS: e = launch_gather_f64(c->dm.m, c->dm.id, nd, dd, 1, 0, s, (uint32_t)c->n); break;
      case SPH_FIELD_CELL: {
        const double *xx[3] = {c->dm.x[0], c->dm.x[1], c->dm.x[2]};
        e = launch_cells_of(c->g, dim, xx, c->dm.id, nd, di, s, (uint32_t)c->n);
        break;
      }
      case SPH_FIELD_U:
        if (!c->mixed) e = launch_gather_rec(c->rec1 + nf, c->dm.id, nd, dd, dim, 0, dim, s, (uint32_t)c->n);
        else e = launch_dummy_fields_mixed(c->P, c->mrec, nf, c->dm.id, nd, field, dst, s, (uint32_t)c->n);
        break;
      case SPH_FIELD_PHI:
        if (!c->mixed) e = launch_gather_rec(c->rec0 + nf, c->dm.id, nd, dd, 1, 3, 1, s, (uint32_t)c->n);
        else e = launch_dummy_fields_mixed(c->P, c->mrec, nf, c->dm.id, nd, field, dst, s, (uint32_t)c->n);
        break;
      case SPH_FIELD_RHO: case SPH_FIELD_P:
        if (!c->mixed) e = launch_rho_p_rec(c->P, c->rec0 + nf, c->dm.id, nd, dd, field == SPH_FIELD_RHO ? 0 : 1, s, (uint32_t)c->n);
        else e = launch_dummy_fields_mixed(c->P, c->mrec, nf, c->dm.id, nd, field, dst, s, (uint32_t)c->n);
        break;
      case SPH_FIELD_MIRROR_SRC:
        if (nd > 0)
          hipLaunchKernelGGL(k_mirror_src_ids, dim3(grid_for(nd)), dim3(kBlock), 0, s, c->dm.src, c->dm.id, fid, nd, di,
                             (uint32_t)c->n);
        break;
      default: break;
    }
  }
  // rate fields (fluid rows)
  if (e == hipSuccess && rate_field) {
    switch (field) {
      case SPH_FIELD_DUDT:
        for (int a = 0; a < dim && e == hipSuccess; ++a) e = launch_gather_f64(c->r.acc[a], fid, nf, dd, dim, a, s, (uint32_t)c->n);
        break;
      case SPH_FIELD_DELTA_U:
        for (int a = 0; a < dim && e == hipSuccess; ++a) e = launch_gather_f64(c->r.dus[a], fid, nf, dd, dim, a, s, (uint32_t)c->n);
        break;
      case SPH_FIELD_NORMAL:
        for (int a = 0; a < dim && e == hipSuccess; ++a) e = launch_gather_f64(c->r.nrm[a], fid, nf, dd, dim, a, s, (uint32_t)c->n);
        break;
      case SPH_FIELD_LAMBDA:
        for (int a = 0; a < 3 && e == hipSuccess; ++a) e = launch_gather_f64(c->r.lam[a], fid, nf, dd, 3, a, s, (uint32_t)c->n);
        break;
      case SPH_FIELD_DPHIDT: e = launch_gather_f64(c->r.dphi, fid, nf, dd, 1, 0, s, (uint32_t)c->n); break;
      case SPH_FIELD_FS: e = launch_gather_u32_bits(c->r.flags, fid, nf, di, kFlagFS, 1, s, (uint32_t)c->n); break;
      case SPH_FIELD_TIC: e = launch_gather_u32_bits(c->r.flags, fid, nf, di, kFlagCons, 0, s, (uint32_t)c->n); break;
      case SPH_FIELD_NNB: e = launch_gather_u32_bits(c->r.nnb, fid, nf, di, 0xffffffffu, 0, s, (uint32_t)c->n); break;
      case SPH_FIELD_FEATURES: e = launch_gather_rows_f32(c->r.feat, fid, nf, kNFeat, (float *)dst, s, (uint32_t)c->n); break;
      case SPH_FIELD_LOGIT: e = launch_gather_u32_bits((const uint32_t *)c->r.logit, fid, nf, di, 0xffffffffu, 0, s, (uint32_t)c->n); break;
      case SPH_FIELD_FS_PATH:
        if (nf > 0) hipLaunchKernelGGL(k_path_of, dim3(grid_for(nf)), dim3(kBlock), 0, s, c->r.flags, fid, nf, di, (uint32_t)c->n);
        break;
      default: break;
    }
  }
  if (e == hipSuccess) e = hipGetLastError();
  sph_status st = hip_check(c, e, "fields");
  if (st != SPH_OK) return st;
  if (!out_on_device) {
    e = hipMemcpyAsync(out, c->stage, bytes, hipMemcpyDeviceToHost, s);
    st = hip_check(c, e, "fields copy");
    if (st != SPH_OK) return st;
    st = c->status != SPH_OK ? c->status : sync_errors(c);
    if (st != SPH_OK) return st;
  }
  return c->status;
}

// ------------------------------------------------------------- neighbours

namespace {

__global__ void k_shift_offsets(const uint32_t *__restrict__ off, uint32_t base, int64_t n, uint32_t *__restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) dst[i] = off[i] - base;
}

}  // namespace

extern "C" sph_status sph_neighbors(sph_ctx *c, int64_t *offsets, int32_t *ids, int64_t cap, int64_t *needed) {
  sph_status st = usable(c);
  if (st != SPH_OK) return st;
  if (!offsets) return SPH_EINVAL;
  if (c->mixed) return fail(c, SPH_EUNSUPPORTED, "neighbour export is defined on the FP64 path");
  if (!c->cells_current) {
    st = rebuild(c, 0);
    if (st != SPH_OK) return st;
    // records of dummies hold positions already (fixed); fluid records rebuilt
  }
  hipStream_t s = c->s;
  const int64_t n = c->n, nf = c->nf;
  uint32_t *cnt = (uint32_t *)c->stage;
  uint32_t *off = cnt + (n + 1);
  hipError_t e = launch_fill_u32(cnt, 0u, n + 1, s);
  if (e == hipSuccess)
    e = launch_nb_count_f64(c->P, c->g, c->rec0, c->cs_f, c->cs_d, (uint32_t)nf, c->cur.id, cnt, s, (uint32_t)n);
  if (e == hipSuccess) e = launch_exclusive_scan(cnt, off, n, c->ss.scan_tmp, s);
  std::vector<uint32_t> hoff((size_t)n + 1);
  if (e == hipSuccess) e = hipMemcpyAsync(hoff.data(), off, sizeof(uint32_t) * (n + 1), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  st = hip_check(c, e, "neighbour count");
  if (st != SPH_OK) return st;
  // the u32 scan wraps beyond 4G entries; check monotonicity
  for (int64_t i = 0; i < n; ++i)
    if (hoff[i + 1] < hoff[i]) return fail(c, SPH_ECAPACITY, "too many neighbour entries");
  const int64_t total = hoff[n];
  if (needed) *needed = total;
  for (int64_t i = 0; i <= n; ++i) offsets[i] = hoff[i];
  if (!ids || total > cap) return total > cap ? SPH_ECAPACITY : SPH_OK;
  // fill in chunks of original rows that fit the staging area
  int32_t *chunk = (int32_t *)(off + (n + 1));
  size_t used = sizeof(uint32_t) * 2 * (size_t)(n + 1);
  size_t room = (c->stage_bytes - used - 4096) / sizeof(int32_t);
  room = room / 2;  // half for ids, half for shifted offsets
  int32_t *cids = chunk;
  uint32_t *coff = (uint32_t *)(chunk + room);
  int64_t r0 = 0;
  while (r0 < n) {
    int64_t r1 = r0;
    while (r1 < n && (int64_t)(hoff[r1 + 1] - hoff[r0]) <= (int64_t)room && (r1 - r0) < (int64_t)room - 2) ++r1;
    if (r1 == r0) return fail(c, SPH_ECAPACITY, "a neighbour row exceeds the staging area");
    // offsets relative to the chunk; the fill writes rows [r0, r1) only
    hipLaunchKernelGGL(k_shift_offsets, dim3(grid_for(n + 1)), dim3(kBlock), 0, s, off, hoff[r0], n, coff);
    e = launch_nb_fill_f64(c->P, c->g, c->rec0, c->cs_f, c->cs_d, (uint32_t)nf, c->cur.id, c->dm.id, coff,
                                 (uint32_t)r0, (uint32_t)r1, cids, s);
    if (e == hipSuccess) e = launch_sort_rows(coff, r0, r1, cids, s);
    int64_t cn = hoff[r1] - hoff[r0];
    if (e == hipSuccess && cn > 0)
      e = hipMemcpyAsync(ids + hoff[r0], cids, sizeof(int32_t) * cn, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    st = hip_check(c, e, "neighbour fill");
    if (st != SPH_OK) return st;
    r0 = r1;
  }
  return sync_errors(c);
}

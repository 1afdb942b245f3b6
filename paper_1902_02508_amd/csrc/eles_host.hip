// Host side of the C ABI declared in include/eles.h: descriptor validation,
// layout of the caller-owned state and workspace buffers, and the launch
// sequence of each call. Nothing here touches field data; every step of the
// filter runs in the device kernels.
#include "eles.h"
#include "eles_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

struct eles_filter_s {
  eles_filter_desc d;
  std::vector<double> y;
  int ygemm;
  eles::OpsView v;
  eles::GradView gv;
  eles_state_layout lay;
  int zt, nzt, nxt, n16;
  size_t npts;
  bool ys_ok;          // the staged stress y pass fits this grid
  eles::YsPlan ys;
  bool xzm_ok;         // the matrix-core stress x/z pass covers this grid
  bool xzm_on = true;  // ... and is selected
  eles::XzmPlan xzm;
  // per-pass event timing
  int prof_max = 0, prof_calls = 0;
  unsigned prof_mask = 0;       // passes timed
  std::vector<hipEvent_t> ev;   // [call][pass][start, stop]; null for passes not timed
  std::vector<int> used;        // [call][pass]
};

namespace {

constexpr double kTailFloor = 1e-17;
constexpr int kMaxNy = 8192;

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }
bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

bool kept(double r, double delta, double tau) { return std::exp(-6.0 * r * r / (delta * delta)) >= tau; }

// Largest offset m (in grid spacings) whose kernel value is kept; -1 if huge.
long half_width(int n, double length, double delta, double tau) {
  const double h = length / n;
  const double cut = delta * std::sqrt(std::log(1.0 / tau) / 6.0);
  if (!(cut / h < 1e6)) return -1;
  long m = (long)std::floor(cut / h);
  while (kept((m + 1) * h, delta, tau)) ++m;
  while (m > 0 && !kept(m * h, delta, tau)) --m;
  return m;
}

struct Plan {
  int mx, mz, mpad, kpad, mpx, kpx, mpz, kpz;
  double tau;
  size_t off[32];   // one per state region (O_END <= 32)
  size_t bytes;
};

enum {
  O_Y, O_WP, O_WM, O_WX64, O_WZ64, O_SHIFT, O_WX32, O_WZ32, O_A32, O_AHI, O_ALO, O_RB, O_PROF,
  O_DX32, O_DXHI, O_DXLO, O_DXB, O_DZHI, O_DZLO, O_DY32, O_DYHI, O_DYLO, O_DYB, O_TWX, O_TWZ, O_END
};
static_assert(O_END <= 32, "Plan::off holds 32 regions");

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int32_t plan_filter(const eles_filter_desc *d, Plan *p) {
  if (!d || !d->y) return ELES_EINVAL;
  if (d->nx < 1 || d->nz < 1 || d->ny < 3 || d->ny > kMaxNy) return ELES_EINVAL;
  if ((double)d->nx * d->ny * d->nz > 2147483647.0) return ELES_ENOTSUP;
  if (!finite_pos(d->lx) || !finite_pos(d->lz)) return ELES_EINVAL;
  if (!finite_pos(d->delta_x) || !finite_pos(d->delta_y) || !finite_pos(d->delta_z)) return ELES_EINVAL;
  if (!std::isfinite(d->tail_tol) || d->tail_tol < 0.0 || d->tail_tol > 1e-2) return ELES_EINVAL;
  if (d->ygemm < ELES_YGEMM_FP32 || d->ygemm > ELES_YGEMM_BF16X3) return ELES_EINVAL;
  const double *y = d->y;
  if (y[0] != -1.0 || y[d->ny - 1] != 1.0) return ELES_EINVAL;
  for (int j = 0; j < d->ny; ++j)
    if (!std::isfinite(y[j]) || (j > 0 && !(y[j] > y[j - 1]))) return ELES_EINVAL;
  // g(0) = sqrt(6/(pi D^2)) must stay finite and D^2 must not underflow
  for (double w : {d->delta_x, d->delta_y, d->delta_z})
    if (w < 1e-150 || w > 1e150) return ELES_ENUMERIC;
  p->tau = d->tail_tol > kTailFloor ? d->tail_tol : kTailFloor;
  const long mx = half_width(d->nx, d->lx, d->delta_x, p->tau);
  const long mz = half_width(d->nz, d->lz, d->delta_z, p->tau);
  if (mx < 0 || mz < 0 || mx > eles::kMaxHalfX || mz > eles::kMaxHalfZ) return ELES_ENOTSUP;
  p->mx = (int)mx;
  p->mz = (int)mz;
  p->mpad = (d->ny + eles::kYBlockM - 1) / eles::kYBlockM * eles::kYBlockM;
  p->kpad = (d->ny + eles::kKAlign - 1) / eles::kKAlign * eles::kKAlign;
  p->mpx = (d->nx + 15) / 16 * 16;
  p->kpx = (d->nx + 31) / 32 * 32;
  p->mpz = (d->nz + 15) / 16 * 16;
  p->kpz = (d->nz + 31) / 32 * 32;
  const size_t ny = d->ny, mk = (size_t)p->mpad * p->kpad;
  const size_t mkx = (size_t)p->mpx * p->kpx, mkz = (size_t)p->mpz * p->kpz;
  const size_t sz[O_END] = {
      ny * 8, ny * ny * 8, ny * ny * 8, (size_t)(2 * mx + 1) * 8, (size_t)(2 * mz + 1) * 8, 3 * ny * 8,
      (size_t)eles::tap_pad_len((int)mx) * 4, (size_t)eles::tap_pad_len((int)mz) * 4,
      4 * mk * 4, 4 * mk * 2, 4 * mk * 2, (size_t)p->mpad * 2 * 4, (size_t)p->mpad * 3 * 4,
      mkx * 4, mkx * 2, mkx * 2, (size_t)p->mpx * 2 * 4, mkz * 2, mkz * 2,
      2 * mk * 4, 2 * mk * 2, 2 * mk * 2, (size_t)p->mpad * 2 * 4, (size_t)d->nx * 8, (size_t)d->nz * 8};
  size_t o = 0;
  for (int k = 0; k < O_END; ++k) {
    p->off[k] = o;
    o += up256(sz[k]);
  }
  p->bytes = o;
  return ELES_OK;
}

eles::OpsView make_view(const eles_filter_desc *d, const Plan &p, char *st) {
  eles::OpsView v;
  v.nx = d->nx;
  v.ny = d->ny;
  v.nz = d->nz;
  v.mx = p.mx;
  v.mz = p.mz;
  v.mpad = p.mpad;
  v.kpad = p.kpad;
  v.lx = d->lx;
  v.lz = d->lz;
  v.dx = d->delta_x;
  v.dy = d->delta_y;
  v.dz = d->delta_z;
  v.tau = p.tau;
  v.y64 = (double *)(st + p.off[O_Y]);
  v.wp64 = (double *)(st + p.off[O_WP]);
  v.wm64 = (double *)(st + p.off[O_WM]);
  v.wx64 = (double *)(st + p.off[O_WX64]);
  v.wz64 = (double *)(st + p.off[O_WZ64]);
  v.shift64 = (double *)(st + p.off[O_SHIFT]);
  v.wx32 = (float *)(st + p.off[O_WX32]);
  v.wz32 = (float *)(st + p.off[O_WZ32]);
  const size_t mk = (size_t)p.mpad * p.kpad;
  for (int w = 0; w < 4; ++w) {
    v.a32[w] = (float *)(st + p.off[O_A32]) + w * mk;
    v.ahi[w] = (uint16_t *)(st + p.off[O_AHI]) + w * mk;
    v.alo[w] = (uint16_t *)(st + p.off[O_ALO]) + w * mk;
  }
  v.rowband = (int *)(st + p.off[O_RB]);
  v.prof32 = (float *)(st + p.off[O_PROF]);
  return v;
}

eles::GradView make_grad_view(const eles_filter_desc *d, const Plan &p, char *st) {
  eles::GradView g;
  g.nx = d->nx;
  g.ny = d->ny;
  g.nz = d->nz;
  g.lx = d->lx;
  g.lz = d->lz;
  g.mpx = p.mpx;
  g.kpx = p.kpx;
  g.mpz = p.mpz;
  g.kpz = p.kpz;
  g.mpy = p.mpad;
  g.kpy = p.kpad;
  g.dx32 = (float *)(st + p.off[O_DX32]);
  g.dxhi = (uint16_t *)(st + p.off[O_DXHI]);
  g.dxlo = (uint16_t *)(st + p.off[O_DXLO]);
  g.dxband = (int *)(st + p.off[O_DXB]);
  g.dzhi = (uint16_t *)(st + p.off[O_DZHI]);
  g.dzlo = (uint16_t *)(st + p.off[O_DZLO]);
  const size_t mk = (size_t)p.mpad * p.kpad;
  for (int w = 0; w < 2; ++w) {
    g.dy32[w] = (float *)(st + p.off[O_DY32]) + w * mk;
    g.dyhi[w] = (uint16_t *)(st + p.off[O_DYHI]) + w * mk;
    g.dylo[w] = (uint16_t *)(st + p.off[O_DYLO]) + w * mk;
  }
  g.dyband = (int *)(st + p.off[O_DYB]);
  eles::sder_plan(d->nx, d->lx, false, &g.sx);
  eles::sder_plan(d->nz, d->lz, true, &g.sz);
  g.sx.tw = (float2 *)(st + p.off[O_TWX]);
  g.sz.tw = (float2 *)(st + p.off[O_TWZ]);
  return g;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  const char *pa = (const char *)a, *pb = (const char *)b;
  return pa < pb + nb && pb < pa + na;
}

// Groups of consecutive 16-row tiles for the staged stress y pass, from the
// operators' row bands. A tile walks its K range [lo, hi) in chunks of 16
// from k0 = lo rounded down to 4, moved down (not below 0) so that the walk
// ends by ny rounded up to 4 where it can; a group stages the union of its
// tiles' walks (rows past ny as zeros), next to its products and its
// operator tiles (4 KiB per chunk). Groups grow to maxt tiles
// while the block's LDS stays within budget; false if no plan fits.
bool plan_ys_groups(const std::vector<int> &rb, int ny, int maxt, size_t budget, eles::YsPlan *out) {
  const int ntile = (ny + 15) / 16;
  const int e = (ny + 3) & ~3;
  std::vector<int> k0(ntile), nc(ntile);
  for (int t = 0; t < ntile; ++t) {
    int lo = 1 << 30, hi = 0;
    for (int r = 0; r < 16; ++r) {
      const int a = rb[2 * (16 * t + r)], b = rb[2 * (16 * t + r) + 1];
      if (b > a) {
        lo = std::min(lo, a);
        hi = std::max(hi, b);
      }
    }
    if (hi == 0) lo = 0;
    int s = lo & ~3;
    const int n = (hi - s + 15) >> 4;
    if (s + 16 * n > e) s = std::max(0, e - 16 * n);
    k0[t] = s;
    nc[t] = n;
  }
  eles::YsPlan p;
  std::memset(&p, 0, sizeof(p));
  auto bytes = [](int chunks, int rows) {
    eles::YsPlan q;
    q.max_chunks = chunks;
    q.lds_rows = rows;
    return eles::ys_lds_bytes(q);
  };
  int nchunk = 0;
  for (int t = 0; t < ntile;) {
    if (p.ngroup == eles::kYsMaxGroups) return false;
    const int start = t;
    int kb = 1 << 30, kend = 0, rows = 0, chunks = 0;
    while (t < ntile && t - start < maxt) {
      const int nkb = std::min(kb, k0[t]), nke = std::max(kend, k0[t] + 16 * nc[t]);
      const int nrows = nke - nkb;
      const int nch = chunks + nc[t];
      if (t > start && (nch > eles::kYsMaxGroupChunks ||
                        bytes(std::max(p.max_chunks, nch), std::max(p.lds_rows, nrows)) > budget))
        break;
      kb = nkb;
      kend = nke;
      rows = nrows;
      chunks = nch;
      ++t;
    }
    if (nchunk + chunks > eles::kYsMaxChunks || chunks > eles::kYsMaxGroupChunks) return false;
    const int g = p.ngroup++;
    p.tile0[g] = start;
    p.ntile[g] = t - start;
    p.kb[g] = kb;
    p.nrow[g] = kend - kb;
    p.chunk0[g] = nchunk;
    p.nchunk[g] = chunks;
    for (int u = start; u < t; ++u)
      for (int c = 0; c < nc[u]; ++c)
        p.chunk[nchunk++] = (k0[u] + 16 * c) | ((u - start) << 16) | ((c == nc[u] - 1) << 24);
    p.max_chunks = std::max(p.max_chunks, chunks);
    p.lds_rows = std::max(p.lds_rows, rows);
  }
  if (eles::ys_lds_bytes(p) > budget) return false;
  *out = p;
  return true;
}

// Plane partials per (quantity, row): one per block of a group on the
// staged path, one per (x, 64-column block) on the other.
int sgs_parts(const eles_filter_s *f, bool staged) {
  return staged ? f->ys.nblk / f->ys.ngroup : eles::y_parts(f->d.nx, f->n16);
}

// Workspace of sgs_stress: the nine x/z-filtered fields, then the plane
// partials.
size_t sgs_ws(const eles_filter_s *f, size_t *off_part) {
  const size_t x = up256(9 * f->npts * sizeof(float));
  int parts = sgs_parts(f, false);
  if (f->ys_ok) parts = std::max(parts, sgs_parts(f, true));
  if (off_part) *off_part = x;
  return x + up256((size_t)9 * f->d.ny * parts * sizeof(double));
}

eles::YArgs y_args(const eles_filter_s *f) {
  eles::YArgs a;
  std::memset(&a, 0, sizeof(a));
  for (int w = 0; w < 4; ++w) {
    a.a32[w] = f->v.a32[w];
    a.ahi[w] = f->v.ahi[w];
    a.alo[w] = f->v.alo[w];
  }
  a.rowband = f->v.rowband;
  a.prof32 = f->v.prof32;
  a.nx = f->d.nx;
  a.ny = f->d.ny;
  a.nz = f->d.nz;
  a.mpad = f->v.mpad;
  a.kpad = f->v.kpad;
  a.n16 = f->n16;
  return a;
}

eles::XzArgs xz_args(const eles_filter_s *f) {
  eles::XzArgs a;
  std::memset(&a, 0, sizeof(a));
  a.wx = f->v.wx32;
  a.wz = f->v.wz32;
  a.nx = f->d.nx;
  a.ny = f->d.ny;
  a.nz = f->d.nz;
  a.mx = f->v.mx;
  a.mz = f->v.mz;
  a.zt = f->zt;
  a.nzt = f->nzt;
  a.nxt = f->nxt;
  return a;
}

// Launch one pass, bracketed by timing events when profiling is on.
template <class F>
hipError_t timed(eles_filter_s *f, int pass, hipStream_t s, F &&launch) {
  const bool on = f->prof_max > 0 && f->prof_calls < f->prof_max && ((f->prof_mask >> pass) & 1u);
  const size_t k = ((size_t)f->prof_calls * ELES_NPASS + pass);
  if (on && hipEventRecord(f->ev[2 * k], s) != hipSuccess) return hipErrorUnknown;
  hipError_t e = launch();
  if (e != hipSuccess) return e;
  if (on) {
    if (hipEventRecord(f->ev[2 * k + 1], s) != hipSuccess) return hipErrorUnknown;
    f->used[k] = 1;
  }
  return hipSuccess;
}

void end_call(eles_filter_s *f) {
  if (f->prof_max > 0 && f->prof_calls < f->prof_max) ++f->prof_calls;
}

void release_events(eles_filter_s *f) {
  for (hipEvent_t e : f->ev)
    if (e) (void)hipEventDestroy(e);
  f->ev.clear();
  f->used.clear();
  f->prof_max = f->prof_calls = 0;
  f->prof_mask = 0;
}

}  // namespace

extern "C" {

const char *eles_status_string(int32_t s) {
  switch (s) {
    case ELES_OK: return "ok";
    case ELES_EINVAL: return "invalid argument";
    case ELES_ENOSPACE: return "buffer too small";
    case ELES_EHIP: return "HIP error";
    case ELES_ENUMERIC: return "numerical range";
    case ELES_ENOTSUP: return "not supported";
    default: return "unknown status";
  }
}

size_t filter_state_bytes(const eles_filter_desc *desc) {
  Plan p;
  if (plan_filter(desc, &p) != ELES_OK) return 0;
  return p.bytes;
}

int32_t filter_setup(const eles_filter_desc *desc, void *state, size_t state_bytes, hipStream_t stream,
                     eles_filter *out) {
  if (!out) return ELES_EINVAL;
  *out = nullptr;
  Plan p;
  int32_t st = plan_filter(desc, &p);
  if (st != ELES_OK) return st;
  if (!state || !aligned16(state)) return ELES_EINVAL;
  if (state_bytes < p.bytes) return ELES_ENOSPACE;
  eles_filter_s *f = new (std::nothrow) eles_filter_s;
  if (!f) return ELES_EINVAL;
  f->d = *desc;
  f->y.assign(desc->y, desc->y + desc->ny);
  f->d.y = f->y.data();
  f->ygemm = desc->ygemm;
  f->v = make_view(desc, p, (char *)state);
  f->gv = make_grad_view(desc, p, (char *)state);
  f->npts = (size_t)desc->nx * desc->ny * desc->nz;
  f->zt = eles::xz_tile_z(desc->nz, p.mz);
  f->nzt = (desc->nz + f->zt - 1) / f->zt;
  f->nxt = (desc->nx + eles::kXzTileX - 1) / eles::kXzTileX;
  f->n16 = (desc->nz + eles::kYTileN - 1) / eles::kYTileN;
  eles_state_layout &L = f->lay;
  L.mx = p.mx;
  L.mz = p.mz;
  L.ny_pad_m = p.mpad;
  L.ny_pad_k = p.kpad;
  L.off_wp64 = p.off[O_WP];
  L.off_wm64 = p.off[O_WM];
  L.off_wx64 = p.off[O_WX64];
  L.off_wz64 = p.off[O_WZ64];
  L.off_y64 = p.off[O_Y];
  L.off_shift = p.off[O_SHIFT];
  L.state_bytes = p.bytes;
  if (hipMemcpyAsync(f->v.y64, f->y.data(), desc->ny * sizeof(double), hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      eles::launch_build_ops(f->v, stream) != hipSuccess ||
      eles::launch_build_grad_ops(f->gv, f->v.y64, stream) != hipSuccess ||
      eles::sder_setup(f->gv.sx, stream) != hipSuccess || eles::sder_setup(f->gv.sz, stream) != hipSuccess) {
    delete f;
    return ELES_EHIP;
  }
  // the y-pass plan needs the operators' row bands on the host
  std::vector<int> rb(2 * (size_t)p.mpad);
  if (hipMemcpyAsync(rb.data(), f->v.rowband, rb.size() * sizeof(int), hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    delete f;
    return ELES_EHIP;
  }
  f->ys_ok = false;
  for (size_t budget : {eles::kYsLdsMax}) {
    if (!plan_ys_groups(rb, desc->ny, eles::kYsMaxTiles, budget, &f->ys)) continue;
    f->ys.nblk = eles::ys_grid(f->ys, desc->nz, desc->nx * f->n16);
    f->ys_ok = f->ys.nblk > 0;
    break;
  }
  L.y_groups = f->ys_ok ? f->ys.ngroup : 0;
  L.y_blocks = f->ys_ok ? f->ys.nblk : 0;
  f->xzm_ok = eles::xzm_plan(desc->nx, desc->ny, desc->nz, p.mx, p.mz, &f->xzm);
  L.xz_waves = f->xzm_ok ? f->xzm.nblk * eles::kXzmWaves : 0;
  L.xz_wide = f->xzm_ok && f->xzm.wide ? 1 : 0;
  *out = f;
  return ELES_OK;
}

int32_t filter_set_ygemm(eles_filter f, int32_t ygemm) {
  if (!f || ygemm < ELES_YGEMM_FP32 || ygemm > ELES_YGEMM_BF16X3) return ELES_EINVAL;
  f->ygemm = ygemm;
  return ELES_OK;
}

int32_t filter_set_xz(eles_filter f, int32_t matrix_cores) {
  if (!f || (matrix_cores != 0 && matrix_cores != 1)) return ELES_EINVAL;
  if (matrix_cores && !f->xzm_ok) return ELES_ENOTSUP;
  f->xzm_on = matrix_cores == 1;
  return ELES_OK;
}

int32_t filter_state_layout(eles_filter f, eles_state_layout *out) {
  if (!f || !out) return ELES_EINVAL;
  *out = f->lay;
  return ELES_OK;
}

size_t filter_workspace_bytes(eles_filter f, int32_t nfields) {
  if (!f || nfields < 1) return 0;
  const int g = nfields < 3 ? nfields : 3;
  return up256((size_t)g * f->npts * sizeof(float));
}

size_t sgs_workspace_bytes(eles_filter f) { return f ? sgs_ws(f, nullptr) : 0; }

int32_t filter_fields(eles_filter f, const float *in, int32_t nfields, const int8_t *parity, float *out,
                      void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!f || !in || !out || !parity || !ws || nfields < 1) return ELES_EINVAL;
  if (!aligned16(in) || !aligned16(out) || !aligned16(ws)) return ELES_EINVAL;
  for (int k = 0; k < nfields; ++k)
    if (parity[k] != 1 && parity[k] != -1) return ELES_EINVAL;
  const size_t n = f->npts, bytes = (size_t)nfields * n * sizeof(float);
  if (overlap(in, bytes, out, bytes)) return ELES_EINVAL;
  if (ws_bytes < filter_workspace_bytes(f, nfields)) return ELES_ENOSPACE;
  if (overlap(ws, ws_bytes, in, bytes) || overlap(ws, ws_bytes, out, bytes)) return ELES_EINVAL;
  float *tmp = (float *)ws;
  for (int g0 = 0; g0 < nfields; g0 += 3) {
    const int nc = nfields - g0 < 3 ? nfields - g0 : 3;
    eles::XzArgs xa = xz_args(f);
    xa.in = in + (size_t)g0 * n;
    xa.in_stride = n;
    xa.out = tmp;
    xa.out_nf = nc;
    xa.mshift = nullptr;
    xa.ncomp = nc;
    if (timed(f, 1, stream, [&] { return eles::launch_xz(xa, false, stream); }) != hipSuccess) return ELES_EHIP;
    eles::YArgs ya = y_args(f);
    ya.in = tmp;
    ya.in_fs = f->d.nz;
    ya.in_ks = (size_t)nc * f->d.nz;
    ya.in_xs = (size_t)f->d.ny * ya.in_ks;
    ya.out = out + (size_t)g0 * n;
    ya.out_fs = n;
    ya.out_ks = f->d.nz;
    ya.out_xs = (size_t)f->d.ny * f->d.nz;
    ya.nfield = nc;
    ya.parity_mask = 0;
    for (int k = 0; k < nc; ++k)
      if (parity[g0 + k] < 0) ya.parity_mask |= 1u << k;
    if (timed(f, 2, stream, [&] { return eles::launch_y(ya, false, f->ygemm, stream); }) != hipSuccess)
      return ELES_EHIP;
  }
  end_call(f);
  return ELES_OK;
}

int32_t sgs_stress(eles_filter f, const float *u, float *ubar, float *tau, double *stats, void *ws,
                   size_t ws_bytes, hipStream_t stream) {
  if (!f || !u || !ubar || !tau || !ws) return ELES_EINVAL;
  if (!aligned16(u) || !aligned16(ubar) || !aligned16(tau) || !aligned16(ws) || (stats && !aligned16(stats)))
    return ELES_EINVAL;
  const size_t n = f->npts, fb = n * sizeof(float);
  if (overlap(u, 3 * fb, ubar, 3 * fb) || overlap(u, 3 * fb, tau, 6 * fb) || overlap(ubar, 3 * fb, tau, 6 * fb))
    return ELES_EINVAL;
  size_t off_part = 0;
  const size_t need = sgs_ws(f, &off_part);
  if (ws_bytes < need) return ELES_ENOSPACE;
  if (overlap(ws, need, u, 3 * fb) || overlap(ws, need, ubar, 3 * fb) || overlap(ws, need, tau, 6 * fb) ||
      (stats && overlap(ws, need, stats, 9 * f->d.ny * sizeof(double))))
    return ELES_EINVAL;
  float *X = (float *)ws;
  double *part = stats ? (double *)((char *)ws + off_part) : nullptr;
  if (timed(f, 0, stream, [&] { return eles::launch_shift_ops(f->v, u, stream); }) != hipSuccess)
    return ELES_EHIP;
  eles::XzArgs xa = xz_args(f);
  xa.in = u;
  xa.in_stride = n;
  xa.out = X;
  xa.out_nf = 9;
  xa.mshift = f->v.prof32;
  xa.ncomp = 3;
  if (timed(f, 1, stream, [&] {
        return f->xzm_ok && f->xzm_on ? eles::launch_xzm(xa, f->xzm, stream) : eles::launch_xz(xa, true, stream);
      }) != hipSuccess)
    return ELES_EHIP;
  eles::YArgs ya = y_args(f);
  ya.in = X;
  ya.in_fs = f->d.nz;
  ya.in_ks = (size_t)9 * f->d.nz;
  ya.in_xs = (size_t)f->d.ny * ya.in_ks;
  ya.ubar = ubar;
  ya.tau = tau;
  ya.part = part;
  ya.nfield = 9;
  const bool staged = f->ys_ok && f->ygemm == ELES_YGEMM_FP32;
  if (timed(f, 2, stream, [&] {
        return staged ? eles::launch_ys(ya, f->ys, stream) : eles::launch_y(ya, true, f->ygemm, stream);
      }) != hipSuccess)
    return ELES_EHIP;
  if (stats) {
    const double inv = 1.0 / ((double)f->d.nx * f->d.nz);
    const int nparts = sgs_parts(f, staged);
    if (timed(f, 3, stream, [&] { return eles::launch_stats(part, stats, f->d.ny, nparts, inv, stream); }) !=
        hipSuccess)
      return ELES_EHIP;
  }
  end_call(f);
  return ELES_OK;
}

int32_t filter_profile_begin(eles_filter f, int32_t max_calls, uint32_t pass_mask) {
  if (!f || max_calls < 1 || max_calls > (1 << 20) || pass_mask == 0 || (pass_mask >> ELES_NPASS))
    return ELES_EINVAL;
  release_events(f);
  const size_t n = (size_t)max_calls * ELES_NPASS;
  f->ev.assign(2 * n, nullptr);
  f->used.assign(n, 0);
  for (size_t i = 0; i < f->ev.size(); ++i)
    if (((pass_mask >> ((i / 2) % ELES_NPASS)) & 1u) && hipEventCreate(&f->ev[i]) != hipSuccess) {
      release_events(f);
      return ELES_EHIP;
    }
  f->prof_mask = pass_mask;
  f->prof_max = max_calls;
  f->prof_calls = 0;
  return ELES_OK;
}

int32_t filter_profile_end(eles_filter f, double *ms, int32_t *launches) {
  if (!f || !ms || !launches || f->prof_max == 0) return ELES_EINVAL;
  for (int p = 0; p < ELES_NPASS; ++p) {
    ms[p] = 0.0;
    launches[p] = 0;
  }
  int32_t st = ELES_OK;
  if (hipDeviceSynchronize() != hipSuccess) st = ELES_EHIP;
  for (size_t k = 0; st == ELES_OK && k < f->used.size(); ++k) {
    if (!f->used[k]) continue;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, f->ev[2 * k], f->ev[2 * k + 1]) != hipSuccess) {
      st = ELES_EHIP;
      break;
    }
    ms[k % ELES_NPASS] += t;
    launches[k % ELES_NPASS] += 1;
  }
  release_events(f);
  return st;
}

void filter_destroy(eles_filter f) {
  if (!f) return;
  release_events(f);
  delete f;
}

}  // extern "C"

// ======================================================================
// learned closure
// ======================================================================

struct eles_closure_s {
  eles::ClosureView c;
  double *norm64;     // device copy of the standardisation moments
  long step;          // Adam steps taken so far
  double gm_coef[3];  // gradient-model coefficients (0: the plain network)
};

namespace {

constexpr int kNorm = 2 * eles::kMlpIn + 2 * eles::kMlpOut;   // 32 moments
constexpr int kNrm32 = 2 * eles::kMlpIn + 4 * eles::kMlpOut;  // derived scales and shifts

enum { C_TH, C_M, C_V, C_W1, C_W2, C_W3, C_W4, C_W2T, C_W3T, C_W4T, C_N64, C_N32, C_END };

size_t closure_layout(size_t *off) {
  const int P = eles::kMlpNParam, H = eles::kMlpHidden, K1 = eles::kMlpInPad;
  const size_t sz[C_END] = {(size_t)P * 4, (size_t)P * 4, (size_t)P * 4, (size_t)H * K1 * 2, (size_t)H * H * 2,
                            (size_t)H * H * 2, (size_t)16 * H * 2, (size_t)H * H * 2, (size_t)H * H * 2,
                            (size_t)H * K1 * 2, (size_t)kNorm * 8, (size_t)kNrm32 * 4};
  size_t o = 0;
  for (int k = 0; k < C_END; ++k) {
    if (off) off[k] = o;
    o += up256(sz[k]);
  }
  return o;
}

bool valid_norms(const double *n) {
  for (int k = 0; k < kNorm; ++k)
    if (!std::isfinite(n[k])) return false;
  for (int k = 0; k < eles::kMlpIn; ++k)
    if (!(n[eles::kMlpIn + k] > 0.0)) return false;
  for (int k = 0; k < eles::kMlpOut; ++k)
    if (!(n[2 * eles::kMlpIn + eles::kMlpOut + k] > 0.0)) return false;
  return true;
}

// Gradient-model coefficients of a handle (NULL: none), host and kernel copies.
void set_coef(eles_closure_s *h, const double *c) {
  bool any = false;
  for (int k = 0; k < 3; ++k) {
    h->gm_coef[k] = c ? c[k] : 0.0;
    h->c.gmc[k] = (float)h->gm_coef[k];
    any = any || h->gm_coef[k] != 0.0;
  }
  h->c.use_gm = any ? 1 : 0;
}

bool valid_coef(const double *c) {
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(c[k]) || c[k] < 0.0) return false;
  return true;
}

// Host-side FP32 scale/shift pairs of the standardisation.
void derive_nrm32(const double *n, float *o) {
  const int I = eles::kMlpIn, O = eles::kMlpOut;
  for (int k = 0; k < I; ++k) {
    o[k] = (float)(1.0 / n[I + k]);
    o[I + k] = (float)(-n[k] / n[I + k]);
  }
  for (int k = 0; k < O; ++k) {
    const double mu = n[2 * I + k], sd = n[2 * I + O + k];
    o[2 * I + k] = (float)(1.0 / sd);
    o[2 * I + O + k] = (float)(-mu / sd);
    o[2 * I + 2 * O + k] = (float)sd;
    o[2 * I + 3 * O + k] = (float)mu;
  }
}

size_t train_ws(int batch, eles::TrainWs *w, char *base) {
  const size_t B = batch, H = eles::kMlpHidden, K1 = eles::kMlpInPad;
  const int nch = (batch + eles::kMlpChunk - 1) / eles::kMlpChunk;
  const int mrows[4] = {64, 64, 64, 16}, ncols[4] = {eles::kMlpIn, 64, 64, 64};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + o : nullptr;
    o += up256(bytes);
    return p;
  };
  eles::TrainWs t{};
  t.x0 = (uint16_t *)take(B * K1 * 2);
  t.x0t = (uint16_t *)take(eles::kMlpIn * B * 2);
  t.tb = (float *)take(B * 8 * 4);
  for (int l = 0; l < 3; ++l) {
    t.h[l] = (uint16_t *)take(B * H * 2);
    t.ht[l] = (uint16_t *)take(H * B * 2);
    t.g[l] = (uint16_t *)take(B * H * 2);
    t.dz[l] = (uint16_t *)take(B * H * 2);
    t.dzt[l] = (uint16_t *)take(H * B * 2);
  }
  t.dy = (uint16_t *)take(B * K1 * 2);
  t.dyt = (uint16_t *)take(16 * B * 2);
  for (int l = 0; l < 4; ++l) {
    t.pw[l] = (float *)take((size_t)nch * mrows[l] * ncols[l] * 4);
    t.pb[l] = (float *)take((size_t)nch * mrows[l] * 4);
  }
  t.lossp = (double *)take(B / 16 * 8);
  if (w) *w = t;
  return o;
}

// Workspace of closure_infer: the features (or, for the exact fallback,
// the filtered velocity and sgs_stress's workspace), the plane partials,
// plane sums for the check when the caller passes no stats, the flag.
struct InferWs {
  size_t off_sgs, off_part, off_stats, off_flag;
};

size_t infer_ws(const eles_filter_s *f, bool exact, InferWs *w) {
  const size_t n = f->npts;
  size_t r0 = up256(10 * n * 4);
  const size_t off_sgs = up256(3 * n * 4);
  if (exact) r0 = std::max(r0, off_sgs + sgs_ws(f, nullptr));
  InferWs o;
  o.off_sgs = off_sgs;
  o.off_part = r0;
  // the row sums of the prediction, or the plane-mean partials of the
  // exact stress after a fallback
  const size_t rows = (size_t)6 * f->d.nx * f->d.ny;
  o.off_stats = o.off_part + up256(std::max(rows, (size_t)eles::plane_mean_parts(6, f->d.ny)) * 8);
  o.off_flag = o.off_stats + up256((size_t)6 * f->d.ny * 8);
  if (w) *w = o;
  return o.off_flag + 256;
}

}  // namespace

extern "C" {

size_t closure_state_bytes(void) { return closure_layout(nullptr); }

int32_t closure_create(void *state, size_t state_bytes, const float *params, const double *norms,
                       const double *gm_coef, hipStream_t stream, eles_closure *out) {
  if (!out) return ELES_EINVAL;
  *out = nullptr;
  if (!state || !params || !norms || !aligned16(state)) return ELES_EINVAL;
  if (gm_coef && !valid_coef(gm_coef)) return ELES_ENUMERIC;
  size_t off[C_END];
  const size_t need = closure_layout(off);
  if (state_bytes < need) return ELES_ENOSPACE;
  for (int k = 0; k < eles::kMlpNParam; ++k)
    if (!std::isfinite(params[k])) return ELES_ENUMERIC;
  if (!valid_norms(norms)) return ELES_ENUMERIC;
  eles_closure_s *h = new (std::nothrow) eles_closure_s;
  if (!h) return ELES_EINVAL;
  char *st = (char *)state;
  eles::ClosureView &c = h->c;
  c.theta = (float *)(st + off[C_TH]);
  c.m = (float *)(st + off[C_M]);
  c.v = (float *)(st + off[C_V]);
  c.w1 = (uint16_t *)(st + off[C_W1]);
  c.w2 = (uint16_t *)(st + off[C_W2]);
  c.w3 = (uint16_t *)(st + off[C_W3]);
  c.w4 = (uint16_t *)(st + off[C_W4]);
  c.w2t = (uint16_t *)(st + off[C_W2T]);
  c.w3t = (uint16_t *)(st + off[C_W3T]);
  c.w4t = (uint16_t *)(st + off[C_W4T]);
  h->norm64 = (double *)(st + off[C_N64]);
  float *n32 = (float *)(st + off[C_N32]);
  const int I = eles::kMlpIn, O = eles::kMlpOut;
  c.fsc = n32;
  c.fsh = n32 + I;
  c.tsc = n32 + 2 * I;
  c.tsh = n32 + 2 * I + O;
  c.isc = n32 + 2 * I + 2 * O;
  c.ish = n32 + 2 * I + 3 * O;
  h->step = 0;
  set_coef(h, gm_coef);
  float nrm[kNrm32];
  derive_nrm32(norms, nrm);
  const size_t pbytes = (size_t)eles::kMlpNParam * 4;
  bool ok = hipMemsetAsync(st, 0, need, stream) == hipSuccess &&
            hipMemcpyAsync(c.theta, params, pbytes, hipMemcpyHostToDevice, stream) == hipSuccess &&
            hipMemcpyAsync(h->norm64, norms, kNorm * 8, hipMemcpyHostToDevice, stream) == hipSuccess &&
            hipMemcpyAsync(n32, nrm, sizeof(nrm), hipMemcpyHostToDevice, stream) == hipSuccess &&
            eles::launch_shadows(c, stream) == hipSuccess && hipStreamSynchronize(stream) == hipSuccess;
  if (!ok) {
    delete h;
    return ELES_EHIP;
  }
  *out = h;
  return ELES_OK;
}

int64_t closure_step(eles_closure c) { return c ? c->step : -1; }

size_t closure_blob_bytes(void) { return (size_t)3 * eles::kMlpNParam * 4 + kNorm * 8 + 8 + 3 * 8; }

int32_t closure_get_params(eles_closure c, void *blob, size_t bytes, hipStream_t stream) {
  if (!c || !blob || bytes < closure_blob_bytes()) return ELES_EINVAL;
  const size_t pb = (size_t)eles::kMlpNParam * 4;
  char *b = (char *)blob;
  // stream-ordered copies; the host reads the blob, so the call waits for
  // the stream
  if (hipMemcpyAsync(b, c->c.theta, pb, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(b + pb, c->c.m, pb, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(b + 2 * pb, c->c.v, pb, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(b + 3 * pb, c->norm64, kNorm * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return ELES_EHIP;
  int64_t st = c->step;
  std::memcpy(b + 3 * pb + kNorm * 8, &st, 8);
  std::memcpy(b + 3 * pb + kNorm * 8 + 8, c->gm_coef, 3 * 8);
  return ELES_OK;
}

int32_t closure_set_params(eles_closure c, const void *blob, size_t bytes, hipStream_t stream) {
  if (!c || !blob || bytes < closure_blob_bytes()) return ELES_EINVAL;
  const size_t pb = (size_t)eles::kMlpNParam * 4;
  const char *b = (const char *)blob;
  const float *f = (const float *)b;
  for (int k = 0; k < 3 * eles::kMlpNParam; ++k)
    if (!std::isfinite(f[k])) return ELES_ENUMERIC;
  const double *n = (const double *)(b + 3 * pb);
  if (!valid_norms(n)) return ELES_ENUMERIC;
  int64_t st;
  std::memcpy(&st, b + 3 * pb + kNorm * 8, 8);
  if (st < 0) return ELES_EINVAL;
  double coef[3];
  std::memcpy(coef, b + 3 * pb + kNorm * 8 + 8, 3 * 8);
  if (!valid_coef(coef)) return ELES_ENUMERIC;
  float nrm[kNrm32];
  derive_nrm32(n, nrm);
  // stream-ordered after the work already queued on the handle; the call
  // waits for the stream because the copies read host memory the caller
  // (and this frame, for nrm) may release on return
  if (hipMemcpyAsync(c->c.theta, b, pb, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(c->c.m, b + pb, pb, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(c->c.v, b + 2 * pb, pb, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(c->norm64, n, kNorm * 8, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync((void *)c->c.fsc, nrm, sizeof(nrm), hipMemcpyHostToDevice, stream) != hipSuccess ||
      eles::launch_shadows(c->c, stream) != hipSuccess || hipStreamSynchronize(stream) != hipSuccess)
    return ELES_EHIP;
  c->step = st;
  set_coef(c, coef);
  return ELES_OK;
}

// d/dx by the dense spectral operator through the y-pass kernel, the field
// seen as one [nx] x [ny nz] slab (BF16x3 products)
int32_t dense_dx(eles_filter f, const float *ubar, float *feat, hipStream_t stream) {
  const size_t n = f->npts;
  const int nx = f->d.nx, ny = f->d.ny, nz = f->d.nz;
  const eles::GradView &g = f->gv;
  eles::YArgs ya = y_args(f);
  for (int w = 0; w < 4; ++w) {
    ya.a32[w] = g.dx32;
    ya.ahi[w] = g.dxhi;
    ya.alo[w] = g.dxlo;
  }
  ya.rowband = g.dxband;
  ya.mpad = g.mpx;
  ya.kpad = g.kpx;
  ya.nx = 1;
  ya.ny = nx;
  ya.nz = ny * nz;
  ya.n16 = (ny * nz + eles::kYTileN - 1) / eles::kYTileN;
  ya.nfield = 3;
  ya.parity_mask = 0;
  ya.in = ubar;
  ya.in_fs = n;
  ya.in_xs = 0;
  ya.in_ks = (size_t)ny * nz;
  ya.out = feat;
  ya.out_fs = 3 * n;
  ya.out_xs = 0;
  ya.out_ks = (size_t)ny * nz;
  return eles::launch_y(ya, false, ELES_YGEMM_BF16X3, stream) == hipSuccess ? ELES_OK : ELES_EHIP;
}

// features 0..8 (the velocity gradient) and, with walldist, feature 9
int32_t gradient_features(eles_filter f, const float *ubar, float *feat, bool walldist, hipStream_t stream) {
  const size_t n = f->npts;
  const int nx = f->d.nx, ny = f->d.ny, nz = f->d.nz;
  const eles::GradView &g = f->gv;
  // d/dx: fast transforms along x where nx factors into 2, 3 and 5, else
  // the dense spectral operator, the field seen as one [nx] x [ny nz] slab
  if (g.sx.nrad) {
    if (eles::launch_sder(g, false, ubar, feat, (long)(3 * n), stream) != hipSuccess) return ELES_EHIP;
  } else if (dense_dx(f, ubar, feat, stream) != ELES_OK) {
    return ELES_EHIP;
  }
  // d/dz with d/dy from the same staged rows where the fused kernel covers
  // the grid
  if (eles::sder_zy_ok(g)) {
    if (eles::launch_sder_zy(g, ubar, feat + 2 * n, feat + n, (long)(3 * n), 0x2, stream) != hipSuccess)
      return ELES_EHIP;
    if (walldist && eles::launch_walldist(f->v.y64, nx, ny, nz, feat + 9 * n, stream) != hipSuccess)
      return ELES_EHIP;
    return ELES_OK;
  }
  // d/dy: three-point difference with the parities of (u1, u2, u3),
  // streamed along each column (grids of three or more rows)
  if (ny >= 3) {
    if (eles::launch_ddy(g, ubar, feat + n, (long)(3 * n), 0x2, stream) != hipSuccess) return ELES_EHIP;
  } else {
    eles::YArgs yb = y_args(f);
    yb.a32[0] = g.dy32[0];
    yb.a32[1] = g.dy32[1];
    yb.ahi[0] = g.dyhi[0];
    yb.ahi[1] = g.dyhi[1];
    yb.alo[0] = g.dylo[0];
    yb.alo[1] = g.dylo[1];
    yb.rowband = g.dyband;
    yb.nfield = 3;
    yb.parity_mask = 0x2;
    yb.in = ubar;
    yb.in_fs = n;
    yb.in_xs = (size_t)ny * nz;
    yb.in_ks = nz;
    yb.out = feat + n;
    yb.out_fs = 3 * n;
    yb.out_xs = (size_t)ny * nz;
    yb.out_ks = nz;
    if (eles::launch_y(yb, false, ELES_YGEMM_FP32, stream) != hipSuccess) return ELES_EHIP;
  }
  // d/dz: fast transforms along the rows, else rows times the transposed
  // dense spectral operator
  if (g.sz.nrad) {
    if (eles::launch_sder(g, true, ubar, feat + 2 * n, (long)(3 * n), stream) != hipSuccess) return ELES_EHIP;
  } else if (eles::launch_dz(g, ubar, feat + 2 * n, (long)(3 * n), stream) != hipSuccess) {
    return ELES_EHIP;
  }
  if (walldist && eles::launch_walldist(f->v.y64, nx, ny, nz, feat + 9 * n, stream) != hipSuccess)
    return ELES_EHIP;
  return ELES_OK;
}

int32_t closure_features(eles_filter f, const float *ubar, float *feat, hipStream_t stream) {
  if (!f || !ubar || !feat || !aligned16(ubar) || !aligned16(feat)) return ELES_EINVAL;
  const size_t n = f->npts;
  if (overlap(ubar, 3 * n * 4, feat, 10 * n * 4)) return ELES_EINVAL;
  return gradient_features(f, ubar, feat, true, stream);
}

size_t closure_moments_workspace_bytes(int32_t nchan) {
  return nchan < 1 ? 0 : up256((size_t)nchan * 1024 * 8);
}

int32_t closure_moments(const float *data, int32_t nchan, int32_t nsnap, int64_t npts, double *out, void *ws,
                        size_t ws_bytes, hipStream_t stream) {
  if (!data || !out || !ws || nchan < 1 || nchan > 64 || nsnap < 1 || npts < 1) return ELES_EINVAL;
  if (ws_bytes < closure_moments_workspace_bytes(nchan)) return ELES_ENOSPACE;
  return eles::launch_moments(data, nchan, nsnap, (long)npts, (double *)ws, 1024, out, stream) == hipSuccess
             ? ELES_OK
             : ELES_EHIP;
}

size_t closure_train_workspace_bytes(int32_t batch) {
  if (batch < 32 || batch % 32) return 0;
  return train_ws(batch, nullptr, nullptr);
}

int32_t closure_train(eles_closure c, const float *feat, const float *tau, int32_t nsnap, int64_t npts,
                      const eles_train_desc *td, float *loss_hist, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!c || !feat || !tau || !td || !ws || nsnap < 1 || npts < 1) return ELES_EINVAL;
  if (td->batch < 32 || td->batch % 32 || td->steps < 0) return ELES_EINVAL;
  if (!(td->lr > 0.0f) || !(td->beta1 >= 0.0f && td->beta1 < 1.0f) || !(td->beta2 >= 0.0f && td->beta2 < 1.0f) ||
      !(td->eps > 0.0f))
    return ELES_EINVAL;
  if ((double)nsnap * npts > 4294967295.0) return ELES_ENOTSUP;
  if (ws_bytes < closure_train_workspace_bytes(td->batch)) return ELES_ENOSPACE;
  eles::TrainWs w;
  train_ws(td->batch, &w, (char *)ws);
  if (hipMemsetAsync(w.dy, 0, (size_t)td->batch * eles::kMlpInPad * 2, stream) != hipSuccess) return ELES_EHIP;
  eles::TrainData d{feat, tau, nsnap, (long)npts};
  for (int s = 0; s < td->steps; ++s) {
    const long t = c->step + s + 1;
    eles::AdamArgs a{};
    a.lr = td->lr;
    a.b1 = td->beta1;
    a.b2 = td->beta2;
    a.eps = td->eps;
    a.bc1 = (float)(1.0 / (1.0 - std::pow((double)td->beta1, (double)t)));
    a.bc2 = (float)(1.0 / (1.0 - std::pow((double)td->beta2, (double)t)));
    a.loss_out = loss_hist ? loss_hist + s : nullptr;
    if (eles::launch_train_step(c->c, d, w, td->seed, t - 1, td->batch, a, stream) != hipSuccess) return ELES_EHIP;
  }
  c->step += td->steps;
  return ELES_OK;
}

size_t closure_infer_workspace_bytes(eles_filter f, int32_t with_fallback) {
  return f ? infer_ws(f, with_fallback != 0, nullptr) : 0;
}

int32_t closure_infer(eles_closure c, eles_filter f, const float *ubar, float *tau_pred, double *stats,
                      int32_t fallback, const float *u_or_null, int32_t *fell_back, void *ws, size_t ws_bytes,
                      hipStream_t stream) {
  if (fell_back) *fell_back = 0;
  if (!c || !f || !ubar || !tau_pred || !ws || !aligned16(tau_pred) || !aligned16(ws) ||
      (stats && !aligned16(stats)))
    return ELES_EINVAL;
  if (fallback < ELES_INFER_UNCHECKED || fallback > ELES_INFER_FALLBACK) return ELES_EINVAL;
  const bool checked = fallback != ELES_INFER_UNCHECKED, exact = fallback == ELES_INFER_FALLBACK;
  if (exact && (!u_or_null || !aligned16(u_or_null))) return ELES_EINVAL;
  InferWs w;
  const size_t need = infer_ws(f, exact, &w);
  if (ws_bytes < need) return ELES_ENOSPACE;
  const size_t n = f->npts, sb = (size_t)6 * f->d.ny * sizeof(double);
  if (overlap(ubar, 3 * n * 4, tau_pred, 6 * n * 4) || overlap(ws, need, tau_pred, 6 * n * 4) ||
      overlap(ws, need, ubar, 3 * n * 4) || (stats && (overlap(stats, sb, ws, need) ||
                                                       overlap(stats, sb, tau_pred, 6 * n * 4))))
    return ELES_EINVAL;
  if (exact && (overlap(u_or_null, 3 * n * 4, tau_pred, 6 * n * 4) || overlap(u_or_null, 3 * n * 4, ws, need)))
    return ELES_EINVAL;
  char *base = (char *)ws;
  float *feat = (float *)base;
  double *part = (double *)(base + w.off_part);
  // the network computes the wall distance itself
  int32_t st = gradient_features(f, ubar, feat, false, stream);
  if (st != ELES_OK) return st;
  // plane means: the caller's stats, or (for the check alone) the
  // workspace's, from the network kernel's row sums
  double *sums = stats ? stats : (checked ? (double *)(base + w.off_stats) : nullptr);
  if (eles::launch_infer(c->c, feat, f->d.nx, f->d.ny, f->d.nz, f->v.y64, tau_pred, sums ? part : nullptr,
                         stream) != hipSuccess)
    return ELES_EHIP;
  if (sums && eles::launch_row_means(part, 6, f->d.nx, f->d.ny, f->d.nz, sums, stream) != hipSuccess)
    return ELES_EHIP;
  if (!checked) return ELES_OK;
  // a NaN or infinity anywhere in tau_pred makes its plane's FP64 sum
  // non-finite; the host reads the device flag back
  int32_t bad = 0;
  int *flag = (int *)(base + w.off_flag);
  if (eles::launch_nonfinite(sums, 6 * f->d.ny, flag, stream) != hipSuccess ||
      hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return ELES_EHIP;
  if (!bad) return ELES_OK;
  if (!exact) return ELES_ENUMERIC;
  // the exact stress replaces the prediction: sgs_stress into tau_pred, its
  // filtered velocity and workspace in the (now free) feature region
  float *ub_exact = (float *)base;
  st = sgs_stress(f, u_or_null, ub_exact, tau_pred, nullptr, base + w.off_sgs, sgs_ws(f, nullptr), stream);
  if (st != ELES_OK) return st;
  if (stats && eles::launch_plane_mean(tau_pred, 6, f->d.nx, f->d.ny, f->d.nz, part, stats, stream) != hipSuccess)
    return ELES_EHIP;
  if (fell_back) *fell_back = 1;
  return ELES_OK;
}

int32_t closure_sample_indices(uint64_t seed, int64_t step, int32_t batch, uint64_t count, int64_t *out,
                               hipStream_t stream) {
  if (!out || batch < 1 || step < 0 || count < 1 || count > 4294967296ull) return ELES_EINVAL;
  return eles::launch_sample(seed, (long)step, batch, count, out, stream) == hipSuccess ? ELES_OK : ELES_EHIP;
}

void closure_destroy(eles_closure c) { delete c; }

}  // extern "C"

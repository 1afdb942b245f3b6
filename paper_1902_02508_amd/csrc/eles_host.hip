// Host side of the C ABI declared in include/eles.h: descriptor validation,
// layout of the caller-owned state and workspace buffers, and the launch
// sequence of each call. Nothing here touches field data; every step of the
// filter runs in the device kernels.
#include "eles.h"
#include "eles_internal.h"

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

struct eles_filter_s {
  eles_filter_desc d;
  std::vector<double> y;
  int ygemm;
  eles::OpsView v;
  eles_state_layout lay;
  int zt, nzt, nxt, n16;
  size_t npts;
  // per-pass event timing
  int prof_max = 0, prof_calls = 0;
  std::vector<hipEvent_t> ev;   // [call][pass][start, stop]
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
  int mx, mz, mpad, kpad;
  double tau;
  size_t off[16];
  size_t bytes;
};

enum { O_Y, O_WP, O_WM, O_WX64, O_WZ64, O_SHIFT, O_WX32, O_WZ32, O_A32, O_AHI, O_ALO, O_RB, O_PROF, O_END };

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
  const size_t ny = d->ny, mk = (size_t)p->mpad * p->kpad;
  const size_t sz[O_END] = {
      ny * 8, ny * ny * 8, ny * ny * 8, (size_t)(2 * mx + 1) * 8, (size_t)(2 * mz + 1) * 8, 3 * ny * 8,
      (size_t)eles::tap_pad_len((int)mx) * 4, (size_t)eles::tap_pad_len((int)mz) * 4,
      4 * mk * 4, 4 * mk * 2, 4 * mk * 2, (size_t)p->mpad * 2 * 4, (size_t)p->mpad * 3 * 4};
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

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  const char *pa = (const char *)a, *pb = (const char *)b;
  return pa < pb + nb && pb < pa + na;
}

size_t sgs_ws(const eles_filter_s *f, size_t *off_part) {
  const size_t x = up256(9 * f->npts * sizeof(float));
  if (off_part) *off_part = x;
  return x + up256((size_t)9 * f->d.ny * eles::y_parts(f->d.nx, f->n16) * sizeof(double));
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
  const bool on = f->prof_max > 0 && f->prof_calls < f->prof_max;
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
    if (e) hipEventDestroy(e);
  f->ev.clear();
  f->used.clear();
  f->prof_max = f->prof_calls = 0;
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
      eles::launch_build_ops(f->v, stream) != hipSuccess) {
    delete f;
    return ELES_EHIP;
  }
  *out = f;
  return ELES_OK;
}

int32_t filter_set_ygemm(eles_filter f, int32_t ygemm) {
  if (!f || ygemm < ELES_YGEMM_FP32 || ygemm > ELES_YGEMM_BF16X3) return ELES_EINVAL;
  f->ygemm = ygemm;
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
    ya.in_nf = nc;
    ya.out = out + (size_t)g0 * n;
    ya.out_stride = n;
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
  if (timed(f, 1, stream, [&] { return eles::launch_xz(xa, true, stream); }) != hipSuccess) return ELES_EHIP;
  eles::YArgs ya = y_args(f);
  ya.in = X;
  ya.in_nf = 9;
  ya.ubar = ubar;
  ya.tau = tau;
  ya.part = part;
  ya.nfield = 9;
  if (timed(f, 2, stream, [&] { return eles::launch_y(ya, true, f->ygemm, stream); }) != hipSuccess)
    return ELES_EHIP;
  if (stats) {
    const int nparts = eles::y_parts(f->d.nx, f->n16);
    const double inv = 1.0 / ((double)f->d.nx * f->d.nz);
    if (timed(f, 3, stream, [&] { return eles::launch_stats(part, stats, f->d.ny, nparts, inv, stream); }) !=
        hipSuccess)
      return ELES_EHIP;
  }
  end_call(f);
  return ELES_OK;
}

int32_t filter_profile_begin(eles_filter f, int32_t max_calls) {
  if (!f || max_calls < 1 || max_calls > (1 << 20)) return ELES_EINVAL;
  release_events(f);
  const size_t n = (size_t)max_calls * ELES_NPASS;
  f->ev.assign(2 * n, nullptr);
  f->used.assign(n, 0);
  for (auto &e : f->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      release_events(f);
      return ELES_EHIP;
    }
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

// Host side of the differential-filter part of the C ABI (include/eles.h):
// descriptor validation, layout of the caller-owned state and workspace,
// and the launch sequence of each call. Every step of the filter runs in
// the kernels of k_dfilt.hip.
#include "eles.h"
#include "eles_internal.h"

#include <cmath>
#include <new>
#include <vector>

struct eles_dfilter_s {
  eles_dfilter_desc d;
  std::vector<double> y;
  eles::DView v;
  size_t npts;
  // timing: events [call][pass][start, stop], used flags [call][pass]
  int prof_max = 0, prof_calls = 0;
  unsigned prof_mask = 0;   // passes timed; the events of the others stay null
  std::vector<hipEvent_t> ev;
  std::vector<char> used;
};

namespace {

static_assert(eles::kDPasses == ELES_DNPASS, "pass count");

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// events of the next call, marking the passes it times; null when off
const hipEvent_t *call_events(eles_dfilter_s *f, bool sgs) {
  if (f->prof_max == 0 || f->prof_calls >= f->prof_max) return nullptr;
  const size_t base = (size_t)f->prof_calls * ELES_DNPASS;
  for (int p = 0; p < ELES_DNPASS; ++p)
    f->used[base + p] = ((f->prof_mask >> p) & 1u) && (sgs || (p != eles::kDPassShift && p != eles::kDPassEpi));
  ++f->prof_calls;
  return f->ev.data() + 2 * base;
}

void release_events(eles_dfilter_s *f) {
  for (hipEvent_t e : f->ev)
    if (e) (void)hipEventDestroy(e);
  f->ev.clear();
  f->used.clear();
  f->prof_max = f->prof_calls = 0;
  f->prof_mask = 0;
}
bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  const char *pa = (const char *)a, *pb = (const char *)b;
  return pa < pb + nb && pb < pa + na;
}

enum { D_Y, D_D64, D_P64, D_S64, D_FX, D_IX, D_FZ, D_IZ, D_LO, D_OP, D_CP, D_INV, D_PROF, D_TWX, D_TWZ, D_END };

struct DPlan {
  eles::DAxis ax, az;
  int hx, hz;
  size_t off[D_END];
  size_t bytes;
};

int32_t plan_d(const eles_dfilter_desc *d, DPlan *p) {
  if (!d || !d->y) return ELES_EINVAL;
  if (d->nx < eles::kDMinN || d->nz < eles::kDMinN || d->ny < 4 || d->ny > 8192) return ELES_EINVAL;
  if (!(std::isfinite(d->lx) && d->lx > 0) || !(std::isfinite(d->lz) && d->lz > 0)) return ELES_EINVAL;
  if (!(std::isfinite(d->a) && d->a > 0)) return ELES_EINVAL;
  const double *y = d->y;
  if (y[0] != -1.0 || y[d->ny - 1] != 1.0) return ELES_EINVAL;
  for (int j = 0; j < d->ny; ++j)
    if (!std::isfinite(y[j]) || (j > 0 && !(y[j] > y[j - 1]))) return ELES_EINVAL;
  // the transforms address one field through 32-bit byte offsets
  if ((double)d->nx * d->ny * d->nz * 4.0 >= 2147483648.0) return ELES_ENOTSUP;
  p->ax = eles::daxis(d->nx);
  p->az = eles::daxis(d->nz);
  p->hx = d->nx / 2;
  p->hz = d->nz / 2;
  const size_t ny = d->ny;
  const size_t nfac = 2 * (size_t)(p->hx + 1) * (p->hz + 1) * ny;
  const size_t sz[D_END] = {ny * 8,
                            6 * ny * 8,
                            3 * ny * 8,
                            3 * ny * 8,
                            eles::dtab_fwd_floats(p->ax) * 4,
                            eles::dtab_inv_floats(p->ax) * 4,
                            eles::dtab_fwd_floats(p->az) * 4,
                            eles::dtab_inv_floats(p->az) * 4,
                            2 * ny * 4,
                            6 * ny * 4,
                            nfac * 4,
                            nfac * 4,
                            3 * ny * 4,
                            (size_t)d->nx * 8,
                            (size_t)d->nz * 8};
  size_t o = 0;
  for (int k = 0; k < D_END; ++k) {
    p->off[k] = o;
    o += up256(sz[k]);
  }
  p->bytes = o;
  return ELES_OK;
}

}  // namespace

extern "C" {

size_t dfilter_state_bytes(const eles_dfilter_desc *desc) {
  DPlan p;
  return plan_d(desc, &p) == ELES_OK ? p.bytes : 0;
}

int32_t dfilter_setup(const eles_dfilter_desc *desc, void *state, size_t state_bytes, hipStream_t stream,
                      eles_dfilter *out) {
  if (!out) return ELES_EINVAL;
  DPlan p;
  const int32_t st = plan_d(desc, &p);
  if (st != ELES_OK) return st;
  if (!state || !aligned16(state)) return ELES_EINVAL;
  if (state_bytes < p.bytes) return ELES_ENOSPACE;
  eles_dfilter_s *f = new (std::nothrow) eles_dfilter_s;
  if (!f) return ELES_EINVAL;
  f->d = *desc;
  f->y.assign(desc->y, desc->y + desc->ny);
  f->d.y = f->y.data();
  f->npts = (size_t)desc->nx * desc->ny * desc->nz;
  char *s = (char *)state;
  eles::DView &v = f->v;
  v.nx = desc->nx;
  v.ny = desc->ny;
  v.nz = desc->nz;
  v.hx = p.hx;
  v.hz = p.hz;
  v.ax = p.ax;
  v.az = p.az;
  v.lx = desc->lx;
  v.lz = desc->lz;
  v.a = desc->a;
  v.y64 = (double *)(s + p.off[D_Y]);
  v.d64 = (double *)(s + p.off[D_D64]);
  v.p64 = (double *)(s + p.off[D_P64]);
  v.scratch64 = (double *)(s + p.off[D_S64]);
  v.fx = (float *)(s + p.off[D_FX]);
  v.ix = (float *)(s + p.off[D_IX]);
  v.fz = (float *)(s + p.off[D_FZ]);
  v.iz = (float *)(s + p.off[D_IZ]);
  v.lo32 = (float *)(s + p.off[D_LO]);
  v.op32 = (float *)(s + p.off[D_OP]);
  v.cp = (float *)(s + p.off[D_CP]);
  v.inv = (float *)(s + p.off[D_INV]);
  v.prof = (float *)(s + p.off[D_PROF]);
  // fast transforms where both periodic lengths factor into 2, 3 and 5
  if (!eles::sder_plan(v.nx, v.lx, false, &v.rx) || !eles::sder_plan(v.nz, v.lz, true, &v.rz))
    v.rx.nrad = v.rz.nrad = 0;
  v.rx.tw = (float2 *)(s + p.off[D_TWX]);
  v.rz.tw = (float2 *)(s + p.off[D_TWZ]);
  if (eles::dfilter_lds_limit(v) != hipSuccess || eles::rfft_setup(v.rx, stream) != hipSuccess ||
      eles::rfft_setup(v.rz, stream) != hipSuccess ||
      hipMemcpyAsync(v.y64, f->y.data(), f->y.size() * sizeof(double), hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      eles::launch_dsetup(v, stream) != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) {
    delete f;
    return ELES_EHIP;
  }
  *out = f;
  return ELES_OK;
}

size_t dfilter_workspace_bytes(eles_dfilter f, int32_t nfields) {
  if (!f || nfields < 1 || nfields > 32) return 0;
  return 2 * up256((size_t)nfields * f->npts * sizeof(float));
}

size_t dfilter_sgs_workspace_bytes(eles_dfilter f) {
  if (!f) return 0;
  return 2 * up256((size_t)eles::kDFields * f->npts * sizeof(float)) +
         up256((size_t)eles::dsgs_parts(f->v) * sizeof(double));
}

int32_t dfilter_fields(eles_dfilter f, const float *in, int32_t nfields, const int8_t *parity, float *out,
                       void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!f || !in || !out || !parity || !ws || nfields < 1 || nfields > 32) return ELES_EINVAL;
  if (!aligned16(in) || !aligned16(out) || !aligned16(ws)) return ELES_EINVAL;
  unsigned pmask = 0;
  for (int k = 0; k < nfields; ++k) {
    if (parity[k] != 1 && parity[k] != -1) return ELES_EINVAL;
    if (parity[k] < 0) pmask |= 1u << k;
  }
  const size_t bytes = (size_t)nfields * f->npts * sizeof(float);
  if (overlap(in, bytes, out, bytes)) return ELES_EINVAL;
  if (ws_bytes < dfilter_workspace_bytes(f, nfields)) return ELES_ENOSPACE;
  if (overlap(ws, ws_bytes, in, bytes) || overlap(ws, ws_bytes, out, bytes)) return ELES_EINVAL;
  float *w0 = (float *)ws;
  float *w1 = (float *)((char *)ws + up256(bytes));
  return eles::launch_dfilter(f->v, in, nfields, pmask, w0, w1, out, stream, call_events(f, false)) == hipSuccess
             ? ELES_OK
             : ELES_EHIP;
}

int32_t dfilter_sgs_stress(eles_dfilter f, const float *u, float *ubar, float *tau, double *stats, void *ws,
                           size_t ws_bytes, hipStream_t stream) {
  if (!f || !u || !ubar || !tau || !ws) return ELES_EINVAL;
  if (!aligned16(u) || !aligned16(ubar) || !aligned16(tau) || !aligned16(ws)) return ELES_EINVAL;
  if (stats && ((uintptr_t)stats & 7u)) return ELES_EINVAL;
  const size_t n = f->npts;
  if (overlap(u, 3 * n * 4, ubar, 3 * n * 4) || overlap(u, 3 * n * 4, tau, 6 * n * 4) ||
      overlap(ubar, 3 * n * 4, tau, 6 * n * 4))
    return ELES_EINVAL;
  if (ws_bytes < dfilter_sgs_workspace_bytes(f)) return ELES_ENOSPACE;
  if (overlap(ws, ws_bytes, u, 3 * n * 4) || overlap(ws, ws_bytes, ubar, 3 * n * 4) ||
      overlap(ws, ws_bytes, tau, 6 * n * 4))
    return ELES_EINVAL;
  const size_t fb = up256((size_t)eles::kDFields * n * sizeof(float));
  float *w0 = (float *)ws;
  float *w1 = (float *)((char *)ws + fb);
  double *part = (double *)((char *)ws + 2 * fb);
  return eles::launch_dsgs(f->v, u, w0, w1, ubar, tau, part, stats, stream, call_events(f, true)) == hipSuccess
             ? ELES_OK
             : ELES_EHIP;
}

int32_t dfilter_profile_begin(eles_dfilter f, int32_t max_calls, uint32_t pass_mask) {
  if (!f || max_calls < 1 || max_calls > (1 << 20) || pass_mask == 0 || (pass_mask >> ELES_DNPASS))
    return ELES_EINVAL;
  release_events(f);
  const size_t n = (size_t)max_calls * ELES_DNPASS;
  f->ev.assign(2 * n, nullptr);
  f->used.assign(n, 0);
  for (size_t i = 0; i < f->ev.size(); ++i)
    if (((pass_mask >> ((i / 2) % ELES_DNPASS)) & 1u) && hipEventCreate(&f->ev[i]) != hipSuccess) {
      release_events(f);
      return ELES_EHIP;
    }
  f->prof_mask = pass_mask;
  f->prof_max = max_calls;
  f->prof_calls = 0;
  return ELES_OK;
}

int32_t dfilter_profile_end(eles_dfilter f, double *ms, int32_t *launches) {
  if (!f || !ms || !launches || f->prof_max == 0) return ELES_EINVAL;
  for (int p = 0; p < ELES_DNPASS; ++p) {
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
    ms[k % ELES_DNPASS] += t;
    launches[k % ELES_DNPASS] += 1;
  }
  release_events(f);
  return st;
}

int32_t dfilter_inverse(eles_dfilter f, const float *in, int32_t nfields, const int8_t *parity, float *out,
                        void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!f || !in || !out || !parity || !ws || nfields < 1 || nfields > 32) return ELES_EINVAL;
  if (!aligned16(in) || !aligned16(out) || !aligned16(ws)) return ELES_EINVAL;
  unsigned pmask = 0;
  for (int k = 0; k < nfields; ++k) {
    if (parity[k] != 1 && parity[k] != -1) return ELES_EINVAL;
    if (parity[k] < 0) pmask |= 1u << k;
  }
  const size_t bytes = (size_t)nfields * f->npts * sizeof(float);
  if (overlap(in, bytes, out, bytes)) return ELES_EINVAL;
  if (ws_bytes < dfilter_workspace_bytes(f, nfields)) return ELES_ENOSPACE;
  if (overlap(ws, ws_bytes, in, bytes) || overlap(ws, ws_bytes, out, bytes)) return ELES_EINVAL;
  float *w0 = (float *)ws;
  float *w1 = (float *)((char *)ws + up256(bytes));
  return eles::launch_dinverse(f->v, in, nfields, pmask, w0, w1, out, stream, call_events(f, false)) == hipSuccess
             ? ELES_OK
             : ELES_EHIP;
}

size_t dfilter_errors_workspace_bytes(eles_dfilter f) {
  if (!f) return 0;
  return up256((size_t)eles::derr_parts(f->v) * sizeof(double));
}

int32_t dfilter_errors(eles_dfilter f, const float *les, const float *dns, double utau_les, double utau_dns,
                       double *out, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!f || !les || !dns || !out || !ws) return ELES_EINVAL;
  if (!aligned16(les) || !aligned16(dns) || !aligned16(ws) || ((uintptr_t)out & 7u)) return ELES_EINVAL;
  if (!(std::isfinite(utau_les) && utau_les > 0) || !(std::isfinite(utau_dns) && utau_dns > 0)) return ELES_EINVAL;
  if (ws_bytes < dfilter_errors_workspace_bytes(f)) return ELES_ENOSPACE;
  const size_t n = 3 * f->npts * sizeof(float);
  if (overlap(ws, ws_bytes, les, n) || overlap(ws, ws_bytes, dns, n) || overlap(ws, ws_bytes, out, 5 * 8) ||
      overlap(out, 5 * 8, les, n) || overlap(out, 5 * 8, dns, n))
    return ELES_EINVAL;
  return eles::launch_derrors(f->v, les, dns, utau_les, utau_dns, (double *)ws, out, stream) == hipSuccess
             ? ELES_OK
             : ELES_EHIP;
}

void dfilter_destroy(eles_dfilter f) {
  if (!f) return;
  release_events(f);
  delete f;
}

}  // extern "C"

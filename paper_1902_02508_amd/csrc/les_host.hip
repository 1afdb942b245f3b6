// Host side of the LES-grid part of the C ABI (include/eles.h): descriptor
// validation, the interpolation weights and derivative stencils (FP64 on
// the host, copied once into the caller-owned state), and the launches.
#include "eles.h"
#include "eles_internal.h"

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

struct eles_les_s {
  eles::LesView v;
  size_t npts, nles;
  std::vector<char> host;   // the state image, kept until the copy has completed
};

namespace {

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }
bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  const char *pa = (const char *)a, *pb = (const char *)b;
  return pa < pb + nb && pb < pa + na;
}

enum { L_IX, L_IY, L_IZ, L_WX, L_WY, L_WZ, L_DB, L_DC, L_LB, L_LC, L_LW, L_END };

struct LPlan {
  size_t off[L_END];
  size_t bytes;
};

bool increasing(const double *y, int n) {
  for (int j = 0; j < n; ++j)
    if (!std::isfinite(y[j]) || (j > 0 && !(y[j] > y[j - 1]))) return false;
  return true;
}

int32_t plan_l(const eles_les_desc *d, LPlan *p) {
  if (!d || !d->y || !d->y_les) return ELES_EINVAL;
  if (d->nx < 1 || d->nz < 1 || d->ny < 3 || d->nx_les < 1 || d->nz_les < 1 || d->ny_les < 3) return ELES_EINVAL;
  if (!increasing(d->y, d->ny) || d->y[0] != -1.0 || d->y[d->ny - 1] != 1.0) return ELES_EINVAL;
  if (!increasing(d->y_les, d->ny_les) || d->y_les[0] < -1.0 || d->y_les[d->ny_les - 1] > 1.0) return ELES_EINVAL;
  const size_t nxl = d->nx_les, nyl = d->ny_les, nzl = d->nz_les, ny = d->ny;
  const size_t sz[L_END] = {nxl * 4, nyl * 4, nzl * 4, nxl * 4, nyl * 4, nzl * 4,
                            ny * 4,  ny * 24, nyl * 4, nyl * 24, nyl * 8};
  size_t o = 0;
  for (int k = 0; k < L_END; ++k) {
    p->off[k] = o;
    o += up256(sz[k]);
  }
  p->bytes = o;
  return ELES_OK;
}

// LES node k of n_les on a period of n DNS nodes: lower node and weight
void periodic(int n_les, int n, int32_t *i0, float *w) {
  for (int k = 0; k < n_les; ++k) {
    const long long num = (long long)k * n;
    i0[k] = (int32_t)(num / n_les);
    w[k] = (float)((double)(num % n_les) / n_les);
  }
}

// LES y node t: the DNS node j <= ny - 2 with y[j] <= t < y[j+1], and the weight of j + 1
void bounded(const double *yl, int nyl, const double *y, int ny, int32_t *j0, float *w) {
  for (int k = 0; k < nyl; ++k) {
    int lo = 0, hi = ny - 2;   // largest j in [0, ny-2] with y[j] <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (y[mid] <= yl[k])
        lo = mid;
      else
        hi = mid - 1;
    }
    j0[k] = lo;
    w[k] = (float)((yl[k] - y[lo]) / (y[lo + 1] - y[lo]));
  }
}

// second-order three-point first derivative on nodes y[0 .. n): central
// inside, one-sided at both ends; base[j] is the stencil's first node
void stencils(const double *y, int n, int32_t *base, double *c) {
  for (int j = 0; j < n; ++j) {
    if (j == 0) {
      const double h1 = y[1] - y[0], h2 = y[2] - y[1];
      base[j] = 0;
      c[3 * j] = -(2 * h1 + h2) / (h1 * (h1 + h2));
      c[3 * j + 1] = (h1 + h2) / (h1 * h2);
      c[3 * j + 2] = -h1 / (h2 * (h1 + h2));
    } else if (j == n - 1) {
      const double h1 = y[j] - y[j - 1], h2 = y[j - 1] - y[j - 2];
      base[j] = n - 3;
      c[3 * j] = h1 / (h2 * (h1 + h2));
      c[3 * j + 1] = -(h1 + h2) / (h1 * h2);
      c[3 * j + 2] = (2 * h1 + h2) / (h1 * (h1 + h2));
    } else {
      const double hm = y[j] - y[j - 1], hp = y[j + 1] - y[j];
      base[j] = j - 1;
      c[3 * j] = -hp / (hm * (hm + hp));
      c[3 * j + 1] = (hp - hm) / (hm * hp);
      c[3 * j + 2] = hm / (hp * (hm + hp));
    }
  }
}

}  // namespace

extern "C" {

size_t les_state_bytes(const eles_les_desc *desc) {
  LPlan p;
  return plan_l(desc, &p) == ELES_OK ? p.bytes : 0;
}

int32_t les_setup(const eles_les_desc *desc, void *state, size_t state_bytes, hipStream_t stream, eles_les *out) {
  if (!out) return ELES_EINVAL;
  LPlan p;
  const int32_t st = plan_l(desc, &p);
  if (st != ELES_OK) return st;
  if (!state || !aligned16(state)) return ELES_EINVAL;
  if (state_bytes < p.bytes) return ELES_ENOSPACE;
  eles_les_s *h = new (std::nothrow) eles_les_s;
  if (!h) return ELES_EINVAL;
  h->host.assign(p.bytes, 0);
  char *b = h->host.data();
  periodic(desc->nx_les, desc->nx, (int32_t *)(b + p.off[L_IX]), (float *)(b + p.off[L_WX]));
  periodic(desc->nz_les, desc->nz, (int32_t *)(b + p.off[L_IZ]), (float *)(b + p.off[L_WZ]));
  bounded(desc->y_les, desc->ny_les, desc->y, desc->ny, (int32_t *)(b + p.off[L_IY]), (float *)(b + p.off[L_WY]));
  stencils(desc->y, desc->ny, (int32_t *)(b + p.off[L_DB]), (double *)(b + p.off[L_DC]));
  stencils(desc->y_les, desc->ny_les, (int32_t *)(b + p.off[L_LB]), (double *)(b + p.off[L_LC]));
  double *lw = (double *)(b + p.off[L_LW]);
  for (int j = 0; j < desc->ny_les; ++j) {
    const double lo = j > 0 ? desc->y_les[j] - desc->y_les[j - 1] : 0.0;
    const double hi = j < desc->ny_les - 1 ? desc->y_les[j + 1] - desc->y_les[j] : 0.0;
    lw[j] = 0.5 * (lo + hi);
  }
  char *s = (char *)state;
  eles::LesView &v = h->v;
  v.nx = desc->nx;
  v.ny = desc->ny;
  v.nz = desc->nz;
  v.nxl = desc->nx_les;
  v.nyl = desc->ny_les;
  v.nzl = desc->nz_les;
  v.ix = (const int *)(s + p.off[L_IX]);
  v.iy = (const int *)(s + p.off[L_IY]);
  v.iz = (const int *)(s + p.off[L_IZ]);
  v.wx = (const float *)(s + p.off[L_WX]);
  v.wy = (const float *)(s + p.off[L_WY]);
  v.wz = (const float *)(s + p.off[L_WZ]);
  v.db = (const int *)(s + p.off[L_DB]);
  v.dc = (const double *)(s + p.off[L_DC]);
  v.lb = (const int *)(s + p.off[L_LB]);
  v.lc = (const double *)(s + p.off[L_LC]);
  v.lw = (const double *)(s + p.off[L_LW]);
  h->npts = (size_t)desc->nx * desc->ny * desc->nz;
  h->nles = (size_t)desc->nx_les * desc->ny_les * desc->nz_les;
  if (hipMemcpyAsync(state, b, p.bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    delete h;
    return ELES_EHIP;
  }
  *out = h;
  return ELES_OK;
}

int32_t les_stress(eles_les h, const float *ubar, const float *tau, float *ubar_les, float *T, hipStream_t stream) {
  if (!h || !ubar || !tau || !ubar_les || !T) return ELES_EINVAL;
  const size_t n = h->npts * 4, nl = h->nles * 4;
  if (overlap(ubar_les, 3 * nl, T, 6 * nl) || overlap(ubar_les, 3 * nl, ubar, 3 * n) ||
      overlap(ubar_les, 3 * nl, tau, 6 * n) || overlap(T, 6 * nl, ubar, 3 * n) || overlap(T, 6 * nl, tau, 6 * n))
    return ELES_EINVAL;
  return eles::launch_les_stress(h->v, ubar, tau, ubar_les, T, stream) == hipSuccess ? ELES_OK : ELES_EHIP;
}

size_t les_commutation_workspace_bytes(eles_les h) {
  if (!h) return 0;
  return up256((size_t)eles::les_comm_parts(h->v) * sizeof(double));
}

int32_t les_commutation(eles_les h, const float *g, double *out, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!h || !g || !out || !ws || ((uintptr_t)out & 7u) || ((uintptr_t)ws & 7u)) return ELES_EINVAL;
  if (ws_bytes < les_commutation_workspace_bytes(h)) return ELES_ENOSPACE;
  if (overlap(ws, ws_bytes, g, h->npts * 4) || overlap(ws, ws_bytes, out, 8)) return ELES_EINVAL;
  return eles::launch_les_commutation(h->v, g, (double *)ws, out, stream) == hipSuccess ? ELES_OK : ELES_EHIP;
}

void les_destroy(eles_les h) { delete h; }

}  // extern "C"

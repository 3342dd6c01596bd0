// C ABI of the DPD step library (declared in include/dpd.h): context set-up,
// validation, buffer management, the per-step launch sequence and getters.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dpd.h"
#include "device.h"
#include "kernels.h"

using dpd::KGeom;
using dpd::KParams;
using dpd::Status;

namespace {

thread_local std::string g_create_error = "no error";

enum Kernel { K_INTEGRATE = 0, K_SCAN_REDUCE, K_SCAN_TOP, K_SCAN_DOWN, K_SCATTER, K_SORT,
              K_FORCE, K_OTHER };
const char *kKernelNames[DPD_NUM_KERNELS] = {"integrate_reflect_bin", "scan_reduce", "scan_top",
                                             "scan_down", "scatter", "sort_cells", "pair_force",
                                             "other"};

struct TimedLaunch {
  int kernel;
  hipEvent_t a, b;
};

}  // namespace

struct dpd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  dpd_allocator al{};
  bool has_al = false;
  std::string err = "no error";
  std::vector<void *> owned;

  int64_t n = 0, nf = 0, nw = 0, ncell = 0;
  int nc[3] = {0, 0, 0};
  int ng[3] = {0, 0, 0};
  int grid_f64 = 0;
  double L[3] = {0, 0, 0}, h[3] = {0, 0, 0};
  dpd_params params{};
  KGeom G{};
  KParams P{};

  float4 *pos[2] = {nullptr, nullptr}, *vel[2] = {nullptr, nullptr}, *frc[2] = {nullptr, nullptr};
  float4 *vt = nullptr;
  int cur = 0;
  int32_t *cell_of = nullptr, *rank_of = nullptr, *count = nullptr, *cstart = nullptr,
          *idx = nullptr, *bsum = nullptr;
  int nscan = 0;
  int32_t *wcstart = nullptr;   // exclusive scan of wall counts per cell (static)
  int32_t *wcell = nullptr;     // cell of each cell-sorted wall (static)
  int32_t *idx_all = nullptr;   // merged per-cell runs: walls (nf + w), then fluid
  int32_t *start_all = nullptr; // start of each cell's merged run
  int32_t *fluid_off = nullptr; // start of each cell's fluid part in the merged run
  void *grid = nullptr;
  uint32_t *bits = nullptr;   // near-interface grid cubes, one bit each
  int64_t nwords = 0;
  int use_mask = 1;
  int64_t flagged_cubes = 0;
  Status *status = nullptr;
  unsigned long long *pair_counter = nullptr;

  uint64_t k = 0;
  int64_t steps = 0;

  bool timing = false;
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> free_events;
  double kernel_ms[DPD_NUM_KERNELS] = {0};
  int64_t kernel_launches[DPD_NUM_KERNELS] = {0};
};

namespace {

int fail(dpd_ctx *c, int code, const std::string &msg) {
  if (c)
    c->err = msg;
  else
    g_create_error = msg;
  return code;
}

int hip_fail(dpd_ctx *c, hipError_t e, const char *where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? DPD_E_NOMEM : DPD_E_DEVICE, m);
}

#define HIP_TRY(ctx, expr)                                      \
  do {                                                          \
    hipError_t e_ = (expr);                                     \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);    \
  } while (0)

void *dalloc(dpd_ctx *c, size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (bytes == 0) bytes = 256;
  void *p = nullptr;
  if (c->has_al) {
    p = c->al.alloc(bytes, (void *)c->stream, c->al.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) c->owned.push_back(p);
  return p;
}

void dfree(dpd_ctx *c, void *p) {
  for (size_t q = 0; q < c->owned.size(); ++q) {
    if (c->owned[q] != p) continue;
    if (c->has_al)
      c->al.free(p, (void *)c->stream, c->al.user);
    else
      (void)hipFree(p);
    c->owned.erase(c->owned.begin() + (std::ptrdiff_t)q);
    return;
  }
}

void release_all(dpd_ctx *c) {
  for (void *p : c->owned) {
    if (c->has_al)
      c->al.free(p, (void *)c->stream, c->al.user);
    else
      (void)hipFree(p);
  }
  c->owned.clear();
  for (auto &t : c->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  c->pending.clear();
  for (auto e : c->free_events) (void)hipEventDestroy(e);
  c->free_events.clear();
}

hipEvent_t get_event(dpd_ctx *c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Collect finished timings (the stream must have been synchronised).
void harvest_timings(dpd_ctx *c) {
  for (auto &t : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      c->kernel_ms[t.kernel] += ms;
      c->kernel_launches[t.kernel] += 1;
    }
    c->free_events.push_back(t.a);
    c->free_events.push_back(t.b);
  }
  c->pending.clear();
}

// Launch helper: brackets a launch with events when timing is on.
template <typename F>
hipError_t timed(dpd_ctx *c, int kernel, F &&launch) {
  if (!c->timing) return launch();
  if (c->pending.size() > 4096) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    harvest_timings(c);
  }
  TimedLaunch t{kernel, get_event(c), get_event(c)};
  (void)hipEventRecord(t.a, c->stream);
  hipError_t e = launch();
  (void)hipEventRecord(t.b, c->stream);
  c->pending.push_back(t);
  return e;
}

int read_status(dpd_ctx *c, Status &st) {
  HIP_TRY(c, hipMemcpyAsync(&st, c->status, sizeof(Status), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return DPD_OK;
}

int latched_error(dpd_ctx *c) {
  Status st;
  int rc = read_status(c, st);
  if (rc) return rc;
  if (st.nonfinite)
    return fail(c, DPD_E_UNSTABLE, "non-finite positions or forces (" +
                                       std::to_string(st.nonfinite) + " events)");
  if (st.unstable)
    return fail(c, DPD_E_UNSTABLE, "a particle moved more than half a cell in one step (" +
                                       std::to_string(st.unstable) + " events)");
  return DPD_OK;
}

// Release a half-built context, keeping its message as the create error.
int abandon_create(dpd_ctx *c, int code) {
  (void)hipStreamSynchronize(c->stream);
  release_all(c);
  g_create_error = c->err;
  delete c;
  return code;
}

bool finite3(const float *p) {
  return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]);
}

// Cell list of the current fluid positions in pos[cur]: bin, scan, scatter, sort.
int build_cells_from_pos(dpd_ctx *c) {
  HIP_TRY(c, timed(c, K_OTHER, [&] {
            return dpd::launch_bin(c->stream, c->G, c->nf, c->pos[c->cur], c->cell_of,
                                   c->rank_of, c->count);
          }));
  return DPD_OK;
}

int scan_scatter_sort(dpd_ctx *c) {
  HIP_TRY(c, timed(c, K_SCAN_REDUCE, [&] {
            return dpd::launch_scan_reduce(c->stream, c->ncell, c->count, c->bsum);
          }));
  HIP_TRY(c, timed(c, K_SCAN_TOP, [&] { return dpd::launch_scan_top(c->stream, c->nscan, c->bsum); }));
  HIP_TRY(c, timed(c, K_SCAN_DOWN, [&] {
            return dpd::launch_scan_down(c->stream, c->ncell, c->count, c->cstart, c->bsum,
                                         c->wcstart, c->start_all, c->fluid_off);
          }));
  HIP_TRY(c, timed(c, K_SCATTER, [&] {
            return dpd::launch_scatter(c->stream, c->nf, c->cell_of, c->rank_of, c->cstart,
                                       c->idx);
          }));
  HIP_TRY(c, timed(c, K_SORT, [&] {
            return dpd::launch_sort_cells(c->stream, c->ncell, c->cstart, c->idx, c->fluid_off,
                                          c->idx_all);
          }));
  HIP_TRY(c, timed(c, K_OTHER, [&] {
            return dpd::launch_fill_walls(c->stream, c->nw, c->nf, c->wcell, c->wcstart,
                                          c->start_all, c->idx_all);
          }));
  return DPD_OK;
}

// Forces at the current state in sorted order; init = 1 keeps velocities.
int force_pass(dpd_ctx *c, int init) {
  const int a = c->cur, b = 1 - c->cur;
  HIP_TRY(c, timed(c, K_FORCE, [&] {
            return dpd::launch_force(c->stream, c->G, c->P, c->nf, c->nw, init, c->pos[a], c->vt,
                                     c->vel[a], c->frc[a], c->idx, c->idx_all, c->start_all,
                                     c->pos[b], c->vel[b], c->frc[b], c->k,
                                     c->status);
          }));
  c->cur = b;
  return DPD_OK;
}

int one_step(dpd_ctx *c) {
  const int a = c->cur;
  HIP_TRY(c, timed(c, K_INTEGRATE, [&] {
            return dpd::launch_integrate(c->stream, c->G, c->P, c->nf, c->pos[a], c->vel[a],
                                         c->frc[a], c->vt, c->cell_of, c->rank_of, c->count,
                                         c->bits, c->use_mask, c->grid, c->grid_f64, c->status);
          }));
  int rc = scan_scatter_sort(c);
  if (rc) return rc;
  c->k += 1;
  rc = force_pass(c, 0);
  if (rc) return rc;
  c->steps += 1;
  return DPD_OK;
}

}  // namespace

extern "C" {

const char *dpd_last_error(const dpd_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

const char *dpd_kernel_name(int32_t i) {
  if (i < 0 || i >= DPD_NUM_KERNELS) return "";
  return kKernelNames[i];
}

int dpd_create(const dpd_box *box, const dpd_particles *pp, const dpd_params *prm,
               const dpd_phi_grid *phi, const dpd_allocator *alloc, void *hip_stream,
               dpd_ctx **out) {
  if (!out) return fail(nullptr, DPD_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!box || !pp || !prm || !phi) return fail(nullptr, DPD_E_INVAL, "NULL argument");
  // ---- validate scalar inputs ----
  const dpd_params &P = *prm;
  for (int a = 0; a < 3; ++a)
    if (!(std::isfinite(box->L[a]) && box->L[a] > 0))
      return fail(nullptr, DPD_E_INVAL, "box edges must be finite and positive");
  if (!(std::isfinite(P.rc) && P.rc > 0)) return fail(nullptr, DPD_E_INVAL, "rc must be > 0");
  if (!(std::isfinite(P.dt) && P.dt > 0)) return fail(nullptr, DPD_E_INVAL, "dt must be > 0");
  if (!(std::isfinite(P.gamma) && P.gamma >= 0) || !(std::isfinite(P.kBT) && P.kBT >= 0))
    return fail(nullptr, DPD_E_INVAL, "gamma and kBT must be finite and >= 0");
  if (!std::isfinite(P.lambda)) return fail(nullptr, DPD_E_INVAL, "lambda must be finite");
  for (int a = 0; a < 4; ++a)
    if (!std::isfinite(P.a[a])) return fail(nullptr, DPD_E_INVAL, "a_ij must be finite");
  if (P.a[1] != P.a[2]) return fail(nullptr, DPD_E_INVAL, "a_ij must be symmetric");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(P.g[a])) return fail(nullptr, DPD_E_INVAL, "g must be finite");
  if (P.replica >= 65536u) return fail(nullptr, DPD_E_INVAL, "replica must be < 65536");
  int nc[3];
  for (int a = 0; a < 3; ++a) {
    nc[a] = (int)std::floor(box->L[a] / P.rc);
    if (nc[a] < 3) return fail(nullptr, DPD_E_INVAL, "box must hold at least 3 cells per axis");
  }
  const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
  if (ncell > (int64_t)1 << 30) return fail(nullptr, DPD_E_INVAL, "too many cells");
  if (!(phi->dtype == 4 || phi->dtype == 8))
    return fail(nullptr, DPD_E_INVAL, "phi dtype must be 4 or 8");
  if (!phi->data) return fail(nullptr, DPD_E_INVAL, "phi data is NULL");
  for (int a = 0; a < 3; ++a) {
    if (phi->n[a] < 2 || !(phi->h[a] > 0))
      return fail(nullptr, DPD_E_INVAL, "phi grid needs >= 2 nodes and h > 0 per axis");
    if (std::fabs(phi->n[a] * phi->h[a] - box->L[a]) > 1e-9 * box->L[a])
      return fail(nullptr, DPD_E_INVAL, "phi grid n*h must equal the box edge");
  }
  const int64_t n = pp->n;
  if (n < 0 || n >= ((int64_t)1 << 31))
    return fail(nullptr, DPD_E_INVAL, "particle count out of range");
  if (n > 0 && (!pp->pos || !pp->vel || !pp->type))
    return fail(nullptr, DPD_E_INVAL, "particle arrays are NULL");

  // ---- bring particle arrays to the host for validation and splitting ----
  std::vector<float> hpos(3 * (size_t)n), hvel(3 * (size_t)n);
  std::vector<int32_t> htype((size_t)n);
  std::vector<uint32_t> hgid((size_t)n);
  if (n > 0) {
    if (pp->on_device) {
      if (hipMemcpy(hpos.data(), pp->pos, 12 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hvel.data(), pp->vel, 12 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(htype.data(), pp->type, 4 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess ||
          (pp->gid && hipMemcpy(hgid.data(), pp->gid, 4 * (size_t)n, hipMemcpyDeviceToHost) !=
                          hipSuccess))
        return fail(nullptr, DPD_E_DEVICE, "copying particle arrays failed");
    } else {
      std::memcpy(hpos.data(), pp->pos, 12 * (size_t)n);
      std::memcpy(hvel.data(), pp->vel, 12 * (size_t)n);
      std::memcpy(htype.data(), pp->type, 4 * (size_t)n);
      if (pp->gid) std::memcpy(hgid.data(), pp->gid, 4 * (size_t)n);
    }
  }
  if (!pp->gid)
    for (int64_t i = 0; i < n; ++i) hgid[i] = (uint32_t)i;
  {
    std::vector<uint8_t> seen((size_t)n, 0);
    for (int64_t i = 0; i < n; ++i) {
      if (hgid[i] >= (uint64_t)n || seen[hgid[i]])
        return fail(nullptr, DPD_E_INVAL, "gid must be a permutation of 0..n-1");
      seen[hgid[i]] = 1;
    }
  }
  std::vector<int64_t> rows_f, rows_w;
  for (int64_t i = 0; i < n; ++i) {
    if (htype[i] != DPD_TYPE_FLUID && htype[i] != DPD_TYPE_WALL)
      return fail(nullptr, DPD_E_INVAL, "type must be 0 (fluid) or 1 (wall)");
    if (!finite3(&hpos[3 * i]) || (htype[i] == DPD_TYPE_FLUID && !finite3(&hvel[3 * i])))
      return fail(nullptr, DPD_E_INVAL, "non-finite particle position or velocity");
    for (int a = 0; a < 3; ++a)
      if (!(hpos[3 * i + a] >= 0.0f && hpos[3 * i + a] < (float)box->L[a]))
        return fail(nullptr, DPD_E_INVAL, "particle position outside [0, L)");
    (htype[i] == DPD_TYPE_FLUID ? rows_f : rows_w).push_back(i);
  }

  // ---- device (after the host-side checks, which need none) ----
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(nullptr, DPD_E_DEVICE, "no HIP device");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, DPD_E_DEVICE, "hipGetDevice failed");
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
      return fail(nullptr, DPD_E_DEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(nullptr, DPD_E_DEVICE,
                  std::string("library built for gfx950, device is ") + prop.gcnArchName);
  }

  // ---- context ----
  dpd_ctx *c = new (std::nothrow) dpd_ctx();
  if (!c) return fail(nullptr, DPD_E_NOMEM, "host allocation failed");
  c->device = dev;
  c->stream = (hipStream_t)hip_stream;
  if (alloc && alloc->alloc && alloc->free) {
    c->al = *alloc;
    c->has_al = true;
  }
  c->params = P;
  c->n = n;
  c->nf = (int64_t)rows_f.size();
  c->nw = (int64_t)rows_w.size();
  c->ncell = ncell;
  c->grid_f64 = phi->dtype == 8;
  for (int a = 0; a < 3; ++a) {
    c->nc[a] = nc[a];
    c->ng[a] = phi->n[a];
    c->L[a] = box->L[a];
    c->h[a] = phi->h[a];
    c->G.L[a] = (float)box->L[a];
    c->G.invw[a] = (float)((double)nc[a] / box->L[a]);
    c->G.nc[a] = nc[a];
    c->G.ng[a] = phi->n[a];
    c->G.inv_h[a] = (float)(1.0 / phi->h[a]);
    c->G.inv_h64[a] = 1.0 / phi->h[a];
    c->G.h[a] = (float)phi->h[a];
  }
  {
    KParams &K = c->P;
    K.a_ff = (float)P.a[0];
    K.a_fw = (float)P.a[1];
    K.gamma = (float)P.gamma;
    K.sigma_rdt = (float)(std::sqrt(2.0 * P.gamma * P.kBT) / std::sqrt(P.dt));
    K.rc2 = (float)(P.rc * P.rc);
    K.inv_rc = (float)(1.0 / P.rc);
    K.dt = (float)P.dt;
    K.hdt = (float)(0.5 * P.dt);
    K.lamdt = (float)(P.lambda * P.dt);
    for (int a = 0; a < 3; ++a) K.g[a] = (float)P.g[a];
    double wmin = box->L[0] / nc[0];
    for (int a = 1; a < 3; ++a) wmin = std::fmin(wmin, box->L[a] / nc[a]);
    K.max_disp2 = (float)(0.25 * wmin * wmin);
    K.key0 = (uint32_t)P.seed;
    K.key1 = (uint32_t)(P.seed >> 32);
    K.replica = P.replica;
  }
  c->use_mask = (P.flags & DPD_FLAG_NO_MASK) ? 0 : 1;

  auto bail = [c](int code) { return abandon_create(c, code); };

  // ---- device buffers ----
  const size_t nf = (size_t)c->nf, nw = (size_t)c->nw;
  const size_t gbytes = (size_t)phi->n[0] * phi->n[1] * phi->n[2] * (size_t)phi->dtype;
  for (int b = 0; b < 2; ++b) {
    c->pos[b] = (float4 *)dalloc(c, 16 * (nf + nw + 1));
    c->vel[b] = (float4 *)dalloc(c, 16 * nf);
    c->frc[b] = (float4 *)dalloc(c, 16 * nf);
  }
  c->vt = (float4 *)dalloc(c, 16 * (nf + nw + 1));
  c->cell_of = (int32_t *)dalloc(c, 4 * (nf > nw ? nf : nw));
  c->rank_of = (int32_t *)dalloc(c, 4 * (nf > nw ? nf : nw));
  c->idx = (int32_t *)dalloc(c, 4 * (nf > nw ? nf : nw));
  c->count = (int32_t *)dalloc(c, 4 * (size_t)ncell);
  c->cstart = (int32_t *)dalloc(c, 4 * ((size_t)ncell + 1));
  c->nscan = dpd::scan_blocks(ncell);
  c->bsum = (int32_t *)dalloc(c, 4 * (size_t)c->nscan);
  c->wcstart = (int32_t *)dalloc(c, 4 * ((size_t)ncell + 1));
  c->wcell = (int32_t *)dalloc(c, 4 * nw);
  c->idx_all = (int32_t *)dalloc(c, 4 * (nf + nw));
  c->start_all = (int32_t *)dalloc(c, 4 * ((size_t)ncell + 1));
  c->fluid_off = (int32_t *)dalloc(c, 4 * (size_t)ncell);
  c->grid = dalloc(c, gbytes);
  c->nwords = ((int64_t)phi->n[0] * phi->n[1] * phi->n[2] + 31) / 32;
  c->bits = (uint32_t *)dalloc(c, 4 * (size_t)c->nwords);
  c->status = (Status *)dalloc(c, sizeof(Status));
  c->pair_counter = (unsigned long long *)dalloc(c, 8);
  for (int b = 0; b < 2; ++b)
    if (!c->pos[b] || !c->vel[b] || !c->frc[b]) return bail(fail(c, DPD_E_NOMEM, "device allocation failed"));
  if (!c->vt || !c->cell_of || !c->rank_of || !c->idx || !c->count || !c->cstart || !c->bsum ||
      !c->wcell || !c->idx_all || !c->start_all || !c->fluid_off || !c->wcstart || !c->grid || !c->bits || !c->status || !c->pair_counter)
    return bail(fail(c, DPD_E_NOMEM, "device allocation failed"));

  // ---- upload ----
  int rc = DPD_OK;
  auto chk = [&](hipError_t e, const char *w) {
    if (e != hipSuccess && rc == DPD_OK) rc = hip_fail(c, e, w);
  };
  chk(hipMemcpyAsync(c->grid, phi->data, gbytes,
                     phi->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream),
      "upload phi");
  chk(dpd::launch_fill_zero(c->stream, c->status, sizeof(Status)), "zero status");
  chk(dpd::launch_fill_zero(c->stream, c->count, 4 * (size_t)ncell), "zero counts");
  chk(dpd::launch_fill_zero(c->stream, c->pair_counter, 8), "zero counter");
  if (rc) return bail(rc);
  {
    // staging of all input rows on the device, released before returning
    const size_t nn = (size_t)(n > 0 ? n : 1);
    float *dpos = (float *)dalloc(c, 12 * nn);
    float *dvel = (float *)dalloc(c, 12 * nn);
    uint32_t *dgid = (uint32_t *)dalloc(c, 4 * nn);
    int64_t *drows_f = (int64_t *)dalloc(c, 8 * (nf > 0 ? nf : 1));
    int64_t *drows_w = (int64_t *)dalloc(c, 8 * (nw > 0 ? nw : 1));
    float4 *wtmp = (float4 *)dalloc(c, 16 * (nw > 0 ? nw : 1));
    if (!dpos || !dvel || !dgid || !drows_f || !drows_w || !wtmp)
      return bail(fail(c, DPD_E_NOMEM, "staging allocation failed"));
    if (n > 0) {
      chk(hipMemcpyAsync(dpos, hpos.data(), 12 * (size_t)n, hipMemcpyHostToDevice, c->stream), "upload pos");
      chk(hipMemcpyAsync(dvel, hvel.data(), 12 * (size_t)n, hipMemcpyHostToDevice, c->stream), "upload vel");
      chk(hipMemcpyAsync(dgid, hgid.data(), 4 * (size_t)n, hipMemcpyHostToDevice, c->stream), "upload gid");
    }
    if (nf > 0) {
      chk(hipMemcpyAsync(drows_f, rows_f.data(), 8 * nf, hipMemcpyHostToDevice, c->stream), "rows");
      chk(dpd::launch_pack(c->stream, (int64_t)nf, dpos, dvel, dgid, drows_f, c->pos[0],
                           c->vel[0], c->vt, c->frc[0]),
          "pack fluid");
    }
    // frozen walls: pack, bin, scan, scatter, sort each cell, permute (once)
    if (nw > 0) {
      chk(hipMemcpyAsync(drows_w, rows_w.data(), 8 * nw, hipMemcpyHostToDevice, c->stream), "rows");
      chk(dpd::launch_pack(c->stream, (int64_t)nw, dpos, nullptr, dgid, drows_w, wtmp, nullptr,
                           nullptr, nullptr),
          "pack walls");
      chk(dpd::launch_bin(c->stream, c->G, (int64_t)nw, wtmp, c->cell_of, c->rank_of, c->count),
          "bin walls");
    }
    chk(dpd::launch_scan_reduce(c->stream, ncell, c->count, c->bsum), "scan");
    chk(dpd::launch_scan_top(c->stream, c->nscan, c->bsum), "scan");
    chk(dpd::launch_scan_down(c->stream, ncell, c->count, c->wcstart, c->bsum, nullptr, nullptr,
                              nullptr),
        "scan");
    if (nw > 0) {
      // walls sorted by cell into the tail of both position buffers (static),
      // with zero predicted velocity
      chk(dpd::launch_scatter(c->stream, (int64_t)nw, c->cell_of, c->rank_of, c->wcstart, c->idx),
          "scatter walls");
      chk(dpd::launch_sort_cells(c->stream, ncell, c->wcstart, c->idx, nullptr, nullptr),
          "sort walls");
      chk(dpd::launch_permute(c->stream, (int64_t)nw, c->idx, wtmp, c->pos[0] + nf, nullptr,
                              nullptr, nullptr, nullptr),
          "permute walls");
      chk(hipMemcpyAsync(c->pos[1] + nf, c->pos[0] + nf, 16 * nw, hipMemcpyDeviceToDevice,
                         c->stream),
          "copy walls");
      chk(dpd::launch_fill_zero(c->stream, c->vt + nf, 16 * nw), "zero wall velocities");
      chk(dpd::launch_cells(c->stream, c->G, (int64_t)nw, c->pos[0] + nf, c->wcell), "wall cells");
    }
    chk(dpd::launch_set_pad(c->stream, c->pos[0] + nf + nw, c->vt + nf + nw), "pad");
    chk(dpd::launch_set_pad(c->stream, c->pos[1] + nf + nw, nullptr), "pad");
    chk(hipStreamSynchronize(c->stream), "sync");
    for (void *q : {(void *)dpos, (void *)dvel, (void *)dgid, (void *)drows_f, (void *)drows_w,
                    (void *)wtmp})
      dfree(c, q);
    if (rc) return bail(rc);
  }
  // near-interface mask and create-time phi check
  {
    chk(dpd::launch_cube_mask(c->stream, c->G, c->grid, c->grid_f64, c->nwords, c->bits), "mask");
    chk(dpd::launch_check_grid(c->stream, c->grid, c->grid_f64,
                               (int64_t)phi->n[0] * phi->n[1] * phi->n[2], c->status),
        "check grid");
    chk(dpd::launch_check_phi(c->stream, c->G, c->grid, c->grid_f64, c->nf, c->pos[0], c->status),
        "check phi");
    if (rc) return bail(rc);
    Status st;
    int r2 = read_status(c, st);
    if (r2) return bail(r2);
    if (st.bad_grid)
      return bail(fail(c, DPD_E_INVAL, std::to_string(st.bad_grid) + " non-finite phi values"));
    if (st.bad_phi)
      return bail(fail(c, DPD_E_INVAL,
                       std::to_string(st.bad_phi) + " fluid particles start at phi < 0"));
    std::vector<uint32_t> hb((size_t)c->nwords);
    chk(hipMemcpy(hb.data(), c->bits, 4 * (size_t)c->nwords, hipMemcpyDeviceToHost),
        "mask readback");
    if (rc) return bail(rc);
    int64_t m = 0;
    for (uint32_t v : hb) m += __builtin_popcount(v);
    c->flagged_cubes = m;
  }
  // initial cell list and forces f(0) with k = 0
  c->cur = 0;
  c->k = 0;
  rc = build_cells_from_pos(c);
  if (!rc) rc = scan_scatter_sort(c);
  if (!rc) rc = force_pass(c, 1);
  if (!rc) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = hip_fail(c, e, "initial forces");
  }
  if (!rc) rc = latched_error(c);
  if (rc) return bail(rc);
  *out = c;
  return DPD_OK;
}

int dpd_step(dpd_ctx *c, int64_t nsteps) {
  if (!c) return DPD_E_INVAL;
  if (nsteps < 0) return fail(c, DPD_E_INVAL, "negative step count");
  for (int64_t s = 0; s < nsteps; ++s) {
    int rc = one_step(c);
    if (rc) return rc;
  }
  return DPD_OK;
}

int dpd_forces(dpd_ctx *c, float *f_out) {
  if (!c) return DPD_E_INVAL;
  if (!f_out) return fail(c, DPD_E_INVAL, "f_out is NULL");
  HIP_TRY(c, dpd::launch_fill_zero(c->stream, f_out, 12 * (size_t)c->n));
  HIP_TRY(c, dpd::launch_export(c->stream, c->G, c->nf, c->pos[c->cur], c->vel[c->cur],
                                c->frc[c->cur], 0, nullptr, nullptr, f_out, nullptr, nullptr));
  return latched_error(c);
}

int dpd_get_state(dpd_ctx *c, float *pos, float *vel, int32_t *events, int32_t *cell_of) {
  if (!c) return DPD_E_INVAL;
  HIP_TRY(c, dpd::launch_export(c->stream, c->G, c->nf, c->pos[c->cur], c->vel[c->cur],
                                c->frc[c->cur], 0, pos, vel, nullptr, events, cell_of));
  HIP_TRY(c, dpd::launch_export(c->stream, c->G, c->nw, c->pos[c->cur] + c->nf, nullptr, nullptr,
                                1, pos, vel,
                                nullptr, events, cell_of));
  return latched_error(c);
}

int dpd_set_state(dpd_ctx *c, const float *pos, const float *vel, const float *force,
                  uint64_t k, int32_t on_device) {
  if (!c) return DPD_E_INVAL;
  if (!pos || !vel || !force) return fail(c, DPD_E_INVAL, "NULL state array");
  const size_t bytes = 12 * (size_t)c->n;
  const float *dp = pos, *dv = vel, *df = force;
  float *stage = nullptr;
  if (!on_device) {
    stage = (float *)dalloc(c, 3 * bytes);
    if (!stage) return fail(c, DPD_E_NOMEM, "staging allocation failed");
    HIP_TRY(c, hipMemcpyAsync(stage, pos, bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(stage + 3 * c->n, vel, bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(stage + 6 * c->n, force, bytes, hipMemcpyHostToDevice, c->stream));
    dp = stage;
    dv = stage + 3 * c->n;
    df = stage + 6 * c->n;
  }
  const int a = c->cur;
  HIP_TRY(c, dpd::launch_import(c->stream, c->nf, c->pos[a], c->vel[a], c->frc[a], dp, dv, df));
  // re-sort: cell list of the new positions, permute into slot order
  HIP_TRY(c, dpd::launch_bin(c->stream, c->G, c->nf, c->pos[a], c->cell_of, c->rank_of, c->count));
  int rc = scan_scatter_sort(c);
  if (rc) return rc;
  const int b = 1 - a;
  HIP_TRY(c, dpd::launch_permute(c->stream, c->nf, c->idx, c->pos[a], c->pos[b], c->vel[a],
                                 c->vel[b], c->frc[a], c->frc[b]));
  c->cur = b;
  c->k = k;
  // validate positions: in box and phi >= 0
  Status before;
  rc = read_status(c, before);
  if (rc) return rc;
  HIP_TRY(c, dpd::launch_check_phi(c->stream, c->G, c->grid, c->grid_f64, c->nf, c->pos[c->cur],
                                   c->status));
  Status after;
  rc = read_status(c, after);
  if (rc) return rc;
  if (stage) dfree(c, stage);
  if (after.bad_phi != before.bad_phi)
    return fail(c, DPD_E_INVAL, "set_state: fluid particles at phi < 0");
  return DPD_OK;
}

int dpd_neighbor_pairs(dpd_ctx *c, uint32_t *pairs, int64_t cap, int64_t *count) {
  if (!c || !count) return DPD_E_INVAL;
  if (cap < 0 || (cap > 0 && !pairs)) return fail(c, DPD_E_INVAL, "bad pair buffer");
  // cell list of the current positions (state is in slot order already; the
  // list is rebuilt so that it matches the positions exactly)
  HIP_TRY(c, dpd::launch_fill_zero(c->stream, c->pair_counter, 8));
  HIP_TRY(c, dpd::launch_bin(c->stream, c->G, c->nf, c->pos[c->cur], c->cell_of, c->rank_of,
                             c->count));
  int rc = scan_scatter_sort(c);
  if (rc) return rc;
  HIP_TRY(c, dpd::launch_pairs(c->stream, c->G, c->P, c->nf, c->pos[c->cur], c->idx, c->idx_all,
                               c->start_all, pairs, cap, c->pair_counter));
  unsigned long long cnt = 0;
  HIP_TRY(c, hipMemcpyAsync(&cnt, c->pair_counter, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *count = (int64_t)cnt;
  return latched_error(c);
}

int dpd_profile(dpd_ctx *c, int32_t axis, int32_t nbins, double *out) {
  if (!c) return DPD_E_INVAL;
  if (axis < 0 || axis > 2 || nbins <= 0 || !out) return fail(c, DPD_E_INVAL, "bad profile arguments");
  HIP_TRY(c, dpd::launch_fill_zero(c->stream, out, 5 * 8 * (size_t)nbins));
  HIP_TRY(c, dpd::launch_profile(c->stream, c->G, c->nf, c->pos[c->cur], c->vel[c->cur], axis,
                                 nbins, out));
  return DPD_OK;
}

int dpd_counters(dpd_ctx *c, int64_t *out) {
  if (!c || !out) return DPD_E_INVAL;
  Status st;
  int rc = read_status(c, st);
  if (rc) return rc;
  out[0] = c->steps;
  out[1] = (int64_t)c->k;
  out[2] = (int64_t)st.bounce;
  out[3] = (int64_t)st.fallback;
  out[4] = c->nf;
  out[5] = c->nw;
  out[6] = c->ncell;
  out[7] = c->flagged_cubes;
  out[9] = (int64_t)st.unstable;
  // fluid particles now in flagged cubes (those that interpolate phi)
  HIP_TRY(c, dpd::launch_fill_zero(c->stream, &c->status->lookups, 8));
  HIP_TRY(c, dpd::launch_count_flagged(c->stream, c->G, c->grid_f64, c->nf, c->pos[c->cur],
                                       c->bits, &c->status->lookups));
  rc = read_status(c, st);
  if (rc) return rc;
  out[8] = (int64_t)st.lookups;
  return DPD_OK;
}

int dpd_kernel_times(dpd_ctx *c, int32_t enable, double *out_ms, int64_t *out_launches) {
  if (!c) return DPD_E_INVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  harvest_timings(c);
  if (out_ms)
    for (int i = 0; i < DPD_NUM_KERNELS; ++i) out_ms[i] = c->kernel_ms[i];
  if (out_launches)
    for (int i = 0; i < DPD_NUM_KERNELS; ++i) out_launches[i] = c->kernel_launches[i];
  if (enable && !c->timing) {
    for (int i = 0; i < DPD_NUM_KERNELS; ++i) {
      c->kernel_ms[i] = 0;
      c->kernel_launches[i] = 0;
    }
  }
  c->timing = enable != 0;
  return DPD_OK;
}

int dpd_sync(dpd_ctx *c) {
  if (!c) return DPD_E_INVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return latched_error(c);
}

void dpd_destroy(dpd_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  release_all(c);
  delete c;
}

int dpd_pair_random(uint64_t seed, uint64_t k, uint32_t replica, const uint32_t *gi,
                    const uint32_t *gj, int64_t n, uint32_t *words, float *xi, void *hip_stream) {
  if (n < 0 || (n > 0 && (!gi || !gj))) return DPD_E_INVAL;
  if (replica >= 65536u) return DPD_E_INVAL;
  hipError_t e = dpd::launch_pair_random((hipStream_t)hip_stream, seed, k, replica, gi, gj, n,
                                         words, xi);
  return e == hipSuccess ? DPD_OK : DPD_E_DEVICE;
}

int dpd_copy_probe(void *dst, const void *src, size_t bytes, void *hip_stream) {
  if (!dst || !src) return DPD_E_INVAL;
  hipError_t e = dpd::launch_copy((hipStream_t)hip_stream, dst, src, bytes);
  return e == hipSuccess ? DPD_OK : DPD_E_DEVICE;
}

}  // extern "C"

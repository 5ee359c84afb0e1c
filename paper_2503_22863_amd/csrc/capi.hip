// C-ABI layer of libgsr: handles, argument checks, workspace management and
// the host side of the device-resident LSQR driver.  All arithmetic of the
// method runs in the kernels (aprod.hip, fused.hip, attitude.hip,
// constraints.hip, lsqr.hip, mlp.hip); this file only validates, allocates
// and enqueues.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <set>
#include <vector>

#include "internal.h"

using namespace gsr;

// ------------------------------------------------------------------ errors
static thread_local char g_err[512] = "";

static int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(call)                                                                                  \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      return fail(e_ == hipErrorOutOfMemory ? GSR_ENOMEM : GSR_EHIP, "%s failed: %s", #call,          \
                  hipGetErrorString(e_));                                                             \
  } while (0)

#define CHK(expr)              \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != GSR_OK) return rc_; \
  } while (0)

extern "C" const char* gsr_last_error(void) { return g_err; }
extern "C" const char* gsr_version(void) { return "gsr 0.1 (gfx950)"; }

// ------------------------------------------------------------------ handle
struct PendingTime {
  int kind;
  hipEvent_t a, b;
};

struct gsr_system {
  SysView s;
  int device = 0;
  int cus = 256;
  int waves_per_cu = 32;
  int att_atomics = 0;  // 1: attitude sums by device atomics instead of the bucketed pass
  int att_tried = 0;    // the bucketed attitude view was built (or could not be) at its first use
  StreamShape sh{};
  AttView av{};
  Scalars* sc = nullptr;
  Scalars* sc_host = nullptr;  // pinned
  Work wk{};
  double* acc = nullptr;  // tail accumulators [tail_len]
  double* S = nullptr;
  int S_valid = 0;
  // LSQR vectors
  double *u = nullptr, *v = nullptr, *vg = nullptr, *w = nullptr, *y = nullptr, *var = nullptr;
  double* gA = nullptr;  // raw astrometric sums of the fused iteration pass
  double* x3 = nullptr;  // attitude window records of vg [n_att][kAttRec], for the star-order fused pass
  double* awr = nullptr;  // attitude window records of vg [n_att][kAttRec], for the regrouped pass
  float* awrf = nullptr;  // the same rounded to FP32, for the regrouped pass with FP32 products
  double* x3a = nullptr;  // attitude window records of aprod 1's x (aprod 1's workspace)
  void* rix = nullptr;   // packed row indices for the fused pass (16 B per row); null: no fused pass
  int fused = 1;         // one pass over the rows per iteration (FP64 products, attitude mode 0 or 3)
  // rows regrouped by attitude window (one pass per iteration where the attitude block exceeds LDS)
  BlkView blk{};
  int blocked = 1;       // use the regrouped copy when it applies
  int blk_maxw = 0;      // cap on its window width (0: as large as LDS allows)
  int blk_failed = 0;    // the copy could not be built (memory or limits): not tried again
  int use_blk = 0;       // the current solve runs on it
  int packed = 0;        // the rows exist only in the regrouped order, in the caller's buffer (gsr_create_packed)
  Scalars* psc = nullptr;  // scalars of the standalone passes over the regrouped rows
  // refinement buffers
  double *xr = nullptr, *xn = nullptr, *nrm2 = nullptr;
  // covariances
  int64_t nsel = 0;
  int32_t dblock = 64;
  int64_t* sel = nullptr;
  double* D = nullptr;
  double* Cacc = nullptr;
  int cov_precond = 0;
  // constraint equations (rows under A; the LSQR u vector has m + ncon entries)
  ConView con{};
  double* con_rhs = nullptr;   // [ncon]
  double* zvec = nullptr;      // [n] zeros (the x of the constrained solve's first pass)
  // covariances for a pair list instead of a dense block (sel = the pairs' distinct unknowns)
  int64_t npairs = 0;
  int32_t *pa = nullptr, *pb = nullptr;  // positions in sel
  double* Cp = nullptr;
  // export of whole d_i blocks (covariance pipeline version 1)
  int32_t eblock = 0;              // 0: off
  double* ering = nullptr;         // device ring [2*eblock][n]
  double* ehost = nullptr;         // caller's host buffer [emax][eblock][n]
  int64_t emax = 0;
  hipStream_t estream = nullptr;   // copies
  hipEvent_t eev[2] = {nullptr, nullptr};  // copy of ring half h done
  hipEvent_t efill = nullptr;      // ring half filled (solve stream)
  int eissued[2] = {0, 0};         // a copy from ring half h is outstanding
  std::vector<char> ecopied;       // block b copied during this solve
  int64_t eblocks = 0;             // blocks of the last solve
  int32_t elast = 0;               // vectors in its last block
  // session
  int in_session = 0;
  int precond = 0;
  int pmode = 0;
  const double* x0 = nullptr;
  int64_t itmax = 0;
  int64_t enq = 0;
  // graph replay of blocks of iterations (launch-bound small systems)
  int use_graphs = 1;
  hipStream_t gstream = nullptr;  // non-blocking stream the graphs are captured and replayed on
  hipGraphExec_t gexec = nullptr;
  hipEvent_t gev[2] = {nullptr, nullptr};
  int64_t gsize = 0;
  uint64_t gkey = 0;
  // timing
  int timing = 0;
  std::vector<hipEvent_t> pool;
  std::vector<PendingTime> pending;
  double tms[5] = {0, 0, 0, 0, 0};
  int64_t tn[5] = {0, 0, 0, 0, 0};
};

static std::mutex g_mu;
static std::set<gsr_system*> g_live;

static int check_handle(gsr_system* s) {
  if (!s) return fail(GSR_EINVAL, "null handle");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_live.count(s)) return fail(GSR_EINVAL, "unknown or destroyed handle");
  return GSR_OK;
}

static int dev_alloc(void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    return fail(GSR_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  if (e != hipSuccess) return fail(GSR_EHIP, "hipMalloc: %s", hipGetErrorString(e));
  return GSR_OK;
}

template <typename T>
static int dalloc(T** p, size_t count) {
  return dev_alloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

static void dfree(void* p) {
  if (p) (void)hipFree(p);
}

static int is_device_ptr(const void* p) {
  if (!p) return 0;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

#define NEED_DEV(p, name)                                                                          \
  do {                                                                                             \
    if (!is_device_ptr(p)) return fail(GSR_EINVAL, "%s must be a device pointer", name);            \
  } while (0)

static int device_lds() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) return 65536;
  return v;
}

int gsr::device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
  return cus;
}

extern "C" int64_t gsr_num_unknowns(const gsr_dims* d) {
  if (!d || d->n_stars < 0 || d->m < 0 || d->n_att < 4 || d->n_instr < 6 || (d->n_glob != 0 && d->n_glob != 1))
    return -1;
  return 5 * d->n_stars + 3 * d->n_att + d->n_instr + d->n_glob;
}

static void reshape(gsr_system* s) { s->sh = stream_shape(s->s, s->cus, s->waves_per_cu); }

static int att_mode(const gsr_system* s) { return att_mode_of(s->s, s->av, s->att_atomics); }

// The attitude-bucketed copy used by the star-order passes when the attitude
// block does not fit in LDS, built at its first use (standalone aprod 2, solves
// that do not run on the regrouped copy).  Without memory for it those passes
// sum the attitude columns with device atomics.
static int ensure_att(gsr_system* s, hipStream_t st) {
  if (s->att_tried || s->s.tail_len <= kLdsTailMax || s->s.m == 0) return GSR_OK;
  s->att_tried = 1;
  HIPCHK(hipStreamSynchronize(st));
  char msg[256] = "";
  const int rc = att_build(s->s, &s->av, s->cus, msg, sizeof msg, st);
  if (rc == GSR_ENOMEM) return GSR_OK;  // att_mode falls back to atomics (view not ready)
  if (rc != GSR_OK) return fail(rc, "attitude view: %s", msg);
  return GSR_OK;
}

static void con_free(gsr_system* s) {
  for (const void* p : {(const void*)s->con.ptr, (const void*)s->con.col, (const void*)s->con.val,
                        (const void*)s->con.tile_e, (const void*)s->con.tile_r, (const void*)s->con.tmp,
                        (const void*)s->con_rhs})
    dfree(const_cast<void*>(p));
  s->con = ConView{};
  s->con_rhs = nullptr;
}

static void release(gsr_system* s) {
  (void)hipDeviceSynchronize();
  dfree(s->sc);
  dfree(s->psc);
  if (s->sc_host) (void)hipHostFree(s->sc_host);
  dfree(s->wk.part_a);
  dfree(s->wk.part_b);
  dfree(s->wk.part_c);
  dfree(s->wk.tickets);
  dfree(s->acc);
  dfree(s->S);
  dfree(s->u);
  dfree(s->v);
  dfree(s->vg);
  dfree(s->w);
  dfree(s->y);
  dfree(s->var);
  dfree(s->gA);
  con_free(s);
  dfree(s->zvec);
  dfree(s->pa);
  dfree(s->pb);
  dfree(s->Cp);
  dfree(s->ering);
  if (s->estream) (void)hipStreamDestroy(s->estream);
  for (hipEvent_t e : {s->eev[0], s->eev[1], s->efill})
    if (e) (void)hipEventDestroy(e);
  dfree(s->x3);
  dfree(s->awr);
  dfree(s->awrf);
  dfree(s->x3a);
  dfree(s->rix);
  dfree(s->xr);
  dfree(s->xn);
  dfree(s->nrm2);
  dfree(s->sel);
  dfree(s->D);
  dfree(s->Cacc);
  att_free(&s->av);
  blk_free(&s->blk);
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  for (auto e : s->gev)
    if (e) (void)hipEventDestroy(e);
  if (s->gstream) (void)hipStreamDestroy(s->gstream);
  for (auto e : s->pool) (void)hipEventDestroy(e);
  for (auto& p : s->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  delete s;
}

static void resolve_scratch(int dev);

// The handle's scalars, reduction partials, tickets and tail accumulators.
static int init_workspaces(gsr_system* s, hipStream_t st) {
  const SysView& v = s->s;
  CHK(dalloc(&s->sc, 1));
  CHK(dalloc(&s->wk.part_a, kPartialSlots));
  CHK(dalloc(&s->wk.part_b, kPartialSlots));
  CHK(dalloc(&s->wk.part_c, kPartialSlots));
  CHK(dalloc(&s->wk.tickets, kTickets));
  CHK(dalloc(&s->acc, (size_t)v.tail_len));
  if (hipHostMalloc((void**)&s->sc_host, sizeof(Scalars), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    s->sc_host = nullptr;
    return fail(GSR_ENOMEM, "pinned host allocation failed");
  }
  if (hipMemsetAsync(s->wk.tickets, 0, kTickets * sizeof(unsigned), st) != hipSuccess ||
      hipMemsetAsync(s->acc, 0, (size_t)v.tail_len * sizeof(double), st) != hipSuccess)
    return fail(GSR_EHIP, "workspace clear failed");
  return GSR_OK;
}

// Argument checks shared by gsr_create and gsr_layout_plan (vals may be absent).
static int check_system_args(const gsr_dims* d, const void* vals, const int64_t* star_row_ptr,
                             const int32_t* att_start, const int32_t* instr_col, int need_vals) {
  if (gsr_num_unknowns(d) < 0)
    return fail(GSR_EINVAL, "bad dims: need n_stars >= 0, m >= 0, n_att >= 4, n_instr >= 6, n_glob in {0,1}");
  if (d->value_type != GSR_F64 && d->value_type != GSR_F32) return fail(GSR_EINVAL, "bad value_type");
  if (d->n_att > INT32_MAX || d->n_instr > INT32_MAX) return fail(GSR_EINVAL, "n_att / n_instr too large");
  NEED_DEV(star_row_ptr, "star_row_ptr");
  if (d->m > 0) {
    if (need_vals) {
      NEED_DEV(vals, "vals");
      if ((uintptr_t)vals % 16) return fail(GSR_EINVAL, "vals must be 16-byte aligned");
    }
    NEED_DEV(att_start, "att_start");
    NEED_DEV(instr_col, "instr_col");
    if ((uintptr_t)instr_col % 8) return fail(GSR_EINVAL, "instr_col must be 8-byte aligned");
    if ((uintptr_t)att_start % 4) return fail(GSR_EINVAL, "att_start must be 4-byte aligned");
  }
  if ((uintptr_t)star_row_ptr % 8) return fail(GSR_EINVAL, "star_row_ptr must be 8-byte aligned");
  if (d->n_stars == 0 && d->m > 0) return fail(GSR_EINVAL, "rows without stars");
  if (d->n_instr + 1 > kLdsTailMax) return fail(GSR_EINVAL, "n_instr above %d is not supported", kLdsTailMax - 1);
  return GSR_OK;
}

static SysView make_view(const gsr_dims* d, const void* vals, const int64_t* star_row_ptr, const int32_t* att_start,
                         const int32_t* instr_col) {
  SysView v{};
  v.n_stars = d->n_stars;
  v.m = d->m;
  v.n_att = d->n_att;
  v.n_instr = d->n_instr;
  v.n_glob = d->n_glob;
  v.value_type = d->value_type;
  v.n_astro = 5 * d->n_stars;
  v.tail_len = 3 * d->n_att + d->n_instr + d->n_glob;
  v.n = v.n_astro + v.tail_len;
  v.vals = vals;
  v.row_ptr = star_row_ptr;
  v.att_start = att_start;
  v.instr_col = instr_col;
  v.has_empty_stars = 0;
  return v;
}

// Index validation on the device: the first bad row or star is reported.
static int validate_indices(SysView& v, hipStream_t st) {
  unsigned long long* bad = nullptr;
  CHK(dalloc(&bad, 3));
  unsigned long long hb[3] = {~0ull, ~0ull, 0ull};
  hipError_t e = hipMemcpyAsync(bad, hb, sizeof hb, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_validate(v, bad, st);
  if (e == hipSuccess) e = hipMemcpyAsync(hb, bad, sizeof hb, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(bad);
  if (e != hipSuccess) return fail(GSR_EHIP, "validation failed: %s", hipGetErrorString(e));
  if (hb[1] != ~0ull) return fail(GSR_EINVAL, "star_row_ptr invalid at star %llu", hb[1]);
  if (v.n_stars > 0) {
    int64_t ends[2];
    if (hipMemcpy(ends, v.row_ptr, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(ends + 1, v.row_ptr + v.n_stars, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(GSR_EHIP, "reading star_row_ptr failed");
    if (ends[0] != 0 || ends[1] != v.m) return fail(GSR_EINVAL, "star_row_ptr must run from 0 to m");
  }
  if (hb[0] != ~0ull) return fail(GSR_EINVAL, "att_start / instr_col out of range at row %llu", hb[0]);
  v.has_empty_stars = hb[2] != 0;
  return GSR_OK;
}

extern "C" int gsr_create(gsr_system** out, const gsr_dims* d, const void* vals, const int64_t* star_row_ptr,
                          const int32_t* att_start, const int32_t* instr_col, gsr_stream stream) {
  if (!out) return fail(GSR_EINVAL, "out is null");
  *out = nullptr;
  CHK(check_system_args(d, vals, star_row_ptr, att_start, instr_col, 1));

  gsr_system* s = new gsr_system();
  hipStream_t st = (hipStream_t)stream;
  s->s = make_view(d, vals, star_row_ptr, att_start, instr_col);
  SysView& v = s->s;
  (void)hipGetDevice(&s->device);
  s->cus = device_cus();
  resolve_scratch(s->device);  // set-up of gsr_aprod1_noalloc, once per device

  int rc = GSR_OK;
  auto bail = [&](int code) {
    release(s);
    return code;
  };
  if ((rc = init_workspaces(s, st))) return bail(rc);
  if ((rc = validate_indices(v, st))) return bail(rc);
  reshape(s);
  if (v.m > 0 && v.n_instr <= 65536) {
    // packed row indices for the fused iteration pass; without memory for them
    // iterations run as separate aprod 1 / aprod 2 passes
    if (hipMalloc(&s->rix, 16 * (size_t)v.m) == hipSuccess) {
      if (launch_pack_rows(v, s->rix, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return bail(fail(GSR_EHIP, "packing row indices failed"));
    } else {
      (void)hipGetLastError();
      s->rix = nullptr;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_live.insert(s);
  }
  *out = s;
  return GSR_OK;
}

// ------------------------------------------------------ rows placed by the caller
// A layout plan: the regrouped row order (records, positions, segments and the
// pass's workspaces) computed from the index data, without coefficients.  The
// caller places its rows with gsr_layout_pack into a buffer of its own, which
// gsr_create_packed then borrows: the library never holds a copy of A.
struct gsr_layout {
  gsr_dims d{};
  SysView v{};  // sizes; the caller's index arrays only during planning
  BlkView bv{};
  int device = 0;
};
static std::set<gsr_layout*> g_layouts;

static int check_layout(gsr_layout* L) {
  if (!L) return fail(GSR_EINVAL, "null layout");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_layouts.count(L)) return fail(GSR_EINVAL, "unknown, destroyed or consumed layout");
  return GSR_OK;
}

static void drop_layout(gsr_layout* L) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_layouts.erase(L);
  }
  delete L;
}

extern "C" int gsr_layout_plan(gsr_layout** out, const gsr_dims* d, const int64_t* star_row_ptr,
                               const int32_t* att_start, const int32_t* instr_col, int32_t max_window,
                               gsr_stream stream) {
  if (!out) return fail(GSR_EINVAL, "out is null");
  *out = nullptr;
  CHK(check_system_args(d, nullptr, star_row_ptr, att_start, instr_col, 0));
  if (d->m <= 0) return fail(GSR_EINVAL, "a layout needs rows (m > 0)");
  if (max_window != 0 && max_window < 4) return fail(GSR_EINVAL, "max_window must be 0 or >= 4");
  hipStream_t st = (hipStream_t)stream;
  gsr_layout* L = new gsr_layout();
  L->d = *d;
  L->v = make_view(d, nullptr, star_row_ptr, att_start, instr_col);
  (void)hipGetDevice(&L->device);
  int rc = validate_indices(L->v, st);
  if (rc != GSR_OK) {
    delete L;
    return rc;
  }
  char msg[256] = "";
  rc = blk_plan(L->v, &L->bv, device_cus(), max_window, device_lds(), msg, sizeof msg, st);
  if (rc != GSR_OK) {
    delete L;
    return fail(rc, "layout: %s", msg);
  }
  L->v.vals = nullptr;
  L->v.row_ptr = nullptr;
  L->v.att_start = nullptr;
  L->v.instr_col = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_layouts.insert(L);
  }
  *out = L;
  return GSR_OK;
}

static void layout_info(const BlkView& b, int active, int owned, gsr_blocked_layout* info) {
  memset(info, 0, sizeof *info);
  info->active = active;
  info->workgroups = b.G;
  info->window = b.Wb;
  info->blocks = b.nb;
  info->padded_rows = b.mp;
  info->segments = b.nseg;
  info->bytes = (int64_t)blk_index_bytes(b);
  info->value_bytes = (int64_t)blk_value_bytes(b);
  info->values_owned = owned;
}

extern "C" int gsr_layout_info(gsr_layout* L, gsr_blocked_layout* info) {
  CHK(check_layout(L));
  if (!info) return fail(GSR_EINVAL, "info is null");
  layout_info(L->bv, 0, 0, info);
  return GSR_OK;
}

extern "C" int gsr_layout_pack(gsr_layout* L, const void* rows, int64_t row0, int64_t count, void* packed,
                               gsr_stream stream) {
  CHK(check_layout(L));
  if (row0 < 0 || count < 0 || row0 + count > L->d.m)
    return fail(GSR_EINVAL, "rows %lld .. %lld outside [0, m = %lld)", (long long)row0, (long long)(row0 + count),
                (long long)L->d.m);
  if (count == 0) return GSR_OK;
  NEED_DEV(rows, "rows");
  NEED_DEV(packed, "packed");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != L->device) return fail(GSR_EINVAL, "the layout's device must be current");
  if ((uintptr_t)rows % 16 || (uintptr_t)packed % 16) return fail(GSR_EINVAL, "rows and packed must be 16-byte aligned");
  HIPCHK(launch_blk_pack(L->bv, rows, row0, count, packed, (hipStream_t)stream));
  return GSR_OK;
}

extern "C" int gsr_layout_destroy(gsr_layout* L) {
  if (!L) return GSR_OK;
  CHK(check_layout(L));
  (void)hipDeviceSynchronize();
  blk_free(&L->bv);
  drop_layout(L);
  return GSR_OK;
}

extern "C" int gsr_create_packed(gsr_system** out, gsr_layout* L, void* packed, gsr_stream stream) {
  if (!out) return fail(GSR_EINVAL, "out is null");
  *out = nullptr;
  CHK(check_layout(L));
  NEED_DEV(packed, "packed");
  if ((uintptr_t)packed % 16) return fail(GSR_EINVAL, "packed must be 16-byte aligned");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != L->device) return fail(GSR_EINVAL, "the layout's device must be current");
  hipStream_t st = (hipStream_t)stream;
  gsr_system* s = new gsr_system();
  s->s = L->v;
  s->device = dev;
  s->cus = device_cus();
  s->packed = 1;
  resolve_scratch(s->device);
  int rc = init_workspaces(s, st);
  if (rc == GSR_OK) rc = dalloc(&s->psc, 1);
  if (rc == GSR_OK && (launch_blk_zero_pad(L->bv, packed, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)) {
    (void)hipGetLastError();
    rc = fail(GSR_EHIP, "clearing the padding rows failed");
  }
  if (rc != GSR_OK) {
    release(s);  // the layout stays with the caller
    return rc;
  }
  reshape(s);
  // the handle takes the layout over; the coefficients stay in the caller's buffer
  s->blk = L->bv;
  s->blk.T = packed;
  s->blk.t_owned = 0;
  s->blk.ready = 1;
  L->bv = BlkView{};
  drop_layout(L);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_live.insert(s);
  }
  *out = s;
  return GSR_OK;
}

extern "C" int gsr_destroy(gsr_system* s) {
  if (!s) return GSR_OK;
  CHK(check_handle(s));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_live.erase(s);
  }
  release(s);
  return GSR_OK;
}

extern "C" int gsr_set_tuning(gsr_system* s, int32_t waves_per_cu, int32_t att_atomics) {
  CHK(check_handle(s));
  if (waves_per_cu < 1 || waves_per_cu > 256 || (att_atomics != 0 && att_atomics != 1))
    return fail(GSR_EINVAL, "waves_per_cu in [1,256], att_atomics in {0,1}");
  s->waves_per_cu = waves_per_cu;
  s->att_atomics = att_atomics;
  reshape(s);
  return GSR_OK;
}

extern "C" int gsr_set_graphs(gsr_system* s, int32_t on) {
  CHK(check_handle(s));
  s->use_graphs = on != 0;
  return GSR_OK;
}

extern "C" int gsr_set_fused(gsr_system* s, int32_t on) {
  CHK(check_handle(s));
  if (s->in_session) return fail(GSR_ESTATE, "gsr_set_fused: a solve is in progress");
  if (s->packed && !on) return fail(GSR_EINVAL, "gsr_set_fused: a handle over packed rows runs the one-pass iteration");
  s->fused = on != 0;
  return GSR_OK;
}

static void drop_graph(gsr_system* s);

extern "C" int gsr_set_blocked(gsr_system* s, int32_t on, int32_t max_window) {
  CHK(check_handle(s));
  if (s->in_session) return fail(GSR_ESTATE, "gsr_set_blocked: a solve is in progress");
  if (max_window != 0 && max_window < 4) return fail(GSR_EINVAL, "max_window must be 0 or >= 4");
  if (s->packed) {
    if (!on || max_window != 0)
      return fail(GSR_EINVAL, "gsr_set_blocked: a packed handle keeps its layout (set max_window in gsr_layout_plan)");
    return GSR_OK;
  }
  if (max_window != s->blk_maxw) {
    (void)hipDeviceSynchronize();
    blk_free(&s->blk);  // rebuilt with the new width when next used
    s->blk_failed = 0;
    drop_graph(s);
  }
  s->blocked = on != 0;
  s->blk_maxw = max_window;
  return GSR_OK;
}

extern "C" int gsr_blocked_info(gsr_system* s, gsr_blocked_layout* info) {
  CHK(check_handle(s));
  if (!info) return fail(GSR_EINVAL, "info is null");
  memset(info, 0, sizeof *info);
  if (!s->blk.ready) return GSR_OK;
  layout_info(s->blk, 1, s->blk.t_owned, info);
  return GSR_OK;
}

// ------------------------------------------------------------------ timing
static int ev_get(gsr_system* s, hipEvent_t* e) {
  if (!s->pool.empty()) {
    *e = s->pool.back();
    s->pool.pop_back();
    return GSR_OK;
  }
  HIPCHK(hipEventCreate(e));
  return GSR_OK;
}

struct TimeScope {
  gsr_system* s;
  int kind;
  hipStream_t st;
  hipEvent_t a{}, b{};
  bool on;
  TimeScope(gsr_system* s_, int k, hipStream_t st_) : s(s_), kind(k), st(st_), on(s_->timing != 0) {
    if (on && (ev_get(s, &a) != GSR_OK || ev_get(s, &b) != GSR_OK || hipEventRecord(a, st) != hipSuccess)) on = false;
  }
  ~TimeScope() {
    if (!on) return;
    if (hipEventRecord(b, st) == hipSuccess) s->pending.push_back({kind, a, b});
  }
};

extern "C" int gsr_timing_enable(gsr_system* s, int32_t on) {
  CHK(check_handle(s));
  s->timing = on != 0;
  return GSR_OK;
}

extern "C" int gsr_timing_get(gsr_system* s, gsr_timing* t) {
  CHK(check_handle(s));
  if (!t) return fail(GSR_EINVAL, "t is null");
  for (auto& p : s->pending) {
    HIPCHK(hipEventSynchronize(p.b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    s->tms[p.kind] += ms;
    s->tn[p.kind] += 1;
    s->pool.push_back(p.a);
    s->pool.push_back(p.b);
  }
  s->pending.clear();
  t->aprod1_ms = s->tms[0];
  t->aprod2_ms = s->tms[1];
  t->tail_ms = s->tms[2];
  t->update_ms = s->tms[3];
  t->syrk_ms = s->tms[4];
  t->aprod1_n = s->tn[0];
  t->aprod2_n = s->tn[1];
  t->tail_n = s->tn[2];
  t->update_n = s->tn[3];
  t->syrk_n = s->tn[4];
  for (int i = 0; i < 5; ++i) {
    s->tms[i] = 0;
    s->tn[i] = 0;
  }
  return GSR_OK;
}

// ------------------------------------------------------------------ products
static int check_product(gsr_system* s, int32_t product) {
  if (product != GSR_PROD_F64 && product != GSR_PROD_F32) return fail(GSR_EINVAL, "bad product mode");
  if (product == GSR_PROD_F32 && s->s.value_type != GSR_F32)
    return fail(GSR_EINVAL, "FP32 products need an FP32 system");
  return GSR_OK;
}

static int ensure_x3a(gsr_system* s) {
  if (!s->x3a) CHK(dalloc(&s->x3a, (size_t)std::max<int64_t>(kAttRec * s->s.n_att, 1)));
  return GSR_OK;
}

// The regrouped rows for a standalone pass: the caller's packed buffer, or the
// library's copy (built at first use) on a handle over rows in star order.
static int ensure_blk(gsr_system* s, hipStream_t st) {
  if (!s->blk.ready) {
    if (s->blk_failed) return fail(GSR_ENOMEM, "the regrouped copy could not be built");
    char msg[256] = "";
    HIPCHK(hipStreamSynchronize(st));
    const int rc = blk_build(s->s, &s->blk, s->cus, s->blk_maxw, device_lds(), msg, sizeof msg, st);
    if (rc != GSR_OK) {
      if (rc != GSR_EHIP) s->blk_failed = 1;
      return fail(rc, "regrouped copy: %s", msg);
    }
  }
  if (!s->psc) CHK(dalloc(&s->psc, 1));
  return GSR_OK;
}

// Work vectors of the standalone passes over the regrouped rows.
static int ensure_blk_vectors(gsr_system* s, int32_t product, hipStream_t st) {
  const size_t nr = (size_t)std::max<int64_t>(kAttRec * s->s.n_att, 1);
  if (!s->awr) CHK(dalloc(&s->awr, nr));
  if (product == GSR_PROD_F32 && !s->awrf) CHK(dalloc(&s->awrf, nr));
  if (!s->gA) CHK(dalloc(&s->gA, (size_t)std::max<int64_t>(s->s.n_astro, 1)));
  if (!s->zvec) {
    CHK(dalloc(&s->zvec, (size_t)s->s.n));
    HIPCHK(launch_fill(s->zvec, s->s.n, 0.0, st));
  }
  return GSR_OK;
}

// Standalone products as one pass over the regrouped rows (the LSQR
// iteration's pass with its own scalars, whose epilogues only record norms):
//   u' = su * u_in + A v (rows in the caller's order; u_in null: u' = A v), written
//   to u_out unless it is null; with want_t also x <- sx * x + A^T u' (every column).
// square = 1: x <- column sums of squares instead (v, u_in ignored).
static int no_session(gsr_system* s) {
  if (s->in_session) return fail(GSR_ESTATE, "a solve is in progress (its u occupies the regrouped rows' vector)");
  return GSR_OK;
}

static int blk_products(gsr_system* s, const double* v, const double* u_in, double* u_out, double su, double* x,
                        double sx, int32_t product, int want_t, int square, int kind, hipStream_t st) {
  CHK(ensure_blk(s, st));
  CHK(ensure_blk_vectors(s, product, st));
  if (s->s.m == 0) return GSR_OK;
  TimeScope ts(s, kind, st);
  const BlkView& bv = s->blk;
  if (!v || square) v = s->zvec;
  if (u_in && !square)
    HIPCHK(launch_blk_permute(bv, u_in, st));
  else
    su = 0.0;
  HIPCHK(launch_att_records(s->s, v, s->awr, st, product == GSR_PROD_F32 ? s->awrf : nullptr));
  HIPCHK(launch_raw_scalars(s->psc, su, sx, st));
  HIPCHK(launch_fblk(s->s, bv, square ? GSR_PROD_F64 : product, v, s->awr, s->awrf, s->acc, s->psc, s->wk, st, 0,
                     square));
  if (want_t || square) {
    HIPCHK(launch_tail_seg(s->s, bv, x, s->acc, nullptr, s->psc, s->wk, st, 1));
  } else {
    // the pass added its instrumental and global sums into the tail accumulators
    HIPCHK(launch_fill(s->acc + 3 * s->s.n_att, s->s.n_instr + s->s.n_glob, 0.0, st));
  }
  if (u_out) HIPCHK(launch_blk_unpermute(bv, u_out, st));
  return GSR_OK;
}

extern "C" int gsr_aprod12(gsr_system* s, const double* v, double* u, double scale_u, double* x, double scale_x,
                           int32_t product, gsr_stream stream) {
  CHK(check_handle(s));
  CHK(check_product(s, product));
  NEED_DEV(v, "v");
  NEED_DEV(x, "x");
  if (s->s.m > 0) NEED_DEV(u, "u");
  if (s->con.ncon > 0) return fail(GSR_EINVAL, "gsr_aprod12 computes with A alone: detach the constraints first");
  CHK(no_session(s));
  if (s->s.m == 0) {
    // no rows: A^T u' = 0
    HIPCHK(launch_scaled_copy(x, x, s->s.n, scale_x, (hipStream_t)stream));
    return GSR_OK;
  }
  return blk_products(s, v, u, u, scale_u, x, scale_x, product, 1, 0, 0, (hipStream_t)stream);
}

extern "C" int gsr_aprod1(gsr_system* s, const double* x, double* y, double scale_y, int32_t product,
                          gsr_stream stream) {
  CHK(check_handle(s));
  CHK(check_product(s, product));
  NEED_DEV(x, "x");
  if (s->s.m > 0) NEED_DEV(y, "y");
  if (s->s.m == 0) return GSR_OK;
  if (s->packed) {
    CHK(no_session(s));
    return blk_products(s, x, y, y, scale_y, nullptr, 0.0, product, 0, 0, 0, (hipStream_t)stream);
  }
  TimeScope ts(s, 0, (hipStream_t)stream);
  CHK(ensure_x3a(s));
  HIPCHK(launch_aprod1(s->s, s->sh, x, s->x3a, y, scale_y, 1.0, product, nullptr, s->wk, 0, (hipStream_t)stream));
  return GSR_OK;
}

// ------------------------------------------------- aprod 1 without allocation
// The only workspace of the standalone aprod 1 is the attitude window records
// of x (kAttRec n_att doubles).  gsr_aprod1_noalloc takes it from this
// file-scope device array instead of a handle allocation; every GPU the
// library runs on holds its own copy for the life of the process.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in symbol): its device address is looked up once per device, with that
// device current, when the first handle on the device is created.
constexpr int64_t kScratchDoubles = (int64_t)1 << 21;  // 16 MiB: attitude blocks up to 131,072 per axis
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static double* g_scratch[kMaxDevices] = {};
static int g_scratch_rc[kMaxDevices] = {};  // 0 not looked up, 1 resolved, -1 lookup failed

static void resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch_rc[dev] != 0) return;
  double* p = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    g_scratch_rc[dev] = -1;
    return;
  }
  g_scratch[dev] = p;
  g_scratch_rc[dev] = 1;
}

extern "C" int gsr_aprod1_noalloc(gsr_system* s, const double* x, double* y, double scale_y, int32_t product,
                                  gsr_stream stream) {
  CHK(check_handle(s));
  CHK(check_product(s, product));
  NEED_DEV(x, "x");
  if (s->s.m > 0) NEED_DEV(y, "y");
  if (s->packed) return fail(GSR_EINVAL, "gsr_aprod1_noalloc runs on handles made by gsr_create");
  if (kAttRec * s->s.n_att > kScratchDoubles)
    return fail(GSR_EINVAL, "16 * n_att = %lld exceeds the no-allocation scratch of %lld doubles",
                (long long)(kAttRec * s->s.n_att), (long long)kScratchDoubles);
  if (s->s.m == 0) return GSR_OK;
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != s->device) return fail(GSR_EINVAL, "the handle's device must be current");
  double* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev >= 0 && dev < kMaxDevices && g_scratch_rc[dev] == 1) ptr = g_scratch[dev];
  }
  if (!ptr) return fail(GSR_EHIP, "the device address of the no-allocation scratch is not available");
  // no timing scope here: recording events may allocate them
  HIPCHK(launch_aprod1(s->s, s->sh, x, ptr, y, scale_y, 1.0, product, nullptr, s->wk, 0, (hipStream_t)stream));
  return GSR_OK;
}

// aprod 2 in LSQR form (sc != nullptr: scale / 1/beta from the device scalars) or standalone.
static int aprod2_launches(gsr_system* s, const double* y, double* x, const double* S, double scale, int32_t product,
                           int square, Scalars* sc, int lsqr_stage, hipStream_t st) {
  // the column norms (square) are taken once: without the bucketed view they use
  // device atomics rather than build it for that alone
  if (!square) CHK(ensure_att(s, st));
  const int mode = att_mode(s);
  {
    TimeScope ts(s, 1, st);
    if (mode == 3 && !square) HIPCHK(launch_partition(s->s, s->av, y, sc, st));
    HIPCHK(launch_aprod2(s->s, s->sh, mode, mode == 3 ? s->av.sv : nullptr, y, x, s->acc, S, scale, 1.0, product, square, sc, s->wk, st));
    if (mode == 3) HIPCHK(launch_att_pass(s->s, s->av, 1.0, product, square, sc, st));
  }
  TimeScope ts(s, 2, st);
  if (sc)
    HIPCHK(launch_tail(s->s, s->av, mode, x, s->acc, S, 0.0, sc, s->wk, lsqr_stage, s->sh.blocks, st));
  else
    HIPCHK(launch_tail(s->s, s->av, mode, x, s->acc, nullptr, scale, nullptr, s->wk, 0, 0, st));
  return GSR_OK;
}

static int aprod2_raw(gsr_system* s, const double* y, double* x, double scale_x, int32_t product, int square,
                      hipStream_t st) {
  return aprod2_launches(s, y, x, nullptr, scale_x, product, square, nullptr, 0, st);
}

extern "C" int gsr_aprod2(gsr_system* s, const double* y, double* x, double scale_x, int32_t product,
                          gsr_stream stream) {
  CHK(check_handle(s));
  CHK(check_product(s, product));
  NEED_DEV(x, "x");
  if (s->s.m > 0) NEED_DEV(y, "y");
  if (s->packed) {
    CHK(no_session(s));
    return blk_products(s, nullptr, y, nullptr, 1.0, x, scale_x, product, 1, 0, 1, (hipStream_t)stream);
  }
  return aprod2_raw(s, y, x, scale_x, product, 0, (hipStream_t)stream);
}

static int ensure_scale(gsr_system* s, hipStream_t st) {
  if (s->S_valid) return GSR_OK;
  if (!s->S) CHK(dalloc(&s->S, (size_t)s->s.n));
  // column sums of squares with the aprod 2 machinery (on packed rows the
  // regrouped pass in its square mode), then 1/sqrt
  if (s->packed && s->s.m > 0)
    CHK(blk_products(s, nullptr, nullptr, nullptr, 0.0, s->S, 0.0, GSR_PROD_F64, 1, 1, 1, st));
  else
    CHK(aprod2_raw(s, nullptr, s->S, 0.0, 0, 1, st));
  HIPCHK(launch_con_sq(s->con, s->S, st));  // columns of [A; C]
  HIPCHK(launch_scale_from_sq(s->s.n, s->S, st));
  s->S_valid = 1;
  return GSR_OK;
}

extern "C" int gsr_column_scale(gsr_system* s, double* out, gsr_stream stream) {
  CHK(check_handle(s));
  hipStream_t st = (hipStream_t)stream;
  CHK(ensure_scale(s, st));
  if (out) {
    NEED_DEV(out, "scale_out");
    HIPCHK(hipMemcpyAsync(out, s->S, (size_t)s->s.n * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  return GSR_OK;
}

// ------------------------------------------------------------------ LSQR
static int check_opts(const gsr_lsqr_opts* o) {
  if (!o) return fail(GSR_EINVAL, "opts is null");
  if (!(o->damp >= 0) || !(o->atol >= 0) || !(o->btol >= 0) || !(o->conlim >= 0) || o->itmax < 0)
    return fail(GSR_EINVAL, "opts: damp, atol, btol, conlim and itmax must be >= 0");
  if (o->precond != 0 && o->precond != 1) return fail(GSR_EINVAL, "opts.precond must be 0 or 1");
  return GSR_OK;
}

// The constraint rows of the LSQR u vector (after its m rows, or alone when the
// rows are packed and u lives in the regrouped order).
static double* u_con(gsr_system* s) { return s->u + (s->packed ? 0 : s->s.m); }

static int ensure_vectors(gsr_system* s) {
  const size_t m = (size_t)s->s.m, n = (size_t)s->s.n;
  // packed rows: u lives in the regrouped order only; this holds the constraint rows
  if (!s->u) CHK(dalloc(&s->u, (s->packed ? 0 : m) + (size_t)s->con.ncon));
  if (!s->v) CHK(dalloc(&s->v, n));
  if (!s->vg) CHK(dalloc(&s->vg, n));
  if (!s->w) CHK(dalloc(&s->w, n));
  if (!s->y) CHK(dalloc(&s->y, n));
  if (!s->var) CHK(dalloc(&s->var, n));
  if (!s->gA) CHK(dalloc(&s->gA, (size_t)std::max<int64_t>(s->s.n_astro, 1)));
  if (!s->x3) CHK(dalloc(&s->x3, (size_t)std::max<int64_t>(kAttRec * s->s.n_att, 1)));
  CHK(ensure_x3a(s));
  return GSR_OK;
}

// Whether an iteration runs as one pass over the rows (plus the attitude and
// tail passes) instead of separate aprod 1 and aprod 2 passes.
static int fused_for(const gsr_system* s, int32_t pmode) {
  const int mode = att_mode(s);
  return s->fused && (mode == 0 || mode == 3) && s->rix != nullptr;
}

static int iteration_fused(const gsr_system* s) { return fused_for(s, s->pmode); }

// Whether a solve runs on the copy regrouped by attitude window.
static int blk_applies(const gsr_system* s) {
  if (s->packed) return 1;
  return s->blocked && s->fused && !s->blk_failed && s->s.m > 0 && s->s.tail_len > kLdsTailMax &&
         s->s.n_instr + 1 <= kLdsTailMax;
}

// The attitude window records that the next row pass reads: the regrouped pass's
// (and their FP32 rounding with FP32 products), or the star-order fused pass's.
static hipError_t att_copy_for_pass(gsr_system* s, const double* v, hipStream_t st) {
  if (s->use_blk) return launch_att_records(s->s, v, s->awr, st, s->pmode == GSR_PROD_F32 ? s->awrf : nullptr);
  return launch_att_records(s->s, v, s->x3, st);
}

// fold_r0: on the regrouped copy, form r0 = b - A x0 inside the first pass
// (u' = u + A vg with vg = -x0, FP64 products) instead of by a separate aprod 1;
// the rounding of r0 then follows the pass's summation order.
static int lsqr_begin(gsr_system* s, const double* b, const double* x0, const gsr_lsqr_opts* o, int32_t product,
                      hipStream_t st, int fold_r0 = 0) {
  CHK(check_opts(o));
  CHK(check_product(s, product));
  if (s->s.m > 0) NEED_DEV(b, "b");
  if (x0) NEED_DEV(x0, "x0");
  if (!blk_applies(s)) CHK(ensure_att(s, st));
  if (s->con.ncon > 0 && (product != GSR_PROD_F64 || !(fused_for(s, product) || blk_applies(s))))
    return fail(GSR_EINVAL, "constraint equations need the fused iteration (FP64 products, fused on, "
                            "attitude in LDS, regrouped or bucketed)");
  CHK(ensure_vectors(s));
  if (o->precond) CHK(ensure_scale(s, st));
  s->use_blk = 0;
  if (blk_applies(s)) {
    if (!s->blk.ready) {
      char msg[256] = "";
      HIPCHK(hipStreamSynchronize(st));
      const int rc = blk_build(s->s, &s->blk, s->cus, s->blk_maxw, device_lds(), msg, sizeof msg, st);
      if (rc == GSR_EHIP) return fail(rc, "regrouped copy: %s", msg);
      if (rc != GSR_OK) s->blk_failed = 1;  // no memory for it, or outside its limits: the bucketed pass
    }
    s->use_blk = s->blk.ready;
  }
  if (!s->use_blk) CHK(ensure_att(s, st));
  if (s->use_blk) {
    const size_t nr = (size_t)std::max<int64_t>(kAttRec * s->s.n_att, 1);
    if (!s->awr) CHK(dalloc(&s->awr, nr));
    if (product == GSR_PROD_F32 && !s->awrf) CHK(dalloc(&s->awrf, nr));
  }
  if (s->con.ncon > 0 && !s->use_blk && !fused_for(s, product))
    return fail(GSR_EINVAL, "constraint equations need the fused iteration (no memory for the regrouped copy "
                            "and no bucketed attitude view)");
  s->precond = o->precond;
  s->pmode = product;
  s->x0 = x0;
  s->itmax = o->itmax;
  s->enq = 0;
  if (s->eblock) {
    HIPCHK(hipStreamSynchronize(s->estream));
    s->eissued[0] = s->eissued[1] = 0;
    s->ecopied.assign((size_t)((o->itmax + s->eblock - 1) / s->eblock + 1), 0);
    s->eblocks = 0;
    s->elast = 0;
  }
  const double* S = o->precond ? s->S : nullptr;

  Scalars h;
  memset(&h, 0, sizeof h);
  h.damp = o->damp;
  h.atol = o->atol;
  h.btol = o->btol;
  h.ctol = o->conlim > 0 ? 1.0 / o->conlim : 0.0;
  h.itmax = o->itmax;
  h.nsel = s->nsel;
  h.dblock = s->dblock;
  h.u_scale = 1.0;  // the constrained solve's first pass forms u' = 1*u + A 0
  *s->sc_host = h;
  HIPCHK(hipMemcpyAsync(s->sc, s->sc_host, sizeof(Scalars), hipMemcpyHostToDevice, st));
  if (s->nsel > 0) {
    if (s->npairs > 0)
      HIPCHK(launch_fill(s->Cp, s->npairs, 0.0, st));
    else
      HIPCHK(launch_fill(s->Cacc, s->nsel * s->nsel, 0.0, st));
    s->cov_precond = o->precond;
  }
  // r0 = [b; c] - [A; C] x0 (on packed rows always inside the first pass)
  const int r0_in_pass = s->use_blk && (fold_r0 || s->packed) && x0;
  double* uc = u_con(s);  // constraint rows of u
  if (!r0_in_pass && !(s->use_blk && !x0)) {
    HIPCHK(launch_copy(b, s->u, s->s.m, st));
    if (x0 && s->s.m > 0)
      HIPCHK(launch_aprod1(s->s, s->sh, x0, s->x3a, s->u, 1.0, -1.0, 0, nullptr, s->wk, 0, st));
  }
  if (s->con.ncon > 0) HIPCHK(launch_copy(s->con_rhs, uc, s->con.ncon, st));
  if (x0) HIPCHK(launch_con_aprod1(s->con, x0, uc, 1.0, -1.0, nullptr, s->wk, st));
  if (s->use_blk) {
    // r0 in the regrouped order; then beta_1 and alpha_1 v_1 by the iteration's
    // own pass with x = 0 (u' = u), or x = -x0 on b when r0 is formed there,
    // and the init steps of the scalar recurrences
    if (!s->zvec) {
      CHK(dalloc(&s->zvec, (size_t)s->s.n));
      HIPCHK(launch_fill(s->zvec, s->s.n, 0.0, st));
    }
    const double* vg0 = s->zvec;
    int32_t pm0 = product;
    if (r0_in_pass) {
      HIPCHK(launch_blk_permute(s->blk, b, st));
      HIPCHK(launch_scaled_copy(x0, s->y, s->s.n, -1.0, st));  // y is free until init_vectors
      vg0 = s->y;
      pm0 = GSR_PROD_F64;
    } else {
      HIPCHK(launch_blk_permute(s->blk, x0 ? s->u : b, st));
    }
    HIPCHK(launch_att_records(s->s, vg0, s->awr, st, pm0 == GSR_PROD_F32 ? s->awrf : nullptr));
    // constraint rows of u stay after the m rows of s->u (uc)
    if (s->con.ncon > 0) HIPCHK(launch_con_aprod1(s->con, s->zvec, uc, 0.0, 1.0, s->sc, s->wk, st));
    HIPCHK(launch_fblk(s->s, s->blk, pm0, vg0, s->awr, s->awrf, s->acc, s->sc, s->wk, st, 1));
    if (s->con.ncon > 0) {
      HIPCHK(launch_seg_reduce(s->s, s->blk, s->gA, s->sc, st));
      HIPCHK(launch_con_aprod2(s->con, s->s.n_astro, uc, s->gA, s->acc, s->sc, st));
      HIPCHK(launch_tail_blk(s->s, s->blk, s->v, s->acc, S, s->gA, s->sc, s->wk, st, 0));
    } else {
      HIPCHK(launch_tail_seg(s->s, s->blk, s->v, s->acc, S, s->sc, s->wk, st, 0));
    }
  } else if (s->con.ncon > 0 || iteration_fused(s)) {
    // beta_1 u_1 = r0 and alpha_1 v_1 = S [A; C]^T u_1 through the iteration's own
    // passes, with x = 0 (u' = u) and the init steps of the scalar recurrences: the
    // first A^T product then takes its operand in the same (unnormalised) form as
    // every later one
    const int mode = att_mode(s);
    if (!s->zvec) {
      CHK(dalloc(&s->zvec, (size_t)s->s.n));
      HIPCHK(launch_fill(s->zvec, s->s.n, 0.0, st));
    }
    HIPCHK(launch_att_records(s->s, s->zvec, s->x3, st));
    if (s->con.ncon > 0) HIPCHK(launch_con_aprod1(s->con, s->zvec, uc, 0.0, 1.0, s->sc, s->wk, st));
    HIPCHK(launch_fused(s->s, s->sh, mode, product, s->zvec, s->x3, s->rix, s->u, s->gA, s->acc, s->sc, s->wk, st,
                        1));
    if (mode == 3) {
      HIPCHK(launch_partition(s->s, s->av, s->u, s->sc, st));
      HIPCHK(launch_att_pass(s->s, s->av, 1.0, product, 0, s->sc, st, 1));
    }
    if (s->con.ncon > 0) HIPCHK(launch_con_aprod2(s->con, s->s.n_astro, uc, s->gA, s->acc, s->sc, st));
    HIPCHK(launch_tail_fused(s->s, s->av, mode, s->v, s->acc, S, s->gA, s->sc, s->wk, st, 0));
  } else {
    HIPCHK(launch_norm_init(s->u, s->s.m, s->sc, s->wk, st));
    // alpha_1 v_1 = S A^T u_1
    CHK(aprod2_launches(s, s->u, s->v, S, 0.0, product, 0, s->sc, 0, st));
  }
  HIPCHK(launch_init_vectors(s->s.n, s->v, s->vg, s->w, s->y, s->var, S, s->sc, st));
  if (s->use_blk || iteration_fused(s)) HIPCHK(att_copy_for_pass(s, o->precond ? s->vg : s->v, st));
  s->in_session = 1;
  return GSR_OK;
}

extern "C" int gsr_lsqr_begin(gsr_system* s, const double* b, const double* x0, const gsr_lsqr_opts* o,
                              gsr_stream stream) {
  CHK(check_handle(s));
  if (!o) return fail(GSR_EINVAL, "opts is null");
  return lsqr_begin(s, b, x0, o, o->product, (hipStream_t)stream);
}

// One LSQR iteration: aprod 1, aprod 2 (+ tail), update, and the covariance
// SYRK when a block of `dblock` columns is complete.
// One covariance update from the buffered columns: SYRK for a dense block, the
// pair dot products for a pair list.
static hipError_t cov_flush(gsr_system* s, hipStream_t st) {
  if (s->npairs > 0) return launch_pairdot(s->D, s->dblock, s->pa, s->pb, s->npairs, s->Cp, s->sc, s->wk, -1, st);
  return launch_syrk(s->D, s->nsel, s->dblock, s->Cacc, s->sc, s->wk, -1, st);
}

// Export: copy ring half h (block b, `rows` vectors) into the caller's buffer on
// the copy stream, after what the solve stream has enqueued so far.
static int export_copy(gsr_system* s, int64_t b, int64_t rows, hipStream_t st) {
  const int h = (int)(b & 1);
  const size_t n = (size_t)s->s.n;
  if (b >= s->emax || rows <= 0) return GSR_OK;
  HIPCHK(hipEventRecord(s->efill, st));
  HIPCHK(hipStreamWaitEvent(s->estream, s->efill, 0));
  HIPCHK(hipMemcpyAsync(s->ehost + (size_t)b * s->eblock * n, s->ering + (size_t)h * s->eblock * n,
                        sizeof(double) * (size_t)rows * n, hipMemcpyDeviceToHost, s->estream));
  HIPCHK(hipEventRecord(s->eev[h], s->estream));
  s->eissued[h] = 1;
  if ((size_t)b < s->ecopied.size()) s->ecopied[(size_t)b] = 1;
  return GSR_OK;
}

static int enqueue_iteration(gsr_system* s, hipStream_t st) {
  const double* S = s->precond ? s->S : nullptr;
  double* vg = s->precond ? s->vg : s->v;
  if (s->eblock && s->enq % s->eblock == 0) {
    // this iteration starts refilling ring half h: its previous copy must be done
    const int h = (int)((s->enq / s->eblock) & 1);
    if (s->eissued[h]) HIPCHK(hipStreamWaitEvent(st, s->eev[h], 0));
  }
  if (s->use_blk) {
    double* uc = u_con(s);  // constraint rows of u
    if (s->con.ncon > 0) {
      TimeScope ts(s, 2, st);
      HIPCHK(launch_con_aprod1(s->con, vg, uc, 0.0, 1.0, s->sc, s->wk, st));
    }
    {
      TimeScope ts(s, 0, st);
      HIPCHK(launch_fblk(s->s, s->blk, s->pmode, vg, s->awr, s->awrf, s->acc, s->sc, s->wk, st));
    }
    if (s->con.ncon > 0) {
      // the constraint rows add into the raw sums between the segment reduction and the tail
      {
        TimeScope ts(s, 1, st);
        HIPCHK(launch_seg_reduce(s->s, s->blk, s->gA, s->sc, st));
      }
      TimeScope ts(s, 2, st);
      HIPCHK(launch_con_aprod2(s->con, s->s.n_astro, uc, s->gA, s->acc, s->sc, st));
      HIPCHK(launch_tail_blk(s->s, s->blk, s->v, s->acc, S, s->gA, s->sc, s->wk, st));
    } else {
      TimeScope ts(s, 2, st);
      HIPCHK(launch_tail_seg(s->s, s->blk, s->v, s->acc, S, s->sc, s->wk, st));
    }
  } else if (iteration_fused(s)) {
    const int mode = att_mode(s);
    double* uc = u_con(s);
    if (s->con.ncon > 0) {
      TimeScope ts(s, 2, st);
      HIPCHK(launch_con_aprod1(s->con, vg, uc, 0.0, 1.0, s->sc, s->wk, st));
    }
    {
      TimeScope ts(s, 0, st);
      HIPCHK(launch_fused(s->s, s->sh, mode, s->pmode, vg, s->x3, s->rix, s->u, s->gA, s->acc, s->sc, s->wk, st));
    }
    if (mode == 3) {
      TimeScope ts(s, 1, st);
      HIPCHK(launch_partition(s->s, s->av, s->u, s->sc, st));
      HIPCHK(launch_att_pass(s->s, s->av, 1.0, s->pmode, 0, s->sc, st, 1));
    }
    if (s->con.ncon > 0) {
      TimeScope ts(s, 2, st);
      HIPCHK(launch_con_aprod2(s->con, s->s.n_astro, uc, s->gA, s->acc, s->sc, st));
    }
    {
      TimeScope ts(s, 2, st);
      HIPCHK(launch_tail_fused(s->s, s->av, mode, s->v, s->acc, S, s->gA, s->sc, s->wk, st));
    }
  } else {
    {
      TimeScope ts(s, 0, st);
      HIPCHK(launch_aprod1(s->s, s->sh, vg, s->x3a, s->u, 0.0, 1.0, s->pmode, s->sc, s->wk, 1, st));
    }
    CHK(aprod2_launches(s, s->u, s->v, S, 0.0, s->pmode, 0, s->sc, 1, st));
  }
  if (s->nsel > 0) {
    TimeScope ts(s, 2, st);
    HIPCHK(launch_cov_gather(s->nsel, s->sel, s->w, s->D, s->sc, s->wk, st));
  }
  {
    TimeScope ts(s, 3, st);
    HIPCHK(launch_update(s->s.n, s->v, vg, s->w, s->y, s->var, S, s->sc, s->wk, st, s->eblock ? s->ering : nullptr,
                         s->eblock ? s->eblock : 1));
    if (s->use_blk || iteration_fused(s)) HIPCHK(att_copy_for_pass(s, vg, st));
  }
  s->enq += 1;
  if (s->nsel > 0 && s->enq % s->dblock == 0) {
    TimeScope ts(s, 4, st);
    HIPCHK(cov_flush(s, st));
  }
  if (s->eblock && s->enq % s->eblock == 0) CHK(export_copy(s, s->enq / s->eblock - 1, s->eblock, st));
  return GSR_OK;
}

static void drop_graph(gsr_system* s) {
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  s->gexec = nullptr;
  s->gsize = 0;
}

// Replays of a captured block of iterations.  The kernels of an iteration are
// identical from one iteration to the next (all per-iteration values live in
// the device scalar struct), so a block captured once is replayed for the
// rest of the solve and for later solves with the same configuration.  The
// graph runs on the handle's own stream, ordered after and before the
// caller's stream by events (the null stream cannot be captured).
static int graph_block(gsr_system* s, int64_t G, hipStream_t st) {
  const uint64_t key = ((uint64_t)s->precond << 0) | ((uint64_t)s->pmode << 1) | ((uint64_t)(s->nsel > 0) << 2) |
                       ((uint64_t)G << 3) | ((uint64_t)s->att_atomics << 40) | ((uint64_t)s->waves_per_cu << 41) |
                       ((uint64_t)s->fused << 56) | ((uint64_t)s->use_blk << 57);
  if (!s->gstream) {
    HIPCHK(hipStreamCreateWithFlags(&s->gstream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&s->gev[0], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&s->gev[1], hipEventDisableTiming));
  }
  HIPCHK(hipEventRecord(s->gev[0], st));
  HIPCHK(hipStreamWaitEvent(s->gstream, s->gev[0], 0));
  if (!s->gexec || s->gkey != key) {
    drop_graph(s);
    const int64_t enq0 = s->enq;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s->gstream, hipStreamCaptureModeThreadLocal));
    int rc = GSR_OK;
    for (int64_t i = 0; i < G && rc == GSR_OK; ++i) rc = enqueue_iteration(s, s->gstream);
    hipError_t e = hipStreamEndCapture(s->gstream, &g);
    s->enq = enq0;
    if (rc != GSR_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(GSR_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      s->gexec = nullptr;
      return fail(GSR_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    s->gkey = key;
    s->gsize = G;
  }
  HIPCHK(hipGraphLaunch(s->gexec, s->gstream));
  HIPCHK(hipEventRecord(s->gev[1], s->gstream));
  HIPCHK(hipStreamWaitEvent(st, s->gev[1], 0));
  s->enq += G;
  return GSR_OK;
}

static int lsqr_iterate(gsr_system* s, int64_t nit, hipStream_t st) {
  // blocks of G iterations by graph replay when no per-kernel timing is requested;
  // with covariances a block is the covariance block, aligned to it
  const int64_t G = s->nsel > 0 ? s->dblock : 16;
  if (s->use_graphs && !s->timing && !s->eblock) {
    while (nit >= G && s->itmax - s->enq >= G && (s->nsel == 0 || s->enq % G == 0)) {
      CHK(graph_block(s, G, st));
      nit -= G;
    }
  }
  for (int64_t i = 0; i < nit && s->enq < s->itmax; ++i) CHK(enqueue_iteration(s, st));
  return GSR_OK;
}

extern "C" int gsr_lsqr_iterate(gsr_system* s, int64_t n_iter, gsr_stream stream) {
  CHK(check_handle(s));
  if (!s->in_session) return fail(GSR_ESTATE, "gsr_lsqr_iterate without gsr_lsqr_begin");
  if (n_iter < 0) return fail(GSR_EINVAL, "n_iter < 0");
  return lsqr_iterate(s, n_iter, (hipStream_t)stream);
}

static int read_status(gsr_system* s, gsr_lsqr_result* r, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(s->sc_host, s->sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const Scalars& h = *s->sc_host;
  if (r) {
    r->istop = h.istop;
    r->itn = h.itn;
    r->rnorm = h.rnorm;
    r->arnorm = h.arnorm;
    r->anorm = sqrt(h.anorm2);
    r->acond = h.acond;
    r->xnorm = h.xnorm;
    r->bnorm = h.bnorm;
    r->outer_steps = 0;
    r->inner_total = h.itn;
  }
  return GSR_OK;
}

extern "C" int gsr_lsqr_status(gsr_system* s, gsr_lsqr_result* r, gsr_stream stream) {
  CHK(check_handle(s));
  if (!s->in_session) return fail(GSR_ESTATE, "no solve in progress");
  return read_status(s, r, (hipStream_t)stream);
}

extern "C" int gsr_lsqr_peek(gsr_system* s, double* x, gsr_stream stream) {
  CHK(check_handle(s));
  if (!s->in_session) return fail(GSR_ESTATE, "no solve in progress");
  NEED_DEV(x, "x");
  HIPCHK(launch_finish(s->s.n, s->y, s->var, s->precond ? s->S : nullptr, s->x0, x, nullptr, (hipStream_t)stream));
  return GSR_OK;
}

static int lsqr_end(gsr_system* s, double* x, double* var, gsr_lsqr_result* r, hipStream_t st) {
  if (x) NEED_DEV(x, "x");
  if (var) NEED_DEV(var, "var");
  if (s->nsel > 0) {
    TimeScope ts(s, 4, st);
    HIPCHK(cov_flush(s, st));
  }
  HIPCHK(launch_finish(s->s.n, s->y, s->var, s->precond ? s->S : nullptr, s->x0, x, var, st));
  CHK(read_status(s, r, st));
  if (s->eblock) {
    // blocks of the iterations actually run; the last, possibly partial, one is
    // copied now unless an eager copy (issued once its block was enqueued) covers it
    const int64_t itn = s->sc_host->itn;  // read_status copied the scalars back
    s->eblocks = (itn + s->eblock - 1) / s->eblock;
    s->elast = (int32_t)(itn - (s->eblocks - 1) * s->eblock);
    if (s->eblocks > 0 && !s->ecopied[(size_t)(s->eblocks - 1)]) CHK(export_copy(s, s->eblocks - 1, s->elast, st));
    HIPCHK(hipStreamSynchronize(s->estream));
  }
  s->in_session = 0;
  return GSR_OK;
}

extern "C" int gsr_lsqr_end(gsr_system* s, double* x, double* var, gsr_lsqr_result* r, gsr_stream stream) {
  CHK(check_handle(s));
  if (!s->in_session) return fail(GSR_ESTATE, "no solve in progress");
  return lsqr_end(s, x, var, r, (hipStream_t)stream);
}

static int lsqr_run(gsr_system* s, hipStream_t st) {
  // enqueue in growing chunks; iterations queued after a stop are no-ops
  int64_t chunk = 8;
  for (;;) {
    CHK(lsqr_iterate(s, chunk, st));
    CHK(read_status(s, nullptr, st));
    if (s->sc_host->done || s->enq >= s->itmax) break;
    chunk = std::min<int64_t>(chunk * 2, 64);
  }
  return GSR_OK;
}

extern "C" int gsr_lsqr_solve(gsr_system* s, const double* b, const double* x0, double* x, double* var,
                              const gsr_lsqr_opts* o, gsr_lsqr_result* r, gsr_stream stream) {
  CHK(check_handle(s));
  if (!o) return fail(GSR_EINVAL, "opts is null");
  NEED_DEV(x, "x");
  hipStream_t st = (hipStream_t)stream;
  CHK(lsqr_begin(s, b, x0, o, o->product, st));
  CHK(lsqr_run(s, st));
  return lsqr_end(s, x, var, r, st);
}

extern "C" int gsr_lsqr_refine(gsr_system* s, const double* b, const double* x0, double* x,
                               const gsr_lsqr_opts* o, gsr_lsqr_result* res, gsr_stream stream) {
  CHK(check_handle(s));
  CHK(check_opts(o));
  if (s->s.value_type != GSR_F32) return fail(GSR_EINVAL, "gsr_lsqr_refine needs an FP32 system");
  if (s->con.ncon > 0) return fail(GSR_EINVAL, "gsr_lsqr_refine does not take constraint equations");
  if (o->outer_max < 1 || !(o->outer_tol >= 0)) return fail(GSR_EINVAL, "outer_max >= 1, outer_tol >= 0");
  // each inner solve would damp its correction dx towards zero, not x towards x0:
  // the outer loop would then converge to the undamped solution, not the damped one
  if (o->damp != 0.0) return fail(GSR_EINVAL, "gsr_lsqr_refine solves the undamped problem (damp must be 0)");
  NEED_DEV(x, "x");
  if (s->s.m > 0) NEED_DEV(b, "b");
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)s->s.n;
  if (!s->xr) CHK(dalloc(&s->xr, n));
  if (!s->xn) CHK(dalloc(&s->xn, n));
  if (!s->nrm2) CHK(dalloc(&s->nrm2, 2));
  if (x0) {
    NEED_DEV(x0, "x0");
    HIPCHK(launch_copy(x0, s->xr, (int64_t)n, st));
  } else {
    HIPCHK(launch_fill(s->xr, (int64_t)n, 0.0, st));
  }
  const int64_t keep_sel = s->nsel;
  const int32_t keep_eblock = s->eblock;
  s->nsel = 0;  // covariances are neither accumulated nor exported across refinement steps
  s->eblock = 0;
  int64_t total = 0;
  int32_t steps = 0;
  double prev = 0.0;  // ||dx|| of the previous outer step
  gsr_lsqr_result last{};
  int rc = GSR_OK;
  for (int32_t it = 0; it < o->outer_max; ++it) {
    // LSQR from the current x on r = b - A x, formed with FP64 products on the
    // stored FP32 coefficients (exact upcast); the solve returns x + dx
    const double* xc = (it > 0 || x0) ? s->xr : nullptr;
    if ((rc = lsqr_begin(s, b, xc, o, o->product, st, 1))) break;
    if ((rc = lsqr_run(s, st))) break;
    if ((rc = lsqr_end(s, s->xn, nullptr, &last, st))) break;
    total += last.itn;
    steps = it + 1;
    if (launch_step_norms((int64_t)n, s->xn, s->xr, s->nrm2, s->wk, st) != hipSuccess) {
      rc = fail(GSR_EHIP, "update launch failed");
      break;
    }
    double h2[2];
    if (hipMemcpyAsync(h2, s->nrm2, sizeof h2, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(GSR_EHIP, "reading norms failed");
      break;
    }
    // stop on a small correction, or when the next one, predicted from the
    // contraction between the last two, is small
    const double d = sqrt(h2[0]), lim = o->outer_tol * sqrt(h2[1]);
    if (d <= lim || (it > 0 && d < prev && d * (d / prev) <= lim)) break;
    prev = d;
  }
  s->nsel = keep_sel;
  s->eblock = keep_eblock;
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(x, s->xr, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  if (res) {
    *res = last;
    res->outer_steps = steps;
    res->inner_total = total;
  }
  return GSR_OK;
}

// ------------------------------------------------------------------ covariances
extern "C" int64_t gsr_cov_bytes(int32_t version, int64_t itn_cov_cp, int64_t count) {
  if ((version != 1 && version != 2) || itn_cov_cp < 0 || count < 0) return -1;
  return 8 * itn_cov_cp * count;  // Eq. (5) with count = N_unk, Eq. (6) with count = N_cov,indexes
}

static void cov_clear(gsr_system* s) {
  for (void* p : {(void*)s->sel, (void*)s->D, (void*)s->Cacc, (void*)s->pa, (void*)s->pb, (void*)s->Cp}) dfree(p);
  s->sel = nullptr;
  s->D = nullptr;
  s->Cacc = nullptr;
  s->pa = s->pb = nullptr;
  s->Cp = nullptr;
  s->nsel = 0;
  s->npairs = 0;
}

// Distinct unknowns of a pair list (sorted) and each pair's two positions in them.
static int pair_index(const int64_t* pairs, int64_t P, int64_t n, std::vector<int64_t>* U, std::vector<int32_t>* a,
                      std::vector<int32_t>* b) {
  U->assign(pairs, pairs + 2 * P);
  for (int64_t v : *U)
    if (v < 0 || v >= n) return fail(GSR_EINVAL, "pair index %lld out of range", (long long)v);
  std::sort(U->begin(), U->end());
  U->erase(std::unique(U->begin(), U->end()), U->end());
  if (U->size() >= ((size_t)1 << 31)) return fail(GSR_EINVAL, "too many distinct pair indexes");
  a->resize((size_t)P);
  b->resize((size_t)P);
  for (int64_t p = 0; p < P; ++p) {
    (*a)[(size_t)p] = (int32_t)(std::lower_bound(U->begin(), U->end(), pairs[2 * p]) - U->begin());
    (*b)[(size_t)p] = (int32_t)(std::lower_bound(U->begin(), U->end(), pairs[2 * p + 1]) - U->begin());
  }
  return GSR_OK;
}

extern "C" int gsr_set_constraints(gsr_system* s, int64_t ncon, const int64_t* ptr, const int64_t* col,
                                   const double* val, const double* rhs) {
  CHK(check_handle(s));
  if (s->in_session) return fail(GSR_ESTATE, "gsr_set_constraints: a solve is in progress");
  if (ncon < 0) return fail(GSR_EINVAL, "ncon < 0");
  if (ncon > 0 && (!ptr || !rhs)) return fail(GSR_EINVAL, "ptr and rhs are needed");
  if (ncon > 0 && (is_device_ptr(ptr) || is_device_ptr(rhs) || (col && is_device_ptr(col)) ||
                   (val && is_device_ptr(val))))
    return fail(GSR_EINVAL, "constraint arrays are host memory");
  const int64_t nnz = ncon > 0 ? ptr[ncon] : 0;
  if (ncon > 0) {
    if (ptr[0] != 0) return fail(GSR_EINVAL, "ptr[0] must be 0");
    if (nnz > 0 && (!col || !val)) return fail(GSR_EINVAL, "col and val are needed");
    for (int64_t i = 0; i < ncon; ++i) {
      if (ptr[i + 1] < ptr[i]) return fail(GSR_EINVAL, "ptr decreases at row %lld", (long long)i);
      for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
        if (col[e] < 0 || col[e] >= s->s.n) return fail(GSR_EINVAL, "col[%lld] out of range", (long long)e);
        if (e > ptr[i] && col[e] <= col[e - 1])
          return fail(GSR_EINVAL, "the columns of constraint row %lld must be strictly increasing", (long long)i);
      }
    }
  }
  (void)hipDeviceSynchronize();
  drop_graph(s);
  con_free(s);
  dfree(s->u);  // its length is m + ncon
  s->u = nullptr;
  s->S_valid = 0;  // the column norms are those of [A; C]
  if (ncon == 0) return GSR_OK;
  // tiles of at most kConTile entries of one row
  std::vector<int64_t> te, tr;
  for (int64_t i = 0; i < ncon; ++i)
    for (int64_t e = ptr[i]; e < ptr[i + 1]; e += kConTile) {
      te.push_back(e);
      tr.push_back(i);
    }
  const int64_t nt = (int64_t)tr.size();
  te.push_back(nnz);
  int64_t *dp = nullptr, *dc = nullptr, *dte = nullptr, *dtr = nullptr;
  double *dv = nullptr, *dtmp = nullptr, *drhs = nullptr;
  int rc = GSR_OK;
  if ((rc = dalloc(&dp, (size_t)ncon + 1)) || (rc = dalloc(&dc, (size_t)std::max<int64_t>(nnz, 1))) ||
      (rc = dalloc(&dv, (size_t)std::max<int64_t>(nnz, 1))) || (rc = dalloc(&dte, (size_t)nt + 1)) ||
      (rc = dalloc(&dtr, (size_t)std::max<int64_t>(nt, 1))) || (rc = dalloc(&dtmp, (size_t)ncon)) ||
      (rc = dalloc(&drhs, (size_t)ncon))) {
    for (void* p : {(void*)dp, (void*)dc, (void*)dv, (void*)dte, (void*)dtr, (void*)dtmp, (void*)drhs}) dfree(p);
    return rc;
  }
  s->con.ncon = ncon;
  s->con.ptr = dp;
  s->con.col = dc;
  s->con.val = dv;
  s->con.ntiles = nt;
  s->con.tile_e = dte;
  s->con.tile_r = dtr;
  s->con.tmp = dtmp;
  s->con_rhs = drhs;
  HIPCHK(hipMemcpy(dp, ptr, sizeof(int64_t) * ((size_t)ncon + 1), hipMemcpyHostToDevice));
  if (nnz > 0) {
    HIPCHK(hipMemcpy(dc, col, sizeof(int64_t) * (size_t)nnz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dv, val, sizeof(double) * (size_t)nnz, hipMemcpyHostToDevice));
  }
  HIPCHK(hipMemcpy(dte, te.data(), sizeof(int64_t) * te.size(), hipMemcpyHostToDevice));
  if (nt > 0) HIPCHK(hipMemcpy(dtr, tr.data(), sizeof(int64_t) * (size_t)nt, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(drhs, rhs, sizeof(double) * (size_t)ncon, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(dtmp, 0, sizeof(double) * (size_t)ncon));
  return GSR_OK;
}

extern "C" int gsr_cov_request(gsr_system* s, const int64_t* sel, int64_t k, int32_t block) {
  CHK(check_handle(s));
  if (k < 0) return fail(GSR_EINVAL, "k < 0");
  if (k > 0 && !sel) return fail(GSR_EINVAL, "sel is null");
  if (block < 1 || block > 1024) return fail(GSR_EINVAL, "block must be in [1, 1024]");
  for (int64_t p = 0; p < k; ++p)
    if (sel[p] < 0 || sel[p] >= s->s.n) return fail(GSR_EINVAL, "sel[%lld] = %lld out of range", (long long)p,
                                                     (long long)sel[p]);
  if (s->in_session) return fail(GSR_ESTATE, "gsr_cov_request: a solve is in progress");
  (void)hipDeviceSynchronize();
  drop_graph(s);
  cov_clear(s);
  if (k == 0) return GSR_OK;
  CHK(dalloc(&s->sel, (size_t)k));
  CHK(dalloc(&s->D, (size_t)k * block));
  CHK(dalloc(&s->Cacc, (size_t)k * k));
  HIPCHK(hipMemcpy(s->sel, sel, (size_t)k * sizeof(int64_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemset(s->Cacc, 0, (size_t)k * k * sizeof(double)));
  s->nsel = k;
  s->dblock = block;
  return GSR_OK;
}

extern "C" int gsr_cov_request_pairs(gsr_system* s, const int64_t* pairs, int64_t P, int32_t block) {
  CHK(check_handle(s));
  if (s->in_session) return fail(GSR_ESTATE, "gsr_cov_request_pairs: a solve is in progress");
  if (P < 0) return fail(GSR_EINVAL, "P < 0");
  if (P > 0 && !pairs) return fail(GSR_EINVAL, "pairs is null");
  if (block < 1 || block > 1024) return fail(GSR_EINVAL, "block must be in [1, 1024]");
  std::vector<int64_t> U;
  std::vector<int32_t> a, b;
  if (P > 0) CHK(pair_index(pairs, P, s->s.n, &U, &a, &b));
  (void)hipDeviceSynchronize();
  drop_graph(s);
  cov_clear(s);
  if (P == 0) return GSR_OK;
  const int64_t k = (int64_t)U.size();
  CHK(dalloc(&s->sel, (size_t)k));
  CHK(dalloc(&s->D, (size_t)k * block));
  CHK(dalloc(&s->pa, (size_t)P));
  CHK(dalloc(&s->pb, (size_t)P));
  CHK(dalloc(&s->Cp, (size_t)P));
  HIPCHK(hipMemcpy(s->sel, U.data(), (size_t)k * sizeof(int64_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->pa, a.data(), (size_t)P * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->pb, b.data(), (size_t)P * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemset(s->Cp, 0, (size_t)P * sizeof(double)));
  s->nsel = k;
  s->npairs = P;
  s->dblock = block;
  return GSR_OK;
}

extern "C" int gsr_cov_get_pairs(gsr_system* s, double* out, gsr_stream stream) {
  CHK(check_handle(s));
  if (s->npairs == 0) return fail(GSR_ESTATE, "no pair list");
  NEED_DEV(out, "out");
  HIPCHK(launch_pair_out(s->Cp, s->npairs, s->pa, s->pb, s->cov_precond ? s->S : nullptr, s->sel, out,
                         (hipStream_t)stream));
  return GSR_OK;
}

extern "C" int gsr_cov_get(gsr_system* s, double* C, gsr_stream stream) {
  CHK(check_handle(s));
  if (s->npairs > 0) return fail(GSR_ESTATE, "the covariance request is a pair list: use gsr_cov_get_pairs");
  if (s->nsel == 0) return fail(GSR_ESTATE, "no covariance selection");
  NEED_DEV(C, "C");
  HIPCHK(launch_cov_out(s->Cacc, s->nsel, s->cov_precond ? s->S : nullptr, s->sel, C, (hipStream_t)stream));
  return GSR_OK;
}

extern "C" int gsr_cov_export(gsr_system* s, double* host, int64_t max_blocks, int32_t block) {
  CHK(check_handle(s));
  if (s->in_session) return fail(GSR_ESTATE, "gsr_cov_export: a solve is in progress");
  if (block < 0 || block > 1024) return fail(GSR_EINVAL, "block must be in [0, 1024]");
  if (block > 0 && (!host || max_blocks < 1)) return fail(GSR_EINVAL, "need a host buffer and max_blocks >= 1");
  if (block > 0 && is_device_ptr(host)) return fail(GSR_EINVAL, "the export buffer must be host memory");
  if (s->ering && block != s->eblock) {
    dfree(s->ering);
    s->ering = nullptr;
  }
  s->eblock = 0;
  s->ehost = nullptr;
  s->emax = 0;
  s->eblocks = 0;
  s->elast = 0;
  if (block == 0) return GSR_OK;
  if (!s->ering) CHK(dalloc(&s->ering, 2 * (size_t)block * (size_t)std::max<int64_t>(s->s.n, 1)));
  if (!s->estream) {
    HIPCHK(hipStreamCreateWithFlags(&s->estream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&s->eev[0], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&s->eev[1], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&s->efill, hipEventDisableTiming));
  }
  s->eblock = block;
  s->ehost = host;
  s->emax = max_blocks;
  drop_graph(s);
  return GSR_OK;
}

extern "C" int gsr_cov_export_status(gsr_system* s, int64_t* blocks, int32_t* last_cols) {
  CHK(check_handle(s));
  if (!blocks || !last_cols) return fail(GSR_EINVAL, "null output");
  *blocks = s->eblocks;
  *last_cols = s->elast;
  return GSR_OK;
}

// Post-hoc covariance accumulation over exported blocks: for each block, the
// rows sel of its vectors are gathered on the host into a pinned [k][block]
// stage, copied, and reduced into Cacc (dense, SYRK) or Cp (pair list).
static int export_accumulate(const double* blocks, int64_t n, int32_t block, int64_t nblocks, int32_t last_cols,
                             const int64_t* sel, int64_t k, double* Cacc, const int32_t* pa, const int32_t* pb,
                             int64_t P, double* Cp, hipStream_t st) {
  double *Dd = nullptr, *stage = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  auto done = [&](int code) {
    (void)hipStreamSynchronize(st);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    dfree(Dd);
    if (stage) (void)hipHostFree(stage);
    return code;
  };
  const size_t kb = (size_t)k * (size_t)block;
  int rc = dalloc(&Dd, 2 * kb);
  if (rc) return done(rc);
  if (hipHostMalloc((void**)&stage, sizeof(double) * 2 * kb, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return done(fail(GSR_ENOMEM, "pinned staging allocation failed"));
  }
  if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess)
    return done(fail(GSR_EHIP, "event creation failed"));
  Work none{};
  for (int64_t b = 0; b < nblocks; ++b) {
    const int h = (int)(b & 1);
    const int64_t cols = (b == nblocks - 1) ? last_cols : block;
    if (b >= 2 && hipEventSynchronize(ev[h]) != hipSuccess) return done(fail(GSR_EHIP, "staging wait failed"));
    // stage[p][c] = d_{b*block+c}[sel[p]]
    double* sg = stage + (size_t)h * kb;
    const double* blk = blocks + (size_t)b * (size_t)block * (size_t)n;
    for (int64_t c = 0; c < cols; ++c) {
      const double* dv = blk + (size_t)c * (size_t)n;
      for (int64_t p = 0; p < k; ++p) sg[(size_t)p * block + c] = dv[sel[p]];
    }
    double* dd = Dd + (size_t)h * kb;
    hipError_t e = hipMemcpyAsync(dd, sg, sizeof(double) * kb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(ev[h], st);
    if (e == hipSuccess)
      e = P > 0 ? launch_pairdot(dd, block, pa, pb, P, Cp, nullptr, none, cols, st)
                : launch_syrk(dd, k, block, Cacc, nullptr, none, cols, st);
    if (e != hipSuccess) return done(fail(GSR_EHIP, "block %lld: %s", (long long)b, hipGetErrorString(e)));
  }
  return done(GSR_OK);
}

static int check_export_args(const double* blocks, int64_t n, int32_t block, int64_t nblocks, int32_t last_cols) {
  if (n < 1 || block < 1 || block > 1024 || nblocks < 0) return fail(GSR_EINVAL, "bad sizes");
  if (nblocks > 0 && (last_cols < 1 || last_cols > block)) return fail(GSR_EINVAL, "last_cols must be in [1, block]");
  if (nblocks > 0 && !blocks) return fail(GSR_EINVAL, "blocks is null");
  if (is_device_ptr(blocks)) return fail(GSR_EINVAL, "blocks must be host memory");
  return GSR_OK;
}

extern "C" int gsr_cov_from_export(const double* blocks, int64_t n, int32_t block, int64_t nblocks, int32_t last_cols,
                                   const int64_t* sel, int64_t k, const double* S, double* C, gsr_stream stream) {
  CHK(check_export_args(blocks, n, block, nblocks, last_cols));
  if (k < 0) return fail(GSR_EINVAL, "k < 0");
  if (k == 0) return GSR_OK;
  if (!sel || is_device_ptr(sel)) return fail(GSR_EINVAL, "sel must be host memory");
  NEED_DEV(C, "C");
  if (S) NEED_DEV(S, "S");
  for (int64_t p = 0; p < k; ++p)
    if (sel[p] < 0 || sel[p] >= n) return fail(GSR_EINVAL, "sel[%lld] out of range", (long long)p);
  hipStream_t st = (hipStream_t)stream;
  double* Cacc = nullptr;
  int64_t* seld = nullptr;
  int rc = GSR_OK;
  if (!(rc = dalloc(&Cacc, (size_t)k * (size_t)k)) && !(rc = dalloc(&seld, (size_t)k))) {
    if (hipMemcpyAsync(seld, sel, sizeof(int64_t) * (size_t)k, hipMemcpyHostToDevice, st) != hipSuccess ||
        launch_fill(Cacc, k * k, 0.0, st) != hipSuccess)
      rc = fail(GSR_EHIP, "cov_from_export set-up failed");
    if (!rc) rc = export_accumulate(blocks, n, block, nblocks, last_cols, sel, k, Cacc, nullptr, nullptr, 0, nullptr, st);
    if (!rc && (launch_cov_out(Cacc, k, S, seld, C, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess))
      rc = fail(GSR_EHIP, "cov_from_export output failed");
  }
  (void)hipStreamSynchronize(st);
  dfree(Cacc);
  dfree(seld);
  return rc;
}

extern "C" int gsr_cov_pairs_from_export(const double* blocks, int64_t n, int32_t block, int64_t nblocks,
                                         int32_t last_cols, const int64_t* pairs, int64_t P, const double* S,
                                         double* out, gsr_stream stream) {
  CHK(check_export_args(blocks, n, block, nblocks, last_cols));
  if (P < 0) return fail(GSR_EINVAL, "P < 0");
  if (P == 0) return GSR_OK;
  if (!pairs || is_device_ptr(pairs)) return fail(GSR_EINVAL, "pairs must be host memory");
  NEED_DEV(out, "out");
  if (S) NEED_DEV(S, "S");
  std::vector<int64_t> U;
  std::vector<int32_t> a, b;
  CHK(pair_index(pairs, P, n, &U, &a, &b));
  const int64_t k = (int64_t)U.size();
  hipStream_t st = (hipStream_t)stream;
  double* Cp = nullptr;
  int32_t *pa = nullptr, *pb = nullptr;
  int64_t* seld = nullptr;
  int rc = GSR_OK;
  if (!(rc = dalloc(&Cp, (size_t)P)) && !(rc = dalloc(&pa, (size_t)P)) && !(rc = dalloc(&pb, (size_t)P)) &&
      !(rc = dalloc(&seld, (size_t)k))) {
    if (hipMemcpyAsync(seld, U.data(), sizeof(int64_t) * (size_t)k, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(pa, a.data(), sizeof(int32_t) * (size_t)P, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(pb, b.data(), sizeof(int32_t) * (size_t)P, hipMemcpyHostToDevice, st) != hipSuccess ||
        launch_fill(Cp, P, 0.0, st) != hipSuccess)
      rc = fail(GSR_EHIP, "cov_pairs_from_export set-up failed");
    if (!rc) rc = export_accumulate(blocks, n, block, nblocks, last_cols, U.data(), k, nullptr, pa, pb, P, Cp, st);
    if (!rc && (launch_pair_out(Cp, P, pa, pb, S, seld, out, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess))
      rc = fail(GSR_EHIP, "cov_pairs_from_export output failed");
  }
  (void)hipStreamSynchronize(st);
  for (void* p : {(void*)Cp, (void*)pa, (void*)pb, (void*)seld}) dfree(p);
  return rc;
}

extern "C" int gsr_syrk(const double* D, int64_t k, int64_t cols, int64_t ldd, double* C, gsr_stream stream) {
  if (k < 0 || cols < 0 || ldd < cols) return fail(GSR_EINVAL, "need k >= 0, 0 <= cols <= ldd");
  if (k == 0 || cols == 0) return GSR_OK;
  NEED_DEV(D, "D");
  NEED_DEV(C, "C");
  Work none{};
  HIPCHK(launch_syrk(D, k, ldd, C, nullptr, none, cols, (hipStream_t)stream));
  return GSR_OK;
}

// ------------------------------------------------------------------ learned warm start

extern "C" int gsr_features(gsr_system* s, const double* b, const double* x_other, double* F, gsr_stream stream) {
  CHK(check_handle(s));
  if (s->packed) return fail(GSR_EINVAL, "gsr_features reads the rows in star order: use a handle from gsr_create");
  if (s->s.m > 0) NEED_DEV(b, "b");
  NEED_DEV(x_other, "x_other");
  if (s->s.n_stars > 0) NEED_DEV(F, "F");
  HIPCHK(launch_features(s->s, b, x_other, F, (hipStream_t)stream));
  return GSR_OK;
}

extern "C" int gsr_mean_rows(const double* X, int64_t k, int64_t len, double* out, gsr_stream stream) {
  if (k < 1 || len < 0) return fail(GSR_EINVAL, "need k >= 1, len >= 0");
  if (len == 0) return GSR_OK;
  NEED_DEV(X, "X");
  NEED_DEV(out, "out");
  HIPCHK(launch_mean_rows(X, k, len, out, (hipStream_t)stream));
  return GSR_OK;
}

struct gsr_mlp {
  int I = 0, H = 0, O = 0;
  int64_t P = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  double *mu_x = nullptr, *sd_x = nullptr, *mu_t = nullptr, *sd_t = nullptr;
  int norm_set = 0;
  int64_t t = 0;
  int64_t cap = 0;
  float *Xs = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Y = nullptr, *Ts = nullptr;
  float *dY = nullptr, *dZ2 = nullptr, *dZ1 = nullptr;
  double* loss = nullptr;
  double* loss_host = nullptr;
  // parameter views
  float *W1() { return p; }
  float *b1() { return p + (int64_t)H * I; }
  float *W2() { return b1() + H; }
  float *b2() { return W2() + (int64_t)H * H; }
  float *W3() { return b2() + H; }
  float *b3() { return W3() + (int64_t)O * H; }
};

static std::set<gsr_mlp*> g_live_mlp;

static int check_mlp(gsr_mlp* n) {
  if (!n) return fail(GSR_EINVAL, "null network");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_live_mlp.count(n)) return fail(GSR_EINVAL, "unknown or destroyed network");
  return GSR_OK;
}

static void mlp_release(gsr_mlp* n) {
  (void)hipDeviceSynchronize();
  for (void* q : {(void*)n->p, (void*)n->g, (void*)n->m, (void*)n->v, (void*)n->mu_x, (void*)n->sd_x,
                  (void*)n->mu_t, (void*)n->sd_t, (void*)n->Xs, (void*)n->Z1, (void*)n->H1, (void*)n->Z2,
                  (void*)n->H2, (void*)n->Y, (void*)n->Ts, (void*)n->dY, (void*)n->dZ2, (void*)n->dZ1,
                  (void*)n->loss})
    dfree(q);
  if (n->loss_host) (void)hipHostFree(n->loss_host);
  delete n;
}

extern "C" int gsr_mlp_create(gsr_mlp** out, int32_t n_in, int32_t n_hidden, int32_t n_out, const double* params) {
  if (!out) return fail(GSR_EINVAL, "out is null");
  *out = nullptr;
  if (n_in < 1 || n_hidden < 1 || n_out < 1 || n_in > 4096 || n_hidden > 4096 || n_out > 4096)
    return fail(GSR_EINVAL, "layer sizes must be in [1, 4096]");
  if (!params) return fail(GSR_EINVAL, "params is null");
  gsr_mlp* n = new gsr_mlp();
  n->I = n_in;
  n->H = n_hidden;
  n->O = n_out;
  n->P = (int64_t)n_hidden * n_in + n_hidden + (int64_t)n_hidden * n_hidden + n_hidden + (int64_t)n_out * n_hidden +
         n_out;
  int rc;
  if ((rc = dalloc(&n->p, n->P)) || (rc = dalloc(&n->g, n->P)) || (rc = dalloc(&n->m, n->P)) ||
      (rc = dalloc(&n->v, n->P)) || (rc = dalloc(&n->mu_x, n_in)) || (rc = dalloc(&n->sd_x, n_in)) ||
      (rc = dalloc(&n->mu_t, n_out)) || (rc = dalloc(&n->sd_t, n_out)) || (rc = dalloc(&n->loss, 1))) {
    mlp_release(n);
    return rc;
  }
  if (hipHostMalloc((void**)&n->loss_host, sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    mlp_release(n);
    return fail(GSR_ENOMEM, "pinned host allocation failed");
  }
  std::vector<float> h((size_t)n->P);
  for (int64_t i = 0; i < n->P; ++i) h[i] = (float)params[i];
  std::vector<double> ones(std::max(n_in, n_out), 1.0), zeros(std::max(n_in, n_out), 0.0);
  if (hipMemcpy(n->p, h.data(), n->P * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(n->m, 0, n->P * sizeof(float)) != hipSuccess || hipMemset(n->v, 0, n->P * sizeof(float)) != hipSuccess ||
      hipMemcpy(n->mu_x, zeros.data(), n_in * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(n->sd_x, ones.data(), n_in * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(n->mu_t, zeros.data(), n_out * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(n->sd_t, ones.data(), n_out * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    mlp_release(n);
    return fail(GSR_EHIP, "network upload failed");
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_live_mlp.insert(n);
  }
  *out = n;
  return GSR_OK;
}

extern "C" int gsr_mlp_destroy(gsr_mlp* n) {
  if (!n) return GSR_OK;
  CHK(check_mlp(n));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_live_mlp.erase(n);
  }
  mlp_release(n);
  return GSR_OK;
}

extern "C" int gsr_mlp_get_params(gsr_mlp* n, double* params) {
  CHK(check_mlp(n));
  if (!params) return fail(GSR_EINVAL, "params is null");
  std::vector<float> h((size_t)n->P);
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(h.data(), n->p, n->P * sizeof(float), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n->P; ++i) params[i] = h[i];
  return GSR_OK;
}

extern "C" int gsr_mlp_fit_norm(gsr_mlp* n, const double* X, const double* T, int64_t N, gsr_stream stream) {
  CHK(check_mlp(n));
  if (N < 1) return fail(GSR_EINVAL, "N < 1");
  NEED_DEV(X, "X");
  NEED_DEV(T, "T");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(mlp_col_stats(X, N, n->I, n->mu_x, n->sd_x, st));
  HIPCHK(mlp_col_stats(T, N, n->O, n->mu_t, n->sd_t, st));
  n->norm_set = 1;
  return GSR_OK;
}

static int mlp_reserve(gsr_mlp* n, int64_t N) {
  if (N <= n->cap) return GSR_OK;
  HIPCHK(hipDeviceSynchronize());
  for (float** q : {&n->Xs, &n->Z1, &n->H1, &n->Z2, &n->H2, &n->Y, &n->Ts, &n->dY, &n->dZ2, &n->dZ1}) {
    dfree(*q);
    *q = nullptr;
  }
  n->cap = 0;
  const size_t I = n->I, H = n->H, O = n->O;
  CHK(dalloc(&n->Xs, N * I));
  CHK(dalloc(&n->Z1, N * H));
  CHK(dalloc(&n->H1, N * H));
  CHK(dalloc(&n->Z2, N * H));
  CHK(dalloc(&n->H2, N * H));
  CHK(dalloc(&n->Y, N * O));
  CHK(dalloc(&n->Ts, N * O));
  CHK(dalloc(&n->dY, N * O));
  CHK(dalloc(&n->dZ2, N * H));
  CHK(dalloc(&n->dZ1, N * H));
  n->cap = N;
  return GSR_OK;
}

// forward on standardized inputs n->Xs (N rows); output n->Y (standardized)
static int mlp_fwd(gsr_mlp* n, int64_t N, hipStream_t st) {
  const int I = n->I, H = n->H, O = n->O;
  GemmArgs g1{(int)N, H, I, n->Xs, I, 1, n->W1(), 1, I, n->H1, H, n->b1(), 1, n->Z1, nullptr};
  HIPCHK(mlp_gemm(g1, 1, st));
  GemmArgs g2{(int)N, H, H, n->H1, H, 1, n->W2(), 1, H, n->H2, H, n->b2(), 1, n->Z2, nullptr};
  HIPCHK(mlp_gemm(g2, 1, st));
  GemmArgs g3{(int)N, O, H, n->H2, H, 1, n->W3(), 1, H, n->Y, O, n->b3(), 0, nullptr, nullptr};
  HIPCHK(mlp_gemm(g3, 1, st));
  return GSR_OK;
}

// gradients of the mean squared error into n->g (loss accumulated into n->loss)
static int mlp_bwd(gsr_mlp* n, int64_t N, hipStream_t st) {
  const int I = n->I, H = n->H, O = n->O;
  const int splits = (int)std::max<int64_t>(1, std::min<int64_t>(64, N / 256));
  float* gW1 = n->g;
  float* gb1 = gW1 + (int64_t)H * I;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (int64_t)H * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + (int64_t)O * H;
  HIPCHK(mlp_mse(n->Y, n->Ts, N * O, n->dY, n->loss, st));
  GemmArgs w3{O, H, (int)N, n->dY, 1, O, n->H2, H, 1, gW3, H, nullptr, 0, nullptr, nullptr};
  HIPCHK(mlp_gemm(w3, splits, st));
  HIPCHK(mlp_colsum(n->dY, N, O, gb3, st));
  GemmArgs h2{(int)N, H, O, n->dY, O, 1, n->W3(), H, 1, n->dZ2, H, nullptr, 0, nullptr, n->Z2};
  HIPCHK(mlp_gemm(h2, 1, st));
  GemmArgs w2{H, H, (int)N, n->dZ2, 1, H, n->H1, H, 1, gW2, H, nullptr, 0, nullptr, nullptr};
  HIPCHK(mlp_gemm(w2, splits, st));
  HIPCHK(mlp_colsum(n->dZ2, N, H, gb2, st));
  GemmArgs h1{(int)N, H, H, n->dZ2, H, 1, n->W2(), H, 1, n->dZ1, H, nullptr, 0, nullptr, n->Z1};
  HIPCHK(mlp_gemm(h1, 1, st));
  GemmArgs w1{H, I, (int)N, n->dZ1, 1, H, n->Xs, I, 1, gW1, I, nullptr, 0, nullptr, nullptr};
  HIPCHK(mlp_gemm(w1, splits, st));
  HIPCHK(mlp_colsum(n->dZ1, N, H, gb1, st));
  return GSR_OK;
}

static int mlp_load(gsr_mlp* n, const double* X, const double* T, int64_t N, hipStream_t st) {
  CHK(mlp_reserve(n, N));
  HIPCHK(mlp_standardize(X, N, n->I, n->mu_x, n->sd_x, n->Xs, st));
  if (T) HIPCHK(mlp_standardize(T, N, n->O, n->mu_t, n->sd_t, n->Ts, st));
  return GSR_OK;
}

extern "C" int gsr_mlp_forward(gsr_mlp* n, const double* X, int64_t N, double* Y, gsr_stream stream) {
  CHK(check_mlp(n));
  if (N < 0) return fail(GSR_EINVAL, "N < 0");
  if (N == 0) return GSR_OK;
  NEED_DEV(X, "X");
  NEED_DEV(Y, "Y");
  hipStream_t st = (hipStream_t)stream;
  CHK(mlp_load(n, X, nullptr, N, st));
  CHK(mlp_fwd(n, N, st));
  HIPCHK(mlp_destandardize(n->Y, N, n->O, n->mu_t, n->sd_t, Y, st));
  return GSR_OK;
}

extern "C" int gsr_mlp_grad(gsr_mlp* n, const double* X, const double* T, int64_t N, double* loss_host,
                            float* grads, gsr_stream stream) {
  CHK(check_mlp(n));
  if (N < 1) return fail(GSR_EINVAL, "N < 1");
  NEED_DEV(X, "X");
  NEED_DEV(T, "T");
  hipStream_t st = (hipStream_t)stream;
  CHK(mlp_load(n, X, T, N, st));
  HIPCHK(hipMemsetAsync(n->loss, 0, sizeof(double), st));
  CHK(mlp_fwd(n, N, st));
  CHK(mlp_bwd(n, N, st));
  if (grads) {
    NEED_DEV(grads, "grads");
    HIPCHK(hipMemcpyAsync(grads, n->g, n->P * sizeof(float), hipMemcpyDeviceToDevice, st));
  }
  HIPCHK(hipMemcpyAsync(n->loss_host, n->loss, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (loss_host) *loss_host = *n->loss_host;
  return GSR_OK;
}

extern "C" int gsr_mlp_train(gsr_mlp* n, const double* X, const double* T, int64_t N, int32_t steps, double lr,
                             double* loss_host, gsr_stream stream) {
  CHK(check_mlp(n));
  if (N < 1 || steps < 0 || !(lr > 0)) return fail(GSR_EINVAL, "need N >= 1, steps >= 0, lr > 0");
  NEED_DEV(X, "X");
  NEED_DEV(T, "T");
  hipStream_t st = (hipStream_t)stream;
  CHK(mlp_load(n, X, T, N, st));
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int32_t i = 0; i < steps; ++i) {
    CHK(mlp_fwd(n, N, st));
    HIPCHK(hipMemsetAsync(n->loss, 0, sizeof(double), st));
    CHK(mlp_bwd(n, N, st));
    n->t += 1;
    const float c1 = (float)(1.0 - pow(0.9, (double)n->t)), c2 = (float)(1.0 - pow(0.999, (double)n->t));
    HIPCHK(mlp_adam(n->p, n->g, n->m, n->v, n->P, (float)lr, b1, b2, eps, c1, c2, st));
  }
  // loss of the final parameters
  HIPCHK(hipMemsetAsync(n->loss, 0, sizeof(double), st));
  CHK(mlp_fwd(n, N, st));
  HIPCHK(mlp_mse(n->Y, n->Ts, N * n->O, n->dY, n->loss, st));
  HIPCHK(hipMemcpyAsync(n->loss_host, n->loss, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (loss_host) *loss_host = *n->loss_host;
  return GSR_OK;
}

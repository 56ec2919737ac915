// runtime.hip -- host side of the C ABI declared in include/lbm.h.
//
// Owns contexts (one lattice each), their device memory, the host step
// loop, the FP64 monitors and batches.  Every entry point validates its
// arguments, returns an lbm_status and records a message; no exception
// crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "kernels.hpp"
#include "lattice.hpp"
#include "probes.hpp"

using namespace lbm;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int bytes_of(int storage) { return storage == LBM_F64 ? 8 : storage == LBM_F32 ? 4 : 2; }

// Monitor scratch: velocity snapshot (3 N values of the compute type),
// per-block partial sums and the 3 final sums.
size_t monitor_bytes(size_t N, int storage) {
  const size_t snap = 3 * N * (storage == LBM_F64 ? 8 : 4);
  return align_up(snap) + align_up(3 * sizeof(double) * 2048) + align_up(4 * sizeof(double));
}

// Elements between consecutive population arrays: N rounded up to 64 (a
// wavefront's worth) plus LBM_STRIDE_PAD elements.  Without the pad, the q
// arrays of a power-of-two lattice start at power-of-two offsets and the q
// streams of one wavefront hit the same memory channels; 1088 elements
// (4352 B in FP32) shift each array by a little over one 4 KB interleave
// step (measured +4 % on 128^3 D3Q18 FP32 AA; neutral at 256^3).
#ifndef LBM_STRIDE_PAD
#define LBM_STRIDE_PAD 1088
#endif
size_t pop_stride(size_t N) { return (N + 63) / 64 * 64 + LBM_STRIDE_PAD; }

size_t population_bytes(int q, size_t N, int storage) {
  return (size_t)q * pop_stride(N) * (size_t)bytes_of(storage);
}

// Monitor runs whose results a context can hold unread (a ring).
constexpr int kMonSlots = 8;

bool is_nee_face(int kind) {
  return kind == LBM_VELOCITY || kind == LBM_PRESSURE || kind == LBM_SYMMETRY_NODE;
}

// Number of nodes on velocity / pressure faces: all nodes minus the box of
// nodes on none of them.
long long nee_node_count(int nx, int ny, int nz, const lbm_spec* sp) {
  const int dim[3] = {nx, ny, nz};
  long long inner = 1;
  bool any = false;
  for (int d = 0; d < 3; ++d) {
    const int lo = is_nee_face(sp->face[2 * d]), hi = is_nee_face(sp->face[2 * d + 1]);
    any = any || lo || hi;
    inner *= std::max(0, dim[d] - lo - hi);
  }
  return any ? (long long)nx * ny * nz - inner : 0;
}

std::string validate(int model, int nx, int ny, int nz, const double* s, const lbm_spec* sp) {
  if (model != 14 && model != 18 && model != 26) return "model must be 14, 18 or 26";
  if (nx < 1 || ny < 1 || nz < 1) return "lattice dimensions must be >= 1";
  const long long N = (long long)nx * ny * nz;
  if (N >= (1LL << 31)) return "lattice too large (nx*ny*nz must be < 2^31)";
  if (!sp) return "spec is NULL";
  if (sp->storage < LBM_F64 || sp->storage > LBM_F16DEV) return "unknown storage";
  if (sp->pattern != LBM_AB && sp->pattern != LBM_AA) return "unknown pattern";
  if (sp->storage == LBM_F16DEV && (sp->f16_scale_log2 < 0 || sp->f16_scale_log2 > 24))
    return "f16_scale_log2 must be in 0..24";
  if (sp->monitor_every < 0) return "monitor_every must be >= 0";
  if (sp->f16_rounding != LBM_ROUND_STOCHASTIC && sp->f16_rounding != LBM_ROUND_NEAREST)
    return "unknown f16_rounding";
  if (sp->collision != LBM_MRT && sp->collision != LBM_BGK) return "unknown collision";
  if (sp->collision == LBM_BGK && s) {
    for (int k = 1; k < model; ++k)
      if (s[k] != s[0]) return "LBM_BGK needs all relaxation rates equal (S = I/tau)";
  }
  for (int d = 0; d < 3; ++d) {
    const int a = sp->face[2 * d], b = sp->face[2 * d + 1];
    if (a < LBM_PERIODIC || a > LBM_SYMMETRY_NODE || b < LBM_PERIODIC || b > LBM_SYMMETRY_NODE)
      return "face kind must be LBM_PERIODIC, LBM_WALL, LBM_SYMMETRY, LBM_VELOCITY, "
             "LBM_PRESSURE or LBM_SYMMETRY_NODE";
    if ((a == LBM_PERIODIC) != (b == LBM_PERIODIC)) return "periodic faces must come in pairs";
    const int dim[3] = {nx, ny, nz};
    if ((is_nee_face(a) || is_nee_face(b)) && dim[d] < 3)
      return "an axis with a velocity, pressure or node-layer symmetry face needs at least 3 "
             "nodes";
  }
  for (int f = 0; f < 6; ++f)
    if (!std::isfinite(sp->face_p[f]) || !std::isfinite(sp->face_pA[f]))
      return "face pressures must be finite";
  for (int f = 0; f < 6; ++f) {
    const double* u = sp->wall_u[f];
    const double m = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!(m < 0.3)) return "wall speed must be < 0.3 (lattice units)";
  }
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(sp->F0[d]) || !std::isfinite(sp->FA[d])) return "force must be finite";
  if (!std::isfinite(sp->FT)) return "FT must be finite";
  if (!std::isfinite(sp->p0)) return "p0 must be finite";
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(sp->u0[d])) return "u0 must be finite";
  if (s) {
    for (int k = 0; k < model; ++k)
      if (!(s[k] >= 0.0 && s[k] < 2.0)) return "relaxation rates must lie in [0, 2)";
  } else {
    return "s_vec is NULL";
  }
  return "";
}

// F(t) = F0 + FA cos(2 pi t / FT) (FT <= 0: F0).
void force_at(const lbm_spec& sp, long long t, double F[3]) {
  double ph = 1.0;
  if (sp.FT > 0.0) ph = std::cos(2.0 * M_PI * (double)t / sp.FT);
  for (int d = 0; d < 3; ++d) F[d] = sp.F0[d] + (sp.FT > 0.0 ? sp.FA[d] * ph : 0.0);
}

bool has_force(const lbm_spec& sp) {
  for (int d = 0; d < 3; ++d)
    if (sp.F0[d] != 0.0 || (sp.FT > 0.0 && sp.FA[d] != 0.0)) return true;
  return false;
}

template <int Q>
void lattice_tables(int (&cx)[26], int (&cy)[26], int (&cz)[26], double (&w)[26], int (&N)[26]) {
  for (int a = 0; a < Q; ++a) {
    cx[a] = Lattice<Q>::cx[a];
    cy[a] = Lattice<Q>::cy[a];
    cz[a] = Lattice<Q>::cz[a];
    w[a] = weight<Q>(a);
    N[a] = Lattice<Q>::N[a];
  }
}

}  // namespace

struct lbm_ctx {
  int q = 0, nx = 0, ny = 0, nz = 0;
  size_t N = 0;
  lbm_spec spec{};
  double s[26] = {};
  hipStream_t stream = nullptr;
  int device = 0;
  void* buf = nullptr;
  bool own_buf = false;
  size_t footprint = 0;
  void* popA = nullptr;  // current copy
  void* popB = nullptr;  // AB: the other copy
  int phase = 0;         // AA: 0 natural layout, 1 swapped
  long long t = 0;
  // monitor
  void* mon_buf = nullptr;  // separately allocated monitor area (when not in buf)
  void* snap = nullptr;
  double* partial = nullptr;
  double* d_res = nullptr;
  bool snap_valid = false;
  long long t_snap = 0;
  long long mon_lag = 0;
  bool mon_ran = false;
  bool mon_pending = false;  // the last monitor run's sums are not yet read
  double mon[3] = {0, 0, 0};
  // Monitor runs in flight: each copies its sums and the sticky flag into a
  // slot of pinned host memory and records that slot's event, in a ring of
  // kMonSlots, so that a poll can read the newest run that has completed
  // while later ones are still queued.
  double* h_mon = nullptr;                   // kMonSlots x 4 doubles
  hipEvent_t mon_ev[kMonSlots] = {};
  bool slot_pending[kMonSlots] = {};
  long long slot_t[kMonSlots] = {};
  int mon_next = 0;                          // slot of the next run
  int mon_last = 0;                          // slot of the last run
  bool mon_reset = true;        // the next run starts the device's non-finite flag afresh
  bool tripped = false;         // a completed monitor run saw a non-finite value
  long long trip_t = -1;        // ... in its run at this time level
  bool forced = false;
  int tx = 1, ty = 1;
  LatticeArgs<double> a64{};
  LatticeArgs<float> a32{};
  // velocity / pressure faces: the nodes on them (in buf) and their values
  int* nee_nodes = nullptr;
  int nee_count = 0;
  NeeArgs<double> e64{};
  NeeArgs<float> e32{};
  // HIP graphs of kGraphSteps steps, by AA parity / A-B buffer order
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;  // where the graphs are recorded (not run)
  bool graph_failed = false;  // a capture failed once: step eagerly from then on
  std::string err;
  void* batch = nullptr;  // batch this context belongs to (or NULL)
};

namespace {

// Message of the last failed lbm_create on this thread (lbm_last_error(NULL)).
thread_local std::string g_create_err;

int fail(lbm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(lbm_ctx* c, hipError_t e, const char* where) {
  return fail(c, LBM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, call)                               \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

// Workgroup order of the step kernels (a lattice, or all active members of
// a batch): one contiguous range of tiles per XCD up to 384 MB of
// populations (beyond: below).  The contiguous ranges, measured on
// D3Q18 AA cavities against dispatch order: FP32 +3 % at 96 MB,
// +1.3 % at 144 MB (128^3), +10-14 % at 172-241 MB, +1.5-3 % at 281-374 MB,
// but -4.6 % at 486 MB and -5.5 % at 1.2 GB (256^3); FP16 deviations
// +2-13 % at 72-308 MB; FP64 unchanged.
#ifndef LBM_XCD_ORDER_MAX_BYTES
#define LBM_XCD_ORDER_MAX_BYTES (384ull << 20)
#endif
// Beyond that size a single lattice hands the XCDs chunks of 4 rows in turn
// (xcd_order 2, a permutation of the low five bits of the workgroup index
// in the step kernel; from HBM +0.4-2.9 % over dispatch order, measured with
// a general chunk code that cost 1.4 % in the cache by spilling scalar
// registers, which this one does not), and a batch hands out chunks of
// LBM_XCD_CHUNK_BATCH workgroups (512 nodes each) per XCD in turn: the
// 256-cavity batch (4.85 GB) +3.1 % at 64 (+0.4 % at 4, +2.7 % at 16).
#ifndef LBM_XCD_CHUNK_BATCH
#define LBM_XCD_CHUNK_BATCH 64
#endif
static_assert(LBM_XCD_CHUNK_BATCH == 0 || (LBM_XCD_CHUNK_BATCH & (LBM_XCD_CHUNK_BATCH - 1)) == 0,
              "LBM_XCD_CHUNK_BATCH must be 0 or a power of two");
// xcd_order of the batch kernels for chunks of K = 2^k workgroups: k + 1
// (K <= 1: chunks of one are the dispatch order, 0).
constexpr int chunk_order(unsigned K) {
  int k = 0;
  while ((1u << k) < K) ++k;
  return K > 1 ? k + 1 : 0;
}
size_t step_bytes(const lbm_ctx& c) {
  return population_bytes(c.q, c.N, c.spec.storage) * (c.spec.pattern == LBM_AB ? 2 : 1);
}
int order_for(size_t bytes, bool batch) {
  if (bytes <= (size_t)LBM_XCD_ORDER_MAX_BYTES) return 1;
  return batch ? chunk_order(LBM_XCD_CHUNK_BATCH) : 2;
}

template <typename C>
void fill_args(const lbm_ctx& c, LatticeArgs<C>& A) {
  int cx[26], cy[26], cz[26], Nk[26];
  double w[26];
  if (c.q == 14)
    lattice_tables<14>(cx, cy, cz, w, Nk);
  else if (c.q == 18)
    lattice_tables<18>(cx, cy, cz, w, Nk);
  else
    lattice_tables<26>(cx, cy, cz, w, Nk);
  std::memset(&A, 0, sizeof(A));
  A.f = c.popA;
  A.g = c.popB ? c.popB : c.popA;
  A.stride = (long long)pop_stride(c.N);
  A.pbytes = A.stride * (c.spec.storage == LBM_F64 ? 8 : c.spec.storage == LBM_F32 ? 4 : 2);
  for (int a = 0; a < 26; ++a) A.pofs[a] = a * A.pbytes;
  A.nx = c.nx;
  A.ny = c.ny;
  A.nz = c.nz;
  A.per_x = c.spec.face[0] == LBM_PERIODIC;
  A.per_y = c.spec.face[2] == LBM_PERIODIC;
  A.per_z = c.spec.face[4] == LBM_PERIODIC;
  A.sym = 0;
  for (int f = 0; f < 6; ++f)
    if (c.spec.face[f] == LBM_SYMMETRY) A.sym |= 1 << f;
  A.tx = c.tx;
  A.ty = c.ty;
  A.xcd_order = order_for(step_bytes(c), false);
  A.tiles_x = (c.nx + c.tx - 1) / c.tx;
  A.tiles_y = (c.ny + c.ty - 1) / c.ty;
  A.fd_tiles_x = make_fastdiv((unsigned)A.tiles_x);
  A.fd_tiles_y = make_fastdiv((unsigned)A.tiles_y);
  A.fd_tx = make_fastdiv((unsigned)A.tx);
  for (int k = 0; k < c.q; ++k) {
    A.sN[k] = (C)(c.s[k] / Nk[k]);
    A.hN[k] = (C)((1.0 - 0.5 * c.s[k]) / Nk[k]);
  }
  const double sc = std::ldexp(1.0, c.spec.f16_scale_log2);
  // Wall term of population a leaving through the face its d-component
  // points at: 6 w_a (c_a . u_w), computed as the FP64 oracle of the paper
  // would (w_a times 6, times the dot product); for FP16 storage in the
  // step kernels' deviation units (times 2^s, exact).
  const double bb_units = c.spec.storage == LBM_F16DEV ? sc : 1.0;
  for (int a = 0; a < c.q; ++a) {
    const int comp[3] = {cx[a], cy[a], cz[a]};
    for (int d = 0; d < 3; ++d) {
      A.bb[a][d] = 0;
      if (!comp[d]) continue;
      const int face = 2 * d + (comp[d] > 0 ? 1 : 0);
      const double* uw = c.spec.wall_u[face];
      const double cu = cx[a] * uw[0] + cy[a] * uw[1] + cz[a] * uw[2];
      A.bb[a][d] = (C)(6.0 * w[a] * cu * bb_units);
    }
  }
  A.scale = (C)sc;
  A.inv_scale = (C)(1.0 / sc);
  // one base per weight class (|c_a|^2 = 1, 2, 3); classes a model lacks
  // are never read
  for (int k = 0; k < 3; ++k) {
    A.base[k] = A.base_s[k] = 0;
    for (int a = 0; a < c.q; ++a)
      if (cx[a] * cx[a] + cy[a] * cy[a] + cz[a] * cz[a] == k + 1) {
        A.base[k] = (C)(3.0 * w[a] * c.spec.p0);
        A.base_s[k] = A.base[k] * A.scale;
        break;
      }
  }
  A.F[0] = A.F[1] = A.F[2] = 0;
  A.tstep = (unsigned)c.t;
  A.f16_sr = c.spec.f16_rounding == LBM_ROUND_STOCHASTIC ? 1 : 0;
  A.omega = (C)c.s[0];
  A.hom = (C)(1.0 - 0.5 * c.s[0]);
}

void refresh_args(lbm_ctx& c) {
  fill_args<double>(c, c.a64);
  fill_args<float>(c, c.a32);
}

const void* args_ptr(lbm_ctx& c) {
  return c.spec.storage == LBM_F64 ? (const void*)&c.a64 : (const void*)&c.a32;
}

// Per-step kernel arguments: the force F(t) and the time level t.
void set_force(lbm_ctx& c, long long t) {
  double F[3];
  force_at(c.spec, t, F);
  for (int d = 0; d < 3; ++d) {
    c.a64.F[d] = F[d];
    c.a32.F[d] = (float)F[d];
  }
  c.a64.tstep = c.a32.tstep = (unsigned)t;
}

void pick_tile(int nx, int ny, int& tx, int& ty) {
  if (nx >= 256) {
    tx = 256;
    ty = 1;
  } else {
    tx = nx;
    ty = std::max(1, std::min(ny, 256 / nx));
  }
}

int ensure_monitor(lbm_ctx* c) {
  if (c->snap) return LBM_OK;
  const size_t snap_b = align_up(3 * c->N * (c->spec.storage == LBM_F64 ? 8 : 4));
  const size_t part_b = align_up(3 * sizeof(double) * 2048);
  const size_t bytes = monitor_bytes(c->N, c->spec.storage);
  char* base = nullptr;
  HIPCHK(c, hipMalloc((void**)&base, bytes));
  c->mon_buf = base;
  c->snap = base;
  c->partial = (double*)(base + snap_b);
  c->d_res = (double*)(base + snap_b + part_b);
  return LBM_OK;
}

// Pinned host slots for the monitor's sums and the events that say a slot
// holds its run's values.
int ensure_monitor_host(lbm_ctx* c) {
  if (!c->h_mon)
    HIPCHK(c, hipHostMalloc((void**)&c->h_mon, kMonSlots * 4 * sizeof(double),
                            hipHostMallocDefault));
  for (int s = 0; s < kMonSlots; ++s)
    if (!c->mon_ev[s]) HIPCHK(c, hipEventCreateWithFlags(&c->mon_ev[s], hipEventDisableTiming));
  return LBM_OK;
}

int trip_fail(lbm_ctx* c) {
  return fail(c, LBM_ENONFINITE,
              "the monitor found a non-finite value (run at t = " + std::to_string(c->trip_t) + ")");
}

// Queue a monitor run: the two reduction passes, then an asynchronous copy
// of the sums and the sticky non-finite flag to pinned host memory.
int run_monitor(lbm_ctx* c) {
  int rc = ensure_monitor(c);
  if (!rc) rc = ensure_monitor_host(c);
  if (rc) return rc;
  set_force(*c, c->t);
  int nb = 0;
  const int phase = c->spec.pattern == LBM_AA ? c->phase : 0;
  HIPCHK(c, launch_monitor(c->q, c->spec.storage, phase, args_ptr(*c), c->snap, c->partial, &nb,
                           c->stream));
  const int flags = (c->snap_valid ? 1 : 0) | (c->mon_reset ? 2 : 0);
  HIPCHK(c, launch_reduce_partials(c->partial, nb, c->d_res, flags, c->stream));
  // a slot kMonSlots runs old that is still unread is reused: the flag the
  // new run copies includes every earlier run's
  const int slot = c->mon_next;
  c->mon_next = (slot + 1) % kMonSlots;
  HIPCHK(c, hipMemcpyAsync(c->h_mon + 4 * slot, c->d_res, 4 * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipEventRecord(c->mon_ev[slot], c->stream));
  c->slot_pending[slot] = true;
  c->slot_t[slot] = c->t;
  c->mon_last = slot;
  c->mon_reset = false;
  c->mon_lag = c->snap_valid ? c->t - c->t_snap : 0;
  c->snap_valid = true;
  c->t_snap = c->t;
  c->mon_ran = true;
  c->mon_pending = true;
  return LBM_OK;
}

// Take over the values of a run whose copy has landed.
void absorb_slot(lbm_ctx* c, int s) {
  const double* h = c->h_mon + 4 * s;
  for (int k = 0; k < 3; ++k) c->mon[k] = h[k];
  if (h[3] != 0.0 && !c->tripped) {
    c->tripped = true;
    c->trip_t = c->slot_t[s];
  }
  c->slot_pending[s] = false;
  if (s == c->mon_last) c->mon_pending = false;
}

// Read, oldest first, every run whose copy has landed; never waits (runs
// complete in stream order, so the first one still in flight ends the scan).
int poll_monitor(lbm_ctx* c) {
  for (int i = 0; i < kMonSlots; ++i) {
    const int s = (c->mon_next + i) % kMonSlots;
    if (!c->slot_pending[s]) continue;
    const hipError_t e = hipEventQuery(c->mon_ev[s]);
    if (e == hipErrorNotReady) {
      (void)hipGetLastError();
      break;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipEventQuery(monitor)");
    absorb_slot(c, s);
  }
  return LBM_OK;
}

// Wait for the last monitor run (not for later work on the stream).
int fetch_monitor(lbm_ctx* c) {
  if (!c->mon_pending) return LBM_OK;
  HIPCHK(c, hipEventSynchronize(c->mon_ev[c->mon_last]));
  return poll_monitor(c);
}

// A new state (lbm_set_f, lbm_init_fields): earlier monitor findings no
// longer apply.
void reset_monitor_state(lbm_ctx* c) {
  c->snap_valid = false;
  c->tripped = false;
  c->trip_t = -1;
  c->mon_reset = true;
  c->mon_pending = false;
  for (bool& p : c->slot_pending) p = false;
}

// RAII device scratch for the non-hot host-data paths.
struct DevTmp {
  void* p = nullptr;
  ~DevTmp() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

extern "C" {

void lbm_spec_default(lbm_spec* sp) {
  if (!sp) return;
  std::memset(sp, 0, sizeof(*sp));
  for (int f = 0; f < 6; ++f) sp->face[f] = LBM_WALL;
  sp->storage = LBM_F32;
  sp->pattern = LBM_AA;
  sp->f16_scale_log2 = 12;
  sp->graphs = 1;
}

size_t lbm_footprint_bytes(int model, int nx, int ny, int nz, const lbm_spec* sp) {
  double s[26];
  for (int k = 0; k < 26; ++k) s[k] = 1.0;
  if (!validate(model, nx, ny, nz, s, sp).empty()) return 0;
  const size_t N = (size_t)nx * ny * nz;
  size_t b = align_up(population_bytes(model, N, sp->storage));
  if (sp->pattern == LBM_AB) b *= 2;
  b += align_up(sizeof(int) * (size_t)nee_node_count(nx, ny, nz, sp));
  if (sp->monitor_every > 0) b += monitor_bytes(N, sp->storage);
  return b;
}

int lbm_create(lbm_ctx** out, int model, int nx, int ny, int nz, const double* s_vec,
               const lbm_spec* sp) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  g_create_err.clear();
  const std::string v = validate(model, nx, ny, nz, s_vec, sp);
  if (!v.empty()) {
    g_create_err = v;
    return LBM_EINVAL;
  }
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ENOMEM;
  c->q = model;
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  c->N = (size_t)nx * ny * nz;
  c->spec = *sp;
  for (int k = 0; k < model; ++k) c->s[k] = s_vec[k];
  c->stream = (hipStream_t)sp->stream;
  c->forced = has_force(c->spec);
  pick_tile(nx, ny, c->tx, c->ty);
  {
    const long long tiles = (long long)((nx + c->tx - 1) / c->tx) * ((ny + c->ty - 1) / c->ty) * nz;
    if (tiles >= (1LL << 30)) {  // the kernels decode tile indices below 2^30
      delete c;
      g_create_err = "lattice needs too many workgroups (rows too short for its size)";
      return LBM_EINVAL;
    }
  }
  (void)hipGetDevice(&c->device);
  const size_t need = lbm_footprint_bytes(model, nx, ny, nz, sp);
  c->footprint = need;
  char* base = nullptr;
  if (sp->dev_buf) {
    if (sp->dev_buf_bytes < need) {
      delete c;
      g_create_err = "dev_buf_bytes below the footprint";
      return LBM_ENOMEM;
    }
    if (((uintptr_t)sp->dev_buf) % kAlign != 0) {
      delete c;
      g_create_err = "dev_buf must be 256-byte aligned";
      return LBM_EINVAL;
    }
    base = (char*)sp->dev_buf;
    c->own_buf = false;
  } else {
    const hipError_t me = hipMalloc((void**)&base, need);
    if (me != hipSuccess) {
      (void)hipGetLastError();
      delete c;
      g_create_err = std::string("hipMalloc: ") + hipGetErrorString(me);
      return LBM_ENOMEM;
    }
    c->own_buf = true;
  }
  c->buf = base;
  const size_t pop = align_up(population_bytes(model, c->N, sp->storage));
  c->popA = base;
  c->popB = sp->pattern == LBM_AB ? base + pop : nullptr;
  size_t off = pop * (sp->pattern == LBM_AB ? 2 : 1);
  c->nee_count = (int)nee_node_count(nx, ny, nz, sp);
  if (c->nee_count > 0) {
    // nodes on velocity / pressure faces, in increasing linear index
    std::vector<int> list;
    list.reserve((size_t)c->nee_count);
    auto on = [&](int v, int n, int d) {
      return (v == 0 && is_nee_face(sp->face[2 * d])) ||
             (v == n - 1 && is_nee_face(sp->face[2 * d + 1]));
    };
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y) {
        const bool row = on(z, nz, 2) || on(y, ny, 1);
        const int base_n = nx * (y + ny * z);
        if (row) {
          for (int x = 0; x < nx; ++x) list.push_back(base_n + x);
        } else {
          if (on(0, nx, 0)) list.push_back(base_n);
          if (nx > 1 && on(nx - 1, nx, 0)) list.push_back(base_n + nx - 1);
        }
      }
    c->nee_nodes = (int*)(base + off);
    off += align_up(sizeof(int) * list.size());
    hipError_t e = list.size() == (size_t)c->nee_count
                       ? hipMemcpy(c->nee_nodes, list.data(), sizeof(int) * list.size(),
                                   hipMemcpyHostToDevice)
                       : hipErrorInvalidValue;
    if (e != hipSuccess) {
      g_create_err = std::string("boundary node list: ") + hipGetErrorString(e);
      lbm_destroy(c);
      return LBM_EDEVICE;
    }
    for (int f = 0; f < 6; ++f) {
      c->e64.kind[f] = c->e32.kind[f] = sp->face[f];
      for (int d = 0; d < 3; ++d) {
        c->e64.u[f][d] = sp->wall_u[f][d];
        c->e32.u[f][d] = (float)sp->wall_u[f][d];
      }
    }
  }
  if (sp->monitor_every > 0) {
    const size_t snap_b = align_up(3 * c->N * (sp->storage == LBM_F64 ? 8 : 4));
    const size_t part_b = align_up(3 * sizeof(double) * 2048);
    c->snap = base + off;
    c->partial = (double*)(base + off + snap_b);
    c->d_res = (double*)(base + off + snap_b + part_b);
  }
  refresh_args(*c);
  set_force(*c, 0);
  const double u0[3] = {sp->u0[0], sp->u0[1], sp->u0[2]};
  hipError_t e = launch_init_eq(c->q, sp->storage, args_ptr(*c), nullptr, nullptr, sp->p0, u0,
                                c->stream);
  if (e != hipSuccess) {
    g_create_err = std::string("initialisation kernel: ") + hipGetErrorString(e);
    lbm_destroy(c);
    return LBM_EDEVICE;
  }
  *out = c;
  return LBM_OK;
}

}  // extern "C"

namespace {

// Steps per captured graph (even, so that the AA parity and the A/B buffer
// order are back where they started).
constexpr int kGraphSteps = 32;

// One time step of the context: the step kernel, the velocity / pressure /
// symmetry-node pass, and the state that goes with them (no monitor).
int eager_step(lbm_ctx* c) {
  set_force(*c, c->t);
  int mode;
  if (c->spec.pattern == LBM_AB) {
    mode = MODE_AB;
  } else {
    mode = c->phase == 0 ? MODE_AA_EVEN : MODE_AA_ODD;
  }
  if (c->spec.collision == LBM_BGK)
    HIPCHK(c, launch_step_bgk(c->q, c->spec.storage, mode, c->forced, args_ptr(*c), c->stream));
  else
    HIPCHK(c, launch_step(c->q, c->spec.storage, mode, c->forced, args_ptr(*c), 0, c->stream));
  if (c->spec.pattern == LBM_AB) {
    std::swap(c->popA, c->popB);
    c->a64.f = c->a32.f = c->popA;
    c->a64.g = c->a32.g = c->popB;
  } else {
    c->phase ^= 1;
  }
  c->t += 1;
  if (c->nee_count > 0) {
    // velocity / pressure faces at the level just reached
    set_force(*c, c->t);
    for (int f = 0; f < 6; ++f) {
      double pf = c->spec.face_p[f];
      if (c->spec.FT > 0.0)
        pf += c->spec.face_pA[f] * std::cos(2.0 * M_PI * (double)c->t / c->spec.FT);
      c->e64.p[f] = pf;
      c->e32.p[f] = (float)pf;
    }
    const int phase = c->spec.pattern == LBM_AA ? c->phase : 0;
    const void* e = c->spec.storage == LBM_F64 ? (const void*)&c->e64 : (const void*)&c->e32;
    HIPCHK(c, launch_nee(c->q, c->spec.storage, phase, args_ptr(*c), e, c->nee_nodes,
                         c->nee_count, c->stream));
  }
  return LBM_OK;
}

// Lattices from this many nodes up step eagerly: their kernels run long
// enough to hide the launch cost, and graph replay measured 0.3 % slower
// at 128^3 (+3 % at 64^3, +8 % at 16x16x32).
constexpr size_t kGraphMaxNodes = size_t(1) << 21;

// Whether graphs pay and consecutive steps launch identical kernels with
// identical arguments (apart from the alternation that an even step count
// undoes).
bool graph_eligible(const lbm_ctx* c) {
  if (!c->spec.graphs || c->graph_failed || c->N >= kGraphMaxNodes) return false;
  if (c->spec.FT > 0.0) return false;               // F(t), face p(t) change every step
  if (c->spec.storage == LBM_F16DEV && c->spec.f16_rounding == LBM_ROUND_STOCHASTIC)
    return false;                                   // rounding bits depend on t
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->stream, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st == hipStreamCaptureStatusNone;          // the caller is not capturing
}

// kGraphSteps steps through the graph for the current parity / buffer order
// (captured on first use).  The launches are recorded on a private stream
// of the context (the legacy null stream, torch's default, cannot be
// captured) and the graph is then launched on the context's stream.
// Returns LBM_OK, or 1 if no graph could be made (the caller then steps
// eagerly), or an error status.
int graph_steps(lbm_ctx* c) {
  const int key = c->spec.pattern == LBM_AA ? c->phase : (c->popA == c->buf ? 0 : 1);
  if (!c->gexec[key]) {
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      c->cap_stream = nullptr;
      c->graph_failed = true;
      return 1;
    }
    const long long t0 = c->t;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      c->graph_failed = true;
      return 1;
    }
    hipStream_t run = c->stream;
    c->stream = c->cap_stream;
    int rc = LBM_OK;
    for (int k = 0; k < kGraphSteps && rc == LBM_OK; ++k) rc = eager_step(c);
    c->stream = run;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->t = t0;  // nothing has run yet; parity and buffer order are back (even count)
    if (rc != LBM_OK || e != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      c->graph_failed = true;
      return rc != LBM_OK ? rc : 1;
    }
    const hipError_t ie = hipGraphInstantiate(&c->gexec[key], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      c->gexec[key] = nullptr;
      (void)hipGetLastError();
      c->graph_failed = true;
      return 1;
    }
  }
  HIPCHK(c, hipGraphLaunch(c->gexec[key], c->stream));
  c->t += kGraphSteps;
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_step(lbm_ctx* c, long long n) {
  if (!c) return LBM_EINVAL;
  if (n < 0) return fail(c, LBM_EINVAL, "n must be >= 0");
  int prc = poll_monitor(c);
  if (prc) return prc;
  if (c->tripped) return trip_fail(c);
  const long long K = c->spec.monitor_every;
  long long i = 0;
  const bool graphs = n >= kGraphSteps && graph_eligible(c);
  while (i < n) {
    int rc = 1;
    if (graphs) {
      // steps left before the next monitor point (a graph never spans one)
      const long long span = K > 0 ? std::min(n - i, K - c->t % K) : n - i;
      if (span >= kGraphSteps) rc = graph_steps(c);
      if (rc == LBM_OK) i += kGraphSteps;
      if (rc < 0) return rc;
    }
    if (rc != LBM_OK) {
      rc = eager_step(c);
      if (rc) return rc;
      i += 1;
    }
    if (K > 0 && c->t % K == 0) {
      // the previous run's findings, if they have landed (no wait)
      rc = poll_monitor(c);
      if (rc) return rc;
      if (c->tripped) return trip_fail(c);
      rc = run_monitor(c);
      if (rc) return rc;
    }
  }
  return LBM_OK;
}

int lbm_macros_device(lbm_ctx* c, double* p_dev, double* u_dev) {
  if (!c) return LBM_EINVAL;
  set_force(*c, c->t);
  const int phase = c->spec.pattern == LBM_AA ? c->phase : 0;
  HIPCHK(c, launch_macros(c->q, c->spec.storage, phase, args_ptr(*c), p_dev, u_dev, c->stream));
  return LBM_OK;
}

int lbm_macros(lbm_ctx* c, double* p, double* u) {
  if (!c) return LBM_EINVAL;
  if (!p && !u) return LBM_OK;
  DevTmp tp, tu;
  if (p) HIPCHK(c, hipMalloc(&tp.p, c->N * sizeof(double)));
  if (u) HIPCHK(c, hipMalloc(&tu.p, 3 * c->N * sizeof(double)));
  int rc = lbm_macros_device(c, (double*)tp.p, (double*)tu.p);
  if (rc) return rc;
  if (p)
    HIPCHK(c, hipMemcpyAsync(p, tp.p, c->N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (u)
    HIPCHK(c, hipMemcpyAsync(u, tu.p, 3 * c->N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

}  // extern "C"

// ---- the allocation-free macros call --------------------------------------
// lbm_macros_noalloc stages p and u of a node range between the macros
// kernel and the copies to the caller's host arrays in this file-scope
// device array instead of memory it allocates: 8 MiB, p, u_x, u_y and u_z
// of up to kNoallocNodes nodes.  Each GPU the library runs on holds its own
// copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not the device memory: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current and
// kept in g_scratch_dev, and only that address is handed to kernels and
// copies.
namespace {
constexpr long long kNoallocNodes = LBM_NOALLOC_MAX_NODES;
constexpr int kMaxDevices = 64;
}  // namespace
static __device__ __align__(256) double scratch[4 * kNoallocNodes];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of this device's scratch (looked up on first use).
int scratch_address(lbm_ctx* c, double** out) {
  if (c->device < 0 || c->device >= kMaxDevices)
    return fail(c, LBM_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[c->device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(c, LBM_EDEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_dev[c->device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_dev[c->device];
  return LBM_OK;
}

// Makes the context's device current for a scope and restores the caller's.
struct DeviceScope {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceScope(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceScope() {
    int now = -1;
    if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
  }
};
}  // namespace

extern "C" {

int lbm_macros_noalloc(lbm_ctx* c, long long n0, long long count, double* p, double* u) {
  if (!c) return LBM_EINVAL;
  if (n0 < 0 || count < 0 || n0 > (long long)c->N || count > (long long)c->N - n0)
    return fail(c, LBM_EINVAL, "node range [n0, n0 + count) outside the lattice");
  if (count > kNoallocNodes)
    return fail(c, LBM_EINVAL,
                "count " + std::to_string(count) + " exceeds the " +
                    std::to_string(kNoallocNodes) +
                    " nodes the static scratch of lbm_macros_noalloc holds (8 MiB)");
  if (count == 0 || (!p && !u)) return LBM_OK;
  DeviceScope scope(c->device);
  if (scope.err != hipSuccess) return hip_fail(c, scope.err, "hipSetDevice");
  double* s = nullptr;
  int rc = scratch_address(c, &s);
  if (rc) return rc;
  set_force(*c, c->t);
  const int phase = c->spec.pattern == LBM_AA ? c->phase : 0;
  HIPCHK(c, launch_macros_range(c->q, c->spec.storage, phase, args_ptr(*c), n0, count, s,
                                c->stream));
  const size_t bytes = (size_t)count * sizeof(double);
  if (p) HIPCHK(c, hipMemcpyAsync(p, s, bytes, hipMemcpyDeviceToHost, c->stream));
  if (u)
    for (int d = 0; d < 3; ++d)
      HIPCHK(c, hipMemcpyAsync(u + (size_t)d * count, s + (size_t)(1 + d) * count, bytes,
                               hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_monitor(lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  return run_monitor(c);
}

int lbm_residual(lbm_ctx* c, double* r) {
  if (!c || !r) return LBM_EINVAL;
  if (!c->mon_ran) return fail(c, LBM_ESTATE, "the monitor has not run");
  int rc = fetch_monitor(c);
  if (rc) return rc;
  // Without an earlier snapshot of this state (lag 0) the difference sum was
  // taken against whatever the snapshot buffer held (fresh memory, or a
  // state replaced since) and means nothing: only sum|u| and the mass
  // speak for the current populations then.
  const bool lagged = c->mon_lag > 0;
  if ((lagged && !std::isfinite(c->mon[0])) || !std::isfinite(c->mon[1]) ||
      !std::isfinite(c->mon[2])) {
    *r = std::numeric_limits<double>::quiet_NaN();
    return fail(c, LBM_ENONFINITE, "monitor found a non-finite value");
  }
  if (!lagged || !(c->mon[1] > 0.0))
    *r = std::numeric_limits<double>::infinity();
  else
    *r = c->mon[0] / ((double)c->mon_lag * c->mon[1]);
  return LBM_OK;
}

int lbm_residual_change(lbm_ctx* c, double* r, long long* lag) {
  if (!c || !r) return LBM_EINVAL;
  if (!c->mon_ran) return fail(c, LBM_ESTATE, "the monitor has not run");
  int rc = fetch_monitor(c);
  if (rc) return rc;
  const bool lagged = c->mon_lag > 0;
  if (lag) *lag = c->mon_lag;
  if ((lagged && !std::isfinite(c->mon[0])) || !std::isfinite(c->mon[1]) ||
      !std::isfinite(c->mon[2])) {
    *r = std::numeric_limits<double>::quiet_NaN();
    return fail(c, LBM_ENONFINITE, "monitor found a non-finite value");
  }
  if (!lagged || !(c->mon[1] > 0.0))
    *r = std::numeric_limits<double>::infinity();
  else
    *r = c->mon[0] / c->mon[1];
  return LBM_OK;
}

int lbm_poll(lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  const int rc = poll_monitor(c);
  if (rc) return rc;
  return c->tripped ? trip_fail(c) : LBM_OK;
}

int lbm_mass(lbm_ctx* c, double* m) {
  if (!c || !m) return LBM_EINVAL;
  if (!c->mon_ran) {
    int rc = run_monitor(c);
    if (rc) return rc;
  }
  int rc = fetch_monitor(c);
  if (rc) return rc;
  *m = c->mon[2];
  if (!std::isfinite(*m)) return fail(c, LBM_ENONFINITE, "monitor found a non-finite mass");
  return LBM_OK;
}

int lbm_get_f(lbm_ctx* c, double* f) {
  if (!c || !f) return LBM_EINVAL;
  DevTmp tmp;
  HIPCHK(c, hipMalloc(&tmp.p, c->N * sizeof(double)));
  const int phase = c->spec.pattern == LBM_AA ? c->phase : 0;
  for (int a = 0; a < c->q; ++a) {
    HIPCHK(c, launch_get_pop(c->q, c->spec.storage, phase, a, args_ptr(*c), (double*)tmp.p,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(f + (size_t)a * c->N, tmp.p, c->N * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return LBM_OK;
}

int lbm_set_f(lbm_ctx* c, const double* f) {
  if (!c || !f) return LBM_EINVAL;
  DevTmp tmp;
  HIPCHK(c, hipMalloc(&tmp.p, c->N * sizeof(double)));
  // the natural layout is written: AA parity restarts at 0
  c->phase = 0;
  for (int a = 0; a < c->q; ++a) {
    HIPCHK(c, hipMemcpyAsync(tmp.p, f + (size_t)a * c->N, c->N * sizeof(double),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_set_pop(c->q, c->spec.storage, a, args_ptr(*c), (const double*)tmp.p,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  reset_monitor_state(c);
  return LBM_OK;
}

int lbm_init_fields(lbm_ctx* c, const double* p, const double* u) {
  if (!c) return LBM_EINVAL;
  DevTmp tp, tu;
  if (p) {
    HIPCHK(c, hipMalloc(&tp.p, c->N * sizeof(double)));
    HIPCHK(c, hipMemcpyAsync(tp.p, p, c->N * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  if (u) {
    HIPCHK(c, hipMalloc(&tu.p, 3 * c->N * sizeof(double)));
    HIPCHK(c, hipMemcpyAsync(tu.p, u, 3 * c->N * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  c->phase = 0;
  set_force(*c, c->t);
  HIPCHK(c, launch_init_eq(c->q, c->spec.storage, args_ptr(*c), (const double*)tp.p,
                           (const double*)tu.p, c->spec.p0, c->spec.u0, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  reset_monitor_state(c);
  return LBM_OK;
}

long long lbm_time(const lbm_ctx* c) { return c ? c->t : -1; }

int lbm_set_time(lbm_ctx* c, long long t) {
  if (!c || t < 0) return LBM_EINVAL;
  c->t = t;
  c->snap_valid = false;
  return LBM_OK;
}

int lbm_info(const lbm_ctx* c, lbm_info_t* info) {
  if (!c || !info) return LBM_EINVAL;
  info->q = c->q;
  info->nx = c->nx;
  info->ny = c->ny;
  info->nz = c->nz;
  info->storage = c->spec.storage;
  info->pattern = c->spec.pattern;
  info->t = c->t;
  info->nodes = c->N;
  info->population_bytes = population_bytes(c->q, c->N, c->spec.storage);
  info->footprint_bytes = c->footprint;
  info->bytes_per_value = bytes_of(c->spec.storage);
  info->graphs = (c->gexec[0] != nullptr) + (c->gexec[1] != nullptr);
  return LBM_OK;
}

int lbm_sync(lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* c) {
  return c ? c->err.c_str() : g_create_err.c_str();
}

const char* lbm_status_string(int s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of device memory";
    case LBM_EDEVICE: return "device error";
    case LBM_ENONFINITE: return "non-finite value";
    case LBM_ESTATE: return "invalid state";
  }
  return "unknown status";
}

int lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_OK;
  if (c->batch) (void)lbm_batch_remove((lbm_batch*)c->batch, c);
  // Wait only when device memory this library allocated is freed; a
  // caller-owned buffer stays valid and its reuse is the caller's (stream-
  // ordered) business, so queued work keeps running.
  if ((c->own_buf && c->buf) || c->mon_buf) (void)hipStreamSynchronize(c->stream);
  if (c->own_buf && c->buf) (void)hipFree(c->buf);
  if (c->mon_buf) (void)hipFree(c->mon_buf);
  for (hipEvent_t& ev : c->mon_ev)
    if (ev) {
      (void)hipEventSynchronize(ev);  // its copy writes into h_mon
      (void)hipEventDestroy(ev);
    }
  if (c->h_mon) (void)hipHostFree(c->h_mon);
  for (auto& g : c->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
  return LBM_OK;
}

int lbm_pattern_probe(void* buf, int q, int elem_bytes, int nx, int ny, int nz,
                      long long stride, int odd, int reps, void* stream) {
  if (!buf || (q != 14 && q != 18 && q != 26) ||
      (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) || nx < 1 || ny < 1 || nz < 1 ||
      stride < (long long)nx * ny * nz || (odd != 0 && odd != 1) || reps < 0)
    return LBM_EINVAL;
  // the step kernels' workgroup order rule for this footprint (up to 384 MB:
  // contiguous ranges per XCD; beyond, dispatch order here)
  const size_t bytes = (size_t)q * (size_t)stride * (size_t)elem_bytes;
  const int xcd = bytes <= (size_t)LBM_XCD_ORDER_MAX_BYTES ? 1 : 0;
  for (int i = 0; i < reps; ++i)
    if (launch_pattern_probe(buf, q, elem_bytes, nx, ny, nz, stride, odd, xcd,
                             (hipStream_t)stream) != hipSuccess)
      return LBM_EDEVICE;
  return LBM_OK;
}

int lbm_copy_probe(void* dst, const void* src, size_t bytes, int reps, void* stream) {
  if (!dst || !src || bytes % 16 || reps < 0) return LBM_EINVAL;
  // the faster workgroup order for the bytes touched (XCD-contiguous from HBM)
  const size_t touched = dst == src ? bytes : 2 * bytes;
  const int xcd = touched > (size_t)LBM_XCD_ORDER_MAX_BYTES ? 1 : 0;
  for (int i = 0; i < reps; ++i)
    if (launch_copy_probe(dst, src, bytes, xcd, (hipStream_t)stream) != hipSuccess)
      return LBM_EDEVICE;
  return LBM_OK;
}

}  // extern "C"

// ============================ batches =======================================
namespace {
struct Member {
  lbm_ctx* ctx;
  long long remaining;
  int tx, ty;  // 0: automatic
};

// Automatic mapping of a member's nodes to workgroups: 256 consecutive
// nodes each ("flat"; measured 2-5 % faster than row tiles for edges that
// are not multiples of 64, equal at 64), or tiles of whole rows for members
// with N >= 2^30 (the flat node index is decoded with multiply-shift
// division, exact below 2^30).
bool member_flat(const Member& m) { return m.tx == 0 && m.ctx->N < (1u << 30); }
}  // namespace

// Launch classes of at least this many tiles (2^22 nodes at 256 nodes a
// tile, 64 tiles per compute unit) run kBatchChunk tiles per workgroup;
// smaller ones one tile per workgroup, so that they keep enough workgroups.
constexpr long long kBatchChunkMinTiles = 16384;

// A member of at least this many nodes that is the only active member of
// its (q, storage) class in a call takes its steps with the single-lattice
// kernels (lbm_step's eager path: the same arithmetic and bits),
// interleaved with the other classes' launches: for such a member the class
// launch is the same work with the batch kernel's member lookup on top (one
// 128^3 D3Q18 FP32 member: 44.5k MLUPS batched, 46.0k alone; FP32 serving
// trace +0.7 % Poisson, +1.4 % saturated), and an FP16 member would miss
// the single-lattice odd step's lean general path (FP16 serving trace,
// saturated: 72.0k against 68.7k MLUPS).  Several large members of one
// class keep sharing its launch (stepping every large FP16 member on its
// own measured 71.6k on the same trace).
// A member whose population buffer spans 4 GiB or more always steps on its
// own: the class kernels address members with 32-bit offsets where that
// pays (the odd step of FP16 and 26-velocity classes).
#ifndef LBM_BATCH_SOLO_NODES
#define LBM_BATCH_SOLO_NODES (1ll << 18)
#endif

struct lbm_batch {
  hipStream_t stream = nullptr;
  std::vector<Member> members;
  std::string err;
  // device staging (grown on demand)
  BatchMember* d_members = nullptr;
  size_t d_members_cap = 0;
  BatchChunk* d_chunks = nullptr;
  size_t d_chunks_cap = 0;
  float* d_ftab = nullptr;
  size_t d_ftab_cap = 0;
  float* d_ntab = nullptr;   // boundary rows (9 floats per member step)
  size_t d_ntab_cap = 0;
  // pinned host staging + the event that says it may be reused
  BatchMember* h_members = nullptr;
  size_t h_members_cap = 0;
  BatchChunk* h_chunks = nullptr;
  size_t h_chunks_cap = 0;
  float* h_ftab = nullptr;
  size_t h_ftab_cap = 0;
  float* h_ntab = nullptr;
  size_t h_ntab_cap = 0;
  hipEvent_t staged = nullptr;
  // monitor staging
  char* d_mon = nullptr;
  size_t d_mon_cap = 0;
};

namespace {
int bfail(lbm_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}
#define BHIP(b, call)                                                         \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) return bfail(b, LBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
int grow_dev(lbm_batch* b, T*& p, size_t& cap, size_t n) {
  if (n <= cap) return LBM_OK;
  if (p) BHIP(b, hipFree(p));
  p = nullptr;
  size_t c = std::max<size_t>(n, cap * 2);
  BHIP(b, hipMalloc((void**)&p, c * sizeof(T)));
  cap = c;
  return LBM_OK;
}
template <typename T>
int grow_host(lbm_batch* b, T*& p, size_t& cap, size_t n) {
  if (n <= cap) return LBM_OK;
  if (p) BHIP(b, hipHostFree(p));
  p = nullptr;
  size_t c = std::max<size_t>(n, cap * 2);
  BHIP(b, hipHostMalloc((void**)&p, c * sizeof(T), hipHostMallocDefault));
  cap = c;
  return LBM_OK;
}
}  // namespace

extern "C" {

int lbm_batch_create(lbm_batch** out, void* stream) {
  if (!out) return LBM_EINVAL;
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_ENOMEM;
  b->stream = (hipStream_t)stream;
  if (hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) {
    delete b;
    return LBM_EDEVICE;
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_add(lbm_batch* b, lbm_ctx* c, long long budget) {
  if (!b || !c || budget < 0) return LBM_EINVAL;
  if (c->batch) return bfail(b, LBM_EINVAL, "context already belongs to a batch");
  if (c->spec.pattern != LBM_AA) return bfail(b, LBM_EINVAL, "batched members must use LBM_AA");
  if (c->spec.storage == LBM_F64)
    return bfail(b, LBM_EINVAL, "batched members must store LBM_F32 or LBM_F16DEV");
  if (c->stream != b->stream) return bfail(b, LBM_EINVAL, "member stream differs from batch stream");
  if (c->spec.collision != LBM_MRT) return bfail(b, LBM_EINVAL, "batched members use LBM_MRT");
  b->members.push_back(Member{c, budget, 0, 0});
  c->batch = b;
  return LBM_OK;
}

int lbm_batch_remove(lbm_batch* b, lbm_ctx* c) {
  if (!b || !c) return LBM_EINVAL;
  for (size_t i = 0; i < b->members.size(); ++i)
    if (b->members[i].ctx == c) {
      b->members.erase(b->members.begin() + i);
      c->batch = nullptr;
      return LBM_OK;
    }
  return bfail(b, LBM_EINVAL, "not a member");
}

int lbm_batch_set_tile(lbm_batch* b, lbm_ctx* c, int tx, int ty) {
  if (!b || !c) return LBM_EINVAL;
  if (tx < 0 || ty < 0 || (long long)tx * ty > 256 || ((tx == 0) != (ty == 0)))
    return bfail(b, LBM_EINVAL, "tile must satisfy 1 <= tx*ty <= 256 (or 0,0)");
  for (auto& m : b->members)
    if (m.ctx == c) {
      m.tx = tx;
      m.ty = ty;
      return LBM_OK;
    }
  return bfail(b, LBM_EINVAL, "not a member");
}

long long lbm_batch_remaining(const lbm_batch* b, const lbm_ctx* c) {
  if (!b || !c) return -1;
  for (const auto& m : b->members)
    if (m.ctx == c) return m.remaining;
  return -1;
}

int lbm_batch_size(const lbm_batch* b) { return b ? (int)b->members.size() : 0; }

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : "null batch"; }

int lbm_batch_step(lbm_batch* b, long long n) {
  if (!b || n < 0) return LBM_EINVAL;
  if (n == 0 || b->members.empty()) return LBM_OK;
  if (n > (1LL << 30)) return bfail(b, LBM_EINVAL, "n too large for one call");
  // active members and their step counts for this call; a large member
  // alone in its (q, storage) class steps on its own (solo)
  std::vector<int> act, solo;
  std::vector<long long> solo_k;
  long long nmax = 0, solo_max = 0;
  size_t ftab_rows = 0, ntab_rows = 0;
  auto model_storage = [&](size_t i) {
    const lbm_ctx* c = b->members[i].ctx;
    return 2 * (c->q == 14 ? 0 : c->q == 18 ? 1 : 2) + (c->spec.storage == LBM_F32 ? 0 : 1);
  };
  int per_class[6] = {};
  for (size_t i = 0; i < b->members.size(); ++i)
    if (std::min(n, b->members[i].remaining) > 0) ++per_class[model_storage(i)];
  for (size_t i = 0; i < b->members.size(); ++i) {
    const long long k = std::min(n, b->members[i].remaining);
    if (k <= 0) continue;
    const lbm_ctx* mc = b->members[i].ctx;
    const bool huge = population_bytes(mc->q, (size_t)mc->N, mc->spec.storage) > 0xffffffffull;
    if (huge || ((long long)mc->N >= (long long)LBM_BATCH_SOLO_NODES &&
                 per_class[model_storage(i)] == 1)) {
      solo.push_back((int)i);
      solo_k.push_back(k);
      solo_max = std::max(solo_max, k);
      continue;
    }
    act.push_back((int)i);
    nmax = std::max(nmax, k);
    if (b->members[i].ctx->forced) ftab_rows += (size_t)k;
    if (b->members[i].ctx->nee_count > 0) ntab_rows += (size_t)k;
  }
  auto solo_substep = [&](long long s) -> int {
    for (size_t j = 0; j < solo.size(); ++j)
      if (s < solo_k[j]) {
        lbm_ctx* c = b->members[solo[j]].ctx;
        const int rc = eager_step(c);
        if (rc) return bfail(b, rc, c->err);
      }
    return LBM_OK;
  };
  auto solo_done = [&]() {
    for (size_t j = 0; j < solo.size(); ++j) b->members[solo[j]].remaining -= solo_k[j];
  };
  if (act.empty()) {
    for (long long s = 0; s < solo_max; ++s) {
      const int rc = solo_substep(s);
      if (rc) return rc;
    }
    solo_done();
    return LBM_OK;
  }
  // One specialised launch per (q, storage) class and step.  For n >= 2 the
  // members run in step with the AA parity of the first active member (one
  // out of step sits out the first substep of this call); for n == 1 the
  // parity is part of the class instead.  Class index: 6 x odd parity
  // (n == 1 only) + 2 x model (0: q = 14, 1: q = 18, 2: q = 26) + FP16.
  constexpr int NG = 12;
  const bool align = n >= 2;
  const int parity = b->members[act[0]].ctx->phase;
  auto cls = [&](int i) {
    const lbm_ctx* c = b->members[i].ctx;
    return (align ? 0 : (c->phase ? 6 : 0)) + 2 * (c->q == 14 ? 0 : c->q == 18 ? 1 : 2) +
           (c->spec.storage == LBM_F32 ? 0 : 1);
  };
  auto cls_q = [](int k) { return (k % 6) < 2 ? 14 : (k % 6) < 4 ? 18 : 26; };
  std::stable_sort(act.begin(), act.end(), [&](int x, int y) { return cls(x) < cls(y); });
  const int nm = (int)act.size();
  int cls_off[NG] = {}, cls_cnt[NG] = {}, cls_forced[NG] = {};
  long long cls_tiles[NG] = {}, cls_steps[NG] = {}, cls_nee[NG] = {};
  // chunks (large classes only): a member's tiles in runs of kBatchChunk,
  // grouped by class
  auto member_tiles = [&](int i) {
    const lbm_ctx* c = b->members[i].ctx;
    if (member_flat(b->members[i])) return (long long)((c->N + 255) / 256);
    int tx = b->members[i].tx, ty = b->members[i].ty;
    if (tx == 0) pick_tile(c->nx, c->ny, tx, ty);
    return (long long)((c->nx + tx - 1) / tx) * ((c->ny + ty - 1) / ty) * c->nz;
  };
  long long all_tiles[NG] = {};
  for (int i : act) all_tiles[cls(i)] += member_tiles(i);
  bool cls_big[NG];
  for (int k = 0; k < NG; ++k) cls_big[k] = all_tiles[k] >= kBatchChunkMinTiles;
  long long nchunks = 0;
  for (int i : act)
    if (cls_big[cls(i)]) nchunks += (member_tiles(i) + kBatchChunk - 1) / kBatchChunk;
  if (nchunks >= (1LL << 31)) return bfail(b, LBM_EINVAL, "too many tiles in one batch");
  long long cls_chunk_off[NG] = {}, cls_chunks[NG] = {};
  // the pinned staging may still be read by the previous upload
  BHIP(b, hipEventSynchronize(b->staged));
  int rc = grow_host(b, b->h_members, b->h_members_cap, (size_t)nm);
  if (!rc) rc = grow_dev(b, b->d_members, b->d_members_cap, (size_t)nm);
  if (!rc) rc = grow_host(b, b->h_chunks, b->h_chunks_cap, std::max<long long>(nchunks, 1));
  if (!rc) rc = grow_dev(b, b->d_chunks, b->d_chunks_cap, std::max<long long>(nchunks, 1));
  if (!rc) rc = grow_host(b, b->h_ftab, b->h_ftab_cap, std::max<size_t>(3 * ftab_rows, 3));
  if (!rc) rc = grow_dev(b, b->d_ftab, b->d_ftab_cap, std::max<size_t>(3 * ftab_rows, 3));
  if (!rc) rc = grow_host(b, b->h_ntab, b->h_ntab_cap, std::max<size_t>(9 * ntab_rows, 9));
  if (!rc) rc = grow_dev(b, b->d_ntab, b->d_ntab_cap, std::max<size_t>(9 * ntab_rows, 9));
  if (rc) return rc;
  size_t frow = 0, nrow = 0;
  long long chunk = 0;
  for (int j = 0; j < nm; ++j) {
    Member& m = b->members[act[j]];
    lbm_ctx* c = m.ctx;
    const int k_cls = cls(act[j]);
    if (cls_cnt[k_cls]++ == 0) {
      cls_off[k_cls] = j;
      cls_chunk_off[k_cls] = chunk;
    }
    long long& tiles = cls_tiles[k_cls];
    BatchMember& bm = b->h_members[j];
    std::memset(&bm, 0, sizeof(bm));
    int tx = m.tx, ty = m.ty;
    if (tx == 0) pick_tile(c->nx, c->ny, tx, ty);
    const int save_tx = c->tx, save_ty = c->ty;
    c->tx = tx;
    c->ty = ty;
    fill_args<float>(*c, bm.a);
    c->tx = save_tx;
    c->ty = save_ty;
    bm.q = c->q;
    bm.storage = c->spec.storage == LBM_F32 ? ST_F32 : ST_F16;
    bm.phase0 = c->phase;
    bm.skip = (align && c->phase != parity) ? 1 : 0;
    const long long k = std::min(n - bm.skip, m.remaining);
    bm.steps = (int)k;
    bm.tile_begin = tiles;
    bm.ntiles = (long long)bm.a.tiles_x * bm.a.tiles_y * c->nz;
    bm.flat = member_flat(m) ? 1 : 0;
    if (bm.flat) {
      bm.ntiles = (long long)((c->N + 255) / 256);
      bm.fd_nx = make_fastdiv((unsigned)c->nx);
      bm.fd_ny = make_fastdiv((unsigned)c->ny);
    }
    tiles += bm.ntiles;
    if (cls_big[k_cls])
      for (long long t0 = 0; t0 < bm.ntiles; t0 += kBatchChunk) {
        b->h_chunks[chunk].member = j - cls_off[k_cls];
        b->h_chunks[chunk].tile = (int)t0;
        ++chunk;
        ++cls_chunks[k_cls];
      }
    cls_steps[k_cls] = std::max(cls_steps[k_cls], k + bm.skip);
    bm.forced = c->forced ? 1 : 0;
    cls_forced[k_cls] |= bm.forced;
    bm.ftab_off = 3LL * (long long)frow;
    if (c->forced) {
      for (long long s = 0; s < k; ++s) {
        double F[3];
        force_at(c->spec, c->t + s, F);
        for (int d = 0; d < 3; ++d) b->h_ftab[3 * (frow + s) + d] = (float)F[d];
      }
      frow += (size_t)k;
    }
    // velocity / pressure / node-layer symmetry faces: after each of its
    // steps, at the level reached, the force and face pressures the
    // single-lattice step uses there
    bm.nee_nodes = c->nee_nodes;
    bm.nee_count = c->nee_count;
    bm.nee_begin = cls_nee[k_cls];
    bm.ntab_off = 9LL * (long long)nrow;
    bm.e = c->e32;
    if (c->nee_count > 0) {
      cls_nee[k_cls] += c->nee_count;
      for (long long s = 0; s < k; ++s) {
        const long long lev = c->t + s + 1;
        double F[3];
        force_at(c->spec, lev, F);
        float* row = b->h_ntab + 9 * (nrow + s);
        for (int d = 0; d < 3; ++d) row[d] = (float)F[d];
        for (int f = 0; f < 6; ++f) {
          double pf = c->spec.face_p[f];
          if (c->spec.FT > 0.0)
            pf += c->spec.face_pA[f] * std::cos(2.0 * M_PI * (double)lev / c->spec.FT);
          row[3 + f] = (float)pf;
        }
      }
      nrow += (size_t)k;
    }
  }
  for (int k = 0; k < NG; ++k)
    if (cls_tiles[k] >= (1LL << 30)) return bfail(b, LBM_EINVAL, "too many tiles in one batch");
  if (chunk != nchunks) return bfail(b, LBM_EINVAL, "internal: chunk count mismatch");
  BHIP(b, hipMemcpyAsync(b->d_members, b->h_members, nm * sizeof(BatchMember),
                         hipMemcpyHostToDevice, b->stream));
  if (nchunks)
    BHIP(b, hipMemcpyAsync(b->d_chunks, b->h_chunks, nchunks * sizeof(BatchChunk),
                           hipMemcpyHostToDevice, b->stream));
  if (frow)
    BHIP(b, hipMemcpyAsync(b->d_ftab, b->h_ftab, 3 * frow * sizeof(float), hipMemcpyHostToDevice,
                           b->stream));
  if (nrow)
    BHIP(b, hipMemcpyAsync(b->d_ntab, b->h_ntab, 9 * nrow * sizeof(float), hipMemcpyHostToDevice,
                           b->stream));
  BHIP(b, hipEventRecord(b->staged, b->stream));
  // the same tile order rule as single lattices, on the populations of all
  // active members (the class launches of a step follow each other)
  size_t act_bytes = 0;
  for (int j = 0; j < nm; ++j) act_bytes += step_bytes(*b->members[act[j]].ctx);
  const int xcd = order_for(act_bytes, true);
  nmax = 0;
  for (int k = 0; k < NG; ++k) nmax = std::max(nmax, cls_steps[k]);
  for (long long s = 0; s < std::max(nmax, solo_max); ++s) {
    for (int k = 0; k < NG; ++k) {
      if (cls_cnt[k] == 0 || s >= cls_steps[k]) continue;
      const int odd = (int)(((align ? parity : k / 6) + s) & 1);
      BatchLaunch L;
      L.members = b->d_members + cls_off[k];
      L.nmembers = cls_cnt[k];
      L.chunks = cls_big[k] ? b->d_chunks + cls_chunk_off[k] : nullptr;
      L.nblocks = cls_big[k] ? cls_chunks[k] : cls_tiles[k];
      L.ftab = b->d_ftab;
      L.substep = (int)s;
      L.xcd_order = xcd;
      BHIP(b, launch_batch_group(cls_q(k), (k & 1) ? ST_F16 : ST_F32,
                                 odd ? MODE_AA_ODD : MODE_AA_EVEN, cls_forced[k] != 0, L,
                                 b->stream));
      if (cls_nee[k] > 0)
        BHIP(b, launch_batch_nee(cls_q(k), (k & 1) ? ST_F16 : ST_F32, odd ? 0 : 1,
                                 b->d_members + cls_off[k], cls_cnt[k], b->d_ntab, (int)s,
                                 cls_nee[k], b->stream));
    }
    const int rc = solo_substep(s);
    if (rc) return rc;
  }
  solo_done();
  for (int j = 0; j < nm; ++j) {
    Member& m = b->members[act[j]];
    const long long k = std::min(n - ((align && m.ctx->phase != parity) ? 1 : 0), m.remaining);
    m.ctx->t += k;
    m.ctx->phase = (int)((m.ctx->phase + k) & 1);
    m.remaining -= k;
  }
  return LBM_OK;
}

int lbm_batch_monitor(lbm_batch* b) {
  if (!b) return LBM_EINVAL;
  // members created with monitor_every > 0 (their footprint holds the
  // monitor scratch)
  std::vector<lbm_ctx*> mons;
  for (auto& m : b->members)
    if (m.ctx->spec.monitor_every > 0) mons.push_back(m.ctx);
  const int nm = (int)mons.size();
  if (nm == 0) return LBM_OK;
  for (lbm_ctx* c : mons) {
    int rc = ensure_monitor(c);
    if (rc) return bfail(b, rc, c->err);
  }
  // layout of the staging block: members | snaps | pofs | bbeg | pcount |
  // phases | partials | out
  std::vector<BatchMember> hm(nm);
  std::vector<void*> snaps(nm);
  std::vector<long long> pofs(nm), bbeg(nm), pcount(nm);
  std::vector<int> phases(nm);
  long long blocks = 0;
  for (int j = 0; j < nm; ++j) {
    lbm_ctx* c = mons[j];
    std::memset(&hm[j], 0, sizeof(BatchMember));
    fill_args<float>(*c, hm[j].a);
    double F[3];
    force_at(c->spec, c->t, F);
    for (int d = 0; d < 3; ++d) hm[j].a.F[d] = (float)F[d];
    hm[j].q = c->q;
    hm[j].storage = c->spec.storage == LBM_F32 ? ST_F32 : ST_F16;
    snaps[j] = c->snap;
    long long nb = ((long long)c->N + 255) / 256;
    nb = std::max(1LL, std::min(nb, 256LL));
    bbeg[j] = blocks;
    pofs[j] = blocks;
    pcount[j] = nb;
    phases[j] = c->phase;
    blocks += nb;
  }
  size_t off = 0;
  auto place = [&](size_t bytes) {
    size_t o = align_up(off);
    off = o + bytes;
    return o;
  };
  const size_t o_m = place(nm * sizeof(BatchMember));
  const size_t o_s = place(nm * sizeof(void*));
  const size_t o_p = place(nm * sizeof(long long));
  const size_t o_b = place(nm * sizeof(long long));
  const size_t o_c = place(nm * sizeof(long long));
  const size_t o_h = place(nm * sizeof(int));
  const size_t o_part = place(3 * blocks * sizeof(double));
  const size_t o_out = place(3 * nm * sizeof(double));
  int rc = grow_dev(b, b->d_mon, b->d_mon_cap, off);
  if (rc) return rc;
  char* d = b->d_mon;
  BHIP(b, hipMemcpyAsync(d + o_m, hm.data(), nm * sizeof(BatchMember), hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipMemcpyAsync(d + o_s, snaps.data(), nm * sizeof(void*), hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipMemcpyAsync(d + o_p, pofs.data(), nm * sizeof(long long), hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipMemcpyAsync(d + o_b, bbeg.data(), nm * sizeof(long long), hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipMemcpyAsync(d + o_c, pcount.data(), nm * sizeof(long long), hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipMemcpyAsync(d + o_h, phases.data(), nm * sizeof(int), hipMemcpyHostToDevice, b->stream));
  BHIP(b, launch_batch_monitor((const BatchMember*)(d + o_m), nm, (void* const*)(d + o_s),
                               (double*)(d + o_part), (const long long*)(d + o_p), blocks,
                               (const long long*)(d + o_b), (const int*)(d + o_h), b->stream));
  BHIP(b, launch_batch_reduce((const double*)(d + o_part), (const long long*)(d + o_p),
                              (const long long*)(d + o_c), nm, (double*)(d + o_out), b->stream));
  std::vector<double> res(3 * nm);
  BHIP(b, hipMemcpyAsync(res.data(), d + o_out, 3 * nm * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  for (int j = 0; j < nm; ++j) {
    lbm_ctx* c = mons[j];
    (void)poll_monitor(c);  // earlier single runs, all done (stream synchronised)
    c->mon[0] = res[3 * j];
    c->mon[1] = res[3 * j + 1];
    c->mon[2] = res[3 * j + 2];
    const bool bad = !std::isfinite(c->mon[1]) || !std::isfinite(c->mon[2]) ||
                     (c->snap_valid && !std::isfinite(c->mon[0]));
    if (bad && !c->tripped) {
      c->tripped = true;
      c->trip_t = c->t;
    }
    c->mon_lag = c->snap_valid ? c->t - c->t_snap : 0;
    c->snap_valid = true;
    c->t_snap = c->t;
    c->mon_ran = true;
    c->mon_pending = false;
  }
  return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_OK;
  (void)hipStreamSynchronize(b->stream);
  for (auto& m : b->members) m.ctx->batch = nullptr;
  if (b->d_members) (void)hipFree(b->d_members);
  if (b->d_chunks) (void)hipFree(b->d_chunks);
  if (b->d_ftab) (void)hipFree(b->d_ftab);
  if (b->d_ntab) (void)hipFree(b->d_ntab);
  if (b->d_mon) (void)hipFree(b->d_mon);
  if (b->h_members) (void)hipHostFree(b->h_members);
  if (b->h_chunks) (void)hipHostFree(b->h_chunks);
  if (b->h_ftab) (void)hipHostFree(b->h_ftab);
  if (b->h_ntab) (void)hipHostFree(b->h_ntab);
  if (b->staged) (void)hipEventDestroy(b->staged);
  delete b;
  return LBM_OK;
}

}  // extern "C"

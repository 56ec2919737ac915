// kernels.hip -- device code of the D3Q14 / D3Q18 / D3Q26 incompressible MRT
// lattice Boltzmann library for gfx950 (arXiv 1503.03337).
//
// Data layout: structure of arrays, population a of node n at
// f[a*stride + n], n = x + nx*(y + ny*z); one thread per node, a workgroup
// covers a tx x ty tile of one x-y plane (tx spans whole rows where it can,
// so a wavefront reads and writes 64 consecutive x).  Every population is
// read once and written once per step: the kernels are HBM-bound
// (2 q b bytes per node, b = bytes per stored value).
//
// One time step (Eq. (mrteq)): collide every node (lattice.hpp), then move
// each post-collision population to x + c_a; across a periodic face the
// destination wraps, across a wall face it returns to x as the opposite
// population minus 6 w_a (c_a . u_w) (half-way bounce-back, moving wall).
// Three memory patterns:
//   AB       read A[a][n]; push f*_a to B[a][n + c_a] (or B[abar][n])
//   AA even  read A[a][n]; write f*_a to A[abar][n] (purely local; minus
//            the wall term when x + c_a is a wall)
//   AA odd   read f_a = A[abar][n - c_a] (or A[a][n] when n - c_a is a
//            wall); push like AB but in place
// AA even + AA odd = two time steps on one copy; each node reads and
// writes exactly the same set of slots within a step, so the in-place
// update has no race.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "lattice.hpp"

namespace lbm {

// Launch helpers read hipGetLastError() after a launch; drop any error an
// earlier, unrelated runtime call left behind so only this launch counts.
static inline void clear_stale_error() { (void)hipGetLastError(); }

// ---- population memory access --------------------------------------------------
// Every population value is touched once per step.  The AB pattern reads a
// copy it never writes in the same step: its loads carry the non-temporal
// hint (measured +20 % on 128^3 D3Q18 FP32).  The AA pattern reads lines it
// writes back right after, where the hint costs ~20 %, so it loads
// normally.  LBM_NT_LOAD forces the hint on every load, LBM_NT_STORE on
// every store (both measured neutral or worse).
#ifndef LBM_NT_LOAD
#define LBM_NT_LOAD 0
#endif
#ifndef LBM_NT_STORE
#define LBM_NT_STORE 0
#endif
// Population pointers are always device global memory.  Saying so with the
// address space lets the compiler use global (not flat) loads and stores
// even when the pointer comes out of a descriptor in memory (the batched
// kernels), which keeps the scalar-load and vector-memory counters apart.
#define LBM_GLOBAL __attribute__((address_space(1)))
template <bool NT, typename S>
__device__ __forceinline__ S pop_load(const S* p) {
  const LBM_GLOBAL S* g = (const LBM_GLOBAL S*)p;
  if (NT || LBM_NT_LOAD) return __builtin_nontemporal_load(g);
  return *g;
}
template <typename S>
__device__ __forceinline__ void pop_store(S* p, S v) {
  LBM_GLOBAL S* g = (LBM_GLOBAL S*)p;
#if LBM_NT_STORE
  __builtin_nontemporal_store(v, g);
#else
  *g = v;
#endif
}

// ---- storage codecs --------------------------------------------------------
template <int ST> struct Codec;
// dec(v, base, 2^-s) and enc(v, base 2^s, 2^s); FP64 and FP32 store the
// value itself.
template <> struct Codec<ST_F64> {
  using S = double;
  using C = double;
  static __device__ __forceinline__ C dec(S v, C, C) { return v; }
  static __device__ __forceinline__ S enc(C v, C, C) { return v; }
};
template <> struct Codec<ST_F32> {
  using S = float;
  using C = float;
  static __device__ __forceinline__ C dec(S v, C, C) { return v; }
  static __device__ __forceinline__ S enc(C v, C, C) { return v; }
};
// FP16 deviation: stored h = fp16((f - base) 2^s).  Both directions are one
// fused multiply-add: h 2^-s and f 2^s are exact products (2^s is a power of
// two), so fma(h, 2^-s, base) rounds exactly like base + h 2^-s, and
// fma(f, 2^s, -base 2^s) exactly like (f - base) 2^s.  (The step kernels
// skip both: they compute on h itself, in deviation units; see step_dec.)
// enc rounds to nearest.  enc_sr rounds stochastically with gfx950's
// v_cvt_sr_f16_f32: the top 13 bits of the random word r are added below
// the 10 mantissa bits FP16 keeps, then the rest is truncated, so a value
// rounds up with probability equal to its distance from the lower FP16
// neighbour (unbiased).  Round-to-nearest applied to a nearly steady state
// rounds the same values the same way every step, and increments below
// half an FP16 ulp (a weak body force, a slow viscous correction) are lost
// every time; the stochastic form keeps them on average.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
template <> struct Codec<ST_F16> {
  using S = _Float16;
  using C = float;
  static __device__ __forceinline__ C dec(S v, C base, C inv_scale) {
    return __builtin_fmaf(static_cast<float>(v), inv_scale, base);
  }
  static __device__ __forceinline__ S enc(C v, C base_s, C scale) {
    return static_cast<_Float16>(__builtin_fmaf(v, scale, -base_s));
  }
  static __device__ __forceinline__ S enc_sr(C v, C base_s, C scale, unsigned r) {
    // the instruction keeps the upper half of its first operand; only the
    // lower half is stored, so r's own register serves (no extra move)
    const half2_t h = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(half2_t, r),
                                                      __builtin_fmaf(v, scale, -base_s), r, false);
    return h[0];
  }
};

// Counter-based random words for the FP16 dither: one hash of (node, time
// level) per node, then a Weyl sequence over the populations (marginally
// uniform top bits at one add each).  Deterministic, so a lattice gives the
// same bits alone or in a batch, in either memory pattern.
__device__ __forceinline__ unsigned node_hash(unsigned n, unsigned t) {
  unsigned x = (n * 0x9E3779B1u) ^ (t * 0x85EBCA77u + 0x165667B1u);
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ unsigned pop_bits(unsigned h, int a) {
  return h + 0x9E3779B9u * (unsigned)(a + 1);
}

// Encode a post-collision value: FP16 stochastically (SR) or to nearest,
// the other storages plainly.  SR is a template argument so that a kernel
// picks the rounding mode once per node, not once per population.
template <int Q, int ST, bool SR>
__device__ __forceinline__ typename Codec<ST>::S enc_step(const LatticeArgs<typename Codec<ST>::C>& A,
                                                          typename Codec<ST>::C v, int slot,
                                                          unsigned h, int a) {
  const typename Codec<ST>::C bs = A.base_s[wclass<Q>(slot)];
  if constexpr (ST == ST_F16 && SR) return Codec<ST>::enc_sr(v, bs, A.scale, pop_bits(h, a));
  return Codec<ST>::enc(v, bs, A.scale);
}
// The same with the mode read per value (code off the per-node hot path).
template <int Q, int ST>
__device__ __forceinline__ typename Codec<ST>::S enc_any(const LatticeArgs<typename Codec<ST>::C>& A,
                                                         typename Codec<ST>::C v, int slot,
                                                         unsigned h, int a) {
  return A.f16_sr ? enc_step<Q, ST, true>(A, v, slot, h, a)
                  : enc_step<Q, ST, false>(A, v, slot, h, a);
}

// Units of the step kernels.  FP16 lattices step in deviation units: the
// collision runs on g = (f - base) 2^s, the stored value itself (the
// deviation form of the collision is in lattice.hpp), so a stored value
// converts to g exactly and the post-collision g is rounded once to FP16,
// with no multiply-add on either side; the arithmetic works on the small
// deviations instead of on base + deviation.  Their wall terms are held in
// the same units (the host scales them by 2^s) and the body force is scaled
// here.  FP32 and FP64 lattices step on f itself.  Everything else (set,
// get, macros, monitors, the boundary pass) stays in f units.
template <int ST>
constexpr bool dev_units() {
  return ST == ST_F16;
}
template <int ST>
__device__ __forceinline__ typename Codec<ST>::C step_dec(typename Codec<ST>::S v) {
  return static_cast<typename Codec<ST>::C>(v);
}
template <int ST, bool SR>
__device__ __forceinline__ typename Codec<ST>::S step_enc(typename Codec<ST>::C v, unsigned h,
                                                          int a) {
  if constexpr (ST == ST_F16) {
    if constexpr (SR) {
      const unsigned r = pop_bits(h, a);
      return __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(half2_t, r), v, r, false)[0];
    } else {
      return static_cast<_Float16>(v);
    }
  } else {
    return v;
  }
}

// ---- neighbour offsets -----------------------------------------------------
// For each axis and direction (-1, +1): the linear-index delta of the
// neighbour (wrapped on periodic axes, 0 across a symmetry plane) and
// whether a wall or a symmetry plane is crossed.
struct Nbr {
  int ox[2], oy[2], oz[2];
  bool wx[2], wy[2], wz[2];
  bool sx[2], sy[2], sz[2];
};

__device__ __forceinline__ void axis_nbr(int c, int n, int per, bool sym_lo, bool sym_hi,
                                         int stride, int (&o)[2], bool (&w)[2], bool (&s)[2]) {
  const bool lo = (c == 0), hi = (c == n - 1);
  o[0] = lo ? (per ? (n - 1) * stride : 0) : -stride;
  o[1] = hi ? (per ? -(n - 1) * stride : 0) : stride;
  s[0] = lo && sym_lo;
  s[1] = hi && sym_hi;
  w[0] = lo && !per && !sym_lo;
  w[1] = hi && !per && !sym_hi;
}

// GEN = false: the caller guarantees 0 < y < ny-1 and 0 < z < nz-1 and that
// neither x face is a symmetry plane, so only x walls and wrap-around need
// handling (per lane); GEN = true handles every axis and face kind.
template <bool GEN, typename C>
__device__ __forceinline__ Nbr make_nbr(const LatticeArgs<C>& A, int x, int y, int z) {
  Nbr b;
  if (GEN) {
    axis_nbr(x, A.nx, A.per_x, A.sym & 1, A.sym & 2, 1, b.ox, b.wx, b.sx);
    axis_nbr(y, A.ny, A.per_y, A.sym & 4, A.sym & 8, A.nx, b.oy, b.wy, b.sy);
    axis_nbr(z, A.nz, A.per_z, A.sym & 16, A.sym & 32, A.nx * A.ny, b.oz, b.wz, b.sz);
  } else {
    axis_nbr(x, A.nx, A.per_x, false, false, 1, b.ox, b.wx, b.sx);
    b.oy[0] = -A.nx;
    b.oy[1] = A.nx;
    b.oz[0] = -A.nx * A.ny;
    b.oz[1] = A.nx * A.ny;
    b.wy[0] = b.wy[1] = b.wz[0] = b.wz[1] = false;
    b.sy[0] = b.sy[1] = b.sz[0] = b.sz[1] = false;
  }
  return b;
}

// Link of population `a` from this node along its velocity (cx,cy,cz):
// offset of the node it lands on, wall flag, the wall term of the crossed
// wall face (z face first, then y, then x) and the slot it lands in (a, or
// its mirror image when symmetry planes are crossed and no wall is).
template <int Q, typename C>
__device__ __forceinline__ void link(const Nbr& b, const LatticeArgs<C>& A, int a, int cx, int cy,
                                     int cz, int& off, bool& wall, C& term, int& slot) {
  off = 0;
  wall = false;
  term = C(0);
  bool fx = false, fy = false, fz = false;
  if (cx) {
    const int k = cx > 0;
    off += b.ox[k];
    fx = b.sx[k];
    if (b.wx[k]) {
      wall = true;
      term = A.bb[a][0];
    }
  }
  if (cy) {
    const int k = cy > 0;
    off += b.oy[k];
    fy = b.sy[k];
    if (b.wy[k]) {
      wall = true;
      term = A.bb[a][1];
    }
  }
  if (cz) {
    const int k = cz > 0;
    off += b.oz[k];
    fz = b.sz[k];
    if (b.wz[k]) {
      wall = true;
      term = A.bb[a][2];
    }
  }
  const int lo = fy ? (fx ? mirror<Q>(a, 3) : mirror<Q>(a, 2)) : (fx ? mirror<Q>(a, 1) : a);
  const int hi = fy ? (fx ? mirror<Q>(a, 7) : mirror<Q>(a, 6))
                    : (fx ? mirror<Q>(a, 5) : mirror<Q>(a, 4));
  slot = fz ? hi : lo;
}

// ---- population addresses ---------------------------------------------------
// Byte address of a stored value: the node's own address p0 = buf + n b
// (one per lane and node), plus the neighbour offset times b, plus the
// population array's offset pofs[slot] (a kernel argument: uniform, no
// multiply in the kernel).  On the inner path (GEN = false: y and z interior,
// no symmetry planes) only the x part of the neighbour offset varies across
// lanes, so each node forms p0 and its two x-shifted copies once and every
// population's address is one 64-bit add of a uniform offset.  The general
// path also handles mirror slots across symmetry planes (slot chosen per
// lane), with slot * pbytes.
template <typename S>
__device__ __forceinline__ const char* lane_ptr(const void* buf, unsigned n) {
  return static_cast<const char*>(buf) + (unsigned long long)n * sizeof(S);
}

// Address of slot `slot` at node n + off on either path (link() semantics:
// off, slot for population a moving along (cx, cy, cz)); px[k] = p0 + the
// x offset of direction k (inner path only).
template <typename S, bool GEN, typename C>
__device__ __forceinline__ const char* link_ptr(const LatticeArgs<C>& A, const Nbr& b,
                                                const char* p0, const char* const (&px)[2],
                                                int cx, int cy, int cz, int off, int slot,
                                                int slot_inner) {
  if constexpr (GEN) {
    return p0 + (long long)off * (long long)sizeof(S) + (long long)slot * A.pbytes;
  } else {
    // slot == slot_inner here (no symmetry planes on the inner path)
    long long u = A.pofs[slot_inner];
    if (cy) u += (long long)b.oy[cy > 0] * (long long)sizeof(S);
    if (cz) u += (long long)b.oz[cz > 0] * (long long)sizeof(S);
    return (cx ? px[cx > 0] : p0) + u;
  }
}

// ---- 32-bit offsets (odd AA step, inner path) ------------------------------
// When the whole population buffer spans less than 4 GiB (O32), the odd AA
// step of the inner path can address it through a buffer resource: byte
// offset = a 32-bit lane offset (vector register) + a 32-bit uniform offset
// (scalar register).  Populations with c_x = 0 sit at a uniform distance
// (pofs plus the y / z row offsets) from a lane offset the whole node
// shares, so their addresses cost no vector instruction at all.  The
// x-moving populations put the whole offset in the lane part:
//   off = (n + o_x) b + U + (m & (W - U))
// with U the uniform part, W the offset of the wall slot at this node and
// m all-ones on the one lane of a row that sits on an x wall (0 elsewhere),
// in modular 32-bit arithmetic whose true value is the offset itself (below
// 2^32): two or three 32-bit vector instructions instead of two 64-bit adds
// and a 64-bit select.  Both register parts are kept non-negative: the
// uniform part of a c_x = 0 link is shifted up by K = (nx ny + nx) b and the
// lane part down by K, which the inner path (y, z >= 1) allows.  The
// gather of f_a and the push of f*_abar touch the same value (the AA
// property), so the push reuses the gather's offsets.  The resource spans
// exactly the population buffer, and every offset formed here lies inside
// it.
using rsrc_t = __amdgpu_buffer_rsrc_t;
template <int Q, typename C>
__device__ __forceinline__ rsrc_t pop_rsrc(const LatticeArgs<C>& A, const void* buf) {
  const long long bytes = A.pofs[Q - 1] + A.pbytes;  // below 2^32 under O32
  // dword 3: 32-bit data format (a raw untyped view for gfx9-family parts)
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(buf), 0, (int)(unsigned)bytes,
                                           0x00020000);
}
template <typename S> struct BufIO;
template <> struct BufIO<double> {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ double load(rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
  }
  static __device__ __forceinline__ void store(double x, rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, v, s, 0);
  }
};
template <> struct BufIO<float> {
  static __device__ __forceinline__ float load(rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  }
  static __device__ __forceinline__ void store(float x, rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, 0);
  }
};
template <> struct BufIO<_Float16> {
  static __device__ __forceinline__ _Float16 load(rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
  }
  static __device__ __forceinline__ void store(_Float16 x, rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, 0);
  }
};

// Lane parts of the inner path: n b, n b - K, (n + o_x[k]) b, and the wall
// masks of the two x directions; K the shift of the uniform parts.
struct Off32 {
  unsigned v0, vs, k, vx[2], wm[2];
};
template <typename S, typename C>
__device__ __forceinline__ Off32 make_off32(const LatticeArgs<C>& A, const Nbr& b, unsigned n) {
  Off32 o;
  const unsigned sz = (unsigned)sizeof(S);
  o.k = ((unsigned)A.nx * (unsigned)A.ny + (unsigned)A.nx) * sz;
  o.v0 = n * sz;
  o.vs = o.v0 - o.k;
  o.vx[0] = (n + (unsigned)b.ox[0]) * sz;
  o.vx[1] = (n + (unsigned)b.ox[1]) * sz;
  o.wm[0] = b.wx[0] ? ~0u : 0u;
  o.wm[1] = b.wx[1] ? ~0u : 0u;
  // hide that the masks are 0 / all-ones: otherwise m & (W - U) + U becomes
  // a select between two scalar values, which costs two moves more per use
  // (one scalar operand per vector instruction)
  asm volatile("" : "+v"(o.wm[0]), "+v"(o.wm[1]));
  return o;
}

// Lane and uniform offsets of the value the odd step gathers as f_a on the
// inner path: slot abar at x - c_a, or slot a of this node when x - c_a lies
// beyond an x wall.
template <int Q, typename S, typename C>
__device__ __forceinline__ void gather_off32(const LatticeArgs<C>& A, const Nbr& b, const Off32& o,
                                             int a, unsigned& vo, unsigned& so) {
  using L = Lattice<Q>;
  const int cx = -L::cx[a], cy = -L::cy[a], cz = -L::cz[a];  // towards x - c_a
  long long u = A.pofs[L::opp[a]];
  if (cy) u += (long long)b.oy[cy > 0] * (long long)sizeof(S);
  if (cz) u += (long long)b.oz[cz > 0] * (long long)sizeof(S);
  if (cx == 0) {
    vo = o.vs;
    so = (unsigned)u + o.k;
  } else {
    const int k = cx > 0;
    const unsigned u32 = (unsigned)u, d = (unsigned)A.pofs[a] - u32;
    vo = o.vx[k] + u32 + (o.wm[k] & d);
    so = 0u;
  }
}

// AA odd step on the inner path through the buffer resource.  The gather
// of population a (slot abar at x - c_a, or slot a here across an x wall)
// and the push of population abar (slot abar at x + c_abar = x - c_a, or
// slot a here across that wall) touch the same value, so the push reuses
// the gather's offsets: vo / so[a] is where f_a came from.
template <int Q, int ST>
__device__ __forceinline__ void read_odd32(const LatticeArgs<typename Codec<ST>::C>& A, unsigned n,
                                           int x, int y, int z, typename Codec<ST>::C (&f)[Q],
                                           unsigned (&vo)[Q], unsigned (&so)[Q]) {
  using CD = Codec<ST>;
  using S = typename CD::S;
  const rsrc_t r = pop_rsrc<Q>(A, A.f);
  const Nbr b = make_nbr<false>(A, x, y, z);
  const Off32 o = make_off32<S>(A, b, n);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    gather_off32<Q, S>(A, b, o, a, vo[a], so[a]);
    f[a] = step_dec<ST>(BufIO<S>::load(r, vo[a], so[a]));
  }
}

// Value population a leaves an inner-path node with: f_a - m bb_a, m = 1 on
// the lane whose x + c_a is a wall and 0 elsewhere (only an x face can be a
// wall there): one fused multiply-add with a per-lane 0/1 factor instead of
// a select and a subtraction per population.  m bb is exact, so the result
// rounds like f_a - bb_a and equals f_a for m = 0 (a zero f_a may come out
// with the other sign: the same value, so every later operation gives the
// same result).
template <int Q, typename C>
__device__ __forceinline__ C leave_inner(const LatticeArgs<C>& A, const C (&mx)[2],
                                         const C (&f)[Q], int a) {
  using L = Lattice<Q>;
  if (L::cx[a] == 0) return f[a];
  return fma2(-mx[L::cx[a] > 0], A.bb[a][0], f[a]);
}

template <int Q, int ST, bool SR>
__device__ __forceinline__ void write_odd32(const LatticeArgs<typename Codec<ST>::C>& A, unsigned n,
                                            int x, int y, int z,
                                            const typename Codec<ST>::C (&f)[Q],
                                            const unsigned (&vo)[Q], const unsigned (&so)[Q]) {
  using CD = Codec<ST>;
  using C = typename CD::C;
  using S = typename CD::S;
  using L = Lattice<Q>;
  const unsigned h = (ST == ST_F16) ? node_hash(n, A.tstep) : 0u;
  const Nbr b = make_nbr<false>(A, x, y, z);
  const C mx[2] = {b.wx[0] ? C(1) : C(0), b.wx[1] ? C(1) : C(0)};
  const rsrc_t r = pop_rsrc<Q>(A, A.f);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int o = L::opp[a];
    BufIO<S>::store(step_enc<ST, SR>(leave_inner<Q>(A, mx, f, a), h, a), r, vo[o], so[o]);
  }
}

// ---- reading the populations of node n ------------------------------------
// PHASE 0: natural layout (AB, AA even).  PHASE 1: AA swapped layout after
// an even step: f_a(x) = A[abar][x - c_a], or, when x - c_a is a wall,
// A[a][x], where the even step already stored the bounced-back value
// f*_abar(x) - 6 w_abar (c_abar . u_w).  When x - c_a lies beyond symmetry
// planes only, the source node keeps x's coordinates along their normals and
// the slot is the mirror image of abar.
// STEP: the values come out in the step kernels' units (dev_units).
template <int Q, int ST, int PHASE, bool GEN, bool NT = false, bool STEP = false>
__device__ __forceinline__ void read_node(const LatticeArgs<typename Codec<ST>::C>& A,
                                          const typename Codec<ST>::S* src, unsigned n, int x,
                                          int y, int z, typename Codec<ST>::C (&f)[Q]) {
  using CD = Codec<ST>;
  using C = typename CD::C;
  using S = typename CD::S;
  using L = Lattice<Q>;
  const char* p0 = lane_ptr<S>(src, n);
  if (PHASE == 0) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const S v = pop_load<NT>((const S*)(p0 + A.pofs[a]));
      f[a] = STEP ? step_dec<ST>(v) : CD::dec(v, A.base[wclass<Q>(a)], A.inv_scale);
    }
  } else {
    const Nbr b = make_nbr<GEN>(A, x, y, z);
    // x - c_a: direction k = (-cx > 0) of the link taken from this node
    const char* const px[2] = {p0 + (long long)b.ox[0] * (long long)sizeof(S),
                               p0 + (long long)b.ox[1] * (long long)sizeof(S)};
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const int o = L::opp[a];
      int off, slot;
      bool wall;
      C term;
      link<Q, C>(b, A, o, -L::cx[a], -L::cy[a], -L::cz[a], off, wall, term, slot);
      const char* nb = link_ptr<S, GEN>(A, b, p0, px, -L::cx[a], -L::cy[a], -L::cz[a], off,
                                        slot, o);
      const char* p = wall ? p0 + A.pofs[a] : nb;
      const S v = pop_load<NT>((const S*)p);
      f[a] = STEP ? step_dec<ST>(v) : CD::dec(v, A.base[wclass<Q>(a)], A.inv_scale);
    }
  }
}

// ---- writing post-collision populations -----------------------------------
// MODE_AA_EVEN: f*_a into slot abar of the same node, minus the wall term
// when x + c_a is a wall (so the value stored is the bounced-back
// population, rounded once, as in the push patterns).  Otherwise push to
// x + c_a (or bounce back into slot abar of this node across a wall, or,
// across symmetry planes only, into the mirror slot of the node reached by
// moving along the planes).  The wall term is +0 off walls and f - (+0) is
// f bit for bit, so every store is f_a - term at a selected address (no
// branch); a slot and its mirror image or opposite share a's weight, hence
// its FP16 base.
template <int Q, int ST, int MODE, bool GEN, bool SR>
__device__ __forceinline__ void write_node(const LatticeArgs<typename Codec<ST>::C>& A,
                                           typename Codec<ST>::S* dst, unsigned n, int x, int y,
                                           int z, const typename Codec<ST>::C (&f)[Q]) {
  using CD = Codec<ST>;
  using C = typename CD::C;
  using S = typename CD::S;
  using L = Lattice<Q>;
  // dither bits of the value population a leaves this node with at level t
  const unsigned h = (ST == ST_F16) ? node_hash(n, A.tstep) : 0u;
  char* p0 = const_cast<char*>(lane_ptr<S>(dst, n));
  const Nbr b = make_nbr<GEN>(A, x, y, z);
  if (MODE == MODE_AA_EVEN) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const int o = L::opp[a];
      int off, slot;
      bool wall;
      C term;
      link<Q, C>(b, A, a, L::cx[a], L::cy[a], L::cz[a], off, wall, term, slot);
      pop_store((S*)(p0 + A.pofs[o]), step_enc<ST, SR>(f[a] - term, h, a));
    }
  } else {
    const char* const px[2] = {p0 + (long long)b.ox[0] * (long long)sizeof(S),
                               p0 + (long long)b.ox[1] * (long long)sizeof(S)};
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const int o = L::opp[a];
      int off, slot;
      bool wall;
      C term;
      link<Q, C>(b, A, a, L::cx[a], L::cy[a], L::cz[a], off, wall, term, slot);
      const char* nb = link_ptr<S, GEN>(A, b, p0, px, L::cx[a], L::cy[a], L::cz[a], off, slot, a);
      char* p = const_cast<char*>(wall ? p0 + A.pofs[o] : nb);
      pop_store((S*)p, step_enc<ST, SR>(f[a] - term, h, a));
    }
  }
}

// ---- one node, one step ------------------------------------------------------
// The collision in the step kernels' units: MRT, or LBGK when BGK; in
// deviation units the body force takes the factor 2^s and products take
// 2^-s (lattice.hpp).
template <int Q, int ST, bool FORCED, bool BGK>
__device__ __forceinline__ void collide_step(const LatticeArgs<typename Codec<ST>::C>& A,
                                             typename Codec<ST>::C (&f)[Q]) {
  using C = typename Codec<ST>::C;
  constexpr bool DEV = dev_units<ST>();
  C F[3] = {A.F[0], A.F[1], A.F[2]};
  if constexpr (DEV && FORCED) {
    F[0] *= A.scale;
    F[1] *= A.scale;
    F[2] *= A.scale;
  }
  if constexpr (BGK) {
    collide_bgk<Q, C, FORCED, DEV>(f, A.omega, A.hom, F, A.inv_scale);
  } else {
    Relax<C> r;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      r.sN[k] = A.sN[k];
      r.hN[k] = A.hN[k];
    }
    collide<Q, C, FORCED, DEV>(f, r, F, A.inv_scale);
  }
}

// RECOMP (general path): the push forms its addresses anew instead of
// keeping the gather's 64-bit addresses live through the collision; the
// coordinates pass through an empty asm statement, so the compiler cannot
// reuse the gather's address arithmetic.
template <int Q, int ST, int MODE, bool FORCED, bool GEN, bool BGK = false, bool RECOMP = false>
__device__ __forceinline__ void node_step(const LatticeArgs<typename Codec<ST>::C>& A, int x, int y,
                                          int z) {
  using CD = Codec<ST>;
  using C = typename CD::C;
  using S = typename CD::S;
  const unsigned n = (unsigned)x + (unsigned)A.nx * ((unsigned)y + (unsigned)A.ny * (unsigned)z);
  C f[Q];
  if (MODE == MODE_AB) {
    read_node<Q, ST, 0, GEN, true, true>(A, static_cast<const S*>(A.f), n, x, y, z, f);
  } else if (MODE == MODE_AA_EVEN) {
    read_node<Q, ST, 0, GEN, false, true>(A, static_cast<const S*>(A.f), n, x, y, z, f);
  } else {
    read_node<Q, ST, 1, GEN, false, true>(A, static_cast<const S*>(A.f), n, x, y, z, f);
  }
  collide_step<Q, ST, FORCED, BGK>(A, f);
  S* dst = static_cast<S*>(MODE == MODE_AB ? A.g : A.f);
  unsigned nw = n;
  if constexpr (RECOMP) asm volatile("" : "+v"(nw), "+v"(x), "+v"(y), "+v"(z));
  if (ST == ST_F16 && A.f16_sr)
    write_node<Q, ST, MODE, GEN, true>(A, dst, nw, x, y, z, f);
  else
    write_node<Q, ST, MODE, GEN, false>(A, dst, nw, x, y, z, f);
}

// The odd AA step of an inner-path node with 32-bit buffer offsets (the
// same arithmetic as node_step; only the addressing differs).
template <int Q, int ST, bool FORCED, bool BGK>
__device__ __forceinline__ void node_step_odd32(const LatticeArgs<typename Codec<ST>::C>& A, int x,
                                                int y, int z) {
  using C = typename Codec<ST>::C;
  const unsigned n = (unsigned)x + (unsigned)A.nx * ((unsigned)y + (unsigned)A.ny * (unsigned)z);
  C f[Q];
  unsigned vo[Q], so[Q];  // where each f_a was read
  read_odd32<Q, ST>(A, n, x, y, z, f, vo, so);
  collide_step<Q, ST, FORCED, BGK>(A, f);
  if (ST == ST_F16 && A.f16_sr)
    write_odd32<Q, ST, true>(A, n, x, y, z, f, vo, so);
  else
    write_odd32<Q, ST, false>(A, n, x, y, z, f, vo, so);
}

// Dispatch on whether this node's wavefront may touch a y or z boundary
// (uniform for a wavefront inside one x-row); lattices with a symmetry plane
// on an x face take the general path everywhere.
template <int Q, int ST, int MODE, bool FORCED, bool BGK = false, bool O32 = false>
__device__ __forceinline__ void node_step_any(const LatticeArgs<typename Codec<ST>::C>& A, int x,
                                              int y, int z) {
  const bool inner =
      (y > 0) & (y < A.ny - 1) & (z > 0) & (z < A.nz - 1) & ((A.sym & 3) == 0);
  if (inner) {
    if constexpr (O32 && MODE == MODE_AA_ODD)
      node_step_odd32<Q, ST, FORCED, BGK>(A, x, y, z);
    else
      node_step<Q, ST, MODE, FORCED, false, BGK>(A, x, y, z);
  } else {
    node_step<Q, ST, MODE, FORCED, true, BGK>(A, x, y, z);
  }
}

// Work item of this workgroup in an XCD-aware order.  Workgroups are
// dispatched to the 8 XCDs in turn (w to XCD w % 8).  xcd_contiguous hands
// XCD k the k-th contiguous range of [0, gridDim.x) (the first
// gridDim.x % 8 XCDs take one item more); xcd_block(c), c >= 2, hands the
// XCDs chunks of 2^(c-1) consecutive items in turn (items past the last
// whole round of 8 chunks keep w), and c = 1 is xcd_contiguous.  Each is a
// bijection on [0, gridDim.x), so neighbouring rows, whose lines the odd AA
// step shares, run in one L2 without changing what any item computes.  The
// single-lattice step does not call xcd_block: its general chunk branch made
// the compiler spill scalar registers there and cost 1.4 % at 128^3.  It
// uses xcd_contiguous, or chunks of 4 written as a bit permutation.
__device__ __forceinline__ unsigned xcd_contiguous() {
  const unsigned G = gridDim.x, q8 = G >> 3, r8 = G & 7u, xc = blockIdx.x & 7u,
                 i = blockIdx.x >> 3;
  return xc < r8 ? xc * (q8 + 1u) + i : r8 * (q8 + 1u) + (xc - r8) * q8 + i;
}

__device__ __forceinline__ unsigned xcd_block(int order) {
  if (order == 1) return xcd_contiguous();
  const unsigned G = gridDim.x, w = blockIdx.x, xc = w & 7u, i = w >> 3;
  const unsigned sh = (unsigned)order - 1u, whole = (G >> (sh + 3u)) << (sh + 3u);
  if (w >= whole) return w;
  return ((i >> sh) << (sh + 3u)) + (xc << sh) + (i & ((1u << sh) - 1u));
}

// The kernel's own arguments re-read from the kernel-argument segment
// behind an empty asm statement: scalar loads at the point of use that the
// compiler cannot hoist into the kernel's entry.  (A kernel with one
// by-value argument finds it at offset 0 of the segment.)
template <typename C>
__device__ __forceinline__ const LatticeArgs<C>& reread_args() {
  typedef const __attribute__((address_space(4))) LatticeArgs<C>* kp_t;
  kp_t p = (kp_t)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return *(const LatticeArgs<C>*)p;
}

// Register budget of the odd AA step.  Its general path (y / z faces,
// symmetry planes) holds every wall term and population offset and, left
// to itself, sets the registers of the whole kernel: the compiler loads
// all arguments at the kernel's entry, spills scalar registers into
// vector-register lanes (reloaded on the inner path too) and keeps the
// gather's 64-bit addresses live through the collision.  A lean general
// path re-reads the arguments where it uses them and forms the push
// addresses anew (RECOMP); the inner path then runs without reloads and
// with fewer vector registers (the D3Q18 FP16 odd step: 62 instead of
// 102, 7 waves per SIMD instead of 4), giving the same bits.  Measured per
// kernel at 128^3 / 256^3: D3Q18 FP16 odd step -4.6 % / -8.4 %, D3Q14 FP16
// -6 % / -7 %; at 128^3 D3Q26 FP16 -19 %, D3Q18 FP64 -2.3 %.  The FP32 odd
// steps lost 1.4-2.8 % with it (6 waves per SIMD instead of 4: more than
// HBM streaming wants there) and keep the plain general path, as do the
// even steps, which moved by -0.8 % to +1.5 %.
template <int Q, int ST, int MODE>
constexpr bool lean_general() {
  return MODE == MODE_AA_ODD && ST != ST_F32;
}

template <int Q, int ST, int MODE, bool FORCED, bool BGK = false, bool O32 = false>
__global__ __launch_bounds__(256) void k_step(LatticeArgs<typename Codec<ST>::C> A) {
  unsigned b = blockIdx.x;
  if (A.xcd_order == 1) {
    b = xcd_contiguous();
  } else if (A.xcd_order == 2 && b < (gridDim.x & ~31u)) {
    // chunks of 4 tiles per XCD in turn (xcd_block(3)): within each run of
    // 32 workgroups, a permutation of the low five bits
    b = (b & ~31u) | ((b & 7u) << 2) | ((b >> 3) & 3u);
  }
  const unsigned r = fast_div(b, A.fd_tiles_x);
  const int bx = (int)(b - r * (unsigned)A.tiles_x);
  const unsigned zz = fast_div(r, A.fd_tiles_y);
  const int by = (int)(r - zz * (unsigned)A.tiles_y);
  const int z = (int)zz;
  const int x = bx * A.tx + (int)threadIdx.x;
  const int y = by * A.ty + (int)threadIdx.y;
  if (x >= A.nx || y >= A.ny) return;
  if constexpr (lean_general<Q, ST, MODE>()) {
    const bool inner =
        (y > 0) & (y < A.ny - 1) & (z > 0) & (z < A.nz - 1) & ((A.sym & 3) == 0);
    if (inner) {
      if constexpr (O32)
        node_step_odd32<Q, ST, FORCED, BGK>(A, x, y, z);
      else
        node_step<Q, ST, MODE, FORCED, false, BGK>(A, x, y, z);
    } else {
      node_step<Q, ST, MODE, FORCED, true, BGK, true>(reread_args<typename Codec<ST>::C>(), x, y,
                                                      z);
    }
  } else {
    node_step_any<Q, ST, MODE, FORCED, BGK, O32>(A, x, y, z);
  }
}

// The odd AA step of the kernels whose vector instructions rival their
// memory traffic (FP16 storage: half the bytes per node for the same
// arithmetic; the 26-velocity model: the largest collision) takes the
// buffer-resource addressing when the population buffer spans less than
// 4 GiB.  Measured per kernel at 128^3 and 256^3: FP16 D3Q18 odd step
// -3.8 % / -3.0 %, D3Q14 FP16 -6 %, D3Q26 FP32 -2.9 %; the FP32 D3Q14 /
// D3Q18 and FP64 odd steps, bound by memory alone, were within +-1 % either
// way and keep the 64-bit addresses, as does every even step (its
// 32-bit-offset form needs fewer registers, runs more waves per SIMD and
// was 0.5-4 % slower).
template <int Q, int ST, int MODE>
constexpr bool odd32_kernel() {
  return MODE == MODE_AA_ODD && (ST == ST_F16 || Q == 26);
}
template <int Q, typename C>
static bool fits_o32(const LatticeArgs<C>& A) {
  return A.pofs[Q - 1] + A.pbytes <= 0xffffffffLL;
}

template <int Q, int ST, int MODE, bool FORCED, bool BGK>
static hipError_t step_launch(const void* args, hipStream_t s) {
  clear_stale_error();
  using C = typename Codec<ST>::C;
  const LatticeArgs<C>& A = *static_cast<const LatticeArgs<C>*>(args);
  const long long blocks = (long long)A.tiles_x * A.tiles_y * A.nz;
  dim3 block(A.tx, A.ty, 1);
  if (odd32_kernel<Q, ST, MODE>() && fits_o32<Q>(A))
    hipLaunchKernelGGL((k_step<Q, ST, MODE, FORCED, BGK, odd32_kernel<Q, ST, MODE>()>),
                       dim3((unsigned)blocks), block, 0, s, A);
  else
    hipLaunchKernelGGL((k_step<Q, ST, MODE, FORCED, BGK>), dim3((unsigned)blocks), block, 0, s, A);
  return hipGetLastError();
}

template <int Q, int ST, bool BGK = false>
static hipError_t step_q_st(int mode, bool forced, const void* args, hipStream_t s) {
  clear_stale_error();
  switch (mode) {
    case MODE_AB:
      return forced ? step_launch<Q, ST, MODE_AB, true, BGK>(args, s)
                    : step_launch<Q, ST, MODE_AB, false, BGK>(args, s);
    case MODE_AA_EVEN:
      return forced ? step_launch<Q, ST, MODE_AA_EVEN, true, BGK>(args, s)
                    : step_launch<Q, ST, MODE_AA_EVEN, false, BGK>(args, s);
    case MODE_AA_ODD:
      return forced ? step_launch<Q, ST, MODE_AA_ODD, true, BGK>(args, s)
                    : step_launch<Q, ST, MODE_AA_ODD, false, BGK>(args, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step_bgk(int q, int storage, int mode, bool forced, const void* args,
                           hipStream_t s) {
  clear_stale_error();
  if (q == 14) {
    if (storage == ST_F64) return step_q_st<14, ST_F64, true>(mode, forced, args, s);
    if (storage == ST_F32) return step_q_st<14, ST_F32, true>(mode, forced, args, s);
    if (storage == ST_F16) return step_q_st<14, ST_F16, true>(mode, forced, args, s);
  } else if (q == 18) {
    if (storage == ST_F64) return step_q_st<18, ST_F64, true>(mode, forced, args, s);
    if (storage == ST_F32) return step_q_st<18, ST_F32, true>(mode, forced, args, s);
    if (storage == ST_F16) return step_q_st<18, ST_F16, true>(mode, forced, args, s);
  } else if (q == 26) {
    if (storage == ST_F64) return step_q_st<26, ST_F64, true>(mode, forced, args, s);
    if (storage == ST_F32) return step_q_st<26, ST_F32, true>(mode, forced, args, s);
    if (storage == ST_F16) return step_q_st<26, ST_F16, true>(mode, forced, args, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step(int q, int storage, int mode, bool forced, const void* args, size_t,
                       hipStream_t s) {
  clear_stale_error();
  if (q == 14) {
    if (storage == ST_F64) return step_q_st<14, ST_F64>(mode, forced, args, s);
    if (storage == ST_F32) return step_q_st<14, ST_F32>(mode, forced, args, s);
    if (storage == ST_F16) return step_q_st<14, ST_F16>(mode, forced, args, s);
  } else if (q == 18) {
    if (storage == ST_F64) return step_q_st<18, ST_F64>(mode, forced, args, s);
    if (storage == ST_F32) return step_q_st<18, ST_F32>(mode, forced, args, s);
    if (storage == ST_F16) return step_q_st<18, ST_F16>(mode, forced, args, s);
  } else if (q == 26) {
    if (storage == ST_F64) return step_q_st<26, ST_F64>(mode, forced, args, s);
    if (storage == ST_F32) return step_q_st<26, ST_F32>(mode, forced, args, s);
    if (storage == ST_F16) return step_q_st<26, ST_F16>(mode, forced, args, s);
  }
  return hipErrorInvalidValue;
}

// ---- grid-stride helpers for the auxiliary kernels -------------------------
__device__ __forceinline__ void node_xyz(long long n, int nx, int ny, int& x, int& y, int& z) {
  x = (int)(n % nx);
  const long long r = n / nx;
  y = (int)(r % ny);
  z = (int)(r / ny);
}

// ---- population get / set / init -------------------------------------------
template <int Q, int ST, int PHASE>
__global__ __launch_bounds__(256) void k_get_pop(LatticeArgs<typename Codec<ST>::C> A, int a,
                                                 double* __restrict__ out) {
  using CD = Codec<ST>;
  using C = typename CD::C;
  const long long N = (long long)A.nx * A.ny * A.nz;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
       n += (long long)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz(n, A.nx, A.ny, x, y, z);
    C f[Q];
    read_node<Q, ST, PHASE, true>(A, static_cast<const typename CD::S*>(A.f), (unsigned)n, x, y, z,
                                  f);
    // select population a without dynamic register indexing
    C v = f[0];
#pragma unroll
    for (int k = 1; k < Q; ++k)
      if (k == a) v = f[k];
    out[n] = (double)v;
  }
}

template <int Q, int ST>
__global__ __launch_bounds__(256) void k_set_pop(LatticeArgs<typename Codec<ST>::C> A, int a,
                                                 const double* __restrict__ in) {
  using CD = Codec<ST>;
  using C = typename CD::C;
  const long long N = (long long)A.nx * A.ny * A.nz;
  typename CD::S* dst = static_cast<typename CD::S*>(A.f) + a * A.stride;
  // weight class of population a, selected without indexing by a
  int cls = 0;
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (k == a) cls = wclass<Q>(k);
  const C base = A.base_s[cls];
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
       n += (long long)gridDim.x * blockDim.x)
    dst[n] = CD::enc((C)in[n], base, A.scale);
}

// Eq. (edf) with Eq. (lamda_alpha): f_a = 3 w_a p + w_a (3 c.u + 9/2 (c.u)^2
// - 3/2 |u|^2), evaluated in FP64 with j = u - F/2.
template <int Q, int ST>
__global__ __launch_bounds__(256) void k_init_eq(LatticeArgs<typename Codec<ST>::C> A,
                                                 const double* __restrict__ p,
                                                 const double* __restrict__ u, double p0, double u0x,
                                                 double u0y, double u0z, double Fx, double Fy,
                                                 double Fz) {
  using CD = Codec<ST>;
  using C = typename CD::C;
  using L = Lattice<Q>;
  const long long N = (long long)A.nx * A.ny * A.nz;
  typename CD::S* dst = static_cast<typename CD::S*>(A.f);
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
       n += (long long)gridDim.x * blockDim.x) {
    const double pn = p ? p[n] : p0;
    const double jx = (u ? u[n] : u0x) - 0.5 * Fx;
    const double jy = (u ? u[N + n] : u0y) - 0.5 * Fy;
    const double jz = (u ? u[2 * N + n] : u0z) - 0.5 * Fz;
    const double jsq = jx * jx + jy * jy + jz * jz;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const double w = weight<Q>(a);
      const double cu = L::cx[a] * jx + L::cy[a] * jy + L::cz[a] * jz;
      const double fe = 3.0 * w * pn + w * (3.0 * cu + 4.5 * cu * cu - 1.5 * jsq);
      dst[a * A.stride + n] = CD::enc((C)fe, A.base_s[wclass<Q>(a)], A.scale);
    }
  }
}

static int aux_blocks(long long N) {
  long long b = (N + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

#define DISPATCH_QST(q, st, CALL)                      \
  do {                                                 \
    if ((q) == 14) {                                   \
      if ((st) == ST_F64) { constexpr int Q_ = 14; constexpr int ST_ = ST_F64; CALL; } \
      if ((st) == ST_F32) { constexpr int Q_ = 14; constexpr int ST_ = ST_F32; CALL; } \
      if ((st) == ST_F16) { constexpr int Q_ = 14; constexpr int ST_ = ST_F16; CALL; } \
    } else if ((q) == 18) {                            \
      if ((st) == ST_F64) { constexpr int Q_ = 18; constexpr int ST_ = ST_F64; CALL; } \
      if ((st) == ST_F32) { constexpr int Q_ = 18; constexpr int ST_ = ST_F32; CALL; } \
      if ((st) == ST_F16) { constexpr int Q_ = 18; constexpr int ST_ = ST_F16; CALL; } \
    } else if ((q) == 26) {                            \
      if ((st) == ST_F64) { constexpr int Q_ = 26; constexpr int ST_ = ST_F64; CALL; } \
      if ((st) == ST_F32) { constexpr int Q_ = 26; constexpr int ST_ = ST_F32; CALL; } \
      if ((st) == ST_F16) { constexpr int Q_ = 26; constexpr int ST_ = ST_F16; CALL; } \
    }                                                  \
    return hipErrorInvalidValue;                       \
  } while (0)

template <int Q, int ST>
static hipError_t get_pop_impl(int phase, const void* args, int a, double* out, hipStream_t s) {
  clear_stale_error();
  using C = typename Codec<ST>::C;
  const LatticeArgs<C>& A = *static_cast<const LatticeArgs<C>*>(args);
  const int nb = aux_blocks((long long)A.nx * A.ny * A.nz);
  if (phase == 0)
    hipLaunchKernelGGL((k_get_pop<Q, ST, 0>), dim3(nb), dim3(256), 0, s, A, a, out);
  else
    hipLaunchKernelGGL((k_get_pop<Q, ST, 1>), dim3(nb), dim3(256), 0, s, A, a, out);
  return hipGetLastError();
}

hipError_t launch_get_pop(int q, int storage, int phase, int a, const void* args, double* out,
                          hipStream_t s) {
  clear_stale_error();
  DISPATCH_QST(q, storage, return (get_pop_impl<Q_, ST_>(phase, args, a, out, s)));
}

template <int Q, int ST>
static hipError_t set_pop_impl(const void* args, int a, const double* in, hipStream_t s) {
  clear_stale_error();
  using C = typename Codec<ST>::C;
  const LatticeArgs<C>& A = *static_cast<const LatticeArgs<C>*>(args);
  const int nb = aux_blocks((long long)A.nx * A.ny * A.nz);
  hipLaunchKernelGGL((k_set_pop<Q, ST>), dim3(nb), dim3(256), 0, s, A, a, in);
  return hipGetLastError();
}

hipError_t launch_set_pop(int q, int storage, int a, const void* args, const double* in,
                          hipStream_t s) {
  clear_stale_error();
  DISPATCH_QST(q, storage, return (set_pop_impl<Q_, ST_>(args, a, in, s)));
}

template <int Q, int ST>
static hipError_t init_impl(const void* args, const double* p, const double* u, double p0,
                            const double* u0, hipStream_t s) {
  clear_stale_error();
  using C = typename Codec<ST>::C;
  const LatticeArgs<C>& A = *static_cast<const LatticeArgs<C>*>(args);
  const int nb = aux_blocks((long long)A.nx * A.ny * A.nz);
  hipLaunchKernelGGL((k_init_eq<Q, ST>), dim3(nb), dim3(256), 0, s, A, p, u, p0, u0[0], u0[1],
                     u0[2], (double)A.F[0], (double)A.F[1], (double)A.F[2]);
  return hipGetLastError();
}

hipError_t launch_init_eq(int q, int storage, const void* args, const double* p, const double* u,
                          double p0, const double* u0, hipStream_t s) {
  clear_stale_error();
  DISPATCH_QST(q, storage, return (init_impl<Q_, ST_>(args, p, u, p0, u0, s)));
}

// ---- non-equilibrium extrapolation (velocity / pressure faces) --------------
// Eq. (edf) in the compute type: f_a = 3 w_a p + w_a (3 c.u + 9/2 (c.u)^2
// - 3/2 |u|^2).
template <int Q, typename C>
__device__ __forceinline__ void feq_c(C p, C ux, C uy, C uz, C (&fe)[Q]) {
  using L = Lattice<Q>;
  const C usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const C w = (C)weight<Q>(a);
    const C cu = (C)L::cx[a] * ux + (C)L::cy[a] * uy + (C)L::cz[a] * uz;
    fe[a] = C(3) * w * p + w * (C(3) * cu + C(4.5) * cu * cu - C(1.5) * usq);
  }
}

// Store the physical populations f of node n in the layout of PHASE: the
// exact inverse of read_node's addressing (each physical population of
// each node has one slot, so stores for one node never touch a slot that
// represents another node's population).
// Only the populations whose bit is set in `sel` are stored.
template <int Q, int ST, int PHASE>
__device__ __forceinline__ void store_node(const LatticeArgs<typename Codec<ST>::C>& A,
                                           typename Codec<ST>::S* dst, unsigned n, int x, int y,
                                           int z, const typename Codec<ST>::C (&f)[Q], unsigned h,
                                           unsigned sel) {
  using C = typename Codec<ST>::C;
  using L = Lattice<Q>;
  const long long st = A.stride;
  if (PHASE == 0) {
#pragma unroll
    for (int a = 0; a < Q; ++a)
      if (sel & (1u << a)) pop_store(dst + a * st + n, enc_any<Q, ST>(A, f[a], a, h, a));
  } else {
    const Nbr b = make_nbr<true>(A, x, y, z);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      if (!(sel & (1u << a))) continue;
      const int o = L::opp[a];
      int off, slot;
      bool wall;
      C term;
      link<Q, C>(b, A, o, -L::cx[a], -L::cy[a], -L::cz[a], off, wall, term, slot);
      const long long idx = wall ? (a * st + n) : (slot * st + (long long)(n + off));
      pop_store(dst + idx, enc_any<Q, ST>(A, f[a], a, h, a));
    }
  }
}

// Node-layer symmetry planes: at a node on such planes, the populations that
// arrive from beyond a plane are replaced by the mirrored populations of the
// same node (which streaming delivered from the layer below); returns the
// mask of replaced populations (0 if the node is on no such plane).
template <int Q, typename C>
__device__ __forceinline__ unsigned mirror_arrivals(const NeeArgs<C>& E, const int (&dim)[3],
                                                    const int (&own)[3], C (&f)[Q]) {
  using L = Lattice<Q>;
  int side[3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
    side[d] = (own[d] == 0 && E.kind[2 * d] == 5) ? -1
              : (own[d] == dim[d] - 1 && E.kind[2 * d + 1] == 5) ? 1 : 0;
  if (!(side[0] | side[1] | side[2])) return 0u;
  C g[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) g[a] = f[a];
  unsigned sel = 0u;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const bool bx = L::cx[a] * side[0] < 0, by = L::cy[a] * side[1] < 0,
               bz = L::cz[a] * side[2] < 0;
    const C lo = by ? (bx ? g[mirror<Q>(a, 3)] : g[mirror<Q>(a, 2)])
                    : (bx ? g[mirror<Q>(a, 1)] : g[a]);
    const C hi = by ? (bx ? g[mirror<Q>(a, 7)] : g[mirror<Q>(a, 6)])
                    : (bx ? g[mirror<Q>(a, 5)] : g[mirror<Q>(a, 4)]);
    f[a] = bz ? hi : lo;
    if (bx | by | bz) sel |= 1u << a;
  }
  return sel;
}

// The pass at one listed boundary node x_b (k_nee: one thread per node of
// a lattice's list; k_batch_nee: of a batch class's lists).  On velocity / pressure faces
// (non-equilibrium extrapolation): inward neighbour x_f (never on such a
// face itself, as each such axis has >= 3 nodes; if it lies on a node-layer
// symmetry plane its arriving populations are taken mirrored, as that
// plane's own pass defines them), its p_f, u_f (Eq. (hgl), u = sum c f +
// F/2) and f_neq = f(x_f) - f_eq(p_f, u_f); then f(x_b) = f_eq(p_b, u_b) +
// f_neq.  Otherwise, on node-layer symmetry planes only: the arriving
// populations become the mirrored ones.  Each thread writes only its own
// node's populations.  It reads its own node, or an inward neighbour on no
// velocity / pressure face; if that neighbour is on a symmetry plane, its
// arrival slots (which the neighbour's own thread may be rewriting) are
// read but not used, the mirrored values standing in for them exactly as
// the owner computes them, so the result does not depend on thread order.
template <int Q, int ST, int PHASE>
__device__ __forceinline__ void nee_node(const LatticeArgs<typename Codec<ST>::C>& A,
                                         const NeeArgs<typename Codec<ST>::C>& E, unsigned n) {
  using CD = Codec<ST>;
  using C = typename CD::C;
  using L = Lattice<Q>;
  const int dim[3] = {A.nx, A.ny, A.nz};
  {
    int x, y, z;
    node_xyz(n, A.nx, A.ny, x, y, z);
    const int own[3] = {x, y, z};
    int src[3] = {x, y, z}, vf = -1, pf = -1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int face = -1;
      const int klo = E.kind[2 * d], khi = E.kind[2 * d + 1];
      if (own[d] == 0 && (klo == 3 || klo == 4)) {
        face = 2 * d;
        src[d] = 1;
      } else if (own[d] == dim[d] - 1 && (khi == 3 || khi == 4)) {
        face = 2 * d + 1;
        src[d] = dim[d] - 2;
      }
      if (face < 0) continue;
      if (E.kind[face] == 3)
        vf = face;  // later axes win: z over y over x
      else
        pf = face;
    }
    const unsigned h = node_hash(n, A.tstep) ^ 0x68E31DA4u;
    if (vf < 0 && pf < 0) {
      // node-layer symmetry planes only
      C f[Q];
      read_node<Q, ST, PHASE, true>(A, static_cast<const typename CD::S*>(A.f), n, x, y, z, f);
      const unsigned sel = mirror_arrivals<Q, C>(E, dim, own, f);
      store_node<Q, ST, PHASE>(A, static_cast<typename CD::S*>(A.f), n, x, y, z, f, h, sel);
      return;
    }
    const unsigned m = (unsigned)src[0] + (unsigned)A.nx * ((unsigned)src[1] + (unsigned)A.ny * (unsigned)src[2]);
    C ff[Q];
    read_node<Q, ST, PHASE, true>(A, static_cast<const typename CD::S*>(A.f), m, src[0], src[1],
                                  src[2], ff);
    (void)mirror_arrivals<Q, C>(E, dim, src, ff);
    C P = C(0), jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      P += ff[a];
      if (L::cx[a]) jx += L::cx[a] > 0 ? ff[a] : -ff[a];
      if (L::cy[a]) jy += L::cy[a] > 0 ? ff[a] : -ff[a];
      if (L::cz[a]) jz += L::cz[a] > 0 ? ff[a] : -ff[a];
    }
    const C ux = jx + C(0.5) * A.F[0], uy = jy + C(0.5) * A.F[1], uz = jz + C(0.5) * A.F[2];
    const C w0 = (C)L::w0;
    const C pf_ = (P - C(1.5) * w0 * (ux * ux + uy * uy + uz * uz)) / (C(3) * (C(1) - w0));
    C fe[Q], fb[Q];
    feq_c<Q, C>(pf_, ux, uy, uz, fe);
    C bx = ux, by = uy, bz = uz, pb = pf_;
    if (vf >= 0) {
      bx = E.u[vf][0];
      by = E.u[vf][1];
      bz = E.u[vf][2];
    }
    if (pf >= 0) pb = E.p[pf];
    feq_c<Q, C>(pb, bx, by, bz, fb);
#pragma unroll
    for (int a = 0; a < Q; ++a) fb[a] += ff[a] - fe[a];
    store_node<Q, ST, PHASE>(A, static_cast<typename CD::S*>(A.f), n, x, y, z, fb, h,
                             (1u << Q) - 1u);
  }
}

template <int Q, int ST, int PHASE>
__global__ __launch_bounds__(256) void k_nee(LatticeArgs<typename Codec<ST>::C> A,
                                             NeeArgs<typename Codec<ST>::C> E,
                                             const int* __restrict__ nodes, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    nee_node<Q, ST, PHASE>(A, E, (unsigned)nodes[i]);
}

template <int Q, int ST>
static hipError_t nee_impl(int phase, const void* args, const void* nee, const int* nodes,
                           int count, hipStream_t s) {
  clear_stale_error();
  using C = typename Codec<ST>::C;
  const LatticeArgs<C>& A = *static_cast<const LatticeArgs<C>*>(args);
  const NeeArgs<C>& E = *static_cast<const NeeArgs<C>*>(nee);
  if (count <= 0) return hipSuccess;
  const int nb = aux_blocks(count);
  if (phase == 0)
    hipLaunchKernelGGL((k_nee<Q, ST, 0>), dim3(nb), dim3(256), 0, s, A, E, nodes, count);
  else
    hipLaunchKernelGGL((k_nee<Q, ST, 1>), dim3(nb), dim3(256), 0, s, A, E, nodes, count);
  return hipGetLastError();
}

hipError_t launch_nee(int q, int storage, int phase, const void* args, const void* nee,
                      const int* nodes, int count, hipStream_t s) {
  clear_stale_error();
  DISPATCH_QST(q, storage, return (nee_impl<Q_, ST_>(phase, args, nee, nodes, count, s)));
}

// ---- macroscopic fields and monitors ----------------------------------------
// P = sum f, j = sum c f (FP64 sums of the decoded values), u = j + F/2,
// p by Eq. (hgl).
template <int Q, typename C>
__device__ __forceinline__ void macro_fp64(const C (&f)[Q], const C (&F)[3], double& P, double& ux,
                                           double& uy, double& uz) {
  using L = Lattice<Q>;
  P = 0.0;
  double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const double v = (double)f[a];
    P += v;
    if (L::cx[a]) jx += L::cx[a] > 0 ? v : -v;
    if (L::cy[a]) jy += L::cy[a] > 0 ? v : -v;
    if (L::cz[a]) jz += L::cz[a] > 0 ? v : -v;
  }
  ux = jx + 0.5 * (double)F[0];
  uy = jy + 0.5 * (double)F[1];
  uz = jz + 0.5 * (double)F[2];
}

// p and u (Eq. (hgl)) of node n in FP64.
template <int Q, int ST, int PHASE>
__device__ __forceinline__ void node_macros(const LatticeArgs<typename Codec<ST>::C>& A,
                                            long long n, double& p, double& ux, double& uy,
                                            double& uz) {
  using CD = Codec<ST>;
  using C = typename CD::C;
  using L = Lattice<Q>;
  const C F[3] = {A.F[0], A.F[1], A.F[2]};
  int x, y, z;
  node_xyz(n, A.nx, A.ny, x, y, z);
  C f[Q];
  read_node<Q, ST, PHASE, true>(A, static_cast<const typename CD::S*>(A.f), (unsigned)n, x, y, z,
                                f);
  double P;
  macro_fp64<Q, C>(f, F, P, ux, uy, uz);
  const double usq = ux * ux + uy * uy + uz * uz;
  p = (P - 1.5 * L::w0 * usq) / (3.0 * (1.0 - L::w0));
}

template <int Q, int ST, int PHASE>
__global__ __launch_bounds__(256) void k_macros(LatticeArgs<typename Codec<ST>::C> A,
                                                double* __restrict__ p, double* __restrict__ u) {
  const long long N = (long long)A.nx * A.ny * A.nz;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
       n += (long long)gridDim.x * blockDim.x) {
    double pn, ux, uy, uz;
    node_macros<Q, ST, PHASE>(A, n, pn, ux, uy, uz);
    if (p) p[n] = pn;
    if (u) {
      u[n] = ux;
      u[N + n] = uy;
      u[2 * N + n] = uz;
    }
  }
}

// Nodes [n0, n0 + count) into out[4 count]: p, then u_x, u_y, u_z, each
// count values (the same arithmetic as k_macros).
template <int Q, int ST, int PHASE>
__global__ __launch_bounds__(256) void k_macros_range(LatticeArgs<typename Codec<ST>::C> A,
                                                      long long n0, long long count,
                                                      double* __restrict__ out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    double pn, ux, uy, uz;
    node_macros<Q, ST, PHASE>(A, n0 + i, pn, ux, uy, uz);
    out[i] = pn;
    out[count + i] = ux;
    out[2 * count + i] = uy;
    out[3 * count + i] = uz;
  }
}

template <int Q, int ST>
static hipError_t macros_impl(int phase, const void* args, double* p, double* u, hipStream_t s) {
  clear_stale_error();
  using C = typename Codec<ST>::C;
  const LatticeArgs<C>& A = *static_cast<const LatticeArgs<C>*>(args);
  const int nb = aux_blocks((long long)A.nx * A.ny * A.nz);
  if (phase == 0)
    hipLaunchKernelGGL((k_macros<Q, ST, 0>), dim3(nb), dim3(256), 0, s, A, p, u);
  else
    hipLaunchKernelGGL((k_macros<Q, ST, 1>), dim3(nb), dim3(256), 0, s, A, p, u);
  return hipGetLastError();
}

hipError_t launch_macros(int q, int storage, int phase, const void* args, double* p, double* u,
                         hipStream_t s) {
  clear_stale_error();
  DISPATCH_QST(q, storage, return (macros_impl<Q_, ST_>(phase, args, p, u, s)));
}

template <int Q, int ST>
static hipError_t macros_range_impl(int phase, const void* args, long long n0, long long count,
                                    double* out, hipStream_t s) {
  clear_stale_error();
  using C = typename Codec<ST>::C;
  const LatticeArgs<C>& A = *static_cast<const LatticeArgs<C>*>(args);
  const long long N = (long long)A.nx * A.ny * A.nz;
  if (n0 < 0 || count < 0 || n0 + count > N) return hipErrorInvalidValue;
  if (count == 0) return hipSuccess;
  const int nb = aux_blocks(count);
  if (phase == 0)
    hipLaunchKernelGGL((k_macros_range<Q, ST, 0>), dim3(nb), dim3(256), 0, s, A, n0, count, out);
  else
    hipLaunchKernelGGL((k_macros_range<Q, ST, 1>), dim3(nb), dim3(256), 0, s, A, n0, count, out);
  return hipGetLastError();
}

hipError_t launch_macros_range(int q, int storage, int phase, const void* args, long long n0,
                               long long count, double* out, hipStream_t s) {
  clear_stale_error();
  DISPATCH_QST(q, storage, return (macros_range_impl<Q_, ST_>(phase, args, n0, count, out, s)));
}

// Deterministic block sum of three FP64 values: wavefront butterfly by
// xor-shuffles, then the 4 wavefront results in fixed order.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    a += __shfl_xor(a, m, 64);
    b += __shfl_xor(b, m, 64);
    c += __shfl_xor(c, m, 64);
  }
  __shared__ double sh[3][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wv] = a;
    sh[1][wv] = b;
    sh[2][wv] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
    b = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    c = (sh[2][0] + sh[2][1]) + (sh[2][2] + sh[2][3]);
  }
}

static constexpr int MON_BLOCKS_MAX = 2048;
int monitor_blocks(long long nodes) {
  long long b = (nodes + 255) / 256;
  if (b > MON_BLOCKS_MAX) b = MON_BLOCKS_MAX;
  if (b < 1) b = 1;
  return (int)b;
}

// Pass 1 over nodes [n_begin, n_end) of one lattice, grid-strided by the
// blocks [0, nblk): sums |u - snap|, |u|, P; snap <- u.
template <int Q, int ST, int PHASE>
__device__ __forceinline__ void monitor_body(const LatticeArgs<typename Codec<ST>::C>& A,
                                             typename Codec<ST>::C* __restrict__ snap, int blk,
                                             int nblk, double& s_du, double& s_u, double& s_P) {
  using CD = Codec<ST>;
  using C = typename CD::C;
  const long long N = (long long)A.nx * A.ny * A.nz;
  const C F[3] = {A.F[0], A.F[1], A.F[2]};
  s_du = s_u = s_P = 0.0;
  for (long long n = blk * 256LL + threadIdx.x; n < N; n += (long long)nblk * 256) {
    int x, y, z;
    node_xyz(n, A.nx, A.ny, x, y, z);
    C f[Q];
    read_node<Q, ST, PHASE, true>(A, static_cast<const typename CD::S*>(A.f), (unsigned)n, x, y, z,
                                  f);
    double P, ux, uy, uz;
    macro_fp64<Q, C>(f, F, P, ux, uy, uz);
    const double o0 = (double)snap[n], o1 = (double)snap[N + n], o2 = (double)snap[2 * N + n];
    s_du += fabs(ux - o0) + fabs(uy - o1) + fabs(uz - o2);
    s_u += fabs(ux) + fabs(uy) + fabs(uz);
    s_P += P;
    snap[n] = (C)ux;
    snap[N + n] = (C)uy;
    snap[2 * N + n] = (C)uz;
  }
  block_sum3(s_du, s_u, s_P);
}

template <int Q, int ST, int PHASE>
__global__ __launch_bounds__(256) void k_monitor(LatticeArgs<typename Codec<ST>::C> A,
                                                 typename Codec<ST>::C* __restrict__ snap,
                                                 double* __restrict__ partial) {
  double a, b, c;
  monitor_body<Q, ST, PHASE>(A, snap, blockIdx.x, gridDim.x, a, b, c);
  if (threadIdx.x == 0) {
    partial[3 * blockIdx.x + 0] = a;
    partial[3 * blockIdx.x + 1] = b;
    partial[3 * blockIdx.x + 2] = c;
  }
}

template <int Q, int ST>
static hipError_t monitor_impl(int phase, const void* args, void* snap, double* partial, int* nbo,
                               hipStream_t s) {
  clear_stale_error();
  using C = typename Codec<ST>::C;
  const LatticeArgs<C>& A = *static_cast<const LatticeArgs<C>*>(args);
  const int nb = monitor_blocks((long long)A.nx * A.ny * A.nz);
  *nbo = nb;
  if (phase == 0)
    hipLaunchKernelGGL((k_monitor<Q, ST, 0>), dim3(nb), dim3(256), 0, s, A, (C*)snap, partial);
  else
    hipLaunchKernelGGL((k_monitor<Q, ST, 1>), dim3(nb), dim3(256), 0, s, A, (C*)snap, partial);
  return hipGetLastError();
}

hipError_t launch_monitor(int q, int storage, int phase, const void* args, void* snap,
                          double* partial, int* nbo, hipStream_t s) {
  clear_stale_error();
  DISPATCH_QST(q, storage, return (monitor_impl<Q_, ST_>(phase, args, snap, partial, nbo, s)));
}

// Pass 2: one workgroup, fixed-order sum of nb partial triples into
// out[0..2], and out[3], a flag that stays 1 once any pass has seen a
// non-finite sum |u| or mass, or (flags bit 0: the snapshot holds an
// earlier u of this state) a non-finite sum |u - snap|; flags bit 1 starts
// the flag afresh (the first pass on new memory or a replaced state).
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ partial,
                                                         int nb, double* __restrict__ out,
                                                         int flags) {
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += partial[3 * i];
    b += partial[3 * i + 1];
    c += partial[3 * i + 2];
  }
  block_sum3(a, b, c);
  if (threadIdx.x == 0) {
    const bool bad = !isfinite(b) || !isfinite(c) || ((flags & 1) && !isfinite(a));
    const bool before = !(flags & 2) && out[3] != 0.0;
    out[0] = a;
    out[1] = b;
    out[2] = c;
    out[3] = (bad || before) ? 1.0 : 0.0;
  }
}

hipError_t launch_reduce_partials(const double* partial, int nb, double* out, int flags,
                                  hipStream_t s) {
  clear_stale_error();
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partial, nb, out, flags);
  return hipGetLastError();
}

// ---- measurement helper: plain streaming copy ---------------------------------
// Each thread moves 2 x 16 bytes, both loads issued before the stores, one
// workgroup per 8 KB.  Of the variants measured on MI355X (1-4 GiB, in place
// and not) this one is the fastest: 4 x 16 B per thread is 3-4 % slower and
// 8 x 16 B 28 % slower; non-temporal stores do not help.  It is the
// achievable-bandwidth reference the step kernels are read against.  The
// workgroup order is the faster one for the footprint: dispatch order in
// the Infinity Cache (151 MB in place: 7.1 TB/s against 6.7 XCD-contiguous),
// XCD-contiguous from HBM (1 GiB in place: 6.0 TB/s against 5.6; 1 GiB to a
// second GiB: 5.90 against 5.82).
__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src,
                                              uint4* __restrict__ dst, long long n16, int xcd) {
  const long long base = (long long)(xcd ? xcd_contiguous() : blockIdx.x) * 512LL + threadIdx.x;
  uint4 v[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const long long i = base + 256LL * k;
    if (i < n16) v[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const long long i = base + 256LL * k;
    if (i < n16) dst[i] = v[k];
  }
}

hipError_t launch_copy_probe(void* dst, const void* src, size_t bytes, int xcd, hipStream_t s) {
  clear_stale_error();
  const long long n16 = (long long)(bytes / 16);
  long long nb = (n16 + 511) / 512;
  if (nb < 1) nb = 1;
  if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)nb), dim3(256), 0, s, (const uint4*)src, (uint4*)dst,
                     n16, xcd);
  return hipGetLastError();
}

// ---- batched execution --------------------------------------------------------
// One launch per time step and (q, storage) class over the tiles of every
// member of the class; the host aligns the members' AA parity (a member out
// of step sits out one substep), so each launch runs exactly the node update
// of k_step for one memory pattern.  A class with any forced member runs the
// force path for all of them (with F = 0 it gives the same bits as the
// unforced path).  A workgroup finds its member by binary search over the
// members' first tile indices (uniform scalar loads).  Per-member
// arithmetic does not depend on the other members, so a member's result is
// the same alone and in any mix.
// Members of a small launch class: one tile per workgroup, the member found
// by binary search over the members' first tiles.
__device__ __forceinline__ int find_member(const BatchMember* __restrict__ ms, int nm,
                                           unsigned tile) {
  int lo = 0, hi = nm - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ms[mid].tile_begin <= (long long)tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Per-node work of a batched step once the member and its tile are known.
template <int Q, int ST, int MODE, bool FORCED>
__device__ __forceinline__ void batch_tile(const BatchMember& m, const float* __restrict__ ftab,
                                           int own, unsigned lt) {
  LatticeArgs<float> A = m.a;
  const unsigned t = threadIdx.x;
  int x, y;
  unsigned zz;
  if (m.flat) {
    // 256 consecutive nodes (every wavefront full and aligned, whatever nx)
    const unsigned n = lt * 256u + t;
    if (n >= (unsigned)A.nx * (unsigned)A.ny * (unsigned)A.nz) return;
    const unsigned r = fast_div(n, m.fd_nx);
    x = (int)(n - r * (unsigned)A.nx);
    zz = fast_div(r, m.fd_ny);
    y = (int)(r - zz * (unsigned)A.ny);
  } else {
    const int tx = A.tx;
    if (t >= (unsigned)(tx * A.ty)) return;
    const unsigned r = fast_div(lt, A.fd_tiles_x);
    const int bx = (int)(lt - r * (unsigned)A.tiles_x);
    zz = fast_div(r, A.fd_tiles_y);
    const int by = (int)(r - zz * (unsigned)A.tiles_y);
    const unsigned ly = fast_div(t, A.fd_tx);
    x = bx * tx + (int)(t - ly * (unsigned)tx);
    y = by * A.ty + (int)ly;
    if (x >= A.nx || y >= A.ny) return;
  }
  A.tstep += (unsigned)own;
  if (FORCED) {
    if (m.forced) {
      const float* Fr = ftab + m.ftab_off + 3LL * own;
      A.F[0] = Fr[0];
      A.F[1] = Fr[1];
      A.F[2] = Fr[2];
    } else {
      A.F[0] = A.F[1] = A.F[2] = 0.0f;
    }
  }
  // every member of a batch class spans less than 4 GiB (larger ones step
  // on their own), so the class takes the single lattice's odd-step choice
  node_step_any<Q, ST, MODE, FORCED, false, odd32_kernel<Q, ST, MODE>()>(A, x, y, (int)zz);
}

template <int Q, int ST, int MODE, bool FORCED>
__global__ __launch_bounds__(256) void k_batch_grp(const BatchMember* __restrict__ ms, int nm,
                                                   const float* __restrict__ ftab, int substep,
                                                   int xcd_order) {
  const unsigned tile = xcd_order ? xcd_block(xcd_order) : blockIdx.x;
  const BatchMember& m = ms[find_member(ms, nm, tile)];
  const int own = substep - m.skip;  // this member's own step within the call
  if (own < 0 || own >= m.steps) return;
  const unsigned lt = tile - (unsigned)m.tile_begin;
  if (lt >= (unsigned)m.ntiles) return;
  batch_tile<Q, ST, MODE, FORCED>(m, ftab, own, lt);
}

// Members of a large launch class: workgroup b runs the kBatchChunk tiles
// of chunks[b] one after the other (fewer, longer-lived workgroups).
template <int Q, int ST, int MODE, bool FORCED>
__global__ __launch_bounds__(256) void k_batch_chunk(const BatchMember* __restrict__ ms,
                                                     const BatchChunk* __restrict__ chunks,
                                                     const float* __restrict__ ftab,
                                                     int substep, int xcd_order) {
  const BatchChunk ch = chunks[xcd_order ? xcd_block(xcd_order) : blockIdx.x];
  const BatchMember& m = ms[ch.member];
  const int own = substep - m.skip;
  if (own < 0 || own >= m.steps) return;
  const unsigned end = (unsigned)min((long long)ch.tile + kBatchChunk, m.ntiles);
  for (unsigned lt = (unsigned)ch.tile; lt < end; ++lt)
    batch_tile<Q, ST, MODE, FORCED>(m, ftab, own, lt);
}

template <int Q, int ST, int MODE, bool FORCED>
static void batch_launch_k(const BatchLaunch& L, hipStream_t s) {
  if (L.chunks)
    hipLaunchKernelGGL((k_batch_chunk<Q, ST, MODE, FORCED>), dim3((unsigned)L.nblocks), dim3(256),
                       0, s, L.members, L.chunks, L.ftab, L.substep, L.xcd_order);
  else
    hipLaunchKernelGGL((k_batch_grp<Q, ST, MODE, FORCED>), dim3((unsigned)L.nblocks), dim3(256), 0,
                       s, L.members, L.nmembers, L.ftab, L.substep, L.xcd_order);
}

template <int Q, int ST>
static void batch_launch_m(int mode, bool forced, const BatchLaunch& L, hipStream_t s) {
  if (mode == MODE_AA_EVEN)
    forced ? batch_launch_k<Q, ST, MODE_AA_EVEN, true>(L, s)
           : batch_launch_k<Q, ST, MODE_AA_EVEN, false>(L, s);
  else
    forced ? batch_launch_k<Q, ST, MODE_AA_ODD, true>(L, s)
           : batch_launch_k<Q, ST, MODE_AA_ODD, false>(L, s);
}

hipError_t launch_batch_group(int q, int storage, int mode, bool forced, const BatchLaunch& L,
                              hipStream_t s) {
  clear_stale_error();
  if (L.nblocks <= 0 || L.nmembers <= 0) return hipSuccess;
  if (L.nblocks >= (1LL << 31) || (mode != MODE_AA_EVEN && mode != MODE_AA_ODD))
    return hipErrorInvalidValue;
  if (q == 14 && storage == ST_F32)
    batch_launch_m<14, ST_F32>(mode, forced, L, s);
  else if (q == 14 && storage == ST_F16)
    batch_launch_m<14, ST_F16>(mode, forced, L, s);
  else if (q == 18 && storage == ST_F32)
    batch_launch_m<18, ST_F32>(mode, forced, L, s);
  else if (q == 18 && storage == ST_F16)
    batch_launch_m<18, ST_F16>(mode, forced, L, s);
  else if (q == 26 && storage == ST_F32)
    batch_launch_m<26, ST_F32>(mode, forced, L, s);
  else if (q == 26 && storage == ST_F16)
    batch_launch_m<26, ST_F16>(mode, forced, L, s);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// The velocity / pressure / node-layer symmetry pass of a batched substep:
// one thread per boundary node of the class's members.  A thread finds its
// member as the last one whose first boundary index is <= its own (members
// without such faces own an empty range) and runs the single-lattice pass
// for that node, with the member's time level, force and face pressures of
// the level just reached (host-computed rows, the same floats as for a
// single lattice), so a member gives the same bits alone, in any mix, and
// as a single lattice.
__device__ __forceinline__ int find_nee_member(const BatchMember* __restrict__ ms, int nm,
                                               long long i) {
  int lo = 0, hi = nm - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ms[mid].nee_begin <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int Q, int ST, int PHASE>
__global__ __launch_bounds__(256) void k_batch_nee(const BatchMember* __restrict__ ms, int nm,
                                                   const float* __restrict__ ntab, int substep,
                                                   long long total) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const BatchMember& m = ms[find_nee_member(ms, nm, i)];
    const long long j = i - m.nee_begin;
    if (j < 0 || j >= m.nee_count) continue;
    const int own = substep - m.skip;
    if (own < 0 || own >= m.steps) continue;
    LatticeArgs<float> A = m.a;
    A.tstep += (unsigned)(own + 1);
    const float* row = ntab + m.ntab_off + 9LL * own;
    A.F[0] = row[0];
    A.F[1] = row[1];
    A.F[2] = row[2];
    NeeArgs<float> E = m.e;
#pragma unroll
    for (int f = 0; f < 6; ++f) E.p[f] = row[3 + f];
    nee_node<Q, ST, PHASE>(A, E, (unsigned)m.nee_nodes[j]);
  }
}

template <int Q, int ST>
static void batch_nee_q(int phase, const BatchMember* ms, int nm, const float* ntab, int substep,
                        long long total, hipStream_t s) {
  const int nb = aux_blocks(total);
  if (phase == 0)
    hipLaunchKernelGGL((k_batch_nee<Q, ST, 0>), dim3(nb), dim3(256), 0, s, ms, nm, ntab, substep,
                       total);
  else
    hipLaunchKernelGGL((k_batch_nee<Q, ST, 1>), dim3(nb), dim3(256), 0, s, ms, nm, ntab, substep,
                       total);
}

hipError_t launch_batch_nee(int q, int storage, int phase, const BatchMember* members,
                            int nmembers, const float* ntab, int substep, long long total,
                            hipStream_t s) {
  clear_stale_error();
  if (total <= 0 || nmembers <= 0) return hipSuccess;
  if (q == 14 && storage == ST_F32)
    batch_nee_q<14, ST_F32>(phase, members, nmembers, ntab, substep, total, s);
  else if (q == 14 && storage == ST_F16)
    batch_nee_q<14, ST_F16>(phase, members, nmembers, ntab, substep, total, s);
  else if (q == 18 && storage == ST_F32)
    batch_nee_q<18, ST_F32>(phase, members, nmembers, ntab, substep, total, s);
  else if (q == 18 && storage == ST_F16)
    batch_nee_q<18, ST_F16>(phase, members, nmembers, ntab, substep, total, s);
  else if (q == 26 && storage == ST_F32)
    batch_nee_q<26, ST_F32>(phase, members, nmembers, ntab, substep, total, s);
  else if (q == 26 && storage == ST_F16)
    batch_nee_q<26, ST_F16>(phase, members, nmembers, ntab, substep, total, s);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Batched monitor: block b belongs to the member whose block range holds it.
__device__ __forceinline__ int find_block_member(const long long* __restrict__ bb, int nm,
                                                 long long blk) {
  int lo = 0, hi = nm - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bb[mid] <= blk)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_batch_monitor(const BatchMember* __restrict__ ms, int nm,
                                                       void* const* __restrict__ snaps,
                                                       double* __restrict__ partial,
                                                       const long long* __restrict__ pofs,
                                                       const long long* __restrict__ bbeg,
                                                       const int* __restrict__ phases) {
  const long long blk = blockIdx.x;
  const int mi = find_block_member(bbeg, nm, blk);
  const BatchMember& m = ms[mi];
  const int lb = (int)(blk - bbeg[mi]);
  const int nblk = (int)((mi + 1 < nm ? bbeg[mi + 1] : (long long)gridDim.x) - bbeg[mi]);
  const int ph = phases[mi];
  double a = 0, b = 0, c = 0;
  float* snap = static_cast<float*>(snaps[mi]);
  LatticeArgs<float> A = m.a;
  if (m.q == 14) {
    if (m.storage == ST_F32) {
      if (ph == 0) monitor_body<14, ST_F32, 0>(A, snap, lb, nblk, a, b, c);
      else monitor_body<14, ST_F32, 1>(A, snap, lb, nblk, a, b, c);
    } else {
      if (ph == 0) monitor_body<14, ST_F16, 0>(A, snap, lb, nblk, a, b, c);
      else monitor_body<14, ST_F16, 1>(A, snap, lb, nblk, a, b, c);
    }
  } else if (m.q == 18) {
    if (m.storage == ST_F32) {
      if (ph == 0) monitor_body<18, ST_F32, 0>(A, snap, lb, nblk, a, b, c);
      else monitor_body<18, ST_F32, 1>(A, snap, lb, nblk, a, b, c);
    } else {
      if (ph == 0) monitor_body<18, ST_F16, 0>(A, snap, lb, nblk, a, b, c);
      else monitor_body<18, ST_F16, 1>(A, snap, lb, nblk, a, b, c);
    }
  } else {
    if (m.storage == ST_F32) {
      if (ph == 0) monitor_body<26, ST_F32, 0>(A, snap, lb, nblk, a, b, c);
      else monitor_body<26, ST_F32, 1>(A, snap, lb, nblk, a, b, c);
    } else {
      if (ph == 0) monitor_body<26, ST_F16, 0>(A, snap, lb, nblk, a, b, c);
      else monitor_body<26, ST_F16, 1>(A, snap, lb, nblk, a, b, c);
    }
  }
  if (threadIdx.x == 0) {
    double* o = partial + 3 * (pofs[mi] + lb);
    o[0] = a;
    o[1] = b;
    o[2] = c;
  }
}

hipError_t launch_batch_monitor(const BatchMember* ms, int nm, void* const* snaps, double* partial,
                                const long long* pofs, long long total_blocks,
                                const long long* bbeg, const int* phases, hipStream_t s) {
  clear_stale_error();
  if (nm <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_monitor, dim3((unsigned)total_blocks), dim3(256), 0, s, ms, nm, snaps,
                     partial, pofs, bbeg, phases);
  return hipGetLastError();
}

// One workgroup per member: fixed-order sum of that member's partials.
__global__ __launch_bounds__(256) void k_batch_reduce(const double* __restrict__ partial,
                                                      const long long* __restrict__ pofs,
                                                      const long long* __restrict__ pcount,
                                                      double* __restrict__ out) {
  const int mi = blockIdx.x;
  const double* p = partial + 3 * pofs[mi];
  const long long nb = pcount[mi];
  double a = 0.0, b = 0.0, c = 0.0;
  for (long long i = threadIdx.x; i < nb; i += 256) {
    a += p[3 * i];
    b += p[3 * i + 1];
    c += p[3 * i + 2];
  }
  block_sum3(a, b, c);
  if (threadIdx.x == 0) {
    out[3 * mi] = a;
    out[3 * mi + 1] = b;
    out[3 * mi + 2] = c;
  }
}

hipError_t launch_batch_reduce(const double* partial, const long long* pofs,
                               const long long* pcount, int nm, double* out, hipStream_t s) {
  clear_stale_error();
  if (nm <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_reduce, dim3(nm), dim3(256), 0, s, partial, pofs, pcount, out);
  return hipGetLastError();
}

}  // namespace lbm

// kernels.hpp -- argument blocks and launch entry points of the device
// code (kernels.hip); used by the host runtime (runtime.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace lbm {

enum Storage { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2 };
// AB: read natural A, collide, push into B.  AA_EVEN: read natural, write
// each post-collision population into its opposite slot of the same node.
// AA_ODD: gather from the neighbours' opposite slots, collide, push.
enum Mode { MODE_AB = 0, MODE_AA_EVEN = 1, MODE_AA_ODD = 2 };

// Division by a fixed divisor d as a multiply and shift, for numerators
// below 2^30: m = ceil(2^(32+l) / d), l = ceil(log2 d); the rounding error
// n (m d - 2^(32+l)) / (d 2^(32+l)) stays below 1/(4d), so the floor is
// exact.
struct FastDiv {
  unsigned long long m;
  unsigned s;  // 32 + l
  unsigned d;
};
inline FastDiv make_fastdiv(unsigned d) {
  unsigned l = 0;
  while ((1ull << l) < d) ++l;
  const unsigned long long m = ((1ull << (32 + l)) + d - 1) / d;
  return FastDiv{m, 32 + l, d};
}
__device__ __forceinline__ unsigned fast_div(unsigned n, const FastDiv& f) {
  return (unsigned)(((unsigned long long)n * f.m) >> f.s);
}

// Everything a lattice kernel needs about one lattice, in compute type C.
template <typename C> struct LatticeArgs {
  void* f;                 // populations (AB: the copy read this step)
  void* g;                 // AB: the copy written this step; AA: == f
  long long stride;        // elements between population arrays (= N)
  long long pbytes;        // stride in bytes of the stored type
  long long pofs[26];      // a * pbytes: byte offset of population array a
  int nx, ny, nz;
  int per_x, per_y, per_z; // periodic axes
  int sym;                 // bit f set: face f (-x,+x,-y,+y,-z,+z) is a
                           // symmetry plane (specular reflection)
  int tx, ty, tiles_x, tiles_y;  // x-y tile of one workgroup
  int xcd_order;           // tile order (workgroup w runs on XCD w % 8):
                           // 0 tile = w; 1 a contiguous range of tiles per
                           // XCD; 2 chunks of 4 tiles per XCD in turn
  C sN[26], hN[26];        // s_k/N_k, (1 - s_k/2)/N_k
  C bb[26][3];             // 6 w_a (c_a . u_w) for link a leaving through
                           // the x / y / z face it crosses (FP16 storage:
                           // times 2^s, the step kernels' deviation units)
  C F[3];                  // body force at this step
  C base[3], base_s[3];    // FP16 deviation base 3 w_a p0 of the axis, edge
                           // and corner populations (|c_a|^2 = 1, 2, 3), and
                           // base 2^s (exact: 2^s is a power of two)
  C scale, inv_scale;      // FP16 2^s, 2^-s
  unsigned tstep;          // time level t of this step (FP16 rounding dither)
  int f16_sr;              // FP16 stores: 1 stochastic rounding, 0 nearest
  FastDiv fd_tiles_x, fd_tiles_y, fd_tx;  // tile decoding without divisions
  C omega, hom;            // LBGK collision: 1/tau, 1 - 1/(2 tau)
};

// Boundary values of the velocity / pressure faces (non-equilibrium
// extrapolation) at the time level being completed.
template <typename C> struct NeeArgs {
  int kind[6];   // 3 velocity face, 4 pressure face, 5 node-layer symmetry
                 // face, anything else: none of these
  C u[6][3];     // velocity of a velocity face
  C p[6];        // pressure of a pressure face at this level
};

// Launches (all asynchronous on `stream`; return a hipError_t).
hipError_t launch_step(int q, int storage, int mode, bool forced, const void* args,
                       size_t args_bytes, hipStream_t stream);
// The same step with the LBGK collision (S = I/tau).
hipError_t launch_step_bgk(int q, int storage, int mode, bool forced, const void* args,
                           hipStream_t stream);
// Decode population a of the current state (phase: 0 natural, 1 AA
// swapped) into FP64 out[N].
hipError_t launch_get_pop(int q, int storage, int phase, int a, const void* args, double* out,
                          hipStream_t stream);
// Non-equilibrium extrapolation on the `count` nodes listed in `nodes`
// (linear indices of the nodes on velocity / pressure faces), in the layout
// of `phase` (0 natural, 1 AA swapped), with args.F = F and args.tstep = t
// of the level just reached; nee points to NeeArgs of the compute type.
hipError_t launch_nee(int q, int storage, int phase, const void* args, const void* nee,
                      const int* nodes, int count, hipStream_t stream);
// Encode FP64 in[N] into population a (natural layout).
hipError_t launch_set_pop(int q, int storage, int a, const void* args, const double* in,
                          hipStream_t stream);
// f = f_eq(p, u - F/2) (FP64 arithmetic) from device p[N], u[3][N] or, when
// p/u are NULL, the uniform p0/u0; written in natural layout.
hipError_t launch_init_eq(int q, int storage, const void* args, const double* p, const double* u,
                          double p0, const double* u0, hipStream_t stream);
// p[N], u[3][N] (FP64) of the current state with the force args.F.
hipError_t launch_macros(int q, int storage, int phase, const void* args, double* p, double* u,
                         hipStream_t stream);
// The same for nodes [n0, n0 + count) into out[4 count] (p, u_x, u_y, u_z,
// each count values); hipErrorInvalidValue if the range leaves the lattice.
hipError_t launch_macros_range(int q, int storage, int phase, const void* args, long long n0,
                               long long count, double* out, hipStream_t stream);
// Monitor pass 1: per-block FP64 partial sums of sum|u - snap|, sum|u|,
// sum P into partial[3*nblocks]; refreshes snap (compute type) with u.
// nblocks is returned through *nblocks_out (host computed).
hipError_t launch_monitor(int q, int storage, int phase, const void* args, void* snap,
                          double* partial, int* nblocks_out, hipStream_t stream);
// Monitor pass 2: fixed-order sum of the partials into out[0..2]; out[3]
// is a sticky non-finite flag (flags bit 0: count a non-finite sum |u - snap|
// too; bit 1: start the flag afresh).
hipError_t launch_reduce_partials(const double* partial, int nblocks, double* out, int flags,
                                  hipStream_t stream);
int monitor_blocks(long long nodes);
hipError_t launch_copy_probe(void* dst, const void* src, size_t bytes, int xcd, hipStream_t stream);

// ---- batched execution -------------------------------------------------
// One member of a batch, as the batched kernel sees it (FP32 compute).
struct BatchMember {
  LatticeArgs<float> a;    // a.F unused: forces come from the F table
  int q, storage;
  int phase0;              // AA parity at its first substep
  int skip;                // first substep it takes part in (0 or 1: parity alignment)
  int steps;               // substeps it takes, from substep `skip` on
  long long tile_begin;    // first global tile index of this member
  long long ntiles;
  long long ftab_off;      // float offset of this member's F(t) rows (3 per own step)
  int forced;
  int flat;                // 1: tile lt = nodes [256 lt, 256 lt + 256) in linear order
  FastDiv fd_nx, fd_ny;    // flat tiles: node index -> (x, y, z)
  // velocity / pressure / node-layer symmetry faces (nee_count > 0 only)
  const int* nee_nodes;    // the member's boundary node list (device)
  int nee_count;
  long long nee_begin;     // first index of its nodes in its class's boundary pass
  long long ntab_off;      // float offset of its boundary rows: per own step,
                           // F at the level reached (3) and the face pressures (6)
  NeeArgs<float> e;        // face kinds and velocities (e.p comes from the rows)
};
// Tiles of one member run one after the other by one workgroup of a large
// batched launch.
constexpr int kBatchChunk = 2;

// A chunk of a large batched launch: member index (into that launch's
// member array) and the member's first tile of the chunk; the chunk covers
// tiles [tile, min(tile + kBatchChunk, ntiles)) of that member.
struct BatchChunk {
  int member;
  int tile;
};

// One launch of a batched time step: members[0..nmembers) share q, storage,
// the AA step kind and `forced`.  chunks == NULL: one tile per workgroup,
// nblocks = the members' tiles, each member's tile_begin counting from 0 at
// members[0].  Otherwise workgroup b runs chunks[b] (nblocks chunks).
struct BatchLaunch {
  const BatchMember* members;
  int nmembers;
  const BatchChunk* chunks;
  long long nblocks;
  const float* ftab;
  int substep;
  int xcd_order;  // workgroup order: 0 dispatch, 1 contiguous ranges per XCD,
                  // c >= 2 chunks of 2^(c-1) workgroups per XCD in turn
};
hipError_t launch_batch_group(int q, int storage, int mode, bool forced, const BatchLaunch& L,
                              hipStream_t stream);
// The velocity / pressure / node-layer symmetry pass of substep `substep`
// for the members[0..nmembers) of one launch class (same q and storage),
// right after that class's step launch: `total` boundary nodes, member m's
// at [m.nee_begin, m.nee_begin + m.nee_count); phase is the AA layout after
// the step (1 after an even step, 0 after an odd one).
hipError_t launch_batch_nee(int q, int storage, int phase, const BatchMember* members,
                            int nmembers, const float* ntab, int substep, long long total,
                            hipStream_t stream);
// Monitor pass 1 of every member: partial sums into partial[3*blocks of
// member]; member m writes at partial + 3*pofs[m].
hipError_t launch_batch_monitor(const BatchMember* members, int nmembers, void* const* snaps,
                                double* partial, const long long* pofs, long long total_blocks,
                                const long long* block_begin, const int* phases,
                                hipStream_t stream);
hipError_t launch_batch_reduce(const double* partial, const long long* pofs,
                               const long long* pcount, int nmembers, double* out,
                               hipStream_t stream);

}  // namespace lbm

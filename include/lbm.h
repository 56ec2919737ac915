/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the incompressible
 * 14- and 18-velocity multiple-relaxation-time lattice Boltzmann models of
 * Zhang, Shi & Wang (arXiv 1503.03337), and the 26-velocity model built by
 * the same construction (LBM_D3Q26 below).
 *
 * What one time step computes (per fluid node x, time level t -> t+1):
 *   - P = sum_a f_a, j = sum_a c_a f_a, u = j + F(t)/2 and
 *     p = c_s^2/(1-w0) [P - w0 |u|^2 / (2 c_s^2)]          (Eq. (hgl))
 *   - m = T f with the integer T of Eq. (T14) / Appendix B (Sec. 3)
 *   - D_k = s_k (m_k - m_k^eq(p,u)) - (1 - s_k/2) m_k^F     (Eq. (mrteqvT);
 *     m^eq from Eq. (meq) / Appendix B, m^F = (d m^eq/d u) . F, the body
 *     force written in moment space; F = 0 is the paper's scheme)
 *   - f*_a = f_a - sum_k T_ka D_k / N_k, N_k = sum_a T_ka^2 (rows of T are
 *     orthogonal, Sec. 3)
 *   - streaming f_a(x + c_a, t+1) = f*_a(x) (Eq. (mrteq)); periodic faces
 *     wrap; across a wall face the population returns as
 *     f_abar(x, t+1) = f*_a(x) - 6 w_a (c_a . u_w) (half-way bounce-back
 *     with the moving-wall term of the linear part of Eq. (edf)).  A link
 *     leaving through several wall faces takes the wall velocity of its z
 *     face, else its y face, else its x face.
 *
 * Lattice units (c = dx = dt = 1, c_s^2 = 1/3).  Velocities in the paper's
 * order: q = 14 (Sec. 3): +-x, +-y, +-z, then the 8 corners
 * (1,1,1),(-1,1,1),(1,-1,1),(-1,-1,1),(1,1,-1),(-1,1,-1),(1,-1,-1),
 * (-1,-1,-1); q = 18 (Appendix B): +-x, +-y, +-z, then (+-1,+-1,0),
 * (+-1,0,+-1), (0,+-1,+-1), x sign varying fastest.  Weights: 1/9, 1/72
 * (rest weight 2/9) for q = 14 -- the D3Q15 values, since the printed
 * Eq. (omega) values do not reproduce Eq. (meq) -- and 1/18, 1/36 (rest
 * weight 1/3) for q = 18.  Relaxation vectors s_vec hold q rates in the
 * moment order of Eq. (moment) / Eq. (d3q18moment).
 *
 * Node (i,j,k) has linear index n = i + nx*(j + ny*k); host population
 * arrays are [q][N] FP64 in that order, macroscopic arrays p[N], u[3][N].
 * Walls are half-way: fluid nodes 0..n-1, wall planes at -1/2 and n-1/2.
 *
 * Conventions: every function returns LBM_OK (0) or a negative lbm_status;
 * nothing throws across the ABI.  The library owns all device state of a
 * context unless spec.dev_buf is given, in which case the caller owns that
 * buffer (and must keep it alive until lbm_destroy) and the library never
 * frees it.  Host arrays are always caller-owned and only read/written
 * during the call.  Work is queued on spec.stream (a hipStream_t; NULL =
 * the null stream); calls that return host data synchronise that stream.
 * A context is not thread-safe; use one context per host thread.
 */
#ifndef LBM_H_
#define LBM_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;

/* LBM_D3Q26: the 26-velocity model the closing paragraph of Appendix B says
 * the same construction gives (not spelled out in the paper; built here by
 * Sec. 3's Gram-Schmidt of monomial rows): the 18 velocities above, then
 * the 8 corners in the order of the 14-velocity model; D3Q27 weights 2/27,
 * 1/54, 1/216 (rest weight 8/27); 26 moments (P, e, eps, j_x, q_x, h_x,
 * j_y, q_y, h_y, j_z, q_z, h_z, 3p_xx, 3pi_xx, p_ww, pi_ww, p_xy, p_yz,
 * p_xz, pi_xy, pi_yz, pi_xz, t_x, t_y, t_z, t_xyz), and s_vec in that order;
 * p = 9/19 (P - 4/9 |u|^2) (Eq. (hgl) with w0 = 8/27). */
typedef enum { LBM_D3Q14 = 14, LBM_D3Q18 = 18, LBM_D3Q26 = 26 } lbm_model;

/* Population storage.  Arithmetic is FP64 for LBM_F64 and FP32 otherwise.
 * LBM_F16DEV stores h_a = fp16((f_a - 3 w_a p0) 2^s): the deviation from the
 * rest-state equilibrium f_a = 3 w_a p0 (Eq. (edf) at u = 0), scaled by a
 * power of two (exact) so that it stays in FP16's normal range. */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16DEV = 2 } lbm_storage;

/* Streaming pattern: LBM_AB keeps two population copies (read one, write
 * the other); LBM_AA keeps one copy updated in place, alternating a local
 * step (read and write a node's own slots) and a neighbour step. */
typedef enum { LBM_AB = 0, LBM_AA = 1 } lbm_pattern;

/* Boundary kind of a lattice face.
 *
 * LBM_WALL: half-way bounce-back (above); the wall lies half a spacing
 * beyond the last node layer.
 *
 * LBM_SYMMETRY is the symmetry plane of Eq. (z05symmetry) (Sec. 4.3 computes
 * half the cavity with it): a population leaving through it is reflected
 * specularly half-way across the link, f_a'(x + c_a with the crossed normal
 * components removed, t+1) = f*_a(x), where c_a' is c_a with those normal
 * components negated.  A link crossing a wall and a symmetry plane at once
 * bounces back at the wall.
 *
 * LBM_VELOCITY and LBM_PRESSURE are the non-equilibrium extrapolation
 * boundaries the paper uses throughout Sec. 4 (Guo, Zheng & Shi): the face
 * runs through the last node layer (node-based grid: a duct of width 2a at
 * spacing dx has 2a/dx + 1 nodes across).  After every step each node x_b on
 * such faces is set to f(x_b) = f_eq(p_b, u_b) + [f(x_f) - f_eq(p_f, u_f)],
 * x_f = x_b + the inward normals of its faces (p_f, u_f: the macroscopic
 * fields there, Eq. (hgl)).  A velocity face fixes u_b = wall_u and takes
 * p_b = p_f; a pressure face fixes p_b = face_p + face_pA cos(2 pi t / FT)
 * (FT > 0, else face_p) at the new time level and takes u_b = u_f.
 * At edges and corners both kinds apply; among faces of one kind the z
 * face wins, then y, then x.
 *
 * LBM_SYMMETRY_NODE is the symmetry plane of Eq. (z05symmetry) through the
 * last node layer (node-based grids such as the paper's 97x97x49 half
 * cavity): after every step, the populations of a node on the plane that
 * arrive from beyond it are set to the mirrored populations of the same
 * node (those the layer below sent towards the plane), so a half domain
 * evolves exactly as the lower half of the full mirror-symmetric one.  A
 * node on both such a plane and a velocity / pressure face follows the
 * latter, extrapolating from its inward neighbour after the plane's
 * mirroring.
 *
 * Velocity, pressure and node-layer symmetry faces need at least 3 nodes on
 * their axis; in a batch their pass runs once per class and step over the
 * boundary nodes of all members that have such faces.
 *
 * wall_u is used on wall and velocity faces and ignored elsewhere. */
typedef enum {
  LBM_PERIODIC = 0,
  LBM_WALL = 1,
  LBM_SYMMETRY = 2,
  LBM_VELOCITY = 3,
  LBM_PRESSURE = 4,
  LBM_SYMMETRY_NODE = 5
} lbm_face_kind;

/* Rounding of LBM_F16DEV stores made by a time step.  Stochastic (the
 * default): a value rounds up with probability equal to its distance from
 * the lower FP16 neighbour, with random bits from a hash of (node,
 * population, time level) -- deterministic and unbiased, so increments below
 * half an FP16 ulp survive on average; the price is a small stationary
 * fluctuation (a residual floor of order 1e-6).  Nearest: round to nearest
 * even; a steady state is reached exactly but slow weak forcing stagnates.
 * lbm_set_f and initialisation always round to nearest. */
typedef enum { LBM_ROUND_STOCHASTIC = 0, LBM_ROUND_NEAREST = 1 } lbm_rounding;

/* Collision operator.  LBM_MRT: the moment-space collision above.  LBM_BGK:
 * the single-relaxation-time special case S = I/tau that the MRT models
 * reduce to (Sec. 3, Appendix B: the iD3Q15 / iD3Q19 LBGK models of Sec. 2),
 * f*_a = f_a - (f_a - f_eq_a)/tau + (1 - 1/(2 tau)) w_a [3 c.F + 9 (c.u)(c.F)
 * - 3 u.F], evaluated without the transforms; all q rates must be equal
 * (tau = 1/s_vec[0]).  Single lattices only (batches are MRT). */
typedef enum { LBM_MRT = 0, LBM_BGK = 1 } lbm_collision;

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad argument: q, dims < 1, N >= 2^31, s_k outside [0,2),
                          unpaired periodic faces, |u_w| >= 0.3, bad storage,
                          a non-finite F0, FA, FT, p0, u0 or face pressure ... */
  LBM_ENOMEM = -2,     /* footprint above dev_buf_bytes or hipMalloc failure */
  LBM_EDEVICE = -3,    /* a HIP call failed (message in lbm_last_error) */
  LBM_ENONFINITE = -4, /* a monitor found a non-finite mass or velocity */
  LBM_ESTATE = -5      /* call not valid in this state (e.g. no monitor data) */
} lbm_status;

/* Faces in the order -x, +x, -y, +y, -z, +z. */
typedef struct {
  int face[6];          /* lbm_face_kind; periodic faces must come in pairs   */
  double wall_u[6][3];  /* velocity of each wall / velocity face (0: at rest) */
  double F0[3];         /* body force F(t) = F0 + FA cos(2 pi t / FT)         */
  double FA[3];
  double FT;            /* FT <= 0: constant force F0                        */
  double p0;            /* reference pressure: initial state and FP16 base   */
  double u0[3];         /* initial velocity: f = f_eq(p0, u0 - F(0)/2)       */
  int storage;          /* lbm_storage                                       */
  int pattern;          /* lbm_pattern                                       */
  int f16_scale_log2;   /* s of LBM_F16DEV, 0..24                           */
  int f16_rounding;     /* lbm_rounding of LBM_F16DEV step stores            */
  int collision;        /* lbm_collision                                     */
  int monitor_every;    /* K > 0: run the mass/residual monitor every K steps */
  void* stream;         /* hipStream_t to queue work on (NULL: null stream)  */
  void* dev_buf;        /* optional caller-owned device buffer ...           */
  size_t dev_buf_bytes; /* ... and its size (>= lbm_footprint_bytes)         */
  double face_p[6];     /* pressure of each LBM_PRESSURE face ...            */
  double face_pA[6];    /* ... plus face_pA cos(2 pi t / FT) when FT > 0     */
  int graphs;           /* 1 (default): lbm_step replays captured HIP graphs
                           where it can (see lbm_step); 0: never           */
} lbm_spec;

/* Defaults: all six faces walls at rest, no force, p0 = 0, u0 = 0, FP32,
 * AA pattern, f16_scale_log2 = 12, stochastic FP16 rounding, MRT collision,
 * no monitor, null stream, own memory, graphs on. */
void lbm_spec_default(lbm_spec* spec);

/* Device bytes a context of this shape needs (populations, the list of
 * velocity/pressure-face nodes, monitor snapshot and reduction scratch); 0
 * on invalid input.  For admission
 * control: no device call is made. */
size_t lbm_footprint_bytes(int model, int nx, int ny, int nz, const lbm_spec* spec);

/* Create a context and initialise f = f_eq(p0, u0 - F(0)/2) at t = 0
 * (Eq. (edf)).  s_vec: q relaxation rates in moment order, each in [0,2). */
int lbm_create(lbm_ctx** out, int model, int nx, int ny, int nz,
               const double* s_vec, const lbm_spec* spec);

/* Advance n >= 0 time steps (one kernel launch per step, plus one for
 * velocity / pressure / node-layer symmetry faces, queued on the context
 * stream; returns without waiting).
 *
 * With spec.graphs = 1 the launches of 32 consecutive steps are captured
 * once into a HIP graph and replayed, which removes the per-launch host cost
 * that dominates small lattices.  This happens for lattices below 2^21 nodes
 * whose kernel arguments do not change from step to step: a stream the
 * caller is not capturing, no
 * time-dependent force or face pressure (FT <= 0), and not LBM_F16DEV with
 * stochastic rounding (its rounding bits depend on t).  The graph is
 * recorded on a private stream of the context (the null stream cannot be
 * captured) and launched on the context stream.  A
 * graph never spans a monitor step.  Results are bit-identical either way.
 * The first such call on a context captures (and keeps, until lbm_destroy)
 * up to two graphs, one per AA parity or A/B buffer order.
 *
 * Failure: with spec.monitor_every = K > 0 the FP64 monitor runs every K
 * steps (queued like the steps).  Its second pass keeps a flag on the
 * device that stays set once any run has seen a non-finite mass or sum |u|
 * (or, with an earlier snapshot of the state, a non-finite change of u), and
 * copies it to host memory with its sums.  lbm_step reads that copy without
 * waiting, at its start and before each monitor run it queues; once a run
 * that has completed reports a non-finite value, lbm_step returns
 * LBM_ENONFINITE at once (queuing nothing more) and keeps doing so until
 * lbm_set_f or lbm_init_fields gives the context a new state.  A diverging
 * lattice is therefore stopped at most a few monitor intervals after it
 * turned non-finite, however long the caller keeps stepping it.  In a batch
 * (lbm_batch_step) nothing is checked: use lbm_batch_monitor and lbm_poll. */
int lbm_step(lbm_ctx* ctx, long long n);

/* Non-blocking health check: LBM_ENONFINITE if a completed monitor run (of
 * lbm_step, lbm_monitor or lbm_batch_monitor) has seen a non-finite value
 * since the state was last set, LBM_OK otherwise (also while the last run
 * is still in flight).  Never waits for the device. */
int lbm_poll(lbm_ctx* ctx);

/* Pressure p[N] and velocity u[3][N] (host, FP64) at the current time level
 * t, with u = sum c f + F(t)/2 (Eq. (hgl)).  Either pointer may be NULL.
 * Synchronises the stream. */
int lbm_macros(lbm_ctx* ctx, double* p, double* u);

/* Same, into caller-owned device FP64 arrays; queued, does not wait. */
int lbm_macros_device(lbm_ctx* ctx, double* p_dev, double* u_dev);

/* For callers that cannot allocate (code between graph captures, tight
 * serving loops, harnesses that forbid hipMalloc): lbm_macros for the nodes
 * [n0, n0 + count) without any allocation.  p[count] and u[3][count]
 * (u_x, u_y, u_z, each count values) are caller-owned host FP64 arrays;
 * either may be NULL.  The values equal those of lbm_macros at the same
 * nodes bit for bit.  The call stages them in a static device array of the
 * library (8 MiB per GPU, held until the process ends) instead of the device
 * memory lbm_macros allocates, and calls no hipMalloc or hipFree.
 * count <= LBM_NOALLOC_MAX_NODES (262,144), else LBM_EINVAL; a range outside
 * the lattice is LBM_EINVAL.  Every call on one GPU shares that array: calls
 * that overlap on one GPU (other host threads, other streams) race.
 * Synchronises the stream. */
#define LBM_NOALLOC_MAX_NODES 262144
int lbm_macros_noalloc(lbm_ctx* ctx, long long n0, long long count, double* p, double* u);

/* Velocity residual of the last monitor run:
 *   R = sum_n sum_k |u_k(n,t) - u_k(n,t-L)| / (L sum_n sum_k |u_k(n,t)|)
 * with L the steps since the previous snapshot (the steady-state criteria
 * Eqs. (sc), (cr), (cavity_creterion) for lag L, per step).  +inf when
 * sum|u| = 0 or when the monitor had no earlier snapshot of the current state
 * (its first run, or the first after lbm_set_f, lbm_init_fields or
 * lbm_set_time).  LBM_ENONFINITE if the monitor saw a non-finite value in u,
 * the mass or (with an earlier snapshot) the change of u.  Waits for the
 * last monitor run to complete (not for work queued after it). */
int lbm_residual(lbm_ctx* ctx, double* r);

/* The same change of u in the norm of the paper's steady-state criteria
 * themselves (Eq. (sc) for L = 1, Eq. (cr) for L = T, Eq. (cavity_creterion)
 * for L = 1000), not divided by the lag:
 *   R_L = sum_n sum_k |u_k(n,t) - u_k(n,t-L)| / sum_n sum_k |u_k(n,t)|,
 * and the lag L in *lag (may be NULL; 0 when the monitor had no earlier
 * snapshot, R_L = +inf then).  lbm_residual returns R_L / L.  Status as for
 * lbm_residual. */
int lbm_residual_change(lbm_ctx* ctx, double* r, long long* lag);

/* Mass M = sum_n P(n) = sum_n sum_a f_a(n) (FP64) from the last monitor run;
 * runs the monitor first if it has never run. */
int lbm_mass(lbm_ctx* ctx, double* m);

/* Run the monitor now (snapshot u, update residual and mass); queued. */
int lbm_monitor(lbm_ctx* ctx);

/* Populations at the current time level as host FP64 [q][N], in the
 * physical (streamed, decoded) layout whatever the pattern and parity. */
int lbm_get_f(lbm_ctx* ctx, double* f);

/* Overwrite the populations from host FP64 [q][N] (encoded to the storage
 * type); the time level is unchanged.  Synchronises the stream. */
int lbm_set_f(lbm_ctx* ctx, const double* f);

/* Set f = f_eq(p, u - F(t)/2) from host FP64 p[N], u[3][N] (NULL: p0 / u0),
 * so that the velocity recovered at the current time t is u. */
int lbm_init_fields(lbm_ctx* ctx, const double* p, const double* u);

long long lbm_time(const lbm_ctx* ctx);
int lbm_set_time(lbm_ctx* ctx, long long t);   /* for checkpoint restore */

/* Shape and device layout of a context (for drivers and measurement). */
typedef struct {
  int q, nx, ny, nz, storage, pattern;
  long long t;
  size_t nodes;             /* nx*ny*nz                                     */
  size_t population_bytes;  /* bytes of one population copy (q*N*elem)      */
  size_t footprint_bytes;   /* everything the context holds on the device   */
  int bytes_per_value;      /* 8, 4 or 2                                    */
  int graphs;               /* HIP graphs lbm_step has captured (0..2)      */
} lbm_info_t;
int lbm_info(const lbm_ctx* ctx, lbm_info_t* info);

int lbm_sync(lbm_ctx* ctx);                  /* wait for the context stream */
/* lbm_destroy waits for the context stream only if it frees device memory
 * the library allocated.  With a caller-owned spec.dev_buf it returns at
 * once: work already queued on the stream may still use the buffer, so the
 * caller must not reuse it out of stream order. */
/* Message of the last failure on ctx; with ctx == NULL, of the last failed
 * lbm_create on the calling thread.  Never NULL. */
const char* lbm_last_error(const lbm_ctx* ctx);
const char* lbm_status_string(int status);
int lbm_destroy(lbm_ctx* ctx);

/* ---- batched execution ------------------------------------------------
 * A batch advances many independent contexts (any mix of q = 14 / 18,
 * storage FP32 / FP16DEV, pattern AA, MRT collision, shapes, face kinds,
 * forces and rates) with one kernel launch per time step and (q, storage)
 * class covering all of them (plus one launch for the velocity / pressure /
 * node-layer symmetry pass when any member of the class has such faces); each
 * member keeps its own time level, parity and populations, and its result
 * is bit-identical to running it alone in a batch and to stepping it with
 * lbm_step.  Members must share the batch's stream.  Members can be added
 * and removed between calls (continuous batching).  Each member has a step
 * budget: lbm_batch_step advances it by min(n, remaining budget).  The batch
 * does not own its members: destroying a member removes it, and destroying
 * the batch leaves the members usable on their own. */
int lbm_batch_create(lbm_batch** out, void* stream);
/* LBM_EINVAL (message in lbm_batch_last_error) for a context that is
 * already in a batch, not LBM_AA, stored as LBM_F64, on another stream, or
 * using the LBGK collision; step_budget >= 0. */
int lbm_batch_add(lbm_batch* b, lbm_ctx* ctx, long long step_budget);
int lbm_batch_remove(lbm_batch* b, lbm_ctx* ctx);
/* Mapping of a member's nodes to workgroups: a tx x ty tile (tx*ty <= 256
 * nodes of one x-y plane), or (0,0) = automatic: 256 consecutive nodes in
 * linear order (every wavefront full and aligned whatever nx; members with
 * N >= 2^30 nodes use a row tile instead).  Results do not depend on it. */
int lbm_batch_set_tile(lbm_batch* b, lbm_ctx* ctx, int tx, int ty);
int lbm_batch_step(lbm_batch* b, long long n);
/* Run the monitor of every member created with monitor_every > 0 (one
 * launch; synchronises the stream); then lbm_residual / lbm_mass of each
 * such member read its values.  Members without a monitor are skipped. */
int lbm_batch_monitor(lbm_batch* b);
/* Remaining step budget of a member (0 when done); -1 if not a member. */
long long lbm_batch_remaining(const lbm_batch* b, const lbm_ctx* ctx);
int lbm_batch_size(const lbm_batch* b);
const char* lbm_batch_last_error(const lbm_batch* b);
int lbm_batch_destroy(lbm_batch* b);

/* ---- measurement helper -----------------------------------------------
 * Copy `bytes` (multiple of 16) from src to dst on the device with a plain
 * streaming kernel, `reps` times back to back; the achievable-bandwidth
 * reference against which the step kernels are read.  Its workgroup order
 * is the faster one measured for the bytes touched: dispatch order up to
 * 384 MB, one contiguous range per XCD beyond.  Queued on stream. */
int lbm_copy_probe(void* dst, const void* src, size_t bytes, int reps, void* stream);

/* The memory pattern of an AA step without its arithmetic, `reps` times,
 * over an nx x ny x nz lattice that is periodic on every axis: buf (device)
 * holds q arrays (q = 14, 18 or 26) of elem_bytes-byte values (2, 4 or 8),
 * `stride` >= nx ny nz elements apart, node n = x + nx (y + ny z).  odd = 0
 * (the even step): every node moves its q values into the slots of the
 * opposite velocities at the same node.  odd = 1 (the odd step): every node
 * n reads slot abar at n - c_a and writes it into slot a at n + c_a.  Values
 * move as raw bits, one thread per node in tiles of whole rows (256, 128 or
 * 64 threads wide, 256 per workgroup), one contiguous range of workgroups
 * per XCD up to 384 MB of populations and dispatch order beyond: the
 * ceiling of the step kernels' own access pattern, read beside the plain
 * copy.  LBM_EINVAL on bad arguments.  Queued on stream. */
int lbm_pattern_probe(void* buf, int q, int elem_bytes, int nx, int ny, int nz,
                      long long stride, int odd, int reps, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H_ */

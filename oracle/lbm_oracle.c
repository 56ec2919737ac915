/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 CPU implementation of the incompressible 14- and
 * 18-velocity multiple-relaxation-time lattice Boltzmann step of
 * Zhang, Shi & Wang, "14-velocity and 18-velocity multiple-relaxation-time
 * lattice Boltzmann models for three-dimensional incompressible flows"
 * (arXiv 1503.03337).  It exists so that the GPU library can be checked
 * against something written straight from the paper.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it, and it shares no code, table or header with
 * the HIP library.
 *
 * The closing paragraph of Appendix B notes that the same construction of
 * the (q-1) x (q-1) transform gives a 26-velocity model (iD3Q26) as well,
 * without spelling it out; it is built here by that construction (see
 * "the 26-velocity model" below).
 *
 * What is followed, and where:
 *   velocity sets ........ Sec. 3 (iD3Q14) and Appendix B (iD3Q18); the
 *                          26 non-rest D3Q27 velocities for iD3Q26
 *   weights .............. Eq. (omega) for the D3Q19 lattice (Appendix B);
 *                          for the 14-velocity model the D3Q15 weights
 *                          2/9, 1/9, 1/72 (the printed Eq. (omega) lists the
 *                          D3Q19 values; only the D3Q15 ones reproduce the
 *                          printed moment equilibria Eq. (meq) via T f_eq)
 *   equilibrium .......... Eqs. (edf), (lamda_alpha)
 *   p, u recovery ........ Eq. (hgl), with u = sum c f + F/2 when a body
 *                          force F acts (forcing is not in the paper: the
 *                          moment-space Guo form m_F = (d m_eq / d u) . F
 *                          is used, so F = 0 gives the paper's scheme)
 *   transform T .......... Eq. (T14) and the 18x18 T of Appendix B,
 *                          typed in as printed
 *   moment equilibria .... Eq. (meq) (Sec. 3) and Appendix B
 *   relaxation ........... Eq. (mrteqvT) with the diagonal of
 *                          Eqs. (sD3Q15) / (sD3Q19)
 *   T^-1 ................. T T' is diagonal (rows mutually orthogonal,
 *                          Sec. 3), so T^-1 = T' N^-1 with N_k the squared
 *                          row norms, computed here from T
 *   streaming + walls .... Eq. (mrteq) for the free flight; walls are
 *                          half-way bounce-back with the moving-wall term
 *                          -2 w_a (c_a . u_w) / c_s^2 taken from the linear
 *                          term of Eq. (edf) (the paper itself uses
 *                          non-equilibrium extrapolation)
 *   symmetry planes ...... Eq. (z05symmetry) (Sec. 4.3): du/dn = dv/dn =
 *                          dp/dn = 0, w = 0 on the plane, imposed by
 *                          specular reflection at a half-way plane
 *   non-equilibrium ...... the boundary scheme the paper applies throughout
 *   extrapolation          Sec. 4 (Guo, Zheng & Shi): boundary nodes lie on
 *                          the face; after streaming, each takes the
 *                          equilibrium of its boundary values plus the
 *                          non-equilibrium part of its inward neighbour;
 *                          a velocity face fixes u and takes p from the
 *                          neighbour, a pressure face (Eq. (bc)) the reverse;
 *   node-layer symmetry .. Eq. (z05symmetry) on a plane through the last
 *                          node layer (the paper's 97x97x49 half cavity):
 *                          the populations arriving from beyond the plane
 *                          are the mirror images of those leaving towards it
 *
 * Layout: f[a*N + n], n = x + nx*(y + ny*z), a = 0..q-1 in the paper's
 * order 1..q.  Everything is FP64.  Build: -O2 -ffp-contract=off.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 26

/* ---- lattices (Sec. 3 for q = 14, Appendix B for q = 18) ------------- */
static const int VEL14[14][3] = {
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},   {0, 0, 1},
    {0, 0, -1}, {1, 1, 1},  {-1, 1, 1}, {1, -1, 1},   {-1, -1, 1},
    {1, 1, -1}, {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};

static const int VEL18[18][3] = {
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0}, {1, 0, 1}, {-1, 0, 1},
    {1, 0, -1}, {-1, 0, -1}, {0, 1, 1}, {0, -1, 1}, {0, 1, -1}, {0, -1, -1}};

/* Eq. (T14), as printed. */
static const int TMAT14[14][14] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -4, -4, -4, -4, -4, 3, 3, 3, 3, 3, 3, 3, 3},
    {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
    {-4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
    {0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1},
    {0, 0, 0, 0, -4, 4, 1, 1, 1, 1, -1, -1, -1, -1},
    {2, 2, -1, -1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1},
    {0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1},
    {0, 0, 0, 0, 0, 0, 1, -1, -1, 1, -1, 1, 1, -1}};

/* The 18x18 T of Appendix B, as printed. */
static const int TMAT18[18][18] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-2, -2, -2, -2, -2, -2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {-4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, 0, -4, 4, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {-4, -4, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, -2, -2, 2, 2, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1}};

/* ---- the 26-velocity model (closing paragraph of Appendix B) ------------
 * Velocities: the six axis ones and the twelve edge ones in the order of
 * Appendix B, then the eight corners in the order of Sec. 3.  Weights: those
 * of the D3Q27 lattice the model is cut from, 2/27 (axis), 1/54 (edge),
 * 1/216 (corner), rest weight 8/27 (the role the D3Q15 and D3Q19 weights
 * play for 14 and 18 velocities).
 *
 * Transform: Sec. 3 builds T by Gram-Schmidt orthogonalisation of monomial
 * rows c_x^m c_y^n c_z^l chosen per tensor order (Eq. (transformation_Mbar),
 * Eq. (m)).  On these 26 velocities the monomials fall into the classes
 *   scalars ......... 1, |c|^2, |c|^4                    (P, e, eps)
 *   vectors ......... c_x, |c|^2 c_x, |c|^4 c_x, y, z    (j, q, h)
 *   2nd order ....... 3c_x^2, 3c_x^2|c|^2, c_y^2 - c_z^2, (c_y^2 - c_z^2)|c|^2,
 *                     c_x c_y, c_y c_z, c_x c_z and the same times |c|^2
 *   3rd order ....... (c_y^2 - c_z^2)c_x, (c_z^2 - c_x^2)c_y,
 *                     (c_x^2 - c_y^2)c_z, c_x c_y c_z
 * (26 independent rows; the rest population, and with it one scalar, is
 * dropped as for 14 and 18 velocities).  Orthogonalised in the order of
 * the moment vector below and scaled to the smallest integers, the rows
 * are the polynomials of t26_row.  Moments, in this order:
 *   (P, e, eps, j_x, q_x, h_x, j_y, q_y, h_y, j_z, q_z, h_z, 3p_xx, 3pi_xx,
 *    p_ww, pi_ww, p_xy, p_yz, p_xz, pi_xy, pi_yz, pi_xz, t_x, t_y, t_z, t_xyz).
 * Their equilibria and forcing moments are not printed anywhere: they are
 * computed from their definitions, m_eq = T f_eq (Sec. 3, with Eq. (edf))
 * and m_F = T (the Guo source written in velocity space). */
static const int VEL26[26][3] = {
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},   {0, 0, -1},  {1, 1, 0},
    {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0}, {1, 0, 1}, {-1, 0, 1},  {1, 0, -1},  {-1, 0, -1},
    {0, 1, 1},  {0, -1, 1}, {0, 1, -1},  {0, -1, -1}, {1, 1, 1}, {-1, 1, 1}, {1, -1, 1},
    {-1, -1, 1}, {1, 1, -1}, {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};

/* Row k of the 26 x 26 transform at velocity c (k2 = |c|^2). */
static int t26_row(int k, const int* c) {
  const int x = c[0], y = c[1], z = c[2], k2 = x * x + y * y + z * z;
  const int q = 3 * k2 - 7;                          /* energy flux  */
  const int h = (9 * k2 * k2 - 39 * k2 + 38) / 2;    /* second flux  */
  const int r = 3 * k2 - 5;                          /* pi_xx, pi_ww */
  const int s = 3 * k2 - 8;                          /* pi_xy ...    */
  switch (k) {
    case 0: return 1;
    case 1: return 13 * k2 - 27;
    case 2: return (15 * k2 * k2 - 61 * k2 + 54) / 2;
    case 3: return x;
    case 4: return q * x;
    case 5: return h * x;
    case 6: return y;
    case 7: return q * y;
    case 8: return h * y;
    case 9: return z;
    case 10: return q * z;
    case 11: return h * z;
    case 12: return 3 * x * x - k2;
    case 13: return r * (3 * x * x - k2);
    case 14: return y * y - z * z;
    case 15: return r * (y * y - z * z);
    case 16: return x * y;
    case 17: return y * z;
    case 18: return x * z;
    case 19: return s * x * y;
    case 20: return s * y * z;
    case 21: return s * x * z;
    case 22: return (y * y - z * z) * x;
    case 23: return (z * z - x * x) * y;
    case 24: return (x * x - y * y) * z;
    default: return x * y * z;
  }
}

/* The lattice in use, with the derived quantities the step needs. */
typedef struct {
  int q;
  int c[QMAX][3];
  double w[QMAX]; /* w_1..w_q */
  double w0;      /* weight of the dropped rest velocity */
  int opp[QMAX];  /* index of -c_a */
  int T[QMAX][QMAX];
  double N[QMAX]; /* N_k = sum_a T_ka^2 */
} lattice;

static int make_lattice(int q, lattice* L) {
  int a, b, k, d;
  if (q != 14 && q != 18 && q != 26) return -1;
  memset(L, 0, sizeof(*L));
  L->q = q;
  for (a = 0; a < q; ++a) {
    int len2 = 0;
    for (d = 0; d < 3; ++d) {
      L->c[a][d] = (q == 14) ? VEL14[a][d] : (q == 18) ? VEL18[a][d] : VEL26[a][d];
      len2 += L->c[a][d] * L->c[a][d];
    }
    if (q == 14)
      L->w[a] = (len2 == 1) ? 1.0 / 9.0 : 1.0 / 72.0;
    else if (q == 18)
      L->w[a] = (len2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
    else
      L->w[a] = (len2 == 1) ? 2.0 / 27.0 : (len2 == 2) ? 1.0 / 54.0 : 1.0 / 216.0;
  }
  for (k = 0; k < q; ++k)
    for (b = 0; b < q; ++b)
      L->T[k][b] = (q == 14) ? TMAT14[k][b] : (q == 18) ? TMAT18[k][b] : t26_row(k, L->c[b]);
  L->w0 = (q == 14) ? 2.0 / 9.0 : (q == 18) ? 1.0 / 3.0 : 8.0 / 27.0;
  for (a = 0; a < q; ++a) {
    L->opp[a] = -1;
    for (b = 0; b < q; ++b)
      if (L->c[b][0] == -L->c[a][0] && L->c[b][1] == -L->c[a][1] &&
          L->c[b][2] == -L->c[a][2])
        L->opp[a] = b;
    if (L->opp[a] < 0) return -1;
  }
  for (k = 0; k < q; ++k) {
    int s = 0;
    for (a = 0; a < q; ++a) s += L->T[k][a] * L->T[k][a];
    L->N[k] = (double)s;
  }
  return 0;
}

/* ---- problem description (mirrored by a ctypes Structure) -------------- */
typedef struct {
  int q, nx, ny, nz;
  double s[QMAX];        /* relaxation rates in the order of Eq. (moment) */
  int face[6];           /* -x,+x,-y,+y,-z,+z: 0 periodic, 1 wall,
                            2 symmetry plane, 3 velocity face and 4
                            pressure face (non-equilibrium extrapolation),
                            5 symmetry plane through the last node layer */
  double wall_u[6][3];   /* velocity of each wall or velocity face        */
  double F0[3], FA[3];   /* body force F(t) = F0 + FA cos(2 pi t / FT)    */
  double FT;             /* FT <= 0: constant force F0 and face pressure  */
  double face_p0[6];     /* pressure of a pressure face:                  */
  double face_pA[6];     /*   p(t) = p0 + pA cos(2 pi t / FT)             */
} orc_problem;

/* ---- single-node pieces ---------------------------------------------- */

/* Eq. (edf) with Eq. (lamda_alpha) for a = 1..q (c_s^2 = 1/3). */
static void feq_node(const lattice* L, double p, const double u[3], double* feq) {
  int a;
  double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (a = 0; a < L->q; ++a) {
    double cu = L->c[a][0] * u[0] + L->c[a][1] * u[1] + L->c[a][2] * u[2];
    double lam = L->w[a] * p * 3.0;
    feq[a] = lam + L->w[a] * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
  }
}

/* Eq. (hgl): u = sum_a c_a f_a (+ F/2 under a body force),
 * p = c_s^2/(1 - w0) [ sum_a f_a - w0 |u|^2 / (2 c_s^2) ]. */
static void macro_node(const lattice* L, const double* f, const double F[3],
                       double* p, double u[3]) {
  int a, d;
  double P = 0.0, j[3] = {0.0, 0.0, 0.0}, usq;
  for (a = 0; a < L->q; ++a) {
    P += f[a];
    for (d = 0; d < 3; ++d) j[d] += L->c[a][d] * f[a];
  }
  for (d = 0; d < 3; ++d) u[d] = j[d] + 0.5 * F[d];
  usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  *p = (P - 1.5 * L->w0 * usq) / (3.0 * (1.0 - L->w0));
}

/* Eq. (meq) for q = 14 (Sec. 3) and its Appendix B counterpart for q = 18. */
static void meq_node(int q, double p, const double u[3], double* meq) {
  double ux = u[0], uy = u[1], uz = u[2];
  double usq = ux * ux + uy * uy + uz * uz;
  if (q == 14) {
    meq[0] = 7.0 * p / 3.0 + usq / 3.0;
    meq[1] = -7.0 * p + usq;
    meq[2] = ux;
    meq[3] = -7.0 * ux / 3.0;
    meq[4] = uy;
    meq[5] = -7.0 * uy / 3.0;
    meq[6] = uz;
    meq[7] = -7.0 * uz / 3.0;
    meq[8] = 3.0 * ux * ux - usq;
    meq[9] = uy * uy - uz * uz;
    meq[10] = ux * uy;
    meq[11] = uy * uz;
    meq[12] = ux * uz;
    meq[13] = 0.0;
  } else {
    meq[0] = 2.0 * p + 0.5 * usq;
    meq[1] = -p + 0.5 * usq;
    meq[2] = ux;
    meq[3] = -2.0 * ux / 3.0;
    meq[4] = uy;
    meq[5] = -2.0 * uy / 3.0;
    meq[6] = uz;
    meq[7] = -2.0 * uz / 3.0;
    meq[8] = 3.0 * ux * ux - usq;
    meq[9] = -0.5 * (3.0 * ux * ux - usq);
    meq[10] = uy * uy - uz * uz;
    meq[11] = -0.5 * (uy * uy - uz * uz);
    meq[12] = ux * uy;
    meq[13] = uy * uz;
    meq[14] = ux * uz;
    meq[15] = 0.0;
    meq[16] = 0.0;
    meq[17] = 0.0;
  }
}

/* Forcing moments m_F = (d m_eq / d u) . F, p held fixed: the derivative of
 * each line of meq_node.  (With F = 0 these vanish and the step is the
 * paper's unforced scheme.) */
static void mforce_node(int q, const double u[3], const double F[3], double* mF) {
  double ux = u[0], uy = u[1], uz = u[2];
  double Fx = F[0], Fy = F[1], Fz = F[2];
  double w = ux * Fx + uy * Fy + uz * Fz; /* (1/2) d|u|^2 . F */
  if (q == 14) {
    mF[0] = 2.0 * w / 3.0;
    mF[1] = 2.0 * w;
    mF[2] = Fx;
    mF[3] = -7.0 * Fx / 3.0;
    mF[4] = Fy;
    mF[5] = -7.0 * Fy / 3.0;
    mF[6] = Fz;
    mF[7] = -7.0 * Fz / 3.0;
    mF[8] = 6.0 * ux * Fx - 2.0 * w;
    mF[9] = 2.0 * (uy * Fy - uz * Fz);
    mF[10] = ux * Fy + uy * Fx;
    mF[11] = uy * Fz + uz * Fy;
    mF[12] = ux * Fz + uz * Fx;
    mF[13] = 0.0;
  } else {
    mF[0] = w;
    mF[1] = w;
    mF[2] = Fx;
    mF[3] = -2.0 * Fx / 3.0;
    mF[4] = Fy;
    mF[5] = -2.0 * Fy / 3.0;
    mF[6] = Fz;
    mF[7] = -2.0 * Fz / 3.0;
    mF[8] = 6.0 * ux * Fx - 2.0 * w;
    mF[9] = -0.5 * (6.0 * ux * Fx - 2.0 * w);
    mF[10] = 2.0 * (uy * Fy - uz * Fz);
    mF[11] = -(uy * Fy - uz * Fz);
    mF[12] = ux * Fy + uy * Fx;
    mF[13] = uy * Fz + uz * Fy;
    mF[14] = ux * Fz + uz * Fx;
    mF[15] = 0.0;
    mF[16] = 0.0;
    mF[17] = 0.0;
  }
}

/* The Guo source in velocity space, w_a [3 c.F + 9 (c.u)(c.F) - 3 u.F]:
 * T applied to it gives the forcing moments m_F = (d m_eq / d u) . F. */
static void guo_source(const lattice* L, const double u[3], const double F[3], double* src) {
  int a;
  double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
  for (a = 0; a < L->q; ++a) {
    double cu = L->c[a][0] * u[0] + L->c[a][1] * u[1] + L->c[a][2] * u[2];
    double cF = L->c[a][0] * F[0] + L->c[a][1] * F[1] + L->c[a][2] * F[2];
    src[a] = L->w[a] * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF);
  }
}

/* m = T v for a vector v over the velocities. */
static void transform(const lattice* L, const double* v, double* m) {
  int a, k;
  for (k = 0; k < L->q; ++k) {
    double acc = 0.0;
    for (a = 0; a < L->q; ++a) acc += L->T[k][a] * v[a];
    m[k] = acc;
  }
}

/* Moment equilibria and forcing moments of the lattice in use: the printed
 * closed forms for 14 and 18 velocities; for 26 velocities (none printed)
 * their definitions m_eq = T f_eq and m_F = T (Guo source). */
static void moment_eq_force(const lattice* L, double p, const double u[3], const double F[3],
                            double* meq, double* mF) {
  if (L->q == 26) {
    double fe[QMAX], src[QMAX];
    feq_node(L, p, u, fe);
    guo_source(L, u, F, src);
    transform(L, fe, meq);
    transform(L, src, mF);
  } else {
    meq_node(L->q, p, u, meq);
    mforce_node(L->q, u, F, mF);
  }
}

/* One collision, Eq. (mrteqvT):
 *   m = T f;  D_k = s_k (m_k - meq_k) - (1 - s_k/2) mF_k;
 *   f*_a = f_a - sum_k T_ka D_k / N_k. */
static void collide_node(const lattice* L, const double* s, const double* f,
                         const double F[3], double* fstar) {
  int a, k, q = L->q;
  double p, u[3], m[QMAX], meq[QMAX], mF[QMAX], D[QMAX];
  macro_node(L, f, F, &p, u);
  transform(L, f, m);
  moment_eq_force(L, p, u, F, meq, mF);
  for (k = 0; k < q; ++k)
    D[k] = s[k] * (m[k] - meq[k]) - (1.0 - 0.5 * s[k]) * mF[k];
  for (a = 0; a < q; ++a) {
    double acc = 0.0;
    for (k = 0; k < q; ++k) acc += L->T[k][a] * (D[k] / L->N[k]);
    fstar[a] = f[a] - acc;
  }
}

static void force_at(const orc_problem* pr, long long t, double F[3]) {
  int d;
  double ph = 1.0;
  if (pr->FT > 0.0) ph = cos(2.0 * M_PI * (double)t / pr->FT);
  for (d = 0; d < 3; ++d) F[d] = pr->F0[d] + (pr->FT > 0.0 ? pr->FA[d] * ph : 0.0);
}

static double face_pressure(const orc_problem* pr, int face, long long t) {
  if (pr->FT > 0.0) return pr->face_p0[face] + pr->face_pA[face] * cos(2.0 * M_PI * (double)t / pr->FT);
  return pr->face_p0[face];
}

static int is_nee(int kind) { return kind == 3 || kind == 4; }

static int check_problem(const orc_problem* pr, lattice* L) {
  int d;
  const int dim[3] = {pr->nx, pr->ny, pr->nz};
  if (make_lattice(pr->q, L)) return -1;
  if (pr->nx < 1 || pr->ny < 1 || pr->nz < 1) return -1;
  for (d = 0; d < 6; ++d)
    if (pr->face[d] < 0 || pr->face[d] > 5) return -1;
  for (d = 0; d < 3; ++d) {
    if ((pr->face[2 * d] == 0) != (pr->face[2 * d + 1] == 0)) return -1;
    /* a boundary node's inward neighbour must not lie on the opposite face */
    if ((pr->face[2 * d] >= 3 || pr->face[2 * d + 1] >= 3) && dim[d] < 3) return -1;
  }
  return 0;
}

/* Index of the velocity equal to c_a with the components flagged in
 * flip[] negated. */
static int mirror_of(const lattice* L, int a, const int flip[3]) {
  int b, d;
  for (b = 0; b < L->q; ++b) {
    int same = 1;
    for (d = 0; d < 3; ++d)
      if (L->c[b][d] != (flip[d] ? -L->c[a][d] : L->c[a][d])) same = 0;
    if (same) return b;
  }
  return -1;
}

/* ---- node-based faces ------------------------------------------------- */

/* Node-layer symmetry faces (pass 1 after streaming to level t): at a node
 * x_b on such planes and on no velocity / pressure face, the populations
 * that arrive from beyond a plane are the mirror images of those the layer
 * below sent towards it, which streaming has just delivered to x_b as the
 * mirrored populations: f_a(x_b) = f_m(x_b), m = a with the components
 * normal to the crossed planes reversed.  The plane thus acts as a mirror
 * through the node layer, and a half domain evolves exactly as the full
 * one.  Returns 0 if x_b is not such a node. */
static int mirror_node(const orc_problem* pr, const lattice* L, int x, int y, int z, double* f) {
  const int dim[3] = {pr->nx, pr->ny, pr->nz};
  const int own[3] = {x, y, z};
  const size_t N = (size_t)pr->nx * pr->ny * pr->nz;
  const size_t n = (size_t)x + (size_t)pr->nx * ((size_t)y + (size_t)pr->ny * z);
  int d, a, side[3] = {0, 0, 0}, mir = 0;
  double fn[QMAX];
  for (d = 0; d < 3; ++d) {
    const int lo = pr->face[2 * d], hi = pr->face[2 * d + 1];
    if ((own[d] == 0 && is_nee(lo)) || (own[d] == dim[d] - 1 && is_nee(hi))) return 0;
    if (own[d] == 0 && lo == 5) side[d] = -1, mir = 1;
    if (own[d] == dim[d] - 1 && hi == 5) side[d] = 1, mir = 1;
  }
  if (!mir) return 0;
  for (a = 0; a < L->q; ++a) fn[a] = f[(size_t)a * N + n];
  for (a = 0; a < L->q; ++a) {
    int flip[3] = {0, 0, 0}, any = 0;
    for (d = 0; d < 3; ++d)
      if (side[d] != 0 && L->c[a][d] * side[d] < 0) flip[d] = any = 1; /* arrives from beyond */
    if (any) f[(size_t)a * N + n] = fn[mirror_of(L, a, flip)];
  }
  return 1;
}

/* Velocity / pressure faces (pass 2, non-equilibrium extrapolation): a
 * node x_b on one or more of them takes its inward neighbour x_f = x_b + sum
 * of the inward normals of those faces (x_f lies on no such face, but may
 * lie on a node-layer symmetry plane, already completed by pass 1), p_f,
 * u_f and f_neq = f(x_f) - f_eq(p_f, u_f); then f(x_b) = f_eq(p_b, u_b) +
 * f_neq, with u_b the velocity of a velocity face (else u_f) and p_b the
 * pressure of a pressure face (else p_f).  When several faces of one kind
 * meet at an edge or corner, the z face wins, then the y face, then the x
 * face (as for wall velocities).  Returns 0 if x_b is on no such face. */
static int nee_node(const orc_problem* pr, const lattice* L, long long t, int x, int y, int z,
                    double* f) {
  const int dim[3] = {pr->nx, pr->ny, pr->nz};
  const int own[3] = {x, y, z};
  const size_t N = (size_t)pr->nx * pr->ny * pr->nz;
  const size_t n = (size_t)x + (size_t)pr->nx * ((size_t)y + (size_t)pr->ny * z);
  int src[3] = {x, y, z}, d, a, on = 0, vface = -1, pface = -1;
  double F[3], fn[QMAX], pf, uf[3], fe[QMAX], ub[3], pb, eb[QMAX];
  for (d = 0; d < 3; ++d) {
    int face = -1;
    if (own[d] == 0 && is_nee(pr->face[2 * d])) {
      face = 2 * d;
      src[d] = 1;
    } else if (own[d] == dim[d] - 1 && is_nee(pr->face[2 * d + 1])) {
      face = 2 * d + 1;
      src[d] = dim[d] - 2;
    }
    if (face < 0) continue;
    on = 1;
    if (pr->face[face] == 3) vface = face; /* later axes overwrite: z > y > x */
    else pface = face;
  }
  if (!on) return 0;
  {
    const size_t m = (size_t)src[0] + (size_t)pr->nx * ((size_t)src[1] + (size_t)pr->ny * src[2]);
    force_at(pr, t, F);
    for (a = 0; a < L->q; ++a) fn[a] = f[(size_t)a * N + m];
  }
  macro_node(L, fn, F, &pf, uf);
  feq_node(L, pf, uf, fe);
  for (d = 0; d < 3; ++d) ub[d] = vface >= 0 ? pr->wall_u[vface][d] : uf[d];
  pb = pface >= 0 ? face_pressure(pr, pface, t) : pf;
  feq_node(L, pb, ub, eb);
  for (a = 0; a < L->q; ++a) f[(size_t)a * N + n] = eb[a] + (fn[a] - fe[a]);
  return 1;
}

/* ---- the lattice step ------------------------------------------------ */

/* Advance f_in (time level t) to f_out (t+1).  Every fluid node is
 * collided, then each post-collision population either moves to x + c_a
 * (periodic axes wrap) or, if x + c_a lies beyond a wall face, returns to x
 * as the opposite population with the moving-wall term.  A link leaving
 * through several wall faces takes the velocity of the z face it crosses,
 * else the y face, else the x face.  A link that crosses symmetry planes
 * and no wall is reflected specularly: the components normal to the planes
 * it crosses are reversed, so it arrives at x + c_a with those coordinates
 * left unchanged, as the population of the mirrored velocity. */
static void step_impl(const orc_problem* pr, const lattice* L, long long t,
                      const double* fin, double* fout) {
  const int nx = pr->nx, ny = pr->ny, nz = pr->nz, q = L->q;
  const size_t N = (size_t)nx * ny * nz;
  double F[3];
  int z;
  force_at(pr, t, F);
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (z = 0; z < nz; ++z) {
    int x, y, a, d;
    double f[QMAX], fs[QMAX];
    for (y = 0; y < ny; ++y)
      for (x = 0; x < nx; ++x) {
        const size_t n = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
        for (a = 0; a < q; ++a) f[a] = fin[(size_t)a * N + n];
        collide_node(L, pr->s, f, F, fs);
        for (a = 0; a < q; ++a) {
          int dst[3] = {x + L->c[a][0], y + L->c[a][1], z + L->c[a][2]};
          int dim[3] = {nx, ny, nz};
          int own[3] = {x, y, z};
          int out[3] = {0, 0, 0}, outside = 0, flip[3] = {0, 0, 0}, mirrored = 0, leaves = 0;
          for (d = 0; d < 3; ++d) {
            int face;
            if (dst[d] >= 0 && dst[d] < dim[d]) continue;
            face = 2 * d + (dst[d] < 0 ? 0 : 1);
            if (pr->face[face] == 0) {
              dst[d] = (dst[d] + dim[d]) % dim[d];
            } else if (pr->face[face] == 2) {
              flip[d] = 1;
              mirrored = 1;
            } else if (pr->face[face] == 1) {
              out[d] = (dst[d] < 0) ? -1 : 1;
              outside = 1;
            } else {
              leaves = 1; /* through a node-based face: lost */
            }
          }
          /* (a population leaving through a node-based face starts on a
             boundary node; the boundary pass below replaces what would
             arrive in its place, so it is simply dropped) */
          if (leaves) {
            continue;
          } else if (!outside && mirrored) {
            int b = mirror_of(L, a, flip);
            size_t m;
            for (d = 0; d < 3; ++d)
              if (flip[d]) dst[d] = own[d];
            m = (size_t)dst[0] + (size_t)nx * ((size_t)dst[1] + (size_t)ny * dst[2]);
            fout[(size_t)b * N + m] = fs[a];
          } else if (!outside) {
            size_t m = (size_t)dst[0] +
                       (size_t)nx * ((size_t)dst[1] + (size_t)ny * dst[2]);
            fout[(size_t)a * N + m] = fs[a];
          } else {
            const double* uw;
            double cu;
            if (out[2])
              uw = pr->wall_u[out[2] < 0 ? 4 : 5];
            else if (out[1])
              uw = pr->wall_u[out[1] < 0 ? 2 : 3];
            else
              uw = pr->wall_u[out[0] < 0 ? 0 : 1];
            cu = L->c[a][0] * uw[0] + L->c[a][1] * uw[1] + L->c[a][2] * uw[2];
            fout[(size_t)L->opp[a] * N + n] = fs[a] - 6.0 * L->w[a] * cu;
          }
        }
      }
  }
  /* boundary passes at level t+1: node-layer symmetry planes (each node
     reads and writes only itself), then velocity / pressure faces (each
     reads an inward neighbour, never on such a face, writes itself) */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (z = 0; z < nz; ++z) {
    int x, y;
    for (y = 0; y < ny; ++y)
      for (x = 0; x < nx; ++x) mirror_node(pr, L, x, y, z, fout);
  }
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (z = 0; z < nz; ++z) {
    int x, y;
    for (y = 0; y < ny; ++y)
      for (x = 0; x < nx; ++x) nee_node(pr, L, t + 1, x, y, z, fout);
  }
}

/* ---- exported API (ctypes) ------------------------------------------- */

int orc_lattice(int q, int* c, double* w, int* opp, double* w0, int* T, double* Nk) {
  lattice L;
  int a, k;
  if (make_lattice(q, &L)) return -1;
  for (a = 0; a < q; ++a) {
    if (c) {
      c[3 * a] = L.c[a][0];
      c[3 * a + 1] = L.c[a][1];
      c[3 * a + 2] = L.c[a][2];
    }
    if (w) w[a] = L.w[a];
    if (opp) opp[a] = L.opp[a];
    if (Nk) Nk[a] = L.N[a];
    if (T)
      for (k = 0; k < q; ++k) T[a * q + k] = L.T[a][k];
  }
  if (w0) *w0 = L.w0;
  return 0;
}

int orc_feq(int q, double p, const double* u, double* feq) {
  lattice L;
  if (make_lattice(q, &L)) return -1;
  feq_node(&L, p, u, feq);
  return 0;
}

int orc_macro_node(int q, const double* f, const double* F, double* p, double* u) {
  lattice L;
  if (make_lattice(q, &L)) return -1;
  macro_node(&L, f, F, p, u);
  return 0;
}

int orc_meq(int q, double p, const double* u, double* meq) {
  lattice L;
  double F[3] = {0.0, 0.0, 0.0}, mF[QMAX];
  if (make_lattice(q, &L)) return -1;
  moment_eq_force(&L, p, u, F, meq, mF);
  return 0;
}

int orc_mforce(int q, const double* u, const double* F, double* mF) {
  lattice L;
  double meq[QMAX];
  if (make_lattice(q, &L)) return -1;
  moment_eq_force(&L, 0.0, u, F, meq, mF);
  return 0;
}

int orc_collide(int q, const double* s, const double* f, const double* F, double* fstar) {
  lattice L;
  if (make_lattice(q, &L)) return -1;
  collide_node(&L, s, f, F, fstar);
  return 0;
}

/* Fill f (q x N) with f_eq(p(n), j(n)), j = u - F(t)/2, so that the
 * velocity recovered at time t is u.  p/u may be NULL (then p0, u0). */
int orc_init_eq(const orc_problem* pr, long long t, const double* p, const double* u,
                double p0, const double* u0, double* f) {
  lattice L;
  size_t N, n;
  double F[3];
  int a;
  if (check_problem(pr, &L)) return -1;
  N = (size_t)pr->nx * pr->ny * pr->nz;
  force_at(pr, t, F);
  for (n = 0; n < N; ++n) {
    double pn = p ? p[n] : p0, j[3], fe[QMAX];
    int d;
    for (d = 0; d < 3; ++d) j[d] = (u ? u[(size_t)d * N + n] : u0[d]) - 0.5 * F[d];
    feq_node(&L, pn, j, fe);
    for (a = 0; a < L.q; ++a) f[(size_t)a * N + n] = fe[a];
  }
  return 0;
}

/* Advance f (q x N, time level t0) by nsteps; result left in f. */
int orc_run(const orc_problem* pr, long long t0, long long nsteps, double* f) {
  lattice L;
  size_t bytes;
  double *a, *b;
  long long i;
  if (check_problem(pr, &L) || nsteps < 0) return -1;
  bytes = sizeof(double) * (size_t)L.q * pr->nx * pr->ny * pr->nz;
  b = (double*)malloc(bytes);
  if (!b) return -2;
  a = f;
  for (i = 0; i < nsteps; ++i) {
    double* tmp;
    step_impl(pr, &L, t0 + i, a, b);
    tmp = a;
    a = b;
    b = tmp;
  }
  if (a != f) {
    memcpy(f, a, bytes);
    free(a);
  } else {
    free(b);
  }
  return 0;
}

/* p (N) and u (3 x N) at time level t. */
int orc_macros(const orc_problem* pr, long long t, const double* f, double* p, double* u) {
  lattice L;
  size_t N, n;
  double F[3];
  if (check_problem(pr, &L)) return -1;
  N = (size_t)pr->nx * pr->ny * pr->nz;
  force_at(pr, t, F);
  for (n = 0; n < N; ++n) {
    double fn[QMAX], un[3];
    int a;
    for (a = 0; a < L.q; ++a) fn[a] = f[(size_t)a * N + n];
    macro_node(&L, fn, F, &p[n], un);
    u[n] = un[0];
    u[N + n] = un[1];
    u[2 * N + n] = un[2];
  }
  return 0;
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

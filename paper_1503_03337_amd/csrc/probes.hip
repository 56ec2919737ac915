// probes.hip -- measurement helpers that move population data the way the
// AA step kernels do, without their arithmetic, to read the step kernels
// against the ceiling of their own memory access pattern.
#include <hip/hip_runtime.h>

#include "lattice.hpp"
#include "probes.hpp"

namespace lbm {

// q arrays of E-byte values, `stride` elements apart, over an nx x ny x nz
// lattice, periodic on every axis.  One thread per node; a workgroup covers
// a tx x ty tile of one x-y plane (tx a multiple of 64, so a wavefront
// covers consecutive x as in the step kernels); with xcd = 1 each XCD takes
// a contiguous range of workgroups (workgroup w runs on XCD w % 8).
//   ODD = false (the even step): node n moves its q values into the slots of
//     the opposite velocities of the same node.
//   ODD = true (the odd step): node n reads slot abar at n - c_a and writes
//     that value into slot a at n + c_a.  Both sets are
//     {(b, n + c_b)}, so the in-place update has no race, as in the step.
template <int Q, typename E, bool ODD>
__global__ __launch_bounds__(256) void k_pattern_probe(E* __restrict__ buf, int nx, int ny,
                                                       int nz, int tiles_x, int tiles_y,
                                                       long long stride, int xcd) {
  using L = Lattice<Q>;
  unsigned b = blockIdx.x;
  if (xcd) {
    const unsigned G = gridDim.x, q8 = G >> 3, r8 = G & 7u, xc = b & 7u, i = b >> 3;
    b = xc < r8 ? xc * (q8 + 1u) + i : r8 * (q8 + 1u) + (xc - r8) * q8 + i;
  }
  const unsigned r = b / (unsigned)tiles_x;
  const int bx = (int)(b - r * (unsigned)tiles_x);
  const int z = (int)(r / (unsigned)tiles_y);
  const int by = (int)(r - (unsigned)z * (unsigned)tiles_y);
  const int x = bx * (int)blockDim.x + (int)threadIdx.x;
  const int y = by * (int)blockDim.y + (int)threadIdx.y;
  if (x >= nx || y >= ny) return;
  const long long sxy = (long long)nx * ny;
  const long long n = x + (long long)nx * (y + (long long)ny * z);
  E v[Q];
  if constexpr (!ODD) {
#pragma unroll
    for (int a = 0; a < Q; ++a) v[a] = buf[a * stride + n];
#pragma unroll
    for (int a = 0; a < Q; ++a) buf[L::opp[a] * stride + n] = v[a];
  } else {
    // neighbour offsets along each axis, k = 0: -1, k = 1: +1 (wrapped)
    const long long ox[2] = {x == 0 ? nx - 1 : -1, x == nx - 1 ? -(nx - 1) : 1};
    const long long oy[2] = {y == 0 ? (long long)(ny - 1) * nx : -(long long)nx,
                             y == ny - 1 ? -(long long)(ny - 1) * nx : (long long)nx};
    const long long oz[2] = {z == 0 ? (nz - 1) * sxy : -sxy, z == nz - 1 ? -(nz - 1) * sxy : sxy};
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      long long m = n;  // n - c_a
      if (L::cx[a]) m += ox[L::cx[a] < 0];
      if (L::cy[a]) m += oy[L::cy[a] < 0];
      if (L::cz[a]) m += oz[L::cz[a] < 0];
      v[a] = buf[L::opp[a] * stride + m];
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      long long m = n;  // n + c_a
      if (L::cx[a]) m += ox[L::cx[a] > 0];
      if (L::cy[a]) m += oy[L::cy[a] > 0];
      if (L::cz[a]) m += oz[L::cz[a] > 0];
      buf[a * stride + m] = v[a];
    }
  }
}

template <int Q, typename E>
static void probe_qe(E* buf, int nx, int ny, int nz, long long stride, int odd, int xcd,
                     hipStream_t s) {
  const int tx = nx >= 256 ? 256 : (nx >= 128 ? 128 : 64), ty = 256 / tx;
  const int tiles_x = (nx + tx - 1) / tx, tiles_y = (ny + ty - 1) / ty;
  const dim3 grid((unsigned)((long long)tiles_x * tiles_y * nz)), block(tx, ty, 1);
  if (odd)
    hipLaunchKernelGGL((k_pattern_probe<Q, E, true>), grid, block, 0, s, buf, nx, ny, nz, tiles_x,
                       tiles_y, stride, xcd);
  else
    hipLaunchKernelGGL((k_pattern_probe<Q, E, false>), grid, block, 0, s, buf, nx, ny, nz, tiles_x,
                       tiles_y, stride, xcd);
}

template <int Q>
static void probe_q(void* buf, int elem, int nx, int ny, int nz, long long stride, int odd,
                    int xcd, hipStream_t s) {
  if (elem == 2)
    probe_qe<Q>((unsigned short*)buf, nx, ny, nz, stride, odd, xcd, s);
  else if (elem == 4)
    probe_qe<Q>((unsigned*)buf, nx, ny, nz, stride, odd, xcd, s);
  else
    probe_qe<Q>((unsigned long long*)buf, nx, ny, nz, stride, odd, xcd, s);
}

hipError_t launch_pattern_probe(void* buf, int q, int elem, int nx, int ny, int nz,
                                long long stride, int odd, int xcd, hipStream_t s) {
  (void)hipGetLastError();
  if ((q != 14 && q != 18 && q != 26) || (elem != 2 && elem != 4 && elem != 8) || nx < 1 ||
      ny < 1 || nz < 1 || (long long)nx * ny * nz > stride)
    return hipErrorInvalidValue;
  const long long tiles = (long long)((nx + 63) / 64) * ((ny + 3) / 4) * nz;
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  if (q == 14) probe_q<14>(buf, elem, nx, ny, nz, stride, odd, xcd, s);
  if (q == 18) probe_q<18>(buf, elem, nx, ny, nz, stride, odd, xcd, s);
  if (q == 26) probe_q<26>(buf, elem, nx, ny, nz, stride, odd, xcd, s);
  return hipGetLastError();
}

}  // namespace lbm

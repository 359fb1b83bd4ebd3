// Device helpers shared by the kernels of libgnorfdtd (not part of the ABI).
#pragma once

#include "gnor_internal.h"

namespace gnor {
namespace {

__device__ __forceinline__ int slab_e(int g, int n, int np) {
  return g < np ? g : (g >= n - np ? g - (n - 2 * np) : -1);
}
__device__ __forceinline__ int slab_h(int g, int n, int np) {
  return g < np ? g : (g >= n - 1 - np ? g - (n - 1 - 2 * np) : -1);
}
// index into an axis-`a` slab array with slab coordinate s replacing axis a
__device__ __forceinline__ size_t slab_index(int a, int s, int i, int j, int k, int nx, int ny,
                                             int np) {
  const int w = 2 * np;
  if (a == 0) return ((size_t)k * ny + j) * w + s;
  if (a == 1) return ((size_t)k * w + s) * nx + i;
  return ((size_t)s * ny + j) * nx + i;
}

struct Tile {
  int bx, by, bz;
  bool ok;
};
// Block b of the launch for tile class c -> tile.  The class's tiles are
// listed in natural order (x fastest, then y, then z); the position in the
// list follows the tile order of the tiling (blocks are dealt round-robin to
// the 8 XCDs).
__device__ __forceinline__ Tile decode_tile(const Tiling& tl, const int* __restrict__ list, int c,
                                            int b) {
  Tile r;
  int pos = b;
  if (tl.xcd == 1) {
    pos = (b & 7) * tl.cper[c] + (b >> 3);
  } else if (tl.xcd == 2) {
    const int rank = b >> 3;  // the block's rank on its XCD
    pos = ((rank / tl.q) * 8 + (b & 7)) * tl.q + rank % tl.q;
  }
  r.ok = pos < tl.cn[c];
  const int t = r.ok ? list[tl.coff[c] + pos] : 0;
  r.bx = t % tl.nbx;
  r.by = (t / tl.nbx) % tl.nby;
  r.bz = t / (tl.nbx * tl.nby);
  return r;
}

// Node scalars of sub-grid node l (Eqs. NonlocalUpdate / GNORUpdate in the
// current form; see Params): the node divergence of J^{n-1/2} (its edges at
// the node and one below along each axis), Phi~_P^n, and Q, the scalar whose
// differences along the edges give the nonlocal force.  One definition for
// every kernel that writes them, so that they agree bit for bit.
template <class T>
__device__ __forceinline__ void store_node_scalars(const Params<T>& p, size_t l, T jx, T jxm, T jy, T jym,
                                                   T jz, T jzm, T pp, T pj) {
  const T div = (jx - jxm) + (jy - jym) + (jz - jzm);
  const T phiP = pp + div;
  p.PPo[l] = phiP;
  p.PJo[l] = div;
  p.Q[l] = p.g1 * phiP + p.g2 * (T(3) * div - pj);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------ auxiliary line
__device__ double source_value(const AuxParams& a, double t) {
  if (a.src_kind == 1) {
    const double u = (t - a.t0) / a.tau;
    return a.e0 * exp(-u * u) * sin(a.omega_c * (t - a.t0));
  }
  if (a.src_kind == 2) {
    if (t < 0.0 || t > 2.0 * M_PI / a.omega_max) return 0.0;
    const double s = 0.5 * (1.0 - cos(a.omega_max * t));
    return a.e0 * s * s * s;
  }
  return 0.0;
}

__device__ void aux_h_block(const AuxParams& a, int tid, int nthr) {
  for (int q = tid; q <= a.n1 - 2; q += nthr) {
    const double d = a.e1[q + 1] - a.e1[q];
    const double ps = a.bh[q] * a.ph[q] + a.ah[q] * d;
    a.ph[q] = ps;
    a.h1[q] -= a.S * (a.kh[q] * d + ps);
  }
}

__device__ void aux_e_block(const AuxParams& a, int sub, int tid, int nthr) {
  for (int q = 1 + tid; q <= a.n1 - 2; q += nthr) {
    const double d = a.h1[q] - a.h1[q - 1];
    const double ps = a.be[q] * a.pe[q] + a.ae[q] * d;
    a.pe[q] = ps;
    // line cell q carries E_x of plane k = q - kAuxOff, layered like the grid
    const int k = q - kAuxOff;
    const double se = k < a.sub_k ? a.SE : (k == a.sub_k ? a.se_avg : a.se_sub);
    a.e1[q] -= se * (a.ke[q] * d + ps);
  }
  const int64_t n = a.step_base[0] + sub;
  // phase table of this step for the running transforms (e^{+i w t})
  const double tJ = ((double)n + 0.5) * a.dt, tE = ((double)n + 1.0) * a.dt;
  for (int m = tid; m < a.nf; m += nthr) {
    double s, c;
    sincos(a.omega[m] * tJ, &s, &c);
    a.phase[m] = c;
    a.phase[a.nf + m] = s;
    sincos(a.omega[m] * tE, &s, &c);
    a.phase[2 * a.nf + m] = c;
    a.phase[3 * a.nf + m] = s;
  }
  __syncthreads();
  if (tid == 0) a.e1[a.src_cell] += source_value(a, (double)(n + 1) * a.dt);
}

// Batch: the blocks of all instances in one launch per class.  Instance q
// owns blocks [blk0[c], blk0[c] + nblk[c]) of class c (for class 0 its tiles,
// then its auxiliary-line block); c = -1 selects the spectra launch's ranges
// (dblk0), c = -2 the TF/SF launch's (fblk0), c = -3 the node scalars'
// (sblk0).  A block finds its instance by
// binary search.  With an XCD-aware tile order the ranges are spaced so that
// instance q's first chunk runs on XCD q % 8; the blocks between the ranges
// exit at once.
template <class T>
__device__ __forceinline__ int find_instance(const BatchEntry<T>* __restrict__ e, int n, int b,
                                             int c) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const BatchEntry<T>& m = entry_at(e, mid);
    const int b0 = c == -1 ? m.dblk0 : (c == -2 ? m.fblk0 : (c == -3 ? m.sblk0 : m.blk0[c]));
    if (b0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// [lo, hi) meets [0, np) or [n - 1 - np, n)  (the E and H slabs of an axis)
__device__ __forceinline__ bool range_in_slabs(int lo, int hi, int n, int np) {
  // [lo, hi) meets [0, np) or [n - 1 - np, n)  (the E and H slabs of an axis)
  return np > 0 && (lo < np || hi > n - 1 - np);
}

}  // namespace
}  // namespace gnor

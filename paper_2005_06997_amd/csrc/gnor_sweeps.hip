// Field sweeps of libgnorfdtd (gfx950): the H and E/J updates as two
// HBM-bound passes (used for batches, for the adjoint's forward recompute
// and as the reference for the fused step).
//
//   k_h   f1 (Sec. III): H^{n+1/2} = H^{n-1/2} - S curl E^n with CPML and the
//         TF/SF corrections that use E_inc^n.  Tiles over the metal sub-grid
//         also evaluate the node scalars of the current form of Eq.
//         (GNORUpdate): Phi_J^{n-1/2} = Div J^{n-1/2},
//         Phi_P^n = Phi_P^{n-1} + Phi_J and Q = g1 Phi_P^n + g2 (3 Phi_J -
//         Phi_J^{n-3/2}).  The class-0 launch also advances the auxiliary
//         line's H half.
//   k_ej  f2 + f4: E^{n+1} and, at metal points, J^{n+1/2} with
//         G_a = Q(node + e_a) - Q(node) (= D_G1 GD^n + D_G2 BDF2(GD) of Eq.
//         GNORUpdate, Eq. GradDiv being Grad of the node divergence), CPML,
//         TF/SF corrections with H_inc^{n+1/2}, and per-wavefront plane sums
//         of J_x for the spectra.  The class-0 launch also advances the
//         auxiliary line's E half (soft source) and writes the step's DFT
//         phase table.
//
// A block owns 64 (x, one wavefront) x TY (y) columns and marches them over
// kz planes; H and the H-slab CPML memory are read from the step's input
// buffers and written to its output buffers.
#include "gnor_device.h"

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

namespace gnor {

namespace {

// ------------------------------------------------------------ tile classes
// Each sweep runs as four launches, one per tile class, so that each class
// gets the register budget (and hence the occupancy) its code needs:
//   class 0: tiles that meet neither metal nor a CPML slab (the bulk of a
//            large grid: the plain Yee update), and in the two-sweep form
//            also the tiles that meet only an x slab (their slab lanes
//            update the x-slab psi behind a tile-uniform branch);
//   class 1: tiles that meet a CPML slab but no metal;
//   class 2: tiles with a metal point within two cells and no slab;
//   class 3: tiles that are both 1 and 2.
// A wavefront marches its column over the tile's planes; every plane's loads
// are issued together, then computed and stored.  Latency is hidden by the
// other resident wavefronts.

// ------------------------------------------------------------------ f1: H
// Cell index of the sweeps: 32-bit in the metal classes and in FP64 (fewer
// registers for addresses: 67 -> 46 VGPRs in the FP32 metal E/J kernel),
// 64-bit elsewhere, which measured faster there.  gnor_create admits at most
// 4e9 < 2^32 cells, and every index a sweep dereferences lies below N.
template <class T, bool METAL>
using CellIdx = typename std::conditional<METAL || sizeof(T) == 8, uint32_t, size_t>::type;

// Store of a field output: nontemporal for sweeps larger than the Infinity
// Cache.  A compile-time choice: the compiler merges the two stores of a
// run-time branch into one plain store.
template <bool NT, class T>
__device__ __forceinline__ void store_field(T* a, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, a);
  else *a = v;
}

// Does the tile, widened by one cell, meet an x slab?  (The host's
// classification makes the same test.)
template <class T>
__device__ __forceinline__ bool tile_meets_x_slab(const Params<T>& p, const Tile& t) {
  const int np = p.cp[0].np;
  return np > 0 && (t.bx * kBX - 1 < np || t.bx * kBX + kBX + 1 > p.nx - 1 - np);
}

// PM: 0 no CPML; 1 any slab (pml_tile: the tile meets one); 2 at most an x
// slab (the plain class in the two-sweep form, which also takes the tiles
// that meet only an x slab: the y and z parts compile away)
template <class T, int TY, bool METAL, int PM, bool NT>
__device__ __forceinline__ void h_tile(const Params<T>& p, const Tile tile, bool pml_tile) {
  constexpr bool PML = PM != 0, PYZ = PM == 1;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int i = tile.bx * kBX + threadIdx.x;
  const int j = tile.by * TY + threadIdx.y;
  if (i >= nx || j >= ny) return;
  const int k0 = tile.bz * p.tl.kz;
  const int k1 = min(nz, k0 + p.tl.kz);
  const size_t sy = nx, sz = (size_t)nx * ny;
  const T* __restrict__ Ex = p.E[0];
  const T* __restrict__ Ey = p.E[1];
  const T* __restrict__ Ez = p.E[2];
  T* __restrict__ Hx = p.H[0];
  T* __restrict__ Hy = p.H[1];
  T* __restrict__ Hz = p.H[2];
  const T* __restrict__ Hi0 = p.Hi[0];  // H^{n-1/2} (input buffer)
  const T* __restrict__ Hi1 = p.Hi[1];
  const T* __restrict__ Hi2 = p.Hi[2];
  const T S = p.S;
  const int np = p.cp[0].np;
  const bool xin = i <= nx - 2, yin = j <= ny - 2;
  const bool cx = i >= 1 && xin && yin;  // H_x columns
  const bool cy = xin && j >= 1 && yin;  // H_y
  const bool cz = xin && yin;            // H_z
  const int sxh = (PML && pml_tile) ? slab_h(i, nx, np) : -1;
  const int syh = (PYZ && pml_tile) ? slab_h(j, ny, np) : -1;
  const CpmlAxis<T>& Z = p.cp[2];
  // the column's x- and y-slab coefficients, in registers for the whole
  // march (the psi stores could alias them, so the compiler cannot hoist them)
  T xb = T(0), xa = T(0), xk = T(1), yb = T(0), ya = T(0), yk = T(1);
  if (sxh >= 0) { xb = p.cp[0].bh[sxh]; xa = p.cp[0].ah[sxh]; xk = p.cp[0].kh[sxh]; }
  if (syh >= 0) { yb = p.cp[1].bh[syh]; ya = p.cp[1].ah[syh]; yk = p.cp[1].kh[syh]; }
  const bool tfx = p.tfsf && i >= p.tf_lo[0] && i <= p.tf_hi[0] - 1;
  const bool tfy_band = tfx && j >= p.tf_lo[1] && j <= p.tf_hi[1];
  const bool tfz_lo = tfx && j == p.tf_lo[1] - 1, tfz_hi = tfx && j == p.tf_hi[1];
  // node scalars: this column inside the metal sub-grid?
  const int lx = i - p.mlo[0], ly = j - p.mlo[1];
  const bool col_sub = METAL && lx >= 0 && ly >= 0 && lx < p.mn[0] && ly < p.mn[1];
  const size_t m1 = p.mn[0], m2 = (size_t)p.mn[0] * p.mn[1];
  const size_t lcol = col_sub ? (size_t)ly * m1 + lx : 0;
  // nodes of the column that touch a metal edge (sub-grid planes [zlo, zhi]);
  // every other node keeps zero node scalars
  int zlo = 1, zhi = 0;
  if (METAL && col_sub) {
    zlo = p.colz[2 * lcol];
    zhi = p.colz[2 * lcol + 1];
  }

  using Idx = CellIdx<T, METAL>;
  Idx id = (Idx)k0 * (Idx)sz + (Idx)j * nx + i;
  T ex0 = Ex[id], ey0 = Ey[id];  // E_x, E_y of plane k (carried up the column)
  T jzm = T(0);                  // J_z one plane below (metal sub-grid)
  if (METAL && col_sub) {
    const int lzm = k0 - 1 - p.mlo[2];
    if (lzm >= 0 && lzm < p.mn[2]) jzm = p.Ji[2][(size_t)lzm * m2 + lcol];
  }
  for (int k = k0; k < k1; ++k, id += sz) {
    const bool zin = k <= nz - 2;
    const bool ux = cx && zin, uy = cy && zin, uz = cz && k >= 1 && zin;
    // loads of the plane (one select per value: a branch that assigns
    // several values on each side can leave them in scratch memory)
    const T ex1 = zin ? Ex[id + sz] : T(0), ey1 = zin ? Ey[id + sz] : T(0);
    const T ez = Ez[id];
    const T ezy = yin ? Ez[id + sy] : T(0), exy = yin ? Ex[id + sy] : T(0);
    const T ezx = xin ? Ez[id + 1] : T(0), eyx = xin ? Ey[id + 1] : T(0);
    const T hx = ux ? Hi0[id] : T(0), hy = uy ? Hi1[id] : T(0), hz = uz ? Hi2[id] : T(0);
    T dyx = ezy - ez, dzx = ey1 - ey0;   // H_x: dy Ez - dz Ey
    T dzy = ex1 - ex0, dxy = ezx - ez;   // H_y: dz Ex - dx Ez
    T dxz = eyx - ey0, dyz = exy - ex0;  // H_z: dx Ey - dy Ex
    if (PML && pml_tile) {
      // CPML-stretched differences kinv d + psi with psi <- b psi + a d
      const int szh = PYZ ? slab_h(k, nz, np) : -1;
      if (PYZ && ux && syh >= 0) {
        const size_t q = slab_index(1, syh, i, j, k, nx, ny, np);
        const T ps = yb * p.psiHi[1][0][q] + ya * dyx;
        p.psiH[1][0][q] = ps;
        dyx = yk * dyx + ps;
      }
      if (szh >= 0) {
        const T zb = Z.bh[szh], za = Z.ah[szh], zk = Z.kh[szh];
        if (ux) {
          const size_t q = slab_index(2, szh, i, j, k, nx, ny, np);
          const T ps = zb * p.psiHi[2][1][q] + za * dzx;
          p.psiH[2][1][q] = ps;
          dzx = zk * dzx + ps;
        }
        if (uy) {
          const size_t q = slab_index(2, szh, i, j, k, nx, ny, np);
          const T ps = zb * p.psiHi[2][0][q] + za * dzy;
          p.psiH[2][0][q] = ps;
          dzy = zk * dzy + ps;
        }
      }
      if (uy && sxh >= 0) {
        const size_t q = slab_index(0, sxh, i, j, k, nx, ny, np);
        const T ps = xb * p.psiHi[0][1][q] + xa * dxy;
        p.psiH[0][1][q] = ps;
        dxy = xk * dxy + ps;
      }
      if (uz && sxh >= 0) {
        const size_t q = slab_index(0, sxh, i, j, k, nx, ny, np);
        const T ps = xb * p.psiHi[0][0][q] + xa * dxz;
        p.psiH[0][0][q] = ps;
        dxz = xk * dxz + ps;
      }
      if (PYZ && uz && syh >= 0) {
        const size_t q = slab_index(1, syh, i, j, k, nx, ny, np);
        const T ps = yb * p.psiHi[1][1][q] + ya * dyz;
        p.psiH[1][1][q] = ps;
        dyz = yk * dyz + ps;
      }
    }
    T cyv = dzy - dxy;
    T czv = dxz - dyz;
    // TF/SF: scattered-field H next to the TF box sees E_inc^n on the TF side
    if (tfy_band) {
      if (k == p.tf_lo[2] - 1) cyv -= (T)p.e1[p.tf_lo[2] + kAuxOff];
      if (k == p.tf_hi[2]) cyv += (T)p.e1[p.tf_hi[2] + kAuxOff];
    }
    if ((tfz_lo || tfz_hi) && k >= p.tf_lo[2] && k <= p.tf_hi[2]) {
      const T inc = (T)p.e1[k + kAuxOff];
      czv += tfz_lo ? inc : -inc;
    }
    if (ux) store_field<NT>(&Hx[id], hx - S * (dyx - dzx));
    if (uy) store_field<NT>(&Hy[id], hy - S * cyv);
    if (uz) store_field<NT>(&Hz[id], hz - S * czv);
    if (METAL) {
      // node scalars of node (i, j, k) of the metal sub-grid
      // J_z is carried from the plane below, so it is read one plane early
      const int lz = k - p.mlo[2];
      const bool sub = lz >= zlo && lz <= zhi;
      const bool rd = lz >= zlo - 1 && lz <= zhi;
      const size_t l = rd ? (size_t)lz * m2 + lcol : 0;
      const T jx = sub ? p.Ji[0][l] : T(0);
      const T jy = sub ? p.Ji[1][l] : T(0);
      const T jz = rd ? p.Ji[2][l] : T(0);
      const T jxm = (sub && lx > 0) ? p.Ji[0][l - 1] : T(0);
      const T jym = (sub && ly > 0) ? p.Ji[1][l - m1] : T(0);
      const T pp = sub ? p.PPi[l] : T(0);
      const T pj = sub ? p.PJi[l] : T(0);
      if (sub) store_node_scalars(p, l, jx, jxm, jy, jym, jz, jzm, pp, pj);
      jzm = jz;
    }
    ex0 = ex1;
    ey0 = ey1;
  }
}

// Critical points of one E component at metal point l: the known part R_u of
// each pole's increment (before E^{n+1}) and their sum, which enters the E
// update; then the increments and polarisations after it (f3).
template <class T>
struct CpState {
  T P[kMaxCP], R[kMaxCP];
};
template <class T>
__device__ __forceinline__ T cp_known(const Params<T>& p, int c, size_t l, T r, T e, T em, CpState<T>& st) {
  T sum = T(0);
#pragma unroll
  for (int u = 0; u < kMaxCP; ++u) {
    if (u < p.ncp) {
      st.P[u] = p.cpP[u][c][l];
      const T q = p.cpQ[u][c][l];
      st.R[u] = p.cpa[u] * st.P[u] + (q - p.cpb[u] * q) + r * (p.cp4[u] * (T(2) * e) - p.cp5[u] * (e - em));
      sum += st.R[u];
    }
  }
  return sum;
}
template <class T>
__device__ __forceinline__ double cp_update(const Params<T>& p, int c, size_t l, T r, T de,
                                            const CpState<T>& st) {
  double inc = 0.0;
#pragma unroll
  for (int u = 0; u < kMaxCP; ++u) {
    if (u < p.ncp) {
      const T q = st.R[u] + r * p.cp3[u] * de;
      p.cpQ[u][c][l] = q;
      p.cpP[u][c][l] = st.P[u] + q;
      inc += (double)q;
    }
  }
  return inc;
}

// ------------------------------------------------------- f2 + f4: E and J
template <class T, int TY, bool METAL, int PM, bool CP, bool NT>
__device__ __forceinline__ void ej_tile(const Params<T>& p, const Tile tile, bool pml_tile) {
  constexpr bool PML = PM != 0, PYZ = PM == 1;  // PM as for h_tile
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int i = tile.bx * kBX + tx;
  const int j = tile.by * TY + ty;
  const int k0 = tile.bz * p.tl.kz;
  const int k1 = min(nz, k0 + p.tl.kz);
  // lanes outside the grid stay in metal tiles (the plane sums of J_x use
  // whole wavefronts) but load and store nothing
  const bool active = i < nx && j < ny;
  if (!METAL && !active) return;
  const size_t sy = nx, sz = (size_t)nx * ny;
  const T* __restrict__ Hx = p.H[0];
  const T* __restrict__ Hy = p.H[1];
  const T* __restrict__ Hz = p.H[2];
  const T* __restrict__ Ex = p.E[0];
  const T* __restrict__ Ey = p.E[1];
  const T* __restrict__ Ez = p.E[2];
  T* __restrict__ Ox = p.O[0];
  T* __restrict__ Oy = p.O[1];
  T* __restrict__ Oz = p.O[2];
  const T SE = p.SE;
  const int np = p.cp[0].np;
  const bool ax = active && i <= nx - 2 && j >= 1 && j <= ny - 2;
  const bool ay = active && i >= 1 && i <= nx - 2 && j <= ny - 2;
  const bool az = active && i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2;
  const int sxe = (PML && pml_tile && active) ? slab_e(i, nx, np) : -1;
  const int sye = (PYZ && pml_tile && active) ? slab_e(j, ny, np) : -1;
  const CpmlAxis<T>& Z = p.cp[2];
  T xb = T(0), xa = T(0), xk = T(1), yb = T(0), ya = T(0), yk = T(1);
  if (sxe >= 0) { xb = p.cp[0].be[sxe]; xa = p.cp[0].ae[sxe]; xk = p.cp[0].ke[sxe]; }
  if (sye >= 0) { yb = p.cp[1].be[sye]; ya = p.cp[1].ae[sye]; yk = p.cp[1].ke[sye]; }
  const bool tf_xband = p.tfsf && i >= p.tf_lo[0] && i <= p.tf_hi[0] - 1 && j >= p.tf_lo[1] &&
                        j <= p.tf_hi[1];
  const bool tf_zside = p.tfsf && j >= p.tf_lo[1] && j <= p.tf_hi[1] &&
                        (i == p.tf_lo[0] || i == p.tf_hi[0]);
  const int lx = i - p.mlo[0], ly = j - p.mlo[1];
  const bool col_sub = METAL && active && lx >= 0 && ly >= 0 && lx < p.mn[0] && ly < p.mn[1];
  const size_t m1 = p.mn[0], m2 = (size_t)p.mn[0] * p.mn[1];
  const size_t lcol = col_sub ? (size_t)ly * m1 + lx : 0;

  using Idx = CellIdx<T, METAL>;
  Idx id = (Idx)k0 * (Idx)sz + (Idx)(active ? j : 0) * nx + (active ? i : 0);
  T hxm = T(0), hym = T(0);  // H at k-1 for the z differences
  if (active && k0 >= 1 && k0 < k1) {
    hxm = Hx[id - sz];
    hym = Hy[id - sz];
  }
  T qz = T(0);  // Q at node (i, j, k+1) for E_z (metal)
  for (int k = k0; k < k1; ++k, id += sz) {
    // E-type ranges in k: E_x, E_y need 1 <= k <= nz-2; E_z needs k <= nz-2
    const bool zin = k >= 1 && k <= nz - 2;
    const bool ux = ax && zin, uy = ay && zin, uz = az && k <= nz - 2;
    const T hx = active ? Hx[id] : T(0), hy = active ? Hy[id] : T(0), hz = active ? Hz[id] : T(0);
    const T hzy = (active && j >= 1) ? Hz[id - sy] : T(0);
    const T hxy = (active && j >= 1) ? Hx[id - sy] : T(0);
    const T hzx = (active && i >= 1) ? Hz[id - 1] : T(0);
    const T hyx = (active && i >= 1) ? Hy[id - 1] : T(0);
    const T ex = ux ? Ex[id] : T(0), ey = uy ? Ey[id] : T(0), ez = uz ? Ez[id] : T(0);
    // curl H (index units): E_x: dy Hz - dz Hy; E_y: dz Hx - dx Hz; E_z: dx Hy - dy Hx
    T d_yx = hz - hzy, d_zx = hy - hym;
    T d_zy = hx - hxm, d_xy = hz - hzx;
    T d_xz = hy - hyx, d_yz = hx - hxy;
    if (PML && pml_tile) {
      const int sze = PYZ ? slab_e(k, nz, np) : -1;
      if (PYZ && ux && sye >= 0) {
        T* q = p.psiE[1][0] + slab_index(1, sye, i, j, k, nx, ny, np);
        const T ps = yb * *q + ya * d_yx;
        *q = ps;
        d_yx = yk * d_yx + ps;
      }
      if (sze >= 0) {
        const T zb = Z.be[sze], za = Z.ae[sze], zk = Z.ke[sze];
        if (ux) {
          T* q = p.psiE[2][1] + slab_index(2, sze, i, j, k, nx, ny, np);
          const T ps = zb * *q + za * d_zx;
          *q = ps;
          d_zx = zk * d_zx + ps;
        }
        if (uy) {
          T* q = p.psiE[2][0] + slab_index(2, sze, i, j, k, nx, ny, np);
          const T ps = zb * *q + za * d_zy;
          *q = ps;
          d_zy = zk * d_zy + ps;
        }
      }
      if (uy && sxe >= 0) {
        T* q = p.psiE[0][1] + slab_index(0, sxe, i, j, k, nx, ny, np);
        const T ps = xb * *q + xa * d_xy;
        *q = ps;
        d_xy = xk * d_xy + ps;
      }
      if (uz && sxe >= 0) {
        T* q = p.psiE[0][0] + slab_index(0, sxe, i, j, k, nx, ny, np);
        const T ps = xb * *q + xa * d_xz;
        *q = ps;
        d_xz = xk * d_xz + ps;
      }
      if (PYZ && uz && sye >= 0) {
        T* q = p.psiE[1][1] + slab_index(1, sye, i, j, k, nx, ny, np);
        const T ps = yb * *q + ya * d_yz;
        *q = ps;
        d_yz = yk * d_yz + ps;
      }
    }
    T cxv = d_yx - d_zx, cyv = d_zy - d_xy, czv = d_xz - d_yz;
    // TF/SF: total-field E next to the box surface sees H_inc^{n+1/2} outside
    if (tf_xband) {
      if (k == p.tf_lo[2]) cxv += (T)p.h1[p.tf_lo[2] - 1 + kAuxOff];
      if (k == p.tf_hi[2]) cxv -= (T)p.h1[p.tf_hi[2] + kAuxOff];
    }
    if (tf_zside && k >= p.tf_lo[2] && k <= p.tf_hi[2] - 1) {
      const T inc = (T)p.h1[k + kAuxOff];
      czv += (i == p.tf_lo[0]) ? -inc : inc;
    }
    // background coefficients of the plane: E_x, E_y on node plane k, E_z
    // half a cell above it (a substrate beyond plane sub_k; see Params)
    const T sexy = k < p.sub_k ? SE : (k == p.sub_k ? p.se_avg : p.se_sub);
    const T sez = k < p.sub_k ? SE : p.se_sub;
    T nx_ = ex + sexy * cxv, ny_ = ey + sexy * cyv, nz_ = ez + sez * czv;
    if (METAL) {
      const int lz = k - p.mlo[2];
      const bool zsub = lz >= 0 && lz < p.mn[2];
      // total-field operation: the cell lies in an absorbing layer, so its
      // metal follows the local Drude model (no nonlocal force G)
      const bool local = PYZ && p.lra_pml && (sxe >= 0 || sye >= 0 || slab_e(k, nz, np) >= 0);
      const size_t l = (col_sub && zsub) ? (size_t)lz * m2 + lcol : 0;
      const uint32_t mb = (col_sub && zsub) ? p.mask[l] : 0u;
      double jsum = 0.0;
      if (mb) {
        // metal points lie >= 2 cells inside the sub-grid: +x, +y, +z nodes exist
        const bool b0 = mb & 1u, b1 = mb & 2u, b2 = mb & 4u;
        const T emx = b0 ? Ox[id] : T(0), emy = b1 ? Oy[id] : T(0), emz = b2 ? Oz[id] : T(0);
        const T jx = b0 ? p.Ji[0][l] : T(0), jy = b1 ? p.Ji[1][l] : T(0);
        const T jz = b2 ? p.Ji[2][l] : T(0);
        const T q = p.Q[l];
        const T qx = b0 ? p.Q[l + 1] : T(0), qy = b1 ? p.Q[l + m1] : T(0);
        qz = b2 ? p.Q[l + m2] : T(0);
        T cS = p.cS, c3 = p.c3, c1 = p.c1, cJ = p.cJ, cG = p.cG, d3 = p.d3, r = T(1);
        if (p.rho) {
          r = (T)p.rho[l];
          d3 = r * p.d3;
          const T inv = T(1) / (p.eps_inf + d3 + (CP ? r * p.c3sum : T(0)));
          cS = p.S * inv; c3 = T(3) * d3 * inv; c1 = d3 * inv; cJ = p.D2 * inv; cG = inv;
        }
        const T ag = p.agam;
        CpState<T> cps;
        if (b0) {
          const T G = local ? T(0) : r * (qx - q);
          const T rs = CP ? cp_known(p, 0, l, r, ex, emx, cps) : T(0);
          const T en = ex + (cS * cxv - c3 * ex - c1 * emx + cJ * jx - cG * (CP ? G + rs : G));
          const T jn = jx + (d3 * (emx + T(2) * ex + en) - ag * jx + G);
          p.Jo[0][l] = jn;
          jsum = (double)jn + (double)p.ebd * ((double)en - (double)ex);
          if (CP) jsum += cp_update(p, 0, l, r, en - ex, cps);
          nx_ = en;
        }
        if (b1) {
          const T G = local ? T(0) : r * (qy - q);
          const T rs = CP ? cp_known(p, 1, l, r, ey, emy, cps) : T(0);
          const T en = ey + (cS * cyv - c3 * ey - c1 * emy + cJ * jy - cG * (CP ? G + rs : G));
          p.Jo[1][l] = jy + (d3 * (emy + T(2) * ey + en) - ag * jy + G);
          if (CP) cp_update(p, 1, l, r, en - ey, cps);
          ny_ = en;
        }
        if (b2) {
          const T G = local ? T(0) : r * (qz - q);
          const T rs = CP ? cp_known(p, 2, l, r, ez, emz, cps) : T(0);
          const T en = ez + (cS * czv - c3 * ez - c1 * emz + cJ * jz - cG * (CP ? G + rs : G));
          p.Jo[2][l] = jz + (d3 * (emz + T(2) * ez + en) - ag * jz + G);
          if (CP) cp_update(p, 2, l, r, en - ez, cps);
          nz_ = en;
        }
      }
      // per-wavefront plane sum of J_x for the spectra (fixed order); a
      // wavefront without metal in the plane keeps its zero entry
      if (zsub && __any(mb != 0u)) {
        const double s = wave_sum(jsum);
        if (tx == 0) {
          const int nbxy = p.tl.nbx * p.tl.nby * TY;
          p.jpart[(size_t)k * nbxy + (tile.by * p.tl.nbx + tile.bx) * TY + ty] = s;
        }
      }
    }
    if (ux) store_field<NT>(&Ox[id], nx_);
    if (uy) store_field<NT>(&Oy[id], ny_);
    if (uz) store_field<NT>(&Oz[id], nz_);
    hxm = hx;
    hym = hy;
  }
}

template <class T, int TY, int CLS, bool NT>
__device__ __forceinline__ void h_class(const Params<T>& p, int b) {
  const Tile tile = decode_tile(p.tl, p.tiles, CLS, b);
  if (!tile.ok) return;
  if (CLS == 0) h_tile<T, TY, false, 2, NT>(p, tile, tile_meets_x_slab(p, tile));
  else if (CLS == 1) h_tile<T, TY, false, 1, NT>(p, tile, true);
  else if (CLS == 2) h_tile<T, TY, true, 0, NT>(p, tile, false);
  else h_tile<T, TY, true, 1, NT>(p, tile, true);
}
template <class T, int TY, int CLS, bool CP, bool NT>
__device__ __forceinline__ void ej_class(const Params<T>& p, int b) {
  const Tile tile = decode_tile(p.tl, p.tiles, CLS, b);
  if (!tile.ok) return;
  if (CLS == 0) ej_tile<T, TY, false, 2, false, NT>(p, tile, tile_meets_x_slab(p, tile));
  else if (CLS == 1) ej_tile<T, TY, false, 1, false, NT>(p, tile, true);
  else if (CLS == 2) ej_tile<T, TY, true, 0, CP, NT>(p, tile, false);
  else ej_tile<T, TY, true, 1, CP, NT>(p, tile, true);
}

// ---------------------------------------------------------------- kernels
// Single simulation: one launch per tile class; the class-0 launch has one
// extra block (the last) that advances the auxiliary line.
// NT: nontemporal field stores (chosen by the host per launch: Params::stream_stores)
template <class T, int TY, int CLS, bool NT>
__global__ void __launch_bounds__(kBX* TY) k_h(Params<T> p, AuxParams a) {
  if (CLS == 0 && (int)blockIdx.x == (int)gridDim.x - 1) {
    aux_h_block(a, threadIdx.y * kBX + threadIdx.x, kBX * TY);
    return;
  }
  h_class<T, TY, CLS, NT>(p, blockIdx.x);
}

// CP: the metal classes with critical points (a separate variant, so the
// plain metal code keeps its registers)
template <class T, int TY, int CLS, bool CP, bool NT>
__global__ void __launch_bounds__(kBX* TY) k_ej(Params<T> p, AuxParams a, int sub) {
  if (CLS == 0 && (int)blockIdx.x == (int)gridDim.x - 1) {
    aux_e_block(a, sub, threadIdx.y * kBX + threadIdx.x, kBX * TY);
    return;
  }
  ej_class<T, TY, CLS, CP, NT>(p, blockIdx.x);
}

// Batch: the blocks of all instances in one launch per class (find_instance
// maps a block to its instance).

template <class T, int TY, int CLS, bool NT>
__global__ void __launch_bounds__(kBX* TY) k_h_batch(const BatchEntry<T>* __restrict__ e, int n) {
  const BatchEntry<T>& en = entry_at(e, find_instance(e, n, blockIdx.x, CLS));
  const int b = blockIdx.x - en.blk0[CLS];
  if (b >= en.nblk[CLS] || (CLS == 2 && !en.two_sweep2)) return;
  if (CLS == 0 && b == en.nblk[0] - 1) {
    aux_h_block(en.a, threadIdx.y * kBX + threadIdx.x, kBX * TY);
    return;
  }
  h_class<T, TY, CLS, NT>(en.p, b);
}

// Class 0's last block of each instance is idle in the E/J sweep: the lines'
// E update is k_aux_e_batch.
template <class T, int TY, int CLS, bool CP, bool NT>
__global__ void __launch_bounds__(kBX* TY) k_ej_batch(const BatchEntry<T>* __restrict__ e, int n) {
  const BatchEntry<T>& en = entry_at(e, find_instance(e, n, blockIdx.x, CLS));
  const int b = blockIdx.x - en.blk0[CLS];
  if (b >= en.nblk[CLS] || (CLS == 0 && b == en.nblk[0] - 1) || (CLS == 2 && !en.two_sweep2)) return;
  ej_class<T, TY, CLS, CP, NT>(en.p, b);
}

// The auxiliary lines' E update of a batch, one block per instance.  A kernel
// of its own rather than a block of the class-0 sweep (as for one
// simulation): there its FP64 source and phase evaluation, reached through
// the instance table, doubled the sweep kernel's registers and halved its
// occupancy.
template <class T>
__global__ void __launch_bounds__(kAuxThreads) k_aux_e_batch(const BatchEntry<T>* __restrict__ e, int sub) {
  aux_e_block(entry_at(e, blockIdx.x).a, sub, threadIdx.x, kAuxThreads);
}

// Soft plane source of total-field operation: E_x^{n+1} += f(t_{n+1}) at
// the E_x points (i + 1/2, j, k) the update reaches (0 <= i <= nx - 2,
// 1 <= j <= ny - 2) of node plane k.  Every thread evaluates f itself (one
// plane: a few hundred FP64 exponentials per block).
template <class T>
__global__ void __launch_bounds__(256) k_plane_source(T* __restrict__ ex, int nx, int ny, int k,
                                                      AuxParams a, int sub) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = 1 + blockIdx.y * 4 + threadIdx.y;
  if (i > nx - 2 || j > ny - 2) return;
  const int64_t n = a.step_base[0] + sub;
  const double f = source_value(a, (double)(n + 1) * a.dt);
  T* q = ex + ((size_t)k * ny + j) * nx + i;
  *q = *q + (T)f;
}

}  // namespace

// ------------------------------------------------------------ host helpers
Tiling make_tiling(int nx, int ny, int nz, int ty, int kz, int xcd) {
  Tiling t{};
  t.ty = ty;
  t.kz = kz;
  t.xcd = xcd;
  t.nbx = (nx + kBX - 1) / kBX;
  t.nby = (ny + ty - 1) / ty;
  t.nbz = (nz + kz - 1) / kz;
  t.q = t.nbx * 8;  // chunk: 8 rows of tiles
  return t;
}

// Does the tile, widened by two cells on every side, contain a metal point?
// (Metal work, node scalars and the fused step's Q halo all lie within that
// distance of a metal point.)  rowx[2 (k ny + j)] .. [+1]: first and last x
// of the metal points of row (j, k) (first > last: none).
static bool tile_meets_metal_host(const Tiling& t, int tile, int nx, int ny, int nz,
                                  const int* rowx) {
  if (!rowx) return false;
  const int bx = tile % t.nbx, by = (tile / t.nbx) % t.nby, bz = tile / (t.nbx * t.nby);
  const int x0 = bx * kBX - 2, x1 = std::min(nx, bx * kBX + kBX) + 1;
  const int y0 = std::max(0, by * t.ty - 2), y1 = std::min(ny - 1, by * t.ty + t.ty + 1);
  const int z0 = std::max(0, bz * t.kz - 2), z1 = std::min(nz - 1, std::min(nz, bz * t.kz + t.kz) + 1);
  for (int k = z0; k <= z1; ++k)
    for (int j = y0; j <= y1; ++j) {
      const int* r = rowx + 2 * ((size_t)k * ny + j);
      if (r[0] <= r[1] && r[0] <= x1 && r[1] >= x0) return true;
    }
  return false;
}

void classify_tiles(Tiling& t, int nx, int ny, int nz, int np, const int* rowx,
                    std::vector<int>& list, bool merge_x, bool merge_x_metal,
                    std::vector<uint8_t>& tile_class) {
  const int T = t.nbx * t.nby * t.nbz;
  std::vector<int> cls[kClasses];
  tile_class.assign(T, 0);
  auto slab = [&](int lo, int hi, int n) { return np > 0 && (lo < np || hi > n - 1 - np); };
  for (int tile = 0; tile < T; ++tile) {
    const int bx = tile % t.nbx, by = (tile / t.nbx) % t.nby, bz = tile / (t.nbx * t.nby);
    const int z0 = bz * t.kz, z1 = std::min(nz, z0 + t.kz);
    // ranges widened by one cell: the fused step also touches the tile's halo
    const bool metal = tile_meets_metal_host(t, tile, nx, ny, nz, rowx);
    const bool px = slab(bx * kBX - 1, bx * kBX + kBX + 1, nx);
    const bool pyz = slab(by * t.ty - 1, by * t.ty + t.ty + 1, ny) || slab(z0 - 1, z1 + 1, nz);
    const int c = metal ? (pyz || (px && !merge_x_metal) ? 3 : 2) : (pyz || (px && !merge_x) ? 1 : 0);
    tile_class[tile] = (uint8_t)c;
    cls[c].push_back(tile);
  }
  list.clear();
  for (int c = 0; c < kClasses; ++c) {
    t.coff[c] = (int)list.size();
    t.cn[c] = (int)cls[c].size();
    list.insert(list.end(), cls[c].begin(), cls[c].end());
    if (t.xcd == 1) t.cper[c] = (t.cn[c] + 7) / 8;
    else if (t.xcd == 2) t.cper[c] = ((t.cn[c] + t.q - 1) / t.q + 7) / 8;  // chunks per XCD
    else t.cper[c] = t.cn[c];
  }
}

int class_blocks(const Tiling& t, int c) {
  if (t.cn[c] == 0) return 0;
  if (t.xcd == 1) return 8 * t.cper[c];
  if (t.xcd == 2) return 8 * t.cper[c] * t.q;
  return t.cn[c];
}

namespace {
template <class T, int CLS, bool NT>
void launch_h_cls_nt(const Params<T>& p, const AuxParams& a, int blocks, hipStream_t s) {
  if (p.tl.ty == 4) hipLaunchKernelGGL((k_h<T, 4, CLS, NT>), dim3(blocks), dim3(kBX, 4), 0, s, p, a);
  else if (p.tl.ty == 8) hipLaunchKernelGGL((k_h<T, 8, CLS, NT>), dim3(blocks), dim3(kBX, 8), 0, s, p, a);
  else hipLaunchKernelGGL((k_h<T, 2, CLS, NT>), dim3(blocks), dim3(kBX, 2), 0, s, p, a);
}
template <class T, int CLS>
void launch_h_cls(const Params<T>& p, const AuxParams& a, hipStream_t s) {
  const int blocks = class_blocks(p.tl, CLS) + (CLS == 0 ? 1 : 0);
  if (blocks == 0) return;
  if (p.stream_stores) launch_h_cls_nt<T, CLS, true>(p, a, blocks, s);
  else launch_h_cls_nt<T, CLS, false>(p, a, blocks, s);
}
template <class T, int CLS, bool CP, bool NT>
void launch_ej_cls_nt(const Params<T>& p, const AuxParams& a, int sub, int blocks, hipStream_t s) {
  if (p.tl.ty == 4) hipLaunchKernelGGL((k_ej<T, 4, CLS, CP, NT>), dim3(blocks), dim3(kBX, 4), 0, s, p, a, sub);
  else if (p.tl.ty == 8) hipLaunchKernelGGL((k_ej<T, 8, CLS, CP, NT>), dim3(blocks), dim3(kBX, 8), 0, s, p, a, sub);
  else hipLaunchKernelGGL((k_ej<T, 2, CLS, CP, NT>), dim3(blocks), dim3(kBX, 2), 0, s, p, a, sub);
}
template <class T, int CLS, bool CP>
void launch_ej_cls(const Params<T>& p, const AuxParams& a, int sub, hipStream_t s) {
  const int blocks = class_blocks(p.tl, CLS) + (CLS == 0 ? 1 : 0);
  if (blocks == 0) return;
  if (p.stream_stores) launch_ej_cls_nt<T, CLS, CP, true>(p, a, sub, blocks, s);
  else launch_ej_cls_nt<T, CLS, CP, false>(p, a, sub, blocks, s);
}
template <class T, int CLS, bool NT>
void launch_h_batch_cls_nt(const BatchEntry<T>* e, int n, int blocks, int ty, hipStream_t s) {
  if (ty == 4) hipLaunchKernelGGL((k_h_batch<T, 4, CLS, NT>), dim3(blocks), dim3(kBX, 4), 0, s, e, n);
  else if (ty == 8) hipLaunchKernelGGL((k_h_batch<T, 8, CLS, NT>), dim3(blocks), dim3(kBX, 8), 0, s, e, n);
  else hipLaunchKernelGGL((k_h_batch<T, 2, CLS, NT>), dim3(blocks), dim3(kBX, 2), 0, s, e, n);
}
template <class T, int CLS>
void launch_h_batch_cls(const BatchEntry<T>* e, int n, int blocks, int ty, bool nt, hipStream_t s) {
  if (blocks == 0) return;
  if (nt) launch_h_batch_cls_nt<T, CLS, true>(e, n, blocks, ty, s);
  else launch_h_batch_cls_nt<T, CLS, false>(e, n, blocks, ty, s);
}
template <class T, int CLS, bool CP, bool NT>
void launch_ej_batch_cls_nt(const BatchEntry<T>* e, int n, int blocks, int ty, hipStream_t s) {
  if (ty == 4) hipLaunchKernelGGL((k_ej_batch<T, 4, CLS, CP, NT>), dim3(blocks), dim3(kBX, 4), 0, s, e, n);
  else if (ty == 8) hipLaunchKernelGGL((k_ej_batch<T, 8, CLS, CP, NT>), dim3(blocks), dim3(kBX, 8), 0, s, e, n);
  else hipLaunchKernelGGL((k_ej_batch<T, 2, CLS, CP, NT>), dim3(blocks), dim3(kBX, 2), 0, s, e, n);
}
template <class T, int CLS, bool CP>
void launch_ej_batch_cls(const BatchEntry<T>* e, int n, int blocks, int ty, bool nt, hipStream_t s) {
  if (blocks == 0) return;
  if (nt) launch_ej_batch_cls_nt<T, CLS, CP, true>(e, n, blocks, ty, s);
  else launch_ej_batch_cls_nt<T, CLS, CP, false>(e, n, blocks, ty, s);
}
}  // namespace

template <class T>
void launch_h_class(const Params<T>& p, const AuxParams& a, int c, hipStream_t s) {
  if (c == 0) launch_h_cls<T, 0>(p, a, s);
  else if (c == 1) launch_h_cls<T, 1>(p, a, s);
  else if (c == 2) launch_h_cls<T, 2>(p, a, s);
  else launch_h_cls<T, 3>(p, a, s);
}
template <class T>
void launch_ej_class(const Params<T>& p, const AuxParams& a, int sub, int c, hipStream_t s) {
  const bool cp = p.ncp > 0;
  if (c == 0) launch_ej_cls<T, 0, false>(p, a, sub, s);
  else if (c == 1) launch_ej_cls<T, 1, false>(p, a, sub, s);
  else if (c == 2) cp ? launch_ej_cls<T, 2, true>(p, a, sub, s) : launch_ej_cls<T, 2, false>(p, a, sub, s);
  else cp ? launch_ej_cls<T, 3, true>(p, a, sub, s) : launch_ej_cls<T, 3, false>(p, a, sub, s);
}
template <class T>
void launch_h(const Params<T>& p, const AuxParams& a, hipStream_t s) {
  for (int c = 0; c < kClasses; ++c) launch_h_class<T>(p, a, c, s);
}
template <class T>
void launch_ej(const Params<T>& p, const AuxParams& a, int sub, hipStream_t s) {
  for (int c = 0; c < kClasses; ++c) launch_ej_class<T>(p, a, sub, c, s);
}
template void launch_h_class<float>(const Params<float>&, const AuxParams&, int, hipStream_t);
template void launch_h_class<double>(const Params<double>&, const AuxParams&, int, hipStream_t);
template void launch_ej_class<float>(const Params<float>&, const AuxParams&, int, int, hipStream_t);
template void launch_ej_class<double>(const Params<double>&, const AuxParams&, int, int, hipStream_t);
template <class T>
void launch_h_batch_class(const BatchEntry<T>* e, int n, int blocks, int ty, int c, bool nt,
                          hipStream_t s) {
  if (c == 0) launch_h_batch_cls<T, 0>(e, n, blocks, ty, nt, s);
  else if (c == 1) launch_h_batch_cls<T, 1>(e, n, blocks, ty, nt, s);
  else if (c == 2) launch_h_batch_cls<T, 2>(e, n, blocks, ty, nt, s);
  else launch_h_batch_cls<T, 3>(e, n, blocks, ty, nt, s);
}
template <class T>
void launch_ej_batch_class(const BatchEntry<T>* e, int n, int blocks, int ty, int c, bool cp, bool nt,
                           hipStream_t s) {
  if (c == 0) launch_ej_batch_cls<T, 0, false>(e, n, blocks, ty, nt, s);
  else if (c == 1) launch_ej_batch_cls<T, 1, false>(e, n, blocks, ty, nt, s);
  else if (c == 2) cp ? launch_ej_batch_cls<T, 2, true>(e, n, blocks, ty, nt, s)
                      : launch_ej_batch_cls<T, 2, false>(e, n, blocks, ty, nt, s);
  else cp ? launch_ej_batch_cls<T, 3, true>(e, n, blocks, ty, nt, s)
          : launch_ej_batch_cls<T, 3, false>(e, n, blocks, ty, nt, s);
}
template <class T>
void launch_aux_e_batch(const BatchEntry<T>* e, int n, int sub, hipStream_t s) {
  hipLaunchKernelGGL((k_aux_e_batch<T>), dim3(n), dim3(kAuxThreads), 0, s, e, sub);
}
template void launch_h_batch_class<float>(const BatchEntry<float>*, int, int, int, int, bool, hipStream_t);
template void launch_h_batch_class<double>(const BatchEntry<double>*, int, int, int, int, bool, hipStream_t);
template void launch_ej_batch_class<float>(const BatchEntry<float>*, int, int, int, int, bool, bool,
                                           hipStream_t);
template void launch_ej_batch_class<double>(const BatchEntry<double>*, int, int, int, int, bool, bool,
                                            hipStream_t);
template void launch_aux_e_batch<float>(const BatchEntry<float>*, int, int, hipStream_t);
template void launch_aux_e_batch<double>(const BatchEntry<double>*, int, int, hipStream_t);
template <class T>
void launch_plane_source(const Params<T>& p, const AuxParams& a, int k, int sub, hipStream_t s) {
  const dim3 grid((p.nx - 1 + 63) / 64, (p.ny - 2 + 3) / 4);
  k_plane_source<T><<<grid, dim3(64, 4), 0, s>>>(p.O[0], p.nx, p.ny, k, a, sub);
}
template void launch_plane_source<float>(const Params<float>&, const AuxParams&, int, int, hipStream_t);
template void launch_plane_source<double>(const Params<double>&, const AuxParams&, int, int, hipStream_t);
template void launch_h<float>(const Params<float>&, const AuxParams&, hipStream_t);
template void launch_h<double>(const Params<double>&, const AuxParams&, hipStream_t);
template void launch_ej<float>(const Params<float>&, const AuxParams&, int, hipStream_t);
template void launch_ej<double>(const Params<double>&, const AuxParams&, int, hipStream_t);

}  // namespace gnor

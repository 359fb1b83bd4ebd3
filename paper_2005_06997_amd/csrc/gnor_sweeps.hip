// Field sweeps of libgnorfdtd (gfx950): the two HBM-bound kernels of a step.
//
//   k_h   f1 (Sec. III): H^{n+1/2} = H^{n-1/2} - S curl E^n with CPML and the
//         TF/SF corrections that use E_inc^n.  Tiles over the metal sub-grid
//         also evaluate the node scalars of the current form of Eq.
//         (GNORUpdate): Phi_J^{n-1/2} = Div J^{n-1/2},
//         Phi_P^n = Phi_P^{n-1} + Phi_J and Q = g1 Phi_P^n + g2 (3 Phi_J -
//         Phi_J^{n-3/2}) (k_h does not read J, Phi or Q, so no halo is
//         needed).  One extra block advances the auxiliary line's H half.
//   k_ej  f2 + f4: E^{n+1} and, at metal points, J^{n+1/2} with
//         G_a = Q(node + e_a) - Q(node) (= D_G1 GD^n + D_G2 BDF2(GD) of Eq.
//         GNORUpdate, Eq. GradDiv being Grad of the node divergence), CPML,
//         TF/SF corrections with H_inc^{n+1/2}, and per-wavefront plane sums
//         of J_x for the spectra.  One extra block advances the auxiliary
//         line's E half (soft source) and writes the step's DFT phase table.
//
// A block owns 64 (x, one wavefront) x TY (y) columns and marches them over
// kz planes.  Every iteration first issues the loads of the NEXT plane, then
// computes and stores the current one, so memory latency overlaps compute
// and stores (register double buffering); no barriers.
#include "gnor_internal.h"

#include <cmath>

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
__device__ __forceinline__ Tile decode_tile(const Tiling& tl, int b) {
  Tile r;
  int t = b;
  if (tl.xcd == 1) {
    t = (b & 7) * tl.per + (b >> 3);
  } else if (tl.xcd == 2) {
    const int rank = b >> 3;  // the block's rank on its XCD
    t = ((rank / tl.q) * 8 + (b & 7)) * tl.q + rank % tl.q;
  }
  r.ok = t < tl.nbx * tl.nby * tl.nbz;
  r.bx = t % tl.nbx;
  r.by = (t / tl.nbx) % tl.nby;
  r.bz = t / (tl.nbx * tl.nby);
  return r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// CPML-stretched difference: kinv d + psi with psi <- b psi + a d (index units)
template <class T>
__device__ __forceinline__ T stretch(T* __restrict__ psi, size_t q, T b, T a, T ki, T d) {
  const T ps = b * psi[q] + a * d;
  psi[q] = ps;
  return ki * d + ps;
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
    a.e1[q] -= a.SE * (a.ke[q] * d + ps);
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
  if (tid == 0) a.e1[kAuxSrc] += source_value(a, (double)(n + 1) * a.dt);
}

// ------------------------------------------------------------------ f1: H
template <class T>
struct HIn {
  T ex1, ey1, ez, ezy, ezx, eyx, exy, hx, hy, hz;  // E at k+1 (own), E at k, H at k
  T jx, jy, jz, jxm, jym, pp, pj;                  // node scalars' inputs at k
};

// One tile of the H sweep (blk: the block's index among the tiles).
template <class T, int TY>
__device__ __forceinline__ void h_tile(const Params<T>& p, int blk) {
  const Tile tile = decode_tile(p.tl, blk);
  if (!tile.ok) return;
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
  const T S = p.S;
  const int np = p.cp[0].np;
  const bool xin = i <= nx - 2, yin = j <= ny - 2;
  const bool cx = i >= 1 && xin && yin;  // H_x columns
  const bool cy = xin && j >= 1 && yin;  // H_y
  const bool cz = xin && yin;            // H_z
  const int sxh = np ? slab_h(i, nx, np) : -1;
  const int syh = np ? slab_h(j, ny, np) : -1;
  const bool tfx = p.tfsf && i >= p.tf_lo[0] && i <= p.tf_hi[0] - 1;
  const bool tfy_band = tfx && j >= p.tf_lo[1] && j <= p.tf_hi[1];
  const bool tfz_lo = tfx && j == p.tf_lo[1] - 1, tfz_hi = tfx && j == p.tf_hi[1];
  // node scalars: this column inside the metal sub-grid?
  const int lx = i - p.mlo[0], ly = j - p.mlo[1];
  const bool col_sub = p.any_metal && lx >= 0 && ly >= 0 && lx < p.mn[0] && ly < p.mn[1];
  const size_t m1 = p.mn[0], m2 = (size_t)p.mn[0] * p.mn[1];
  const size_t lcol = col_sub ? (size_t)ly * m1 + lx : 0;

  auto load = [&](int k, size_t id, HIn<T>& v) {
    const bool zin = k <= nz - 2;
    v.ex1 = zin ? Ex[id + sz] : T(0);
    v.ey1 = zin ? Ey[id + sz] : T(0);
    v.ez = Ez[id];
    v.ezy = yin ? Ez[id + sy] : T(0);
    v.ezx = xin ? Ez[id + 1] : T(0);
    v.eyx = xin ? Ey[id + 1] : T(0);
    v.exy = yin ? Ex[id + sy] : T(0);
    v.hx = (cx && zin) ? Hx[id] : T(0);
    v.hy = (cy && zin) ? Hy[id] : T(0);
    v.hz = (cz && k >= 1 && zin) ? Hz[id] : T(0);
    const int lz = k - p.mlo[2];
    if (col_sub && lz >= 0 && lz < p.mn[2]) {
      const size_t l = (size_t)lz * m2 + lcol;
      v.jx = p.Ji[0][l]; v.jy = p.Ji[1][l]; v.jz = p.Ji[2][l];
      v.jxm = lx > 0 ? p.Ji[0][l - 1] : T(0);
      v.jym = ly > 0 ? p.Ji[1][l - m1] : T(0);
      v.pp = p.PPi[l]; v.pj = p.PJi[l];
    } else {
      v.jx = v.jy = v.jz = v.jxm = v.jym = v.pp = v.pj = T(0);
    }
  };

  size_t id = (size_t)k0 * sz + (size_t)j * nx + i;
  T ex0 = Ex[id], ey0 = Ey[id];
  T jzm = T(0);  // J_z one plane below (own column)
  if (col_sub) {
    const int lzm = k0 - 1 - p.mlo[2];
    if (lzm >= 0 && lzm < p.mn[2]) jzm = p.Ji[2][(size_t)lzm * m2 + lcol];
  }
  HIn<T> cur, nxt;
  load(k0, id, cur);
  for (int k = k0; k < k1; ++k, id += sz) {
    if (k + 1 < k1) load(k + 1, id + sz, nxt);
    const bool zin = k <= nz - 2;
    const bool ux = cx && zin, uy = cy && zin, uz = cz && k >= 1 && zin;
    T dyx = cur.ezy - cur.ez, dzx = cur.ey1 - ey0;   // H_x: dy Ez - dz Ey
    T dzy = cur.ex1 - ex0, dxy = cur.ezx - cur.ez;   // H_y: dz Ex - dx Ez
    T dxz = cur.eyx - ey0, dyz = cur.exy - ex0;      // H_z: dx Ey - dy Ex
    if (np) {
      const int szh = slab_h(k, nz, np);
      const CpmlAxis<T>& X = p.cp[0];
      const CpmlAxis<T>& Y = p.cp[1];
      const CpmlAxis<T>& Z = p.cp[2];
      if (ux && syh >= 0) dyx = stretch(p.psiH[1][0], slab_index(1, syh, i, j, k, nx, ny, np), Y.bh[syh], Y.ah[syh], Y.kh[syh], dyx);
      if (ux && szh >= 0) dzx = stretch(p.psiH[2][1], slab_index(2, szh, i, j, k, nx, ny, np), Z.bh[szh], Z.ah[szh], Z.kh[szh], dzx);
      if (uy && szh >= 0) dzy = stretch(p.psiH[2][0], slab_index(2, szh, i, j, k, nx, ny, np), Z.bh[szh], Z.ah[szh], Z.kh[szh], dzy);
      if (uy && sxh >= 0) dxy = stretch(p.psiH[0][1], slab_index(0, sxh, i, j, k, nx, ny, np), X.bh[sxh], X.ah[sxh], X.kh[sxh], dxy);
      if (uz && sxh >= 0) dxz = stretch(p.psiH[0][0], slab_index(0, sxh, i, j, k, nx, ny, np), X.bh[sxh], X.ah[sxh], X.kh[sxh], dxz);
      if (uz && syh >= 0) dyz = stretch(p.psiH[1][1], slab_index(1, syh, i, j, k, nx, ny, np), Y.bh[syh], Y.ah[syh], Y.kh[syh], dyz);
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
    if (ux) Hx[id] = cur.hx - S * (dyx - dzx);
    if (uy) Hy[id] = cur.hy - S * cyv;
    if (uz) Hz[id] = cur.hz - S * czv;
    // node scalars of node (i, j, k) of the metal sub-grid
    const int lz = k - p.mlo[2];
    if (col_sub && lz >= 0 && lz < p.mn[2]) {
      const T div = (cur.jx - cur.jxm) + (cur.jy - cur.jym) + (cur.jz - jzm);
      const T phiP = cur.pp + div;
      const size_t l = (size_t)lz * m2 + lcol;
      p.PPo[l] = phiP;
      p.PJo[l] = div;
      p.Q[l] = p.g1 * phiP + p.g2 * (T(3) * div - cur.pj);
    }
    jzm = cur.jz;
    ex0 = cur.ex1;
    ey0 = cur.ey1;
    cur = nxt;
  }
}

// ------------------------------------------------------- f2 + f4: E and J
template <class T>
struct EIn {
  T hx, hy, hz, hzy, hzx, hyx, hxy;  // H at k (own and -x, -y neighbours)
  T ex, ey, ez;                      // E^n
  T emx, emy, emz;                   // E^{n-1} (metal)
  T jx, jy, jz;                      // J^{n-1/2} (metal)
  T q, qx, qy;                       // Q at node k, k + e_x, k + e_y (metal)
  uint8_t mb;
};

// One tile of the E/J sweep.
template <class T, int TY>
__device__ __forceinline__ void ej_tile(const Params<T>& p, int blk) {
  const int tx = threadIdx.x, ty = threadIdx.y;
  const Tile tile = decode_tile(p.tl, blk);
  if (!tile.ok) return;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int i = tile.bx * kBX + tx;
  const int j = tile.by * TY + ty;
  const int k0 = tile.bz * p.tl.kz;
  const int k1 = min(nz, k0 + p.tl.kz);
  const bool active = i < nx && j < ny;
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
  const int sxe = np ? slab_e(i, nx, np) : -1;
  const int sye = np ? slab_e(j, ny, np) : -1;
  const bool tf_xband = p.tfsf && i >= p.tf_lo[0] && i <= p.tf_hi[0] - 1 && j >= p.tf_lo[1] &&
                        j <= p.tf_hi[1];
  const bool tf_zside = p.tfsf && j >= p.tf_lo[1] && j <= p.tf_hi[1] &&
                        (i == p.tf_lo[0] || i == p.tf_hi[0]);
  const int x0 = tile.bx * kBX, y0 = tile.by * TY;
  const bool metal_tile = p.any_metal && x0 < p.mlo[0] + p.mn[0] && x0 + kBX > p.mlo[0] &&
                          y0 < p.mlo[1] + p.mn[1] && y0 + TY > p.mlo[1] &&
                          k0 < p.mlo[2] + p.mn[2] && k1 > p.mlo[2];
  const int lx = i - p.mlo[0], ly = j - p.mlo[1];
  const bool col_sub = metal_tile && active && lx >= 0 && ly >= 0 && lx < p.mn[0] && ly < p.mn[1];
  const size_t m1 = p.mn[0], m2 = (size_t)p.mn[0] * p.mn[1];
  const size_t lcol = col_sub ? (size_t)ly * m1 + lx : 0;
  auto mask_at = [&](int k) -> uint8_t {
    const int lz = k - p.mlo[2];
    return (col_sub && k < k1 && lz >= 0 && lz < p.mn[2]) ? p.mask[(size_t)lz * m2 + lcol] : 0;
  };
  // E-type ranges in k: E_x, E_y need 1 <= k <= nz-2; E_z needs k <= nz-2
  auto load = [&](int k, size_t id, uint8_t mb, EIn<T>& v) {
    const bool zin = k >= 1 && k <= nz - 2;
    v.hx = active ? Hx[id] : T(0);
    v.hy = active ? Hy[id] : T(0);
    v.hz = active ? Hz[id] : T(0);
    v.hzy = (active && j >= 1) ? Hz[id - sy] : T(0);
    v.hzx = (active && i >= 1) ? Hz[id - 1] : T(0);
    v.hyx = (active && i >= 1) ? Hy[id - 1] : T(0);
    v.hxy = (active && j >= 1) ? Hx[id - sy] : T(0);
    v.ex = (ax && zin) ? Ex[id] : T(0);
    v.ey = (ay && zin) ? Ey[id] : T(0);
    v.ez = (az && k <= nz - 2) ? Ez[id] : T(0);
    v.mb = mb;
    if (mb) {
      const size_t l = (size_t)(k - p.mlo[2]) * m2 + lcol;
      v.emx = (mb & 1u) ? Ox[id] : T(0);
      v.emy = (mb & 2u) ? Oy[id] : T(0);
      v.emz = (mb & 4u) ? Oz[id] : T(0);
      v.jx = (mb & 1u) ? p.Ji[0][l] : T(0);
      v.jy = (mb & 2u) ? p.Ji[1][l] : T(0);
      v.jz = (mb & 4u) ? p.Ji[2][l] : T(0);
      // metal points lie >= 2 cells inside the sub-grid: +x, +y, +z nodes exist
      v.q = p.Q[l];
      v.qx = (mb & 1u) ? p.Q[l + 1] : T(0);
      v.qy = (mb & 2u) ? p.Q[l + m1] : T(0);
    } else {
      v.emx = v.emy = v.emz = v.jx = v.jy = v.jz = v.q = v.qx = v.qy = T(0);
    }
  };

  size_t id = (size_t)k0 * sz + (size_t)j * nx + i;
  T hxm = T(0), hym = T(0);  // H at k-1 for the z differences
  if (active && k0 >= 1) {
    hxm = Hx[id - sz];
    hym = Hy[id - sz];
  }
  uint8_t mk1 = mask_at(k0 + 1);
  EIn<T> cur, nxt;
  load(k0, id, mask_at(k0), cur);
  T qz = T(0);  // Q at node (i, j, k+1) for E_z
  for (int k = k0; k < k1; ++k, id += sz) {
    const uint8_t mk2 = mask_at(k + 2);
    if (k + 1 < k1) load(k + 1, id + sz, mk1, nxt);
    if (cur.mb & 4u) qz = p.Q[(size_t)(k + 1 - p.mlo[2]) * m2 + lcol];
    const bool zin = k >= 1 && k <= nz - 2;
    const bool ux = ax && zin, uy = ay && zin, uz = az && k <= nz - 2;
    // curl H (index units): E_x: dy Hz - dz Hy; E_y: dz Hx - dx Hz; E_z: dx Hy - dy Hx
    T d_yx = cur.hz - cur.hzy, d_zx = cur.hy - hym;
    T d_zy = cur.hx - hxm, d_xy = cur.hz - cur.hzx;
    T d_xz = cur.hy - cur.hyx, d_yz = cur.hx - cur.hxy;
    if (np) {
      const int sze = slab_e(k, nz, np);
      const CpmlAxis<T>& X = p.cp[0];
      const CpmlAxis<T>& Y = p.cp[1];
      const CpmlAxis<T>& Z = p.cp[2];
      if (ux && sye >= 0) d_yx = stretch(p.psiE[1][0], slab_index(1, sye, i, j, k, nx, ny, np), Y.be[sye], Y.ae[sye], Y.ke[sye], d_yx);
      if (ux && sze >= 0) d_zx = stretch(p.psiE[2][1], slab_index(2, sze, i, j, k, nx, ny, np), Z.be[sze], Z.ae[sze], Z.ke[sze], d_zx);
      if (uy && sze >= 0) d_zy = stretch(p.psiE[2][0], slab_index(2, sze, i, j, k, nx, ny, np), Z.be[sze], Z.ae[sze], Z.ke[sze], d_zy);
      if (uy && sxe >= 0) d_xy = stretch(p.psiE[0][1], slab_index(0, sxe, i, j, k, nx, ny, np), X.be[sxe], X.ae[sxe], X.ke[sxe], d_xy);
      if (uz && sxe >= 0) d_xz = stretch(p.psiE[0][0], slab_index(0, sxe, i, j, k, nx, ny, np), X.be[sxe], X.ae[sxe], X.ke[sxe], d_xz);
      if (uz && sye >= 0) d_yz = stretch(p.psiE[1][1], slab_index(1, sye, i, j, k, nx, ny, np), Y.be[sye], Y.ae[sye], Y.ke[sye], d_yz);
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
    T nx_ = cur.ex + SE * cxv, ny_ = cur.ey + SE * cyv, nz_ = cur.ez + SE * czv;
    double jsum = 0.0;
    const uint8_t mb = cur.mb;
    if (mb) {
      const size_t l = (size_t)(k - p.mlo[2]) * m2 + lcol;
      T cS = p.cS, c3 = p.c3, c1 = p.c1, cJ = p.cJ, cG = p.cG, d3 = p.d3, r = T(1);
      if (p.rho) {
        r = (T)p.rho[l];
        d3 = r * p.d3;
        const T inv = T(1) / (p.eps_inf + d3);
        cS = p.S * inv; c3 = T(3) * d3 * inv; c1 = d3 * inv; cJ = p.D2 * inv; cG = inv;
      }
      const T ag = p.agam;
      if (mb & 1u) {
        const T G = r * (cur.qx - cur.q);
        const T en = cur.ex + (cS * cxv - c3 * cur.ex - c1 * cur.emx + cJ * cur.jx - cG * G);
        const T jn = cur.jx + (d3 * (cur.emx + T(2) * cur.ex + en) - ag * cur.jx + G);
        p.Jo[0][l] = jn;
        jsum = (double)jn + (double)p.ebd * ((double)en - (double)cur.ex);
        nx_ = en;
      }
      if (mb & 2u) {
        const T G = r * (cur.qy - cur.q);
        const T en = cur.ey + (cS * cyv - c3 * cur.ey - c1 * cur.emy + cJ * cur.jy - cG * G);
        p.Jo[1][l] = cur.jy + (d3 * (cur.emy + T(2) * cur.ey + en) - ag * cur.jy + G);
        ny_ = en;
      }
      if (mb & 4u) {
        const T G = r * (qz - cur.q);
        const T en = cur.ez + (cS * czv - c3 * cur.ez - c1 * cur.emz + cJ * cur.jz - cG * G);
        p.Jo[2][l] = cur.jz + (d3 * (cur.emz + T(2) * cur.ez + en) - ag * cur.jz + G);
        nz_ = en;
      }
    }
    if (ux) Ox[id] = nx_;
    if (uy) Oy[id] = ny_;
    if (uz) Oz[id] = nz_;
    // per-wavefront plane sum of J_x for the spectra (fixed order)
    const int lz = k - p.mlo[2];
    if (metal_tile && lz >= 0 && lz < p.mn[2]) {
      const double s = wave_sum(jsum);
      if (tx == 0) {
        const int nbxy = p.tl.nbx * p.tl.nby * TY;
        p.jpart[(size_t)k * nbxy + (tile.by * p.tl.nbx + tile.bx) * TY + ty] = s;
      }
    }
    hxm = cur.hx;
    hym = cur.hy;
    cur = nxt;
    mk1 = mk2;
  }
}

// ---------------------------------------------------------------- kernels
// Single simulation: tiles, then the auxiliary-line block last.
template <class T, int TY>
__global__ void __launch_bounds__(kBX* TY) k_h(Params<T> p, AuxParams a) {
  if ((int)blockIdx.x == (int)gridDim.x - 1) {
    aux_h_block(a, threadIdx.y * kBX + threadIdx.x, kBX * TY);
    return;
  }
  h_tile<T, TY>(p, blockIdx.x);
}

template <class T, int TY>
__global__ void __launch_bounds__(kBX* TY) k_ej(Params<T> p, AuxParams a, int sub) {
  if ((int)blockIdx.x == (int)gridDim.x - 1) {
    aux_e_block(a, sub, threadIdx.y * kBX + threadIdx.x, kBX * TY);
    return;
  }
  ej_tile<T, TY>(p, blockIdx.x);
}

// Batch: the blocks of all instances in one launch.  Instance q owns blocks
// [blk0, blk0 + nblk) (its tiles, then its auxiliary-line block); a block
// finds its instance by binary search over the table.
template <class T>
__device__ __forceinline__ int find_instance(const BatchEntry<T>* __restrict__ e, int n, int b,
                                             bool dft) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((dft ? e[mid].dblk0 : e[mid].hblk0) <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class T, int TY>
__global__ void __launch_bounds__(kBX* TY) k_h_batch(const BatchEntry<T>* __restrict__ e, int n) {
  const BatchEntry<T>& en = e[find_instance(e, n, blockIdx.x, false)];
  const int b = blockIdx.x - en.hblk0;
  if (b == en.hnblk - 1) {
    aux_h_block(en.a, threadIdx.y * kBX + threadIdx.x, kBX * TY);
    return;
  }
  h_tile<T, TY>(en.p, b);
}

template <class T, int TY>
__global__ void __launch_bounds__(kBX* TY) k_ej_batch(const BatchEntry<T>* __restrict__ e, int n,
                                                      int sub) {
  const BatchEntry<T>& en = e[find_instance(e, n, blockIdx.x, false)];
  const int b = blockIdx.x - en.hblk0;
  if (b == en.hnblk - 1) {
    aux_e_block(en.a, sub, threadIdx.y * kBX + threadIdx.x, kBX * TY);
    return;
  }
  ej_tile<T, TY>(en.p, b);
}

}  // namespace

Tiling make_tiling(int nx, int ny, int nz, int ty, int kz, int xcd) {
  Tiling t;
  t.ty = ty;
  t.kz = kz;
  t.xcd = xcd;
  t.nbx = (nx + kBX - 1) / kBX;
  t.nby = (ny + ty - 1) / ty;
  t.nbz = (nz + kz - 1) / kz;
  const int tiles = t.nbx * t.nby * t.nbz;
  t.q = t.nbx * 8;  // chunk: 8 rows of tiles
  if (xcd == 2) t.per = ((tiles + t.q - 1) / t.q + 7) / 8;  // chunks per XCD
  else t.per = (tiles + 7) / 8;
  return t;
}

int sweep_blocks(const Tiling& t) {
  // + the auxiliary-line block
  const int tiles = t.xcd == 1 ? 8 * t.per : (t.xcd == 2 ? 8 * t.per * t.q : t.nbx * t.nby * t.nbz);
  return tiles + 1;
}

template <class T>
void launch_h(const Params<T>& p, const AuxParams& a, hipStream_t s) {
  const int blocks = sweep_blocks(p.tl);
  if (p.tl.ty == 4) hipLaunchKernelGGL((k_h<T, 4>), dim3(blocks), dim3(kBX, 4), 0, s, p, a);
  else if (p.tl.ty == 8) hipLaunchKernelGGL((k_h<T, 8>), dim3(blocks), dim3(kBX, 8), 0, s, p, a);
  else hipLaunchKernelGGL((k_h<T, 2>), dim3(blocks), dim3(kBX, 2), 0, s, p, a);
}
template <class T>
void launch_ej(const Params<T>& p, const AuxParams& a, int sub, hipStream_t s) {
  const int blocks = sweep_blocks(p.tl);
  if (p.tl.ty == 4) hipLaunchKernelGGL((k_ej<T, 4>), dim3(blocks), dim3(kBX, 4), 0, s, p, a, sub);
  else if (p.tl.ty == 8) hipLaunchKernelGGL((k_ej<T, 8>), dim3(blocks), dim3(kBX, 8), 0, s, p, a, sub);
  else hipLaunchKernelGGL((k_ej<T, 2>), dim3(blocks), dim3(kBX, 2), 0, s, p, a, sub);
}

template <class T>
void launch_h_batch(const BatchEntry<T>* e, int n, int blocks, int ty, hipStream_t s) {
  if (ty == 4) hipLaunchKernelGGL((k_h_batch<T, 4>), dim3(blocks), dim3(kBX, 4), 0, s, e, n);
  else if (ty == 8) hipLaunchKernelGGL((k_h_batch<T, 8>), dim3(blocks), dim3(kBX, 8), 0, s, e, n);
  else hipLaunchKernelGGL((k_h_batch<T, 2>), dim3(blocks), dim3(kBX, 2), 0, s, e, n);
}
template <class T>
void launch_ej_batch(const BatchEntry<T>* e, int n, int blocks, int ty, int sub, hipStream_t s) {
  if (ty == 4) hipLaunchKernelGGL((k_ej_batch<T, 4>), dim3(blocks), dim3(kBX, 4), 0, s, e, n, sub);
  else if (ty == 8) hipLaunchKernelGGL((k_ej_batch<T, 8>), dim3(blocks), dim3(kBX, 8), 0, s, e, n, sub);
  else hipLaunchKernelGGL((k_ej_batch<T, 2>), dim3(blocks), dim3(kBX, 2), 0, s, e, n, sub);
}
template void launch_h_batch<float>(const BatchEntry<float>*, int, int, int, hipStream_t);
template void launch_h_batch<double>(const BatchEntry<double>*, int, int, int, hipStream_t);
template void launch_ej_batch<float>(const BatchEntry<float>*, int, int, int, int, hipStream_t);
template void launch_ej_batch<double>(const BatchEntry<double>*, int, int, int, int, hipStream_t);

template void launch_h<float>(const Params<float>&, const AuxParams&, hipStream_t);
template void launch_h<double>(const Params<double>&, const AuxParams&, hipStream_t);
template void launch_ej<float>(const Params<float>&, const AuxParams&, int, hipStream_t);
template void launch_ej<double>(const Params<double>&, const AuxParams&, int, hipStream_t);

}  // namespace gnor

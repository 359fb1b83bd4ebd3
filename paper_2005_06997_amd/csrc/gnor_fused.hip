// Fused step of libgnorfdtd (gfx950): f1, f2 and f4 of Sec. III in one pass
// over the grid.  The two-pass form (k_h then k_ej) reads E^n twice and
// writes then re-reads H^{n+1/2}: 18 words per plain Yee cell.  Here a tile
// computes H^{n+1/2} and immediately E^{n+1} from it: 12 words per cell
// (read E^n, H^{n-1/2}; write H^{n+1/2}, E^{n+1}).
//
// Block: TY "row" wavefronts (rows j0 .. j0+TY-1, 64 columns x0 .. x0+63 on
// the lanes) and two "halo" wavefronts, marching the planes of the tile.  Per
// plane k (every wavefront issues all its loads of the plane as one batch):
//   1. each row wavefront computes H^{n+1/2} of its row (stored, and put in
//      LDS for its neighbours); in metal tiles also the node scalars of plane
//      k+1 (Phi_P, Phi_J stored; Q into LDS);
//      the halo wavefronts recompute, from E^n and H^{n-1/2}, the H values
//      the tile's E update needs from outside it (row j0-1: H_x, H_z; column
//      x0-1: H_z, H_y) and the Q values of row j0+TY and column x0+64;
//   2. barrier;
//   3. each row wavefront computes E^{n+1} (and J^{n+1/2}) of its row.
// H at plane k-1 of the own column is carried in registers; at the first
// plane of a tile it is recomputed.  Because halos are recomputed, H and the
// H-slab CPML memory are read from the step's input buffers and written to
// its output buffers, so no tile sees another tile's new values.
//
// The E update's TF/SF corrections need H_inc^{n+1/2}; it is evaluated from
// the auxiliary line (E_inc^n, H_inc^{n-1/2}) with the line's own update.
// The line itself is advanced afterwards by a one-block launch (k_aux).
#include "gnor_device.h"

#include <algorithm>

namespace gnor {

namespace {

// H_inc^{n+1/2} at line index q (the auxiliary line's H update, not stored)
__device__ __forceinline__ double h_inc(const AuxParams& a, int q) {
  const double d = a.e1[q + 1] - a.e1[q];
  const double ps = a.bh[q] * a.ph[q] + a.ah[q] * d;
  return a.h1[q] - a.S * (a.kh[q] * d + ps);
}

// Compiler-only fence (no instruction): the loads issued before it stay there,
// so every wavefront pays one memory round trip per plane instead of having
// each load sunk next to its (often conditional) use.
__device__ __forceinline__ void issue_fence() { __asm__ volatile("" ::: "memory"); }

// ---------------------------------------------------------------- halo cells
// Inputs of the H update at one cell, loaded in one batch (clamped addresses;
// values that the cell does not use are never read).
template <class T>
struct HLoads {
  T ex, ey, ez, ex1, ey1, ezy, exy, ezx, eyx, hx, hy, hz;
  T s_yx, s_zx, s_zy, s_xy, s_xz, s_yz;  // psi_H^{n-1/2}
  T xb, xa, xk, yb, ya, yk, zb, za, zk;  // CPML coefficients of the cell's slabs
};

template <class T, bool PML>
__device__ __forceinline__ void h_load(const Params<T>& p, int i, int j, int k, HLoads<T>& v) {
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int ic = min(max(i, 0), nx - 1), jc = min(max(j, 0), ny - 1), kc = min(max(k, 0), nz - 1);
  const size_t sy = nx, sz = (size_t)nx * ny;
  const size_t id = ((size_t)kc * ny + jc) * nx + ic;
  const size_t dz = kc <= nz - 2 ? sz : 0, dy = jc <= ny - 2 ? sy : 0, dx = ic <= nx - 2 ? 1 : 0;
  v.ex = p.E[0][id]; v.ey = p.E[1][id]; v.ez = p.E[2][id];
  v.ex1 = p.E[0][id + dz]; v.ey1 = p.E[1][id + dz];
  v.ezy = p.E[2][id + dy]; v.exy = p.E[0][id + dy];
  v.ezx = p.E[2][id + dx]; v.eyx = p.E[1][id + dx];
  v.hx = p.Hi[0][id]; v.hy = p.Hi[1][id]; v.hz = p.Hi[2][id];
  if (PML) {
    const int np = p.cp[0].np;
    const int sx = max(slab_h(ic, nx, np), 0), sy_ = max(slab_h(jc, ny, np), 0);
    const int sz_ = max(slab_h(kc, nz, np), 0);
    v.s_yx = p.psiHi[1][0][slab_index(1, sy_, ic, jc, kc, nx, ny, np)];
    v.s_yz = p.psiHi[1][1][slab_index(1, sy_, ic, jc, kc, nx, ny, np)];
    v.s_zx = p.psiHi[2][1][slab_index(2, sz_, ic, jc, kc, nx, ny, np)];
    v.s_zy = p.psiHi[2][0][slab_index(2, sz_, ic, jc, kc, nx, ny, np)];
    v.s_xy = p.psiHi[0][1][slab_index(0, sx, ic, jc, kc, nx, ny, np)];
    v.s_xz = p.psiHi[0][0][slab_index(0, sx, ic, jc, kc, nx, ny, np)];
    v.xb = p.cp[0].bh[sx]; v.xa = p.cp[0].ah[sx]; v.xk = p.cp[0].kh[sx];
    v.yb = p.cp[1].bh[sy_]; v.ya = p.cp[1].ah[sy_]; v.yk = p.cp[1].kh[sy_];
    v.zb = p.cp[2].bh[sz_]; v.za = p.cp[2].ah[sz_]; v.zk = p.cp[2].kh[sz_];
  }
}

// H^{n+1/2} at cell (i, j, k) from loaded inputs; nothing is stored.  Cells
// outside the grid and components the update does not touch give 0 (such H
// points are never updated and stay 0).
template <class T, bool PML>
__device__ __forceinline__ void h_eval(const Params<T>& p, int i, int j, int k, bool want_x,
                                       bool want_y, bool want_z, const HLoads<T>& v, T& hx, T& hy,
                                       T& hz) {
  hx = hy = hz = T(0);
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  if (i < 0 || j < 0 || k < 0 || i >= nx || j >= ny || k >= nz) return;
  const bool xin = i <= nx - 2, yin = j <= ny - 2, zin = k <= nz - 2;
  const bool ux = want_x && i >= 1 && xin && yin && zin;
  const bool uy = want_y && xin && j >= 1 && yin && zin;
  const bool uz = want_z && xin && yin && k >= 1 && zin;
  T dyx = v.ezy - v.ez, dzx = v.ey1 - v.ey;  // H_x: dy Ez - dz Ey
  T dzy = v.ex1 - v.ex, dxy = v.ezx - v.ez;  // H_y: dz Ex - dx Ez
  T dxz = v.eyx - v.ey, dyz = v.exy - v.ex;  // H_z: dx Ey - dy Ex
  if (PML) {
    const int np = p.cp[0].np;
    const bool sx = slab_h(i, nx, np) >= 0, sy = slab_h(j, ny, np) >= 0, sz = slab_h(k, nz, np) >= 0;
    if (sy) { dyx = v.yk * dyx + (v.yb * v.s_yx + v.ya * dyx); dyz = v.yk * dyz + (v.yb * v.s_yz + v.ya * dyz); }
    if (sz) { dzx = v.zk * dzx + (v.zb * v.s_zx + v.za * dzx); dzy = v.zk * dzy + (v.zb * v.s_zy + v.za * dzy); }
    if (sx) { dxy = v.xk * dxy + (v.xb * v.s_xy + v.xa * dxy); dxz = v.xk * dxz + (v.xb * v.s_xz + v.xa * dxz); }
  }
  T cyv = dzy - dxy, czv = dxz - dyz;
  if (p.tfsf && i >= p.tf_lo[0] && i <= p.tf_hi[0] - 1) {
    if (j >= p.tf_lo[1] && j <= p.tf_hi[1]) {
      if (k == p.tf_lo[2] - 1) cyv -= (T)p.e1[p.tf_lo[2] + kAuxOff];
      if (k == p.tf_hi[2]) cyv += (T)p.e1[p.tf_hi[2] + kAuxOff];
    }
    if ((j == p.tf_lo[1] - 1 || j == p.tf_hi[1]) && k >= p.tf_lo[2] && k <= p.tf_hi[2]) {
      const T inc = (T)p.e1[k + kAuxOff];
      czv += (j == p.tf_lo[1] - 1) ? inc : -inc;
    }
  }
  if (ux) hx = v.hx - p.S * (dyx - dzx);
  if (uy) hy = v.hy - p.S * cyv;
  if (uz) hz = v.hz - p.S * czv;
}

// Inputs of the node scalars at one node (clamped addresses; act = the node
// touches a metal edge, else Q = 0).
template <class T>
struct QLoads {
  T jx, jy, jz, jxm, jym, jzm, pp, pj;
  bool act;
};
template <class T>
__device__ __forceinline__ void q_load(const Params<T>& p, int i, int j, int k, QLoads<T>& v) {
  const int lx = i - p.mlo[0], ly = j - p.mlo[1], lz = k - p.mlo[2];
  const bool in = lx >= 0 && ly >= 0 && lz >= 0 && lx < p.mn[0] && ly < p.mn[1] && lz < p.mn[2];
  const size_t m1 = p.mn[0], m2 = (size_t)p.mn[0] * p.mn[1];
  const size_t col = in ? (size_t)ly * m1 + lx : 0;
  const int zlo = p.colz[2 * col], zhi = p.colz[2 * col + 1];
  v.act = in && lz >= zlo && lz <= zhi;
  const size_t l = v.act ? (size_t)lz * m2 + col : 0;
  v.jx = p.Ji[0][l]; v.jy = p.Ji[1][l]; v.jz = p.Ji[2][l];
  v.jxm = p.Ji[0][(v.act && lx > 0) ? l - 1 : 0];
  v.jym = p.Ji[1][(v.act && ly > 0) ? l - m1 : 0];
  v.jzm = p.Ji[2][(v.act && lz > 0) ? l - m2 : 0];
  v.pp = p.PPi[l]; v.pj = p.PJi[l];
}
// Q = g1 Phi_P^n + g2 (3 Phi_J^{n-1/2} - Phi_J^{n-3/2}) with Phi_P^n = Phi_P^{n-1} +
// Phi_J^{n-1/2}, Phi_J^{n-1/2} = Div J^{n-1/2}; returns Phi_P^n, Phi_J^{n-1/2} too.
template <class T>
__device__ __forceinline__ T q_eval(const Params<T>& p, int i, int j, int k, const QLoads<T>& v,
                                    T& phiP, T& div) {
  phiP = div = T(0);
  if (!v.act) return T(0);
  const int lx = i - p.mlo[0], ly = j - p.mlo[1], lz = k - p.mlo[2];
  const T jxm = lx > 0 ? v.jxm : T(0), jym = ly > 0 ? v.jym : T(0), jzm = lz > 0 ? v.jzm : T(0);
  div = (v.jx - jxm) + (v.jy - jym) + (v.jz - jzm);
  phiP = v.pp + div;
  return p.g1 * phiP + p.g2 * (T(3) * div - v.pj);
}

template <class T, int TY>
struct StepLds {
  T hz[2][TY + 1][kBX + 1];  // H_z of rows j0-1 .. j0+TY-1; [..][0] = column x0-1
  T hx[2][TY + 1][kBX];      // H_x of rows j0-1 .. j0+TY-1
  T hy[2][TY][kBX + 1];      // H_y of rows j0 .. j0+TY-1; [..][0] = column x0-1
};
template <class T, int TY>
struct StepLdsQ {
  T q[3][TY + 1][kBX + 1];   // Q of rows j0 .. j0+TY; [..][kBX] = column x0+64
};

// ---------------------------------------------------------------- one tile
template <class T, int TY, bool METAL, bool PML>
__device__ __forceinline__ void step_tile(const Params<T>& p, const AuxParams& a, const Tile tile,
                                          bool pml_tile, StepLds<T, TY>& L, StepLdsQ<T, TY>* LQ) {
  const int l = threadIdx.x, w = threadIdx.y;
  // wavefronts TY and TY+1 compute the halo: row j0-1 (and Q of row j0+TY),
  // column x0-1 (and Q of column x0+64) on lanes < TY
  const bool halo = w >= TY;
  const bool hrow = w == TY;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int x0 = tile.bx * kBX, j0 = tile.by * TY;
  const int i = x0 + l, j = j0 + w;
  const int k0 = tile.bz * p.tl.kz;
  const int k1 = min(nz, k0 + p.tl.kz);
  const bool active = !halo && i < nx && j < ny;
  const size_t sy = nx, sz = (size_t)nx * ny;
  const int np = p.cp[0].np;
  const bool pml = PML && pml_tile;
  // ---- row wavefront: per-column constants
  const bool xin = i <= nx - 2, yin = j <= ny - 2;
  const bool cx = active && i >= 1 && xin && yin;  // H update columns
  const bool cy = active && xin && j >= 1 && yin;
  const bool cz = active && xin && yin;
  const bool ax = active && i <= nx - 2 && j >= 1 && j <= ny - 2;  // E update columns
  const bool ay = active && i >= 1 && i <= nx - 2 && j <= ny - 2;
  const bool az = active && i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2;
  const int sxh = (pml && active) ? slab_h(i, nx, np) : -1;
  const int syh = (pml && active) ? slab_h(j, ny, np) : -1;
  const int sxe = (pml && active) ? slab_e(i, nx, np) : -1;
  const int sye = (pml && active) ? slab_e(j, ny, np) : -1;
  T hxb = T(0), hxa = T(0), hxk = T(1), hyb = T(0), hya = T(0), hyk = T(1);
  T exb = T(0), exa = T(0), exk = T(1), eyb = T(0), eya = T(0), eyk = T(1);
  if (sxh >= 0) { hxb = p.cp[0].bh[sxh]; hxa = p.cp[0].ah[sxh]; hxk = p.cp[0].kh[sxh]; }
  if (syh >= 0) { hyb = p.cp[1].bh[syh]; hya = p.cp[1].ah[syh]; hyk = p.cp[1].kh[syh]; }
  if (sxe >= 0) { exb = p.cp[0].be[sxe]; exa = p.cp[0].ae[sxe]; exk = p.cp[0].ke[sxe]; }
  if (sye >= 0) { eyb = p.cp[1].be[sye]; eya = p.cp[1].ae[sye]; eyk = p.cp[1].ke[sye]; }
  const bool tfx = p.tfsf && active && i >= p.tf_lo[0] && i <= p.tf_hi[0] - 1;
  const bool tfy_band = tfx && j >= p.tf_lo[1] && j <= p.tf_hi[1];
  const bool tfz_lo = tfx && j == p.tf_lo[1] - 1, tfz_hi = tfx && j == p.tf_hi[1];
  const bool tf_zside = p.tfsf && active && j >= p.tf_lo[1] && j <= p.tf_hi[1] &&
                        (i == p.tf_lo[0] || i == p.tf_hi[0]);
  // the TF/SF incident values of the tile's planes are uniform: E_inc^n read
  // and H_inc^{n+1/2} evaluated per plane only where a correction applies
  // metal sub-grid column of the row lane
  const int lx = i - p.mlo[0], ly = j - p.mlo[1];
  const bool col_sub = METAL && active && lx >= 0 && ly >= 0 && lx < p.mn[0] && ly < p.mn[1];
  const size_t m1 = p.mn[0], m2 = (size_t)p.mn[0] * p.mn[1];
  const size_t lcol = col_sub ? (size_t)ly * m1 + lx : 0;
  int zlo = 1, zhi = 0;  // nodes of the column that touch a metal edge
  if (METAL && col_sub) {
    zlo = p.colz[2 * lcol];
    zhi = p.colz[2 * lcol + 1];
  }
  const T S = p.S, SE = p.SE;

  // ---- carried state (row wavefronts)
  const size_t id_base = active ? ((size_t)j * nx + i) : 0;
  T ex0 = T(0), ey0 = T(0);  // E_x, E_y^n of plane k
  T hxm = T(0), hym = T(0);  // H_x, H_y^{n+1/2} of plane k-1
  T jcx = T(0), jcy = T(0), jcz = T(0), qc = T(0);  // J^{n-1/2} and Q at plane k (metal)
  uint32_t mbk = 0u;         // metal bits of plane k
  {
    // first plane: E^n and the H of plane k0-1 (recomputed) / halo state
    HLoads<T> v;
    h_load<T, PML>(p, i, j, k0 - 1, v);
    T ex_ = T(0), ey_ = T(0);
    if (active) {
      const size_t id0 = (size_t)k0 * sz + id_base;
      ex_ = p.E[0][id0];
      ey_ = p.E[1][id0];
    }
    QLoads<T> qv;
    if (METAL) {
      if (!halo) q_load(p, i, j, k0, qv);
      else if (hrow) q_load(p, x0 + l, j0 + TY, k0, qv);
      else q_load(p, x0 + kBX, j0 + min(l, TY - 1), k0, qv);
    }
    uint32_t m0 = 0u;
    if (METAL) {
      const int lz = k0 - p.mlo[2];
      const bool ok = col_sub && lz >= 0 && lz < p.mn[2];
      const uint32_t mm = p.mask[ok ? (size_t)lz * m2 + lcol : 0];
      m0 = ok ? mm : 0u;
    }
    issue_fence();
    ex0 = ex_;
    ey0 = ey_;
    if (active) {
      T hz_;
      h_eval<T, PML>(p, i, j, k0 - 1, true, true, false, v, hxm, hym, hz_);
    }
    if (METAL) {
      mbk = m0;
      T pP, dv;
      if (hrow) {
        LQ->q[k0 % 3][TY][l] = q_eval(p, x0 + l, j0 + TY, k0, qv, pP, dv);
      } else if (halo) {
        const T qq = q_eval(p, x0 + kBX, j0 + min(l, TY - 1), k0, qv, pP, dv);
        if (l < TY) LQ->q[k0 % 3][l][kBX] = qq;
      } else {
        qc = q_eval(p, i, j, k0, qv, pP, dv);
        if (qv.act) {
          const size_t ll = (size_t)(k0 - p.mlo[2]) * m2 + lcol;
          p.PPo[ll] = pP;
          p.PJo[ll] = dv;
          p.Q[ll] = qc;  // for two-sweep neighbours (hybrid form)
        }
        jcx = qv.act ? qv.jx : T(0);
        jcy = qv.act ? qv.jy : T(0);
        jcz = qv.act ? qv.jz : T(0);
        LQ->q[k0 % 3][w][l] = qc;
      }
    }
  }

  for (int k = k0; k < k1; ++k) {
    const int b = k & 1;
    const bool zin = k <= nz - 2;
    T hxc = T(0), hyc = T(0), hzc = T(0);  // H^{n+1/2} of the own cell at plane k
    T ex_k = ex0, ey_k = ey0, ez_k = T(0);  // E^n of the own cell at plane k
    T qn = T(0), jnx = T(0), jny = T(0), jnz = T(0);  // Q and J at plane k+1
    // E-slab CPML memory and metal inputs of plane k (used after the barrier)
    T t_yx = T(0), t_zx = T(0), t_zy = T(0), t_xy = T(0), t_xz = T(0), t_yz = T(0);
    T ezb = T(0), eza = T(0), ezk = T(1);
    T emx = T(0), emy = T(0), emz = T(0), rr = T(1);
    const int sze = pml ? slab_e(k, nz, np) : -1;
    const bool zin_e = k >= 1 && k <= nz - 2;
    const bool vx = ax && zin_e, vy = ay && zin_e, vz = az && k <= nz - 2;
    // ================= phase 1: H^{n+1/2} (and node scalars of plane k+1)
    if (halo) {
      // H that the E update needs from outside the tile (row j0-1: H_x, H_z;
      // column x0-1: H_z, H_y) and Q of plane k+1 beyond it (row j0+TY,
      // column x0+64)
      const int hi_ = hrow ? x0 + l : x0 - 1, hj = hrow ? j0 - 1 : j0 + min(l, TY - 1);
      const int qi = hrow ? x0 + l : x0 + kBX, qj = hrow ? j0 + TY : j0 + min(l, TY - 1);
      HLoads<T> v;
      h_load<T, PML>(p, hi_, hj, k, v);
      QLoads<T> qq;
      if (METAL) q_load(p, qi, qj, k + 1, qq);
      issue_fence();
      T hx_, hy_, hz_;
      h_eval<T, PML>(p, hi_, hj, k, hrow, !hrow, true, v, hx_, hy_, hz_);
      T qv_ = T(0);
      if (METAL) {
        T pP, dv;
        qv_ = q_eval(p, qi, qj, k + 1, qq, pP, dv);
      }
      if (hrow) {
        L.hx[b][0][l] = hx_;
        L.hz[b][0][l + 1] = hz_;
        if (METAL) LQ->q[(k + 1) % 3][TY][l] = qv_;
      } else if (l < TY) {
        L.hz[b][l + 1][0] = hz_;
        L.hy[b][l][0] = hy_;
        if (METAL) LQ->q[(k + 1) % 3][l][kBX] = qv_;
      }
    } else {
      const bool ux = cx && zin, uy = cy && zin, uz = cz && k >= 1 && zin;
      const size_t id = (size_t)k * sz + id_base;
      // ---- the plane's loads, one batch
      const size_t up = (active && zin) ? sz : 0;
      const T ex1r = p.E[0][id + up], ey1r = p.E[1][id + up];
      const T ezr = p.E[2][id];
      const T ezyr = p.E[2][id + ((active && yin) ? sy : 0)];
      const T exyr = p.E[0][id + ((active && yin) ? sy : 0)];
      const T ezxr = p.E[2][id + ((active && xin) ? 1 : 0)];
      const T eyxr = p.E[1][id + ((active && xin) ? 1 : 0)];
      const T hxr = p.Hi[0][id], hyr = p.Hi[1][id], hzr = p.Hi[2][id];
      T s_yx = T(0), s_zx = T(0), s_zy = T(0), s_xy = T(0), s_xz = T(0), s_yz = T(0);
      T hzb = T(0), hza = T(0), hzk = T(1);
      int szh = -1;
      if (pml) {
        szh = slab_h(k, nz, np);
        const int zs = max(szh, 0), zse = max(sze, 0), xs = max(sxh, 0), ys = max(syh, 0);
        const int xse = max(sxe, 0), yse = max(sye, 0);
        const int ic = active ? i : 0, jc = active ? j : 0;
        s_yx = p.psiHi[1][0][slab_index(1, ys, ic, jc, k, nx, ny, np)];
        s_yz = p.psiHi[1][1][slab_index(1, ys, ic, jc, k, nx, ny, np)];
        s_zx = p.psiHi[2][1][slab_index(2, zs, ic, jc, k, nx, ny, np)];
        s_zy = p.psiHi[2][0][slab_index(2, zs, ic, jc, k, nx, ny, np)];
        s_xy = p.psiHi[0][1][slab_index(0, xs, ic, jc, k, nx, ny, np)];
        s_xz = p.psiHi[0][0][slab_index(0, xs, ic, jc, k, nx, ny, np)];
        t_yx = p.psiE[1][0][slab_index(1, yse, ic, jc, k, nx, ny, np)];
        t_yz = p.psiE[1][1][slab_index(1, yse, ic, jc, k, nx, ny, np)];
        t_zx = p.psiE[2][1][slab_index(2, zse, ic, jc, k, nx, ny, np)];
        t_zy = p.psiE[2][0][slab_index(2, zse, ic, jc, k, nx, ny, np)];
        t_xy = p.psiE[0][1][slab_index(0, xse, ic, jc, k, nx, ny, np)];
        t_xz = p.psiE[0][0][slab_index(0, xse, ic, jc, k, nx, ny, np)];
        hzb = p.cp[2].bh[zs]; hza = p.cp[2].ah[zs]; hzk = p.cp[2].kh[zs];
        ezb = p.cp[2].be[zse]; eza = p.cp[2].ae[zse]; ezk = p.cp[2].ke[zse];
      }
      QLoads<T> qv;
      uint32_t mnext = 0u;
      if (METAL) {
        // node inputs of plane k+1, metal bits of plane k+1, E^{n-1} and the
        // design weight of plane k
        q_load(p, i, j, k + 1, qv);
        qv.act = qv.act && col_sub && k + 1 < nz;
        const int lz1 = k + 1 - p.mlo[2];
        const bool ok1 = col_sub && lz1 >= 0 && lz1 < p.mn[2];
        const uint32_t mm = p.mask[ok1 ? (size_t)lz1 * m2 + lcol : 0];
        mnext = ok1 ? mm : 0u;
        const size_t ll = mbk ? (size_t)(k - p.mlo[2]) * m2 + lcol : 0;
        emx = p.O[0][(mbk & 1u) ? id : 0];
        emy = p.O[1][(mbk & 2u) ? id : 0];
        emz = p.O[2][(mbk & 4u) ? id : 0];
        if (p.rho) rr = (T)p.rho[ll];
      }
      issue_fence();
      // ---- f1: H^{n+1/2} of the own row
      if (active) {
        ez_k = ezr;
        const T ex1 = zin ? ex1r : T(0), ey1 = zin ? ey1r : T(0);
        const T ezy = yin ? ezyr : T(0), exy = yin ? exyr : T(0);
        const T ezx = xin ? ezxr : T(0), eyx = xin ? eyxr : T(0);
        T dyx = ezy - ez_k, dzx = ey1 - ey0;  // H_x: dy Ez - dz Ey
        T dzy = ex1 - ex0, dxy = ezx - ez_k;  // H_y: dz Ex - dx Ez
        T dxz = eyx - ey0, dyz = exy - ex0;   // H_z: dx Ey - dy Ex
        if (pml) {
          if (ux && syh >= 0) {
            const T ps = hyb * s_yx + hya * dyx;
            p.psiH[1][0][slab_index(1, syh, i, j, k, nx, ny, np)] = ps;
            dyx = hyk * dyx + ps;
          }
          if (ux && szh >= 0) {
            const T ps = hzb * s_zx + hza * dzx;
            p.psiH[2][1][slab_index(2, szh, i, j, k, nx, ny, np)] = ps;
            dzx = hzk * dzx + ps;
          }
          if (uy && szh >= 0) {
            const T ps = hzb * s_zy + hza * dzy;
            p.psiH[2][0][slab_index(2, szh, i, j, k, nx, ny, np)] = ps;
            dzy = hzk * dzy + ps;
          }
          if (uy && sxh >= 0) {
            const T ps = hxb * s_xy + hxa * dxy;
            p.psiH[0][1][slab_index(0, sxh, i, j, k, nx, ny, np)] = ps;
            dxy = hxk * dxy + ps;
          }
          if (uz && sxh >= 0) {
            const T ps = hxb * s_xz + hxa * dxz;
            p.psiH[0][0][slab_index(0, sxh, i, j, k, nx, ny, np)] = ps;
            dxz = hxk * dxz + ps;
          }
          if (uz && syh >= 0) {
            const T ps = hyb * s_yz + hya * dyz;
            p.psiH[1][1][slab_index(1, syh, i, j, k, nx, ny, np)] = ps;
            dyz = hyk * dyz + ps;
          }
        }
        T cyv = dzy - dxy, czv = dxz - dyz;
        // TF/SF: scattered-field H next to the TF box sees E_inc^n on the TF side
        if (tfy_band) {
          if (k == p.tf_lo[2] - 1) cyv -= (T)p.e1[p.tf_lo[2] + kAuxOff];
          if (k == p.tf_hi[2]) cyv += (T)p.e1[p.tf_hi[2] + kAuxOff];
        }
        if ((tfz_lo || tfz_hi) && k >= p.tf_lo[2] && k <= p.tf_hi[2]) {
          const T inc = (T)p.e1[k + kAuxOff];
          czv += tfz_lo ? inc : -inc;
        }
        if (ux) { hxc = hxr - S * (dyx - dzx); p.H[0][id] = hxc; }
        if (uy) { hyc = hyr - S * cyv; p.H[1][id] = hyc; }
        if (uz) { hzc = hzr - S * czv; p.H[2][id] = hzc; }
        ex0 = ex1;
        ey0 = ey1;
      }
      L.hz[b][w + 1][l + 1] = hzc;
      L.hx[b][w + 1][l] = hxc;
      L.hy[b][w][l + 1] = hyc;
      if (METAL) {
        // node scalars of plane k+1 (the tile's own planes are stored)
        T pP, dv;
        qv.jzm = jcz;  // J_z one plane below = J_z at plane k (0 if that node is inactive)
        qn = q_eval(p, i, j, k + 1, qv, pP, dv);
        if (qv.act && k + 1 < k1) {
          const size_t ll = (size_t)(k + 1 - p.mlo[2]) * m2 + lcol;
          p.PPo[ll] = pP;
          p.PJo[ll] = dv;
          p.Q[ll] = qn;
        }
        jnx = qv.act ? qv.jx : T(0);
        jny = qv.act ? qv.jy : T(0);
        jnz = qv.act ? qv.jz : T(0);
        LQ->q[(k + 1) % 3][w][l] = qn;
        // carried to the next plane
        mbk = mnext | (mbk << 8);  // low byte: plane k+1; next byte: plane k (below)
      }
    }
    __syncthreads();
    // ================= phase 2: E^{n+1} and J^{n+1/2} of the own row
    if (!halo) {
      double jsum = 0.0;
      bool any_m = false;
      const uint32_t mb = METAL ? ((mbk >> 8) & 0xffu) : 0u;
      if (active) {
        const size_t id = (size_t)k * sz + id_base;
        const T hzy = L.hz[b][w][l + 1], hxy = L.hx[b][w][l];
        const T hzx = L.hz[b][w + 1][l], hyx = L.hy[b][w][l];
        const T exn = vx ? ex_k : T(0), eyn = vy ? ey_k : T(0), ezn = vz ? ez_k : T(0);
        T d_yx = hzc - hzy, d_zx = hyc - hym;
        T d_zy = hxc - hxm, d_xy = hzc - hzx;
        T d_xz = hyc - hyx, d_yz = hxc - hxy;
        if (pml) {
          if (vx && sye >= 0) {
            const T ps = eyb * t_yx + eya * d_yx;
            p.psiE[1][0][slab_index(1, sye, i, j, k, nx, ny, np)] = ps;
            d_yx = eyk * d_yx + ps;
          }
          if (vx && sze >= 0) {
            const T ps = ezb * t_zx + eza * d_zx;
            p.psiE[2][1][slab_index(2, sze, i, j, k, nx, ny, np)] = ps;
            d_zx = ezk * d_zx + ps;
          }
          if (vy && sze >= 0) {
            const T ps = ezb * t_zy + eza * d_zy;
            p.psiE[2][0][slab_index(2, sze, i, j, k, nx, ny, np)] = ps;
            d_zy = ezk * d_zy + ps;
          }
          if (vy && sxe >= 0) {
            const T ps = exb * t_xy + exa * d_xy;
            p.psiE[0][1][slab_index(0, sxe, i, j, k, nx, ny, np)] = ps;
            d_xy = exk * d_xy + ps;
          }
          if (vz && sxe >= 0) {
            const T ps = exb * t_xz + exa * d_xz;
            p.psiE[0][0][slab_index(0, sxe, i, j, k, nx, ny, np)] = ps;
            d_xz = exk * d_xz + ps;
          }
          if (vz && sye >= 0) {
            const T ps = eyb * t_yz + eya * d_yz;
            p.psiE[1][1][slab_index(1, sye, i, j, k, nx, ny, np)] = ps;
            d_yz = eyk * d_yz + ps;
          }
        }
        T cxv = d_yx - d_zx, cyv = d_zy - d_xy, czv = d_xz - d_yz;
        // TF/SF with H_inc^{n+1/2} (evaluated from the line)
        if (tfy_band) {
          if (k == p.tf_lo[2]) cxv += (T)h_inc(a, p.tf_lo[2] - 1 + kAuxOff);
          if (k == p.tf_hi[2]) cxv -= (T)h_inc(a, p.tf_hi[2] + kAuxOff);
        }
        if (tf_zside && k >= p.tf_lo[2] && k <= p.tf_hi[2] - 1) {
          const T inc = (T)h_inc(a, k + kAuxOff);
          czv += (i == p.tf_lo[0]) ? -inc : inc;
        }
        T nx_ = exn + SE * cxv, ny_ = eyn + SE * cyv, nz_ = ezn + SE * czv;
        if (METAL && mb) {
          any_m = true;
          const size_t ll = (size_t)(k - p.mlo[2]) * m2 + lcol;
          const bool b0 = mb & 1u, b1 = mb & 2u, b2 = mb & 4u;
          const T qx = LQ->q[k % 3][w][l + 1];
          const T qy = LQ->q[k % 3][w + 1][l];
          T cS = p.cS, c3 = p.c3, c1 = p.c1, cJ = p.cJ, cG = p.cG, d3 = p.d3;
          const T r = rr;
          if (p.rho) {
            d3 = r * p.d3;
            const T inv = T(1) / (p.eps_inf + d3);
            cS = p.S * inv; c3 = T(3) * d3 * inv; c1 = d3 * inv; cJ = p.D2 * inv; cG = inv;
          }
          const T ag = p.agam;
          if (b0) {
            const T G = r * (qx - qc);
            const T en = exn + (cS * cxv - c3 * exn - c1 * emx + cJ * jcx - cG * G);
            const T jn = jcx + (d3 * (emx + T(2) * exn + en) - ag * jcx + G);
            p.Jo[0][ll] = jn;
            jsum = (double)jn + (double)p.ebd * ((double)en - (double)exn);
            nx_ = en;
          }
          if (b1) {
            const T G = r * (qy - qc);
            const T en = eyn + (cS * cyv - c3 * eyn - c1 * emy + cJ * jcy - cG * G);
            p.Jo[1][ll] = jcy + (d3 * (emy + T(2) * eyn + en) - ag * jcy + G);
            ny_ = en;
          }
          if (b2) {
            const T G = r * (qn - qc);
            const T en = ezn + (cS * czv - c3 * ezn - c1 * emz + cJ * jcz - cG * G);
            p.Jo[2][ll] = jcz + (d3 * (emz + T(2) * ezn + en) - ag * jcz + G);
            nz_ = en;
          }
        }
        if (vx) p.O[0][id] = nx_;
        if (vy) p.O[1][id] = ny_;
        if (vz) p.O[2][id] = nz_;
      }
      if (METAL) {
        // per-wavefront plane sum of J_x for the spectra (fixed order; all
        // lanes take part); a wavefront without metal keeps its zero entry
        const int lz = k - p.mlo[2];
        if (lz >= 0 && lz < p.mn[2] && __any(any_m)) {
          const double s_ = wave_sum(jsum);
          if (l == 0) {
            const int nbxy = p.tl.nbx * p.tl.nby * TY;
            p.jpart[(size_t)k * nbxy + (tile.by * p.tl.nbx + tile.bx) * TY + w] = s_;
          }
        }
        mbk &= 0xffu;
      }
      hxm = hxc;
      hym = hyc;
      qc = qn;
      jcx = jnx;
      jcy = jny;
      jcz = jnz;
    }
  }
}

template <class T, int TY, int CLS>
__global__ void __launch_bounds__(kBX*(TY + 2)) k_step(Params<T> p, AuxParams a) {
  __shared__ StepLds<T, TY> L;
  const Tile tile = decode_tile(p.tl, p.tiles, CLS, blockIdx.x);
  if (!tile.ok) return;
  if constexpr (CLS == 0) {
    step_tile<T, TY, false, false>(p, a, tile, false, L, nullptr);
  } else if constexpr (CLS == 1) {
    step_tile<T, TY, false, true>(p, a, tile, true, L, nullptr);
  } else if constexpr (CLS == 2) {
    __shared__ StepLdsQ<T, TY> LQ;
    step_tile<T, TY, true, false>(p, a, tile, false, L, &LQ);
  } else {
    __shared__ StepLdsQ<T, TY> LQ;
    step_tile<T, TY, true, true>(p, a, tile, true, L, &LQ);
  }
}

// The auxiliary line's step (H half, then E half with the soft source and the
// spectra's phase table), after the fused sweep has read E_inc^n.
__global__ void __launch_bounds__(256) k_aux(AuxParams a, int sub) {
  aux_h_block(a, threadIdx.x, blockDim.x);
  __syncthreads();
  aux_e_block(a, sub, threadIdx.x, blockDim.x);
}

template <class T, int CLS>
void launch_step_cls(const Params<T>& p, const AuxParams& a, hipStream_t s) {
  const int blocks = class_blocks(p.tl, CLS);
  if (blocks == 0) return;
  if (p.tl.ty == 4) hipLaunchKernelGGL((k_step<T, 4, CLS>), dim3(blocks), dim3(kBX, 6), 0, s, p, a);
  else if (p.tl.ty == 8) hipLaunchKernelGGL((k_step<T, 8, CLS>), dim3(blocks), dim3(kBX, 10), 0, s, p, a);
  else hipLaunchKernelGGL((k_step<T, 2, CLS>), dim3(blocks), dim3(kBX, 4), 0, s, p, a);
}

}  // namespace

template <class T>
void launch_step_class(const Params<T>& p, const AuxParams& a, int c, hipStream_t s) {
  if (c == 0) launch_step_cls<T, 0>(p, a, s);
  else if (c == 1) launch_step_cls<T, 1>(p, a, s);
  else if (c == 2) launch_step_cls<T, 2>(p, a, s);
  else launch_step_cls<T, 3>(p, a, s);
}
void launch_aux(const AuxParams& a, int sub, hipStream_t s) {
  hipLaunchKernelGGL(k_aux, dim3(1), dim3(256), 0, s, a, sub);
}
template <class T>
void launch_step(const Params<T>& p, const AuxParams& a, int sub, hipStream_t s) {
  for (int c = 0; c < kClasses; ++c) launch_step_class<T>(p, a, c, s);
  launch_aux(a, sub, s);
}
template void launch_step_class<float>(const Params<float>&, const AuxParams&, int, hipStream_t);
template void launch_step_class<double>(const Params<double>&, const AuxParams&, int, hipStream_t);
template void launch_step<float>(const Params<float>&, const AuxParams&, int, hipStream_t);
template void launch_step<double>(const Params<double>&, const AuxParams&, int, hipStream_t);

}  // namespace gnor

// One-pass step of the tiles without metal (gfx950): f1 and f2 of Sec. III
// fused, with the CPML (Roden-Gedney) memory of the slabs a tile meets.  The
// plain class (at most an x slab) and the CPML class (a y or z slab) are
// separate launches with their own register budgets.  The two-sweep
// form reads E^n twice and writes, then re-reads, H^{n+1/2}: 18 field words
// per cell.  Here a tile computes H^{n+1/2} and, at once, E^{n+1} from it:
// 12 words (read E^n and H^{n-1/2}, write H^{n+1/2} and E^{n+1}).
//
// Each wavefront owns one row (64 cells along x) of the tile and marches it
// up the tile's planes.  The E update at (i, j, k) needs H^{n+1/2} at
// (i-1, j, k), (i, j-1, k) and (i, j, k-1).  The plane below is carried in
// registers; the column to the left (H_y, H_z) is the left lane's (a lane
// shuffle), the row below (H_x, H_z) the wavefront below's, through LDS, one
// barrier per plane.  Only the tile's edges recompute halo H from E^n and
// H^{n-1/2}: the first lane of a row that of column x-1, the block's first
// row that of row y-1.  Likewise E at column x+1 is the right lane's, the
// last lane loading the next tile's.  Per cell and plane that is 8 loads,
// against 22 when every wavefront recomputed its halo itself (which ran no
// faster than the two sweeps: the loads, not the bytes, set its pace).  Only
// a cell's own H is stored, and H is read from the step's input buffer and
// written to its output buffer.
//
// TF/SF: the one-pass kernels leave the corrections out.  They are linear
// and sit on the faces of the TF box, so k_tfsf_fix adds them afterwards, at
// the points of one class's tiles only (one launch per one-pass class that
// meets the shell of the TF box): to H^{n+1/2} on the faces the E_inc^n
// terms, and to E^{n+1} the E update's share of those terms plus its own
// H_inc^{n+1/2} terms (evaluated from the line's state with the line's own H
// update; the line advances after the fix).  The background coefficients
// follow the planes (a substrate beyond sub_k).
#include "gnor_device.h"

namespace gnor {

namespace {

template <bool NT, class T>
__device__ __forceinline__ void put(T* a, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, a);
  else *a = v;
}

// H update ranges (PEC walls on the outer node planes): the H point exists and
// is updated iff these hold
__device__ __forceinline__ bool upd_hx(int i, int j, int k, int nx, int ny, int nz) {
  return i >= 1 && i <= nx - 2 && j >= 0 && j <= ny - 2 && k >= 0 && k <= nz - 2;
}
__device__ __forceinline__ bool upd_hy(int i, int j, int k, int nx, int ny, int nz) {
  return i >= 0 && i <= nx - 2 && j >= 1 && j <= ny - 2 && k >= 0 && k <= nz - 2;
}
__device__ __forceinline__ bool upd_hz(int i, int j, int k, int nx, int ny, int nz) {
  return i >= 0 && i <= nx - 2 && j >= 0 && j <= ny - 2 && k >= 1 && k <= nz - 2;
}

// Compiler-only fence: the loads issued before it stay before it (one memory
// round trip per plane).
__device__ __forceinline__ void load_fence() { __asm__ volatile("" ::: "memory"); }

// Neighbour lanes of the wavefront (one row of 64 cells along x): the value
// of lane + 1 and of lane - 1 (a lane without such a neighbour gets its own).
template <class T>
__device__ __forceinline__ T from_right(T v) { return __shfl_down(v, 1, kBX); }
template <class T>
__device__ __forceinline__ T from_left(T v) { return __shfl_up(v, 1, kBX); }

// x-slab coefficients at one position (b = 1, a = 0, k = 1 outside the slab)
template <class T>
struct XCoef {
  T b, a, k;
};
template <class T>
__device__ __forceinline__ XCoef<T> xcoef(const T* b, const T* a, const T* kk, int s) {
  XCoef<T> c{T(1), T(0), T(1)};
  if (s >= 0) { c.b = b[s]; c.a = a[s]; c.k = kk[s]; }
  return c;
}
// CPML-stretched x difference: kinv d + psi, psi <- b psi + a d
template <class T>
__device__ __forceinline__ T xstretch(const XCoef<T>& c, T d, T psi_old, T& psi_new) {
  psi_new = c.b * psi_old + c.a * d;
  return c.k * d + psi_new;
}

// The loads of one plane of a column: E^n around the cell, H^{n-1/2} and
// x-slab memory (of the H and of the E update); E at column x+1 (last lane,
// from the next tile); what the recomputed halos need (first lane: column
// x-1; first row: row y-1).
template <class T>
struct PlaneIn {
  T ez = T(0), ex1 = T(0), ey1 = T(0), ezy = T(0), exy = T(0), hx = T(0), hy = T(0), hz = T(0);
  T sy_ = T(0), sz_ = T(0), ey_ = T(0), ez_ = T(0);
  T ezr = T(0), eyr = T(0);
  T ezl = T(0), eyl = T(0), exl1 = T(0), exly = T(0), hyo = T(0), hzo = T(0), syl = T(0), szl = T(0);
  T eyd1 = T(0), ezd = T(0), exd = T(0), hxo = T(0), hzd_o = T(0), szd = T(0), eydr = T(0);
  // y and z slabs: psi_H of the cell (H_x: dy E_z, dz E_y; H_y: dz E_x; H_z:
  // dy E_x), psi_E of the cell (E_x: dy H_z, dz H_y; E_y: dz H_x; E_z: dy
  // H_x), and the psi_H the recomputed halos need
  T pyx = T(0), pyz = T(0), pzx = T(0), pzy = T(0);
  T qyx = T(0), qyz = T(0), qzx = T(0), qzy = T(0);
  T pyzl = T(0), pzyl = T(0), pyxd = T(0), pyzd = T(0), pzxd = T(0);
};

// y- and z-slab positions of a column's plane (tiles that meet a y or z
// slab): slab-array indices of the cell's H and E points and of its row y-1
// (axis-1 arrays: ((k 2 np + s) nx + i); axis-2: ((s ny + j) nx + i)), and
// whether each lies in its slab (uniform over a row, resp. a plane)
struct YZAt {
  uint32_t qy = 0, qye = 0, qyd = 0, qz = 0, qze = 0;
  bool yh = false, ye = false, yd = false, zh = false, ze = false;
};

template <class T, bool XS, bool YZ>
__device__ __forceinline__ void load_plane(const Params<T>& p, PlaneIn<T>& v, uint32_t id, uint32_t dzp,
                                           uint32_t dyp, uint32_t sy, uint32_t qs, uint32_t qsl,
                                           uint32_t qse, uint32_t sq, const YZAt& yz, bool act,
                                           bool first, bool last, bool rd) {
  const T* __restrict__ Ex = p.E[0];
  const T* __restrict__ Ey = p.E[1];
  const T* __restrict__ Ez = p.E[2];
  if (act) {
    v.ez = Ez[id];
    v.ex1 = Ex[id + dzp]; v.ey1 = Ey[id + dzp];
    v.ezy = Ez[id + dyp]; v.exy = Ex[id + dyp];
    v.hx = p.Hi[0][id]; v.hy = p.Hi[1][id]; v.hz = p.Hi[2][id];
    if (XS) {
      v.sy_ = p.psiHi[0][1][qs]; v.sz_ = p.psiHi[0][0][qs];
      v.ey_ = p.psiE[0][1][qse]; v.ez_ = p.psiE[0][0][qse];
    }
  }
  if (last) { v.ezr = Ez[id + 1]; v.eyr = Ey[id + 1]; }
  if (first) {
    const uint32_t ql = id - 1;
    v.ezl = Ez[ql]; v.eyl = Ey[ql]; v.exl1 = Ex[ql + dzp]; v.exly = Ex[ql + dyp];
    v.hyo = p.Hi[1][ql]; v.hzo = p.Hi[2][ql];
    if (XS) { v.syl = p.psiHi[0][1][qsl]; v.szl = p.psiHi[0][0][qsl]; }
  }
  if (rd) {
    const uint32_t qd = id - sy;
    v.ezd = Ez[qd]; v.eyd1 = Ey[qd + dzp]; v.exd = Ex[qd];
    v.hxo = p.Hi[0][qd]; v.hzd_o = p.Hi[2][qd];
    if (XS) v.szd = p.psiHi[0][0][qs - sq];
    if (last) v.eydr = Ey[qd + 1];
  }
  if (YZ) {
    if (act && yz.yh) { v.pyx = p.psiHi[1][0][yz.qy]; v.pyz = p.psiHi[1][1][yz.qy]; }
    if (act && yz.zh) { v.pzx = p.psiHi[2][1][yz.qz]; v.pzy = p.psiHi[2][0][yz.qz]; }
    if (act && yz.ye) { v.qyx = p.psiE[1][0][yz.qye]; v.qyz = p.psiE[1][1][yz.qye]; }
    if (act && yz.ze) { v.qzx = p.psiE[2][1][yz.qze]; v.qzy = p.psiE[2][0][yz.qze]; }
    if (first && yz.yh) v.pyzl = p.psiHi[1][1][yz.qy - 1];
    if (first && yz.zh) v.pzyl = p.psiHi[2][0][yz.qz - 1];
    if (rd && yz.yd) { v.pyxd = p.psiHi[1][0][yz.qyd]; v.pyzd = p.psiHi[1][1][yz.qyd]; }
    if (rd && yz.zh) v.pzxd = p.psiHi[2][1][yz.qz - sy];
  }
}

// Rows of H_x^{n+1/2} and H_z^{n+1/2} of one plane, shared by the wavefronts
// of a block; two planes deep, so that one barrier per plane suffices (a
// wavefront overwrites a plane's rows only after the barrier of the next
// plane, which every reader of that plane has passed).
template <class T, int TY>
struct HRows {
  T h[2][2][TY][kBX];  // [plane & 1][0: H_x, 1: H_z][row][lane]
};

// What the E update of a metal point reads besides the fields: E^{n-1} (in
// the output buffer, which it overwrites), J^{n-1/2}, the density weight, and
// Q at the cell's node and at the nodes one cell up each axis.
template <class T>
struct MetalIn {
  T em[3] = {T(0), T(0), T(0)}, j[3] = {T(0), T(0), T(0)}, qa[3] = {T(0), T(0), T(0)};
  T q = T(0), r = T(1);
};

// XS: the tile meets an x slab (the other tiles run code free of the CPML
// terms); YZ: it may meet a y or z slab as well (the CPML class); METAL: the
// metal class (no slab), whose E update includes the nonlocal metal points
// (Eqs. NonlocalUpdate / GNORUpdate in the current form, without critical
// points) from node scalars written before the launch (k_nodes)
template <class T, int TY, bool NT, bool XS, bool YZ, bool METAL>
__device__ __forceinline__ void fplain_tile(const Params<T>& p, const Tile tile,
                                            HRows<T, TY>& sh) {
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  // a wavefront is one row (blockDim.x = 64): its row index is uniform, and
  // so are the row's y-slab positions and coefficients (said explicitly in
  // the CPML class: 13 fewer VGPRs there, FP64 1.177 -> 1.162 ms per step on
  // the 320^3 sphere; the plain class measured no gain)
  const int lane = threadIdx.x;
  const int ty = YZ ? __builtin_amdgcn_readfirstlane(threadIdx.y) : (int)threadIdx.y;
  const int i = tile.bx * kBX + lane;
  const int j = tile.by * TY + ty;
  // lanes and rows outside the grid load and store nothing but take part in
  // the shuffles and barriers
  const bool act = i < nx && j < ny;
  const int k0 = tile.bz * p.tl.kz;
  const int k1 = min(nz, k0 + p.tl.kz);
  // 32-bit cell indices (at most 4e9 cells): one offset register serves the
  // loads of all arrays at that cell
  const uint32_t sy = nx, sz = (uint32_t)nx * ny;
  const T* __restrict__ Ex = p.E[0];
  const T* __restrict__ Ey = p.E[1];
  const T* __restrict__ Ez = p.E[2];
  T* __restrict__ Hx = p.H[0];
  T* __restrict__ Hy = p.H[1];
  T* __restrict__ Hz = p.H[2];
  T* __restrict__ Ox = p.O[0];
  T* __restrict__ Oy = p.O[1];
  T* __restrict__ Oz = p.O[2];
  const T S = p.S;
  // neighbours that exist: x+1, y+1 (inside the grid), x-1, y-1
  const bool xp = i <= nx - 2, yp = j <= ny - 2, xm = i >= 1, ym = j >= 1;
  const uint32_t dyp = yp ? sy : 0;
  // the row's first lane recomputes H at column x-1 (the left tile's), its
  // last lane loads E at column x+1; the block's first row recomputes H at
  // row y-1 (the tile below's); every other halo value comes from a
  // neighbouring lane or from the shared rows
  const bool first = act && lane == 0 && xm;
  const bool last = act && lane == kBX - 1 && xp;
  const bool low = ty == 0;  // uniform over the wavefront
  // E update ranges of the column
  const bool ax = act && i <= nx - 2 && j >= 1 && j <= ny - 2;
  const bool ay = act && i >= 1 && i <= nx - 2 && j <= ny - 2;
  const bool az = act && i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2;
  // x slab (tiles that meet one): the H-slab positions of the column and of
  // column x-1, the E-slab position of the column, their coefficients, and
  // slab-array indices (axis-0 slab arrays: ((k ny + j) 2 np + s)).  H points
  // exist up to n - 2 along an axis, and so do their slab positions (-1 on
  // the last node plane, where no H point is updated)
  const int np = p.cp[0].np;
  const int sxh = (XS && act && i <= nx - 2) ? slab_h(i, nx, np) : -1;
  const int sxl = (XS && first) ? slab_h(i - 1, nx, np) : -1;
  const int sxe = (XS && act) ? slab_e(i, nx, np) : -1;
  XCoef<T> ch{T(1), T(0), T(1)}, cl{T(1), T(0), T(1)}, ce{T(1), T(0), T(1)};
  if (XS) {
    const CpmlAxis<T>& X = p.cp[0];
    ch = xcoef(X.bh, X.ah, X.kh, sxh);
    cl = xcoef(X.bh, X.ah, X.kh, sxl);
    ce = xcoef(X.be, X.ae, X.ke, sxe);
  }
  const uint32_t w2 = 2 * np;
  const uint32_t sq = w2;                 // one row in a slab array
  const uint32_t sp = (uint32_t)ny * w2;  // one plane
  const uint32_t jr = act ? (uint32_t)j : 0;
  uint32_t qs = ((uint32_t)k0 * ny + jr) * w2 + (uint32_t)max(sxh, 0);
  uint32_t qsl = ((uint32_t)k0 * ny + jr) * w2 + (uint32_t)max(sxl, 0);
  uint32_t qse = ((uint32_t)k0 * ny + jr) * w2 + (uint32_t)max(sxe, 0);
  // y slab (uniform over the row): H- and E-slab positions of the row and the
  // H-slab position of row y-1, with their coefficients
  const int syh = (YZ && j <= ny - 2) ? slab_h(j, ny, np) : -1;
  const int sye = (YZ && j < ny) ? slab_e(j, ny, np) : -1;
  const int syd = (YZ && low && ym && j < ny) ? slab_h(j - 1, ny, np) : -1;
  XCoef<T> cyh{T(1), T(0), T(1)}, cye{T(1), T(0), T(1)}, cyd{T(1), T(0), T(1)};
  if (YZ) {
    const CpmlAxis<T>& Y = p.cp[1];
    cyh = xcoef(Y.bh, Y.ah, Y.kh, syh);
    cye = xcoef(Y.be, Y.ae, Y.ke, sye);
    cyd = xcoef(Y.bh, Y.ah, Y.kh, syd);
  }
  const CpmlAxis<T>& Z = p.cp[2];
  const uint32_t ic = act ? (uint32_t)i : 0;
  // metal: the column's place in the metal sub-grid; the metal bits of a
  // plane are loaded a plane ahead, so that the plane's metal loads go out
  // with its other loads
  const int lxm = i - p.mlo[0], lym = j - p.mlo[1];
  const bool col_sub = METAL && act && lxm >= 0 && lym >= 0 && lxm < p.mn[0] && lym < p.mn[1];
  const uint32_t m1 = METAL ? (uint32_t)p.mn[0] : 0u, m2 = METAL ? m1 * (uint32_t)p.mn[1] : 0u;
  const uint32_t lcol = col_sub ? (uint32_t)lym * m1 + (uint32_t)lxm : 0u;
  uint32_t mbn = 0u;
  if (METAL && col_sub && k0 - p.mlo[2] >= 0 && k0 - p.mlo[2] < p.mn[2])
    mbn = p.mask[(uint32_t)(k0 - p.mlo[2]) * m2 + lcol];

  uint32_t id = act ? (uint32_t)k0 * sz + (uint32_t)j * nx + i : 0;
  // carried: E_x, E_y of plane k at the column, E_x of column x-1 (first
  // lane) and E_y of row y-1 (first row); H_x, H_y^{n+1/2} of plane k-1
  T ex0 = act ? Ex[id] : T(0), ey0 = act ? Ey[id] : T(0);
  T exl0 = first ? Ex[id - 1] : T(0);
  T eyd0 = (low && act && ym) ? Ey[id - sy] : T(0);
  T hxm = T(0), hym = T(0);
  if (act && k0 >= 1) {
    // H_x, H_y^{n+1/2} of plane k0-1 (recomputed; stored by the tile below)
    const uint32_t q = id - sz;
    const T exq = Ex[q], eyq = Ey[q], ezq = Ez[q];
    const T ezy = Ez[q + dyp], ezx = Ez[q + (xp ? 1 : 0)];
    const T hx_ = p.Hi[0][q], hy_ = p.Hi[1][q];
    const T psy = XS ? p.psiHi[0][1][qs - sp] : T(0);
    T dxy = ezx - ezq, psn;
    if (XS && sxh >= 0) dxy = xstretch(ch, dxy, psy, psn);
    T dyx = ezy - ezq, dzx = ey0 - eyq, dzy = ex0 - exq;
    if (YZ) {
      if (syh >= 0) {
        const uint32_t qy = ((uint32_t)(k0 - 1) * w2 + (uint32_t)syh) * sy + ic;
        dyx = xstretch(cyh, dyx, p.psiHi[1][0][qy], psn);
      }
      const int szm = slab_h(k0 - 1, nz, np);
      if (szm >= 0) {
        const XCoef<T> czm = xcoef(Z.bh, Z.ah, Z.kh, szm);
        const uint32_t qz = ((uint32_t)szm * ny + jr) * sy + ic;
        dzx = xstretch(czm, dzx, p.psiHi[2][1][qz], psn);
        dzy = xstretch(czm, dzy, p.psiHi[2][0][qz], psn);
      }
    }
    hxm = upd_hx(i, j, k0 - 1, nx, ny, nz) ? hx_ - S * (dyx - dzx) : hx_;
    hym = upd_hy(i, j, k0 - 1, nx, ny, nz) ? hy_ - S * (dzy - dxy) : hy_;
  }
  const bool rd = low && act && ym;  // the first row loads row y-1
  for (int k = k0; k < k1; ++k, id += sz, qs += sp, qsl += sp, qse += sp) {
    const bool zp = k <= nz - 2;
    // ---- the plane's loads, issued together (one memory round trip per
    // plane; issuing them a plane ahead measured no faster)
    YZAt yz;
    XCoef<T> czh{T(1), T(0), T(1)}, cze{T(1), T(0), T(1)};
    if (YZ) {
      const int szh = k <= nz - 2 ? slab_h(k, nz, np) : -1, sze = slab_e(k, nz, np);
      yz.yh = syh >= 0; yz.ye = sye >= 0; yz.yd = syd >= 0;
      yz.zh = szh >= 0; yz.ze = sze >= 0;
      const uint32_t kr = (uint32_t)k * w2;
      yz.qy = (kr + (uint32_t)max(syh, 0)) * sy + ic;
      yz.qye = (kr + (uint32_t)max(sye, 0)) * sy + ic;
      yz.qyd = (kr + (uint32_t)max(syd, 0)) * sy + ic;
      yz.qz = ((uint32_t)max(szh, 0) * ny + jr) * sy + ic;
      yz.qze = ((uint32_t)max(sze, 0) * ny + jr) * sy + ic;
      czh = xcoef(Z.bh, Z.ah, Z.kh, szh);
      cze = xcoef(Z.be, Z.ae, Z.ke, sze);
    }
    PlaneIn<T> cur;
    load_plane<T, XS, YZ>(p, cur, id, zp ? sz : 0, dyp, sy, qs, qsl, qse, sq, yz, act, first, last, rd);
    MetalIn<T> mt;
    uint32_t mb = 0u, l = 0u;
    bool zsub = false;
    if (METAL) {
      const int lz = k - p.mlo[2];
      zsub = lz >= 0 && lz < p.mn[2];  // uniform over the block
      l = (col_sub && zsub) ? (uint32_t)lz * m2 + lcol : 0u;
      mb = mbn;
      mbn = (col_sub && lz + 1 >= 0 && lz + 1 < p.mn[2]) ? p.mask[(uint32_t)(lz + 1) * m2 + lcol] : 0u;
      // metal points lie two cells inside the sub-grid: the upper nodes exist
      if (mb & 1u) { mt.em[0] = Ox[id]; mt.j[0] = p.Ji[0][l]; mt.qa[0] = p.Q[l + 1]; }
      if (mb & 2u) { mt.em[1] = Oy[id]; mt.j[1] = p.Ji[1][l]; mt.qa[1] = p.Q[l + m1]; }
      if (mb & 4u) { mt.em[2] = Oz[id]; mt.j[2] = p.Ji[2][l]; mt.qa[2] = p.Q[l + m2]; }
      if (mb) {
        mt.q = p.Q[l];
        if (p.rho) mt.r = (T)p.rho[l];
      }
    }
    load_fence();
    const T ez = cur.ez, ex1 = cur.ex1, ey1 = cur.ey1, ezy = cur.ezy, exy = cur.exy;
    const T hx = cur.hx, hy = cur.hy, hz = cur.hz, sy_ = cur.sy_, sz_ = cur.sz_;
    const T ezr = cur.ezr, eyr = cur.eyr;
    const T ezl = cur.ezl, eyl = cur.eyl, exl1 = cur.exl1, exly = cur.exly, hyo = cur.hyo, hzo = cur.hzo;
    const T syl = cur.syl, szl = cur.szl;
    const T eyd1 = cur.eyd1, ezd = cur.ezd, exd = cur.exd, hxo = cur.hxo, hzd_o = cur.hzd_o;
    const T szd = cur.szd, eydr = cur.eydr;
    // E_z, E_y of plane k at column x+1: the right lane's (the last lane
    // takes the next tile's; a column without x+1 uses its own, as an H
    // point there is not updated)
    T ezx = from_right(ez), eyx = from_right(ey0);
    if (last) { ezx = ezr; eyx = eyr; }
    if (!xp) { ezx = ez; eyx = ey0; }
    // ---- H^{n+1/2} of the cell
    T dxy = ezx - ez, dxz = eyx - ey0;  // x differences of H_y, H_z
    T psy = T(0), psz = T(0);
    if (XS && sxh >= 0) {
      dxy = xstretch(ch, dxy, sy_, psy);
      dxz = xstretch(ch, dxz, sz_, psz);
    }
    const bool uhx = act && upd_hx(i, j, k, nx, ny, nz), uhy = act && upd_hy(i, j, k, nx, ny, nz);
    const bool uhz = act && upd_hz(i, j, k, nx, ny, nz);
    T dyx = ezy - ez, dzx = ey1 - ey0, dzy = ex1 - ex0, dyz = exy - ex0;
    if (YZ) {
      T ps;
      if (yz.yh) {
        dyx = xstretch(cyh, dyx, cur.pyx, ps);
        if (uhx) p.psiH[1][0][yz.qy] = ps;
        dyz = xstretch(cyh, dyz, cur.pyz, ps);
        if (uhz) p.psiH[1][1][yz.qy] = ps;
      }
      if (yz.zh) {
        dzx = xstretch(czh, dzx, cur.pzx, ps);
        if (uhx) p.psiH[2][1][yz.qz] = ps;
        dzy = xstretch(czh, dzy, cur.pzy, ps);
        if (uhy) p.psiH[2][0][yz.qz] = ps;
      }
    }
    const T hxn = uhx ? hx - S * (dyx - dzx) : hx;
    const T hyn = uhy ? hy - S * (dzy - dxy) : hy;
    const T hzn = uhz ? hz - S * (dxz - dyz) : hz;
    if (uhx) put<NT>(&Hx[id], hxn);
    if (uhy) put<NT>(&Hy[id], hyn);
    if (uhz) put<NT>(&Hz[id], hzn);
    if (XS && sxh >= 0) {
      if (uhy) p.psiH[0][1][qs] = psy;
      if (uhz) p.psiH[0][0][qs] = psz;
    }
    const int b = k & 1;
    sh.h[b][0][ty][lane] = hxn;
    sh.h[b][1][ty][lane] = hzn;
    // ---- halo H^{n+1/2} of column x-1 (H_y, H_z): the left lane's; the
    // first lane recomputes the left tile's from E^n and H^{n-1/2}
    T hyl = from_left(hyn), hzl = from_left(hzn);
    if (first) {
      T dy_ = ez - ezl, dz_ = ey0 - eyl, ps;
      if (XS && sxl >= 0) {
        dy_ = xstretch(cl, dy_, syl, ps);
        dz_ = xstretch(cl, dz_, szl, ps);
      }
      T dzyl = exl1 - exl0, dyzl = exly - exl0;
      if (YZ && yz.zh) dzyl = xstretch(czh, dzyl, cur.pzyl, ps);
      if (YZ && yz.yh) dyzl = xstretch(cyh, dyzl, cur.pyzl, ps);
      hyl = upd_hy(i - 1, j, k, nx, ny, nz) ? hyo - S * (dzyl - dy_) : hyo;
      hzl = upd_hz(i - 1, j, k, nx, ny, nz) ? hzo - S * (dz_ - dyzl) : hzo;
      exl0 = exl1;
    }
    // ---- halo H^{n+1/2} of row y-1 (H_x, H_z): the shared row below; the
    // first row recomputes the tile below's
    T hxd = T(0), hzd = T(0);
    if (low) {
      T eydx = from_right(eyd0);  // E_y(i+1, j-1, k)
      if (last) eydx = eydr;
      if (!xp) eydx = eyd0;
      if (rd) {
        T d = eydx - eyd0, ps;
        if (XS && sxh >= 0) d = xstretch(ch, d, szd, ps);
        T dyxd = ez - ezd, dzxd = eyd1 - eyd0, dyzd = ex0 - exd;
        if (YZ && yz.yd) {
          dyxd = xstretch(cyd, dyxd, cur.pyxd, ps);
          dyzd = xstretch(cyd, dyzd, cur.pyzd, ps);
        }
        if (YZ && yz.zh) dzxd = xstretch(czh, dzxd, cur.pzxd, ps);
        hxd = upd_hx(i, j - 1, k, nx, ny, nz) ? hxo - S * (dyxd - dzxd) : hxo;
        hzd = upd_hz(i, j - 1, k, nx, ny, nz) ? hzd_o - S * (d - dyzd) : hzd_o;
      }
      eyd0 = eyd1;
    }
    __syncthreads();
    if (!low && ym) {
      hxd = sh.h[b][0][ty - 1][lane];
      hzd = sh.h[b][1][ty - 1][lane];
    }
    // ---- E^{n+1}
    const bool kin = k >= 1 && k <= nz - 2;
    const bool uex = ax && kin, uey = ay && kin, uez = az && zp;
    T d_xy = hzn - hzl, d_xz = hyn - hyl;  // x differences of E_y, E_z
    if (XS && sxe >= 0) {
      T ps;
      if (uey) {
        d_xy = xstretch(ce, d_xy, cur.ey_, ps);
        p.psiE[0][1][qse] = ps;
      }
      if (uez) {
        d_xz = xstretch(ce, d_xz, cur.ez_, ps);
        p.psiE[0][0][qse] = ps;
      }
    }
    T d_yx = hzn - hzd, d_zx = hyn - hym, d_zy = hxn - hxm, d_yz = hxn - hxd;
    if (YZ) {
      T ps;
      if (yz.ye) {
        if (uex) {
          d_yx = xstretch(cye, d_yx, cur.qyx, ps);
          p.psiE[1][0][yz.qye] = ps;
        }
        if (uez) {
          d_yz = xstretch(cye, d_yz, cur.qyz, ps);
          p.psiE[1][1][yz.qye] = ps;
        }
      }
      if (yz.ze) {
        if (uex) {
          d_zx = xstretch(cze, d_zx, cur.qzx, ps);
          p.psiE[2][1][yz.qze] = ps;
        }
        if (uey) {
          d_zy = xstretch(cze, d_zy, cur.qzy, ps);
          p.psiE[2][0][yz.qze] = ps;
        }
      }
    }
    T cxv = d_yx - d_zx;  // dy H_z - dz H_y
    T cyv = d_zy - d_xy;  // dz H_x - dx H_z
    T czv = d_xz - d_yz;  // dx H_y - dy H_x
    const T sexy = k < p.sub_k ? p.SE : (k == p.sub_k ? p.se_avg : p.se_sub);
    const T sez = k < p.sub_k ? p.SE : p.se_sub;
    T enx = ex0 + sexy * cxv, eny = ey0 + sexy * cyv, enz = ez + sez * czv;
    if (METAL) {
      // metal points: E^{n+1} and J^{n+1/2} together (the same update as
      // the two-sweep E/J kernel's), and the wavefront's share of the plane
      // sum of J_x for the extinction transform
      double jsum = 0.0;
      if (mb) {
        // total-field operation: a metal point in an absorbing layer (here
        // the x slab) follows the local Drude model (no nonlocal force)
        const bool local = XS && p.lra_pml && sxe >= 0;
        T cS = p.cS, c3 = p.c3, c1 = p.c1, cJ = p.cJ, cG = p.cG, d3 = p.d3, r = T(1);
        if (p.rho) {
          r = mt.r;
          d3 = r * p.d3;
          // the two-sweep kernel's divisor without critical points (its
          // pole term a literal zero), so that the forms round alike
          const T inv = T(1) / (p.eps_inf + d3 + T(0));
          cS = p.S * inv; c3 = T(3) * d3 * inv; c1 = d3 * inv; cJ = p.D2 * inv; cG = inv;
        }
        const T ag = p.agam;
        if (mb & 1u) {
          const T G = local ? T(0) : r * (mt.qa[0] - mt.q);
          const T en = ex0 + (cS * cxv - c3 * ex0 - c1 * mt.em[0] + cJ * mt.j[0] - cG * G);
          const T jn = mt.j[0] + (d3 * (mt.em[0] + T(2) * ex0 + en) - ag * mt.j[0] + G);
          p.Jo[0][l] = jn;
          jsum = (double)jn + (double)p.ebd * ((double)en - (double)ex0);
          enx = en;
        }
        if (mb & 2u) {
          const T G = local ? T(0) : r * (mt.qa[1] - mt.q);
          const T en = ey0 + (cS * cyv - c3 * ey0 - c1 * mt.em[1] + cJ * mt.j[1] - cG * G);
          p.Jo[1][l] = mt.j[1] + (d3 * (mt.em[1] + T(2) * ey0 + en) - ag * mt.j[1] + G);
          eny = en;
        }
        if (mb & 4u) {
          const T G = local ? T(0) : r * (mt.qa[2] - mt.q);
          const T en = ez + (cS * czv - c3 * ez - c1 * mt.em[2] + cJ * mt.j[2] - cG * G);
          p.Jo[2][l] = mt.j[2] + (d3 * (mt.em[2] + T(2) * ez + en) - ag * mt.j[2] + G);
          enz = en;
        }
      }
      if (zsub && __any(mb != 0u)) {
        const double s = wave_sum(jsum);
        if (lane == 0) {
          const int nbxy = p.tl.nbx * p.tl.nby * TY;
          p.jpart[(size_t)k * nbxy + (tile.by * p.tl.nbx + tile.bx) * TY + ty] = s;
        }
      }
    }
    if (uex) put<NT>(&Ox[id], enx);
    if (uey) put<NT>(&Oy[id], eny);
    if (uez) put<NT>(&Oz[id], enz);
    // ---- carry up the column
    ex0 = ex1;
    ey0 = ey1;
    hxm = hxn;
    hym = hyn;
  }
}

// Class 0 of the two-sweep tiling (plain tiles, and tiles that meet only an
// x slab), one launch over the class list in its tile order.  A block whose
// tile meets an x slab (the test the tile classes use) takes the x-slab code.
// One launch keeps the tiles of a row of the grid in flight together: the
// row's bytes are fetched by neighbouring blocks at about the same time, and
// a tile's x halo is its neighbour's, still in the L2.  Split into a launch
// for the tiles without an x slab (8 waves per SIMD) and one for the x-slab
// tiles, the same work took 9 % longer.
template <class T, int TY, bool NT>
__global__ void __launch_bounds__(kBX* TY) k_fplain(Params<T> p) {
  __shared__ HRows<T, TY> sh;
  const Tile tile = decode_tile(p.tl, p.tiles, 0, blockIdx.x);
  if (!tile.ok) return;  // uniform over the block
  const int np = p.cp[0].np, x0 = tile.bx * kBX;
  if (np > 0 && (x0 - 1 < np || x0 + kBX + 1 > p.nx - 1 - np)) fplain_tile<T, TY, NT, true, false, false>(p, tile, sh);
  else fplain_tile<T, TY, NT, false, false, false>(p, tile, sh);
}

// Class 1 (tiles without metal that meet a y or z slab, and maybe an x slab)
// in one pass: a kernel of its own, whose larger register budget the plain
// tiles do not share.
template <class T, int TY, bool NT>
__global__ void __launch_bounds__(kBX* TY) k_fplain_pml(Params<T> p) {
  __shared__ HRows<T, TY> sh;
  const Tile tile = decode_tile(p.tl, p.tiles, 1, blockIdx.x);
  if (!tile.ok) return;
  fplain_tile<T, TY, NT, true, true, false>(p, tile, sh);
}

// Class 2 (metal tiles that meet no slab but maybe an x slab) in one pass,
// without critical points; its node scalars come from k_nodes, launched
// before it.  Held to 6 wavefronts per SIMD in FP32 (80 VGPRs and a 12-byte
// spill, against 82 and 5 wavefronts unbounded; 0.6 % faster per step on
// the 320^3 sphere) and to 4 in FP64 (128 VGPRs and a 36-byte spill,
// against 136 and 3: the class 349.6 -> 333.4 us there).
template <class T, int TY, bool NT>
__global__ void __launch_bounds__(kBX* TY, sizeof(T) == 4 ? 6 : 4) k_fplain_metal(Params<T> p) {
  __shared__ HRows<T, TY> sh;
  const Tile tile = decode_tile(p.tl, p.tiles, 2, blockIdx.x);
  if (!tile.ok) return;
  const int np = p.cp[0].np, x0 = tile.bx * kBX;
  if (np > 0 && (x0 - 1 < np || x0 + kBX + 1 > p.nx - 1 - np)) fplain_tile<T, TY, NT, true, false, true>(p, tile, sh);
  else fplain_tile<T, TY, NT, false, false, true>(p, tile, sh);
}

// Node scalars of every node of the metal sub-grid that lies on a metal edge
// (its column's planes zlo .. zhi; the other nodes keep zero), from
// J^{n-1/2} and the previous node scalars, the step's inputs.  One thread per
// sub-grid node, x fastest.  (One thread per column and run of 8 planes,
// marching them, took 42 us per step on the 320^3 sphere: too few loads in
// flight.)
template <class T>
__device__ __forceinline__ void nodes_at(const Params<T>& p, long t) {
  const int m0 = p.mn[0];
  const long C = (long)m0 * p.mn[1];
  if (t >= C * p.mn[2]) return;
  const int col = (int)(t % C), lz = (int)(t / C);
  if (lz < p.colz[2 * col] || lz > p.colz[2 * col + 1]) return;
  const int lx = col % m0, ly = col / m0;
  const size_t l = (size_t)t, m1 = (size_t)m0, m2 = (size_t)C;
  const T jx = p.Ji[0][l], jy = p.Ji[1][l], jz = p.Ji[2][l];
  const T jxm = lx > 0 ? p.Ji[0][l - 1] : T(0);
  const T jym = ly > 0 ? p.Ji[1][l - m1] : T(0);
  const T jzm = lz > 0 ? p.Ji[2][l - m2] : T(0);
  store_node_scalars(p, l, jx, jxm, jy, jym, jz, jzm, p.PPi[l], p.PJi[l]);
}
template <class T>
__global__ void __launch_bounds__(256) k_nodes(Params<T> p) {
  nodes_at(p, (long)blockIdx.x * 256 + threadIdx.x);
}

template <class T, bool NT>
void launch_fplain_nt(const Params<T>& p, int cls, hipStream_t s) {
  const int blocks = class_blocks(p.tl, cls);
  if (cls == 0) {
    if (p.tl.ty == 4) hipLaunchKernelGGL((k_fplain<T, 4, NT>), dim3(blocks), dim3(kBX, 4), 0, s, p);
    else if (p.tl.ty == 8) hipLaunchKernelGGL((k_fplain<T, 8, NT>), dim3(blocks), dim3(kBX, 8), 0, s, p);
    else hipLaunchKernelGGL((k_fplain<T, 2, NT>), dim3(blocks), dim3(kBX, 2), 0, s, p);
  } else if (cls == 1) {
    if (p.tl.ty == 4) hipLaunchKernelGGL((k_fplain_pml<T, 4, NT>), dim3(blocks), dim3(kBX, 4), 0, s, p);
    else if (p.tl.ty == 8) hipLaunchKernelGGL((k_fplain_pml<T, 8, NT>), dim3(blocks), dim3(kBX, 8), 0, s, p);
    else hipLaunchKernelGGL((k_fplain_pml<T, 2, NT>), dim3(blocks), dim3(kBX, 2), 0, s, p);
  } else {
    if (p.tl.ty == 4) hipLaunchKernelGGL((k_fplain_metal<T, 4, NT>), dim3(blocks), dim3(kBX, 4), 0, s, p);
    else if (p.tl.ty == 8) hipLaunchKernelGGL((k_fplain_metal<T, 8, NT>), dim3(blocks), dim3(kBX, 8), 0, s, p);
    else hipLaunchKernelGGL((k_fplain_metal<T, 2, NT>), dim3(blocks), dim3(kBX, 2), 0, s, p);
  }
}

// ------------------------------------------------------- TF/SF corrections
// H_inc^{n+1/2} at line cell q from E_inc^n and the line's H^{n-1/2} (the
// line's own H update; the line advances after the correction)
__device__ __forceinline__ double line_h_next(const AuxParams& a, int q) {
  const double d = a.e1[q + 1] - a.e1[q];
  const double ps = a.bh[q] * a.ph[q] + a.ah[q] * d;
  return a.h1[q] - a.S * (a.kh[q] * d + ps);
}
// The TF/SF terms of H^{n+1/2} at an H_y and an H_z point (zero off the
// faces): -S times the E_inc^n terms the two-sweep H update adds to its curl
template <class T>
__device__ __forceinline__ T tf_dhy(const Params<T>& p, int i, int j, int k) {
  if (i < p.tf_lo[0] || i > p.tf_hi[0] - 1 || j < p.tf_lo[1] || j > p.tf_hi[1]) return T(0);
  if (k == p.tf_lo[2] - 1) return p.S * (T)p.e1[p.tf_lo[2] + kAuxOff];
  if (k == p.tf_hi[2]) return -(p.S * (T)p.e1[p.tf_hi[2] + kAuxOff]);
  return T(0);
}
template <class T>
__device__ __forceinline__ T tf_dhz(const Params<T>& p, int i, int j, int k) {
  if (i < p.tf_lo[0] || i > p.tf_hi[0] - 1 || k < p.tf_lo[2] || k > p.tf_hi[2]) return T(0);
  if (j == p.tf_lo[1] - 1) return -(p.S * (T)p.e1[k + kAuxOff]);
  if (j == p.tf_hi[1]) return p.S * (T)p.e1[k + kAuxOff];
  return T(0);
}

// One thread per point of the shell of the TF box: the box widened by one
// cell, [lo - 1, hi + 1], without its inside [lo + 1, hi - 1], each point
// once: the planes k in {lo-1, lo, hi, hi+1} (whole widened rows), then the
// rows j in {lo-1, lo, hi, hi+1} of the planes lo+1 .. hi-1, then the
// columns i in {lo-1, lo, hi, hi+1} of rows lo+1 .. hi-1 of those planes.
// Every TF/SF term, and every E point whose curl holds one, lies in it.
// Only points of tiles of class cls are touched (a point of a two-sweep tile
// is left alone: those sweeps apply the terms themselves; one of the other
// one-pass class, to that class's own launch); there the terms go to H^{n+1/2} and
// the E update's share of the H terms of its curl (the one-pass kernels took
// every H of that curl without them) plus its own H_inc terms to E^{n+1}.
// Point t of the shell, at tiles of classes c0 .. c1.
template <class T>
__device__ __forceinline__ void tfsf_fix_point(const Params<T>& p, const AuxParams& a, int t, int c0,
                                               int c1) {
  const int* lo = p.tf_lo;
  const int* hi = p.tf_hi;
  const int Lx = hi[0] - lo[0] + 3, Ly = hi[1] - lo[1] + 3, Lz = hi[2] - lo[2] + 3;
  const int nZ = 4 * Lx * Ly, nY = 4 * (Lz - 4) * Lx, nX = 4 * (Ly - 4) * (Lz - 4);
  int i, j, k;
  if (t < nZ) {
    const int q = t / (Lx * Ly);
    i = lo[0] - 1 + t % Lx;
    j = lo[1] - 1 + (t / Lx) % Ly;
    k = q < 2 ? lo[2] - 1 + q : hi[2] + (q - 2);
  } else if ((t -= nZ) < nY) {
    const int q = t / (Lx * (Lz - 4));
    i = lo[0] - 1 + t % Lx;
    k = lo[2] + 1 + (t / Lx) % (Lz - 4);
    j = q < 2 ? lo[1] - 1 + q : hi[1] + (q - 2);
  } else if ((t -= nY) < nX) {
    const int q = t / ((Ly - 4) * (Lz - 4));
    j = lo[1] + 1 + t % (Ly - 4);
    k = lo[2] + 1 + (t / (Ly - 4)) % (Lz - 4);
    i = q < 2 ? lo[0] - 1 + q : hi[0] + (q - 2);
  } else {
    return;
  }
  const Tiling& tl = p.tl;
  const int c = p.tile_class[((k / tl.kz) * tl.nby + j / tl.ty) * tl.nbx + i / kBX];
  if (c < c0 || c > c1) return;
  const size_t id = ((size_t)k * p.ny + j) * p.nx + i;
  const T dhy = tf_dhy(p, i, j, k), dhz = tf_dhz(p, i, j, k);
  if (dhy != T(0)) p.H[1][id] += dhy;
  if (dhz != T(0)) p.H[2][id] += dhz;
  const T sexy = k < p.sub_k ? p.SE : (k == p.sub_k ? p.se_avg : p.se_sub);
  const T sez = k < p.sub_k ? p.SE : p.se_sub;
  // E_x: dy H_z - dz H_y, and H_inc on the z faces
  T cx = (dhz - tf_dhz(p, i, j - 1, k)) - (dhy - tf_dhy(p, i, j, k - 1));
  if (i >= lo[0] && i <= hi[0] - 1 && j >= lo[1] && j <= hi[1]) {
    if (k == lo[2]) cx += (T)line_h_next(a, lo[2] - 1 + kAuxOff);
    if (k == hi[2]) cx -= (T)line_h_next(a, hi[2] + kAuxOff);
  }
  if (cx != T(0)) p.O[0][id] += sexy * cx;
  // E_y: dz H_x - dx H_z
  const T cy = tf_dhz(p, i - 1, j, k) - dhz;
  if (cy != T(0)) p.O[1][id] += sexy * cy;
  // E_z: dx H_y - dy H_x, and H_inc on the x faces
  T cz = dhy - tf_dhy(p, i - 1, j, k);
  if ((i == lo[0] || i == hi[0]) && j >= lo[1] && j <= hi[1] && k >= lo[2] && k <= hi[2] - 1) {
    const T inc = (T)line_h_next(a, k + kAuxOff);
    cz += (i == lo[0]) ? -inc : inc;
  }
  if (cz != T(0)) p.O[2][id] += sez * cz;
}

template <class T>
__global__ void __launch_bounds__(256) k_tfsf_fix(Params<T> p, AuxParams a, int cls) {
  tfsf_fix_point(p, a, blockIdx.x * 256 + threadIdx.x, cls, cls);
}

// ------------------------------------------------------------------ batches
// Step form 3 of a batch: the one-pass class CLS of every instance in one
// launch (class 0's last block of an instance, its line's block in the two
// sweeps, stays idle: the lines take a launch of their own, k_aux_batch).
template <class T, int TY, bool NT, int CLS>
__global__ void __launch_bounds__(kBX* TY) k_fplain_batch(const BatchEntry<T>* __restrict__ e, int n) {
  __shared__ HRows<T, TY> sh;
  const BatchEntry<T>& en = entry_at(e, find_instance(e, n, blockIdx.x, CLS));
  const int b = blockIdx.x - en.blk0[CLS];
  if (b >= en.nblk[CLS] || (CLS == 0 && b == en.nblk[0] - 1) || (CLS == 2 && en.two_sweep2)) return;
  const Params<T>& p = en.p;
  const Tile tile = decode_tile(p.tl, p.tiles, CLS, b);
  if (!tile.ok) return;
  if (CLS == 1) {
    fplain_tile<T, TY, NT, true, true, false>(p, tile, sh);
  } else if (CLS == 2) {
    const int np = p.cp[0].np, x0 = tile.bx * kBX;
    if (np > 0 && (x0 - 1 < np || x0 + kBX + 1 > p.nx - 1 - np)) fplain_tile<T, TY, NT, true, false, true>(p, tile, sh);
    else fplain_tile<T, TY, NT, false, false, true>(p, tile, sh);
  } else {
    const int np = p.cp[0].np, x0 = tile.bx * kBX;
    if (np > 0 && (x0 - 1 < np || x0 + kBX + 1 > p.nx - 1 - np)) fplain_tile<T, TY, NT, true, false, false>(p, tile, sh);
    else fplain_tile<T, TY, NT, false, false, false>(p, tile, sh);
  }
}

// The TF/SF corrections of every instance at the points of its one-pass
// tiles (classes 0 and 1, and 2 unless its metal tiles take the two sweeps),
// after those classes' launches.
template <class T>
__global__ void __launch_bounds__(256) k_tfsf_fix_batch(const BatchEntry<T>* __restrict__ e, int n) {
  const BatchEntry<T>& en = entry_at(e, find_instance(e, n, blockIdx.x, -2));
  const int b = blockIdx.x - en.fblk0;
  if (b >= en.fnblk) return;
  tfsf_fix_point(en.p, en.a, b * 256 + threadIdx.x, 0, en.two_sweep2 ? 1 : 2);
}

// The node scalars of every instance (before the metal class's one-pass
// launch), block range sblk0 .. sblk0 + snblk of each instance.
template <class T>
__global__ void __launch_bounds__(256) k_nodes_batch(const BatchEntry<T>* __restrict__ e, int n) {
  const BatchEntry<T>& en = entry_at(e, find_instance(e, n, blockIdx.x, -3));
  const int b = blockIdx.x - en.sblk0;
  if (b >= en.snblk) return;
  nodes_at(en.p, (long)b * 256 + threadIdx.x);
}

// The lines' whole step, one block per instance (as k_aux for one simulation).
template <class T>
__global__ void __launch_bounds__(kAuxThreads) k_aux_batch(const BatchEntry<T>* __restrict__ e, int sub) {
  const AuxParams& a = entry_at(e, blockIdx.x).a;
  aux_h_block(a, threadIdx.x, kAuxThreads);
  __syncthreads();
  aux_e_block(a, sub, threadIdx.x, kAuxThreads);
}

template <class T, int CLS, bool NT>
void launch_fplain_batch_cls(const BatchEntry<T>* e, int n, int blocks, int ty, hipStream_t s) {
  if (ty == 4) hipLaunchKernelGGL((k_fplain_batch<T, 4, NT, CLS>), dim3(blocks), dim3(kBX, 4), 0, s, e, n);
  else if (ty == 8) hipLaunchKernelGGL((k_fplain_batch<T, 8, NT, CLS>), dim3(blocks), dim3(kBX, 8), 0, s, e, n);
  else hipLaunchKernelGGL((k_fplain_batch<T, 2, NT, CLS>), dim3(blocks), dim3(kBX, 2), 0, s, e, n);
}

}  // namespace

template <class T>
void launch_fplain(const Params<T>& p, const AuxParams& a, int cls, bool fix, hipStream_t s) {
  if (p.tl.cn[cls] == 0) return;
  if (cls == 2 && p.any_metal) {
    const int nb = node_blocks(p.mn);
    if (nb > 0) hipLaunchKernelGGL(k_nodes<T>, dim3(nb), dim3(256), 0, s, p);
  }
  if (p.stream_stores) launch_fplain_nt<T, true>(p, cls, s);
  else launch_fplain_nt<T, false>(p, cls, s);
  if (p.tfsf && fix)
    hipLaunchKernelGGL(k_tfsf_fix<T>, dim3(tfsf_fix_blocks(p.tf_lo, p.tf_hi)), dim3(256), 0, s, p, a, cls);
}
template void launch_fplain<float>(const Params<float>&, const AuxParams&, int, bool, hipStream_t);
template void launch_fplain<double>(const Params<double>&, const AuxParams&, int, bool, hipStream_t);

int node_blocks(const int mn[3]) {
  const long t = (long)mn[0] * mn[1] * mn[2];
  return (int)((t + 255) / 256);
}

int tfsf_fix_blocks(const int lo[3], const int hi[3]) {
  const long Lx = hi[0] - lo[0] + 3, Ly = hi[1] - lo[1] + 3, Lz = hi[2] - lo[2] + 3;
  const long n = 4 * Lx * Ly + 4 * (Lz - 4) * Lx + 4 * (Ly - 4) * (Lz - 4);
  return (int)((n + 255) / 256);
}

template <class T>
void launch_fplain_batch(const BatchEntry<T>* e, int n, int blocks, int ty, int cls, bool nt,
                         hipStream_t s) {
  if (blocks == 0) return;
  if (cls == 0) nt ? launch_fplain_batch_cls<T, 0, true>(e, n, blocks, ty, s)
                   : launch_fplain_batch_cls<T, 0, false>(e, n, blocks, ty, s);
  else if (cls == 1) nt ? launch_fplain_batch_cls<T, 1, true>(e, n, blocks, ty, s)
                        : launch_fplain_batch_cls<T, 1, false>(e, n, blocks, ty, s);
  else nt ? launch_fplain_batch_cls<T, 2, true>(e, n, blocks, ty, s)
          : launch_fplain_batch_cls<T, 2, false>(e, n, blocks, ty, s);
}
template <class T>
void launch_nodes_batch(const BatchEntry<T>* e, int n, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_nodes_batch<T>, dim3(blocks), dim3(256), 0, s, e, n);
}
template void launch_nodes_batch<float>(const BatchEntry<float>*, int, int, hipStream_t);
template void launch_nodes_batch<double>(const BatchEntry<double>*, int, int, hipStream_t);
template <class T>
void launch_tfsf_fix_batch(const BatchEntry<T>* e, int n, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_tfsf_fix_batch<T>, dim3(blocks), dim3(256), 0, s, e, n);
}
template <class T>
void launch_aux_batch(const BatchEntry<T>* e, int n, int sub, hipStream_t s) {
  hipLaunchKernelGGL(k_aux_batch<T>, dim3(n), dim3(kAuxThreads), 0, s, e, sub);
}
template void launch_fplain_batch<float>(const BatchEntry<float>*, int, int, int, int, bool, hipStream_t);
template void launch_fplain_batch<double>(const BatchEntry<double>*, int, int, int, int, bool, hipStream_t);
template void launch_tfsf_fix_batch<float>(const BatchEntry<float>*, int, int, hipStream_t);
template void launch_tfsf_fix_batch<double>(const BatchEntry<double>*, int, int, hipStream_t);
template void launch_aux_batch<float>(const BatchEntry<float>*, int, int, hipStream_t);
template void launch_aux_batch<double>(const BatchEntry<double>*, int, int, hipStream_t);

}  // namespace gnor

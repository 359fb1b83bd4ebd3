// One-pass step of the plain tiles (gfx950): f1 and f2 of Sec. III fused for
// tiles that meet neither metal nor a CPML slab.  The two-sweep form reads
// E^n twice and writes, then re-reads, H^{n+1/2}: 18 field words per cell.
// Here a tile computes H^{n+1/2} and, at once, E^{n+1} from it: 12 words
// (read E^n and H^{n-1/2}, write H^{n+1/2} and E^{n+1}).
//
// Each wavefront owns one row (64 cells along x) of the tile and marches it
// up the tile's planes, independent of every other wavefront: no LDS, no
// barrier.  The E update at (i, j, k) needs H^{n+1/2} at (i-1, j, k),
// (i, j-1, k) and (i, j, k-1).  The plane below is carried in registers; the
// row below (H_x, H_z) and the column to the left (H_y, H_z) are recomputed
// from E^n and H^{n-1/2}, whose values the neighbouring wavefronts load too
// (cache hits).  Only a cell's own H is stored, so no wavefront sees another
// one's new values, and H is read from the step's input buffer and written
// to its output buffer.
//
// TF/SF corrections: the H update takes E_inc^n from the auxiliary line; the
// E update takes H_inc^{n+1/2}, evaluated from the line's state with the
// line's own update (the line itself advances after this launch).  The
// background coefficients follow the planes (a substrate beyond sub_k).
#include "gnor_device.h"

namespace gnor {

namespace {

template <bool NT, class T>
__device__ __forceinline__ void put(T* a, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, a);
  else *a = v;
}

// H_inc^{n+1/2} at line cell q from E_inc^n, H_inc^{n-1/2} (the line's H update)
__device__ __forceinline__ double fp_h_inc(const AuxParams& a, int q) {
  const double d = a.e1[q + 1] - a.e1[q];
  const double ps = a.bh[q] * a.ph[q] + a.ah[q] * d;
  return a.h1[q] - a.S * (a.kh[q] * d + ps);
}

// TF/SF terms of the H update at (i, j, k) (index units, before the factor
// -S): the H_y term of the plane faces and the H_z term of the y faces.
template <class T>
__device__ __forceinline__ void tf_h(const Params<T>& p, int i, int j, int k, T& ty_, T& tz_) {
  ty_ = tz_ = T(0);
  if (!p.tfsf || i < p.tf_lo[0] || i > p.tf_hi[0] - 1) return;
  if (j >= p.tf_lo[1] && j <= p.tf_hi[1]) {
    if (k == p.tf_lo[2] - 1) ty_ = -(T)p.e1[p.tf_lo[2] + kAuxOff];
    if (k == p.tf_hi[2]) ty_ = (T)p.e1[p.tf_hi[2] + kAuxOff];
  }
  if ((j == p.tf_lo[1] - 1 || j == p.tf_hi[1]) && k >= p.tf_lo[2] && k <= p.tf_hi[2]) {
    const T inc = (T)p.e1[k + kAuxOff];
    tz_ = (j == p.tf_lo[1] - 1) ? inc : -inc;
  }
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

// The loads of one plane k of a column: E^n around the cell and the H^{n-1/2}
// and E^n the halo H values need (row y-1: H_x, H_z; column x-1: H_y, H_z),
// and, in x-slab tiles, the H-slab CPML memory of those H values.
template <class T>
struct PlaneLoads {
  T ez, ex1, ey1, ezx, eyx, ezy, exy, hx, hy, hz;  // own cell
  T ezd, eyd1, eydx, exd, hxd, hzd;                // row y-1
  T ezl, eyl, exl1, exly, hyl, hzl;                // column x-1
  T sy_, sz_, szd, syl, szl;                       // psi_H^{n-1/2}: own H_y, H_z; H_z(y-1); H_y, H_z(x-1)
};

template <class T, bool XS>
__device__ __forceinline__ void load_plane(const Params<T>& p, uint32_t id, uint32_t dzp, uint32_t dxp,
                                           uint32_t dyp, uint32_t dxm, uint32_t dym, uint32_t qs,
                                           uint32_t qsl, uint32_t sq, PlaneLoads<T>& v) {
  const T* __restrict__ Ex = p.E[0];
  const T* __restrict__ Ey = p.E[1];
  const T* __restrict__ Ez = p.E[2];
  v.ez = Ez[id];
  v.ex1 = Ex[id + dzp]; v.ey1 = Ey[id + dzp];
  v.ezx = Ez[id + dxp]; v.eyx = Ey[id + dxp];
  v.ezy = Ez[id + dyp]; v.exy = Ex[id + dyp];
  v.hx = p.Hi[0][id]; v.hy = p.Hi[1][id]; v.hz = p.Hi[2][id];
  const uint32_t qd = id - dym, ql = id - dxm;
  v.ezd = Ez[qd]; v.eyd1 = Ey[qd + dzp]; v.eydx = Ey[qd + dxp]; v.exd = Ex[qd];
  v.hxd = p.Hi[0][qd]; v.hzd = p.Hi[2][qd];
  v.ezl = Ez[ql]; v.eyl = Ey[ql]; v.exl1 = Ex[ql + dzp]; v.exly = Ex[ql + dyp];
  v.hyl = p.Hi[1][ql]; v.hzl = p.Hi[2][ql];
  if (XS) {
    // x-slab memory at (slab column, j, k): own and row y-1 (column qs),
    // column x-1 (column qsl); sq steps one row
    v.sy_ = p.psiHi[0][1][qs]; v.sz_ = p.psiHi[0][0][qs];
    v.szd = p.psiHi[0][0][qs - (dym ? sq : 0)];
    v.syl = p.psiHi[0][1][qsl]; v.szl = p.psiHi[0][0][qsl];
  }
}

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

template <class T, int TY, bool NT, bool XS>
__device__ __forceinline__ void fplain_tile(const Params<T>& p, const AuxParams& a, const Tile tile) {
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int i = tile.bx * kBX + threadIdx.x;
  const int j = tile.by * TY + threadIdx.y;
  if (i >= nx || j >= ny) return;
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
  const uint32_t dxp = xp ? 1 : 0, dyp = yp ? sy : 0, dxm = xm ? 1 : 0, dym = ym ? sy : 0;
  // E update ranges of the column
  const bool ax = i <= nx - 2 && j >= 1 && j <= ny - 2;
  const bool ay = i >= 1 && i <= nx - 2 && j <= ny - 2;
  const bool az = i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2;
  const bool tf_xband = p.tfsf && i >= p.tf_lo[0] && i <= p.tf_hi[0] - 1 && j >= p.tf_lo[1] &&
                        j <= p.tf_hi[1];
  const bool tf_zside = p.tfsf && j >= p.tf_lo[1] && j <= p.tf_hi[1] &&
                        (i == p.tf_lo[0] || i == p.tf_hi[0]);
  // x slab (tiles that meet one): the H-slab positions of the column and of
  // column x-1, the E-slab position of the column, their coefficients, and
  // slab-array indices (axis-0 slab arrays: ((k ny + j) 2 np + s))
  const int np = p.cp[0].np;
  const int sxh = XS ? slab_h(i, nx, np) : -1;
  const int sxl = (XS && xm) ? slab_h(i - 1, nx, np) : -1;
  const int sxe = XS ? slab_e(i, nx, np) : -1;
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
  uint32_t qs = ((uint32_t)k0 * ny + j) * w2 + (uint32_t)max(sxh, 0);
  uint32_t qsl = ((uint32_t)k0 * ny + j) * w2 + (uint32_t)max(sxl, 0);
  uint32_t qse = ((uint32_t)k0 * ny + j) * w2 + (uint32_t)max(sxe, 0);

  uint32_t id = (uint32_t)k0 * sz + (uint32_t)j * nx + i;
  // carried: E_x, E_y of plane k at the column, of the column x-1 (E_x) and
  // of the row y-1 (E_y); H_x, H_y^{n+1/2} of plane k-1 at the column
  T ex0 = Ex[id], ey0 = Ey[id];
  T exl0 = Ex[id - dxm], eyd0 = Ey[id - dym];
  T hxm = T(0), hym = T(0);
  if (k0 >= 1) {
    // H_x, H_y^{n+1/2} of plane k0-1 (recomputed; stored by the tile below)
    const uint32_t q = id - sz;
    const T exq = Ex[q], eyq = Ey[q], ezq = Ez[q];
    const T ezy = Ez[q + dyp], ezx = Ez[q + dxp];
    const T hx_ = p.Hi[0][q], hy_ = p.Hi[1][q];
    const T psy = XS ? p.psiHi[0][1][qs - sp] : T(0);
    T tyv, tzv;
    tf_h(p, i, j, k0 - 1, tyv, tzv);
    T dxy = ezx - ezq, psn;
    if (XS && sxh >= 0) dxy = xstretch(ch, dxy, psy, psn);
    hxm = upd_hx(i, j, k0 - 1, nx, ny, nz) ? hx_ - S * ((ezy - ezq) - (ey0 - eyq)) : hx_;
    hym = upd_hy(i, j, k0 - 1, nx, ny, nz) ? hy_ - S * (((ex0 - exq) - dxy) + tyv) : hy_;
  }
  for (int k = k0; k < k1; ++k, id += sz, qs += sp, qsl += sp, qse += sp) {
    const bool zp = k <= nz - 2;
    // ---- the plane's loads, issued together (one memory round trip per
    // plane; issuing the next plane's loads a plane ahead measured no faster)
    PlaneLoads<T> cur;
    load_plane<T, XS>(p, id, zp ? sz : 0, dxp, dyp, dxm, dym, qs, qsl, sq, cur);
    load_fence();
    const PlaneLoads<T>& v = cur;
    // ---- H^{n+1/2} of the cell
    T tyv, tzv;
    tf_h(p, i, j, k, tyv, tzv);
    T dxy = v.ezx - v.ez, dxz = v.eyx - ey0;  // x differences of H_y, H_z
    T psy = T(0), psz = T(0);
    if (XS && sxh >= 0) {
      dxy = xstretch(ch, dxy, v.sy_, psy);
      dxz = xstretch(ch, dxz, v.sz_, psz);
    }
    const bool uhx = upd_hx(i, j, k, nx, ny, nz), uhy = upd_hy(i, j, k, nx, ny, nz);
    const bool uhz = upd_hz(i, j, k, nx, ny, nz);
    const T hxn = uhx ? v.hx - S * ((v.ezy - v.ez) - (v.ey1 - ey0)) : v.hx;
    const T hyn = uhy ? v.hy - S * (((v.ex1 - ex0) - dxy) + tyv) : v.hy;
    const T hzn = uhz ? v.hz - S * ((dxz - (v.exy - ex0)) + tzv) : v.hz;
    if (uhx) put<NT>(&Hx[id], hxn);
    if (uhy) put<NT>(&Hy[id], hyn);
    if (uhz) put<NT>(&Hz[id], hzn);
    if (XS && sxh >= 0) {
      if (uhy) p.psiH[0][1][qs] = psy;
      if (uhz) p.psiH[0][0][qs] = psz;
    }
    // ---- halo H^{n+1/2}: row y-1 (H_x, H_z), column x-1 (H_y, H_z)
    T hxd = T(0), hzd = T(0), hyl = T(0), hzl = T(0);
    if (ym) {
      T tyd, tzd;
      tf_h(p, i, j - 1, k, tyd, tzd);
      T d = v.eydx - eyd0, ps;
      if (XS && sxh >= 0) d = xstretch(ch, d, v.szd, ps);
      hxd = upd_hx(i, j - 1, k, nx, ny, nz) ? v.hxd - S * ((v.ez - v.ezd) - (v.eyd1 - eyd0)) : v.hxd;
      hzd = upd_hz(i, j - 1, k, nx, ny, nz) ? v.hzd - S * ((d - (ex0 - v.exd)) + tzd) : v.hzd;
    }
    if (xm) {
      T tyl, tzl;
      tf_h(p, i - 1, j, k, tyl, tzl);
      T dy_ = v.ez - v.ezl, dz_ = ey0 - v.eyl, ps;
      if (XS && sxl >= 0) {
        dy_ = xstretch(cl, dy_, v.syl, ps);
        dz_ = xstretch(cl, dz_, v.szl, ps);
      }
      hyl = upd_hy(i - 1, j, k, nx, ny, nz) ? v.hyl - S * (((v.exl1 - exl0) - dy_) + tyl) : v.hyl;
      hzl = upd_hz(i - 1, j, k, nx, ny, nz) ? v.hzl - S * ((dz_ - (v.exly - exl0)) + tzl) : v.hzl;
    }
    // ---- E^{n+1}
    const bool kin = k >= 1 && k <= nz - 2;
    const bool uex = ax && kin, uey = ay && kin, uez = az && zp;
    T d_xy = hzn - hzl, d_xz = hyn - hyl;  // x differences of E_y, E_z
    if (XS && sxe >= 0) {
      if (uey) {
        T* q = p.psiE[0][1] + qse;
        T ps;
        d_xy = xstretch(ce, d_xy, *q, ps);
        *q = ps;
      }
      if (uez) {
        T* q = p.psiE[0][0] + qse;
        T ps;
        d_xz = xstretch(ce, d_xz, *q, ps);
        *q = ps;
      }
    }
    T cxv = (hzn - hzd) - (hyn - hym);  // dy H_z - dz H_y
    T cyv = (hxn - hxm) - d_xy;         // dz H_x - dx H_z
    T czv = d_xz - (hxn - hxd);         // dx H_y - dy H_x
    if (tf_xband) {
      if (k == p.tf_lo[2]) cxv += (T)fp_h_inc(a, p.tf_lo[2] - 1 + kAuxOff);
      if (k == p.tf_hi[2]) cxv -= (T)fp_h_inc(a, p.tf_hi[2] + kAuxOff);
    }
    if (tf_zside && k >= p.tf_lo[2] && k <= p.tf_hi[2] - 1) {
      const T inc = (T)fp_h_inc(a, k + kAuxOff);
      czv += (i == p.tf_lo[0]) ? -inc : inc;
    }
    const T sexy = k < p.sub_k ? p.SE : (k == p.sub_k ? p.se_avg : p.se_sub);
    const T sez = k < p.sub_k ? p.SE : p.se_sub;
    if (uex) put<NT>(&Ox[id], ex0 + sexy * cxv);
    if (uey) put<NT>(&Oy[id], ey0 + sexy * cyv);
    if (uez) put<NT>(&Oz[id], v.ez + sez * czv);
    // ---- carry up the column
    ex0 = v.ex1;
    ey0 = v.ey1;
    exl0 = v.exl1;
    eyd0 = v.eyd1;
    hxm = hxn;
    hym = hyn;
  }
}

// Class 0 of the two-sweep tiling (plain tiles, and tiles that meet only an
// x slab: their x-slab CPML behind a tile-uniform branch)
template <class T, int TY, bool NT>
__global__ void __launch_bounds__(kBX* TY) k_fplain(Params<T> p, AuxParams a) {
  const Tile tile = decode_tile(p.tl, p.tiles, 0, blockIdx.x);
  if (!tile.ok) return;
  const int np = p.cp[0].np;
  const bool xs = np > 0 && (tile.bx * kBX - 1 < np || tile.bx * kBX + kBX + 1 > p.nx - 1 - np);
  if (xs) fplain_tile<T, TY, NT, true>(p, a, tile);
  else fplain_tile<T, TY, NT, false>(p, a, tile);
}

template <class T, bool NT>
void launch_fplain_nt(const Params<T>& p, const AuxParams& a, int blocks, hipStream_t s) {
  if (p.tl.ty == 4) hipLaunchKernelGGL((k_fplain<T, 4, NT>), dim3(blocks), dim3(kBX, 4), 0, s, p, a);
  else if (p.tl.ty == 8) hipLaunchKernelGGL((k_fplain<T, 8, NT>), dim3(blocks), dim3(kBX, 8), 0, s, p, a);
  else hipLaunchKernelGGL((k_fplain<T, 2, NT>), dim3(blocks), dim3(kBX, 2), 0, s, p, a);
}

}  // namespace

template <class T>
void launch_fplain(const Params<T>& p, const AuxParams& a, hipStream_t s) {
  const int blocks = class_blocks(p.tl, 0);
  if (blocks == 0) return;
  if (p.stream_stores) launch_fplain_nt<T, true>(p, a, blocks, s);
  else launch_fplain_nt<T, false>(p, a, blocks, s);
}
template void launch_fplain<float>(const Params<float>&, const AuxParams&, hipStream_t);
template void launch_fplain<double>(const Params<double>&, const AuxParams&, hipStream_t);

}  // namespace gnor

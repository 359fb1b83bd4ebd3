// Discrete adjoint of the GNOR-FDTD step (gfx950): the exact transpose of the
// step the forward sweeps compute, run backward in time, for gradients of an
// extinction cross section with respect to a design density rho.
//
// The forward step is three linear maps of the state (TF/SF and the source
// are forcing terms and have no transpose):
//   (A) H' = H - S (h1 - h2),   h = kinv d + psi_H',  psi_H' = b psi_H + a d,
//       d = forward differences of E                         (f1, Sec. III)
//   (B) Phi_J' = Div J,  Phi_P' = Phi_P + Phi_J',  Q = g1 Phi_P' + g2 (3 Phi_J' - Phi_J)
//   (C) curl = c1 - c2,  c = kinv d + psi_E',  psi_E' = b psi_E + a d,
//       d = backward differences of H';
//       vacuum:  E' = E + SE curl
//       metal:   E' = E + cS curl - c3 E - c1 Em + cJ J - cG rho dQ,
//                J' = J + rho d3 (Em + 2E + E') - a_g J + rho dQ,   Em' = E
//       (current form of Eqs. GNORUpdate and discreteamperes, Sec. III; in
//       the design region d3 -> rho d3 inside cS, c3, c1, cJ, cG)
// and the adjoint step applies C^T, B^T, A^T in that order.  Each transposed
// difference operator is a gather: the adjoint of a raw difference d at a
// point is stored (D arrays) and collected by the points it read.
//
// Kernels, one thread per cell:
//   k_adj_e         C^T pointwise: adjoint E', Em', J', psi_E; dQ adjoints;
//                   difference adjoints D of the curl; gradient at design cells
//   k_adj_h_gather  H-bar += (backward-difference curl)^T D
//   k_adj_node      B^T: Q-bar from dQ adjoints; Phi adjoints
//   k_adj_j         J-bar += Div^T Phi_J-bar (metal points) and the objective's
//                   source for the previous step
//   k_adj_h         A^T pointwise: psi_H adjoints, difference adjoints D
//   k_adj_e_gather  E-bar += (forward-difference curl)^T D
#include "gnor_internal.h"

#include <cmath>

namespace gnor {

namespace {

__device__ __forceinline__ int a_slab_e(int g, int n, int np) {
  return g < np ? g : (g >= n - np ? g - (n - 2 * np) : -1);
}
__device__ __forceinline__ int a_slab_h(int g, int n, int np) {
  return g < np ? g : (g >= n - 1 - np ? g - (n - 1 - 2 * np) : -1);
}
__device__ __forceinline__ size_t a_slab_index(int a, int s, int i, int j, int k, int nx, int ny,
                                               int np) {
  const int w = 2 * np;
  if (a == 0) return ((size_t)k * ny + j) * w + s;
  if (a == 1) return ((size_t)k * w + s) * nx + i;
  return ((size_t)s * ny + j) * nx + i;
}

// forward update ranges (PEC walls): E_c and H_c
__device__ __forceinline__ bool e_upd(int c, int i, int j, int k, int nx, int ny, int nz) {
  const int ii[3] = {i, j, k}, nn[3] = {nx, ny, nz};
  for (int d = 0; d < 3; ++d) {
    const int lo = d == c ? 0 : 1;
    if (ii[d] < lo || ii[d] > nn[d] - 2) return false;
  }
  return true;
}
__device__ __forceinline__ bool h_upd(int c, int i, int j, int k, int nx, int ny, int nz) {
  const int ii[3] = {i, j, k}, nn[3] = {nx, ny, nz};
  for (int d = 0; d < 3; ++d) {
    const int lo = d == c ? 1 : 0;
    if (ii[d] < lo || ii[d] > nn[d] - 2) return false;
  }
  return true;
}

// adjoint of "c = kinv d + psi', psi' = b psi + a d" given c-bar: returns
// d-bar and updates psi-bar (in place) for a slab cell
template <class T>
__device__ __forceinline__ T adj_stretch(T* psib, size_t q, T b, T a, T ki, T cbar) {
  const T tot = psib[q] + cbar;
  psib[q] = b * tot;
  return ki * cbar + a * tot;
}

#define CELL_INDEX                                                           \
  const int i = blockIdx.x * 64 + threadIdx.x;                               \
  const int j = blockIdx.y * 4 + threadIdx.y;                                \
  const int k = blockIdx.z;                                                  \
  const Params<T>& p = A.p;                                                  \
  const int nx = p.nx, ny = p.ny, nz = p.nz;                                 \
  if (i >= nx || j >= ny) return;                                            \
  const size_t sy = nx, sz = (size_t)nx * ny;                                \
  const size_t id = (size_t)k * sz + (size_t)j * nx + i;                     \
  (void)sy;                                                                  \
  (void)sz

// ------------------------------------------------------------------ C^T
template <class T>
__global__ void __launch_bounds__(256) k_adj_e(AdjParams<T> A) {
  CELL_INDEX;
  const int np = p.cp[0].np;
  const int lx = i - p.mlo[0], ly = j - p.mlo[1], lz = k - p.mlo[2];
  const bool in_sub = p.any_metal && lx >= 0 && ly >= 0 && lz >= 0 && lx < p.mn[0] &&
                      ly < p.mn[1] && lz < p.mn[2];
  const size_t l = in_sub ? ((size_t)lz * p.mn[1] + ly) * p.mn[0] + lx : 0;
  const uint8_t mb = in_sub ? p.mask[l] : 0;
  // design cell?
  const int dx0 = i - A.dlo[0], dy0 = j - A.dlo[1], dz0 = k - A.dlo[2];
  const bool des = A.grad && dx0 >= 0 && dy0 >= 0 && dz0 >= 0 && dx0 < A.dn[0] && dy0 < A.dn[1] &&
                   dz0 < A.dn[2];
  const size_t dl = des ? ((size_t)dz0 * A.dn[1] + dy0) * A.dn[0] + dx0 : 0;
  const size_t Nd = (size_t)A.dn[0] * A.dn[1] * A.dn[2];
  double g = 0.0;
  const int ii[3] = {i, j, k};
  for (int c = 0; c < 3; ++c) {
    T* Db1 = A.D[2 * c];
    T* Db2 = A.D[2 * c + 1];
    if (!e_upd(c, i, j, k, nx, ny, nz)) {
      Db1[id] = T(0);
      Db2[id] = T(0);
      continue;  // E' = E there: E-bar passes unchanged
    }
    const T eb = A.Eb[c][id];
    T curlb;
    if ((mb >> c) & 1u) {
      const T r = p.rho ? (T)p.rho[l] : T(1);
      const T d3 = r * p.d3;
      const T inv = T(1) / (p.eps_inf + d3);
      const T cS = p.S * inv, c3 = T(3) * d3 * inv, c1 = d3 * inv, cJ = p.D2 * inv, cG = inv;
      const T jb = A.Jb[c][l];
      const T ob = A.Ob[c][l];
      const T etot = eb + d3 * jb;  // adjoint of E' including its use in J'
      A.Eb[c][id] = etot * (T(1) - c3) + T(2) * d3 * jb + ob;
      A.Ob[c][l] = -c1 * etot + d3 * jb;
      A.Jb[c][l] = cJ * etot + (T(1) - p.agam) * jb;
      A.dQb[c][l] = -cG * r * etot + r * jb;
      curlb = cS * etot;
      if (des) {
        // d L / d rho from this step: etot dE'/drho + jb (d3 (Em + 2E + E') + dQ)
        const T* fE = A.fE;
        const size_t lev = (size_t)A.lev_base;  // level of E^n
        const T En = fE[(lev * 3 + c) * Nd + dl];
        const T Em = fE[((lev - 1) * 3 + c) * Nd + dl];
        const T Ep = fE[((lev + 1) * 3 + c) * Nd + dl];
        const T dQ = A.fdQ[((size_t)A.t_idx * 3 + c) * Nd + dl];
        const T dEdr = (-T(3) * p.d3 * En - p.d3 * Em - dQ - p.d3 * (Ep - En)) * inv;
        g += (double)etot * (double)dEdr + (double)jb * (double)(p.d3 * (Em + T(2) * En + Ep) + dQ);
      }
    } else {
      // vacuum (or non-metal component): E' = E + SE curl, E-bar unchanged
      curlb = p.SE * eb;
      if (in_sub) A.dQb[c][l] = T(0);
    }
    // difference adjoints of the curl with CPML: curl = c1 - c2
    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
    T d1 = curlb, d2 = -curlb;
    if (np) {
      const int s1 = a_slab_e(ii[a1], a1 == 0 ? nx : (a1 == 1 ? ny : nz), np);
      const int s2 = a_slab_e(ii[a2], a2 == 0 ? nx : (a2 == 1 ? ny : nz), np);
      const CpmlAxis<T>& X1 = p.cp[a1];
      const CpmlAxis<T>& X2 = p.cp[a2];
      if (s1 >= 0)
        d1 = adj_stretch(A.psiEb[a1][0], a_slab_index(a1, s1, i, j, k, nx, ny, np), X1.be[s1], X1.ae[s1],
                         X1.ke[s1], d1);
      if (s2 >= 0)
        d2 = adj_stretch(A.psiEb[a2][1], a_slab_index(a2, s2, i, j, k, nx, ny, np), X2.be[s2], X2.ae[s2],
                         X2.ke[s2], d2);
    }
    Db1[id] = d1;
    Db2[id] = d2;
  }
  if (des) A.grad[dl] += g;
}

// H-bar_h(m) += D_{h+1,1}(m) - D_{h+1,1}(m + e_{h+2}) + D_{h+2,2}(m) - D_{h+2,2}(m + e_{h+1})
template <class T>
__global__ void __launch_bounds__(256) k_adj_h_gather(AdjParams<T> A) {
  CELL_INDEX;
  const size_t st[3] = {1, sy, sz};
  const int ii[3] = {i, j, k}, nn[3] = {nx, ny, nz};
  for (int h = 0; h < 3; ++h) {
    const int c1 = (h + 1) % 3, c2 = (h + 2) % 3;
    const T* D1 = A.D[2 * c1];
    const T* D2 = A.D[2 * c2 + 1];
    T s = D1[id] + D2[id];
    const int e1 = (h + 2) % 3, e2 = (h + 1) % 3;
    if (ii[e1] + 1 < nn[e1]) s -= D1[id + st[e1]];
    if (ii[e2] + 1 < nn[e2]) s -= D2[id + st[e2]];
    A.Hb[h][id] += s;
  }
}

// ------------------------------------------------------------------ B^T
// Q-bar(node) = sum_c dQ-bar_c(node - e_c) - dQ-bar_c(node);
// Phi_P'-bar = PP-bar + g1 Q-bar; Phi_J'-bar = PJ-bar + Phi_P'-bar + 3 g2 Q-bar;
// PP-bar <- Phi_P'-bar; PJ-bar <- -g2 Q-bar.
template <class T>
__global__ void __launch_bounds__(256) k_adj_node(AdjParams<T> A) {
  const Params<T>& p = A.p;
  const size_t M = (size_t)p.mn[0] * p.mn[1] * p.mn[2];
  const size_t l = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (l >= M) return;
  const int x = (int)(l % p.mn[0]);
  const int y = (int)((l / p.mn[0]) % p.mn[1]);
  const int z = (int)(l / ((size_t)p.mn[0] * p.mn[1]));
  const size_t s1 = p.mn[0], s2 = (size_t)p.mn[0] * p.mn[1];
  T q = -(A.dQb[0][l] + A.dQb[1][l] + A.dQb[2][l]);
  if (x > 0) q += A.dQb[0][l - 1];
  if (y > 0) q += A.dQb[1][l - s1];
  if (z > 0) q += A.dQb[2][l - s2];
  const T pp = A.PPb[l] + p.g1 * q;
  const T pj = A.PJb[l] + pp + T(3) * p.g2 * q;
  A.PPb[l] = pp;
  A.PJb[l] = -p.g2 * q;
  A.phiJb[l] = pj;
}

// J-bar_d(m) += Phi_J'-bar(m) - Phi_J'-bar(m + e_d) at metal points; then the
// objective's source for the step before: J-bar_x += C_L (cos(w t) B_re(k) +
// sin(w t) B_im(k)), t = (n_prev + 1/2) dt.
template <class T>
__global__ void __launch_bounds__(256) k_adj_j(AdjParams<T> A, int64_t n_prev) {
  const Params<T>& p = A.p;
  const size_t M = (size_t)p.mn[0] * p.mn[1] * p.mn[2];
  const size_t l = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (l >= M) return;
  const uint8_t mb = p.mask[l];
  if (!mb) return;
  const int x = (int)(l % p.mn[0]);
  const int y = (int)((l / p.mn[0]) % p.mn[1]);
  const int z = (int)(l / ((size_t)p.mn[0] * p.mn[1]));
  const size_t st[3] = {1, (size_t)p.mn[0], (size_t)p.mn[0] * p.mn[1]};
  const int xx[3] = {x, y, z};
  const T f0 = A.phiJb[l];
  for (int d = 0; d < 3; ++d) {
    if (!((mb >> d) & 1u)) continue;
    T v = f0;
    if (xx[d] + 1 < p.mn[d]) v -= A.phiJb[l + st[d]];
    A.Jb[d][l] += v;
  }
  if ((mb & 1u) && n_prev >= 0) {
    const int k = z + p.mlo[2];
    const double t = ((double)n_prev + 0.5) * A.dt;
    double sn, cs;
    sincos(A.omega * t, &sn, &cs);
    A.Jb[0][l] += (T)(A.CL * (cs * A.Bre[k] + sn * A.Bim[k]));
  }
}

// ------------------------------------------------------------------ A^T
template <class T>
__global__ void __launch_bounds__(256) k_adj_h(AdjParams<T> A) {
  CELL_INDEX;
  const int np = p.cp[0].np;
  const int ii[3] = {i, j, k};
  for (int h = 0; h < 3; ++h) {
    T* D1 = A.D[2 * h];
    T* D2 = A.D[2 * h + 1];
    if (!h_upd(h, i, j, k, nx, ny, nz)) {
      D1[id] = T(0);
      D2[id] = T(0);
      continue;
    }
    const T hb = A.Hb[h][id];
    // H' = H - S (h1 - h2): adjoints of the stretched differences
    T d1 = -p.S * hb, d2 = p.S * hb;
    const int a1 = (h + 1) % 3, a2 = (h + 2) % 3;
    if (np) {
      const int s1 = a_slab_h(ii[a1], a1 == 0 ? nx : (a1 == 1 ? ny : nz), np);
      const int s2 = a_slab_h(ii[a2], a2 == 0 ? nx : (a2 == 1 ? ny : nz), np);
      const CpmlAxis<T>& X1 = p.cp[a1];
      const CpmlAxis<T>& X2 = p.cp[a2];
      if (s1 >= 0)
        d1 = adj_stretch(A.psiHb[a1][0], a_slab_index(a1, s1, i, j, k, nx, ny, np), X1.bh[s1], X1.ah[s1],
                         X1.kh[s1], d1);
      if (s2 >= 0)
        d2 = adj_stretch(A.psiHb[a2][1], a_slab_index(a2, s2, i, j, k, nx, ny, np), X2.bh[s2], X2.ah[s2],
                         X2.kh[s2], d2);
    }
    D1[id] = d1;
    D2[id] = d2;
  }
}

// E-bar_c(m) += D_{c+1,1}(m - e_{c+2}) - D_{c+1,1}(m) + D_{c+2,2}(m - e_{c+1}) - D_{c+2,2}(m)
template <class T>
__global__ void __launch_bounds__(256) k_adj_e_gather(AdjParams<T> A) {
  CELL_INDEX;
  const size_t st[3] = {1, sy, sz};
  const int ii[3] = {i, j, k};
  for (int c = 0; c < 3; ++c) {
    const int h1 = (c + 1) % 3, h2 = (c + 2) % 3;
    const T* D1 = A.D[2 * h1];
    const T* D2 = A.D[2 * h2 + 1];
    T s = -(D1[id] + D2[id]);
    const int e1 = (c + 2) % 3, e2 = (c + 1) % 3;
    if (ii[e1] >= 1) s += D1[id - st[e1]];
    if (ii[e2] >= 1) s += D2[id - st[e2]];
    A.Eb[c][id] += s;
  }
}

// Forward values of the design region for the gradient: E^{n+1} (level
// lev_base + 1 of the store, read from the buffer the step wrote) and
// dQ_c = Q(node + e_c) - Q(node) of the step.
template <class T>
__global__ void __launch_bounds__(256) k_store_design(AdjParams<T> A, int store_e_only,
                                                      const T* Ex, const T* Ey, const T* Ez, int lev) {
  const Params<T>& p = A.p;
  const size_t Nd = (size_t)A.dn[0] * A.dn[1] * A.dn[2];
  const size_t dl = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (dl >= Nd) return;
  const int x = (int)(dl % A.dn[0]);
  const int y = (int)((dl / A.dn[0]) % A.dn[1]);
  const int z = (int)(dl / ((size_t)A.dn[0] * A.dn[1]));
  const int i = x + A.dlo[0], j = y + A.dlo[1], k = z + A.dlo[2];
  const size_t id = ((size_t)k * p.ny + j) * p.nx + i;
  T* fE = const_cast<T*>(A.fE);
  fE[((size_t)lev * 3 + 0) * Nd + dl] = Ex[id];
  fE[((size_t)lev * 3 + 1) * Nd + dl] = Ey[id];
  fE[((size_t)lev * 3 + 2) * Nd + dl] = Ez[id];
  if (store_e_only) return;
  const int lx = i - p.mlo[0], ly = j - p.mlo[1], lz = k - p.mlo[2];
  const size_t l = ((size_t)lz * p.mn[1] + ly) * p.mn[0] + lx;
  const T q0 = p.Q[l];
  T* fdQ = const_cast<T*>(A.fdQ);
  fdQ[((size_t)A.t_idx * 3 + 0) * Nd + dl] = p.Q[l + 1] - q0;
  fdQ[((size_t)A.t_idx * 3 + 1) * Nd + dl] = p.Q[l + p.mn[0]] - q0;
  fdQ[((size_t)A.t_idx * 3 + 2) * Nd + dl] = p.Q[l + (size_t)p.mn[0] * p.mn[1]] - q0;
}

}  // namespace

template <class T>
void launch_adjoint_step(const AdjParams<T>& A, int64_t n_prev, hipStream_t s) {
  const dim3 blk(64, 4), grd((A.p.nx + 63) / 64, (A.p.ny + 3) / 4, A.p.nz);
  const size_t M = (size_t)A.p.mn[0] * A.p.mn[1] * A.p.mn[2];
  const dim3 g1((unsigned)((M + 255) / 256));
  hipLaunchKernelGGL(k_adj_e<T>, grd, blk, 0, s, A);
  hipLaunchKernelGGL(k_adj_h_gather<T>, grd, blk, 0, s, A);
  if (A.p.any_metal) {
    hipLaunchKernelGGL(k_adj_node<T>, g1, dim3(256), 0, s, A);
    hipLaunchKernelGGL(k_adj_j<T>, g1, dim3(256), 0, s, A, n_prev);
  }
  hipLaunchKernelGGL(k_adj_h<T>, grd, blk, 0, s, A);
  hipLaunchKernelGGL(k_adj_e_gather<T>, grd, blk, 0, s, A);
}
template <class T>
void launch_adjoint_source(const AdjParams<T>& A, int64_t n, hipStream_t s) {
  // the objective's source for step n alone (phiJb must be zero)
  const size_t M = (size_t)A.p.mn[0] * A.p.mn[1] * A.p.mn[2];
  hipLaunchKernelGGL(k_adj_j<T>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, A, n);
}
template <class T>
void launch_store_design(const AdjParams<T>& A, int store_e_only, const T* Ex, const T* Ey,
                         const T* Ez, int lev, hipStream_t s) {
  const size_t Nd = (size_t)A.dn[0] * A.dn[1] * A.dn[2];
  hipLaunchKernelGGL(k_store_design<T>, dim3((unsigned)((Nd + 255) / 256)), dim3(256), 0, s, A,
                     store_e_only, Ex, Ey, Ez, lev);
}

template void launch_adjoint_step<float>(const AdjParams<float>&, int64_t, hipStream_t);
template void launch_adjoint_step<double>(const AdjParams<double>&, int64_t, hipStream_t);
template void launch_adjoint_source<float>(const AdjParams<float>&, int64_t, hipStream_t);
template void launch_adjoint_source<double>(const AdjParams<double>&, int64_t, hipStream_t);
template void launch_store_design<float>(const AdjParams<float>&, int, const float*, const float*,
                                         const float*, int, hipStream_t);
template void launch_store_design<double>(const AdjParams<double>&, int, const double*, const double*,
                                          const double*, int, hipStream_t);

}  // namespace gnor

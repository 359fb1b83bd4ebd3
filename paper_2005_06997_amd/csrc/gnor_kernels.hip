// HIP kernels of libgnorfdtd (gfx950).  Memory-bound stencils: one thread per
// cell, x fastest (coalesced), blocks of kBX x kBY cells of one z plane.
//
// Step n (Sec. III update order, f3 absent):
//   k_h       H^{n+1/2} from E^n (f1), CPML, TF/SF corrections with E_inc^n
//   k_aux_h   auxiliary line H_inc^{n+1/2}
//   k_ej      E^{n+1} (f2) and, at metal points, J^{n+1/2} (f4 in current
//             form) with the node scalars, CPML, TF/SF with H_inc^{n+1/2},
//             per-block plane sums of J_x for the spectra
//   k_aux_e   auxiliary line E_inc^{n+1} and the soft source
//   k_dft     running FP64 transforms of the induced current and E_inc
//   k_flux_*  staging / blocked accumulation of the flux-box transforms
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

// CPML-stretched derivative: kinv d + psi, psi <- b psi + a d (index units)
template <class T, bool HTYPE>
__device__ __forceinline__ T stretched(const Params<T>& p, int a, int t, int g, int i, int j,
                                       int k, T d) {
  const CpmlAxis<T>& ax = p.cp[a];
  if (ax.np == 0) return d;
  const int s = HTYPE ? slab_h(g, ax.n, ax.np) : slab_e(g, ax.n, ax.np);
  if (s < 0) return d;
  T* psi = HTYPE ? p.psiH[a][t] : p.psiE[a][t];
  const size_t q = slab_index(a, s, i, j, k, p.nx, p.ny, ax.np);
  const T b = HTYPE ? ax.bh[s] : ax.be[s];
  const T c = HTYPE ? ax.ah[s] : ax.ae[s];
  const T ki = HTYPE ? ax.kh[s] : ax.ke[s];
  const T ps = b * psi[q] + c * d;
  psi[q] = ps;
  return ki * d + ps;
}

template <class T>
__global__ void __launch_bounds__(kBX* kBY) k_h(Params<T> p) {
  const int i = blockIdx.x * kBX + threadIdx.x;
  const int j = blockIdx.y * kBY + threadIdx.y;
  const int k = blockIdx.z;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  if (i >= nx || j >= ny) return;
  const size_t sy = nx, sz = (size_t)nx * ny;
  const size_t id = (size_t)k * sz + (size_t)j * nx + i;
  const T* Ex = p.E[0];
  const T* Ey = p.E[1];
  const T* Ez = p.E[2];
  const bool in_tf = p.tfsf != 0;
  // H_x at (i, j+1/2, k+1/2): i in [1, nx-2], j in [0, ny-2], k in [0, nz-2]
  if (i >= 1 && i <= nx - 2 && j <= ny - 2 && k <= nz - 2) {
    const T dy = Ez[id + sy] - Ez[id];
    const T dz = Ey[id + sz] - Ey[id];
    const T curl = stretched<T, true>(p, 1, 0, j, i, j, k, dy) - stretched<T, true>(p, 2, 1, k, i, j, k, dz);
    p.H[0][id] -= p.S * curl;
  }
  // H_y at (i+1/2, j, k+1/2): i in [0, nx-2], j in [1, ny-2], k in [0, nz-2]
  if (i <= nx - 2 && j >= 1 && j <= ny - 2 && k <= nz - 2) {
    const T dz = Ex[id + sz] - Ex[id];
    const T dx = Ez[id + 1] - Ez[id];
    T curl = stretched<T, true>(p, 2, 0, k, i, j, k, dz) - stretched<T, true>(p, 0, 1, i, i, j, k, dx);
    if (in_tf && i >= p.tf_lo[0] && i <= p.tf_hi[0] - 1 && j >= p.tf_lo[1] && j <= p.tf_hi[1]) {
      if (k == p.tf_lo[2] - 1) curl -= (T)p.e1[p.tf_lo[2] + kAuxOff];
      if (k == p.tf_hi[2]) curl += (T)p.e1[p.tf_hi[2] + kAuxOff];
    }
    p.H[1][id] -= p.S * curl;
  }
  // H_z at (i+1/2, j+1/2, k): i in [0, nx-2], j in [0, ny-2], k in [1, nz-2]
  if (i <= nx - 2 && j <= ny - 2 && k >= 1 && k <= nz - 2) {
    const T dx = Ey[id + 1] - Ey[id];
    const T dy = Ex[id + sy] - Ex[id];
    T curl = stretched<T, true>(p, 0, 0, i, i, j, k, dx) - stretched<T, true>(p, 1, 1, j, i, j, k, dy);
    if (in_tf && i >= p.tf_lo[0] && i <= p.tf_hi[0] - 1 && k >= p.tf_lo[2] && k <= p.tf_hi[2]) {
      if (j == p.tf_lo[1] - 1) curl += (T)p.e1[k + kAuxOff];
      if (j == p.tf_hi[1]) curl -= (T)p.e1[k + kAuxOff];
    }
    p.H[2][id] -= p.S * curl;
  }
}

// Node scalars at local sub-grid node (x, y, z): Phi_J^{n-1/2} = Div J~^{n-1/2}
// (index units, zero outside the sub-grid), Phi_P^n = Phi_P^{n-1} + Phi_J,
// and Q = g1 Phi_P^n + g2 (3 Phi_J^{n-1/2} - Phi_J^{n-3/2}).
template <class T>
struct NodeVals {
  T phiJ, phiP, q;
};

template <class T>
__device__ __forceinline__ NodeVals<T> node_vals(const Params<T>& p, int x, int y, int z) {
  NodeVals<T> v{T(0), T(0), T(0)};
  const int m0 = p.mn[0], m1 = p.mn[1], m2 = p.mn[2];
  if (x < 0 || y < 0 || z < 0 || x >= m0 || y >= m1 || z >= m2) return v;
  const size_t l = ((size_t)z * m1 + y) * m0 + x;
  const size_t s1 = m0, s2 = (size_t)m0 * m1;
  T div = p.Ji[0][l] + p.Ji[1][l] + p.Ji[2][l];
  if (x > 0) div -= p.Ji[0][l - 1];
  if (y > 0) div -= p.Ji[1][l - s1];
  if (z > 0) div -= p.Ji[2][l - s2];
  v.phiJ = div;
  v.phiP = p.PPi[l] + div;
  v.q = p.g1 * v.phiP + p.g2 * (T(3) * div - p.PJi[l]);
  return v;
}

template <class T>
__global__ void __launch_bounds__(kBX* kBY) k_ej(Params<T> p) {
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i = blockIdx.x * kBX + tx;
  const int j = blockIdx.y * kBY + ty;
  const int k = blockIdx.z;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const size_t sy = nx, sz = (size_t)nx * ny;
  const bool valid = i < nx && j < ny;
  const size_t id = (size_t)k * sz + (size_t)j * (size_t)nx + (size_t)i;
  // sub-grid coordinates
  const int lx = i - p.mlo[0], ly = j - p.mlo[1], lz = k - p.mlo[2];
  const bool in_sub = valid && lx >= 0 && ly >= 0 && lz >= 0 && lx < p.mn[0] && ly < p.mn[1] &&
                      lz < p.mn[2];
  const size_t l = in_sub ? ((size_t)lz * p.mn[1] + ly) * p.mn[0] + lx : 0;
  const uint8_t mbits = in_sub ? p.mask[l] : 0;
  double jsum = 0.0;
  if (valid) {
    const T* Hx = p.H[0];
    const T* Hy = p.H[1];
    const T* Hz = p.H[2];
    NodeVals<T> nv0{T(0), T(0), T(0)};
    if (in_sub) {
      nv0 = node_vals(p, lx, ly, lz);
      p.PPo[l] = nv0.phiP;
      p.PJo[l] = nv0.phiJ;
    }
    for (int c = 0; c < 3; ++c) {
      // update range of E_c
      bool upd;
      if (c == 0) upd = i <= nx - 2 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2;
      else if (c == 1) upd = i >= 1 && i <= nx - 2 && j <= ny - 2 && k >= 1 && k <= nz - 2;
      else upd = i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && k <= nz - 2;
      if (!upd) continue;
      const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
      const size_t st1 = a1 == 0 ? 1 : (a1 == 1 ? sy : sz);
      const size_t st2 = a2 == 0 ? 1 : (a2 == 1 ? sy : sz);
      const T* Ha2 = a2 == 0 ? Hx : (a2 == 1 ? Hy : Hz);
      const T* Ha1 = a1 == 0 ? Hx : (a1 == 1 ? Hy : Hz);
      const int g1i = a1 == 0 ? i : (a1 == 1 ? j : k);
      const int g2i = a2 == 0 ? i : (a2 == 1 ? j : k);
      const T d1 = Ha2[id] - Ha2[id - st1];
      const T d2 = Ha1[id] - Ha1[id - st2];
      T curl = stretched<T, false>(p, a1, 0, g1i, i, j, k, d1) -
               stretched<T, false>(p, a2, 1, g2i, i, j, k, d2);
      if (p.tfsf) {
        if (c == 0 && i >= p.tf_lo[0] && i <= p.tf_hi[0] - 1 && j >= p.tf_lo[1] && j <= p.tf_hi[1]) {
          if (k == p.tf_lo[2]) curl += (T)p.h1[p.tf_lo[2] - 1 + kAuxOff];
          if (k == p.tf_hi[2]) curl -= (T)p.h1[p.tf_hi[2] + kAuxOff];
        }
        if (c == 2 && j >= p.tf_lo[1] && j <= p.tf_hi[1] && k >= p.tf_lo[2] && k <= p.tf_hi[2] - 1) {
          if (i == p.tf_lo[0]) curl -= (T)p.h1[k + kAuxOff];
          if (i == p.tf_hi[0]) curl += (T)p.h1[k + kAuxOff];
        }
      }
      const T en = p.E[c][id];
      if (!((mbits >> c) & 1u)) {
        p.O[c][id] = en + p.SE * curl;
        continue;
      }
      // metal point: f2 + f4 in current form
      int ox = lx, oy = ly, oz = lz;
      if (c == 0) ++ox;
      if (c == 1) ++oy;
      if (c == 2) ++oz;
      const NodeVals<T> nv1 = node_vals(p, ox, oy, oz);
      T cS = p.cS, c3 = p.c3, c1 = p.c1, cJ = p.cJ, cG = p.cG, d3 = p.d3;
      T G = nv1.q - nv0.q;
      if (p.rho) {
        const T r = (T)p.rho[l];
        d3 = r * p.d3;
        const T inv = T(1) / (p.eps_inf + d3);
        cS = p.S * inv; c3 = T(3) * d3 * inv; c1 = d3 * inv; cJ = p.D2 * inv; cG = inv;
        G = r * G;
      }
      const T em = p.O[c][id];
      const T jo = p.Ji[c][l];
      const T enew = en + (cS * curl - c3 * en - c1 * em + cJ * jo - cG * G);
      const T jnew = jo + (d3 * (em + T(2) * en + enew) - p.agam * jo + G);
      p.O[c][id] = enew;
      p.Jo[c][l] = jnew;
      if (c == 0) jsum = (double)jnew + (double)p.ebd * ((double)enew - (double)en);
    }
  }
  // deterministic per-block plane sum of J_x (spectra)
  const bool block_in_sub =
      (int)(blockIdx.x * kBX) < p.mlo[0] + p.mn[0] && (int)(blockIdx.x * kBX + kBX) > p.mlo[0] &&
      (int)(blockIdx.y * kBY) < p.mlo[1] + p.mn[1] && (int)(blockIdx.y * kBY + kBY) > p.mlo[1] &&
      k >= p.mlo[2] && k < p.mlo[2] + p.mn[2];
  if (block_in_sub) {
    __shared__ double red[kBX * kBY];
    const int t = ty * kBX + tx;
    red[t] = jsum;
    __syncthreads();
    for (int w = kBX * kBY / 2; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) p.jpart[(size_t)k * (p.nbx * p.nby) + blockIdx.y * p.nbx + blockIdx.x] = red[0];
  }
}

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

__global__ void __launch_bounds__(256) k_aux_h(AuxParams a) {
  for (int q = threadIdx.x; q <= a.n1 - 2; q += blockDim.x) {
    const double d = a.e1[q + 1] - a.e1[q];
    const double ps = a.bh[q] * a.ph[q] + a.ah[q] * d;
    a.ph[q] = ps;
    a.h1[q] -= a.S * (a.kh[q] * d + ps);
  }
}

__global__ void __launch_bounds__(256) k_aux_e(AuxParams a, int sub) {
  for (int q = 1 + threadIdx.x; q <= a.n1 - 2; q += blockDim.x) {
    const double d = a.h1[q] - a.h1[q - 1];
    const double ps = a.be[q] * a.pe[q] + a.ae[q] * d;
    a.pe[q] = ps;
    a.e1[q] -= a.SE * (a.ke[q] * d + ps);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t n = a.step_base[0] + sub;
    a.e1[kAuxSrc] += source_value(a, (double)(n + 1) * a.dt);
  }
}

// One block per grid plane: FP64 running transforms (factor dt, e^{+i w t}).
__global__ void __launch_bounds__(128) k_dft(DftParams d, int sub) {
  const int k = blockIdx.x;
  const int64_t n = d.step_base[0] + sub;
  if (d.every > 1 && (n % d.every) != 0) return;
  const double tJ = ((double)n + 0.5) * d.dt;
  const double tE = ((double)n + 1.0) * d.dt;
  __shared__ double red[128];
  const bool has_j = k >= d.kz0 && k < d.kz1;
  double s = 0.0;
  if (has_j) {
    const double* src = d.jpart + (size_t)k * d.nbxy;
    for (int b = threadIdx.x; b < d.nbxy; b += 128) s += src[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 64; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    s = red[0];
  }
  const double ei = d.e1[k + kAuxOff];
  for (int m = threadIdx.x; m < d.nf; m += 128) {
    const size_t q = (size_t)k * d.nf + m;
    double sn, cs;
    if (has_j) {
      sincos(d.omega[m] * tJ, &sn, &cs);
      d.a_re[q] += (d.wdt * cs) * s;
      d.a_im[q] += (d.wdt * sn) * s;
    }
    sincos(d.omega[m] * tE, &sn, &cs);
    d.b_re[q] += d.wdt * cs * ei;
    d.b_im[q] += d.wdt * sn * ei;
  }
}

__global__ void k_advance(int64_t* base, int64_t count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) base[0] += count;
}

// Flux staging: desc[3 s] = kind (0: E_c sample, 1: H_c averaged across the
// face), desc[3 s + 1] = component, desc[3 s + 2] = stride of the face
// normal; sidx[s] = linear cell index.
template <class T>
__global__ void __launch_bounds__(256) k_flux_stage(FluxParams f, Params<T> p, const int64_t* sidx,
                                                    int sub) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= f.nsamp) return;
  const int64_t n = f.step_base[0] + sub;
  const int slot = (int)(n % f.slots);
  const int kind = f.desc[3 * s];
  const int c = f.desc[3 * s + 1];
  const int64_t st = f.desc[3 * s + 2];
  const int64_t idx = sidx[s];
  double v;
  if (kind == 0) v = (double)p.O[c][idx];  // E^{n+1}
  else v = 0.5 * ((double)p.H[c][idx - st] + (double)p.H[c][idx]);  // H^{n+1/2}
  f.stage[(size_t)slot * f.nsamp + s] = v;
}

// acc[m][s] += sum_{b in [lo, hi)} wdt e^{i w_m t_b} stage[b][s], where slot b
// holds step w0 + b; E samples are stamped (n+1) dt, H samples (n+1/2) dt.
__global__ void __launch_bounds__(256) k_flux_acc(FluxParams f, const int* lo_ptr, int sub) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  const int64_t n_last = f.step_base[0] + sub;
  const int hi = (int)(n_last % f.slots) + 1;
  const int64_t w0 = n_last - (hi - 1);
  const int lo = lo_ptr[0];
  __shared__ double ph[2][2][64];  // [kind][cos/sin][slot]
  double v[64];
  const bool ok = s < f.nsamp;
  const int kind = ok ? f.desc[3 * s] : 0;
#pragma unroll
  for (int b = 0; b < 64; ++b) v[b] = (ok && b >= lo && b < hi) ? f.stage[(size_t)b * f.nsamp + s] : 0.0;
  for (int m = 0; m < f.nf; ++m) {
    __syncthreads();
    if (threadIdx.x < 128) {
      const int b = threadIdx.x & 63;
      const int kd = threadIdx.x >> 6;
      const double t = ((double)(w0 + b) + (kd == 0 ? 1.0 : 0.5)) * f.dt;
      double sn, cs;
      sincos(f.omega[m] * t, &sn, &cs);
      ph[kd][0][b] = f.wdt * cs;
      ph[kd][1][b] = f.wdt * sn;
    }
    __syncthreads();
    if (!ok) continue;
    double re = 0.0, im = 0.0;
    for (int b = lo; b < hi; ++b) {
      re += ph[kind][0][b] * v[b];
      im += ph[kind][1][b] * v[b];
    }
    const size_t q = (size_t)m * f.nsamp + s;
    f.acc_re[q] += re;
    f.acc_im[q] += im;
  }
}

__global__ void k_flux_set(int* lo_ptr, FluxParams f, int sub) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int64_t n_last = f.step_base[0] + sub;
    const int hi = (int)(n_last % f.slots) + 1;
    lo_ptr[0] = hi == f.slots ? 0 : hi;
  }
}

// out[box * nf + m] = sum over the box's (E, H) sample pairs of
// w_p Re(E conj(H)) (fixed order, deterministic).
__global__ void __launch_bounds__(256) k_flux_reduce(const double* are, const double* aim,
                                                     const double* pw, int npairs, int np0, int nf,
                                                     double* out) {
  const int m = blockIdx.x, box = blockIdx.y;
  const int p0 = box == 0 ? 0 : np0, p1 = box == 0 ? np0 : npairs;
  const int nsamp = 2 * npairs;
  const double* re = are + (size_t)m * nsamp;
  const double* im = aim + (size_t)m * nsamp;
  double s = 0.0;
  for (int p = p0 + threadIdx.x; p < p1; p += 256)
    s += pw[p] * (re[2 * p] * re[2 * p + 1] + im[2 * p] * im[2 * p + 1]);
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(size_t)box * nf + m] = red[0];
}

template <class T>
__global__ void __launch_bounds__(256) k_nonfinite(const T* a, size_t n, int* flag) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * 256;
  int bad = 0;
  for (; i < n; i += stride) bad |= !isfinite(a[i]);
  if (bad) atomicOr(flag, 1);
}

}  // namespace

template <class T>
void launch_h(const Params<T>& p, int, hipStream_t s) {
  dim3 blk(kBX, kBY, 1), grd((p.nx + kBX - 1) / kBX, (p.ny + kBY - 1) / kBY, p.nz);
  hipLaunchKernelGGL(k_h<T>, grd, blk, 0, s, p);
}
template <class T>
void launch_ej(const Params<T>& p, int, hipStream_t s) {
  dim3 blk(kBX, kBY, 1), grd((p.nx + kBX - 1) / kBX, (p.ny + kBY - 1) / kBY, p.nz);
  hipLaunchKernelGGL(k_ej<T>, grd, blk, 0, s, p);
}
void launch_aux_h(const AuxParams& p, int, hipStream_t s) {
  hipLaunchKernelGGL(k_aux_h, dim3(1), dim3(256), 0, s, p);
}
void launch_aux_e(const AuxParams& p, int sub, hipStream_t s) {
  hipLaunchKernelGGL(k_aux_e, dim3(1), dim3(256), 0, s, p, sub);
}
void launch_dft(const DftParams& p, int sub, hipStream_t s) {
  hipLaunchKernelGGL(k_dft, dim3(p.nz), dim3(128), 0, s, p, sub);
}
void launch_advance(int64_t* base, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, base, count);
}
template <class T>
void launch_flux_stage(const FluxParams& f, const Params<T>& p, const int64_t* sidx, int sub,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_flux_stage<T>, dim3((f.nsamp + 255) / 256), dim3(256), 0, s, f, p, sidx, sub);
}
void launch_flux_accumulate(const FluxParams& f, int* lo_ptr, int sub, hipStream_t s) {
  hipLaunchKernelGGL(k_flux_acc, dim3((f.nsamp + 255) / 256), dim3(256), 0, s, f, lo_ptr, sub);
  hipLaunchKernelGGL(k_flux_set, dim3(1), dim3(64), 0, s, lo_ptr, f, sub);
}
void launch_flux_reduce(const double* are, const double* aim, const double* pw, int npairs,
                        int npairs_box0, int nf, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_flux_reduce, dim3(nf, 2), dim3(256), 0, s, are, aim, pw, npairs, npairs_box0, nf,
                     out);
}
template <class T>
void launch_nonfinite(const T* a, size_t n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite<T>, dim3(1024), dim3(256), 0, s, a, n, flag);
}

template void launch_h<float>(const Params<float>&, int, hipStream_t);
template void launch_h<double>(const Params<double>&, int, hipStream_t);
template void launch_ej<float>(const Params<float>&, int, hipStream_t);
template void launch_ej<double>(const Params<double>&, int, hipStream_t);
template void launch_flux_stage<float>(const FluxParams&, const Params<float>&, const int64_t*, int,
                                       hipStream_t);
template void launch_flux_stage<double>(const FluxParams&, const Params<double>&, const int64_t*, int,
                                        hipStream_t);
template void launch_nonfinite<float>(const float*, size_t, int*, hipStream_t);
template void launch_nonfinite<double>(const double*, size_t, int*, hipStream_t);

}  // namespace gnor

// Spectral read-out kernels of libgnorfdtd (gfx950), all FP64.
//
//   k_dft          blocks [0, nz): running transforms (factor dt, e^{+i w t})
//                  of the plane sums of the induced current J_x (stamped
//                  (n+1/2) dt) and of the incident line E_inc (stamped
//                  (n+1) dt), with the step's phase table from the E sweep;
//                  blocks [nz, ...): staging of the flux-box samples (E on
//                  the face, H averaged across it)
//   k_flux_phase   phase table of one accumulation window
//   k_flux_acc     acc[m][s] += sum_b wdt e^{i w_m t_b} stage[b][s]: the
//                  staged window folded into the flux-box transforms
//   k_flux_reduce  sum over sample pairs of w_p Re(E conj(H)) per box and
//                  frequency (fixed order)
#include "gnor_internal.h"

#include <cmath>

namespace gnor {

namespace {

// Block blk of the spectra launch of one simulation.
template <class T>
__device__ __forceinline__ void dft_block(const DftParams& d, const FluxParams& f, const Params<T>& p,
                                          int sub, int blk) {
  const int64_t n = d.step_base[0] + sub;
  if (blk < d.nz) {
    const int k = blk;
    if (d.nf == 0 || (d.every > 1 && (n % d.every) != 0)) return;
    __shared__ double red[256];
    const bool has_j = k >= d.kz0 && k < d.kz1;
    double s = 0.0;
    if (has_j) {
      const double* src = d.jpart + (size_t)k * d.nbxy;
      for (int b = threadIdx.x; b < d.nbxy; b += 256) s += src[b];
      red[threadIdx.x] = s;
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
      }
      s = red[0];
    }
    const double ei = d.e1[k + kAuxOff];
    const int nf = d.nf;
    for (int m = threadIdx.x; m < nf; m += 256) {
      const size_t q = (size_t)k * nf + m;
      if (has_j) {
        d.a_re[q] += (d.wdt * d.phase[m]) * s;
        d.a_im[q] += (d.wdt * d.phase[nf + m]) * s;
      }
      d.b_re[q] += d.wdt * d.phase[2 * nf + m] * ei;
      d.b_im[q] += d.wdt * d.phase[3 * nf + m] * ei;
    }
    return;
  }
  // flux staging: pair q -> (segment, face point)
  const int q = (blk - d.nz) * 256 + threadIdx.x;
  if (q >= f.npairs) return;
  int sgi = 0;
  while (sgi + 1 < f.nseg && q >= f.seg[sgi + 1].first) ++sgi;
  const FluxSeg& g = f.seg[sgi];
  const int r = q - g.first;
  int c[3];
  c[g.a] = g.p;
  c[g.in_axis] = g.in_lo + r % g.n_in;
  c[g.out_axis] = g.out_lo + r / g.n_in;
  const size_t sy = f.nx, sz = (size_t)f.nx * f.ny;
  const size_t idx = (size_t)c[2] * sz + (size_t)c[1] * sy + c[0];
  const size_t st = g.a == 0 ? 1 : (g.a == 1 ? sy : sz);
  const int slot = (int)(n % kFluxSlots);
  const double e = (double)p.O[g.ecomp][idx];  // E^{n+1}
  const double h = 0.5 * ((double)p.H[g.hcomp][idx - st] + (double)p.H[g.hcomp][idx]);  // H^{n+1/2}
  f.stage[(size_t)slot * f.nsamp + q] = e;
  f.stage[(size_t)slot * f.nsamp + f.npairs + q] = h;
}

template <class T>
__global__ void __launch_bounds__(256) k_dft(DftParams d, FluxParams f, Params<T> p, int sub) {
  dft_block<T>(d, f, p, sub, blockIdx.x);
}

// Batch: instance q owns blocks [dblk0, dblk0 + dnblk) of the launch.
template <class T>
__global__ void __launch_bounds__(256) k_dft_batch(const BatchEntry<T>* __restrict__ e, int n, int sub) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (e[mid].dblk0 <= (int)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const BatchEntry<T>& en = e[lo];
  dft_block<T>(en.d, en.f, en.p, sub, blockIdx.x - en.dblk0);
}

__global__ void k_advance(int64_t* base, int64_t count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) base[0] += count;
}

template <class T>
__global__ void k_advance_batch(const BatchEntry<T>* __restrict__ e, int n, int64_t count) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) const_cast<int64_t*>(e[q].p.step_base)[0] += count;
}

// ptab[m][kind][cos|sin][b] = wdt e^{i w_m t_b}; slot b of the window holds
// step w0 + b; E samples are stamped (n+1) dt, H samples (n+1/2) dt.
__global__ void __launch_bounds__(2 * kFluxSlots) k_flux_phase(FluxParams f, int sub) {
  const int m = blockIdx.x;
  const int64_t n_last = f.step_base[0] + sub;
  const int64_t w0 = n_last - (n_last % kFluxSlots);
  const int b = threadIdx.x % kFluxSlots;
  const int kind = threadIdx.x / kFluxSlots;
  const double t = ((double)(w0 + b) + (kind == 0 ? 1.0 : 0.5)) * f.dt;
  double s, c;
  sincos(f.omega[m] * t, &s, &c);
  double* out = f.ptab + ((size_t)m * 2 + kind) * 2 * kFluxSlots;
  out[b] = f.wdt * c;
  out[kFluxSlots + b] = f.wdt * s;
}

// acc[m][s] += sum_{b in [lo, hi)} ptab[m][kind(s)][.][b] stage[b][s]
__global__ void __launch_bounds__(256) k_flux_acc(FluxParams f, const int* lo_ptr, int sub) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  const int64_t n_last = f.step_base[0] + sub;
  const int hi = (int)(n_last % kFluxSlots) + 1;
  const int lo = lo_ptr[0];
  const bool ok = s < f.nsamp;
  const int kind = (ok && s >= f.npairs) ? 1 : 0;
  double v[kFluxSlots];
#pragma unroll
  for (int b = 0; b < kFluxSlots; ++b)
    v[b] = (ok && b >= lo && b < hi) ? f.stage[(size_t)b * f.nsamp + s] : 0.0;
  __shared__ double ph[2][2][kFluxSlots];
  for (int m = 0; m < f.nf; ++m) {
    __syncthreads();
    if (threadIdx.x < 4 * kFluxSlots) {
      const double* src = f.ptab + (size_t)m * 4 * kFluxSlots;
      (&ph[0][0][0])[threadIdx.x] = src[threadIdx.x];
    }
    __syncthreads();
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int b = 0; b < kFluxSlots; ++b) {
      re += ph[kind][0][b] * v[b];
      im += ph[kind][1][b] * v[b];
    }
    if (ok) {
      const size_t q = (size_t)m * f.nsamp + s;
      f.acc_re[q] += re;
      f.acc_im[q] += im;
    }
  }
}

__global__ void k_flux_set(int* lo_ptr, FluxParams f, int sub) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int64_t n_last = f.step_base[0] + sub;
    const int hi = (int)(n_last % kFluxSlots) + 1;
    lo_ptr[0] = hi == kFluxSlots ? 0 : hi;
  }
}

// out[box * nf + m] = sum over the box's (E, H) pairs of w_p Re(E conj(H~))
__global__ void __launch_bounds__(256) k_flux_reduce(const double* are, const double* aim,
                                                     const double* pw, int npairs, int np0, int nf,
                                                     double* out) {
  const int m = blockIdx.x, box = blockIdx.y;
  const int p0 = box == 0 ? 0 : np0, p1 = box == 0 ? np0 : npairs;
  const size_t nsamp = 2 * (size_t)npairs;
  const double* re = are + (size_t)m * nsamp;
  const double* im = aim + (size_t)m * nsamp;
  double s = 0.0;
  for (int q = p0 + threadIdx.x; q < p1; q += 256)
    s += pw[q] * (re[q] * re[npairs + q] + im[q] * im[npairs + q]);
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

int dft_blocks(const DftParams& d, const FluxParams& f) { return d.nz + (f.npairs + 255) / 256; }

template <class T>
void launch_dft_stage(const DftParams& d, const FluxParams& f, const Params<T>& p, int sub,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_dft<T>, dim3(dft_blocks(d, f)), dim3(256), 0, s, d, f, p, sub);
}
template <class T>
void launch_dft_batch(const BatchEntry<T>* e, int n, int blocks, int sub, hipStream_t s) {
  hipLaunchKernelGGL(k_dft_batch<T>, dim3(blocks), dim3(256), 0, s, e, n, sub);
}
template <class T>
void launch_advance_batch(const BatchEntry<T>* e, int n, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_advance_batch<T>, dim3((n + 63) / 64), dim3(64), 0, s, e, n, count);
}
template void launch_dft_batch<float>(const BatchEntry<float>*, int, int, int, hipStream_t);
template void launch_dft_batch<double>(const BatchEntry<double>*, int, int, int, hipStream_t);
template void launch_advance_batch<float>(const BatchEntry<float>*, int, int64_t, hipStream_t);
template void launch_advance_batch<double>(const BatchEntry<double>*, int, int64_t, hipStream_t);
void launch_advance(int64_t* base, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, base, count);
}
void launch_flux_accumulate(const FluxParams& f, int* lo_ptr, int sub, hipStream_t s) {
  hipLaunchKernelGGL(k_flux_phase, dim3(f.nf), dim3(2 * kFluxSlots), 0, s, f, sub);
  hipLaunchKernelGGL(k_flux_acc, dim3((f.nsamp + 255) / 256), dim3(256), 0, s, f, lo_ptr, sub);
  hipLaunchKernelGGL(k_flux_set, dim3(1), dim3(64), 0, s, lo_ptr, f, sub);
}
void launch_flux_reduce(const double* are, const double* aim, const double* pw, int npairs,
                        int npairs_box0, int nf, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_flux_reduce, dim3(nf, 2), dim3(256), 0, s, are, aim, pw, npairs, npairs_box0,
                     nf, out);
}
template <class T>
void launch_nonfinite(const T* a, size_t n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite<T>, dim3(1024), dim3(256), 0, s, a, n, flag);
}

template void launch_dft_stage<float>(const DftParams&, const FluxParams&, const Params<float>&, int,
                                      hipStream_t);
template void launch_dft_stage<double>(const DftParams&, const FluxParams&, const Params<double>&, int,
                                       hipStream_t);
template void launch_nonfinite<float>(const float*, size_t, int*, hipStream_t);
template void launch_nonfinite<double>(const double*, size_t, int*, hipStream_t);

}  // namespace gnor

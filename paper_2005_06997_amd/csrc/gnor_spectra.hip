// Spectral read-out kernels of libgnorfdtd (gfx950), all FP64.
//
//   k_dft          blocks [0, nz): running transforms (factor dt, e^{+i w t})
//                  of the plane sums of the induced current J_x (stamped
//                  (n+1/2) dt) and of the incident line E_inc (stamped
//                  (n+1) dt), with the step's phase table from the E sweep;
//                  blocks [nz, ...): staging of the flux-box samples (E on
//                  the face, H averaged across it), the x-normal faces one
//                  thread per grid row)
//   k_flux_phase   phase table of one accumulation window (matrix-core
//                  fragments)
//   k_flux_acc     acc[s][m] += sum_b wdt e^{i w_m t_b} stage[b][s]: the
//                  staged window folded into the flux-box transforms, on the
//                  FP64 matrix cores (each sample's transforms contiguous)
//   k_flux_reduce  sums of w_p Re(E conj(H)) over chunks of sample pairs,
//   k_flux_sum     then over a box's chunks, per frequency (fixed order)
//   k_maps         near-field and density maps on one grid plane: running
//                  transforms of E (stamped (n+1) dt) and of n - n0 from the
//                  step's node scalars Phi~_P^n (stamped n dt)
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
  // flux staging: E^{n+1} on the face, H^{n+1/2} averaged across it
  const int u = (blk - d.nz) * 256 + threadIdx.x;
  const size_t sy = f.nx, sz = (size_t)f.nx * f.ny;
  double* stage = f.stage + (size_t)(n % kFluxSlots) * f.nsamp;
  if (u < f.xnrow) {
    // one (y, z) row: the samples of every x-normal face on it (inner index
    // y, outer z; the H neighbour across the face is the row's previous cell)
    const int j = f.xj0 + u % f.xnj, k = f.xk0 + u / f.xnj;
    for (int sgi = 0; sgi < f.nseg; ++sgi) {
      const FluxSeg& g = f.seg[sgi];
      if (g.a != 0) continue;
      const int ri = j - g.in_lo, ro = k - g.out_lo;
      if (ri < 0 || ri >= g.n_in || ro < 0 || ro >= g.count / g.n_in) continue;
      const int q = g.first + ro * g.n_in + ri;
      const size_t idx = (size_t)k * sz + (size_t)j * sy + g.p;
      stage[q] = (double)p.O[g.ecomp][idx];
      stage[f.npairs + q] = 0.5 * ((double)p.H[g.hcomp][idx - 1] + (double)p.H[g.hcomp][idx]);
    }
    return;
  }
  // the r-th pair of the faces whose normal is y or z -> (segment, face point)
  int r = u - f.xnrow;
  if (r >= f.nrest) return;
  int sgi = 0;
  for (; sgi < f.nseg; ++sgi) {
    if (f.seg[sgi].a == 0) continue;
    if (r < f.seg[sgi].count) break;
    r -= f.seg[sgi].count;
  }
  if (sgi == f.nseg) return;
  const FluxSeg& g = f.seg[sgi];
  int c[3];
  c[g.a] = g.p;
  c[g.in_axis] = g.in_lo + r % g.n_in;
  c[g.out_axis] = g.out_lo + r / g.n_in;
  const size_t idx = (size_t)c[2] * sz + (size_t)c[1] * sy + c[0];
  const size_t st = g.a == 1 ? sy : sz;
  const int q = g.first + r;
  stage[q] = (double)p.O[g.ecomp][idx];
  stage[f.npairs + q] = 0.5 * ((double)p.H[g.hcomp][idx - st] + (double)p.H[g.hcomp][idx]);
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
    if (entry_at(e, mid).dblk0 <= (int)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const BatchEntry<T>& en = entry_at(e, lo);
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

// The window's fold acc += P_kind V is a matrix product: rows R = 2m + c of
// P (c = 0: wdt cos(w_m t_b), c = 1: wdt sin(w_m t_b)), columns b = window
// slots, V[b][s] = stage[b][s].  It runs on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64: 16 rows x 16 samples x 4 slots per instruction).
// Register layouts of that instruction, lane l of the wavefront:
//   A (16 x 4):  A[l % 16][l / 16]
//   B (4 x 16):  B[l / 16][l % 16]
//   D (16 x 16): D[4 r + l / 16][l % 16] in element r of the double4.
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kFluxKB = kFluxSlots / 4;  // 4-slot steps per window
constexpr int kFluxTW = 13;              // row tiles per wavefront

// row tiles of P (2 nf rows, 16 per tile), padded to whole wavefront groups
__host__ __device__ __forceinline__ int flux_row_tiles(int nf) {
  const int t = (nf + 7) / 8;
  return (t + kFluxTW - 1) / kFluxTW * kFluxTW;
}

// ptab[kind][g][kb][t][l] = A fragment of row tile g kFluxTW + t, slots
// 4kb .. 4kb+3 (zero for rows past 2 nf and slots outside the unfolded part
// [lo, hi) of the window): the fragments one wavefront loads per step are
// contiguous.  Slot b holds step w0 + b; E samples are stamped (n+1) dt, H
// samples (n+1/2) dt.
__global__ void __launch_bounds__(256) k_flux_phase(FluxParams f, const int* lo_ptr, int sub) {
  const int T = flux_row_tiles(f.nf);
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= 2 * T * kFluxKB * 64) return;
  const int l = idx & 63;
  const int q = idx >> 6;
  const int kb = q / kFluxTW % kFluxKB;
  const int gq = q / kFluxTW / kFluxKB;  // kind * (T / kFluxTW) + row group
  const int t = (gq % (T / kFluxTW)) * kFluxTW + q % kFluxTW;
  const int kind = gq / (T / kFluxTW);
  const int b = 4 * kb + (l >> 4);
  const int R = 16 * t + (l & 15);
  const int m = R >> 1;
  const int64_t n_last = f.step_base[0] + sub;
  const int64_t w0 = n_last - (n_last % kFluxSlots);
  const int hi = (int)(n_last % kFluxSlots) + 1;
  const int lo = lo_ptr[0];
  double v = 0.0;
  if (m < f.nf && b >= lo && b < hi) {
    const double tb = ((double)(w0 + b) + (kind == 0 ? 1.0 : 0.5)) * f.dt;
    double sn, cs;
    sincos(f.omega[m] * tb, &sn, &cs);
    v = f.wdt * ((R & 1) ? sn : cs);
  }
  f.ptab[idx] = v;
}

// One wavefront: 16 samples (a column tile) of one kind x up to kFluxTW row
// tiles.  Blocks of 4 wavefronts take 4 adjacent column tiles; the row groups
// of a column group are consecutive blocks of one XCD (blocks are dealt
// round-robin to the 8 XCDs), so the group's stage columns are read from
// HBM once.
__global__ void __launch_bounds__(256) k_flux_acc(FluxParams f, const int* lo_ptr, int sub, int ncg8) {
  const int T = flux_row_tiles(f.nf);
  const int WT = T / kFluxTW;
  const int bid = blockIdx.x;
  const int xcd = bid & 7, r = bid >> 3;
  const int g = r % WT;
  const int rest = r / WT;                  // [kind][column group / 8]
  const int kind = rest / (ncg8 >> 3);
  const int cg = (rest % (ncg8 >> 3)) * 8 + xcd;
  const int l = threadIdx.x & 63;
  const int ct = cg * 4 + (threadIdx.x >> 6);
  const int col = ct * 16 + (l & 15);        // pair index of this lane's sample
  if (kind > 1 || ct * 16 >= f.npairs) return;  // whole wavefront
  const bool colok = col < f.npairs;
  // lanes past the last pair read (and never store) the kind's first sample
  const size_t s = (size_t)kind * f.npairs + (colok ? col : 0);
  const int t0 = g * kFluxTW;
  const int64_t n_last = f.step_base[0] + sub;
  const int hi = (int)(n_last % kFluxSlots) + 1;
  const int lo = lo_ptr[0];
  const size_t ns = f.nsamp;
  // the window's sum, added to the running transforms at the end
  dbl4 acc[kFluxTW];
#pragma unroll
  for (int t = 0; t < kFluxTW; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
  const double* pa = f.ptab + (size_t)(kind * WT + g) * kFluxKB * kFluxTW * 64 + l;
  // 4-slot steps covering [lo, hi), widened to whole groups of 8 steps
  // inside the window (the extra steps have zero phase factors)
  constexpr int G = 8;
  int kb0 = lo >> 2, kb1 = (hi + 3) >> 2;
  {
    const int cnt = (kb1 - kb0 + G - 1) / G * G;
    kb1 = min(kFluxKB, kb0 + cnt);
    kb0 = kb1 - cnt;
  }
  if (kb0 == kb1) return;  // nothing staged since the last fold
  // Operands of step kb: A fragments pa[(kb kFluxTW + t) 64] (phase table,
  // cache-resident), loaded one fold ahead into two buffers in turn, and the
  // B fragment from the staging ring (HBM).  The B fragments of a group of 8
  // steps are loaded together one group ahead: memory counters retire in
  // order, so a B load issued with each fold would hold up the next fold's A
  // operands for a full HBM round trip.  Slots outside [lo, hi) meet zero
  // phase factors; the ring holds finite values there (zeroed at reset,
  // earlier samples after).
  auto load_a = [&](int kb, double (&a)[kFluxTW]) {
#pragma unroll
    for (int t = 0; t < kFluxTW; ++t) a[t] = pa[((size_t)kb * kFluxTW + t) * 64];
  };
  auto load_b = [&](int kb, double (&b)[G]) {
#pragma unroll
    for (int j = 0; j < G; ++j) b[j] = f.stage[(size_t)(4 * (kb + j) + (l >> 4)) * ns + s];
  };
  auto fold = [&](const double (&a)[kFluxTW], double v) {
#pragma unroll
    for (int t = 0; t < kFluxTW; ++t)
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], v, acc[t], 0, 0, 0);
  };
  double a0[kFluxTW], a1[kFluxTW], bq[G], bn[G];
  load_b(kb0, bq);
  load_a(kb0, a0);
  // scheduling barriers keep each load group ahead of its use
  for (int kb = kb0; kb < kb1; kb += G) {
    const int nx = kb + G < kb1 ? kb + G : kb;  // the last group's reloads are not used
    load_a(kb + 1, a1);
    load_b(nx, bn);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < G; j += 2) {
      fold(a0, bq[j]);
      __builtin_amdgcn_sched_barrier(0);
      load_a(j + 2 < G ? kb + j + 2 : nx, a0);
      __builtin_amdgcn_sched_barrier(0);
      fold(a1, bq[j + 1]);
      __builtin_amdgcn_sched_barrier(0);
      if (j + 3 < G) load_a(kb + j + 3, a1);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 0; j < G; ++j) bq[j] = bn[j];
  }
  // acc[s][R] (R = 2m + c): the wavefront's 16 samples are 16 consecutive
  // runs of 2 nf doubles, and the four elements q of a tile t fill its
  // 16-row slice of each
  // run in turn.  Tiles go in groups of 7 whose 28 loads are all issued
  // before the group's stores (rows past 2 nf read the run's last element
  // and store nothing): 2 round trips per lane instead of one guarded round
  // trip per element, within the registers of the fold loop.
  double* const dst = f.acc + s * (2 * (size_t)f.nf);
  const int rlast = 2 * f.nf - 1;
  constexpr int TG = 7;
#pragma unroll
  for (int tg = 0; tg < kFluxTW; tg += TG) {
    double old[TG][4];
#pragma unroll
    for (int u = 0; u < TG; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (tg + u < kFluxTW) old[u][q] = dst[min(16 * (t0 + tg + u) + 4 * q + (l >> 4), rlast)];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < TG; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int R = 16 * (t0 + tg + u) + 4 * q + (l >> 4);
        if (tg + u < kFluxTW && colok && R <= rlast) dst[R] = old[u][q] + acc[tg + u][q];
      }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One thread per plane point; the block's phase factors of the step in LDS.
template <class T>
__global__ void __launch_bounds__(256) k_maps(MapParams<T> m, int sub) {
  const int64_t n = m.step_base[0] + sub;
  if (m.every > 1 && (n % m.every) != 0) return;  // the whole launch
  __shared__ double ph[4][8];  // cos, sin of w t_E; cos, sin of w t_N
  const int t = threadIdx.x;
  if (t < m.nmap) {
    double sn, cs;
    sincos(m.omega[t] * ((double)(n + 1) * m.dt), &sn, &cs);
    ph[0][t] = cs;
    ph[1][t] = sn;
    sincos(m.omega[t] * ((double)n * m.dt), &sn, &cs);
    ph[2][t] = cs;
    ph[3][t] = sn;
  }
  __syncthreads();
  const double wdt = m.dt * (m.every > 1 ? m.every : 1);
  if (blockIdx.x == 0 && t < m.nmap) {
    const double ei = m.e1[m.norm_k + kAuxOff];
    m.inc[2 * t] += wdt * ph[0][t] * ei;
    m.inc[2 * t + 1] += wdt * ph[1][t] * ei;
  }
  const int plane = m.nu * m.nv;
  const int q = blockIdx.x * 256 + t;
  if (q >= plane) return;
  const int ua = m.axis == 0 ? 1 : 0, va = m.axis == 2 ? 1 : 2;
  int c[3];
  c[m.axis] = m.index;
  c[ua] = q % m.nu;
  c[va] = q / m.nu;
  const size_t id = ((size_t)c[2] * m.ny + c[1]) * m.nx + c[0];
  const double e[3] = {(double)m.E[0][id], (double)m.E[1][id], (double)m.E[2][id]};
  const int lx = c[0] - m.mlo[0], ly = c[1] - m.mlo[1], lz = c[2] - m.mlo[2];
  double dens = 0.0;
  if (m.PP && lx >= 0 && ly >= 0 && lz >= 0 && lx < m.mn[0] && ly < m.mn[1] && lz < m.mn[2])
    dens = (double)m.PP[((size_t)lz * m.mn[1] + ly) * m.mn[0] + lx] * m.nscale;
  const size_t qs = (size_t)m.nmap * plane;  // stride between quantities
  for (int k = 0; k < m.nmap; ++k) {
    const size_t o = (size_t)k * plane + q;
    for (int a = 0; a < 3; ++a) {
      m.acc[(2 * a) * qs + o] += (wdt * ph[0][k]) * e[a];
      m.acc[(2 * a + 1) * qs + o] += (wdt * ph[1][k]) * e[a];
    }
    m.acc[6 * qs + o] += (wdt * ph[2][k]) * dens;
    m.acc[7 * qs + o] += (wdt * ph[3][k]) * dens;
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
// part[b][m] = sum over the pairs p of chunk b of w_p Re(E conj(H~)) at
// frequency m, in pair order: block b takes chunk b (box 0's chunks first,
// kFluxChunk pairs each, none across the boxes' boundary), thread i the
// frequencies m = i, i + 128, ... (a wavefront reads a pair's transforms
// as one contiguous run)
__global__ void __launch_bounds__(128) k_flux_reduce(const double* acc, const double* pw, int npairs,
                                                     int np0, int nf, double* part) {
  const int b = blockIdx.x;
  const int nb0 = (np0 + kFluxChunk - 1) / kFluxChunk;
  const int p0 = b < nb0 ? b * kFluxChunk : np0 + (b - nb0) * kFluxChunk;
  const int p1 = min(p0 + kFluxChunk, b < nb0 ? np0 : npairs);
  const size_t rs = 2 * (size_t)nf;
  for (int m = threadIdx.x; m < nf; m += 128) {
    double s = 0.0;
    for (int q = p0; q < p1; ++q) {
      const double* e = acc + (size_t)q * rs + 2 * m;
      const double* h = acc + (size_t)(npairs + q) * rs + 2 * m;
      s += pw[q] * (e[0] * h[0] + e[1] * h[1]);
    }
    part[(size_t)b * nf + m] = s;
  }
}

// out[box nf + m] = the box's chunk sums in chunk order
__global__ void k_flux_sum(const double* part, int nb0, int nb, int nf, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * nf) return;
  const int box = i / nf, m = i - box * nf;
  double s = 0.0;
  for (int b = box == 0 ? 0 : nb0; b < (box == 0 ? nb0 : nb); ++b) s += part[(size_t)b * nf + m];
  out[i] = s;
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

int dft_blocks(const DftParams& d, const FluxParams& f) { return d.nz + (f.xnrow + f.nrest + 255) / 256; }

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
template <class T>
void launch_maps(const MapParams<T>& m, int sub, hipStream_t s) {
  if (m.nmap <= 0) return;
  hipLaunchKernelGGL(k_maps<T>, dim3((m.nu * m.nv + 255) / 256), dim3(256), 0, s, m, sub);
}
template void launch_maps<float>(const MapParams<float>&, int, hipStream_t);
template void launch_maps<double>(const MapParams<double>&, int, hipStream_t);

size_t flux_ptab_doubles(int nf) { return (size_t)2 * flux_row_tiles(nf) * kFluxKB * 64; }

void launch_flux_accumulate(const FluxParams& f, int* lo_ptr, int sub, hipStream_t s) {
  const int T = flux_row_tiles(f.nf);
  const int WT = T / kFluxTW;
  const int nct = (f.npairs + 15) / 16;          // column tiles per kind
  const int ncg8 = ((nct + 3) / 4 + 7) / 8 * 8;  // column groups per kind, padded to 8
  const int phase_threads = 2 * T * kFluxKB * 64;
  hipLaunchKernelGGL(k_flux_phase, dim3((phase_threads + 255) / 256), dim3(256), 0, s, f,
                     (const int*)lo_ptr, sub);
  hipLaunchKernelGGL(k_flux_acc, dim3(2 * ncg8 * WT), dim3(256), 0, s, f, (const int*)lo_ptr, sub,
                     ncg8);
  hipLaunchKernelGGL(k_flux_set, dim3(1), dim3(64), 0, s, lo_ptr, f, sub);
}
void launch_flux_reduce(const double* acc, const double* pw, int npairs, int npairs_box0, int nf,
                        double* part, double* out, hipStream_t s) {
  const int nb = flux_reduce_chunks(npairs, npairs_box0);
  const int nb0 = (npairs_box0 + kFluxChunk - 1) / kFluxChunk;
  if (nb > 0)
    hipLaunchKernelGGL(k_flux_reduce, dim3(nb), dim3(128), 0, s, acc, pw, npairs, npairs_box0, nf, part);
  hipLaunchKernelGGL(k_flux_sum, dim3((2 * nf + 255) / 256), dim3(256), 0, s, part, nb0, nb, nf, out);
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

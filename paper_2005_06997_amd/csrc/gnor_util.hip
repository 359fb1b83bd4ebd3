// Small kernels of libgnorfdtd outside the time step: the design density
// (checked and scattered into the metal sub-grid's weight array from a
// device array), the free-electron density read-out, and a fill kernel for
// clears that a captured graph may hold.
//
//   k_design_check    flags any design density outside [0, 1] (or NaN)
//   k_design_scatter  rho[z][y][x] of the design box -> weight of the
//                     metal sub-grid (the weight scales wp^2, beta^2 and D)
//   k_density         n - n0 = div P_f^n / e at the sub-grid's nodes (Eq. Nsol),
//                     from the node scalar Phi~_P^{n-1} of the last H sweep and
//                     the node divergence of J^{n-1/2} (P^n - P^{n-1} = dt J)
// and the static device buffer of gnor_batch_create_static.
#include "gnor_internal.h"

#include <mutex>

// Parameter tables of a batch made by gnor_batch_create_static (callers that
// cannot allocate device memory).  One copy per GPU, held until the process
// ends.  In host code this name is only a stand-in: the device address of a
// GPU's copy is looked up once per device (static_table_address) and only
// that address is ever handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[gnor::kStaticTableBytes];

namespace gnor {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {};

__global__ void __launch_bounds__(256) k_design_check(const float* __restrict__ rho, size_t n,
                                                      int* flag) {
  int bad = 0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float r = rho[i];
    bad |= !(r >= 0.0f && r <= 1.0f);
  }
  if (bad) atomicOr(flag, 1);
}

__global__ void __launch_bounds__(256) k_design_scatter(const float* __restrict__ rho, DesignMap d,
                                                        float* __restrict__ weight) {
  const size_t nd = (size_t)d.dn[0] * d.dn[1] * d.dn[2];
  for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < nd; q += (size_t)gridDim.x * 256) {
    const int x = (int)(q % d.dn[0]);
    const int y = (int)((q / d.dn[0]) % d.dn[1]);
    const int z = (int)(q / ((size_t)d.dn[0] * d.dn[1]));
    const size_t l = ((size_t)(z + d.off[2]) * d.mn[1] + (y + d.off[1])) * d.mn[0] + (x + d.off[0]);
    weight[l] = rho[q];
  }
}

// Node (lx, ly, lz) of the sub-grid: Phi~_P^{n-1} + sum_a (J~_a(node) -
// J~_a(node - e_a)), in index units scaled by eps0 / dx (so that the
// product with `scale` is n - n0 in m^-3).  J vanishes on the sub-grid's
// outer halo (metal lies at least one cell inside it), so a neighbour off
// the sub-grid contributes zero.
template <class T>
__global__ void __launch_bounds__(256) k_density(const T* __restrict__ pp, const T* __restrict__ jx,
                                                 const T* __restrict__ jy, const T* __restrict__ jz,
                                                 int m0, int m1, int m2, double scale,
                                                 double* __restrict__ out) {
  const size_t M = (size_t)m0 * m1 * m2;
  for (size_t l = (size_t)blockIdx.x * 256 + threadIdx.x; l < M; l += (size_t)gridDim.x * 256) {
    const int lx = (int)(l % m0), ly = (int)((l / m0) % m1), lz = (int)(l / ((size_t)m0 * m1));
    double v = (double)pp[l];
    v += (double)jx[l] - (lx > 0 ? (double)jx[l - 1] : 0.0);
    v += (double)jy[l] - (ly > 0 ? (double)jy[l - m0] : 0.0);
    v += (double)jz[l] - (lz > 0 ? (double)jz[l - (size_t)m0 * m1] : 0.0);
    out[l] = v * scale;
  }
}

__global__ void __launch_bounds__(256) k_fill_zero(uint32_t* __restrict__ a, size_t nwords) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < nwords; i += (size_t)gridDim.x * 256)
    a[i] = 0u;
}

unsigned grid_for(size_t n) {
  const size_t b = (n + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

void launch_design_check(const float* rho, size_t n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_design_check, dim3(grid_for(n)), dim3(256), 0, s, rho, n, flag);
}
void launch_design_scatter(const float* rho, const DesignMap& d, float* weight, hipStream_t s) {
  const size_t nd = (size_t)d.dn[0] * d.dn[1] * d.dn[2];
  hipLaunchKernelGGL(k_design_scatter, dim3(grid_for(nd)), dim3(256), 0, s, rho, d, weight);
}
template <class T>
void launch_density(const T* pp, const T* jx, const T* jy, const T* jz, const int mn[3], double scale,
                    double* out, hipStream_t s) {
  const size_t M = (size_t)mn[0] * mn[1] * mn[2];
  hipLaunchKernelGGL(k_density<T>, dim3(grid_for(M)), dim3(256), 0, s, pp, jx, jy, jz, mn[0], mn[1],
                     mn[2], scale, out);
}
template void launch_density<float>(const float*, const float*, const float*, const float*,
                                    const int[3], double, double*, hipStream_t);
template void launch_density<double>(const double*, const double*, const double*, const double*,
                                     const int[3], double, double*, hipStream_t);
hipError_t static_table_address(int* device, void** addr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[dev]) {
    // with device `dev` current: the address of this device's copy
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = p;
  }
  *device = dev;
  *addr = g_scratch_addr[dev];
  return hipSuccess;
}

void launch_fill_zero(void* a, size_t bytes, hipStream_t s) {
  const size_t nw = bytes / 4;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(nw)), dim3(256), 0, s, static_cast<uint32_t*>(a), nw);
}

}  // namespace gnor

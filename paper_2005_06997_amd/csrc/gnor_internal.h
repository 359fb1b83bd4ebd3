// Internal definitions shared by the host runtime and the HIP kernels of
// libgnorfdtd.  Not part of the ABI.
//
// Units inside the library are scaled so that every update coefficient is
// O(1) (important for FP32 storage):
//   E~ = E (V/m),  H~ = eta0 H,  J~ = J dt / eps0,  P~ = P / eps0,
//   node scalars Phi~_P = dx div P / eps0 and Phi~_J = dx dt div J / eps0,
// so that, with S = c dt / dx and integer-index differences D_a,
//   H~  -= S curl_idx E                           (f1, Sec. III)
//   E   += (S / eps_b) curl_idx H~                (vacuum)
// and in the metal (f2 + f4 of Sec. III rewritten for the current):
//   E^{n+1} = E^n + [S curl H~ - 3 d3 E^n - d3 E^{n-1} + D2 J~ - G] / (eps_inf + d3)
//   J~^{n+1/2} = J~ - a_g J~ + d3 (E^{n-1} + 2 E^n + E^{n+1}) + G
// with d3 = D3 / eps0, a_g = 1 + D2 = gamma dt / (1 + gamma dt / 2), and
// G_a = Q(node + e_a) - Q(node), Q = g1 Phi~_P^n + g2 (3 Phi~_J^{n-1/2} - Phi~_J^{n-3/2}),
// g1 = D_G1 / dx^2, g2 = D_G2 / dx^2, Phi~_P^n = Phi~_P^{n-1} + Phi~_J^{n-1/2}.
// This is Eq. (GNORUpdate) with D1 = 1 - D2, grad(div P) = Grad(Div P)
// (Eq. GradDiv is exactly the gradient of the node divergence), and the BDF2
// combination 3 GD^n - 4 GD^{n-1} + GD^{n-2} = Grad(dt (3 Div J^{n-1/2} -
// Div J^{n-3/2})).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace gnor {

// Auxiliary incident line: CPML cells at each end, offset of grid plane k = 0,
// soft-source cell.
constexpr int kAuxPml = 20;
constexpr int kAuxOff = 25;
constexpr int kAuxSrc = 22;

// Field sweeps: blocks of 64 (x, one wavefront) x TY (y) columns, each column
// marching over kz planes.
constexpr int kBX = 64;
constexpr int kMaxCP = 4;        // critical points per material
constexpr int kFluxSlots = 256;  // flux staging depth (steps per accumulation)
constexpr int kAuxThreads = 256;  // threads of a batch's auxiliary-line block
// Field stores of a sweep go nontemporal when its field traffic (9 words per
// cell) exceeds this: larger sweeps cycle the 256 MB Infinity Cache anyway,
// and keeping their one-shot outputs out of it leaves it to the re-read halo
// (320^3 FP32: 0.76 -> 0.69 ms per step); a smaller grid's outputs are
// re-read from it by the next sweep (160^3 FP32: 12 % slower streamed).
constexpr double kStreamStoreBytes = 256.0 * 1024 * 1024;
constexpr int kClasses = 4;     // tile classes of a sweep (plain, CPML, metal, metal + CPML)

template <class T>
struct CpmlAxis {
  int n;          // nodes along the axis
  int np;         // slab thickness (0 = none)
  const T* be;    // [2 np] at integer positions (E updates)
  const T* ae;
  const T* ke;
  const T* bh;    // [2 np] at half-integer positions (H updates)
  const T* ah;
  const T* kh;
};

// Tiling of a sweep: tiles of 64 x ty columns by kz planes, numbered x
// fastest, then y, then z, and split into kClasses classes (plain Yee, CPML,
// metal, metal + CPML) that run as separate launches.  Within a class's launch, block b
// takes a position in the class's tile list according to the tile order
// (blocks are dealt to the 8 XCDs round-robin):
//   0: natural order;
//   1: XCD bands: position (b mod 8) * per + b / 8, so each XCD owns a
//      contiguous band of the list and neighbouring tiles share its L2;
//   2: chunks of q positions dealt round-robin to the XCDs, each XCD sweeping
//      its chunk's consecutive positions (balanced and local).
struct Tiling {
  int ty, kz;
  int xcd;        // tile order 0, 1 or 2 (above)
  int nbx, nby, nbz;
  int q;          // chunk size for order 2 (8 rows of tiles)
  int cn[kClasses];    // tiles per class
  int coff[kClasses];  // offset of each class's list in the tile list
  int cper[kClasses];  // positions (order 1) or chunks (order 2) per XCD, per class
};

// Auxiliary line state (FP64 always).
struct AuxParams {
  int n1;
  double S, SE;
  // substrate (see Params::sub_k): line cell q carries plane q - kAuxOff
  int sub_k;
  double se_avg, se_sub;
  double* e1;
  double* h1;
  double* pe;
  double* ph;
  const double* be;
  const double* ae;
  const double* ke;
  const double* bh;
  const double* ah;
  const double* kh;
  int src_kind;
  int src_cell;   // line cell of the soft source (kAuxSrc, or the source plane + kAuxOff)
  double e0, omega_c, tau, t0, omega_max, dt;
  // phase table of the step for the spectra: [cos tJ, sin tJ, cos tE, sin tE][nf]
  int nf;
  const double* omega;
  double* phase;
  int every;
  const int64_t* step_base;
};

// Device pointers and coefficients of one simulation (one precision).
template <class T>
struct Params {
  int nx, ny, nz;
  T S;            // Courant number: H coefficient
  T SE;           // S / eps_b: vacuum E coefficient
  // dielectric substrate: E_x, E_y on planes k > sub_k and E_z on planes
  // k >= sub_k use se_sub = S / eps_sub, E_x, E_y on plane sub_k use se_avg
  // (the mean permittivity); sub_k = nz + 1 without a substrate
  int sub_k;
  T se_avg, se_sub;
  // full-grid fields
  T* E[3];        // E^n
  T* O[3];        // E^{n-1} (read at metal points) -> E^{n+1} (written everywhere)
  const T* Hi[3]; // H^{n-1/2} (the step's input buffer)
  T* H[3];        // H^{n+1/2} (the step's output buffer)
  // metal sub-grid [mlo, mlo + mn)
  int any_metal;
  int stream_stores;  // store H and E^{n+1} nontemporally (see kStreamStoreBytes)
  int mlo[3], mn[3];
  const uint8_t* mask;  // sub-grid, bit c = P_c is metal
  const int* colz;      // per sub-grid column: first and last plane of nodes on a metal edge
  const float* rho;     // optional per-cell weight of wp^2, beta^2, D (sub-grid); null = 1
  const T* Ji[3];
  T* Jo[3];
  const T* PPi;
  T* PPo;
  const T* PJi;
  T* PJo;
  T* Q;                 // Q of the step's node scalars (written by k_h, read by k_ej)
  T eps_inf, d3, agam, D2, g1, g2, ebd;  // ebd = eps_inf - eps_b
  T cS, c3, c1, cJ, cG;                   // E metal coefficients divided by (eps_inf + d3 + c3sum)
  // critical points (bound electrons) at the metal points, per pole u:
  // P = P_CP/eps0 and its last increment Q on the sub-grid, updated in place;
  // Q^{n+1} = cpa P + (1 - cpb) Q + cp4 (2 E^n) - cp5 (E^n - E^{n-1}) + cp3 (E^{n+1} - E^n)
  int ncp;
  T cpa[kMaxCP], cpb[kMaxCP], cp3[kMaxCP], cp4[kMaxCP], cp5[kMaxCP];
  T c3sum;              // sum of cp3 (in the E divisor)
  T* cpP[kMaxCP][3];
  T* cpQ[kMaxCP][3];
  // CPML memory: psi[axis][t], t = 0 for component (axis+2)%3, 1 for (axis+1)%3;
  // psi_E is updated in place, psi_H read from psiHi and written to psiH
  T* psiE[3][2];
  const T* psiHi[3][2];
  T* psiH[3][2];
  CpmlAxis<T> cp[3];
  // total-field operation: metal points in cells within np of a face follow
  // the local Drude model (G = 0 there; tiles of class 3 only)
  int lra_pml;
  // TF/SF
  int tfsf;
  int tf_lo[3], tf_hi[3];
  const double* e1;
  const double* h1;
  // per-(plane, tile, wavefront) partial sums of the induced current J_x
  double* jpart;      // [nz][nbx * nby * ty]
  Tiling tl;
  const int* tiles;   // tile lists of the classes, back to back
  const uint8_t* tile_class;  // class of every tile (tile order x, y, z)
  const int64_t* step_base;
};

// One face segment of the flux boxes: (E, H) sample pairs on a rectangle of
// the face plane p (normal axis a); pair q of the segment lies at
// inner = q % n_in, outer = q / n_in.
struct FluxSeg {
  int first;          // first pair index
  int count;
  int a, p;
  int ecomp, hcomp;   // E component sampled on the face, H component averaged across it
  int in_axis, out_axis;
  int in_lo, out_lo, n_in;
};
constexpr int kMaxSeg = 24;

struct DftParams {
  int nz, nf;
  int kz0, kz1;          // planes [kz0, kz1) carry induced current
  int nbxy;              // partial sums per plane
  const double* jpart;
  const double* phase;   // [4][nf] from the auxiliary block of the E sweep
  double wdt;
  int every;
  const double* e1;      // auxiliary line, E_inc^{n+1}
  double* a_re;          // [nz][nf]
  double* a_im;
  double* b_re;
  double* b_im;
  const int64_t* step_base;
};

// Flux monitors: samples staged every step, accumulated every kFluxSlots.
// Sample s < npairs is the E sample of pair s, s >= npairs the H sample of
// pair s - npairs.
struct FluxParams {
  int npairs, nsamp;     // nsamp = 2 npairs
  int nf;
  int nseg;
  FluxSeg seg[kMaxSeg];
  int nx, ny;
  // staging order of the sampling launch: first one thread per (y, z) row of
  // the union of the x-normal faces (rows [xj0, xj0 + xnj) x [xk0, ...),
  // xnrow rows in all), which stages every x-normal sample on its row (a
  // gather of one value per row, whichever thread takes it); then the nrest
  // pairs of the faces whose normal is y or z, in segment order
  int xj0, xnj, xk0, xnrow;
  int nrest;
  double* stage;         // [kFluxSlots][nsamp]
  double* acc;           // [nsamp][2 nf]: sample s, frequency m: re at 2m, im at 2m + 1
  const double* omega;
  double* ptab;          // window phase factors as matrix fragments (flux_ptab_doubles)
  double dt, wdt;
  const int64_t* step_base;
};

// Near-field and density maps on one grid plane (running transforms).
template <class T>
struct MapParams {
  int axis, index, nmap, every;
  int nu, nv, nx, ny;               // plane size; grid strides
  const double* omega;              // [nmap]
  double* acc;                      // [8][nmap][nv][nu]
  double* inc;                      // [nmap][2]
  double dt, nscale;                // nscale: Phi~_P -> n - n0 (eps0 / (dx e))
  int mlo[3], mn[3];                // metal sub-grid
  const T* E[3];                    // E^{n+1}
  const T* PP;                      // Phi~_P^n on the sub-grid (this step's node scalars)
  const double* e1;                 // auxiliary line (E_inc^{n+1})
  int norm_k;
  const int64_t* step_base;
};

// Adjoint state and workspace (all device pointers).
template <class T>
struct AdjParams {
  Params<T> p;             // forward coefficients, masks, CPML profiles, Q
  T* Eb[3];                // adjoint of E (full grid)
  T* Hb[3];                // adjoint of H
  T* Ob[3];                // adjoint of E^{n-1} at metal points (sub-grid)
  T* Jb[3];                // adjoint of J (sub-grid)
  T* PPb;                  // adjoints of the node scalars (sub-grid)
  T* PJb;
  T* phiJb;                // workspace: adjoint of Phi_J' of the step
  T* dQb[3];               // workspace: adjoints of dQ_c at metal points
  T* D[6];                 // workspace: adjoints of raw differences, [2 c + term]
  T* psiEb[3][2];          // adjoint CPML memory
  T* psiHb[3][2];
  // design region (cells [dlo, dlo + dn)) and stored forward values
  int dlo[3], dn[3];
  const T* fE;             // [level][3][Nd] E at levels n0-1 .. n1 of a segment
  const T* fdQ;            // [step][3][Nd] dQ_c of each step of the segment
  int lev_base;            // level of E^n for the step being transposed
  int t_idx;               // index of that step within the segment
  double* grad;            // [Nd] d objective / d rho
  // objective: sigma_ext(omega) = sum_n sum_k w_n(k) (plane sum of J~_x)
  double dt, omega, CL;
  const double* Bre;       // [nz] incident transform at omega
  const double* Bim;
};

template <class T>
void launch_adjoint_step(const AdjParams<T>& A, int64_t n_prev, hipStream_t s);
template <class T>
void launch_adjoint_source(const AdjParams<T>& A, int64_t n, hipStream_t s);
template <class T>
void launch_store_design(const AdjParams<T>& A, int store_e_only, const T* Ex, const T* Ey,
                         const T* Ez, int lev, hipStream_t s);

// One instance of a batch: its parameters and its block ranges in the batched
// sweep launches of each tile class (blk0[c] .. blk0[c] + nblk[c]; class 0
// ends with the instance's auxiliary-line block), in the batched spectra
// launch (dblk0 .. dblk0 + dnblk), in the batched TF/SF launch of step
// form 3 (fblk0 .. fblk0 + fnblk; none where no one-pass tile meets the
// shell of the TF box) and in its node-scalar launch (sblk0 .. sblk0 +
// snblk; none without metal).
template <class T>
struct BatchEntry {
  Params<T> p;
  AuxParams a;
  DftParams d;
  FluxParams f;
  int blk0[kClasses], nblk[kClasses];
  int dblk0, dnblk;
  int fblk0, fnblk;
  int sblk0, snblk;
  // 1: the instance's metal tiles (class 2) take the two sweeps in the
  // batch's current step form (form 0, or critical points); 0: one pass
  int two_sweep2;
};

// Entry i of a batch table on the device.  The table is written before a
// launch and only read during it, so it is read through the constant
// address space: its loads are then invariant, and the compiler reloads an
// instance's parameters where they are used instead of holding them all in
// registers (which had lowered the batched kernels' occupancy).
template <class T>
__device__ __forceinline__ const BatchEntry<T>& entry_at(const BatchEntry<T>* e, int i) {
  typedef __attribute__((address_space(4))) const BatchEntry<T> ConstEntry;
  return *(const BatchEntry<T>*)((ConstEntry*)e + i);
}

// one class of the batched sweeps (blocks: that class's blocks of all instances)
template <class T>
void launch_h_batch_class(const BatchEntry<T>* e, int n, int blocks, int ty, int c, bool nt,
                          hipStream_t s);
template <class T>
void launch_ej_batch_class(const BatchEntry<T>* e, int n, int blocks, int ty, int c, bool cp, bool nt,
                           hipStream_t s);
// the auxiliary lines' E update of every instance (one block each), step sub
// of the chunk: after the H sweep, before the spectra
template <class T>
void launch_aux_e_batch(const BatchEntry<T>* e, int n, int sub, hipStream_t s);
// Step form 3 of a batch (gnor_fplain.hip): one-pass class cls (0, 1 or 2) of
// every instance (blocks: that class's blocks of all instances); the TF/SF
// corrections at the one-pass points of every instance (blocks: the sum of
// fnblk); and the lines' whole step (H and E, one block per instance), after
// the TF/SF launch and before the E/J sweeps of the metal classes
template <class T>
void launch_fplain_batch(const BatchEntry<T>* e, int n, int blocks, int ty, int cls, bool nt,
                         hipStream_t s);
template <class T>
void launch_tfsf_fix_batch(const BatchEntry<T>* e, int n, int blocks, hipStream_t s);
// the node scalars of every instance's metal sub-grid (blocks: the sum of
// snblk), before the metal class's one-pass launch
template <class T>
void launch_nodes_batch(const BatchEntry<T>* e, int n, int blocks, hipStream_t s);
// blocks of the node-scalar launch for a metal sub-grid of mn nodes
int node_blocks(const int mn[3]);
template <class T>
void launch_aux_batch(const BatchEntry<T>* e, int n, int sub, hipStream_t s);
// blocks of the TF/SF launch for a TF box [lo, hi] (the points of its shell)
int tfsf_fix_blocks(const int lo[3], const int hi[3]);
template <class T>
void launch_dft_batch(const BatchEntry<T>* e, int n, int blocks, int sub, hipStream_t s);
template <class T>
void launch_advance_batch(const BatchEntry<T>* e, int n, int64_t count, hipStream_t s);
// blocks of the class-c launch of one simulation (without the auxiliary block)
int class_blocks(const Tiling& t, int c);
int dft_blocks(const DftParams& d, const FluxParams& f);

// one tile class of a sweep (class 0 also advances the auxiliary line)
template <class T>
void launch_h_class(const Params<T>& p, const AuxParams& a, int c, hipStream_t s);
template <class T>
void launch_ej_class(const Params<T>& p, const AuxParams& a, int sub, int c, hipStream_t s);
// fused step (H, E/J in one pass; one launch per tile class) and the
// auxiliary line's step, which must follow it
template <class T>
void launch_step_class(const Params<T>& p, const AuxParams& a, int c, hipStream_t s);
void launch_aux(const AuxParams& a, int sub, hipStream_t s);
// one-pass step of tile class cls (gnor_fplain.hip; 0: no metal, at most an
// x slab; 1: no metal, a y or z slab; 2: metal, no slab, no critical points,
// its node scalars first) and, if fix, the TF/SF corrections at that class's
// points; before the line's step
template <class T>
void launch_fplain(const Params<T>& p, const AuxParams& a, int cls, bool fix, hipStream_t s);
template <class T>
void launch_step(const Params<T>& p, const AuxParams& a, int sub, hipStream_t s);
// soft plane source of total-field operation: E_x^{n+1} += f(t_{n+1}) on node
// plane k (after every E/J sweep of the step)
template <class T>
void launch_plane_source(const Params<T>& p, const AuxParams& a, int k, int sub, hipStream_t s);
template <class T>
void launch_h(const Params<T>& p, const AuxParams& a, hipStream_t s);
template <class T>
void launch_ej(const Params<T>& p, const AuxParams& a, int sub, hipStream_t s);
template <class T>
void launch_dft_stage(const DftParams& d, const FluxParams& f, const Params<T>& p, int sub,
                      hipStream_t s);
void launch_advance(int64_t* base, int64_t count, hipStream_t s);
void launch_flux_accumulate(const FluxParams& f, int* lo_ptr, int sub, hipStream_t s);
size_t flux_ptab_doubles(int nf);
template <class T>
void launch_maps(const MapParams<T>& m, int sub, hipStream_t s);
// pair chunks of the flux reduction (each within one box) and their partial sums
constexpr int kFluxChunk = 512;
inline int flux_reduce_chunks(int npairs, int npairs_box0) {
  return (npairs_box0 + kFluxChunk - 1) / kFluxChunk + (npairs - npairs_box0 + kFluxChunk - 1) / kFluxChunk;
}
void launch_flux_reduce(const double* acc, const double* pw, int npairs, int npairs_box0, int nf,
                        double* part, double* out, hipStream_t s);
template <class T>
void launch_nonfinite(const T* a, size_t n, int* flag, hipStream_t s);

// Design box inside the metal sub-grid: dn cells per axis, starting at
// sub-grid cell off; the sub-grid has mn cells per axis.
struct DesignMap {
  int dn[3], off[3], mn[3];
};
// any rho outside [0, 1] (or NaN) sets *flag
void launch_design_check(const float* rho, size_t n, int* flag, hipStream_t s);
// rho[z][y][x] of the design box -> the sub-grid weight array
void launch_design_scatter(const float* rho, const DesignMap& d, float* weight, hipStream_t s);
// n - n0 (m^-3) at the sub-grid nodes from Phi~_P^{n-1} and J~^{n-1/2}
template <class T>
void launch_density(const T* pp, const T* jx, const T* jy, const T* jz, const int mn[3], double scale,
                    double* out, hipStream_t s);
// zero `bytes` (a multiple of 4) with a kernel (graph-safe clear)
void launch_fill_zero(void* a, size_t bytes, hipStream_t s);

// The library's one static device buffer: the parameter tables of a batch
// made by gnor_batch_create_static, at most kStaticBatchMax instances.
constexpr size_t kStaticTableBytes = size_t(1) << 20;
constexpr int kStaticBatchMax = 128;
// Device address of the current device's copy (looked up once per device,
// with that device current) and the device's ordinal.
hipError_t static_table_address(int* device, void** addr);
Tiling make_tiling(int nx, int ny, int nz, int ty, int kz, int xcd);
// Classify the tiles (metal: a metal point within two cells, by the per-row
// x extents rowx of the metal points, null = no metal; CPML: slabs of np
// cells within one cell; classes 0 plain, 1 CPML, 2 metal, 3 metal + CPML)
// and fill the class counts, offsets and per-XCD counts of t; list receives
// the class lists back to back.  merge_x: tiles without metal that meet only
// an x slab go to class 0, whose two-sweep and one-pass (form 3) kernels
// update the x-slab psi of such tiles (the fused kernels of forms 1 and 2
// have no CPML in class 0: false for them).  merge_x_metal: likewise metal
// tiles that meet only an x slab go to class 2 (form 3 without critical
// points, whose one-pass metal kernel carries the x-slab psi).
// Each class lists its tiles in natural order (x fastest, then y, then z).
// tile_class receives the class of every tile (tile order x, y, z).
void classify_tiles(Tiling& t, int nx, int ny, int nz, int np, const int* rowx,
                    std::vector<int>& list, bool merge_x, bool merge_x_metal,
                    std::vector<uint8_t>& tile_class);

}  // namespace gnor

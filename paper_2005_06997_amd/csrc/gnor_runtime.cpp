// Host runtime of libgnorfdtd: the C ABI declared in include/gnor_fdtd.h.
//
// One simulation owns a caller-provided device buffer, carved into a static
// region (masks, CPML and auxiliary-line profiles, monitor descriptors,
// frequencies) and a state region (fields, currents, node scalars, CPML
// memory, auxiliary line, accumulators, step counter) that gnor_reset zeroes.
// Steps are enqueued on the bound stream, either directly or from captured
// HIP graphs of a fixed number of steps.
#include "../../include/gnor_fdtd.h"
#include "gnor_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

namespace {

constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kElementaryCharge = 1.602176634e-19;  // C
constexpr int kFieldDensity = 21;  // gnor_get_field index of n - n0
double eps0() { return 1.0 / (kMu0 * kC0 * kC0); }
double eta0() { return std::sqrt(kMu0 / eps0()); }

struct Err {
  gnor_status st;
  std::string msg;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Region planner: assigns 256-byte aligned offsets.
// Every region is followed by a 33 x 256-byte gap, so that equally sized
// field arrays (e.g. 320^3 x 4 B = 2^17 x 1000 B) do not all start on the
// same large power of two: the same cell of every array then maps to
// different HBM channels.
struct Planner {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += align_up(bytes) + kSkew;
    return o;
  }
  static constexpr size_t kSkew = 33 * 256;
};

struct Layout {
  // static region
  size_t mask = 0, rho = 0, cpml[3] = {0, 0, 0}, aux_prof = 0, omega = 0, fpw = 0, tiles = 0, tile_class = 0,
         colz = 0, map_om = 0;
  // scratch outside the state: density read-out (M doubles), the flags of
  // gnor_check_finite and of the design-density check
  size_t dens = 0, chk = 0, dflag = 0;
  size_t static_end = 0;
  // state region
  size_t state_begin = 0;
  size_t E[2][3] = {{0}}, H[2][3] = {{0}};
  size_t J[2][3] = {{0}}, PP[2] = {0, 0}, PJ[2] = {0, 0}, Q = 0;
  size_t cpP[gnor::kMaxCP][3] = {{0}}, cpQ[gnor::kMaxCP][3] = {{0}};  // critical points
  size_t psiE[3][2] = {{0}}, psiH[2][3][2] = {{{0}}};
  size_t aux = 0, phase = 0, jpart = 0, dft = 0, fstage = 0, facc = 0, ptab = 0, step = 0,
         flux_lo = 0, flag = 0, fsum = 0, fpart = 0, maps = 0, map_inc = 0;
  size_t state_end = 0;
};

}  // namespace

struct gnor_sim {
  gnor_grid_desc g{};
  gnor_material_desc mat{};
  gnor_source_desc src{};
  std::vector<double> omega;
  gnor_monitor_desc mon{};
  bool have_material = false, have_source = false, have_monitors = false, bound = false;
  std::vector<uint8_t> mask;     // full grid
  int mlo[3] = {0, 0, 0}, mn[3] = {0, 0, 0};  // metal sub-grid (with halo)
  bool any_metal = false;
  // design region [dlo, dhi) of cells with densities rho (x fastest)
  bool design = false;
  int dlo[3] = {0, 0, 0}, dhi[3] = {0, 0, 0};
  std::vector<float> rho;
  size_t N = 0, M = 0;
  int elem = 8;                  // bytes per field value
  double dt = 0;
  int n1 = 0;
  int nbx = 0, nby = 0;
  // flux plan
  int nsamp = 0, npairs = 0, npairs_box0 = 0, slots = gnor::kFluxSlots;
  std::vector<gnor::FluxSeg> fseg;
  std::vector<double> fpw;
  int tile_ty = 2, tile_kz = 8, tile_xcd = 2;    // sweep tiling (autotuned)
  gnor::Tiling tl{};                              // that tiling with its tile classes
  std::vector<int> tile_list;                     // the classes' tile lists (host copy)
  std::vector<uint8_t> tile_class;                // class of every tile (host copy)
  bool tf_shell[gnor::kClasses] = {};             // a tile of class c holds a point of the TF box's shell
  std::vector<int> rowx;                          // x extent of the metal points per (y, z) row
  // step form: 0 H and E/J sweeps, 1 one-pass fused step, 2 hybrid, 3 fused
  // plain tiles (see hybrid_fused)
  int mode = 0;
  gnor_map_desc maps{};                           // near-field / density maps (nmap = 0: off)
  std::vector<double> map_omega;
  Layout L;
  char* dev = nullptr;
  size_t dev_bytes = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // the tile classes of a sweep run concurrently: class 0 on the bound
  // stream, classes 1 and 2 on two side streams (fork / join by events)
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
  bool concurrent = true;  // false: the class launches one after another on the bound stream
  int64_t step = 0;
  int graph_chunk = 64;
  hipGraphExec_t graph = nullptr;
  int graph_steps = 0;
  // non-finite watchdog of gnor_run: E is scanned after every chunk of steps
  // (flag in the state region, sticky until reset or load); the host reads
  // a chunk's flag while the next chunk runs, on a stream of its own
  bool watchdog = true;
  hipStream_t wstream = nullptr;
  hipEvent_t wev[2] = {nullptr, nullptr};
  int wslot = 0;
  bool wpending = false;  // the last scanned chunk's flag has not been read yet
  int64_t wsince = 0;     // steps enqueued since the last scan
  std::string last_error;
};

namespace {

gnor_status fail(gnor_sim* s, gnor_status st, const std::string& m) {
  if (s) s->last_error = m;
  return st;
}

#define HIPCHECK(sim, call)                                                              \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(sim, GNOR_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// CPML coefficients at a depth (cells) into a layer of L cells.
void pml_coeffs(const gnor_grid_desc& g, double dt, double depth, int L, double& b, double& a,
                double& kinv) {
  b = 1.0; a = 0.0; kinv = 1.0;
  if (L <= 0 || depth <= 0.0) return;
  const double m = g.pml_order;
  const double smax = g.pml_sigma_scale * (m + 1.0) / (eta0() * g.dx * std::sqrt(g.eps_background));
  const double u = depth / L;
  const double sigma = smax * std::pow(u, m);
  const double kappa = 1.0 + (g.pml_kappa_max - 1.0) * std::pow(u, m);
  const double alpha = g.pml_alpha_max * (1.0 - u);
  b = std::exp(-(sigma / kappa + alpha) * dt / eps0());
  a = sigma > 0.0 ? sigma * (b - 1.0) / (kappa * (sigma + kappa * alpha)) : 0.0;
  kinv = 1.0 / kappa;
}
double layer_depth(double x, int n, int L) {
  double d = 0.0;
  if (x < L) d = L - x;
  if (x > (n - 1 - L)) d = x - (n - 1 - L);
  return d;
}

void plan_flux(gnor_sim* s) {
  // Face segments of the two monitor boxes.  A segment is a rectangle of
  // (E, H) sample pairs on one face; its inner index runs along x whenever x
  // is tangential (coalesced staging loads).  Pair weights: outward sign x
  // dx^2 x trapezoid weight along the face direction in which the samples sit
  // on integer positions; E_b H_c pairs count +, E_c H_b pairs count -.
  s->fseg.clear(); s->fpw.clear();
  s->nsamp = s->npairs = s->npairs_box0 = 0;
  if (!s->have_monitors || !s->mon.flux_enabled || s->mon.nfreq <= 0) return;
  const double h2 = s->g.dx * s->g.dx;
  int first = 0;
  for (int box = 0; box < 2; ++box) {
    const int32_t* lo = box == 0 ? s->mon.abs_lo : s->mon.sca_lo;
    const int32_t* hi = box == 0 ? s->mon.abs_hi : s->mon.sca_hi;
    for (int a = 0; a < 3; ++a)
      for (int side = -1; side <= 1; side += 2) {
        const int p = side < 0 ? lo[a] : hi[a];
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        for (int kind = 0; kind < 2; ++kind) {
          // kind 0: E_b at half-integer b, integer c, with H_c;
          // kind 1: E_c at integer b, half-integer c, with H_b
          gnor::FluxSeg g{};
          g.a = a; g.p = p;
          g.ecomp = kind == 0 ? b : c;
          g.hcomp = kind == 0 ? c : b;
          const int nb = kind == 0 ? hi[b] - lo[b] : hi[b] - lo[b] + 1;
          const int nc = kind == 0 ? hi[c] - lo[c] + 1 : hi[c] - lo[c];
          const bool inner_c = (c == 0);
          g.in_axis = inner_c ? c : b;
          g.out_axis = inner_c ? b : c;
          g.in_lo = inner_c ? lo[c] : lo[b];
          g.out_lo = inner_c ? lo[b] : lo[c];
          g.n_in = inner_c ? nc : nb;
          const int n_out = inner_c ? nb : nc;
          g.first = first;
          g.count = nb * nc;
          for (int r = 0; r < g.count; ++r) {
            const int ii = g.in_lo + r % g.n_in, oo = g.out_lo + r / g.n_in;
            const int pb = inner_c ? oo : ii, pc = inner_c ? ii : oo;  // b and c coordinates
            double wt;
            if (kind == 0) wt = (pc == lo[c] || pc == hi[c]) ? 0.5 : 1.0;
            else wt = (pb == lo[b] || pb == hi[b]) ? 0.5 : 1.0;
            s->fpw.push_back((kind == 0 ? 1.0 : -1.0) * side * h2 * wt);
          }
          (void)n_out;
          first += g.count;
          s->fseg.push_back(g);
        }
      }
    if (box == 0) s->npairs_box0 = first;
  }
  s->npairs = first;
  s->nsamp = 2 * first;
}

// points of the map plane
size_t map_plane(const gnor_sim* s) {
  const int n[3] = {s->g.nx, s->g.ny, s->g.nz};
  const int a = s->maps.axis;
  return (size_t)n[a == 0 ? 1 : 0] * n[a == 2 ? 1 : 2];
}

void plan_layout(gnor_sim* s) {
  Layout& L = s->L;
  L = Layout();
  Planner P;
  const size_t N = s->N, M = s->M;
  const int e = s->elem;
  const int np = s->g.npml;
  L.mask = P.take(M);
  L.colz = P.take((size_t)2 * s->mn[0] * s->mn[1] * 4);
  L.rho = P.take(M * sizeof(float));
  for (int a = 0; a < 3; ++a) L.cpml[a] = P.take((size_t)6 * 2 * np * e + 8);
  L.aux_prof = P.take((size_t)6 * s->n1 * 8);
  L.omega = P.take((size_t)std::max(1, s->mon.nfreq) * 8);
  L.fpw = P.take((size_t)s->npairs * 8 + 8);
  // tile lists: room for the finest tiling (ty = 2, kz = 1)
  L.tiles = P.take((size_t)s->nbx * ((s->g.ny + 1) / 2) * s->g.nz * 4 + 4);
  L.tile_class = P.take((size_t)s->nbx * ((s->g.ny + 1) / 2) * s->g.nz + 4);
  L.map_om = P.take((size_t)std::max(1, s->maps.nmap) * 8);
  L.dens = P.take(M * 8);
  L.chk = P.take(4);
  L.dflag = P.take(4);
  L.static_end = P.off;
  L.state_begin = P.off;
  for (int pp = 0; pp < 2; ++pp)
    for (int c = 0; c < 3; ++c) L.E[pp][c] = P.take(N * e);
  // H^{n-1/2} in H[n mod 2]; a step writes H^{n+1/2} into the other buffer
  for (int pp = 0; pp < 2; ++pp)
    for (int c = 0; c < 3; ++c) L.H[pp][c] = P.take(N * e);
  for (int pp = 0; pp < 2; ++pp) {
    for (int c = 0; c < 3; ++c) L.J[pp][c] = P.take(M * e);
    L.PP[pp] = P.take(M * e);
    L.PJ[pp] = P.take(M * e);
  }
  L.Q = P.take(M * e);
  for (int u = 0; u < s->mat.ncp; ++u)
    for (int c = 0; c < 3; ++c) {
      L.cpP[u][c] = P.take(M * e);
      L.cpQ[u][c] = P.take(M * e);
    }
  const size_t nx = s->g.nx, ny = s->g.ny, nz = s->g.nz;
  const size_t slab[3] = {nz * ny * 2 * np, nz * 2 * np * nx, 2 * np * ny * nx};
  for (int a = 0; a < 3; ++a)
    for (int t = 0; t < 2; ++t) {
      L.psiE[a][t] = P.take(slab[a] * e + 8);
      for (int pp = 0; pp < 2; ++pp) L.psiH[pp][a][t] = P.take(slab[a] * e + 8);
    }
  L.aux = P.take((size_t)4 * s->n1 * 8);
  L.phase = P.take((size_t)4 * std::max(1, s->mon.nfreq) * 8);
  // partial sums per (plane, tile, wavefront): at most nbx * (ny + 8) per plane
  L.jpart = P.take(nz * (size_t)s->nbx * (ny + 8) * 8);
  L.dft = P.take((size_t)4 * nz * std::max(1, s->mon.nfreq) * 8);
  L.fstage = P.take((size_t)s->slots * s->nsamp * 8 + 8);
  L.facc = P.take((size_t)2 * std::max(1, s->mon.nfreq) * s->nsamp * 8 + 8);
  L.ptab = P.take(gnor::flux_ptab_doubles(std::max(1, s->mon.nfreq)) * 8);
  L.fsum = P.take((size_t)2 * std::max(1, s->mon.nfreq) * 8);
  L.fpart = P.take((size_t)gnor::flux_reduce_chunks(s->npairs, s->npairs_box0) * std::max(1, s->mon.nfreq) * 8 + 8);
  L.maps = P.take((size_t)8 * s->maps.nmap * map_plane(s) * 8 + 8);
  L.map_inc = P.take((size_t)2 * std::max(1, s->maps.nmap) * 8);
  L.step = P.take(8);
  L.flux_lo = P.take(4);
  L.flag = P.take(4);
  L.state_end = P.off;
}

template <class T>
T* ptr(gnor_sim* s, size_t off) {
  return reinterpret_cast<T*>(s->dev + off);
}

template <class T>
gnor::Params<T> make_params(gnor_sim* s, int parity) {
  gnor::Params<T> p{};
  const gnor_grid_desc& g = s->g;
  p.nx = g.nx; p.ny = g.ny; p.nz = g.nz;
  const double S = g.courant;
  p.S = (T)S;
  p.SE = (T)(S / g.eps_background);
  const bool sub = g.eps_substrate > 0.0;
  p.sub_k = sub ? g.substrate_k : g.nz + 1;
  p.se_avg = (T)(sub ? S / (0.5 * (g.eps_background + g.eps_substrate)) : S / g.eps_background);
  p.se_sub = (T)(sub ? S / g.eps_substrate : S / g.eps_background);
  const int a = parity & 1, b = a ^ 1;
  for (int c = 0; c < 3; ++c) {
    p.E[c] = ptr<T>(s, s->L.E[a][c]);
    p.O[c] = ptr<T>(s, s->L.E[b][c]);
    p.Hi[c] = ptr<T>(s, s->L.H[a][c]);
    p.H[c] = ptr<T>(s, s->L.H[b][c]);
    p.Ji[c] = ptr<T>(s, s->L.J[a][c]);
    p.Jo[c] = ptr<T>(s, s->L.J[b][c]);
  }
  p.PPi = ptr<T>(s, s->L.PP[a]); p.PPo = ptr<T>(s, s->L.PP[b]);
  p.PJi = ptr<T>(s, s->L.PJ[a]); p.PJo = ptr<T>(s, s->L.PJ[b]);
  p.Q = ptr<T>(s, s->L.Q);
  p.any_metal = s->any_metal ? 1 : 0;
  p.stream_stores = 9.0 * (double)s->N * sizeof(T) > gnor::kStreamStoreBytes ? 1 : 0;
  for (int d = 0; d < 3; ++d) { p.mlo[d] = s->mlo[d]; p.mn[d] = s->mn[d]; }
  p.mask = ptr<uint8_t>(s, s->L.mask);
  p.colz = ptr<int>(s, s->L.colz);
  p.rho = s->design ? ptr<float>(s, s->L.rho) : nullptr;
  // metal coefficients (Sec. III), scaled by eps0 and dx^2
  const double dt = s->dt, dx = g.dx;
  const double gam = s->mat.gamma, wp = s->mat.wp, beta = s->mat.beta, D = s->mat.diffusion;
  const double Dd = gam / (2 * dt) + 1.0 / (dt * dt);
  const double D2 = (gam / (2 * dt) - 1.0 / (dt * dt)) / Dd;
  const double d3 = wp * wp / (4.0 * Dd);          // D3 / eps0
  const double agam = gam * dt / (1.0 + gam * dt / 2.0);  // 1 + D2 without cancellation
  const double eta = beta * beta + D * gam;
  const double g1 = eta / Dd / (dx * dx);
  const double g2 = D / (2.0 * dt * Dd) / (dx * dx);
  const double ei = s->mat.eps_inf;
  // critical points, Eq. (critpointupdate) divided by eps0, as increments:
  // Q = (P_CP^{n+1} - P_CP^n) / eps0 = a P + (1 - b) Q + c4 (2 E^n)
  //   - c5 (E^n - E^{n-1}) + c3 (E^{n+1} - E^n), with a = C_1p + C_2p - 1 and
  // b = 1 + C_2p (so that C_3p + C_4p + C_5p = 2 C_4p); the sin(phi) part of
  // C_3p and C_5p is A Omega sin(phi) / (dt C_p)
  double c3sum = 0.0;
  p.ncp = s->mat.ncp;
  for (int u = 0; u < s->mat.ncp; ++u) {
    const double A = s->mat.cp_A[u], Om = s->mat.cp_Omega[u], Ga = s->mat.cp_Gamma[u];
    const double ph = s->mat.cp_phi[u];
    const double w2 = Om * Om + Ga * Ga;
    const double Cp = Ga / dt + 1.0 / (dt * dt) + w2 / 4.0;
    const double c4 = A * Om * (Om * std::cos(ph) - Ga * std::sin(ph)) / Cp;
    const double sn = A * Om * std::sin(ph) / (dt * Cp);
    p.cpa[u] = (T)(-w2 / Cp);
    p.cpb[u] = (T)(2.0 * Ga / (dt * Cp));
    p.cp3[u] = (T)(c4 / 2.0 - sn);
    p.cp4[u] = (T)c4;
    p.cp5[u] = (T)(c4 / 2.0 + sn);
    c3sum += c4 / 2.0 - sn;
    for (int c = 0; c < 3; ++c) {
      p.cpP[u][c] = ptr<T>(s, s->L.cpP[u][c]);
      p.cpQ[u][c] = ptr<T>(s, s->L.cpQ[u][c]);
    }
  }
  p.c3sum = (T)c3sum;
  const double inv = 1.0 / (ei + d3 + c3sum);
  p.eps_inf = (T)ei; p.d3 = (T)d3; p.agam = (T)agam; p.D2 = (T)D2; p.g1 = (T)g1; p.g2 = (T)g2;
  p.ebd = (T)(ei - g.eps_background);
  p.cS = (T)(S * inv); p.c3 = (T)(3.0 * d3 * inv); p.c1 = (T)(d3 * inv); p.cJ = (T)(D2 * inv);
  p.cG = (T)inv;
  const int np = g.npml;
  const int nn[3] = {g.nx, g.ny, g.nz};
  for (int ax = 0; ax < 3; ++ax) {
    for (int t = 0; t < 2; ++t) {
      p.psiE[ax][t] = ptr<T>(s, s->L.psiE[ax][t]);
      p.psiHi[ax][t] = ptr<T>(s, s->L.psiH[a][ax][t]);
      p.psiH[ax][t] = ptr<T>(s, s->L.psiH[b][ax][t]);
    }
    gnor::CpmlAxis<T>& c = p.cp[ax];
    c.n = nn[ax]; c.np = np;
    T* base = ptr<T>(s, s->L.cpml[ax]);
    c.be = base; c.ae = base + 2 * np; c.ke = base + 4 * np;
    c.bh = base + 6 * np; c.ah = base + 8 * np; c.kh = base + 10 * np;
  }
  p.tfsf = g.total_field ? 0 : 1;
  p.lra_pml = g.total_field ? 1 : 0;
  for (int d = 0; d < 3; ++d) { p.tf_lo[d] = g.tf_lo[d]; p.tf_hi[d] = g.tf_hi[d]; }
  double* aux = ptr<double>(s, s->L.aux);
  p.e1 = aux; p.h1 = aux + s->n1;
  p.jpart = ptr<double>(s, s->L.jpart);
  p.tl = s->tl;
  p.tiles = ptr<int>(s, s->L.tiles);
  p.tile_class = ptr<uint8_t>(s, s->L.tile_class);
  p.step_base = ptr<int64_t>(s, s->L.step);
  return p;
}

gnor::AuxParams make_aux(gnor_sim* s) {
  gnor::AuxParams a{};
  a.n1 = s->n1;
  a.S = s->g.courant;
  a.SE = s->g.courant / s->g.eps_background;
  const bool sub = s->g.eps_substrate > 0.0;
  a.sub_k = sub ? s->g.substrate_k : s->g.nz + 1;
  a.se_avg = sub ? s->g.courant / (0.5 * (s->g.eps_background + s->g.eps_substrate)) : a.SE;
  a.se_sub = sub ? s->g.courant / s->g.eps_substrate : a.SE;
  double* st = ptr<double>(s, s->L.aux);
  a.e1 = st; a.h1 = st + s->n1; a.pe = st + 2 * s->n1; a.ph = st + 3 * s->n1;
  const double* pr = ptr<double>(s, s->L.aux_prof);
  a.be = pr; a.ae = pr + s->n1; a.ke = pr + 2 * s->n1;
  a.bh = pr + 3 * s->n1; a.ah = pr + 4 * s->n1; a.kh = pr + 5 * s->n1;
  a.src_kind = s->have_source ? s->src.kind : 0;
  a.src_cell = s->g.total_field ? s->g.source_k + gnor::kAuxOff : gnor::kAuxSrc;
  a.e0 = s->src.e0; a.omega_c = s->src.omega_c; a.tau = s->src.tau; a.t0 = s->src.t0;
  a.omega_max = s->src.omega_max; a.dt = s->dt;
  a.nf = s->mon.nfreq;
  a.omega = ptr<double>(s, s->L.omega);
  a.phase = ptr<double>(s, s->L.phase);
  a.every = std::max(1, s->mon.dft_every);
  a.step_base = ptr<int64_t>(s, s->L.step);
  return a;
}

gnor::DftParams make_dft(gnor_sim* s) {
  gnor::DftParams d{};
  d.nz = s->g.nz; d.nf = s->mon.nfreq;
  d.kz0 = s->any_metal ? s->mlo[2] : 0;
  d.kz1 = s->any_metal ? s->mlo[2] + s->mn[2] : 0;
  const gnor::Tiling tl = gnor::make_tiling(s->g.nx, s->g.ny, s->g.nz, s->tile_ty, s->tile_kz, s->tile_xcd);
  d.nbxy = tl.nbx * tl.nby * tl.ty;
  d.jpart = ptr<double>(s, s->L.jpart);
  d.phase = ptr<double>(s, s->L.phase);
  d.every = std::max(1, s->mon.dft_every);
  d.wdt = s->dt * d.every;
  d.e1 = ptr<double>(s, s->L.aux);
  const size_t nzf = (size_t)s->g.nz * std::max(1, s->mon.nfreq);
  double* base = ptr<double>(s, s->L.dft);
  d.a_re = base; d.a_im = base + nzf; d.b_re = base + 2 * nzf; d.b_im = base + 3 * nzf;
  d.step_base = ptr<int64_t>(s, s->L.step);
  return d;
}

gnor::FluxParams make_flux(gnor_sim* s) {
  gnor::FluxParams f{};
  f.npairs = s->npairs; f.nsamp = s->nsamp; f.nf = s->mon.nfreq;
  f.nseg = (int)s->fseg.size();
  for (int q = 0; q < f.nseg; ++q) f.seg[q] = s->fseg[q];
  f.nx = s->g.nx; f.ny = s->g.ny;
  // the rows (y, z) that the x-normal faces cover, and the other faces' pairs
  int j0 = INT_MAX, j1 = INT_MIN, k0 = INT_MAX, k1 = INT_MIN;
  for (int q = 0; q < f.nseg; ++q) {
    const gnor::FluxSeg& g = f.seg[q];
    if (g.a != 0) { f.nrest += g.count; continue; }  // x-normal faces run y inside, z outside
    j0 = std::min(j0, g.in_lo); j1 = std::max(j1, g.in_lo + g.n_in);
    k0 = std::min(k0, g.out_lo); k1 = std::max(k1, g.out_lo + g.count / g.n_in);
  }
  if (j0 < j1) { f.xj0 = j0; f.xnj = j1 - j0; f.xk0 = k0; f.xnrow = (j1 - j0) * (k1 - k0); }
  f.stage = ptr<double>(s, s->L.fstage);
  f.acc = ptr<double>(s, s->L.facc);
  f.omega = ptr<double>(s, s->L.omega);
  f.ptab = ptr<double>(s, s->L.ptab);
  f.dt = s->dt; f.wdt = s->dt;
  f.step_base = ptr<int64_t>(s, s->L.step);
  return f;
}

template <class T>
gnor::MapParams<T> make_maps(gnor_sim* s, int parity) {
  gnor::MapParams<T> m{};
  const int n[3] = {s->g.nx, s->g.ny, s->g.nz};
  m.axis = s->maps.axis; m.index = s->maps.index; m.nmap = s->maps.nmap;
  m.every = std::max(1, s->maps.every);
  m.nu = n[m.axis == 0 ? 1 : 0]; m.nv = n[m.axis == 2 ? 1 : 2];
  m.nx = s->g.nx; m.ny = s->g.ny;
  m.omega = ptr<double>(s, s->L.map_om);
  m.acc = ptr<double>(s, s->L.maps);
  m.inc = ptr<double>(s, s->L.map_inc);
  m.dt = s->dt;
  m.nscale = eps0() / (s->g.dx * kElementaryCharge);  // Phi~_P = dx div P / eps0; n - n0 = div P / e
  for (int d = 0; d < 3; ++d) { m.mlo[d] = s->mlo[d]; m.mn[d] = s->mn[d]; }
  const int b = (parity & 1) ^ 1;
  for (int c = 0; c < 3; ++c) m.E[c] = ptr<T>(s, s->L.E[b][c]);
  m.PP = s->any_metal ? ptr<T>(s, s->L.PP[b]) : nullptr;
  m.e1 = ptr<double>(s, s->L.aux);
  m.norm_k = s->mon.norm_k;
  m.step_base = ptr<int64_t>(s, s->L.step);
  return m;
}

// Enqueue one step; `sub` is the step's offset from the device step counter.
// The four tile-class launches of a sweep, concurrently: classes 0 and 3 on
// st, classes 1 and 2 on the side streams, joined back into st.  (Also inside a
// graph capture of st: the side streams join the capture through the fork
// event.)  launch(c, stream) enqueues class c.
// Fork/join events order the class streams of one device: no timing and no
// system-scope fence (the kernels' own completion makes their writes visible
// on the device; only the host reads results, after a stream synchronize).
constexpr unsigned kJoinEventFlags = hipEventDisableTiming | hipEventDisableSystemFence;

// c3_side: class 3 after class 1 on the first side stream (the first half of
// form 3, whose one-pass class-0 launches keep the bound stream busy longest).
// active(c): whether launch(c) launches anything; with at most one such
// class the launches stay on the bound stream, without the fork and join
// (their events cost about 10 us of idle GPU per join in a replayed graph:
// form 3's second half has only class 3's E/J sweep).
template <class F, class A>
void enqueue_classes(gnor_sim* s, hipStream_t st, F launch, A active, bool c3_side = false) {
  int n_active = 0;
  for (int c = 0; c < gnor::kClasses; ++c) n_active += active(c) ? 1 : 0;
  if (!s->concurrent || n_active <= 1) {
    for (int c = 0; c < gnor::kClasses; ++c)
      if (active(c)) launch(c, st);
    return;
  }
  (void)hipEventRecord(s->ev_fork, st);
  for (int q = 0; q < 2; ++q) (void)hipStreamWaitEvent(s->side[q], s->ev_fork, 0);
  auto go = [&](int c, hipStream_t q) {
    if (active(c)) launch(c, q);
  };
  go(0, st);
  if (!c3_side) go(3, st);  // metal + CPML: small grids (usually empty otherwise)
  go(1, s->side[0]);
  if (c3_side) go(3, s->side[0]);
  go(2, s->side[1]);
  for (int q = 0; q < 2; ++q) {
    (void)hipEventRecord(s->ev_join[q], s->side[q]);
    (void)hipStreamWaitEvent(st, s->ev_join[q], 0);
  }
}

// Hybrid step form: the tile classes without CPML (plain, and metal unless
// the material has critical points, which the fused kernel lacks) run the
// one-pass fused step; the CPML classes run the two sweeps.  Order:
//   1. fused classes and H sweeps of the others, concurrently (inputs E^n,
//      H^{n-1/2} are never written in a step; the fused kernels evaluate
//      H_inc^{n+1/2} from the line and store the node scalars Q their
//      two-sweep neighbours read);
//   2. the auxiliary line (after every reader of E_inc^n);
//   3. E/J sweeps of the two-sweep classes (they read H^{n+1/2} of fused
//      neighbours and H_inc^{n+1/2}).
// Form 3: the tiles without metal, class 0 (at most an x slab within one
// cell) and class 1 (a y or z slab), and, without critical points, the metal
// tiles without a slab (class 2, after a launch that writes the node
// scalars) take the one-pass kernels of gnor_fplain.hip, each followed on its
// stream by its TF/SF launch where its tiles meet the shell of the TF box;
// the metal tiles in a slab (class 3) take the two sweeps.
bool hybrid_fused(const gnor_sim* s, int c) {
  if (s->mode == 3) return c <= 1 || (c == 2 && s->mat.ncp == 0);
  return c == 0 || (c == 2 && s->mat.ncp == 0);
}

// First half of a step: the H sweep (mode 0), the fused step (mode 1), or
// phase 1 of the hybrid form.
template <class T>
void enqueue_first(gnor_sim* s, const gnor::Params<T>& p, const gnor::AuxParams& a, int mode,
                   hipStream_t st) {
  // classes with tiles; in the two sweeps class 0's launch also carries the
  // line's block
  auto tiles = [&](int c) { return s->tl.cn[c] > 0; };
  auto swept = [&](int c) { return c == 0 || s->tl.cn[c] > 0; };
  if (mode == 1) {
    enqueue_classes(s, st, [&](int c, hipStream_t q) { gnor::launch_step_class<T>(p, a, c, q); }, tiles);
  } else if (mode == 2 || mode == 3) {
    enqueue_classes(s, st, [&](int c, hipStream_t q) {
      if (!hybrid_fused(s, c)) gnor::launch_h_class<T>(p, a, c, q);
      else if (mode == 3) gnor::launch_fplain<T>(p, a, c, s->tf_shell[c], q);
      else gnor::launch_step_class<T>(p, a, c, q);
    }, tiles, mode == 3);
  } else {
    enqueue_classes(s, st, [&](int c, hipStream_t q) { gnor::launch_h_class<T>(p, a, c, q); }, swept);
  }
}
// Second half: the E/J sweep (mode 0), the auxiliary line (mode 1), or the
// line and then the E/J sweeps of the two-sweep classes (mode 2).
template <class T>
void enqueue_second(gnor_sim* s, const gnor::Params<T>& p, const gnor::AuxParams& a, int sub, int mode,
                    hipStream_t st) {
  if (mode == 1) {
    gnor::launch_aux(a, sub, st);
  } else if (mode == 2 || mode == 3) {
    gnor::launch_aux(a, sub, st);
    enqueue_classes(s, st, [&](int c, hipStream_t q) { gnor::launch_ej_class<T>(p, a, sub, c, q); },
                    [&](int c) { return !hybrid_fused(s, c) && s->tl.cn[c] > 0; });
  } else {
    enqueue_classes(s, st, [&](int c, hipStream_t q) { gnor::launch_ej_class<T>(p, a, sub, c, q); },
                    [&](int c) { return c == 0 || s->tl.cn[c] > 0; });
  }
}

template <class T>
void enqueue_step(gnor_sim* s, int parity, int sub, int mode, hipStream_t st) {
  const gnor::Params<T> p = make_params<T>(s, parity);
  const gnor::AuxParams a = make_aux(s);
  enqueue_first<T>(s, p, a, mode, st);
  enqueue_second<T>(s, p, a, sub, mode, st);
  if (s->g.total_field) gnor::launch_plane_source<T>(p, a, s->g.source_k, sub, st);
  if (s->mon.nfreq > 0) gnor::launch_dft_stage<T>(make_dft(s), make_flux(s), p, sub, st);
  if (s->maps.nmap > 0) gnor::launch_maps<T>(make_maps<T>(s, parity), sub, st);
}

void enqueue_flux_acc(gnor_sim* s, int sub, hipStream_t st) {
  gnor::launch_flux_accumulate(make_flux(s), ptr<int>(s, s->L.flux_lo), sub, st);
}

// mode: the step form (the sim's setting; the adjoint's forward recompute
// uses the two sweeps, whose stored Q it needs everywhere)
void enqueue_steps_eager(gnor_sim* s, int64_t n0, int64_t count, hipStream_t st, int mode) {
  // steps n0 .. n0+count-1; the device counter holds n0 on entry
  for (int64_t q = 0; q < count; ++q) {
    const int64_t n = n0 + q;
    const int sub = (int)q;
    if (s->g.precision == GNOR_FP32) enqueue_step<float>(s, (int)(n & 1), sub, mode, st);
    else enqueue_step<double>(s, (int)(n & 1), sub, mode, st);
    if (s->nsamp > 0 && (n % s->slots) == s->slots - 1) enqueue_flux_acc(s, sub, st);
  }
  gnor::launch_advance(ptr<int64_t>(s, s->L.step), count, st);
}

void drop_graph(gnor_sim* s) {
  if (s->graph) (void)hipGraphExecDestroy(s->graph);
  s->graph = nullptr;
  s->graph_steps = 0;
}

gnor_status build_graph(gnor_sim* s, int steps) {
  drop_graph(s);
  hipGraph_t gr = nullptr;
  HIPCHECK(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
  // the chunk always starts at an even step aligned to the flux staging depth
  enqueue_steps_eager(s, 0, steps, s->stream, s->mode);
  HIPCHECK(s, hipStreamEndCapture(s->stream, &gr));
  hipError_t e = hipGraphInstantiate(&s->graph, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e != hipSuccess) {
    s->graph = nullptr;
    return fail(s, GNOR_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  s->graph_steps = steps;
  return GNOR_OK;
}

int chunk_alignment(const gnor_sim* s) {
  return s->nsamp > 0 ? std::max(2, s->slots) : 2;  // slots is even
}

gnor_status check_ready(gnor_sim* s) {
  if (!s) return GNOR_E_INVALID_ARG;
  if (!s->bound) return fail(s, GNOR_E_STATE, "gnor_bind_memory has not been called");
  return GNOR_OK;
}

// Per-cell weight of the metal's wp^2, beta^2 and D on the sub-grid: rho in
// the design region, 1 elsewhere.
gnor_status upload_rho(gnor_sim* s) {
  std::vector<float> r(s->M, 1.0f);
  const int dn[3] = {s->dhi[0] - s->dlo[0], s->dhi[1] - s->dlo[1], s->dhi[2] - s->dlo[2]};
  for (int z = 0; z < dn[2]; ++z)
    for (int y = 0; y < dn[1]; ++y)
      for (int x = 0; x < dn[0]; ++x) {
        const int lx = x + s->dlo[0] - s->mlo[0], ly = y + s->dlo[1] - s->mlo[1],
                  lz = z + s->dlo[2] - s->mlo[2];
        r[((size_t)lz * s->mn[1] + ly) * s->mn[0] + lx] = s->rho[((size_t)z * dn[1] + y) * dn[0] + x];
      }
  HIPCHECK(s, hipMemcpy(s->dev + s->L.rho, r.data(), r.size() * 4, hipMemcpyHostToDevice));
  return GNOR_OK;
}

// Do the tiles that meet only an x slab join class 0?  Yes for the step forms
// whose class-0 kernels carry the x-slab CPML (the two-sweep plain kernels and
// the one-pass plain kernel of form 3), no for the fused kernel of forms 1, 2.
bool merge_x_slabs(int mode) { return mode == 0 || mode == 3; }
// Do the metal tiles that meet only an x slab join class 2?  Yes where that
// class takes the one-pass metal kernel, which carries the x-slab CPML: form
// 3 without critical points.
bool merge_x_metal(const gnor_sim* s, int mode) { return mode == 3 && s->mat.ncp == 0; }

// Tile classes of the current tiling and step form; uploaded when the memory
// is bound (after the stream's queued steps, which read the old lists).
gnor_status plan_tiles(gnor_sim* s) {
  const gnor_grid_desc& g = s->g;
  s->tl = gnor::make_tiling(g.nx, g.ny, g.nz, s->tile_ty, s->tile_kz, s->tile_xcd);
  if (s->any_metal && s->rowx.empty()) {
    // x extent of the metal points of every (y, z) row
    s->rowx.assign((size_t)2 * g.ny * g.nz, 0);
    for (size_t r = 0; r < (size_t)g.ny * g.nz; ++r) {
      const uint8_t* row = s->mask.data() + r * g.nx;
      int lo = 1, hi = 0;
      for (int x = 0; x < g.nx; ++x)
        if (row[x]) {
          if (lo > hi) lo = x;
          hi = x;
        }
      s->rowx[2 * r] = lo;
      s->rowx[2 * r + 1] = hi;
    }
  }
  // x-slab tiles join the plain class in forms 0 and 3 (merge_x_slabs), and
  // the metal class in form 3 without critical points (merge_x_metal)
  gnor::classify_tiles(s->tl, g.nx, g.ny, g.nz, g.npml, s->any_metal ? s->rowx.data() : nullptr,
                       s->tile_list, merge_x_slabs(s->mode), merge_x_metal(s, s->mode), s->tile_class);
  // Which classes hold points of the shell of the TF box ([lo-1, hi+1]
  // without [lo+1, hi-1]), where the one-pass kernels need their TF/SF
  // launch: a tile does iff it meets the widened box and does not lie inside
  // the inner one (the shell is two cells thick, so a tile, a box of
  // consecutive cells, that reaches from the inner box to beyond it meets it)
  for (int c = 0; c < gnor::kClasses; ++c) s->tf_shell[c] = false;
  if (!g.total_field) {
    const gnor::Tiling& t = s->tl;
    for (size_t tile = 0; tile < s->tile_class.size(); ++tile) {
      const int bx = (int)(tile % t.nbx), by = (int)((tile / t.nbx) % t.nby), bz = (int)(tile / ((size_t)t.nbx * t.nby));
      const int a0[3] = {bx * gnor::kBX, by * t.ty, bz * t.kz};
      const int a1[3] = {std::min(g.nx, a0[0] + gnor::kBX) - 1, std::min(g.ny, a0[1] + t.ty) - 1,
                         std::min(g.nz, a0[2] + t.kz) - 1};
      bool meets = true, inside = true;
      for (int d = 0; d < 3; ++d) {
        meets = meets && a1[d] >= g.tf_lo[d] - 1 && a0[d] <= g.tf_hi[d] + 1;
        inside = inside && a0[d] >= g.tf_lo[d] + 1 && a1[d] <= g.tf_hi[d] - 1;
      }
      if (meets && !inside) s->tf_shell[s->tile_class[tile]] = true;
    }
  }
  if (s->bound && !s->tile_list.empty()) {
    HIPCHECK(s, hipStreamSynchronize(s->stream));
    HIPCHECK(s, hipMemcpy(s->dev + s->L.tiles, s->tile_list.data(), s->tile_list.size() * 4,
                          hipMemcpyHostToDevice));
    HIPCHECK(s, hipMemcpy(s->dev + s->L.tile_class, s->tile_class.data(), s->tile_class.size(),
                          hipMemcpyHostToDevice));
  }
  return GNOR_OK;
}

// Change the step form; the class lists depend on it (see plan_tiles).
gnor_status set_mode(gnor_sim* s, int mode) {
  if (mode == s->mode) return GNOR_OK;
  const bool replan = merge_x_slabs(mode) != merge_x_slabs(s->mode) ||
                      merge_x_metal(s, mode) != merge_x_metal(s, s->mode);
  s->mode = mode;
  drop_graph(s);
  return replan ? plan_tiles(s) : GNOR_OK;
}

gnor_status upload_static(gnor_sim* s) {
  const gnor_grid_desc& g = s->g;
  // metal sub-grid mask
  std::vector<uint8_t> sub(s->M, 0);
  for (int z = 0; z < s->mn[2]; ++z)
    for (int y = 0; y < s->mn[1]; ++y)
      for (int x = 0; x < s->mn[0]; ++x) {
        const size_t gi = ((size_t)(z + s->mlo[2]) * g.ny + (y + s->mlo[1])) * g.nx + (x + s->mlo[0]);
        sub[((size_t)z * s->mn[1] + y) * s->mn[0] + x] = s->any_metal ? s->mask[gi] : 0;
      }
  HIPCHECK(s, hipMemcpy(s->dev + s->L.mask, sub.data(), s->M, hipMemcpyHostToDevice));
  // per sub-grid column, the first and last plane of nodes that touch a metal
  // edge (E_a point with bit a set); node scalars elsewhere stay zero
  {
    const int m0 = s->mn[0], m1 = s->mn[1], m2 = s->mn[2];
    std::vector<int> colz((size_t)2 * m0 * m1);
    auto at = [&](int x, int y, int z) -> unsigned {
      if (x < 0 || y < 0 || z < 0) return 0u;
      return sub[((size_t)z * m1 + y) * m0 + x];
    };
    for (int y = 0; y < m1; ++y)
      for (int x = 0; x < m0; ++x) {
        int lo = 1, hi = 0;
        for (int z = 0; z < m2; ++z) {
          const bool act = at(x, y, z) != 0u || (at(x - 1, y, z) & 1u) || (at(x, y - 1, z) & 2u) ||
                           (at(x, y, z - 1) & 4u);
          if (act) {
            if (lo > hi) lo = z;
            hi = z;
          }
        }
        colz[2 * ((size_t)y * m0 + x)] = lo;
        colz[2 * ((size_t)y * m0 + x) + 1] = hi;
      }
    HIPCHECK(s, hipMemcpy(s->dev + s->L.colz, colz.data(), colz.size() * 4, hipMemcpyHostToDevice));
  }
  if (s->design) {
    const gnor_status st = upload_rho(s);
    if (st != GNOR_OK) return st;
  }
  // CPML profiles per axis: be, ae, ke, bh, ah, kh over the 2 npml slab cells
  const int np = g.npml;
  const int nn[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < 3; ++a) {
    std::vector<double> pr((size_t)12 * np, 0.0);
    for (int sl = 0; sl < 2 * np; ++sl) {
      const int ge = sl < np ? sl : sl + (nn[a] - 2 * np);
      const int gh = sl < np ? sl : sl + (nn[a] - 1 - 2 * np);
      pml_coeffs(g, s->dt, layer_depth((double)ge, nn[a], np), np, pr[sl], pr[2 * np + sl], pr[4 * np + sl]);
      pml_coeffs(g, s->dt, layer_depth(gh + 0.5, nn[a], np), np, pr[6 * np + sl], pr[8 * np + sl],
                 pr[10 * np + sl]);
    }
    if (np > 0) {
      if (g.precision == GNOR_FP32) {
        std::vector<float> f(pr.begin(), pr.end());
        HIPCHECK(s, hipMemcpy(s->dev + s->L.cpml[a], f.data(), f.size() * 4, hipMemcpyHostToDevice));
      } else {
        HIPCHECK(s, hipMemcpy(s->dev + s->L.cpml[a], pr.data(), pr.size() * 8, hipMemcpyHostToDevice));
      }
    }
  }
  // auxiliary line profiles
  std::vector<double> ap((size_t)6 * s->n1);
  for (int q = 0; q < s->n1; ++q) {
    pml_coeffs(g, s->dt, layer_depth((double)q, s->n1, gnor::kAuxPml), gnor::kAuxPml, ap[q],
               ap[s->n1 + q], ap[2 * s->n1 + q]);
    pml_coeffs(g, s->dt, layer_depth(q + 0.5, s->n1, gnor::kAuxPml), gnor::kAuxPml, ap[3 * s->n1 + q],
               ap[4 * s->n1 + q], ap[5 * s->n1 + q]);
  }
  HIPCHECK(s, hipMemcpy(s->dev + s->L.aux_prof, ap.data(), ap.size() * 8, hipMemcpyHostToDevice));
  if (s->mon.nfreq > 0)
    HIPCHECK(s, hipMemcpy(s->dev + s->L.omega, s->omega.data(), s->omega.size() * 8, hipMemcpyHostToDevice));
  if (s->nsamp > 0) {
    HIPCHECK(s, hipMemcpy(s->dev + s->L.fpw, s->fpw.data(), s->fpw.size() * 8, hipMemcpyHostToDevice));
  }
  if (s->maps.nmap > 0)
    HIPCHECK(s, hipMemcpy(s->dev + s->L.map_om, s->map_omega.data(), s->map_omega.size() * 8,
                          hipMemcpyHostToDevice));
  return GNOR_OK;
}

void prepare(gnor_sim* s) {
  const gnor_grid_desc& g = s->g;
  s->elem = g.precision == GNOR_FP32 ? 4 : 8;
  s->N = (size_t)g.nx * g.ny * g.nz;
  s->n1 = g.nz + 2 * gnor::kAuxOff;
  s->nbx = (g.nx + gnor::kBX - 1) / gnor::kBX;
  s->nby = 0;
  if (!s->any_metal) {
    for (int d = 0; d < 3; ++d) { s->mlo[d] = 0; s->mn[d] = 1; }
  }
  s->M = (size_t)s->mn[0] * s->mn[1] * s->mn[2];
  plan_flux(s);
  plan_layout(s);
}

}  // namespace

// ============================================================ C ABI
extern "C" {

const char* gnor_status_string(gnor_status st) {
  switch (st) {
    case GNOR_OK: return "ok";
    case GNOR_E_INVALID_ARG: return "invalid argument";
    case GNOR_E_UNSTABLE: return "unstable time step";
    case GNOR_E_OUT_OF_MEMORY: return "out of host memory";
    case GNOR_E_DEVICE: return "HIP device error";
    case GNOR_E_STATE: return "call out of order";
    case GNOR_E_BUFFER_TOO_SMALL: return "buffer too small";
    case GNOR_E_NONFINITE: return "non-finite field values";
  }
  return "unknown status";
}

const char* gnor_last_error(const gnor_sim* s) { return s ? s->last_error.c_str() : "null sim"; }

gnor_status gnor_create(const gnor_grid_desc* g, gnor_sim** out) {
  if (!g || !out) return GNOR_E_INVALID_ARG;
  *out = nullptr;
  if (g->nx < 4 || g->ny < 4 || g->nz < 4 || !(g->dx > 0.0) || !(g->eps_background > 0.0))
    return GNOR_E_INVALID_ARG;
  // at most 4e9 cells: the sweeps index cells with 32-bit integers
  if ((double)g->nx * g->ny * g->nz > 4.0e9) return GNOR_E_INVALID_ARG;
  if (g->precision != GNOR_FP32 && g->precision != GNOR_FP64) return GNOR_E_INVALID_ARG;
  if (!(g->eps_substrate >= 0.0) || (g->eps_substrate > 0.0 && (g->substrate_k < 0 || g->substrate_k >= g->nz)))
    return GNOR_E_INVALID_ARG;
  if (!(g->courant > 0.0) || g->courant >= 1.0 / std::sqrt(3.0)) return GNOR_E_UNSTABLE;
  if (g->npml < 0 || 2 * g->npml + 4 > std::min(g->nx, std::min(g->ny, g->nz))) return GNOR_E_INVALID_ARG;
  const int n[3] = {g->nx, g->ny, g->nz};
  if (g->total_field != 0 && g->total_field != 1) return GNOR_E_INVALID_ARG;
  if (g->total_field) {
    if (g->eps_substrate > 0.0) return GNOR_E_INVALID_ARG;
    if (g->source_k < g->npml + 1 || g->source_k > g->nz - 2 - g->npml) return GNOR_E_INVALID_ARG;
  } else {
    for (int d = 0; d < 3; ++d)
      if (g->tf_lo[d] < g->npml + 1 || g->tf_hi[d] > n[d] - 2 - g->npml || g->tf_hi[d] - g->tf_lo[d] < 4)
        return GNOR_E_INVALID_ARG;
  }
  gnor_sim* s = new (std::nothrow) gnor_sim();
  if (!s) return GNOR_E_OUT_OF_MEMORY;
  s->g = *g;
  s->dt = g->courant * g->dx / kC0;
  *out = s;
  return GNOR_OK;
}

void gnor_destroy(gnor_sim* s) {
  if (!s) return;
  drop_graph(s);
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  for (int q = 0; q < 2; ++q) {
    if (s->side[q]) (void)hipStreamDestroy(s->side[q]);
    if (s->ev_join[q]) (void)hipEventDestroy(s->ev_join[q]);
  }
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->wstream) (void)hipStreamDestroy(s->wstream);
  for (int q = 0; q < 2; ++q)
    if (s->wev[q]) (void)hipEventDestroy(s->wev[q]);
  delete s;
}

gnor_status gnor_set_material(gnor_sim* s, const uint8_t* mask, const gnor_material_desc* m) {
  if (!s || !m) return GNOR_E_INVALID_ARG;
  if (s->bound) return fail(s, GNOR_E_STATE, "material must be set before gnor_bind_memory");
  if (!(m->wp >= 0) || !(m->gamma >= 0) || !(m->beta >= 0) || !(m->diffusion >= 0) || !(m->eps_inf > 0))
    return fail(s, GNOR_E_INVALID_ARG, "material parameters must be non-negative (eps_inf > 0)");
  if (m->ncp < 0 || m->ncp > gnor::kMaxCP)
    return fail(s, GNOR_E_INVALID_ARG, "ncp must lie in [0, 4]");
  for (int u = 0; u < m->ncp; ++u)
    if (!std::isfinite(m->cp_A[u]) || !(m->cp_Omega[u] >= 0) || !(m->cp_Gamma[u] >= 0) ||
        !std::isfinite(m->cp_phi[u]))
      return fail(s, GNOR_E_INVALID_ARG, "critical points need finite A, phi and Omega, Gamma >= 0");
  if (m->ncp > 0 && s->mode == 1)
    return fail(s, GNOR_E_INVALID_ARG, "the fused step has no critical-point terms (gnor_set_fused 0 first)");
  const gnor_grid_desc& g = s->g;
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  s->mask.assign(N, 0);
  s->rowx.clear();
  int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
  const int nn[3] = {g.nx, g.ny, g.nz};
  bool any = false;
  if (mask) {
    for (int k = 0; k < g.nz; ++k)
      for (int j = 0; j < g.ny; ++j)
        for (int i = 0; i < g.nx; ++i) {
          const size_t q = ((size_t)k * g.ny + j) * g.nx + i;
          const uint8_t b = mask[q] & 7u;
          if (mask[q] & ~7u) return fail(s, GNOR_E_INVALID_ARG, "mask bytes may only use bits 0-2");
          if (!b) continue;
          const int ii[3] = {i, j, k};
          if (g.eps_substrate > 0.0 && k >= g.substrate_k)
            return fail(s, GNOR_E_INVALID_ARG, "metal must lie below the substrate plane");
          for (int d = 0; d < 3; ++d) {
            if (g.total_field) {
              if (ii[d] < 1 || ii[d] > nn[d] - 2)
                return fail(s, GNOR_E_INVALID_ARG, "metal must lie off the outer node planes");
            } else if (ii[d] < g.tf_lo[d] + 2 || ii[d] > g.tf_hi[d] - 2) {
              char buf[160];
              std::snprintf(buf, sizeof buf,
                            "metal at (%d,%d,%d) is not 2 cells inside the TF box: nonlocal material "
                            "must stay in the total-field region", i, j, k);
              return fail(s, GNOR_E_INVALID_ARG, buf);
            }
            lo[d] = std::min(lo[d], ii[d]);
            hi[d] = std::max(hi[d], ii[d]);
          }
          s->mask[q] = b;
          any = true;
        }
  }
  s->any_metal = any;
  if (any)
    for (int d = 0; d < 3; ++d) { s->mlo[d] = lo[d] - 1; s->mn[d] = hi[d] - lo[d] + 3; }
  s->mat = *m;
  s->have_material = true;
  s->design = false;
  return GNOR_OK;
}

gnor_status gnor_set_design(gnor_sim* s, const int32_t* lo, const int32_t* hi, const float* rho) {
  if (!s || !lo || !hi) return GNOR_E_INVALID_ARG;
  if (!s->have_material) return fail(s, GNOR_E_STATE, "gnor_set_material must come first");
  if (s->bound) return fail(s, GNOR_E_STATE, "the design region must be set before gnor_bind_memory");
  if (s->g.eps_substrate > 0.0) return fail(s, GNOR_E_INVALID_ARG, "design regions do not cover a substrate");
  if (s->g.total_field) return fail(s, GNOR_E_INVALID_ARG, "design regions need the TF/SF source");
  const gnor_grid_desc& g = s->g;
  size_t nd = 1;
  for (int d = 0; d < 3; ++d) {
    if (hi[d] <= lo[d] || lo[d] < g.tf_lo[d] + 2 || hi[d] - 1 > g.tf_hi[d] - 2)
      return fail(s, GNOR_E_INVALID_ARG,
                  "design region must be non-empty and lie 2 cells inside the TF box");
    nd *= (size_t)(hi[d] - lo[d]);
  }
  if (rho)
    for (size_t q = 0; q < nd; ++q)
      if (!(rho[q] >= 0.0f && rho[q] <= 1.0f)) return fail(s, GNOR_E_INVALID_ARG, "rho must lie in [0, 1]");
  int mlo[3], mhi[3];
  for (int d = 0; d < 3; ++d) {
    mlo[d] = s->any_metal ? std::min(s->mlo[d] + 1, lo[d]) : lo[d];
    mhi[d] = s->any_metal ? std::max(s->mlo[d] + s->mn[d] - 2, hi[d] - 1) : hi[d] - 1;
  }
  for (int k = lo[2]; k < hi[2]; ++k)
    for (int j = lo[1]; j < hi[1]; ++j)
      for (int i = lo[0]; i < hi[0]; ++i) s->mask[((size_t)k * g.ny + j) * g.nx + i] = 7;
  s->rowx.clear();
  s->any_metal = true;
  for (int d = 0; d < 3; ++d) {
    s->mlo[d] = mlo[d] - 1;
    s->mn[d] = mhi[d] - mlo[d] + 3;
    s->dlo[d] = lo[d];
    s->dhi[d] = hi[d];
  }
  if (rho) s->rho.assign(rho, rho + nd);
  else s->rho.assign(nd, 1.0f);
  s->design = true;
  return GNOR_OK;
}

gnor_status gnor_update_design(gnor_sim* s, const float* rho_dev) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  if (!s->design) return fail(s, GNOR_E_STATE, "no design region");
  if (!rho_dev) return fail(s, GNOR_E_INVALID_ARG, "null density pointer");
  // check on the device (stream-ordered after the queued steps), then scatter
  int* flag = ptr<int>(s, s->L.dflag);
  gnor::launch_fill_zero(flag, 4, s->stream);
  gnor::launch_design_check(rho_dev, s->rho.size(), flag, s->stream);
  int bad = 0;
  HIPCHECK(s, hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, s->stream));
  HIPCHECK(s, hipStreamSynchronize(s->stream));
  if (bad) return fail(s, GNOR_E_INVALID_ARG, "rho must lie in [0, 1]");
  gnor::DesignMap d{};
  for (int a = 0; a < 3; ++a) {
    d.dn[a] = s->dhi[a] - s->dlo[a];
    d.off[a] = s->dlo[a] - s->mlo[a];
    d.mn[a] = s->mn[a];
  }
  gnor::launch_design_scatter(rho_dev, d, ptr<float>(s, s->L.rho), s->stream);
  HIPCHECK(s, hipGetLastError());
  return GNOR_OK;
}

gnor_status gnor_set_source(gnor_sim* s, const gnor_source_desc* src) {
  if (!s || !src) return GNOR_E_INVALID_ARG;
  if (s->bound) return fail(s, GNOR_E_STATE, "source must be set before gnor_bind_memory");
  if (src->kind < 0 || src->kind > 2) return fail(s, GNOR_E_INVALID_ARG, "unknown source kind");
  if (src->kind == 1 && !(src->tau > 0)) return fail(s, GNOR_E_INVALID_ARG, "tau must be positive");
  if (src->kind == 2 && !(src->omega_max > 0)) return fail(s, GNOR_E_INVALID_ARG, "omega_max must be positive");
  s->src = *src;
  s->have_source = true;
  return GNOR_OK;
}

gnor_status gnor_set_monitors(gnor_sim* s, const gnor_monitor_desc* m) {
  if (!s || !m) return GNOR_E_INVALID_ARG;
  if (s->bound) return fail(s, GNOR_E_STATE, "monitors must be set before gnor_bind_memory");
  if (m->nfreq < 0 || (m->nfreq > 0 && !m->omega)) return fail(s, GNOR_E_INVALID_ARG, "bad frequency list");
  if (m->norm_k < 0 || m->norm_k >= s->g.nz) return fail(s, GNOR_E_INVALID_ARG, "norm_k outside the grid");
  if (m->dft_every < 0) return fail(s, GNOR_E_INVALID_ARG, "dft_every must be >= 0");
  if (m->flux_enabled) {
    if (s->g.total_field) return fail(s, GNOR_E_INVALID_ARG, "flux boxes need the TF/SF source");
    if (m->dft_every > 1) return fail(s, GNOR_E_INVALID_ARG, "flux boxes require dft_every = 1");
    const gnor_grid_desc& g = s->g;
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) {
      if (m->abs_lo[d] <= g.tf_lo[d] || m->abs_hi[d] >= g.tf_hi[d] || m->abs_hi[d] - m->abs_lo[d] < 1)
        return fail(s, GNOR_E_INVALID_ARG, "absorption box must lie strictly inside the TF box");
      if (m->sca_lo[d] >= g.tf_lo[d] - 1 || m->sca_hi[d] <= g.tf_hi[d] + 1 ||
          m->sca_lo[d] < g.npml + 1 || m->sca_hi[d] > n[d] - 2 - g.npml)
        return fail(s, GNOR_E_INVALID_ARG,
                    "scattering box must enclose the TF box with a spare cell and stay out of the CPML");
    }
  }
  s->mon = *m;
  s->omega.assign(m->omega, m->omega + m->nfreq);
  s->mon.omega = nullptr;
  s->have_monitors = true;
  return GNOR_OK;
}

gnor_status gnor_set_maps(gnor_sim* s, const gnor_map_desc* m) {
  if (!s || !m) return GNOR_E_INVALID_ARG;
  if (s->bound) return fail(s, GNOR_E_STATE, "maps must be set before gnor_bind_memory");
  const int n[3] = {s->g.nx, s->g.ny, s->g.nz};
  if (m->nmap < 0 || m->nmap > 8 || (m->nmap > 0 && !m->omega))
    return fail(s, GNOR_E_INVALID_ARG, "nmap must lie in [0, 8] with a frequency list");
  if (m->axis < 0 || m->axis > 2) return fail(s, GNOR_E_INVALID_ARG, "map axis must be 0, 1 or 2");
  if (m->index < 0 || m->index >= n[m->axis]) return fail(s, GNOR_E_INVALID_ARG, "map plane outside the grid");
  if (m->every < 1) return fail(s, GNOR_E_INVALID_ARG, "map every must be >= 1");
  s->maps = *m;
  s->map_omega.assign(m->omega, m->omega + m->nmap);
  s->maps.omega = nullptr;
  return GNOR_OK;
}

gnor_status gnor_get_maps(gnor_sim* s, double* fields, double* inc, size_t count) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  const size_t nq = (size_t)8 * s->maps.nmap * map_plane(s);
  if (count != nq) return fail(s, GNOR_E_BUFFER_TOO_SMALL, "count must be 8 * nmap * plane points");
  if (nq == 0) return GNOR_OK;
  HIPCHECK(s, hipStreamSynchronize(s->stream));
  if (fields) HIPCHECK(s, hipMemcpy(fields, s->dev + s->L.maps, nq * 8, hipMemcpyDeviceToHost));
  if (inc) HIPCHECK(s, hipMemcpy(inc, s->dev + s->L.map_inc, (size_t)2 * s->maps.nmap * 8, hipMemcpyDeviceToHost));
  return GNOR_OK;
}

size_t gnor_required_bytes(const gnor_sim* cs) {
  if (!cs) return 0;
  gnor_sim* s = const_cast<gnor_sim*>(cs);
  prepare(s);
  return s->L.state_end + 256;
}

gnor_status gnor_reset(gnor_sim* s) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  HIPCHECK(s, hipMemsetAsync(s->dev + s->L.state_begin, 0, s->L.state_end - s->L.state_begin, s->stream));
  HIPCHECK(s, hipStreamSynchronize(s->stream));
  s->step = 0;
  s->wpending = false;
  s->wsince = 0;
  return GNOR_OK;
}

gnor_status gnor_bind_memory(gnor_sim* s, void* dptr, size_t bytes, void* stream) {
  if (!s || !dptr) return GNOR_E_INVALID_ARG;
  if (!s->have_material) return fail(s, GNOR_E_STATE, "gnor_set_material has not been called");
  if (!s->have_monitors) {
    gnor_monitor_desc m{};
    m.norm_k = s->g.nz / 2;
    gnor_set_monitors(s, &m);
  }
  if (((uintptr_t)dptr) & 255u) return fail(s, GNOR_E_INVALID_ARG, "device buffer must be 256-byte aligned");
  prepare(s);
  if (bytes < s->L.state_end) return fail(s, GNOR_E_BUFFER_TOO_SMALL, "device buffer smaller than gnor_required_bytes");
  drop_graph(s);
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  s->own_stream = false;
  s->stream = reinterpret_cast<hipStream_t>(stream);
  if (!s->stream) {
    HIPCHECK(s, hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    s->own_stream = true;
  }
  if (!s->side[0]) {
    for (int q = 0; q < 2; ++q) {
      HIPCHECK(s, hipStreamCreateWithFlags(&s->side[q], hipStreamNonBlocking));
      HIPCHECK(s, hipEventCreateWithFlags(&s->ev_join[q], kJoinEventFlags));
    }
    HIPCHECK(s, hipEventCreateWithFlags(&s->ev_fork, kJoinEventFlags));
  }
  if (!s->wstream) {
    HIPCHECK(s, hipStreamCreateWithFlags(&s->wstream, hipStreamNonBlocking));
    for (int q = 0; q < 2; ++q) HIPCHECK(s, hipEventCreateWithFlags(&s->wev[q], kJoinEventFlags));
  }
  s->wpending = false;
  s->dev = reinterpret_cast<char*>(dptr);
  s->dev_bytes = bytes;
  s->bound = true;
  gnor_status st = upload_static(s);
  if (st != GNOR_OK) return st;
  st = plan_tiles(s);
  if (st != GNOR_OK) return st;
  return gnor_reset(s);
}

gnor_status gnor_set_class_streams(gnor_sim* s, int32_t on) {
  if (!s || (on != 0 && on != 1)) return GNOR_E_INVALID_ARG;
  if ((on != 0) != s->concurrent) {
    s->concurrent = on != 0;
    drop_graph(s);
  }
  return GNOR_OK;
}

gnor_status gnor_set_fused(gnor_sim* s, int32_t on) {
  if (!s || on < 0 || on > 3) return GNOR_E_INVALID_ARG;
  if (on == 1 && s->have_material && s->mat.ncp > 0)
    return fail(s, GNOR_E_INVALID_ARG, "the fused step has no critical-point terms");
  if ((on == 1 || on == 2) && s->g.eps_substrate > 0.0)
    return fail(s, GNOR_E_INVALID_ARG, "the fused and hybrid step forms have no substrate");
  if (on == 1 && s->g.total_field)
    return fail(s, GNOR_E_INVALID_ARG, "the fused step has no local-Drude absorbing layers");
  return set_mode(s, on);
}

gnor_status gnor_set_graph_chunk(gnor_sim* s, int32_t steps) {
  if (!s) return GNOR_E_INVALID_ARG;
  if (steps < 0 || (steps & 1)) return fail(s, GNOR_E_INVALID_ARG, "graph chunk must be even and >= 0");
  s->graph_chunk = steps;
  drop_graph(s);
  return GNOR_OK;
}

}  // extern "C"

namespace {

// Watchdog: scan E^n (the state after the last enqueued step) for NaN / Inf
// into the sticky flag and mark the scan with an event.
void watch_scan(gnor_sim* s) {
  int* flag = ptr<int>(s, s->L.flag);
  const int parity = (int)(s->step & 1);
  for (int c = 0; c < 3; ++c) {
    if (s->g.precision == GNOR_FP32)
      gnor::launch_nonfinite<float>(ptr<float>(s, s->L.E[parity][c]), s->N, flag, s->stream);
    else
      gnor::launch_nonfinite<double>(ptr<double>(s, s->L.E[parity][c]), s->N, flag, s->stream);
  }
  s->wslot ^= 1;
  (void)hipEventRecord(s->wev[s->wslot], s->stream);
  s->wpending = true;
}

// Read the flag of the scan marked by event slot `slot` (waits for that scan
// only, not for work queued after it).
gnor_status watch_read(gnor_sim* s, int slot) {
  int h = 0;
  HIPCHECK(s, hipStreamWaitEvent(s->wstream, s->wev[slot], 0));
  HIPCHECK(s, hipMemcpyAsync(&h, ptr<int>(s, s->L.flag), 4, hipMemcpyDeviceToHost, s->wstream));
  HIPCHECK(s, hipStreamSynchronize(s->wstream));
  return h ? fail(s, GNOR_E_NONFINITE, "non-finite value in E (watchdog)") : GNOR_OK;
}

}  // namespace

extern "C" {

gnor_status gnor_set_watchdog(gnor_sim* s, int32_t on) {
  if (!s || (on != 0 && on != 1)) return GNOR_E_INVALID_ARG;
  s->watchdog = on != 0;
  return GNOR_OK;
}

gnor_status gnor_run(gnor_sim* s, int64_t nsteps) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  if (nsteps < 0) return fail(s, GNOR_E_INVALID_ARG, "nsteps < 0");
  // a finished scan of an earlier call already flagged the state
  if (s->watchdog && s->wpending && hipEventQuery(s->wev[s->wslot]) == hipSuccess) {
    s->wpending = false;
    st = watch_read(s, s->wslot);
    if (st != GNOR_OK) return st;
  }
  int64_t left = nsteps;
  const int align = chunk_alignment(s);
  int chunk = s->graph_chunk;
  if (chunk > 0) chunk = std::max(align, chunk / align * align);
  // steps between watchdog scans: the graph chunk (eager runs: 64), counted
  // across calls (a caller stepping one step at a time scans as rarely)
  const int64_t period = chunk > 0 ? chunk : 64;
  while (left > 0) {
    int64_t n;
    if (chunk > 0 && (s->step % align) == 0 && left >= chunk) {
      if (!s->graph || s->graph_steps != chunk) {
        st = build_graph(s, chunk);
        if (st != GNOR_OK) return st;
      }
      HIPCHECK(s, hipGraphLaunch(s->graph, s->stream));
      n = chunk;
    } else {
      // eager steps until the next aligned chunk start (or the end)
      n = std::min(left, period);
      if (chunk > 0) {
        const int64_t to_align = (align - (s->step % align)) % align;
        n = to_align > 0 ? std::min(left, to_align) : std::min(left, (int64_t)chunk);
        if (to_align == 0 && left < chunk) n = left;
      }
      enqueue_steps_eager(s, s->step, n, s->stream, s->mode);
      HIPCHECK(s, hipGetLastError());
    }
    s->step += n;
    left -= n;
    s->wsince += n;
    if (s->watchdog && s->wsince >= period) {
      s->wsince = 0;
      // the previous scan's flag is read while this chunk runs
      const bool had = s->wpending;
      watch_scan(s);
      HIPCHECK(s, hipGetLastError());
      if (had) {
        st = watch_read(s, s->wslot ^ 1);
        if (st != GNOR_OK) return st;
      }
    }
  }
  return GNOR_OK;
}

gnor_status gnor_synchronize(gnor_sim* s) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  HIPCHECK(s, hipStreamSynchronize(s->stream));
  if (s->watchdog && s->wpending) {
    s->wpending = false;
    return watch_read(s, s->wslot);
  }
  return GNOR_OK;
}

int64_t gnor_step_index(const gnor_sim* s) { return s ? s->step : -1; }

gnor_status gnor_get_dft(gnor_sim* s, double* are, double* aim, double* bre, double* bim) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  const size_t nzf = (size_t)s->g.nz * s->mon.nfreq;
  if (nzf == 0) return GNOR_OK;
  HIPCHECK(s, hipStreamSynchronize(s->stream));
  std::vector<double> buf(4 * nzf);
  HIPCHECK(s, hipMemcpy(buf.data(), s->dev + s->L.dft, 4 * nzf * 8, hipMemcpyDeviceToHost));
  const double aconv = eps0() / s->dt;  // J~ = J dt / eps0
  for (size_t q = 0; q < nzf; ++q) {
    if (are) are[q] = buf[q] * aconv;
    if (aim) aim[q] = buf[nzf + q] * aconv;
    if (bre) bre[q] = buf[2 * nzf + q];
    if (bim) bim[q] = buf[3 * nzf + q];
  }
  return GNOR_OK;
}

}  // extern "C"

extern "C" {

gnor_status gnor_flush_spectra(gnor_sim* s) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  // fold the staged flux samples of the current window (a no-op right after
  // a fold); the next window fold takes only the slots staged after this
  if (s->nsamp > 0 && s->step > 0 && (s->step % s->slots) != 0) {
    enqueue_flux_acc(s, -1, s->stream);  // last staged step = counter - 1
    HIPCHECK(s, hipGetLastError());
  }
  return GNOR_OK;
}

gnor_status gnor_get_spectra(gnor_sim* s, double* inc, double* ext, double* absn, double* sca) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  const int nf = s->mon.nfreq;
  if (nf == 0) return GNOR_OK;
  std::vector<double> fs(2 * (size_t)nf, 0.0);
  if (s->nsamp > 0) {
    // fold the partially filled staging window into the accumulators
    st = gnor_flush_spectra(s);
    if (st != GNOR_OK) return st;
    gnor::launch_flux_reduce(ptr<double>(s, s->L.facc), ptr<double>(s, s->L.fpw), s->npairs,
                             s->npairs_box0, nf, ptr<double>(s, s->L.fpart), ptr<double>(s, s->L.fsum),
                             s->stream);
    HIPCHECK(s, hipGetLastError());
    HIPCHECK(s, hipStreamSynchronize(s->stream));
    HIPCHECK(s, hipMemcpy(fs.data(), s->dev + s->L.fsum, fs.size() * 8, hipMemcpyDeviceToHost));
  }
  const int nz = s->g.nz;
  std::vector<double> are((size_t)nz * nf), aim((size_t)nz * nf), bre((size_t)nz * nf), bim((size_t)nz * nf);
  st = gnor_get_dft(s, are.data(), aim.data(), bre.data(), bim.data());
  if (st != GNOR_OK) return st;
  const double h3 = s->g.dx * s->g.dx * s->g.dx;
  for (int m = 0; m < nf; ++m) {
    const size_t qc = (size_t)s->mon.norm_k * nf + m;
    const double b2 = bre[qc] * bre[qc] + bim[qc] * bim[qc];
    if (inc) inc[m] = b2;
    double acc = 0.0;
    for (int k = 0; k < nz; ++k) {
      const size_t q = (size_t)k * nf + m;
      acc += are[q] * bre[q] + aim[q] * bim[q];
    }
    if (ext) ext[m] = eta0() * h3 * acc / b2;
    // flux sums are of Re(E conj(H~)) with H~ = eta0 H: flux_SI = sum / eta0
    if (absn) absn[m] = s->nsamp > 0 ? -fs[m] / b2 : 0.0;
    if (sca) sca[m] = s->nsamp > 0 ? fs[nf + m] / b2 : 0.0;
  }
  return GNOR_OK;
}

gnor_status gnor_get_field(gnor_sim* s, int32_t which, double* dst, size_t count) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  if (!dst) return GNOR_E_INVALID_ARG;
  if (count != s->N) return fail(s, GNOR_E_BUFFER_TOO_SMALL, "count must be nx*ny*nz");
  const bool density = which == kFieldDensity;
  if (!density && (which < 0 || which >= 9 + 3 * s->mat.ncp))
    return fail(s, GNOR_E_INVALID_ARG, "field index out of range");
  const int parity = (int)(s->step & 1);
  if (density) {
    std::memset(dst, 0, s->N * 8);
    if (!s->any_metal) return GNOR_OK;
    // div P_f^n at the nodes: Phi~_P^{n-1} (left by the last H sweep in the
    // buffer of this parity) plus the node divergence of J~^{n-1/2}
    const double scale = eps0() / (s->g.dx * kElementaryCharge);
    double* out = ptr<double>(s, s->L.dens);
    if (s->g.precision == GNOR_FP32)
      gnor::launch_density<float>(ptr<float>(s, s->L.PP[parity]), ptr<float>(s, s->L.J[parity][0]),
                                  ptr<float>(s, s->L.J[parity][1]), ptr<float>(s, s->L.J[parity][2]),
                                  s->mn, scale, out, s->stream);
    else
      gnor::launch_density<double>(ptr<double>(s, s->L.PP[parity]), ptr<double>(s, s->L.J[parity][0]),
                                   ptr<double>(s, s->L.J[parity][1]), ptr<double>(s, s->L.J[parity][2]),
                                   s->mn, scale, out, s->stream);
    HIPCHECK(s, hipGetLastError());
    std::vector<double> v(s->M);
    HIPCHECK(s, hipMemcpyAsync(v.data(), out, s->M * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(s, hipStreamSynchronize(s->stream));
    const gnor_grid_desc& g = s->g;
    for (int z = 0; z < s->mn[2]; ++z)
      for (int y = 0; y < s->mn[1]; ++y)
        for (int x = 0; x < s->mn[0]; ++x)
          dst[((size_t)(z + s->mlo[2]) * g.ny + (y + s->mlo[1])) * g.nx + (x + s->mlo[0])] =
              v[((size_t)z * s->mn[1] + y) * s->mn[0] + x];
    return GNOR_OK;
  }
  HIPCHECK(s, hipStreamSynchronize(s->stream));
  const int c = which % 3;
  const bool fp32 = s->g.precision == GNOR_FP32;
  auto fetch = [&](size_t off, size_t n, std::vector<double>& out) -> gnor_status {
    out.resize(n);
    if (fp32) {
      std::vector<float> f(n);
      HIPCHECK(s, hipMemcpy(f.data(), s->dev + off, n * 4, hipMemcpyDeviceToHost));
      for (size_t q = 0; q < n; ++q) out[q] = f[q];
    } else {
      HIPCHECK(s, hipMemcpy(out.data(), s->dev + off, n * 8, hipMemcpyDeviceToHost));
    }
    return GNOR_OK;
  };
  std::vector<double> v;
  if (which < 3) {
    st = fetch(s->L.E[parity][c], s->N, v);
    if (st != GNOR_OK) return st;
    std::memcpy(dst, v.data(), s->N * 8);
  } else if (which < 6) {
    st = fetch(s->L.H[s->step & 1][c], s->N, v);
    if (st != GNOR_OK) return st;
    const double k = 1.0 / eta0();
    for (size_t q = 0; q < s->N; ++q) dst[q] = v[q] * k;
  } else {
    std::memset(dst, 0, s->N * 8);
    if (s->any_metal) {
      // J (sub-grid, scaled increment of P_f) or P_CP,u / eps0 (sub-grid)
      const bool cp = which >= 9;
      st = fetch(cp ? s->L.cpP[(which - 9) / 3][c] : s->L.J[parity][c], s->M, v);
      if (st != GNOR_OK) return st;
      const double k = cp ? eps0() : eps0() / s->dt;
      const gnor_grid_desc& g = s->g;
      for (int z = 0; z < s->mn[2]; ++z)
        for (int y = 0; y < s->mn[1]; ++y)
          for (int x = 0; x < s->mn[0]; ++x)
            dst[((size_t)(z + s->mlo[2]) * g.ny + (y + s->mlo[1])) * g.nx + (x + s->mlo[0])] =
                v[((size_t)z * s->mn[1] + y) * s->mn[0] + x] * k;
    }
  }
  return GNOR_OK;
}

gnor_status gnor_get_aux(gnor_sim* s, double* e1, double* h1, size_t count) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  if (count != (size_t)s->n1) return fail(s, GNOR_E_BUFFER_TOO_SMALL, "count must be nz + 50");
  HIPCHECK(s, hipStreamSynchronize(s->stream));
  std::vector<double> buf(2 * (size_t)s->n1);
  HIPCHECK(s, hipMemcpy(buf.data(), s->dev + s->L.aux, buf.size() * 8, hipMemcpyDeviceToHost));
  if (e1) std::memcpy(e1, buf.data(), s->n1 * 8);
  if (h1)
    for (int q = 0; q < s->n1; ++q) h1[q] = buf[s->n1 + q] / eta0();
  return GNOR_OK;
}

size_t gnor_state_bytes(const gnor_sim* s) {
  if (!s || !s->bound) return 0;
  return s->L.state_end - s->L.state_begin + 8;
}

gnor_status gnor_save_state(gnor_sim* s, void* dst, size_t bytes) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  if (!dst) return GNOR_E_INVALID_ARG;
  const size_t n = s->L.state_end - s->L.state_begin;
  if (bytes < n + 8) return fail(s, GNOR_E_BUFFER_TOO_SMALL, "state buffer too small");
  HIPCHECK(s, hipStreamSynchronize(s->stream));
  std::memcpy(dst, &s->step, 8);
  HIPCHECK(s, hipMemcpy(static_cast<char*>(dst) + 8, s->dev + s->L.state_begin, n, hipMemcpyDeviceToHost));
  return GNOR_OK;
}

gnor_status gnor_load_state(gnor_sim* s, const void* src, size_t bytes) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  if (!src) return GNOR_E_INVALID_ARG;
  const size_t n = s->L.state_end - s->L.state_begin;
  if (bytes < n + 8) return fail(s, GNOR_E_BUFFER_TOO_SMALL, "state buffer too small");
  HIPCHECK(s, hipStreamSynchronize(s->stream));
  std::memcpy(&s->step, src, 8);
  HIPCHECK(s, hipMemcpy(s->dev + s->L.state_begin, static_cast<const char*>(src) + 8, n, hipMemcpyHostToDevice));
  s->wpending = false;
  return GNOR_OK;
}

gnor_status gnor_check_finite(gnor_sim* s) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  int* flag = ptr<int>(s, s->L.chk);
  HIPCHECK(s, hipMemsetAsync(flag, 0, 4, s->stream));
  const int parity = (int)(s->step & 1);
  for (int c = 0; c < 3; ++c) {
    if (s->g.precision == GNOR_FP32) {
      gnor::launch_nonfinite<float>(ptr<float>(s, s->L.E[parity][c]), s->N, flag, s->stream);
      gnor::launch_nonfinite<float>(ptr<float>(s, s->L.H[s->step & 1][c]), s->N, flag, s->stream);
    } else {
      gnor::launch_nonfinite<double>(ptr<double>(s, s->L.E[parity][c]), s->N, flag, s->stream);
      gnor::launch_nonfinite<double>(ptr<double>(s, s->L.H[s->step & 1][c]), s->N, flag, s->stream);
    }
  }
  int h = 0;
  HIPCHECK(s, hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, s->stream));
  HIPCHECK(s, hipStreamSynchronize(s->stream));
  return h ? fail(s, GNOR_E_NONFINITE, "non-finite value in E or H") : GNOR_OK;
}

gnor_status gnor_profile_kernels(gnor_sim* s, int64_t nsteps, double* ms, int32_t count) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  if (!ms || count < 5 || nsteps <= 0) return GNOR_E_INVALID_ARG;
  constexpr int NC = gnor::kClasses;
  // events around: the class launches of the first sweep (H, or the fused
  // step), the class launches of the E/J sweep (two-sweep form) or the
  // auxiliary line (fused form), the spectra, the flux accumulation, the
  // step counter
  // Every step gets its own events and the host synchronizes once at the end,
  // so the queue never drains and no interval holds host launch latency.
  constexpr int NE = 2 * NC + 4;
  if (nsteps > 4096) return fail(s, GNOR_E_INVALID_ARG, "profile: at most 4096 steps");
  // the events are destroyed on every return path
  struct Events {
    std::vector<hipEvent_t> v;
    ~Events() {
      for (hipEvent_t e : v)
        if (e) (void)hipEventDestroy(e);
    }
  } events;
  events.v.assign((size_t)nsteps * NE, nullptr);
  std::vector<hipEvent_t>& evs = events.v;
  // timing only: no system-scope fence (no L2 write-back inside the intervals)
  for (auto& e : evs) HIPCHECK(s, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  double acc[NE - 1] = {};
  const bool fp32 = s->g.precision == GNOR_FP32;
  const int mode = s->mode;
  const bool fused = mode == 1;
  // each half timed as a whole: concurrent classes, and the hybrid form (its
  // fused classes span both halves); the form with one-pass plain tiles, run
  // serially, times class 0's one-pass launches (with their TF/SF fix) in the
  // first half's class-0 slot and the line in the second's
  const bool whole = s->concurrent || mode == 2;
  const bool plain1 = mode == 3;
  for (int64_t q = 0; q < nsteps; ++q) {
    const int64_t n = s->step;
    const int parity = (int)(n & 1);
    const hipStream_t str = s->stream;
    const gnor::AuxParams a = make_aux(s);
    hipEvent_t* ev = evs.data() + (size_t)q * NE;
    (void)hipEventRecord(ev[0], str);
    if (whole) {
      // each half of the step timed as a whole, its classes running
      // concurrently as in a normal run (per-class entries stay 0)
      if (fp32) enqueue_first<float>(s, make_params<float>(s, parity), a, mode, str);
      else enqueue_first<double>(s, make_params<double>(s, parity), a, mode, str);
      (void)hipEventRecord(ev[NC], str);
      if (fp32) enqueue_second<float>(s, make_params<float>(s, parity), a, 0, mode, str);
      else enqueue_second<double>(s, make_params<double>(s, parity), a, 0, mode, str);
      (void)hipEventRecord(ev[2 * NC], str);
    }
    for (int c = 0; c < NC && !whole; ++c) {
      if (fused) {
        if (fp32) gnor::launch_step_class<float>(make_params<float>(s, parity), a, c, str);
        else gnor::launch_step_class<double>(make_params<double>(s, parity), a, c, str);
      } else if (plain1 && hybrid_fused(s, c)) {
        if (fp32) gnor::launch_fplain<float>(make_params<float>(s, parity), a, c, s->tf_shell[c], str);
        else gnor::launch_fplain<double>(make_params<double>(s, parity), a, c, s->tf_shell[c], str);
      } else {
        if (fp32) gnor::launch_h_class<float>(make_params<float>(s, parity), a, c, str);
        else gnor::launch_h_class<double>(make_params<double>(s, parity), a, c, str);
      }
      (void)hipEventRecord(ev[1 + c], str);
    }
    for (int c = 0; c < NC && !whole; ++c) {
      if (fused || (plain1 && hybrid_fused(s, c))) {
        if (c == 0) gnor::launch_aux(a, 0, str);
      } else {
        if (fp32) gnor::launch_ej_class<float>(make_params<float>(s, parity), a, 0, c, str);
        else gnor::launch_ej_class<double>(make_params<double>(s, parity), a, 0, c, str);
      }
      (void)hipEventRecord(ev[1 + NC + c], str);
    }
    if (s->g.total_field) {  // timed with the spectra
      if (fp32) gnor::launch_plane_source<float>(make_params<float>(s, parity), a, s->g.source_k, 0, str);
      else gnor::launch_plane_source<double>(make_params<double>(s, parity), a, s->g.source_k, 0, str);
    }
    if (s->mon.nfreq > 0) {
      if (fp32) gnor::launch_dft_stage<float>(make_dft(s), make_flux(s), make_params<float>(s, parity), 0, str);
      else gnor::launch_dft_stage<double>(make_dft(s), make_flux(s), make_params<double>(s, parity), 0, str);
    }
    if (s->maps.nmap > 0) {
      if (fp32) gnor::launch_maps<float>(make_maps<float>(s, parity), 0, str);
      else gnor::launch_maps<double>(make_maps<double>(s, parity), 0, str);
    }
    (void)hipEventRecord(ev[1 + 2 * NC], str);
    if (s->nsamp > 0 && (n % s->slots) == s->slots - 1) enqueue_flux_acc(s, 0, str);
    (void)hipEventRecord(ev[2 + 2 * NC], str);
    gnor::launch_advance(ptr<int64_t>(s, s->L.step), 1, str);
    (void)hipEventRecord(ev[3 + 2 * NC], str);
    HIPCHECK(s, hipGetLastError());
    s->step += 1;
  }
  HIPCHECK(s, hipStreamSynchronize(s->stream));
  for (int64_t q = 0; q < nsteps; ++q) {
    const hipEvent_t* ev = evs.data() + (size_t)q * NE;
    auto elapsed = [&](int from, int to) {
      float t = 0.f;
      (void)hipEventElapsedTime(&t, ev[from], ev[to]);
      return (double)t;
    };
    if (whole) {  // ev[0], ev[NC] and ev[2 NC] bound the halves
      acc[NC - 1] += elapsed(0, NC);
      acc[2 * NC - 1] += elapsed(NC, 2 * NC);
    } else {
      for (int e = 0; e < 2 * NC; ++e) acc[e] += elapsed(e, e + 1);
    }
    for (int e = 2 * NC; e < NE - 1; ++e) acc[e] += elapsed(e, e + 1);
  }
  const double inv = 1.0 / (double)nsteps;
  double first = 0.0, second = 0.0;
  for (int c = 0; c < NC; ++c) {
    first += acc[c] * inv;
    second += acc[NC + c] * inv;
  }
  double out[6 + 2 * NC];
  out[0] = fused ? 0.0 : first;
  out[1] = fused ? 0.0 : second;
  out[2] = acc[2 * NC] * inv;
  out[3] = fused ? first + second : 0.0;
  out[4] = acc[2 * NC + 1] * inv;
  for (int c = 0; c < NC; ++c) {
    out[5 + c] = whole ? 0.0 : acc[c] * inv;
    out[5 + NC + c] = (fused || whole) ? 0.0 : acc[NC + c] * inv;
  }
  out[5 + 2 * NC] = fused ? second : 0.0;
  for (int i = 0; i < count && i < 6 + 2 * NC; ++i) ms[i] = out[i];
  return GNOR_OK;
}

gnor_status gnor_tile_classes(const gnor_sim* s, int32_t* counts) {
  if (!s || !counts) return GNOR_E_INVALID_ARG;
  for (int c = 0; c < gnor::kClasses; ++c) counts[c] = s->tl.cn[c];
  return GNOR_OK;
}

gnor_status gnor_tile_class_cells(const gnor_sim* s, int64_t* cells, int64_t* slab_dirs) {
  if (!s || !cells || !slab_dirs) return GNOR_E_INVALID_ARG;
  if (!s->bound) return GNOR_E_STATE;
  const gnor_grid_desc& g = s->g;
  const gnor::Tiling& t = s->tl;
  const int n[3] = {g.nx, g.ny, g.nz}, np = g.npml;
  // cells of [lo, hi) on an axis of n nodes that lie in its slabs
  auto in_slab = [np](int lo, int hi, int nn) -> int64_t {
    if (np <= 0) return 0;
    const int a = std::max(0, std::min(hi, np) - lo);
    const int b = std::max(0, hi - std::max(lo, nn - np));
    return a + b;
  };
  for (int c = 0; c < gnor::kClasses; ++c) {
    cells[c] = 0;
    slab_dirs[c] = 0;
    for (int q = 0; q < t.cn[c]; ++q) {
      const int tile = s->tile_list[t.coff[c] + q];
      const int b[3] = {tile % t.nbx, (tile / t.nbx) % t.nby, tile / (t.nbx * t.nby)};
      const int w[3] = {gnor::kBX, t.ty, t.kz};
      int lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        lo[d] = b[d] * w[d];
        hi[d] = std::min(n[d], lo[d] + w[d]);
      }
      const int64_t e[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
      cells[c] += e[0] * e[1] * e[2];
      slab_dirs[c] += in_slab(lo[0], hi[0], n[0]) * e[1] * e[2] + in_slab(lo[1], hi[1], n[1]) * e[0] * e[2] +
                      in_slab(lo[2], hi[2], n[2]) * e[0] * e[1];
    }
  }
  return GNOR_OK;
}

gnor_status gnor_set_tiling(gnor_sim* s, int32_t ty, int32_t kz, int32_t xcd) {
  if (!s) return GNOR_E_INVALID_ARG;
  if (!(ty == 2 || ty == 4 || ty == 8) || kz < 1 || kz > s->g.nz || xcd < 0 || xcd > 2)
    return fail(s, GNOR_E_INVALID_ARG, "tiling: ty must be 2, 4 or 8, 1 <= kz <= nz, tile order 0, 1 or 2");
  if (ty != s->tile_ty || kz != s->tile_kz || xcd != s->tile_xcd) {
    s->tile_ty = ty;
    s->tile_kz = kz;
    s->tile_xcd = xcd;
    drop_graph(s);
    const gnor_status st = plan_tiles(s);
    if (st != GNOR_OK) return st;
    if (s->bound) {
      // partial sums are indexed by tile: clear stale entries of the old tiling
      const size_t jbytes = (size_t)s->g.nz * s->nbx * (s->g.ny + 8) * 8;
      HIPCHECK(s, hipMemsetAsync(s->dev + s->L.jpart, 0, jbytes, s->stream));
      HIPCHECK(s, hipStreamSynchronize(s->stream));
    }
  }
  return GNOR_OK;
}

gnor_status gnor_autotune(gnor_sim* s, int32_t trial_steps, int32_t* ty_out, int32_t* kz_out,
                          int32_t* xcd_out, double* ms_out) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  if (s->step != 0) return fail(s, GNOR_E_STATE, "autotune runs before the first step (state is reset afterwards)");
  if (trial_steps < 2) trial_steps = 2;
  const int tys[3] = {2, 4, 8};
  const int nz = s->g.nz;
  const int kzs[8] = {2, 3, 4, 8, 16, 32, 64, nz};
  // on every return path: the events destroyed, the graph chunk restored,
  // and (on failure) the tiling the search started from set back
  struct Restore {
    gnor_sim* s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int chunk, ty, kz, xcd;
    bool done = false;
    ~Restore() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      s->graph_chunk = chunk;
      if (!done) (void)gnor_set_tiling(s, ty, kz, xcd);
    }
  } guard{s, nullptr, nullptr, s->graph_chunk, s->tile_ty, s->tile_kz, s->tile_xcd};
  HIPCHECK(s, hipEventCreate(&guard.e0));
  HIPCHECK(s, hipEventCreate(&guard.e1));
  hipEvent_t e0 = guard.e0, e1 = guard.e1;
  s->graph_chunk = 0;
  // ms per step of one tiling over `steps` steps (after two warm-up steps)
  auto trial = [&](int ty, int kz, int x, int steps, double* ms) -> gnor_status {
    gnor_status r = gnor_set_tiling(s, ty, kz, x);
    if (r == GNOR_OK) r = gnor_run(s, 2);
    if (r != GNOR_OK) return r;
    (void)hipEventRecord(e0, s->stream);
    r = gnor_run(s, steps);
    if (r != GNOR_OK) return r;
    (void)hipEventRecord(e1, s->stream);
    HIPCHECK(s, hipEventSynchronize(e1));
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    *ms = t / steps;
    return GNOR_OK;
  };
  // every candidate once, then the four fastest again, three times each over
  // four times the steps, keeping each one's best (single short trials
  // differ by a few per cent from run to run)
  struct Cand { double ms; int ty, kz, x; };
  std::vector<Cand> cands;
  for (int x = 0; x < 3; ++x)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 8; ++b) {
        const int kz = std::min(kzs[b], nz);
        if (b > 0 && kz <= std::min(kzs[b - 1], nz)) continue;  // clamped duplicate
        Cand c{0.0, tys[a], kz, x};
        st = trial(c.ty, c.kz, c.x, trial_steps, &c.ms);
        if (st != GNOR_OK) return st;
        cands.push_back(c);
      }
  std::sort(cands.begin(), cands.end(), [](const Cand& u, const Cand& v) { return u.ms < v.ms; });
  double best = 1e300;
  int bty = s->tile_ty, bkz = s->tile_kz, bxcd = s->tile_xcd;
  for (int rep = 0; rep < 3; ++rep)
    for (size_t q = 0; q < cands.size() && q < 4; ++q) {
      double ms = 0.0;
      st = trial(cands[q].ty, cands[q].kz, cands[q].x, 4 * trial_steps, &ms);
      if (st != GNOR_OK) return st;
      if (ms < best) { best = ms; bty = cands[q].ty; bkz = cands[q].kz; bxcd = cands[q].x; }
    }
  s->graph_chunk = guard.chunk;
  st = gnor_set_tiling(s, bty, bkz, bxcd);
  if (st != GNOR_OK) return st;
  guard.done = true;
  st = gnor_reset(s);
  if (st != GNOR_OK) return st;
  if (ty_out) *ty_out = bty;
  if (kz_out) *kz_out = bkz;
  if (xcd_out) *xcd_out = bxcd;
  if (ms_out) *ms_out = best;
  return GNOR_OK;
}

// ----------------------------------------------------------------- voxelisers
gnor_status gnor_voxelize_spheres(int32_t nx, int32_t ny, int32_t nz, double dx, int32_t n,
                                  const double* cr, uint8_t* out) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || !(dx > 0) || n < 0 || (n > 0 && !cr) || !out)
    return GNOR_E_INVALID_ARG;
  // quantise centre and radius to 2^-20 cell; exact int64 comparison
  std::vector<long long> q((size_t)4 * n);
  for (int s = 0; s < n; ++s)
    for (int t = 0; t < 4; ++t) q[4 * s + t] = std::llround(cr[4 * s + t] / dx * 1048576.0);
  const long long one = 1048576, half = 524288;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        uint8_t bits = 0;
        const long long X = i * one, Y = j * one, Z = k * one;
        for (int c = 0; c < 3; ++c) {
          const long long px = X + (c == 0 ? half : 0), py = Y + (c == 1 ? half : 0), pz = Z + (c == 2 ? half : 0);
          for (int s = 0; s < n; ++s) {
            const long long ex = px - q[4 * s], ey = py - q[4 * s + 1], ez = pz - q[4 * s + 2];
            const long long r = q[4 * s + 3];
            if (ex * ex + ey * ey + ez * ez < r * r) { bits |= (uint8_t)(1u << c); break; }
          }
        }
        out[((size_t)k * ny + j) * nx + i] = bits;
      }
  return GNOR_OK;
}

}  // extern "C"

namespace {
// Inside test of the star (sphere + sphere-capped cones), FP64 in a fixed
// operation order (this file is compiled with -ffp-contract=off).
bool star_point(const double* d, double x, double y, double z) {
  const double ox = x - d[0], oy = y - d[1], oz = z - d[2];
  const double R = d[3], rt = d[4], tn = d[5], sn = d[6];
  const int nt = (int)d[7];
  const double r2 = ox * ox + oy * oy + oz * oz;
  if (r2 < R * R) return true;
  for (int t = 0; t < nt; ++t) {
    const double* a = d + 8 + 4 * t;
    const double s_cap = R + a[3] - rt;
    const double s_apex = s_cap + rt / sn;
    const double s_tan = s_cap + rt * sn;
    const double s = ox * a[0] + oy * a[1] + oz * a[2];
    const double q2 = r2 - s * s;
    if (s >= 0.0 && s <= s_tan) {
      const double rad = (s_apex - s) * tn;
      if (q2 < rad * rad) return true;
    }
    const double ux = ox - s_cap * a[0], uy = oy - s_cap * a[1], uz = oz - s_cap * a[2];
    if (ux * ux + uy * uy + uz * uz < rt * rt) return true;
  }
  return false;
}
}  // namespace

extern "C" gnor_status gnor_voxelize_star(int32_t nx, int32_t ny, int32_t nz, double dx, const double* d,
                                          int32_t len, uint8_t* out) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || !(dx > 0) || !d || !out || len < 8) return GNOR_E_INVALID_ARG;
  if (len != 8 + 4 * (int)d[7]) return GNOR_E_INVALID_ARG;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const double xi = (double)i * dx, yj = (double)j * dx, zk = (double)k * dx;
        const double xh = ((double)i + 0.5) * dx, yh = ((double)j + 0.5) * dx, zh = ((double)k + 0.5) * dx;
        uint8_t b = 0;
        if (star_point(d, xh, yj, zk)) b |= 1u;
        if (star_point(d, xi, yh, zk)) b |= 2u;
        if (star_point(d, xi, yj, zh)) b |= 4u;
        out[((size_t)k * ny + j) * nx + i] = b;
      }
  return GNOR_OK;
}

// ============================================================ batches
// Many independent simulations stepped in lockstep: each phase of a step is
// ONE launch over the tiles of every instance (block -> instance through a
// device table of per-instance parameters, one table per ping-pong parity).
struct gnor_batch {
  std::vector<gnor_sim*> sims;
  int n = 0;
  bool fp32 = true;
  int ty = 2;
  char* tab = nullptr;       // two tables of n entries (parity 0, parity 1), caller memory
  size_t entry_bytes = 0;
  int hblocks[gnor::kClasses] = {0, 0, 0, 0}, dblocks = 0, fblocks = 0, sblocks = 0;
  // step form: 0 two sweeps; 3 the tiles without metal in one pass (as
  // gnor_set_fused(sim, 3) for one simulation)
  int form = 0;
  // concurrent class launches, as for a single simulation (serial on the
  // batch's stream for a batch made by gnor_batch_create_static)
  bool concurrent = true;
  int static_dev = -1;       // device whose static table this batch uses (-1: caller table)
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
  std::vector<int> tiling;   // (ty, kz, order) of every instance at creation
  bool any_dft = false, any_flux = false, any_cp = false, all_cp = false;
  bool stream_stores = false;  // nontemporal field stores (by the batch's total size)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipGraphExec_t graph = nullptr;
  int graph_steps = 0, graph_chunk = 64;
  int64_t step = 0;
  std::string last_error;
};

namespace {

gnor_status bfail(gnor_batch* b, gnor_status st, const std::string& m) {
  if (b) b->last_error = m;
  return st;
}

#define BHIPCHECK(b, call)                                                                 \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return bfail(b, GNOR_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

template <class T>
gnor_status batch_tables(gnor_batch* b) {
  std::vector<gnor::BatchEntry<T>> tab(2 * (size_t)b->n);
  // one launch sweeps every instance: stream the field stores by the total
  double cells = 0.0;
  for (int q = 0; q < b->n; ++q) cells += (double)b->sims[q]->N;
  const int stream = 9.0 * cells * sizeof(T) > gnor::kStreamStoreBytes ? 1 : 0;
  b->stream_stores = stream != 0;
  for (int parity = 0; parity < 2; ++parity) {
    int h0[gnor::kClasses] = {0, 0, 0, 0}, d0 = 0, f0 = 0, s0 = 0;
    for (int q = 0; q < b->n; ++q) {
      gnor_sim* s = b->sims[q];
      gnor::BatchEntry<T>& e = tab[(size_t)parity * b->n + q];
      e.p = make_params<T>(s, parity);
      e.p.stream_stores = stream;
      e.a = make_aux(s);
      e.d = make_dft(s);
      e.f = make_flux(s);
      for (int c = 0; c < gnor::kClasses; ++c) {
        // XCD-aware tile orders: the instance's first chunk goes to XCD q % 8
        // (its tiles keep their grouping by XCD under any start; the rotation
        // spreads the partly filled chunks of small instances over the XCDs)
        e.blk0[c] = e.p.tl.xcd != 0 ? (h0[c] + 7) / 8 * 8 + q % 8 : h0[c];
        e.nblk[c] = gnor::class_blocks(e.p.tl, c) + (c == 0 ? 1 : 0);  // + auxiliary block
        h0[c] = e.blk0[c] + e.nblk[c];
      }
      e.dblk0 = d0;
      e.dnblk = s->mon.nfreq > 0 ? gnor::dft_blocks(e.d, e.f) : 0;
      d0 += e.dnblk;
      // step form 3: the metal tiles take one pass unless the instance has
      // critical points (as for one simulation); the TF/SF launch covers the
      // instance's shell where one of its one-pass classes meets it; the
      // node-scalar launch covers the metal sub-grid of instances whose metal
      // tiles take one pass
      e.two_sweep2 = (b->form != 3 || s->mat.ncp > 0) ? 1 : 0;
      const bool shell = s->tf_shell[0] || s->tf_shell[1] || (s->tf_shell[2] && !e.two_sweep2);
      e.fblk0 = f0;
      e.fnblk = (e.p.tfsf && shell) ? gnor::tfsf_fix_blocks(e.p.tf_lo, e.p.tf_hi) : 0;
      f0 += e.fnblk;
      e.sblk0 = s0;
      e.snblk = (!e.two_sweep2 && s->any_metal) ? gnor::node_blocks(e.p.mn) : 0;
      s0 += e.snblk;
    }
    for (int c = 0; c < gnor::kClasses; ++c) b->hblocks[c] = h0[c];
    b->dblocks = d0;
    b->fblocks = f0;
    b->sblocks = s0;
  }
  b->entry_bytes = sizeof(gnor::BatchEntry<T>);
  BHIPCHECK(b, hipMemcpy(b->tab, tab.data(), tab.size() * b->entry_bytes, hipMemcpyHostToDevice));
  return GNOR_OK;
}

// device bytes of the two parameter tables of a batch of n instances
size_t batch_table_bytes(int n, bool fp32) {
  const size_t e = fp32 ? sizeof(gnor::BatchEntry<float>) : sizeof(gnor::BatchEntry<double>);
  return 2 * (size_t)n * e;
}

template <class T>
void batch_enqueue(gnor_batch* b, int64_t n0, int64_t count, hipStream_t st) {
  const gnor::BatchEntry<T>* tabs = reinterpret_cast<const gnor::BatchEntry<T>*>(b->tab);
  for (int64_t q = 0; q < count; ++q) {
    const int64_t n = n0 + q;
    const gnor::BatchEntry<T>* t = tabs + (size_t)(n & 1) * b->n;
    const int sub = (int)q;
    auto classes = [&](auto launch) {
      if (!b->concurrent) {
        for (int c = 0; c < gnor::kClasses; ++c) launch(c, st);
        return;
      }
      (void)hipEventRecord(b->ev_fork, st);
      for (int q2 = 0; q2 < 2; ++q2) (void)hipStreamWaitEvent(b->side[q2], b->ev_fork, 0);
      launch(0, st);
      launch(3, st);
      launch(1, b->side[0]);
      launch(2, b->side[1]);
      for (int q2 = 0; q2 < 2; ++q2) {
        (void)hipEventRecord(b->ev_join[q2], b->side[q2]);
        (void)hipStreamWaitEvent(st, b->ev_join[q2], 0);
      }
    };
    if (b->form == 3) {
      // the tiles without metal in one pass beside the metal classes' H
      // sweeps; then the TF/SF terms at the one-pass points, the lines'
      // step, and the metal classes' E/J sweeps
      // (the metal tiles of instances with critical points keep the two
      // sweeps: in those launches the other instances' blocks exit at once,
      // and the reverse in the one-pass launch)
      classes([&](int c, hipStream_t q2) {
        if (c <= 1) {
          gnor::launch_fplain_batch<T>(t, b->n, b->hblocks[c], b->ty, c, b->stream_stores, q2);
        } else if (c == 2) {
          if (b->sblocks > 0) gnor::launch_nodes_batch<T>(t, b->n, b->sblocks, q2);
          if (!b->all_cp) gnor::launch_fplain_batch<T>(t, b->n, b->hblocks[2], b->ty, 2, b->stream_stores, q2);
          if (b->any_cp) gnor::launch_h_batch_class<T>(t, b->n, b->hblocks[2], b->ty, 2, b->stream_stores, q2);
        } else {
          gnor::launch_h_batch_class<T>(t, b->n, b->hblocks[c], b->ty, c, b->stream_stores, q2);
        }
      });
      gnor::launch_tfsf_fix_batch<T>(t, b->n, b->fblocks, st);
      gnor::launch_aux_batch<T>(t, b->n, sub, st);
      classes([&](int c, hipStream_t q2) {
        if (c == 3 || (c == 2 && b->any_cp))
          gnor::launch_ej_batch_class<T>(t, b->n, b->hblocks[c], b->ty, c, b->any_cp, b->stream_stores, q2);
      });
    } else {
      classes([&](int c, hipStream_t q2) {
        gnor::launch_h_batch_class<T>(t, b->n, b->hblocks[c], b->ty, c, b->stream_stores, q2);
      });
      classes([&](int c, hipStream_t q2) {
        gnor::launch_ej_batch_class<T>(t, b->n, b->hblocks[c], b->ty, c, b->any_cp, b->stream_stores, q2);
        // the lines' E beside the sweep, after the short metal class
        if (c == 2) gnor::launch_aux_e_batch<T>(t, b->n, sub, q2);
      });
    }
    if (b->any_dft && b->dblocks > 0) gnor::launch_dft_batch<T>(t, b->n, b->dblocks, sub, st);
    if (b->any_flux && (n % gnor::kFluxSlots) == gnor::kFluxSlots - 1)
      for (gnor_sim* s : b->sims)
        if (s->nsamp > 0) enqueue_flux_acc(s, sub, st);
  }
  gnor::launch_advance_batch<T>(tabs, b->n, count, st);
}

void batch_enqueue_any(gnor_batch* b, int64_t n0, int64_t count, hipStream_t st) {
  if (b->fp32) batch_enqueue<float>(b, n0, count, st);
  else batch_enqueue<double>(b, n0, count, st);
}

}  // namespace

extern "C" {

size_t gnor_batch_required_bytes(int32_t n, gnor_sim* const* sims) {
  if (n < 1 || !sims || !sims[0]) return 0;
  return batch_table_bytes(n, sims[0]->g.precision == GNOR_FP32);
}

}  // extern "C"

namespace {

// The batch that currently owns each device's static table (null: none).
std::mutex g_static_mutex;
gnor_batch* g_static_owner[64] = {};

// Shared by both creation calls.  concurrent: fork the class launches onto
// two side streams (the static variant creates no streams or events and
// launches the classes one after another on the caller's stream).
gnor_status batch_create_impl(int32_t n, gnor_sim* const* sims, void* stream, void* table,
                              bool concurrent, gnor_batch** out) {
  gnor_batch* b = new (std::nothrow) gnor_batch();
  if (!b) return GNOR_E_OUT_OF_MEMORY;
  b->n = n;
  b->concurrent = concurrent;
  for (int q = 0; q < n; ++q) {
    gnor_sim* s = sims[q];
    if (!s || !s->bound || s->maps.nmap > 0) { delete b; return GNOR_E_STATE; }  // no maps in batches
    if (s->g.total_field) { delete b; return GNOR_E_INVALID_ARG; }  // no plane source in batches
    if (q > 0 && (s->g.precision != sims[0]->g.precision || s->step != sims[0]->step ||
                  s->tile_ty != sims[0]->tile_ty)) {
      delete b;
      return GNOR_E_INVALID_ARG;  // one precision, one step index, one tile height
    }
    for (int r = 0; r < q; ++r)
      if (sims[r] == s) { delete b; return GNOR_E_INVALID_ARG; }
    b->sims.push_back(s);
    b->tiling.insert(b->tiling.end(), {s->tile_ty, s->tile_kz, s->tile_xcd});
    b->any_dft = b->any_dft || s->mon.nfreq > 0;
    b->any_flux = b->any_flux || s->nsamp > 0;
    b->any_cp = b->any_cp || s->mat.ncp > 0;
    b->all_cp = (q == 0 || b->all_cp) && s->mat.ncp > 0;
  }
  b->fp32 = sims[0]->g.precision == GNOR_FP32;
  b->tab = static_cast<char*>(table);
  b->ty = sims[0]->tile_ty;
  b->step = sims[0]->step;
  b->stream = reinterpret_cast<hipStream_t>(stream);
  if (!b->stream) {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) { delete b; return GNOR_E_DEVICE; }
    b->own_stream = true;
  }
  if (concurrent) {
    for (int q = 0; q < 2; ++q) {
      if (hipStreamCreateWithFlags(&b->side[q], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&b->ev_join[q], kJoinEventFlags) != hipSuccess) {
        gnor_batch_destroy(b);
        return GNOR_E_DEVICE;
      }
    }
    if (hipEventCreateWithFlags(&b->ev_fork, kJoinEventFlags) != hipSuccess) {
      gnor_batch_destroy(b);
      return GNOR_E_DEVICE;
    }
  }
  // the instances' own queued work must be complete before the batch runs;
  // their tile lists are those of the batch's step form (form 0 at first:
  // in form 3 metal tiles that meet only an x slab are listed with the metal
  // class, whose two-sweep kernels lack the x-slab terms)
  for (gnor_sim* s : b->sims) {
    if (hipStreamSynchronize(s->stream) != hipSuccess) { gnor_batch_destroy(b); return GNOR_E_DEVICE; }
    if (set_mode(s, 0) != GNOR_OK) { gnor_batch_destroy(b); return GNOR_E_DEVICE; }
  }
  const gnor_status st = b->fp32 ? batch_tables<float>(b) : batch_tables<double>(b);
  if (st != GNOR_OK) { gnor_batch_destroy(b); return st; }
  *out = b;
  return GNOR_OK;
}

}  // namespace

extern "C" {

gnor_status gnor_batch_create(int32_t n, gnor_sim* const* sims, void* stream, void* table,
                              size_t table_bytes, gnor_batch** out) {
  if (!out || n < 1 || !sims || !table) return GNOR_E_INVALID_ARG;
  *out = nullptr;
  if (!sims[0] || table_bytes < batch_table_bytes(n, sims[0]->g.precision == GNOR_FP32) ||
      (((uintptr_t)table) & 255u))
    return GNOR_E_BUFFER_TOO_SMALL;
  return batch_create_impl(n, sims, stream, table, true, out);
}

gnor_status gnor_batch_create_static(int32_t n, gnor_sim* const* sims, void* stream, gnor_batch** out) {
  if (!out || n < 1 || !sims || !sims[0] || !stream) return GNOR_E_INVALID_ARG;
  *out = nullptr;
  if (n > gnor::kStaticBatchMax) return GNOR_E_BUFFER_TOO_SMALL;
  const size_t need = batch_table_bytes(n, sims[0]->g.precision == GNOR_FP32);
  if (need > gnor::kStaticTableBytes) return GNOR_E_BUFFER_TOO_SMALL;
  int dev = 0;
  void* tab = nullptr;
  if (gnor::static_table_address(&dev, &tab) != hipSuccess) return GNOR_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_static_mutex);
  // the batch that held this device's table must have finished reading it
  gnor_batch* prev = g_static_owner[dev];
  if (prev && hipStreamSynchronize(prev->stream) != hipSuccess) return GNOR_E_DEVICE;
  gnor_batch* b = nullptr;
  const gnor_status st = batch_create_impl(n, sims, stream, tab, false, &b);
  if (st != GNOR_OK) return st;
  b->static_dev = dev;
  g_static_owner[dev] = b;  // `prev` (if any) is refused from now on
  *out = b;
  return GNOR_OK;
}

void gnor_batch_destroy(gnor_batch* b) {
  if (!b) return;
  if (b->static_dev >= 0) {
    // its queued kernels read the device's static table: let them finish
    std::lock_guard<std::mutex> lock(g_static_mutex);
    (void)hipStreamSynchronize(b->stream);
    if (g_static_owner[b->static_dev] == b) g_static_owner[b->static_dev] = nullptr;
  }
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  for (int q = 0; q < 2; ++q) {
    if (b->side[q]) (void)hipStreamDestroy(b->side[q]);
    if (b->ev_join[q]) (void)hipEventDestroy(b->ev_join[q]);
  }
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  delete b;
}

gnor_status gnor_batch_set_form(gnor_batch* b, int32_t form) {
  if (!b || (form != 0 && form != 3)) return GNOR_E_INVALID_ARG;
  if (form != b->form) {
    // the queued steps of the old form finish first (they read the same state
    // and the parameter tables, which name the form's launches per instance)
    BHIPCHECK(b, hipStreamSynchronize(b->stream));
    b->form = form;
    // the instances take the form too (their tile lists follow it)
    for (gnor_sim* s : b->sims)
      if (set_mode(s, form) != GNOR_OK) return bfail(b, GNOR_E_DEVICE, "re-planning an instance's tiles failed");
    const gnor_status st = b->fp32 ? batch_tables<float>(b) : batch_tables<double>(b);
    if (st != GNOR_OK) return st;
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_steps = 0;
  }
  return GNOR_OK;
}

gnor_status gnor_batch_set_graph_chunk(gnor_batch* b, int32_t steps) {
  if (!b || steps < 0 || (steps & 1)) return GNOR_E_INVALID_ARG;
  b->graph_chunk = steps;
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  b->graph_steps = 0;
  return GNOR_OK;
}

gnor_status gnor_batch_run(gnor_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) return GNOR_E_INVALID_ARG;
  if (b->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mutex);
    if (g_static_owner[b->static_dev] != b)
      return bfail(b, GNOR_E_STATE, "a later gnor_batch_create_static on this GPU took over the static table");
  }
  for (size_t q = 0; q < b->sims.size(); ++q) {
    const gnor_sim* s = b->sims[q];
    if (s->step != b->step) return bfail(b, GNOR_E_STATE, "an instance was stepped outside the batch");
    if (s->tile_ty != b->tiling[3 * q] || s->tile_kz != b->tiling[3 * q + 1] ||
        s->tile_xcd != b->tiling[3 * q + 2])
      return bfail(b, GNOR_E_STATE, "an instance's tiling changed after the batch was created");
  }
  const int align = b->any_flux ? gnor::kFluxSlots : 2;
  int chunk = b->graph_chunk > 0 ? std::max(align, b->graph_chunk / align * align) : 0;
  int64_t left = nsteps;
  while (left > 0) {
    if (chunk > 0 && (b->step % align) == 0 && left >= chunk) {
      if (!b->graph || b->graph_steps != chunk) {
        if (b->graph) (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
        hipGraph_t gr = nullptr;
        BHIPCHECK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        batch_enqueue_any(b, 0, chunk, b->stream);
        BHIPCHECK(b, hipStreamEndCapture(b->stream, &gr));
        const hipError_t e = hipGraphInstantiate(&b->graph, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) {
          b->graph = nullptr;
          return bfail(b, GNOR_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        b->graph_steps = chunk;
      }
      BHIPCHECK(b, hipGraphLaunch(b->graph, b->stream));
      b->step += chunk;
      left -= chunk;
    } else {
      int64_t m = left;
      if (chunk > 0) {
        const int64_t to_align = (align - (b->step % align)) % align;
        m = to_align > 0 ? std::min(left, to_align) : left;
      }
      batch_enqueue_any(b, b->step, m, b->stream);
      BHIPCHECK(b, hipGetLastError());
      b->step += m;
      left -= m;
    }
  }
  for (gnor_sim* s : b->sims) s->step = b->step;
  return GNOR_OK;
}

gnor_status gnor_batch_synchronize(gnor_batch* b) {
  if (!b) return GNOR_E_INVALID_ARG;
  BHIPCHECK(b, hipStreamSynchronize(b->stream));
  return GNOR_OK;
}

const char* gnor_batch_last_error(const gnor_batch* b) { return b ? b->last_error.c_str() : "null batch"; }

}  // extern "C"

// ============================================================ gradients
// Objective: sigma_ext(omega_m) of a run of nsteps steps from rest, as
// returned by gnor_get_spectra.  Its gradient with respect to the design
// densities is the exact discrete adjoint of the run: a forward pass keeps a
// full-state checkpoint every ckpt_every steps; the backward pass, segment by
// segment from the last, restores the segment's checkpoint, recomputes its
// steps while storing the design region's E and dQ, then transposes the
// segment's steps in reverse order (gnor_adjoint.hip).
namespace {

int nz_of(const gnor_sim* s) { return s->g.nz; }

// Workspace of a gradient, carved from the caller's buffer: checkpoints,
// then (zeroed) the adjoint fields and CPML memory, the gradient's incident
// transform and the design region's stored forward values.
struct GradPlan {
  size_t ck = 0, zero = 0, Eb[3] = {}, Hb[3] = {}, D[6] = {}, Ob[3] = {}, Jb[3] = {}, dQb[3] = {};
  size_t PPb = 0, PJb = 0, phi = 0, psiE[3][2] = {}, psiH[3][2] = {}, B = 0, fE = 0, fdQ = 0;
  size_t total = 0;
};

GradPlan plan_gradient(const gnor_sim* s, int64_t nsteps, int C) {
  GradPlan G;
  const size_t N = s->N, M = s->M, w = s->elem;
  const gnor_grid_desc& g = s->g;
  const int np = g.npml;
  const size_t nd = (size_t)(s->dhi[0] - s->dlo[0]) * (s->dhi[1] - s->dlo[1]) * (s->dhi[2] - s->dlo[2]);
  const size_t sbytes = s->L.state_end - s->L.state_begin;
  const size_t nseg = (size_t)((nsteps + C - 1) / C);
  Planner P;
  G.ck = P.take(sbytes * nseg);
  G.zero = P.off;  // everything from here on is zeroed
  for (int c = 0; c < 3; ++c) { G.Eb[c] = P.take(N * w); G.Hb[c] = P.take(N * w); }
  for (int q = 0; q < 6; ++q) G.D[q] = P.take(N * w);
  for (int c = 0; c < 3; ++c) { G.Ob[c] = P.take(M * w); G.Jb[c] = P.take(M * w); G.dQb[c] = P.take(M * w); }
  G.PPb = P.take(M * w); G.PJb = P.take(M * w); G.phi = P.take(M * w);
  const size_t nxs = g.nx, nys = g.ny, nzs = g.nz;
  const size_t slab[3] = {nzs * nys * 2 * np, nzs * 2 * np * nxs, 2 * np * nys * nxs};
  for (int a = 0; a < 3; ++a)
    for (int t = 0; t < 2; ++t) {
      G.psiE[a][t] = P.take(slab[a] * w + 8);
      G.psiH[a][t] = P.take(slab[a] * w + 8);
    }
  G.B = P.take((size_t)2 * nz_of(s) * 8);
  G.fE = P.take((size_t)(C + 2) * 3 * nd * w);
  G.fdQ = P.take((size_t)C * 3 * nd * w);
  G.total = P.off;
  return G;
}

template <class T>
gnor_status gradient_impl(gnor_sim* s, int64_t nsteps, int C, int m, char* ws, double* objective,
                          double* grad_dev) {
  const gnor_grid_desc& g = s->g;
  const int nz = g.nz, nf = s->mon.nfreq;
  const int dn[3] = {s->dhi[0] - s->dlo[0], s->dhi[1] - s->dlo[1], s->dhi[2] - s->dlo[2]};
  const size_t nd = (size_t)dn[0] * dn[1] * dn[2];
  const size_t sbytes = s->L.state_end - s->L.state_begin;
  const int nseg = (int)((nsteps + C - 1) / C);
  const hipStream_t st = s->stream;
  const GradPlan G = plan_gradient(s, nsteps, C);
  const size_t o_ck = G.ck, o_zero = G.zero, total = G.total;
  HIPCHECK(s, hipMemsetAsync(ws + o_zero, 0, total - o_zero, st));
  HIPCHECK(s, hipMemsetAsync(grad_dev, 0, nd * 8, st));

  // ---- forward pass with checkpoints
  gnor_status rc = gnor_reset(s);
  if (rc != GNOR_OK) return rc;
  for (int seg = 0; seg < nseg; ++seg) {
    const int64_t len = std::min<int64_t>(C, nsteps - (int64_t)seg * C);
    HIPCHECK(s, hipMemcpyAsync(ws + o_ck + sbytes * seg, s->dev + s->L.state_begin, sbytes,
                               hipMemcpyDeviceToDevice, st));
    rc = gnor_run(s, len);
    if (rc != GNOR_OK) return rc;
  }
  std::vector<double> ext(nf), are((size_t)nz * nf), aim((size_t)nz * nf), bre((size_t)nz * nf),
      bim((size_t)nz * nf);
  rc = gnor_get_spectra(s, nullptr, ext.data(), nullptr, nullptr);
  if (rc != GNOR_OK) return rc;
  rc = gnor_get_dft(s, are.data(), aim.data(), bre.data(), bim.data());
  if (rc != GNOR_OK) return rc;
  if (objective) *objective = ext[m];
  std::vector<double> B(2 * (size_t)nz);
  for (int k = 0; k < nz; ++k) {
    B[k] = bre[(size_t)k * nf + m];
    B[nz + k] = bim[(size_t)k * nf + m];
  }
  const double b2 = B[s->mon.norm_k] * B[s->mon.norm_k] + B[nz + s->mon.norm_k] * B[nz + s->mon.norm_k];
  HIPCHECK(s, hipMemcpy(ws + G.B, B.data(), B.size() * 8, hipMemcpyHostToDevice));

  // ---- adjoint
  gnor::AdjParams<T> A{};
  A.p = make_params<T>(s, 0);
  for (int c = 0; c < 3; ++c) {
    A.Eb[c] = reinterpret_cast<T*>(ws + G.Eb[c]);
    A.Hb[c] = reinterpret_cast<T*>(ws + G.Hb[c]);
    A.Ob[c] = reinterpret_cast<T*>(ws + G.Ob[c]);
    A.Jb[c] = reinterpret_cast<T*>(ws + G.Jb[c]);
    A.dQb[c] = reinterpret_cast<T*>(ws + G.dQb[c]);
  }
  for (int q = 0; q < 6; ++q) A.D[q] = reinterpret_cast<T*>(ws + G.D[q]);
  A.PPb = reinterpret_cast<T*>(ws + G.PPb);
  A.PJb = reinterpret_cast<T*>(ws + G.PJb);
  A.phiJb = reinterpret_cast<T*>(ws + G.phi);
  for (int a = 0; a < 3; ++a)
    for (int t = 0; t < 2; ++t) {
      A.psiEb[a][t] = reinterpret_cast<T*>(ws + G.psiE[a][t]);
      A.psiHb[a][t] = reinterpret_cast<T*>(ws + G.psiH[a][t]);
    }
  for (int d = 0; d < 3; ++d) { A.dlo[d] = s->dlo[d]; A.dn[d] = dn[d]; }
  A.fE = reinterpret_cast<const T*>(ws + G.fE);
  A.fdQ = reinterpret_cast<const T*>(ws + G.fdQ);
  A.grad = grad_dev;
  A.dt = s->dt;
  A.omega = s->omega[m];
  // sigma_ext = eta0 dx^3 sum_k Re(A conj B) / |B(norm_k)|^2 with A = (eps0/dt) sum_n dt e^{i w t} J~-sums
  A.CL = eta0() * g.dx * g.dx * g.dx * s->dt * (eps0() / s->dt) / b2;
  A.Bre = reinterpret_cast<const double*>(ws + G.B);
  A.Bim = A.Bre + nz;
  gnor::launch_adjoint_source<T>(A, nsteps - 1, st);
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int64_t n0 = (int64_t)seg * C;
    const int len = (int)std::min<int64_t>(C, nsteps - n0);
    HIPCHECK(s, hipMemcpyAsync(s->dev + s->L.state_begin, ws + o_ck + sbytes * seg, sbytes,
                               hipMemcpyDeviceToDevice, st));
    s->step = n0;
    const int par = (int)(n0 & 1);
    gnor::launch_store_design<T>(A, 1, ptr<T>(s, s->L.E[par ^ 1][0]), ptr<T>(s, s->L.E[par ^ 1][1]),
                                 ptr<T>(s, s->L.E[par ^ 1][2]), 0, st);
    gnor::launch_store_design<T>(A, 1, ptr<T>(s, s->L.E[par][0]), ptr<T>(s, s->L.E[par][1]),
                                 ptr<T>(s, s->L.E[par][2]), 1, st);
    for (int t = 0; t < len; ++t) {
      enqueue_steps_eager(s, s->step, 1, st, false);
      s->step += 1;
      const int q = (int)((n0 + t + 1) & 1);
      A.t_idx = t;
      gnor::launch_store_design<T>(A, 0, ptr<T>(s, s->L.E[q][0]), ptr<T>(s, s->L.E[q][1]),
                                   ptr<T>(s, s->L.E[q][2]), t + 2, st);
    }
    for (int t = len - 1; t >= 0; --t) {
      A.lev_base = t + 1;
      A.t_idx = t;
      gnor::launch_adjoint_step<T>(A, n0 + t - 1, st);
    }
    HIPCHECK(s, hipGetLastError());
  }
  HIPCHECK(s, hipStreamSynchronize(st));
  return GNOR_OK;
}

}  // namespace

extern "C" size_t gnor_gradient_required_bytes(const gnor_sim* s, int64_t nsteps, int32_t ckpt_every) {
  if (!s || !s->bound || !s->design || nsteps < 1 || ckpt_every < 1) return 0;
  return plan_gradient(s, nsteps, ckpt_every).total + 256;
}

extern "C" gnor_status gnor_gradient(gnor_sim* s, int64_t nsteps, int32_t ckpt_every, int32_t m_target,
                                     void* workspace, size_t workspace_bytes, double* objective,
                                     double* grad) {
  gnor_status st = check_ready(s);
  if (st != GNOR_OK) return st;
  if (!s->design) return fail(s, GNOR_E_STATE, "no design region (gnor_set_design)");
  if (!grad || nsteps < 1 || ckpt_every < 1) return fail(s, GNOR_E_INVALID_ARG, "bad gradient arguments");
  if (!workspace || (((uintptr_t)workspace) & 255u))
    return fail(s, GNOR_E_INVALID_ARG, "workspace must be a 256-byte aligned device buffer");
  if (workspace_bytes < plan_gradient(s, nsteps, ckpt_every).total)
    return fail(s, GNOR_E_BUFFER_TOO_SMALL, "workspace smaller than gnor_gradient_required_bytes");
  if (m_target < 0 || m_target >= s->mon.nfreq) return fail(s, GNOR_E_INVALID_ARG, "m_target outside the frequency list");
  if (s->mon.dft_every > 1) return fail(s, GNOR_E_INVALID_ARG, "gradients need dft_every = 1");
  if (s->mat.ncp > 0) return fail(s, GNOR_E_INVALID_ARG, "gradients do not cover critical points");
  if (s->g.eps_substrate > 0.0) return fail(s, GNOR_E_INVALID_ARG, "gradients do not cover a substrate");
  if (s->maps.nmap > 0) return fail(s, GNOR_E_STATE, "gradients replay steps: turn the maps off");
  if (s->mat.eps_inf != s->g.eps_background)
    return fail(s, GNOR_E_INVALID_ARG, "gradients need eps_inf = eps_background");
  // the backward pass needs the stored Q of each recomputed step, so the whole
  // gradient (forward pass included) runs on the two-sweep kernels
  const int mode = s->mode;
  st = set_mode(s, 0);
  if (st != GNOR_OK) return st;
  char* ws = static_cast<char*>(workspace);
  st = s->g.precision == GNOR_FP32 ? gradient_impl<float>(s, nsteps, ckpt_every, m_target, ws, objective, grad)
                                   : gradient_impl<double>(s, nsteps, ckpt_every, m_target, ws, objective, grad);
  const gnor_status st2 = set_mode(s, mode);
  return st != GNOR_OK ? st : st2;
}

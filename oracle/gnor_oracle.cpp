// GNOR-FDTD oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, FP64 CPU implementation of the hydrodynamic (nonlocal Drude
// and GNOR) FDTD time step of Baxter, Cala Lesina & Ramunno, "Parallel FDTD
// modelling of nonlocality in plasmonics" (arXiv:2005.06997).  Only the test
// suite, the smoke check and the benchmark's CPU-baseline leg may load it.
// It shares no code, header or constant table with the GPU library; every
// formula here is written from the paper (or, where the paper is silent, from
// the textbook definition named beside it).
//
// What it follows literally:
//   * Yee positions of E, H and P: Sec. III, Table I.
//   * Update order H -> E -> P_CP -> P_f (f1, f2, f3, f4): Sec. III.
//   * N critical points (bound electrons), Eq. (CritPoint): the f3 update
//     Eq. (critpointupdate) with C_p, C_1p .. C_5p, and their terms in the E
//     update, obtained by putting Eq. (critpointupdate) into Eq.
//     (discreteamperes) as Sec. III describes.  Two readings (the printed
//     coefficients disagree with that derivation and with Eq. (CritPoint)):
//     the sum of C_4p enters the E^n coefficient with a minus sign, and the
//     sin(phi_p) part of C_3p and C_5p is eps0 A_p Omega_p sin(phi_p) /
//     (dt C_p), which makes the discrete susceptibility tend to Eq.
//     (CritPoint) as dt -> 0.  The poles act where P_f does (the metal), with
//     the metal weight scaling A_p.
//   * P_f update: Eq. (NonlocalUpdate) with D1, D2, D3, D_NL, D_d, and its
//     GNOR form Eq. (GNORUpdate) with D_G1, D_G2 and the BDF2 time derivative
//     of grad(div P): Sec. III.
//   * grad(div P) at the three P positions written out term by term as in
//     Eq. (GradDiv), with P = 0 outside the metal (Pekar condition, end of
//     Sec. III), evaluated only where P_f is updated.
//   * E update from the discrete Ampere law Eq. (discreteamperes) combined
//     with the P_f update (the two E-update equations of Sec. III), using the
//     stored histories E^{n-1}, P^{n-1}, GD^{n-1}, GD^{n-2} ("GNOR requires
//     additional memory", Sec. III).
// Where the paper is silent (its Sec. V only names them), the following are
// textbook constructions:
//   * Convolutional PML (Roden-Gedney recursive convolution, polynomial
//     grading) behind which the domain is closed by PEC walls.
//   * Total-field/scattered-field plane-wave source for x-polarised light
//     travelling along +z, fed by a 1D auxiliary Yee line with the same dx,
//     dt and background.
//   * Running discrete Fourier transforms (e^{+i w t}, factor dt) of the
//     induced current (extinction by the volume optical theorem), of the
//     incident field, and of tangential E and H on two flux boxes
//     (absorption: total field inside the TF box; scattering: scattered
//     field outside it).
//   * Total-field operation, for metal that reaches the boundary (a plasmonic
//     substrate) where TF/SF cannot hold it: a soft plane source on E_x of
//     one node plane, and the remedy the end of Sec. III gives -- metal
//     inside the absorbing layers follows the local (LRA) Drude model, the
//     nonlocal model holds everywhere else.
//   * Near-field and free-electron density maps on one grid plane (the field
//     and density distributions of Sec. V): running transforms of E_x, E_y,
//     E_z at their Yee points of the plane (stamped (n+1) dt) and of the
//     density n - n0 = div P_f / e of Eq. (Nsol) at its nodes (backward
//     differences of P_f^n, stamped n dt), every map_every steps.
// A templated scalar lets the same code run on dual numbers, which gives the
// exact directional derivative of an objective with respect to the metal
// weights (forward-mode differentiation).
//
// Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -shared -fPIC

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace {

// Physical constants (SI).  mu0 is the CODATA 2018 value.
constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 1.25663706212e-6;
inline double eps0() { return 1.0 / (kMu0 * kC0 * kC0); }
inline double eta0() { return std::sqrt(kMu0 / eps0()); }

// Auxiliary 1D incident line: CPML thickness, offset of 3D plane k = 0, and
// the soft-source cell.  These are part of the problem definition.
constexpr int kAuxPml = 20;
constexpr int kAuxOff = 25;
constexpr int kAuxSrc = 22;

// ---------------------------------------------------------------- dual numbers
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}  // NOLINT(implicit)
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
inline Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
inline Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
inline Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
inline Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
inline Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
inline Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
inline Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
inline double der(double) { return 0.0; }
inline double der(Dual x) { return x.d; }

}  // namespace

extern "C" {

// Problem description (the oracle's own; mirrored by oracle/oracle.py).
typedef struct {
  int32_t nx, ny, nz;
  int32_t periodic;  // 1: periodic in all three axes (test mode; npml = 0, no TF/SF)
  double dx, courant, eps_b;
  int32_t npml;
  double pml_order, pml_sigma_scale, pml_kappa_max, pml_alpha_max;
  int32_t tfsf;
  int32_t tf_lo[3], tf_hi[3];
  int32_t model;  // 0: GNOR update, 1: nonlocal-Drude update
  double wp, gamma, beta, diff, eps_inf;
  int32_t src_kind;  // 0 none, 1 modulated Gaussian, 2 raised cosine
  double e0, omega_c, tau, t0, omega_max;
  int32_t nfreq, dft_every, norm_k;
  int32_t flux;
  int32_t abs_lo[3], abs_hi[3], sca_lo[3], sca_hi[3];
  int32_t threads;
  // critical points (Eq. CritPoint): ncp poles, A_p, Omega_p [rad/s],
  // Gamma_p [rad/s], phi_p [rad]
  int32_t ncp;
  double cp_A[4], cp_Omega[4], cp_Gamma[4], cp_phi[4];
  // maps: plane map_index normal to map_axis, nmap frequencies, every
  // map_every steps
  int32_t map_axis, map_index, nmap, map_every;
  double map_omega[8];
  // dielectric substrate: the half-space z > sub_k (node planes) has relative
  // permittivity eps_sub when eps_sub > 0 (0: uniform background eps_b)
  double eps_sub;
  int32_t sub_k;
  // total-field operation (no TF/SF; metal may reach into the absorbing
  // layers, where it follows the local Drude model): a soft plane source on
  // E_x of node plane source_k, with the pulse the 1D line also takes at
  // that plane (the line then only gives the incident reference transform)
  int32_t total_field, source_k;
  // periodic in x and y (CPML only on the z faces): a laterally infinite
  // layered problem on a grid a few cells wide (test mode)
  int32_t periodic_xy;
} or_config;

}  // extern "C"

namespace {

template <class R>
struct Sim {
  or_config c{};
  int nx = 0, ny = 0, nz = 0;
  size_t N = 0;
  double dt = 0, dx = 0;
  long step = 0;
  // coefficients of the P_f update (Sec. III)
  double Dd = 0, D1 = 0, D2 = 0, D3 = 0, DNL = 0, DG1 = 0, DG2 = 0, eta = 0;
  std::vector<uint8_t> mask;  // bit c: P_c is updated at this Yee point
  std::vector<R> w;           // per-cell weight of the metal's wp^2, beta^2, D
  std::vector<R> E[3], Em[3], H[3], P[3], Pm[3], GD[3], GD1[3], GD2[3];
  // critical points: P_CP,p^n and P_CP,p^{n-1}, and the coefficients of
  // Eq. (critpointupdate)
  int ncp = 0;
  std::vector<R> PC[4][3], PCm[4][3];
  double C1p[4] = {}, C2p[4] = {}, C3p[4] = {}, C4p[4] = {}, C5p[4] = {};
  std::vector<R> psiE[3][3], psiH[3][3];  // psi[component][derivative axis]
  // CPML coefficients per axis at integer (e) and half-integer (h) positions
  std::vector<double> be[3], ae[3], ke[3], bh[3], ah[3], kh[3];
  // 1D auxiliary line
  int n1 = 0;
  std::vector<double> e1, h1, pe1, ph1, be1, ae1, ke1, bh1, ah1, kh1;
  // DFT
  std::vector<double> omega;
  std::vector<R> Are, Aim;          // [k][m] induced-current transform per plane
  std::vector<double> Bre, Bim;     // [k][m] incident-field transform per plane
  struct Face {
    int a, side, p;                 // normal axis, side (-1 lo, +1 hi), plane
    int b, cc;                      // tangential axes (cyclic after a)
    int lob, hib, loc, hic;
    std::vector<R> Eb_re, Eb_im, Hc_re, Hc_im, Ec_re, Ec_im, Hb_re, Hb_im;
  };
  std::vector<Face> faces[2];       // 0: absorption box, 1: scattering box
  // maps: [quantity][m][v][u], quantity Re/Im of E_x, E_y, E_z, n - n0
  int nmap = 0, mu = 0, mv = 0;
  std::vector<R> maps;
  std::vector<double> map_inc;      // [m][re, im] incident transform at norm_k

  size_t id(int i, int j, int k) const { return ((size_t)k * ny + j) * nx + i; }
  // is axis `a` periodic (all three in periodic mode; x and y with periodic_xy)
  bool per(int a) const { return c.periodic || (c.periodic_xy && a < 2); }
  int wrap(int i, int n, int a) const { return per(a) ? ((i % n) + n) % n : i; }
  R at(const std::vector<R>& a, int i, int j, int k) const {
    i = wrap(i, nx, 0); j = wrap(j, ny, 1); k = wrap(k, nz, 2);
    if (i < 0 || j < 0 || k < 0 || i >= nx || j >= ny || k >= nz) {
      std::fprintf(stderr, "oracle: index (%d,%d,%d) out of range\n", i, j, k);
      std::abort();
    }
    return a[id(i, j, k)];
  }

  // ---------------------------------------------------------- CPML profiles
  // Polynomial grading of order m over npml cells; depth measured at each
  // field's own position; sigma_max = scale (m+1) / (eta0 dx sqrt(eps_b)).
  void pml_coeffs(double depth, int L, double& b, double& a, double& kinv) const {
    b = 1.0; a = 0.0; kinv = 1.0;
    if (L <= 0 || depth <= 0.0) return;
    const double m = c.pml_order;
    const double smax = c.pml_sigma_scale * (m + 1.0) / (eta0() * dx * std::sqrt(c.eps_b));
    const double u = depth / L;
    const double sigma = smax * std::pow(u, m);
    const double kappa = 1.0 + (c.pml_kappa_max - 1.0) * std::pow(u, m);
    const double alpha = c.pml_alpha_max * (1.0 - u);
    b = std::exp(-(sigma / kappa + alpha) * dt / eps0());
    a = sigma > 0.0 ? sigma * (b - 1.0) / (kappa * (sigma + kappa * alpha)) : 0.0;
    kinv = 1.0 / kappa;
  }
  static double depth_at(double x, int n, int L) {
    // x in cells; nodes run 0..n-1; absorbing layers [0, L] and [n-1-L, n-1]
    double d = 0.0;
    if (x < L) d = L - x;
    if (x > (n - 1 - L)) d = x - (n - 1 - L);
    return d;
  }

  // Background permittivity at an E point: eps_b, or eps_sub beyond the
  // substrate plane.  E_x and E_y lie on the node planes (on the interface
  // plane itself: the mean of the two), E_z half a cell above its node.
  double eps_at(int comp, int k) const {
    if (!(c.eps_sub > 0.0)) return c.eps_b;
    if (comp == 2) return (k + 0.5 > c.sub_k) ? c.eps_sub : c.eps_b;
    if (k > c.sub_k) return c.eps_sub;
    if (k == c.sub_k) return 0.5 * (c.eps_b + c.eps_sub);
    return c.eps_b;
  }

  double source(double t) const {
    if (c.src_kind == 1) {
      const double u = (t - c.t0) / c.tau;
      return c.e0 * std::exp(-u * u) * std::sin(c.omega_c * (t - c.t0));
    }
    if (c.src_kind == 2) {
      if (t < 0.0 || t > 2.0 * M_PI / c.omega_max) return 0.0;
      const double s = 0.5 * (1.0 - std::cos(c.omega_max * t));
      return c.e0 * s * s * s;
    }
    return 0.0;
  }

  void init(const or_config& cfg, const uint8_t* m, const R* weight, const double* om) {
    c = cfg;
    nx = c.nx; ny = c.ny; nz = c.nz;
    N = (size_t)nx * ny * nz;
    dx = c.dx;
    dt = c.courant * dx / kC0;
    // Sec. III, Eqs. (d1)-(dd) and the GNOR coefficients D_G1, D_G2.
    Dd = c.gamma / (2.0 * dt) + 1.0 / (dt * dt);
    D1 = 2.0 / (Dd * dt * dt);
    D2 = (c.gamma / (2.0 * dt) - 1.0 / (dt * dt)) / Dd;
    D3 = eps0() * c.wp * c.wp / (4.0 * Dd);
    DNL = c.beta * c.beta / Dd;
    eta = c.beta * c.beta + c.diff * c.gamma;
    DG1 = eta / Dd;
    DG2 = c.diff / (2.0 * dt * Dd);
    // f3 coefficients, Eq. (critpointupdate) (sin term and sign: see top)
    ncp = c.ncp < 0 ? 0 : (c.ncp > 4 ? 4 : c.ncp);
    for (int q = 0; q < ncp; ++q) {
      const double A = c.cp_A[q], Om = c.cp_Omega[q], Ga = c.cp_Gamma[q], ph = c.cp_phi[q];
      const double s2 = Om * Om + Ga * Ga;
      const double Cp = Ga / dt + 1.0 / (dt * dt) + s2 / 4.0;
      C1p[q] = (2.0 / (dt * dt) - s2 / 2.0) / Cp;
      C2p[q] = (Ga / dt - 1.0 / (dt * dt) - s2 / 4.0) / Cp;
      C4p[q] = eps0() * A * Om * (Om * std::cos(ph) - Ga * std::sin(ph)) / Cp;
      C3p[q] = C4p[q] / 2.0 - eps0() * A * Om * std::sin(ph) / (dt * Cp);
      C5p[q] = C4p[q] / 2.0 + eps0() * A * Om * std::sin(ph) / (dt * Cp);
    }
    mask.assign(m, m + N);
    w.assign(N, R(0.0));
    for (size_t p = 0; p < N; ++p) w[p] = weight ? weight[p] : R(mask[p] ? 1.0 : 0.0);
    for (int d = 0; d < 3; ++d) {
      E[d].assign(N, R(0.0)); Em[d].assign(N, R(0.0)); H[d].assign(N, R(0.0));
      P[d].assign(N, R(0.0)); Pm[d].assign(N, R(0.0)); GD[d].assign(N, R(0.0));
      GD1[d].assign(N, R(0.0)); GD2[d].assign(N, R(0.0));
      for (int e = 0; e < 3; ++e) { psiE[d][e].assign(N, R(0.0)); psiH[d][e].assign(N, R(0.0)); }
      for (int q = 0; q < ncp; ++q) { PC[q][d].assign(N, R(0.0)); PCm[q][d].assign(N, R(0.0)); }
    }
    const int ns[3] = {nx, ny, nz};
    for (int d = 0; d < 3; ++d) {
      const int n = ns[d];
      const int L = per(d) ? 0 : c.npml;
      be[d].resize(n); ae[d].resize(n); ke[d].resize(n);
      bh[d].resize(n); ah[d].resize(n); kh[d].resize(n);
      for (int i = 0; i < n; ++i) {
        pml_coeffs(depth_at((double)i, n, L), L, be[d][i], ae[d][i], ke[d][i]);
        pml_coeffs(depth_at(i + 0.5, n, L), L, bh[d][i], ah[d][i], kh[d][i]);
      }
    }
    n1 = nz + 2 * kAuxOff;
    e1.assign(n1, 0.0); h1.assign(n1, 0.0); pe1.assign(n1, 0.0); ph1.assign(n1, 0.0);
    be1.resize(n1); ae1.resize(n1); ke1.resize(n1); bh1.resize(n1); ah1.resize(n1); kh1.resize(n1);
    for (int q = 0; q < n1; ++q) {
      pml_coeffs(depth_at((double)q, n1, kAuxPml), kAuxPml, be1[q], ae1[q], ke1[q]);
      pml_coeffs(depth_at(q + 0.5, n1, kAuxPml), kAuxPml, bh1[q], ah1[q], kh1[q]);
    }
    omega.assign(om, om + c.nfreq);
    Are.assign((size_t)nz * c.nfreq, R(0.0)); Aim.assign((size_t)nz * c.nfreq, R(0.0));
    Bre.assign((size_t)nz * c.nfreq, 0.0); Bim.assign((size_t)nz * c.nfreq, 0.0);
    if (c.flux) {
      make_faces(0, c.abs_lo, c.abs_hi);
      make_faces(1, c.sca_lo, c.sca_hi);
    }
    nmap = c.nmap < 0 ? 0 : (c.nmap > 8 ? 8 : c.nmap);
    const int ua = c.map_axis == 0 ? 1 : 0, va = c.map_axis == 2 ? 1 : 2;
    mu = ns[ua]; mv = ns[va];
    maps.assign((size_t)8 * nmap * mu * mv, R(0.0));
    map_inc.assign((size_t)2 * nmap, 0.0);
    step = 0;
  }

  void make_faces(int box, const int32_t* lo, const int32_t* hi) {
    faces[box].clear();
    for (int a = 0; a < 3; ++a) {
      for (int side = -1; side <= 1; side += 2) {
        Face f;
        f.a = a; f.side = side; f.p = side < 0 ? lo[a] : hi[a];
        f.b = (a + 1) % 3; f.cc = (a + 2) % 3;
        f.lob = lo[f.b]; f.hib = hi[f.b]; f.loc = lo[f.cc]; f.hic = hi[f.cc];
        const size_t nb = f.hib - f.lob, nc = f.hic - f.loc;
        const size_t n_b = nb * (nc + 1) * c.nfreq;  // E_b / H_c points
        const size_t n_c = (nb + 1) * nc * c.nfreq;  // E_c / H_b points
        f.Eb_re.assign(n_b, R(0.0)); f.Eb_im.assign(n_b, R(0.0));
        f.Hc_re.assign(n_b, R(0.0)); f.Hc_im.assign(n_b, R(0.0));
        f.Ec_re.assign(n_c, R(0.0)); f.Ec_im.assign(n_c, R(0.0));
        f.Hb_re.assign(n_c, R(0.0)); f.Hb_im.assign(n_c, R(0.0));
        faces[box].push_back(std::move(f));
      }
    }
  }

  bool active(int comp, size_t p) const { return (mask[p] >> comp) & 1u; }

  // Update ranges.  With PEC walls behind the CPML the tangential E on the
  // outer node planes and the normal H on them stay zero; a field sitting
  // half a cell beyond the last node plane does not exist.
  void erange(int comp, int axis, int& lo, int& hi) const {
    const int n = axis == 0 ? nx : axis == 1 ? ny : nz;
    if (per(axis)) { lo = 0; hi = n - 1; return; }
    if (axis == comp) { lo = 0; hi = n - 2; } else { lo = 1; hi = n - 2; }
  }
  void hrange(int comp, int axis, int& lo, int& hi) const {
    const int n = axis == 0 ? nx : axis == 1 ? ny : nz;
    if (per(axis)) { lo = 0; hi = n - 1; return; }
    if (axis == comp) { lo = 1; hi = n - 2; } else { lo = 0; hi = n - 2; }
  }

  bool in_tf_e(int comp, int i, int j, int k) const {
    // E_comp at (i,j,k) belongs to the total-field region
    const int* lo = c.tf_lo; const int* hi = c.tf_hi;
    const int ii[3] = {i, j, k};
    for (int d = 0; d < 3; ++d) {
      const int h = (d == comp) ? hi[d] - 1 : hi[d];
      if (ii[d] < lo[d] || ii[d] > h) return false;
    }
    return true;
  }

  // ------------------------------------------------------------------- f1: H
  void update_h() {
    const double ch = dt / kMu0;
    const double einc_scale = dt / (kMu0 * dx);
    for (int comp = 0; comp < 3; ++comp) {
      const int a1 = (comp + 1) % 3, a2 = (comp + 2) % 3;
      int lo[3], hi[3];
      for (int d = 0; d < 3; ++d) hrange(comp, d, lo[d], hi[d]);
#pragma omp parallel for schedule(static) num_threads(c.threads > 0 ? c.threads : 1)
      for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
          for (int i = lo[0]; i <= hi[0]; ++i) {
            // curl_comp E = d_{a1} E_{a2} - d_{a2} E_{a1}; forward differences
            const int ii[3] = {i, j, k};
            int p1[3] = {i, j, k}, p2[3] = {i, j, k};
            p1[a1] += 1; p2[a2] += 1;
            const R d1 = (at(E[a2], p1[0], p1[1], p1[2]) - at(E[a2], i, j, k)) / dx;
            const R d2 = (at(E[a1], p2[0], p2[1], p2[2]) - at(E[a1], i, j, k)) / dx;
            const size_t p = id(i, j, k);
            R& s1 = psiH[comp][a1][p];
            R& s2 = psiH[comp][a2][p];
            s1 = bh[a1][ii[a1]] * s1 + ah[a1][ii[a1]] * d1;
            s2 = bh[a2][ii[a2]] * s2 + ah[a2][ii[a2]] * d2;
            const R curl = (kh[a1][ii[a1]] * d1 + s1) - (kh[a2][ii[a2]] * d2 + s2);
            H[comp][p] = H[comp][p] - ch * curl;
          }
    }
    if (c.tfsf && !c.periodic) {
      // Scattered-field H next to the TF box sees E_inc(k) on the TF side.
      const int* lo = c.tf_lo; const int* hi = c.tf_hi;
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0] - 1; ++i) {
          H[1][id(i, j, lo[2] - 1)] += einc_scale * e1[lo[2] + kAuxOff];
          H[1][id(i, j, hi[2])] -= einc_scale * e1[hi[2] + kAuxOff];
        }
      for (int k = lo[2]; k <= hi[2]; ++k)
        for (int i = lo[0]; i <= hi[0] - 1; ++i) {
          H[2][id(i, lo[1] - 1, k)] -= einc_scale * e1[k + kAuxOff];
          H[2][id(i, hi[1], k)] += einc_scale * e1[k + kAuxOff];
        }
    }
  }

  // 1D auxiliary line: H_inc^{n+1/2} from E_inc^n
  void update_h1() {
    const double ch = dt / (kMu0 * dx);
    for (int q = 0; q <= n1 - 2; ++q) {
      const double d = e1[q + 1] - e1[q];
      ph1[q] = bh1[q] * ph1[q] + ah1[q] * d;
      h1[q] -= ch * (kh1[q] * d + ph1[q]);
    }
  }
  // 1D auxiliary line: E_inc^{n+1} from H_inc^{n+1/2}, then the soft source
  void update_e1(double t_next) {
    for (int q = 1; q <= n1 - 2; ++q) {
      // line cell q carries E_x of grid plane q - kAuxOff (layered like the grid)
      const double ce = dt / (eps0() * eps_at(0, q - kAuxOff) * dx);
      const double d = h1[q] - h1[q - 1];
      pe1[q] = be1[q] * pe1[q] + ae1[q] * d;
      e1[q] -= ce * (ke1[q] * d + pe1[q]);
    }
    e1[c.total_field ? c.source_k + kAuxOff : kAuxSrc] += source(t_next);
  }

  // Total-field source: E_x^{n+1} += f(t_{n+1}) on node plane source_k (at
  // every E_x point the update reaches), after the E and P_f updates.
  void plane_source(double t_next) {
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) erange(0, d, lo[d], hi[d]);
    const int k = c.source_k;
    if (k < lo[2] || k > hi[2]) return;
    const double f = source(t_next);
    for (int j = lo[1]; j <= hi[1]; ++j)
      for (int i = lo[0]; i <= hi[0]; ++i) E[0][id(i, j, k)] += f;
  }

  // Inside the absorbing layers (cell (i, j, k) within npml cells of a
  // non-periodic face)?  In total-field operation metal there follows the
  // local Drude model (the remedy of the end of Sec. III for nonlocal
  // material that reaches the boundary).
  bool in_pml(int i, int j, int k) const {
    const int L = c.npml;
    if (L <= 0) return false;
    const int ii[3] = {i, j, k}, ns[3] = {nx, ny, nz};
    for (int d = 0; d < 3; ++d)
      if (!per(d) && (ii[d] < L || ii[d] > ns[d] - 1 - L)) return true;
    return false;
  }
  // weight of the nonlocal (beta^2, D) terms at cell (i, j, k)
  double nonlocal_on(int i, int j, int k) const { return (c.total_field && in_pml(i, j, k)) ? 0.0 : 1.0; }

  // ------------------------------------------------- Eq. (GradDiv), term by term
  R grad_div(int comp, int i, int j, int k, const std::vector<R>* Pa) const {
    const double h2 = dx * dx;
    const auto& Px = Pa[0]; const auto& Py = Pa[1]; const auto& Pz = Pa[2];
    if (comp == 0) {  // at (i+1/2, j, k)
      return (at(Px, i + 1, j, k) - 2.0 * at(Px, i, j, k) + at(Px, i - 1, j, k)) / h2 +
             (at(Py, i + 1, j, k) - at(Py, i + 1, j - 1, k) - at(Py, i, j, k) + at(Py, i, j - 1, k)) / h2 +
             (at(Pz, i + 1, j, k) - at(Pz, i + 1, j, k - 1) - at(Pz, i, j, k) + at(Pz, i, j, k - 1)) / h2;
    }
    if (comp == 1) {  // at (i, j+1/2, k)
      return (at(Py, i, j + 1, k) - 2.0 * at(Py, i, j, k) + at(Py, i, j - 1, k)) / h2 +
             (at(Px, i, j + 1, k) - at(Px, i - 1, j + 1, k) - at(Px, i, j, k) + at(Px, i - 1, j, k)) / h2 +
             (at(Pz, i, j + 1, k) - at(Pz, i, j + 1, k - 1) - at(Pz, i, j, k) + at(Pz, i, j, k - 1)) / h2;
    }
    // at (i, j, k+1/2)
    return (at(Pz, i, j, k + 1) - 2.0 * at(Pz, i, j, k) + at(Pz, i, j, k - 1)) / h2 +
           (at(Px, i, j, k + 1) - at(Px, i - 1, j, k + 1) - at(Px, i, j, k) + at(Px, i - 1, j, k)) / h2 +
           (at(Py, i, j, k + 1) - at(Py, i, j - 1, k + 1) - at(Py, i, j, k) + at(Py, i, j - 1, k)) / h2;
  }

  // ------------------------------------------------------- f2 (E) and f4 (P_f)
  void update_e_p() {
    // grad(div P^n) where P_f is updated; zero elsewhere
    for (int comp = 0; comp < 3; ++comp) {
#pragma omp parallel for schedule(static) num_threads(c.threads > 0 ? c.threads : 1)
      for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
          for (int i = 0; i < nx; ++i) {
            const size_t p = id(i, j, k);
            GD[comp][p] = active(comp, p) ? grad_div(comp, i, j, k, P) : R(0.0);
          }
    }
    const double hinc_scale = 1.0 / dx;
    const double e0ei = eps0() * c.eps_inf;
    std::vector<R> Enew[3];
    for (int comp = 0; comp < 3; ++comp) {
      Enew[comp] = E[comp];
      const int a1 = (comp + 1) % 3, a2 = (comp + 2) % 3;
      int lo[3], hi[3];
      for (int d = 0; d < 3; ++d) erange(comp, d, lo[d], hi[d]);
#pragma omp parallel for schedule(static) num_threads(c.threads > 0 ? c.threads : 1)
      for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
          for (int i = lo[0]; i <= hi[0]; ++i) {
            // curl_comp H = d_{a1} H_{a2} - d_{a2} H_{a1}; backward differences
            const int ii[3] = {i, j, k};
            int m1[3] = {i, j, k}, m2[3] = {i, j, k};
            m1[a1] -= 1; m2[a2] -= 1;
            const R d1 = (at(H[a2], i, j, k) - at(H[a2], m1[0], m1[1], m1[2])) / dx;
            const R d2 = (at(H[a1], i, j, k) - at(H[a1], m2[0], m2[1], m2[2])) / dx;
            const size_t p = id(i, j, k);
            R& s1 = psiE[comp][a1][p];
            R& s2 = psiE[comp][a2][p];
            s1 = be[a1][ii[a1]] * s1 + ae[a1][ii[a1]] * d1;
            s2 = be[a2][ii[a2]] * s2 + ae[a2][ii[a2]] * d2;
            R curl = (ke[a1][ii[a1]] * d1 + s1) - (ke[a2][ii[a2]] * d2 + s2);
            if (c.tfsf && !c.periodic) curl += tfsf_e(comp, i, j, k) * hinc_scale;
            if (!active(comp, p)) {
              Enew[comp][p] = E[comp][p] + dt / (eps0() * eps_at(comp, k)) * curl;
            } else {
              const R d3 = w[p] * D3;
              const R rhs_gd = nonlocal_on(i, j, k) * ((c.model == 1)
                  ? (w[p] * DNL) * GD[comp][p]
                  : (w[p] * DG1) * GD[comp][p] +
                    (w[p] * DG2) * (3.0 * GD[comp][p] - 4.0 * GD1[comp][p] + GD2[comp][p]));
              R num = dt * curl + (e0ei - 2.0 * d3) * E[comp][p] - d3 * Em[comp][p] -
                      (D1 - 1.0) * P[comp][p] - D2 * Pm[comp][p] - rhs_gd;
              R den = e0ei + d3;
              for (int q = 0; q < ncp; ++q) {
                num = num - (w[p] * C4p[q]) * E[comp][p] - (w[p] * C5p[q]) * Em[comp][p] -
                      (C1p[q] - 1.0) * PC[q][comp][p] - C2p[q] * PCm[q][comp][p];
                den = den + w[p] * C3p[q];
              }
              Enew[comp][p] = num / den;
            }
          }
    }
    // f3: P_CP,p^{n+1}, Eq. (critpointupdate), where P_f is updated
    for (int q = 0; q < ncp; ++q)
      for (int comp = 0; comp < 3; ++comp) {
        std::vector<R> Pn(N, R(0.0));
#pragma omp parallel for schedule(static) num_threads(c.threads > 0 ? c.threads : 1)
        for (int k = 0; k < nz; ++k)
          for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
              const size_t p = id(i, j, k);
              if (!active(comp, p)) continue;
              Pn[p] = C1p[q] * PC[q][comp][p] + C2p[q] * PCm[q][comp][p] +
                      w[p] * (C3p[q] * Enew[comp][p] + C4p[q] * E[comp][p] + C5p[q] * Em[comp][p]);
            }
        PCm[q][comp].swap(PC[q][comp]);
        PC[q][comp].swap(Pn);
      }
    // f4: P_f^{n+1} (Eqs. NonlocalUpdate / GNORUpdate) at metal points only
    std::vector<R> Pnew[3];
    for (int comp = 0; comp < 3; ++comp) {
      Pnew[comp].assign(N, R(0.0));
#pragma omp parallel for schedule(static) num_threads(c.threads > 0 ? c.threads : 1)
      for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
          for (int i = 0; i < nx; ++i) {
            const size_t p = id(i, j, k);
            if (!active(comp, p)) continue;
            const R d3 = w[p] * D3;
            const R gd = nonlocal_on(i, j, k) * ((c.model == 1)
                ? (w[p] * DNL) * GD[comp][p]
                : (w[p] * DG1) * GD[comp][p] +
                  (w[p] * DG2) * (3.0 * GD[comp][p] - 4.0 * GD1[comp][p] + GD2[comp][p]));
            Pnew[comp][p] = D1 * P[comp][p] + D2 * Pm[comp][p] +
                            d3 * (Em[comp][p] + 2.0 * E[comp][p] + Enew[comp][p]) + gd;
          }
    }
    for (int comp = 0; comp < 3; ++comp) {
      Em[comp].swap(E[comp]);
      E[comp].swap(Enew[comp]);
      Pm[comp].swap(P[comp]);
      P[comp].swap(Pnew[comp]);
      GD2[comp].swap(GD1[comp]);
      GD1[comp] = GD[comp];
    }
  }

  // TF/SF correction for E (in units of H, i.e. before the 1/dx)
  double tfsf_e(int comp, int i, int j, int k) const {
    const int* lo = c.tf_lo; const int* hi = c.tf_hi;
    double s = 0.0;
    if (comp == 0 && i >= lo[0] && i <= hi[0] - 1 && j >= lo[1] && j <= hi[1]) {
      if (k == lo[2]) s += h1[lo[2] - 1 + kAuxOff];
      if (k == hi[2]) s -= h1[hi[2] + kAuxOff];
    }
    if (comp == 2 && j >= lo[1] && j <= hi[1] && k >= lo[2] && k <= hi[2] - 1) {
      if (i == lo[0]) s -= h1[k + kAuxOff];
      if (i == hi[0]) s += h1[k + kAuxOff];
    }
    return s;
  }

  // ---------------------------------------------------------------- DFTs
  void accumulate(long n) {
    if (c.nfreq <= 0) return;
    if (c.dft_every > 1 && (n % c.dft_every) != 0) return;
    const double wdt = dt * (c.dft_every > 1 ? c.dft_every : 1);
    const double tJ = (n + 0.5) * dt, tE = (n + 1.0) * dt;
    const int nf = c.nfreq;
    std::vector<double> cJ(nf), sJ(nf), cE(nf), sE(nf);
    for (int m = 0; m < nf; ++m) {
      cJ[m] = std::cos(omega[m] * tJ); sJ[m] = std::sin(omega[m] * tJ);
      cE[m] = std::cos(omega[m] * tE); sE[m] = std::sin(omega[m] * tE);
    }
    const double e0d = eps0() * (c.eps_inf - c.eps_b);
    // planes are independent (each plane's sum keeps its own fixed order)
#pragma omp parallel for schedule(static) num_threads(c.threads > 0 ? c.threads : 1)
    for (int k = 0; k < nz; ++k) {
      // induced current J_x^{n+1/2} = (P^{n+1}-P^n)/dt, plus the bound parts
      // eps0 (eps_inf - eps_b) dE/dt and dP_CP,p/dt inside the metal, summed
      // over the plane
      R s(0.0);
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          const size_t p = id(i, j, k);
          if (!active(0, p)) continue;
          s += (P[0][p] - Pm[0][p]) / dt + e0d * (E[0][p] - Em[0][p]) / dt;
          for (int q = 0; q < ncp; ++q) s += (PC[q][0][p] - PCm[q][0][p]) / dt;
        }
      const double ei = (k + kAuxOff < n1) ? e1[k + kAuxOff] : 0.0;
      for (int m = 0; m < nf; ++m) {
        const size_t q = (size_t)k * nf + m;
        Are[q] += (wdt * cJ[m]) * s;
        Aim[q] += (wdt * sJ[m]) * s;
        Bre[q] += wdt * cE[m] * ei;
        Bim[q] += wdt * sE[m] * ei;
      }
    }
    if (!c.flux) return;
    for (int box = 0; box < 2; ++box)
      for (auto& f : faces[box]) accumulate_face(f, wdt, cE, sE, cJ, sJ);
  }

  // P_f^n (held in Pm after a step) at index (i, j, k), zero off the grid
  R pm_at(int comp, int i, int j, int k) const {
    if (i < 0 || j < 0 || k < 0 || i >= nx || j >= ny || k >= nz) return R(0.0);
    return Pm[comp][id(i, j, k)];
  }

  void accumulate_maps(long n) {
    if (nmap <= 0) return;
    const int every = c.map_every > 1 ? c.map_every : 1;
    if (every > 1 && (n % every) != 0) return;
    const double wdt = dt * every;
    const double tE = (n + 1.0) * dt, tN = (double)n * dt;
    const double qe = 1.602176634e-19;  // elementary charge (C), Eq. (Nsol)
    const int ua = c.map_axis == 0 ? 1 : 0, va = c.map_axis == 2 ? 1 : 2;
    for (int m = 0; m < nmap; ++m) {
      const double w = c.map_omega[m];
      const double ce = std::cos(w * tE), se = std::sin(w * tE);
      const double cn = std::cos(w * tN), sn = std::sin(w * tN);
      const size_t plane = (size_t)mu * mv;
      for (int v = 0; v < mv; ++v)
        for (int u = 0; u < mu; ++u) {
          int ii[3];
          ii[c.map_axis] = c.map_index; ii[ua] = u; ii[va] = v;
          const int i = ii[0], j = ii[1], k = ii[2];
          const size_t q = (size_t)v * mu + u;
          for (int comp = 0; comp < 3; ++comp) {
            const R e = E[comp][id(i, j, k)];
            maps[(size_t)(2 * comp) * nmap * plane + m * plane + q] += (wdt * ce) * e;
            maps[(size_t)(2 * comp + 1) * nmap * plane + m * plane + q] += (wdt * se) * e;
          }
          const R dens = ((pm_at(0, i, j, k) - pm_at(0, i - 1, j, k)) +
                          (pm_at(1, i, j, k) - pm_at(1, i, j - 1, k)) +
                          (pm_at(2, i, j, k) - pm_at(2, i, j, k - 1))) / (dx * qe);
          maps[(size_t)6 * nmap * plane + m * plane + q] += (wdt * cn) * dens;
          maps[(size_t)7 * nmap * plane + m * plane + q] += (wdt * sn) * dens;
        }
      const double ei = e1[c.norm_k + kAuxOff];
      map_inc[2 * m] += wdt * ce * ei;
      map_inc[2 * m + 1] += wdt * se * ei;
    }
  }

  R comp_at(const std::vector<R>* F, int comp, int a, int p, int b, int ib, int cc, int ic) const {
    int ii[3];
    ii[a] = p; ii[b] = ib; ii[cc] = ic;
    return at(F[comp], ii[0], ii[1], ii[2]);
  }

  void accumulate_face(Face& f, double wdt, const std::vector<double>& cE, const std::vector<double>& sE,
                       const std::vector<double>& cJ, const std::vector<double>& sJ) {
    const int nf = c.nfreq;
    const int nb = f.hib - f.lob, nc = f.hic - f.loc;
    // E_b at (p, j+1/2, k) and H_c averaged across the plane, same point
    // (every sample point owns its accumulators: rows run in parallel)
#pragma omp parallel for schedule(static) num_threads(c.threads > 0 ? c.threads : 1)
    for (int kk = 0; kk <= nc; ++kk)
      for (int jj = 0; jj < nb; ++jj) {
        const int jb = f.lob + jj, kc = f.loc + kk;
        const R eb = comp_at(E, f.b, f.a, f.p, f.b, jb, f.cc, kc);
        const R hc = 0.5 * (comp_at(H, f.cc, f.a, f.p - 1, f.b, jb, f.cc, kc) +
                            comp_at(H, f.cc, f.a, f.p, f.b, jb, f.cc, kc));
        const size_t base = ((size_t)kk * nb + jj) * nf;
        for (int m = 0; m < nf; ++m) {
          f.Eb_re[base + m] += (wdt * cE[m]) * eb; f.Eb_im[base + m] += (wdt * sE[m]) * eb;
          f.Hc_re[base + m] += (wdt * cJ[m]) * hc; f.Hc_im[base + m] += (wdt * sJ[m]) * hc;
        }
      }
    // E_c at (p, j, k+1/2) and H_b averaged across the plane
#pragma omp parallel for schedule(static) num_threads(c.threads > 0 ? c.threads : 1)
    for (int kk = 0; kk < nc; ++kk)
      for (int jj = 0; jj <= nb; ++jj) {
        const int jb = f.lob + jj, kc = f.loc + kk;
        const R ec = comp_at(E, f.cc, f.a, f.p, f.b, jb, f.cc, kc);
        const R hb = 0.5 * (comp_at(H, f.b, f.a, f.p - 1, f.b, jb, f.cc, kc) +
                            comp_at(H, f.b, f.a, f.p, f.b, jb, f.cc, kc));
        const size_t base = ((size_t)kk * (nb + 1) + jj) * nf;
        for (int m = 0; m < nf; ++m) {
          f.Ec_re[base + m] += (wdt * cE[m]) * ec; f.Ec_im[base + m] += (wdt * sE[m]) * ec;
          f.Hb_re[base + m] += (wdt * cJ[m]) * hb; f.Hb_im[base + m] += (wdt * sJ[m]) * hb;
        }
      }
  }

  // outward flux  sum dA Re(E x H*) . n  at frequency m (trapezoid weights on edges)
  R box_flux(int box, int m) const {
    R total(0.0);
    for (int fi = 0; fi < (int)faces[box].size(); ++fi) total += face_flux(box, fi, m);
    return total;
  }
  // outward flux through one face (faces ordered -x, +x, -y, +y, -z, +z)
  R face_flux(int box, int fi, int m) const {
    const int nf = c.nfreq;
    R total(0.0);
    {
      const Face& f = faces[box][fi];
      const int nb = f.hib - f.lob, nc = f.hic - f.loc;
      R s(0.0);
      for (int kk = 0; kk <= nc; ++kk)
        for (int jj = 0; jj < nb; ++jj) {
          const double wt = (kk == 0 || kk == nc) ? 0.5 : 1.0;
          const size_t q = ((size_t)kk * nb + jj) * nf + m;
          s += wt * (f.Eb_re[q] * f.Hc_re[q] + f.Eb_im[q] * f.Hc_im[q]);
        }
      for (int kk = 0; kk < nc; ++kk)
        for (int jj = 0; jj <= nb; ++jj) {
          const double wt = (jj == 0 || jj == nb) ? 0.5 : 1.0;
          const size_t q = ((size_t)kk * (nb + 1) + jj) * nf + m;
          s -= wt * (f.Ec_re[q] * f.Hb_re[q] + f.Ec_im[q] * f.Hb_im[q]);
        }
      total += (double)f.side * dx * dx * s;
    }
    return total;
  }

  void spectra(double* inc, R* ext, R* absn, R* sca) const {
    const int nf = c.nfreq;
    const int kc = c.norm_k;
    const double h3 = dx * dx * dx;
    for (int m = 0; m < nf; ++m) {
      const size_t qc = (size_t)kc * nf + m;
      const double b2 = Bre[qc] * Bre[qc] + Bim[qc] * Bim[qc];
      if (inc) inc[m] = b2;
      R s(0.0);
      for (int k = 0; k < nz; ++k) {
        const size_t q = (size_t)k * nf + m;
        s += Are[q] * Bre[q] + Aim[q] * Bim[q];  // Re(A conj(B))
      }
      if (ext) ext[m] = (eta0() * h3) * s / b2;
      if (c.flux) {
        if (absn) absn[m] = -eta0() * box_flux(0, m) / b2;
        if (sca) sca[m] = eta0() * box_flux(1, m) / b2;
      } else {
        if (absn) absn[m] = R(0.0);
        if (sca) sca[m] = R(0.0);
      }
    }
  }

  void run(long nsteps) {
    for (long s = 0; s < nsteps; ++s) {
      const long n = step;
      update_h();                    // H^{n+1/2}, uses E_inc^n
      if (c.tfsf || c.total_field) update_h1();  // H_inc^{n+1/2}
      update_e_p();                  // E^{n+1}, P^{n+1}; uses H_inc^{n+1/2}
      if (c.total_field) plane_source((n + 1) * dt);
      if (c.tfsf || c.src_kind) update_e1((n + 1) * dt);  // E_inc^{n+1}
      accumulate(n);
      accumulate_maps(n);
      ++step;
    }
  }
};

// ------------------------------------------------------------- voxelisers
// Spheres: each P_c Yee point is tested against each sphere with an exact
// integer comparison after quantising coordinates to 2^-20 cell.
void vox_spheres(int nx, int ny, int nz, double dx, int n, const double* cr, uint8_t* out) {
  std::vector<long long> q(4 * (size_t)n);
  for (int s = 0; s < n; ++s)
    for (int t = 0; t < 4; ++t) q[4 * s + t] = std::llround(cr[4 * s + t] / dx * 1048576.0);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        uint8_t bits = 0;
        for (int comp = 0; comp < 3; ++comp) {
          // position in units of 2^-20 cell
          long long px = (long long)i * 1048576, py = (long long)j * 1048576, pz = (long long)k * 1048576;
          if (comp == 0) px += 524288;
          if (comp == 1) py += 524288;
          if (comp == 2) pz += 524288;
          for (int s = 0; s < n; ++s) {
            const long long ddx = px - q[4 * s], ddy = py - q[4 * s + 1], ddz = pz - q[4 * s + 2];
            const long long r = q[4 * s + 3];
            if (ddx * ddx + ddy * ddy + ddz * ddz < r * r) { bits |= (uint8_t)(1u << comp); break; }
          }
        }
        out[((size_t)k * ny + j) * nx + i] = bits;
      }
}

// Star: sphere of radius R plus sphere-capped cones (half-angle theta, rounded
// apex of radius r_tip whose far point lies L past the sphere surface).
// desc = [cx, cy, cz, R, r_tip, tan_half, sin_half, ntips, (ax, ay, az, L) x ntips]
bool star_inside(const double* desc, double x, double y, double z) {
  const double dxp = x - desc[0], dyp = y - desc[1], dzp = z - desc[2];
  const double R = desc[3], rt = desc[4], tn = desc[5], sn = desc[6];
  const int nt = (int)desc[7];
  const double r2 = dxp * dxp + dyp * dyp + dzp * dzp;
  if (r2 < R * R) return true;
  for (int t = 0; t < nt; ++t) {
    const double* tip = desc + 8 + 4 * t;
    const double ax = tip[0], ay = tip[1], az = tip[2], L = tip[3];
    const double s_cap = R + L - rt;
    const double s_apex = s_cap + rt / sn;
    const double s_tan = s_cap + rt * sn;
    const double s = dxp * ax + dyp * ay + dzp * az;
    const double q2 = r2 - s * s;
    if (s >= 0.0 && s <= s_tan) {
      const double rad = (s_apex - s) * tn;
      if (q2 < rad * rad) return true;
    }
    const double ux = dxp - s_cap * ax, uy = dyp - s_cap * ay, uz = dzp - s_cap * az;
    if (ux * ux + uy * uy + uz * uz < rt * rt) return true;
  }
  return false;
}

void vox_star(int nx, int ny, int nz, double dx, const double* desc, uint8_t* out) {
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        uint8_t bits = 0;
        const double xi = (double)i * dx, yj = (double)j * dx, zk = (double)k * dx;
        const double xh = ((double)i + 0.5) * dx, yh = ((double)j + 0.5) * dx, zh = ((double)k + 0.5) * dx;
        if (star_inside(desc, xh, yj, zk)) bits |= 1u;
        if (star_inside(desc, xi, yh, zk)) bits |= 2u;
        if (star_inside(desc, xi, yj, zh)) bits |= 4u;
        out[((size_t)k * ny + j) * nx + i] = bits;
      }
}

}  // namespace

// ======================================================================== C API
extern "C" {

typedef struct or_sim or_sim;

or_sim* or_create(const or_config* cfg, const uint8_t* mask, const double* weight, const double* omega) {
  auto* s = new Sim<double>();
  s->init(*cfg, mask, weight, omega);
  return reinterpret_cast<or_sim*>(s);
}
void or_destroy(or_sim* h) { delete reinterpret_cast<Sim<double>*>(h); }
void or_run(or_sim* h, long nsteps) { reinterpret_cast<Sim<double>*>(h)->run(nsteps); }
long or_step_index(const or_sim* h) { return reinterpret_cast<const Sim<double>*>(h)->step; }
double or_dt(const or_sim* h) { return reinterpret_cast<const Sim<double>*>(h)->dt; }

// which: 0-2 E^n, 3-5 H^{n-1/2}, 6-8 J^{n-1/2} = (P^n - P^{n-1})/dt, 9-11 P^n,
//        12-14 P^{n-1}, 15-17 E^{n-1}, 18-20 GD^{n-1}, 21-23 GD^{n-2},
//        24 + 6q + (0-2) P_CP,q^n, 24 + 6q + (3-5) P_CP,q^{n-1}
int or_get(const or_sim* h, int which, double* out) {
  const auto* s = reinterpret_cast<const Sim<double>*>(h);
  const int c = which % 3;
  const size_t N = s->N;
  if (which >= 24) {
    const int q = (which - 24) / 6, lev = (which - 24) % 6 / 3;
    if (q >= s->ncp) return 1;
    std::memcpy(out, (lev == 0 ? s->PC[q][c] : s->PCm[q][c]).data(), N * 8);
    return 0;
  }
  switch (which / 3) {
    case 0: std::memcpy(out, s->E[c].data(), N * 8); return 0;
    case 1: std::memcpy(out, s->H[c].data(), N * 8); return 0;
    case 2: for (size_t p = 0; p < N; ++p) out[p] = (s->P[c][p] - s->Pm[c][p]) / s->dt; return 0;
    case 3: std::memcpy(out, s->P[c].data(), N * 8); return 0;
    case 4: std::memcpy(out, s->Pm[c].data(), N * 8); return 0;
    case 5: std::memcpy(out, s->Em[c].data(), N * 8); return 0;
    case 6: std::memcpy(out, s->GD1[c].data(), N * 8); return 0;
    case 7: std::memcpy(out, s->GD2[c].data(), N * 8); return 0;
    default: return 1;
  }
}
int or_set(or_sim* h, int which, const double* in) {
  auto* s = reinterpret_cast<Sim<double>*>(h);
  const int c = which % 3;
  const size_t N = s->N;
  std::vector<double>* dst = nullptr;
  if (which >= 24) {
    const int q = (which - 24) / 6, lev = (which - 24) % 6 / 3;
    if (q >= s->ncp) return 1;
    dst = lev == 0 ? &s->PC[q][c] : &s->PCm[q][c];
    std::memcpy(dst->data(), in, N * 8);
    return 0;
  }
  switch (which / 3) {
    case 0: dst = &s->E[c]; break;
    case 1: dst = &s->H[c]; break;
    case 3: dst = &s->P[c]; break;
    case 4: dst = &s->Pm[c]; break;
    case 5: dst = &s->Em[c]; break;
    case 6: dst = &s->GD1[c]; break;
    case 7: dst = &s->GD2[c]; break;
    default: return 1;
  }
  std::memcpy(dst->data(), in, N * 8);
  return 0;
}
void or_get_aux(const or_sim* h, double* e1, double* h1) {
  const auto* s = reinterpret_cast<const Sim<double>*>(h);
  if (e1) std::memcpy(e1, s->e1.data(), s->n1 * 8);
  if (h1) std::memcpy(h1, s->h1.data(), s->n1 * 8);
}
int or_aux_len(const or_sim* h) { return reinterpret_cast<const Sim<double>*>(h)->n1; }
void or_get_dft(const or_sim* h, double* are, double* aim, double* bre, double* bim) {
  const auto* s = reinterpret_cast<const Sim<double>*>(h);
  const size_t n = s->Are.size();
  std::memcpy(are, s->Are.data(), n * 8); std::memcpy(aim, s->Aim.data(), n * 8);
  std::memcpy(bre, s->Bre.data(), n * 8); std::memcpy(bim, s->Bim.data(), n * 8);
}
void or_spectra(const or_sim* h, double* inc, double* ext, double* absn, double* sca) {
  reinterpret_cast<const Sim<double>*>(h)->spectra(inc, ext, absn, sca);
}
double or_box_flux(const or_sim* h, int box, int m) {
  return reinterpret_cast<const Sim<double>*>(h)->box_flux(box, m);
}
double or_face_flux(const or_sim* h, int box, int face, int m) {
  return reinterpret_cast<const Sim<double>*>(h)->face_flux(box, face, m);
}

// Maps: fields [8][nmap][mv][mu] (Re/Im of E_x, E_y, E_z transforms, V s/m,
// then of the density transform, s/m^3), inc [nmap][2].  Returns the plane
// size mu * mv.
long or_get_maps(const or_sim* h, double* fields, double* inc) {
  const auto* s = reinterpret_cast<const Sim<double>*>(h);
  if (fields) std::memcpy(fields, s->maps.data(), s->maps.size() * 8);
  if (inc) std::memcpy(inc, s->map_inc.data(), s->map_inc.size() * 8);
  return (long)s->mu * s->mv;
}

// Forward-mode derivative: the metal weight is w = weight + t * direction and
// the result is sigma_ext(omega[m_target]) after nsteps and its derivative
// with respect to t at t = 0.
int or_directional(const or_config* cfg, const uint8_t* mask, const double* weight,
                   const double* direction, const double* omega, long nsteps, int m_target,
                   double* value, double* deriv) {
  const size_t N = (size_t)cfg->nx * cfg->ny * cfg->nz;
  std::vector<Dual> wd(N);
  for (size_t p = 0; p < N; ++p) wd[p] = Dual(weight[p], direction ? direction[p] : 0.0);
  Sim<Dual> s;
  s.init(*cfg, mask, wd.data(), omega);
  s.run(nsteps);
  std::vector<Dual> ext(cfg->nfreq);
  s.spectra(nullptr, ext.data(), nullptr, nullptr);
  *value = val(ext[m_target]);
  *deriv = der(ext[m_target]);
  return 0;
}

void or_voxelize_spheres(int nx, int ny, int nz, double dx, int n, const double* cxyz_r, uint8_t* out) {
  vox_spheres(nx, ny, nz, dx, n, cxyz_r, out);
}
void or_voxelize_star(int nx, int ny, int nz, double dx, const double* desc, uint8_t* out) {
  vox_star(nx, ny, nz, dx, desc, out);
}
// Constants the oracle uses: 0 c0, 1 mu0, 2 eps0, 3 eta0, 4-6 auxiliary line
// (CPML cells, offset of plane k = 0, source cell).
double or_constants(int which) {
  switch (which) {
    case 0: return kC0;
    case 1: return kMu0;
    case 2: return eps0();
    case 3: return eta0();
    case 4: return kAuxPml;
    case 5: return kAuxOff;
    case 6: return kAuxSrc;
    default: return 0.0;
  }
}

}  // extern "C"

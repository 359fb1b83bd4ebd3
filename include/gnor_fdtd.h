/*
 * gnor_fdtd.h -- C ABI of libgnorfdtd, an MI355X (gfx950) implementation of
 * the hydrodynamic (nonlocal Drude) and GNOR FDTD time step of Baxter,
 * Cala Lesina & Ramunno, "Parallel FDTD modelling of nonlocality in
 * plasmonics" (arXiv:2005.06997).
 *
 * The problem statement is the paper's: a uniform Yee grid (Sec. III,
 * Table I), a free-electron metal described by the Drude parameters wp and
 * gamma plus the hydrodynamic pressure coefficient beta and the GNOR
 * diffusion constant D (Sec. II, Eqs. NonlocDrude and GNOR), the Pekar
 * boundary condition (P_f = 0 outside the metal, end of Sec. III), nonlocal
 * material confined to the total-field region of a TF/SF plane-wave source
 * (end of Sec. III), a CPML-terminated domain (Sec. V), and absorption /
 * extinction spectra read from the run (Sec. V).
 *
 * Conventions
 *  - Units are SI.  Arrays are x-fastest, index ((k * ny) + j) * nx + i.
 *  - Yee positions (Sec. III, Table I): E_x and P_x at (i+1/2, j, k),
 *    E_y at (i, j+1/2, k), E_z at (i, j, k+1/2); H_x at (i, j+1/2, k+1/2),
 *    H_y at (i+1/2, j, k+1/2), H_z at (i+1/2, j+1/2, k).  nx, ny, nz count
 *    nodes including the CPML; PEC walls sit on the outer node planes.
 *  - Time: E^n at n dt, H at (n - 1/2) dt; a step advances H to n+1/2 and
 *    E, P_f to n+1 (update order of Sec. III: f1, f2, f4).
 *  - Ownership: the caller allocates ONE device buffer of
 *    gnor_required_bytes() bytes and a HIP stream and binds both with
 *    gnor_bind_memory(); the library carves all device state out of that
 *    buffer, never frees it, and enqueues all work on that stream.  The
 *    gradient's workspace and a batch's parameter tables are further caller
 *    buffers (gnor_gradient_required_bytes, gnor_batch_required_bytes): the
 *    library allocates no device memory.  Host inputs are copied before a
 *    call returns; outputs go to caller arrays.
 *  - Errors: every call returns a gnor_status; nothing is thrown across the
 *    ABI.  gnor_last_error() gives a message for the last failure on a sim.
 *  - Threads: one gnor_sim must not be used by two host threads at once.
 */
#ifndef GNOR_FDTD_H
#define GNOR_FDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gnor_sim gnor_sim;
typedef struct gnor_batch gnor_batch;

typedef enum {
  GNOR_OK = 0,
  GNOR_E_INVALID_ARG = 1,     /* a size, pointer or parameter is out of range */
  GNOR_E_UNSTABLE = 2,        /* Courant number outside (0, 1/sqrt(3)) */
  GNOR_E_OUT_OF_MEMORY = 3,   /* host allocation failed */
  GNOR_E_DEVICE = 4,          /* a HIP call failed */
  GNOR_E_STATE = 5,           /* call out of order (e.g. run before bind) */
  GNOR_E_BUFFER_TOO_SMALL = 6,/* caller buffer smaller than required */
  GNOR_E_NONFINITE = 7        /* the non-finite watchdog found NaN/Inf */
} gnor_status;

typedef enum { GNOR_FP32 = 0, GNOR_FP64 = 1 } gnor_precision;

/* Grid, absorbing layers and TF/SF box.
 * dx: cell size (m); courant: S = c dt / dx, must lie in (0, 1/sqrt(3)).
 * npml: CPML thickness in cells on every face (0 = bare PEC box).  The
 * layers use polynomial grading of order pml_order, sigma_max =
 * pml_sigma_scale (m+1) / (eta0 dx sqrt(eps_background)), kappa rising to
 * pml_kappa_max and alpha falling from pml_alpha_max (Roden-Gedney CPML).
 * tf_lo/tf_hi: node indices of the TF box [tf_lo, tf_hi] (inclusive); the
 * box must lie outside the CPML with one spare cell.  precision: storage and
 * arithmetic type of fields, free-electron current and CPML memory; the
 * spectral accumulators are always FP64. */
typedef struct {
  int32_t nx, ny, nz;
  double dx, courant;
  int32_t npml;
  double pml_order, pml_sigma_scale, pml_kappa_max, pml_alpha_max;
  double eps_background;
  int32_t tf_lo[3], tf_hi[3];
  int32_t precision; /* gnor_precision */
  /* Dielectric substrate: with eps_substrate > 0 the half-space beyond node
   * plane substrate_k (z > substrate_k dx) has relative permittivity
   * eps_substrate; E_x and E_y on that plane take the mean of the two, E_z
   * half a cell above a node takes the permittivity of its side.  The 1D
   * incident line carries the same layers, so the TF/SF source injects the
   * layered (Fresnel) plane wave at normal incidence.  0 = no substrate.
   * With a substrate: every metal point must lie below plane substrate_k
   * (in eps_background), and the fused and hybrid step forms and the design
   * gradient are refused (GNOR_E_INVALID_ARG).  The CPML keeps the
   * eps_background grading on both sides. */
  double eps_substrate;
  int32_t substrate_k;
  /* Total-field operation (end of Sec. III: geometries that TF/SF cannot
   * hold, such as a plasmonic substrate).  total_field = 1: no TF/SF box
   * (tf_lo/tf_hi are ignored); the source is soft on node plane source_k,
   * E_x^{n+1} += f(t_{n+1}) at every E_x point of the plane, added after the
   * E and current updates of the step; metal may reach into the CPML (any
   * node index in [1, n - 2] per axis), and there it follows the local Drude
   * model: the beta^2 and D terms are dropped at metal points in cells
   * within npml of a face.  The 1D line carries the same soft source at line
   * cell source_k + 25, so the spectra normalise by its wave.  source_k must
   * lie in [npml + 1, nz - 2 - npml].  Not available with a substrate, flux
   * boxes, a design region or gradient, batches, or the fused step form 1
   * (GNOR_E_INVALID_ARG).  0 = TF/SF as above. */
  int32_t total_field;
  int32_t source_k;
} gnor_grid_desc;

/* Free-electron metal (Sec. II): wp (rad/s), gamma (rad/s), beta (m/s; the
 * hydrodynamic pressure coefficient is beta^2), diffusion D (m^2/s; GNOR,
 * eta = beta^2 + D gamma), eps_inf (background permittivity of the metal).
 * beta = D = 0 is the local Drude model; D = 0 the nonlocal Drude model.
 *
 * Bound electrons: ncp (0..4) critical points of Eq. (CritPoint), pole p
 * with amplitude cp_A[p], frequency cp_Omega[p] (rad/s), width cp_Gamma[p]
 * (rad/s) and phase cp_phi[p] (rad).  Their polarisation is updated at the
 * metal points after E (f3, Eq. critpointupdate) and enters the E update and
 * the extinction current.  With ncp > 0 the fused one-pass step and the
 * design gradient are not available (GNOR_E_INVALID_ARG). */
#define GNOR_MAX_CP 4
typedef struct {
  double wp, gamma, beta, diffusion, eps_inf;
  int32_t ncp;
  double cp_A[GNOR_MAX_CP], cp_Omega[GNOR_MAX_CP], cp_Gamma[GNOR_MAX_CP], cp_phi[GNOR_MAX_CP];
} gnor_material_desc;

/* Plane-wave source: x-polarised, travelling along +z, injected through the
 * TF/SF box from a 1D auxiliary line (same dx, dt, background; 20-cell CPML
 * at both ends; node k of the grid is line cell k + 25; soft source at line
 * cell 22).  kind 1: e0 exp(-((t - t0)/tau)^2) sin(omega_c (t - t0));
 * kind 2: e0 [(1 - cos(omega_max t))/2]^3 for 0 <= t <= 2 pi / omega_max
 * (the raised-cosine pulse of Sec. V); kind 0: no source. */
typedef struct {
  int32_t kind;
  double e0, omega_c, tau, t0, omega_max;
} gnor_source_desc;

/* Spectral monitors: running DFTs (factor dt, e^{+i w t}) at nfreq angular
 * frequencies omega[] (rad/s), every dft_every-th step.  norm_k: grid plane
 * whose incident transform normalises the cross sections.  flux_enabled:
 * also accumulate tangential E and H on the faces of the absorption box
 * (abs_lo..abs_hi, inside the TF box) and the scattering box (sca_lo..sca_hi,
 * outside it, outside the CPML). */
typedef struct {
  int32_t nfreq;
  const double *omega;
  int32_t norm_k;
  int32_t dft_every;
  int32_t flux_enabled;
  int32_t abs_lo[3], abs_hi[3];
  int32_t sca_lo[3], sca_hi[3];
} gnor_monitor_desc;

/* Create a simulation for a grid.  Checks sizes (each of nx, ny, nz >= 4;
 * at most 4e9 cells, since the sweeps index cells with 32-bit integers; the
 * TF box and the CPML as described above) and the Courant number
 * (GNOR_E_UNSTABLE if S >= 1/sqrt(3)).  *out receives an opaque handle. */
gnor_status gnor_create(const gnor_grid_desc *grid, gnor_sim **out);
void gnor_destroy(gnor_sim *sim);

/* Metal: mask is a host array of nx*ny*nz bytes, bit c (c = 0, 1, 2) set iff
 * P_c at that cell's Yee point is inside the metal (Pekar condition, Sec.
 * III).  Every metal point must lie at least 2 cells inside the TF box
 * (nonlocal material only in the total-field region, end of Sec. III);
 * otherwise GNOR_E_INVALID_ARG. */
gnor_status gnor_set_material(gnor_sim *sim, const uint8_t *mask, const gnor_material_desc *mat);
gnor_status gnor_set_source(gnor_sim *sim, const gnor_source_desc *src);
gnor_status gnor_set_monitors(gnor_sim *sim, const gnor_monitor_desc *mon);

/* Device bytes needed for the current material and monitors. */
size_t gnor_required_bytes(const gnor_sim *sim);

/* Bind the caller's device buffer (>= gnor_required_bytes, 256-byte aligned)
 * and HIP stream (NULL = default stream), upload the problem and zero the
 * state (step index 0).  Must follow set_material/set_source/set_monitors. */
gnor_status gnor_bind_memory(gnor_sim *sim, void *device_ptr, size_t bytes, void *hip_stream);

/* Zero all fields, currents, CPML memory and accumulators (step index 0). */
gnor_status gnor_reset(gnor_sim *sim);

/* Enqueue nsteps leapfrog steps on the bound stream (asynchronous).  Steps
 * are replayed from captured HIP graphs in chunks (gnor_set_graph_chunk).
 * Non-finite watchdog (on by default, gnor_set_watchdog): after every chunk
 * of steps (the graph chunk; 64 steps when graphs are off; counted across
 * calls) a scan of E^n for NaN / Inf sets a device flag that is part of the
 * state (cleared by gnor_reset, restored by gnor_load_state).  While the
 * next chunk runs, gnor_run waits for the previous chunk's scan only and
 * returns GNOR_E_NONFINITE if it found one (the steps enqueued so far still
 * run); gnor_synchronize reads the last scan's flag after the stream drains
 * and returns GNOR_E_NONFINITE the same way. */
gnor_status gnor_run(gnor_sim *sim, int64_t nsteps);
gnor_status gnor_synchronize(gnor_sim *sim);
/* on = 1 (default) or 0; INVALID_ARG otherwise. */
gnor_status gnor_set_watchdog(gnor_sim *sim, int32_t on);
int64_t gnor_step_index(const gnor_sim *sim);

/* Steps per captured graph (even; 0 = launch every kernel directly). */
gnor_status gnor_set_graph_chunk(gnor_sim *sim, int32_t steps);

/* Cross sections (m^2) per monitor frequency, any pointer may be NULL:
 * inc = |B(norm_k, w)|^2 (incident spectral energy, (V s/m)^2);
 * ext = eta0 dx^3 sum_k Re(A(k, w) conj(B(k, w))) / inc with A the transform
 *       of the plane-summed induced current J_x (volume optical theorem);
 * abs = -eta0 (outward flux of Re(E x H*) through the absorption box) / inc;
 * sca = +eta0 (outward flux through the scattering box) / inc.
 * Synchronises the stream. */
gnor_status gnor_get_spectra(gnor_sim *sim, double *inc, double *ext, double *abs_, double *sca);

/* Enqueue (asynchronously, on the bound stream) the fold of the flux-box
 * samples staged since the last fold into the FP64 accumulators.  Steps
 * stage their samples and fold them every 256 steps; gnor_get_spectra folds
 * a partly filled window itself.  This call lets a caller put that fold
 * where it wants it (for example inside a timed region).  A no-op without
 * flux boxes or right after a fold. */
gnor_status gnor_flush_spectra(gnor_sim *sim);

/* Raw transforms (SI): A[k][m], B[k][m] as separate real/imag arrays of
 * nz * nfreq doubles each. */
gnor_status gnor_get_dft(gnor_sim *sim, double *a_re, double *a_im, double *b_re, double *b_im);

/* Near-field and free-electron density maps (the field and density
 * distributions of Sec. V): running transforms (factor every*dt, e^{+i w t})
 * on the grid plane `index` normal to `axis` (0 x, 1 y, 2 z) at nmap (<= 8)
 * angular frequencies omega[] (rad/s).  E_x, E_y and E_z are taken at their
 * Yee points of the plane and stamped (n+1) dt; the free-electron density
 * n - n0 = div P_f / e (Eq. Nsol) at the plane's nodes, from P_f^n (backward
 * differences), stamped n dt; every `every` steps (1 = each step).  Plane
 * coordinates (u, v) are the two other axes in x, y, z order, u fastest.
 * Set before gnor_bind_memory (nmap = 0 turns the maps off).  Not with
 * batches or gnor_gradient (GNOR_E_STATE). */
typedef struct {
  int32_t axis, index, nmap, every;
  const double *omega;
} gnor_map_desc;
gnor_status gnor_set_maps(gnor_sim *sim, const gnor_map_desc *maps);

/* Map transforms: fields receives 8 * nmap * nu * nv doubles, [quantity][m]
 * [v][u] with quantity = Re, Im of E_x, E_y, E_z (V s/m), then Re, Im of
 * n - n0 (s/m^3); inc receives 2 * nmap doubles, [m][Re, Im] of the incident
 * field's transform at plane norm_k (V s/m).  count = 8 * nmap * nu * nv.
 * Synchronises the stream. */
gnor_status gnor_get_maps(gnor_sim *sim, double *fields, double *inc, size_t count);

/* Copy one field to host as nx*ny*nz doubles in SI units:
 * 0-2 E^n (V/m), 3-5 H^{n-1/2} (A/m), 6-8 J^{n-1/2} = dP_f/dt (A/m^2),
 * 9 + 3p + c (p < ncp): component c of the critical-point polarisation
 * P_CP,p^n (C/m^2; zero outside the metal),
 * 21 (GNOR_FIELD_DENSITY): the free-electron density n - n0 = div P_f^n / e
 * (m^-3, Eq. Nsol) at the nodes (i, j, k), with backward differences of the
 * Yee-staggered P_f^n (zero away from the metal).
 * count must be nx*ny*nz.  Synchronises the stream. */
#define GNOR_FIELD_DENSITY 21
gnor_status gnor_get_field(gnor_sim *sim, int32_t which, double *host_dst, size_t count);

/* Auxiliary line E_inc^n, H_inc^{n-1/2} (SI), n1 = nz + 50 doubles each. */
gnor_status gnor_get_aux(gnor_sim *sim, double *e1, double *h1, size_t count);

/* Full state snapshot (fields, currents, node scalars, CPML memory,
 * auxiliary line, accumulators, step index) to/from host memory.  The image
 * is the library's device layout of this simulation's state, unversioned:
 * load it only into a simulation of the same description, with the same
 * library build. */
size_t gnor_state_bytes(const gnor_sim *sim);
gnor_status gnor_save_state(gnor_sim *sim, void *host_dst, size_t bytes);
gnor_status gnor_load_state(gnor_sim *sim, const void *host_src, size_t bytes);

/* Non-finite watchdog: scans E and H; GNOR_E_NONFINITE if any is NaN/Inf. */
gnor_status gnor_check_finite(gnor_sim *sim);

/* Average device time per launch (ms) of each kernel over nsteps steps run
 * with events around every launch on the bound stream (no graphs; the host
 * waits once, after the last step, so the queue never drains; 1 <= nsteps
 * <= 4096, INVALID_ARG otherwise):
 * ms[0] H sweep (with the auxiliary line's H half), ms[1] E/J sweep (with the
 * auxiliary line's E half), ms[2] spectra and flux staging, ms[3] fused step
 * (when fused; see below), ms[4] flux accumulation (per step, amortised).
 * count must be >= 5; the state advances by nsteps. */
gnor_status gnor_profile_kernels(gnor_sim *sim, int64_t nsteps, double *ms, int32_t count);

/* The field update runs as one launch per tile class: 0 tiles that meet
 * neither metal nor a CPML slab, 1 tiles that meet a CPML slab only, 2 tiles
 * with a metal point within two cells, 3 tiles that are both 2 and 1 (a tile
 * meets a slab with a one-cell margin); in the two-sweep form class 0 also
 * takes the tiles that meet only an x slab (gnor_tile_classes counts them
 * there).  By default a step is the two-sweep form (H sweep, then E/J
 * sweep); gnor_set_fused(sim, 1) selects one fused pass (H and E/J together,
 * 12 instead of 18 field words moved per cell) plus a one-block launch that
 * advances the auxiliary line; gnor_set_fused(sim, 2) the hybrid form: the
 * fused pass for the tiles that meet no CPML slab (classes 0 and 2; class 2
 * stays two-sweep with critical points), then the auxiliary line, then the
 * E/J sweep of the CPML classes, whose H sweep ran alongside the fused
 * tiles; gnor_set_fused(sim, 3) the same order with classes 0 (x-slab tiles
 * included), 1 and, without critical points, 2 in one pass, by lighter
 * kernels whose wavefronts share halo H through lane shuffles and LDS (class
 * 2 after a launch that writes the step's node scalars), each class's launch
 * followed by a small one that adds the TF/SF terms on the faces of the TF
 * box at that class's points, and class 3 in two sweeps (critical points, a
 * substrate and total-field operation allowed).  All forms give the same
 * fields up to rounding; gnor_gradient always uses the two-sweep form; a
 * batch its own (gnor_batch_set_form).
 * gnor_profile_kernels times each sweep as it runs: with concurrent class
 * launches (the default, see gnor_set_class_streams) a sweep is timed from its
 * fork to its join; with serial class launches, count >= 14 also returns
 * ms[5 + c] the H sweep's (or the fused step's) class c and ms[9 + c] the E/J
 * sweep's class c (0 otherwise); ms[13] is the auxiliary-line launch of the
 * fused form.  In fused form ms[0] = ms[1] = 0 and ms[3] holds the fused step
 * (classes + auxiliary line); in hybrid form ms[0] is the first phase (fused
 * tiles and H sweeps) and ms[1] the second (auxiliary line and E/J sweeps);
 * in form 3 with serial class launches ms[5 + c] is one-pass class c (with
 * its TF/SF launch, and for class 2 its node scalars) and ms[9] the
 * auxiliary line.
 * gnor_tile_classes writes the number of tiles of each class of the current
 * tiling to counts[0..3] (valid once the memory is bound).
 * gnor_tile_class_cells writes, per class c, the grid cells its tiles cover
 * (tiles clipped to the grid) to cells[c] and the (cell, axis) pairs among
 * them that lie in that axis's CPML slab to slab_dirs[c] (valid once the
 * memory is bound). 
 * gnor_set_fused: on must be 0, 1, 2 or 3 (INVALID_ARG otherwise; 1 also
 * with critical points, 1 and 2 also with a substrate). */
gnor_status gnor_set_fused(gnor_sim *sim, int32_t on);

/* The four tile-class launches of a sweep run concurrently (on = 1, the
 * default: classes 0 and 3 on the bound stream, classes 1 and 2 on two side streams
 * of the library, joined back by events, also inside graphs) or one after
 * another on the bound stream (on = 0; for profilers that time each
 * launch).  INVALID_ARG unless on is 0 or 1. */
gnor_status gnor_set_class_streams(gnor_sim *sim, int32_t on);
gnor_status gnor_tile_classes(const gnor_sim *sim, int32_t *counts);
gnor_status gnor_tile_class_cells(const gnor_sim *sim, int64_t *cells, int64_t *slab_dirs);

/* Sweep tiling: each block owns 64 (x) x ty (y) columns over kz planes;
 * ty in {2, 4, 8}, 1 <= kz <= nz.  Blocks are dealt to the 8 XCDs
 * round-robin; tile_order chooses which tiles a block takes within its
 * class: 0 natural order (neighbouring tiles on different XCDs), 1 one
 * contiguous band of tiles per XCD (neighbours share its L2), 2 chunks of 8
 * tile rows dealt round-robin to the XCDs (balanced and local).  Fields do
 * not depend on the tiling; spectra only through FP64 summation order.
 * Errors: INVALID_ARG for other values. */
gnor_status gnor_set_tiling(gnor_sim *sim, int32_t ty, int32_t kz, int32_t tile_order);

/* Autotuner: times every candidate tiling (ty in {2, 4, 8}, kz in {2, 3, 4,
 * 8, 16, 32, 64, nz} clamped to nz, tile_order in {0, 1, 2}) over
 * trial_steps directly launched steps, times the four fastest three more
 * times over 4 * trial_steps steps and keeps the fastest of those timings.  Must be called at
 * step index 0; the state is reset afterwards.  Outputs (any may be NULL):
 * chosen ty, kz, tile_order and its ms per step (from the second timing). */
gnor_status gnor_autotune(gnor_sim *sim, int32_t trial_steps, int32_t *ty, int32_t *kz,
                          int32_t *tile_order, double *ms_per_step);

/* Voxelisers.  Spheres: n spheres as (cx, cy, cz, r) in metres from node
 * (0,0,0); a P_c point is inside iff its squared distance to a centre is
 * strictly below r^2 after quantising all coordinates to 2^-20 cell (exact
 * integer test).  Star: desc = [cx, cy, cz, R, r_tip, tan(theta),
 * sin(theta), ntips, (ax, ay, az, L) x ntips]: sphere of radius R plus
 * sphere-capped cones of half-angle theta along unit axes a whose rounded
 * apex (radius r_tip) ends L beyond the sphere surface; FP64 tests in a
 * fixed operation order.  mask_out receives nx*ny*nz bytes. */
gnor_status gnor_voxelize_spheres(int32_t nx, int32_t ny, int32_t nz, double dx, int32_t n,
                                  const double *cxyz_r, uint8_t *mask_out);
gnor_status gnor_voxelize_star(int32_t nx, int32_t ny, int32_t nz, double dx, const double *desc,
                               int32_t desc_len, uint8_t *mask_out);

/* Design region for gradients: cells [lo, hi) (node indices, x fastest) whose
 * three P components are all treated as metal with per-cell density rho in
 * [0, 1] scaling wp^2, beta^2 and D (gamma unchanged; rho = 0 leaves P = 0).
 * The region replaces any fixed metal inside it and must lie 2 cells inside
 * the TF box.  Call after gnor_set_material, before gnor_bind_memory;
 * rho_init is a HOST array of prod(hi - lo) floats copied before return
 * (NULL: density 1), uploaded by gnor_bind_memory.
 * gnor_update_design replaces the densities of a bound simulation from a
 * DEVICE array rho_device of prod(hi - lo) floats (x fastest, 4-byte
 * aligned, read in stream order on the bound stream; the state is not
 * reset).  It checks the values on the device and synchronises the stream:
 * any value outside [0, 1] (or NaN) gives GNOR_E_INVALID_ARG and leaves the
 * densities unchanged. */
gnor_status gnor_set_design(gnor_sim *sim, const int32_t lo[3], const int32_t hi[3], const float *rho_init);
gnor_status gnor_update_design(gnor_sim *sim, const float *rho_device);

/* Objective sigma_ext(omega[m_target]) (as gnor_get_spectra) of nsteps steps
 * from rest, and its exact discrete-adjoint gradient with respect to the
 * design densities.  Forward pass with a full-state checkpoint every
 * ckpt_every steps; backward pass segment by segment with recomputation.
 * Needs dft_every = 1 and eps_inf = eps_background.
 * workspace: caller DEVICE buffer of at least
 * gnor_gradient_required_bytes(sim, nsteps, ckpt_every) bytes, 256-byte
 * aligned (checkpoints, adjoint fields, per-segment design-region history;
 * the library writes it and never frees it); gnor_gradient_required_bytes
 * returns 0 before gnor_bind_memory or without a design region.
 * objective: HOST double (may be NULL); grad: DEVICE array of prod(hi - lo)
 * doubles, x fastest, overwritten.  Synchronises the stream before return;
 * the simulation state afterwards is unspecified (gnor_reset).  Errors:
 * GNOR_E_BUFFER_TOO_SMALL for a short workspace, INVALID_ARG for an
 * unaligned one or bad counts, STATE without a design region. */
size_t gnor_gradient_required_bytes(const gnor_sim *sim, int64_t nsteps, int32_t ckpt_every);
gnor_status gnor_gradient(gnor_sim *sim, int64_t nsteps, int32_t ckpt_every, int32_t m_target,
                          void *workspace, size_t workspace_bytes, double *objective, double *grad);

/* Batches: n independent simulations (bound, same precision, same step
 * index, same tile height) stepped in lockstep; every phase of a step is one
 * launch per tile class over the tiles of all instances (and one launch
 * advances every instance's incident line).  The batch enqueues on hip_stream
 * (NULL: a stream of its own); call gnor_batch_synchronize before reading an
 * instance.  Instances must not be stepped outside the batch while it is in
 * use (GNOR_E_STATE).  table: caller DEVICE buffer of at least
 * gnor_batch_required_bytes(n, sims) bytes, 256-byte aligned, that holds the
 * batch's two per-instance parameter tables until gnor_batch_destroy (the
 * library writes it at creation and never frees it); a short or unaligned
 * buffer gives GNOR_E_BUFFER_TOO_SMALL.  The non-finite watchdog of gnor_run
 * does not run inside batches.  Results equal those of the instances run
 * one by one. */
size_t gnor_batch_required_bytes(int32_t n, gnor_sim *const *sims);
gnor_status gnor_batch_create(int32_t n, gnor_sim *const *sims, void *hip_stream, void *table,
                              size_t table_bytes, gnor_batch **out);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * batch as gnor_batch_create, with its parameter tables in the library's one
 * static device buffer instead of a caller buffer.  That buffer is 1 MiB per
 * GPU, held until the process ends, and takes at most 128 instances (more:
 * GNOR_E_BUFFER_TOO_SMALL).  The call allocates nothing and creates no
 * streams or events: hip_stream must be a stream the caller made (NULL:
 * GNOR_E_INVALID_ARG), and the batch launches its tile classes one after
 * another on it.  Every static batch on a GPU shares that GPU's buffer: a
 * new one waits for the previous one's queued work, then takes the buffer
 * over, and the previous one is refused from then on (gnor_batch_run:
 * GNOR_E_STATE).  Calls on one GPU from two host threads at once race.
 * Results equal gnor_batch_create's, bit for bit. */
gnor_status gnor_batch_create_static(int32_t n, gnor_sim *const *sims, void *hip_stream,
                                     gnor_batch **out);
gnor_status gnor_batch_run(gnor_batch *batch, int64_t nsteps);
gnor_status gnor_batch_synchronize(gnor_batch *batch);
gnor_status gnor_batch_set_graph_chunk(gnor_batch *batch, int32_t steps);
/* Step form of a batch (Sec. III: f1 and f2 of every instance, one launch
 * per phase over all instances): 0 two sweeps (the default), 3 the tiles
 * without metal in one pass, the metal tiles in two sweeps, as
 * gnor_set_fused(sim, 3) for one simulation.  The instances take the
 * batch's form (gnor_batch_create sets them to form 0): their tile lists
 * follow it.  Results equal single runs of the same form bit for bit.  Waits
 * for the batch's queued steps when the form changes.  INVALID_ARG unless
 * form is 0 or 3. */
gnor_status gnor_batch_set_form(gnor_batch *batch, int32_t form);
const char *gnor_batch_last_error(const gnor_batch *batch);
void gnor_batch_destroy(gnor_batch *batch);

const char *gnor_status_string(gnor_status s);
const char *gnor_last_error(const gnor_sim *sim);

#ifdef __cplusplus
}
#endif
#endif /* GNOR_FDTD_H */

/*
 * lbm.h -- C ABI of the MI355X lattice-Boltzmann nanochannel library
 * (liblbm.so).  Hot path of the Keldysh-lattice-Boltzmann method of
 * arXiv 2403.15768: water in a nanochannel (Sec. 2) as one lattice-Boltzmann
 * population set (Sec. 4), driven by a bulk pressure-gradient force (Eq. 2),
 * closed at the liquid/solid interface by a friction wall whose per-node
 * coefficient is the linear drag of Eq. 5 / Eq. 27, with periodic inlet and
 * outlet (Sec. 4.2).
 *
 * Conventions shared by every call:
 *  - Every function returns lbm_status (0 = LBM_OK).  Nothing aborts, throws
 *    or prints.  lbm_last_error() describes the last failure of a context.
 *  - Units are lattice units (dx = dt = 1).  The paper's mapping dx = 1 nm,
 *    dt = 1 ps (Sec. 6) is the caller's business.
 *  - Device memory is owned by the caller: lbm_create() borrows an arena of
 *    lbm_footprint() bytes (256-byte aligned) and never frees it.  Host
 *    arrays are owned by the caller and only touched during the call.
 *  - A context is used from one host thread and runs on the HIP stream given
 *    at creation.  lbm_step() and the kernel part of lbm_set_* are
 *    asynchronous; device errors are latched and returned by the next
 *    synchronising call (lbm_sync, lbm_invariants, lbm_flux, lbm_mass,
 *    lbm_get_*, lbm_run_to_steady).
 *  - Population order: D2Q9 uses the paper's numbering beside Eqs. 19-21
 *    (0 rest, 1 +x, 2 +y, 3 -x, 4 -y, 5 (+,+), 6 (-,+), 7 (-,-), 8 (+,-));
 *    D3Q19: 0 rest, 1..6 = +x,-x,+y,-y,+z,-z, 7..18 = (+,+,0), (-,-,0),
 *    (+,-,0), (-,+,0), (+,0,+), (-,0,-), (+,0,-), (-,0,+), (0,+,+), (0,-,-),
 *    (0,+,-), (0,-,+).
 *  - Dense host fields are laid out [z][y][x] (x fastest), populations
 *    [i][z][y][x].  Wall nodes are numbered in increasing linear index
 *    x + nx (y + ny z) ("canonical order").
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* bad argument; nothing changed */
  LBM_ENOMEM = -2,    /* arena too small */
  LBM_EDEVICE = -3,   /* a HIP call failed (message in lbm_last_error) */
  LBM_ENOTCONV = -4,  /* run_to_steady reached max_steps */
  LBM_EDIVERGED = -5, /* NaN/Inf in the flux or mass */
  LBM_ESTATE = -6     /* call not valid in the context's current state */
} lbm_status;

typedef enum { LBM_D2Q9 = 9, LBM_D3Q19 = 19 } lbm_lattice;

/* Storage and arithmetic:
 *  F64  stores and computes in double;
 *  F32  stores float and computes in double (FP32 arithmetic would feed the
 *       rounding error of the computed moments back into every collision as
 *       a momentum source that accumulates over the slowest viscous time to
 *       ~1e-4 of the flow);
 *  F16S stores half-precision deviations from the rest equilibrium, scaled
 *       by 2^12, and computes in float.
 * Storage narrower than the arithmetic is rounded stochastically (counter-
 * based random bits from the context's step and cell), which keeps results
 * reproducible bit for bit; round-to-nearest would stall the approach to
 * steady state once the per-step change drops below half an ulp.  Flux and
 * mass reductions are double in every mode. */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2 } lbm_precision;

/* SLAB: walls half a link below y = 0 and above y = ny-1, z periodic (D2Q9
 *       requires SLAB or MASKED with nz = 1).
 * DUCT: walls on both y and both z faces, half a link outside the box.
 * TUBE: circular wall of radius tube_radius around the x axis through
 *       (tube_cy, tube_cz); cells with (y-cy)^2 + (z-cz)^2 < R^2 are fluid;
 *       interpolated (Bouzidi) bounce-back at the curved wall.
 * MASKED: walls that vary along x -- corrugated, wrinkled or stepped walls,
 *       posts -- the design freedom of Sec. 5.1: the SLAB box with the
 *       points of the (x, y) plane flagged in `solid` solid for every z
 *       (z periodic).  Half-way bounce-back on every wall link; the slip
 *       half of the wall rule takes, for each wall link i of a node, the
 *       node's own population of one link k pointing into the solid, chosen
 *       so that each such k serves exactly one i (mass stays exact): by
 *       preference, over i in increasing direction index among the k still
 *       free, the reflection (c_x, -c_y, -c_z) about a y-normal wall (the
 *       SLAB's transverse reversal: an x-uniform mask is the SLAB exactly),
 *       then (-c_x, c_y, -c_z) about an x-normal step face, then -c_i, then
 *       the lowest-numbered free k.  Wall nodes are numbered as in every
 *       geometry (increasing x + nx (y + ny z)).  Thermal noise works as
 *       everywhere; no moving wall, electron sheets, open ends or batches
 *       (LBM_EINVAL).
 * x is periodic in every geometry (inlet/outlet option 1 of Sec. 4.2) unless
 * lbm_set_open_ends opens it (option 2). */
typedef enum { LBM_SLAB = 0, LBM_DUCT = 1, LBM_TUBE = 2, LBM_MASKED = 3 } lbm_geometry;

typedef struct {
  int lattice;   /* lbm_lattice */
  int precision; /* lbm_precision */
  int geometry;  /* lbm_geometry */
  int nx, ny, nz;
  double tube_radius, tube_cy, tube_cz; /* TUBE only */
  double tau;                           /* BGK relaxation time, > 0.5 */
  double rho0;                          /* reference density */
  double force[3];          /* body-force density (the bulk force of Eq. 2) */
  double wall_velocity_top; /* != 0: the y = ny-1/2 wall of SLAB/DUCT moves
                               along x at this speed as a no-slip wall
                               (Couette check); 0 otherwise */
  const uint8_t *solid;     /* MASKED only: nx * ny bytes, host, index
                               x + nx y, nonzero = solid; read by
                               lbm_footprint / lbm_create only (not kept);
                               ignored by the other geometries */
} lbm_params;

/* Synthetic surface-response spectra of the friction quadrature (units
 * hbar = k_B = 1, lengths in units of the gap d):
 *   raw(Omega) = C sum_a sum_b dq dw q_a^3 e^{-2 q_a d}
 *                  Im g_s Im g_l / (sinh^2(w_b / 2T) S),
 *   C = 1/(8 pi^2 T), q_a = (a+1/2) dq, dq = q_max/nq, w_b = (b+1/2) dw,
 *   dw = w_max/nw, responses at (q_a, w_b), each a damped oscillator
 *   A W / (W - w^2 - i gamma w):
 *   g_s: A = 1, W = P = Omega^2 q d (dispersion = 1) or Omega^2 (dispersion = 0),
 *        gamma = gamma_s;
 *   g_l: A = a_l, W = w_l^2 + v_l^2 q^2, gamma = gamma_l;
 *   S = |1 - g_s g_l e^{-2 q d}|^2 (coupling = 1: the two surfaces screen
 *       each other repeatedly) or 1 (coupling = 0).
 * coupling must be 0 or 1, v_l finite and >= 0.  coupling = 0, v_l = 0 is
 * the unscreened, non-dispersive form (a faster kernel).
 * Lattice friction of node k: lambda_k = lambda_target raw(Omega_k)/raw(omega0).
 * Stand-in for the friction coefficients of the Keldysh analysis (appendix,
 * Eq. 27), which the paper does not give in closed form. */
typedef struct {
  double T, omega0, gamma_s, omega_l, gamma_l, a_l, d;
  int nq, nw;
  double q_max, w_max;
  double lambda_target;
  int dispersion;
  int coupling;
  double v_l;
} lbm_spectral;

typedef struct lbm_ctx lbm_ctx; /* opaque */

/* Device bytes lbm_create() needs for a channel (the nanochannel of Sec. 2:
 * its box, wall geometry and lattice) -- populations, wall tables,
 * reduction partials; for admission by footprint.  LBM_EINVAL on bad
 * parameters. */
lbm_status lbm_footprint(const lbm_params *p, size_t *bytes);

/* Set up a channel: classify cells and wall links (Sec. 4.2 boundary sites),
 * carve the arena, set no-slip walls (lambda = +inf) and the rest state
 * g_i = 0 (f_i = w_i rho0).  arena: device pointer, >= footprint bytes,
 * 256-byte aligned, owned by the caller.  hip_stream: a hipStream_t (NULL =
 * default stream). */
lbm_status lbm_create(const lbm_params *p, void *arena, size_t arena_bytes,
                      void *hip_stream, lbm_ctx **out);
void lbm_destroy(lbm_ctx *ctx); /* never frees the arena */

/* Fluid cells, and wall nodes: the fluid sites next to the liquid/solid
 * interface, where the boundary rules of Sec. 4.2 apply (a site with a
 * link whose upstream point is solid). */
lbm_status lbm_fluid_count(const lbm_ctx *ctx, size_t *n);
lbm_status lbm_wall_count(const lbm_ctx *ctx, size_t *n);
/* xyz: host, 3*wall_count int32 (x, y, z) per wall node, canonical order */
lbm_status lbm_wall_coords(const lbm_ctx *ctx, int32_t *xyz);
/* links: host, wall_count * Q doubles: fraction q in (0, 1] of the link from
 * the node to the wall along -c_i for every wall link (0.5 on planar walls),
 * 0 where the upstream point is fluid (the interface links of Sec. 4.2). */
lbm_status lbm_wall_links(const lbm_ctx *ctx, double *links);

/* Friction per wall node, lattice units, canonical order: lambda >= 0,
 * +inf = no slip (bounce-back, end of Sec. 4.2), 0 = free slip.  The wall
 * rule mixes bounce-back and transverse reversal with r = 3l/(1+3l), which
 * gives slip length nu/lambda on planar walls.  on_device != 0: lambda is a
 * device pointer.  n must equal wall_count.  Negative or NaN -> LBM_EINVAL
 * (nothing changed).  Synchronous. */
lbm_status lbm_set_friction(lbm_ctx *ctx, const double *lambda, size_t n,
                            int on_device);
/* Run the friction quadrature on the GPU for every wall node (Omega: the
 * node's plasmon frequency, canonical order, n = wall_count) and set the wall
 * from the result: the linear friction coefficient of the Keldysh analysis
 * (appendix, Eq. 27) as a (q, omega) sum over the two surfaces' response
 * spectra (lbm_spectral above), the plasmon frequency standing for the
 * charge-carrier density of Sec. 5.1.  Host or device Omega (finite, >= 0,
 * else LBM_EINVAL); bad spectral parameters -> LBM_EINVAL.  Synchronous. */
lbm_status lbm_set_friction_spectral(lbm_ctx *ctx, const lbm_spectral *sp,
                                     const double *omega, size_t n,
                                     int on_device);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * friction quadrature of lbm_set_friction_spectral without a context.
 * omega: device, n plasmon frequencies (finite, >= 0; not checked here: a
 * bad value gives a NaN lambda); lambda: device, n doubles out, the lattice
 * friction lambda_target raw(Omega_k) / raw(omega0), bit for bit what
 * lbm_set_friction_spectral computes for the same spectra and frequencies
 * (lambda may alias omega).  Both arrays are owned by the caller.
 * hip_stream: a hipStream_t (NULL = default stream); asynchronous, no
 * synchronisation, no allocation, no memset, so it may be captured.  The raw
 * quadrature sums live in a fixed device array of LBM_STATIC_MAX_NODES + 1
 * doubles (8 MiB) per GPU, held until the process ends and shared by every
 * call on that GPU: calls that overlap on one GPU (on different streams
 * without ordering) race.  n > LBM_STATIC_MAX_NODES or invalid spectral
 * parameters -> LBM_EINVAL; a failed launch -> LBM_EDEVICE. */
#define LBM_STATIC_MAX_NODES ((size_t)1 << 20)
lbm_status lbm_friction_quadrature_static(const lbm_spectral *sp, const double *omega, size_t n,
                                          double *lambda, void *hip_stream);

/* Current friction: lambda (lattice units) and, after a spectral set, the raw
 * quadrature sums (raw has wall_count + 1 entries, the last being
 * raw(omega0)); either pointer may be NULL.  Host arrays. */
lbm_status lbm_get_friction(lbm_ctx *ctx, double *lambda, double *raw);

/* Thermal fluctuations (fluctuating LB).  Sec. 3.2, Eq. 6: the classical
 * fluctuation-dissipation theorem fixes the random momentum flux; Sec. 4,
 * Eq. 17: the fluctuating LB equation adds it as a local source along
 * w_i (c_ia c_ib - c_s^2 delta_ab).  From the next step on, every fluid cell's
 * post-collision populations gain a zero-mean Gaussian term xi_i:
 *   LBM_NOISE_STRESS  the paper's source: a random symmetric tensor P with
 *       <P_ab P_cd> = A^2 c_s^4 (d_ac d_bd + d_ad d_bc), xi_i = w_i/(2 c_s^4)
 *       P:(c_i c_i - c_s^2 I);
 *   LBM_NOISE_ALL     every non-conserved direction: xi = A times the part of
 *       (sqrt(w_i) z_i) orthogonal to mass and momentum, z_i iid normals;
 * A^2 = mu (1 - (1 - 1/tau)^2), mu = 3 rho0 kT.  LBM_NOISE_ALL holds the
 * equilibrium populations at variance mu w_i, so that <rho u_a^2> = kT and
 * <(rho - rho0)^2> = 3 rho0 kT per site at every wavelength; the stress
 * source alone gives that only at long wavelengths (about 0.6 kT per site at
 * tau = 0.7).  kT is in lattice units (0 switches the noise off; the mode is
 * then ignored).  Random numbers: Philox4x64-10 (Salmon et al., SC'11) under
 * key (seed, 0) with counter (x + nx (y + ny z), step, block, 0), each 64-bit
 * word giving two Box-Muller normals from 23-bit uniforms (|z| <= 5.77),
 * transformed in binary64 with F64 storage and in binary32 (hardware log2,
 * sin, cos) with F32 and F16S storage, so a run is reproducible bit for bit and a restart from lbm_set_state continues
 * the same sequence.  Mass is conserved exactly; momentum too where the walls
 * conserve it.  kT < 0, NaN, Inf or an unknown mode -> LBM_EINVAL.
 * Synchronous (finishes queued work). */
typedef enum { LBM_NOISE_STRESS = 1, LBM_NOISE_ALL = 2 } lbm_noise;
lbm_status lbm_set_thermal(lbm_ctx *ctx, double kT, int mode, uint64_t seed);

/* One-point closure of the quantum fluctuations (Sec. 4, Eq. 18): the
 * two-point quantum correlator of the fluctuating forces (Eq. 7), whose lag
 * dependence Gamma_ab the Keldysh analysis would supply, averaged over
 * spatial lags r and time lags s into a one-point tensor
 *   m_ab = sum_r sum_s W_x(r) W_t(s) Gamma_ab(r, s),
 * which scales the variance of each component of the random stress of the
 * stress-source noise (LBM_NOISE_STRESS): P_ab -> sqrt(m_ab) P_ab, the same
 * Philox normals as the classical noise.  gamma: host, 6 * nr * ns doubles,
 * the components xx, yy, zz, xy, xz, yz in that order, each an nr x ns table
 * indexed [r][s]; wx (nr) and wt (ns) the weights.  A 2-D lattice ignores
 * zz, xz and yz.  Every m_ab must be finite and >= 0 (else LBM_EINVAL); a
 * unit correlator with weights summing to one gives the classical noise bit
 * for bit; gamma == NULL restores it.  Takes effect with the stress-source
 * noise (lbm_set_thermal); kept across lbm_set_thermal calls.  Batches carry
 * each member's factors.  Synchronous (finishes queued work). */
lbm_status lbm_set_noise_closure(lbm_ctx *ctx, const double *gamma, int nr, int ns,
                                 const double *wx, const double *wt);

/* Open x ends: the Neumann-like inlet and outlet of Sec. 4.2 (the option the
 * paper sets beside periodic ends) in place of periodic x.  From the next
 * step on, a fluid link of the first (last) node of an x-line that would
 * pull from x = -1 (x = nx) reads a ghost node instead.  The ghost copies the
 * populations of its neighbour inside the box -- the boundary node b in the
 * ghost's own column -- moved along the local equilibrium to the density
 * prescribed at that end (zero normal gradient of velocity and of the
 * non-equilibrium part; Dirichlet density, i.e. pressure c_s^2 rho):
 *   ghost_i = g_i(b) + w_i (rho_bc - rho_b) (1 + 3 c_i.u_b + 4.5 (c_i.u_b)^2
 *                                             - 1.5 u_b.u_b),
 * rho_b = rho0 + sum_k g_k(b), u_b = sum_k g_k(b) c_k / rho_b, rho_bc =
 * rho_in at x = -1 and rho_out at x = nx.  A pressure drop rho_in > rho_out
 * then drives the flow of the body force c_s^2 (rho_in - rho_out) / (nx + 1).
 * On a TUBE an interpolated wall link whose node behind (x + c_i) lies
 * beyond an end reads the ghost there (of the boundary node of that column).
 * A MASKED wall continues past each end as that end's row of the mask, which
 * must be the same at both ends (x = 0 and x = nx - 1): the wall links are
 * then those of the periodic channel.  Fields, flux and mass take the ghosts
 * too; mass is no longer conserved.  open = 0 restores periodic x (the
 * densities are then ignored).  Requires nx >= 2, no electron sheets, finite
 * densities > 0, equal end rows of a mask (else LBM_EINVAL); batches refuse
 * such channels.  Synchronous (finishes queued work). */
lbm_status lbm_set_open_ends(lbm_ctx *ctx, int open, double rho_in, double rho_out);

/* Electron wind (SLAB, DUCT and TUBE).  Sec. 3.3 describes the electrons of the solid
 * as a fluid dragged by, and dragging, the water; Sec. 4 gives each species
 * its own set of distributions; Eq. 5 / Eq. 27 make the interfacial force a
 * drag on the relative velocity, equal and opposite for the two species.
 * Every solid column next to the water (a "shell") carries one electron line
 * along x -- shells y = -1 and y = ny (by z), then for a duct z = -1 and
 * z = nz (by y), nshell = 2 nz (+ 2 ny for a duct); for a TUBE the solid
 * columns with a fluid column next to them along y or z, by increasing
 * y + ny z (lbm_shell_count): D1Q3
 * populations (c = 0, +1, -1; w = 2/3, 1/6, 1/6; stored as deviations from
 * w_i rho_e0, double), BGK with tau_e, Guo forcing with
 *   F = force_e (a field drive along x) + F_wall - gamma_e rho_e u_e
 * (the last term: drag on the lattice).  The water's wall rule keeps its
 * mixture r BB + (1 - r) (transverse reversal), but the bounce-back half
 * reflects off a wall moving with the electrons of the solid point x - c_i,
 *   BB_i = g_opp(i)(x) + 6 w_i rho0 c_ix u_e(x - c_i),
 * (on a TUBE the interpolated bounce-back, the moving-wall term divided by
 * 2q where the wall lies farther than half a link, as Bouzidi, Firdaouss and
 * Lallemand move their walls, so that a uniform flow at u_e stays exact),
 * and F_wall hands the electrons exactly the axial momentum the water gains
 * there (the free-slip half exchanges none), so water plus electrons change
 * axial momentum only by the external forces and the lattice drag.  Each
 * step runs the electrons first (from the water state of that step), then
 * the water with that u_e.  At steady state the lines' drag takes exactly
 * what the forces put in, gamma_e sum rho_e u_e = F_x N_fluid + force_e
 * N_lines; in a slab the sheets then move at one U_e and the water is the
 * slip-Poiseuille profile shifted by it.
 * Requires a SLAB, DUCT or TUBE (MASKED gives LBM_EINVAL; so does a TUBE
 * whose wall touches the box's edge, where no solid column holds a line),
 * wall_velocity_top == 0, periodic x ends, tau_e > 1/2, rho_e0 > 0,
 * gamma_e >= 0, finite values (else LBM_EINVAL); tau_e == 0 switches the
 * sheets off.
 * Fields, flux and mass (the moments the next collision would see) take
 * the wall velocity from the last step's u_e.
 * Switching on resets the electrons to rest.  The electron and phonon lines
 * are part of the checkpoint (lbm_get_state / lbm_set_state) while they are
 * on; lbm_transfer_state copies the water only; a batch takes channels with
 * lines when all its members have them.  Synchronous. */
lbm_status lbm_set_electrons(lbm_ctx *ctx, double tau_e, double rho_e0,
                             double gamma_e, double force_e);
/* u_e of the last step (nshell * nx doubles, [shell][x]) and the current
 * electron populations (3 * nshell * nx, [i][shell][x]); host arrays,
 * either may be NULL.  LBM_ESTATE if the sheets are off.  Synchronous. */
lbm_status lbm_get_electrons(lbm_ctx *ctx, double *ue, double *pops);

/* Phonon lines (Sec. 3.4): a third population set, one D1Q3 line beside every
 * electron line, BGK with tau_p around rho_p0.  The electron-phonon drag acts
 * equal and opposite on the two (Eq. 27): -G (u_e - u_p) on the electrons and
 * +G (u_e - u_p) on the phonons, G = gamma_ep rho_e at the node; the crystal
 * damps the phonons, -gamma_pc rho_p u_p.  Phonons do not touch the water.
 * With Guo's half-forces both velocities come from one 2 x 2 solve per node,
 * in the electron step.  Water, electrons and phonons then change axial
 * momentum only by the external forces and the two crystal drags; at steady
 * state U_p = G U_e / (G + gamma_pc rho_p0).  Requires the electron lines
 * on (else LBM_EINVAL); tau_p > 1/2, rho_p0 > 0, gamma_pc, gamma_ep >= 0,
 * finite; tau_p == 0 switches them off; lbm_set_electrons switches them off.
 * Resets the phonons to rest.  Synchronous. */
lbm_status lbm_set_phonons(lbm_ctx *ctx, double tau_p, double rho_p0, double gamma_pc,
                           double gamma_ep);
/* u_p of the last step (nshell * nx doubles) and the current phonon
 * populations (3 * nshell * nx, [i][shell][x]); host arrays, either may be
 * NULL.  LBM_ESTATE if the phonons are off.  Synchronous. */
lbm_status lbm_get_phonons(lbm_ctx *ctx, double *up, double *pops);
/* Number of electron shells (lines along x; Sec. 3.3, the electrons of the
 * solid next to the water) of the channel: SLAB 2 nz, DUCT 2 nz + 2 ny, TUBE
 * the solid columns with a fluid column next to them along y or z (numbered
 * by increasing y + ny z), 0 otherwise. */
lbm_status lbm_shell_count(const lbm_ctx *ctx, size_t *n);

/* Autotuner of the channel kernels: the block width (threads per workgroup
 * along an x-line: 64, 128, 256 or 512, no wider than the x-line) of the
 * step kernel of this kind of channel (lattice, storage, geometry, noise
 * form, electron lines, open ends, and a size bucket: log2 of nx and of the
 * fluid columns).  Takes the width a previous search chose in this process,
 * else times 20 real steps of this channel at every allowed width and keeps
 * and caches the fastest, the default width unless another is more than 1 %
 * faster.  The search starts from a host copy of the checkpoint
 * (lbm_state_bytes of host memory, LBM_ENOMEM without it) and puts it back:
 * state, electron and phonon lines, step count and a pending checked step
 * are as before the call.  flags LBM_TUNE_RETIME searches
 * even if cached.  *bx and *us (the chosen width's step time in
 * microseconds, 0 when taken from the cache) may be NULL.  Results never
 * depend on the width: the step's arithmetic is per cell, and the
 * reductions (invariants, checked steps) keep the default blocks.
 * Synchronous. */
#define LBM_TUNE_RETIME 1
lbm_status lbm_tune(lbm_ctx *ctx, int flags, int *bx, double *us);
/* Set the step kernel's block width directly (as lbm_tune; 0: the default,
 * min(nx rounded up to 64, 512)); LBM_EINVAL for a width not allowed.
 * Synchronous. */
lbm_status lbm_set_block(lbm_ctx *ctx, int bx);

/* Advance nsteps >= 0 time steps (asynchronous).  One step is the LB update
 * of Sec. 4 for the water: pull streaming, the wall rule at the liquid/solid
 * links (Sec. 4.2; Navier-slip friction of Eq. 5 / Eq. 27), BGK collision
 * with the bulk force of Eq. 2 as a Guo source; plus the species and noise
 * switched on by the lbm_set_* calls below. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t nsteps);
/* Run to the steady state the paper's permeability questions ask for (the
 * steady flux through the channel, Sec. 5.1): step in chunks of
 * check_every until |Q(a) - Q(b)| < rel_tol |Q(a)| for the fluxes Q of two
 * states check_every steps apart, or max_steps (LBM_ENOTCONV) or a NaN/Inf
 * (LBM_EDIVERGED).  Each chunk's last step reduces the flux of the state it
 * reads (lbm_step_checked), so the flux compared is that of one step before
 * each chunk's end (the first chunk's against the starting state).
 * steps_taken may be NULL.  Synchronous. */
lbm_status lbm_run_to_steady(lbm_ctx *ctx, double rel_tol, int64_t check_every,
                             int64_t max_steps, int64_t *steps_taken);
/* Advance nsteps >= 1 steps like lbm_step, the last of which also sums in
 * FP64, per block, the flux and mass of the populations its collision sees:
 * the invariants of the state one step before the end (asynchronous).  For
 * planar and tube walls without noise, electron lines, masked walls or open
 * ends the sums are fused into that step (no extra pass over the state) and
 * equal lbm_invariants' bit for bit with F64 and F32 storage; otherwise a
 * separate moments pass runs before the last step. */
lbm_status lbm_step_checked(lbm_ctx *ctx, int64_t nsteps);
/* Finish the reduction of the last lbm_step_checked: out as lbm_invariants
 * for the state at step *at_step (may be NULL), the step before that call's
 * end.  LBM_ESTATE if no checked step ran since the context's last
 * reduction pass or state change (lbm_invariants, lbm_get_field,
 * lbm_set_state, ...).  Synchronous; may be called again (same result). */
lbm_status lbm_checked_invariants(lbm_ctx *ctx, double out[3], int64_t *at_step);

/* Invariants of the current state (the moments the next collision sees):
 * out[0] = flux Q = (1/nx) sum_fluid rho u_x -- the mass flow through a
 * cross-section, the permeability measure of Sec. 5.1 --, out[1] = mass
 * M = sum_fluid rho (conserved by Eq. 1 with periodic ends and planar
 * walls), out[2] = sum_fluid (rho - rho0).  Deterministic FP64 reductions.
 * lbm_flux and lbm_mass return out[0] and out[1].  NaN/Inf ->
 * LBM_EDIVERGED.  Synchronous. */
lbm_status lbm_invariants(lbm_ctx *ctx, double out[3]);
/* The same invariants, enqueued: host_out[0..2] (flux, mass, mass deviation)
 * are written when the context's stream reaches this point (the caller
 * waits for the stream or an event recorded after the call before reading
 * them; NaN/Inf are not flagged).  host_out: page-locked host memory
 * (hipHostMalloc or a pinned allocation of the caller's), 3 doubles, owned by
 * the caller and valid until then; with pageable memory the copy, and the
 * call, wait for the stream.  Asynchronous: a serving loop checks many
 * channels without draining the queue once per channel. */
lbm_status lbm_invariants_async(lbm_ctx *ctx, double *host_out);
lbm_status lbm_flux(lbm_ctx *ctx, double *q);
lbm_status lbm_mass(lbm_ctx *ctx, double *m);
/* The hydrodynamic fields of Eqs. 1-2 as the LB moments of Sec. 4 (the
 * populations the next collision sees, with Guo's half-force): which: 0 rho,
 * 1 u_x, 2 u_y, 3 u_z; host_out: nz*ny*nx doubles, 0 on solid cells.
 * Synchronous. */
lbm_status lbm_get_field(lbm_ctx *ctx, int which, double *host_out);
/* The distribution functions of Sec. 4 as shifted post-collision
 * populations g_i = f_i - w_i rho0, doubles, host_out: Q*nz*ny*nx
 * ([i][z][y][x]), 0 on solid cells.  Synchronous. */
lbm_status lbm_get_populations(lbm_ctx *ctx, double *host_out);
/* The inverse: replace the state by host_in (same layout; solid cells
 * ignored), rounded to nearest in the storage precision, and set the step
 * counter to step >= 0.  A NaN, or a value the storage cannot hold (half:
 * |g| > 65504 / 2^12), is rejected with LBM_EINVAL and the state left
 * unchanged.  Synchronous. */
lbm_status lbm_set_populations(lbm_ctx *ctx, const double *host_in, int64_t step);

/* Checkpoint: the populations in storage precision plus the step counter;
 * with electron lines on (lbm_set_electrons) also the electron and phonon
 * populations and their velocities of the last step, so that a restored run
 * continues the same run.  lbm_state_bytes gives the size for the context's
 * current settings (LBM_EINVAL on a size mismatch, e.g. a state taken with
 * the lines on restored with them off); get/set are synchronous; set
 * restores a state bit for bit. */
lbm_status lbm_state_bytes(const lbm_ctx *ctx, size_t *bytes);
lbm_status lbm_get_state(lbm_ctx *ctx, void *host_buf, size_t bytes,
                         int64_t *step);
lbm_status lbm_set_state(lbm_ctx *ctx, const void *host_buf, size_t bytes,
                         int64_t step);

/* Time steps taken (the context's own counter: it selects the buffer and
 * the counter-based random bits of each step). */
lbm_status lbm_step_count(const lbm_ctx *ctx, int64_t *step);

/* Copy the state of src into dst: populations (converted to dst's storage
 * precision, round to nearest), step counter and friction.  Both contexts
 * must have the same lattice, geometry and box; their precisions may differ
 * (e.g. a half-precision run handed to a float context to finish: the
 * mixed-precision solve; the paper fixes no precision).  Waits for src; the
 * copy runs on dst's stream and is complete on return. */
lbm_status lbm_transfer_state(lbm_ctx *dst, lbm_ctx *src);

/* ---- Batches (many channels, one kernel launch per step and group) --------
 * The batching the configurations of many uneven channels and of the
 * serving loop ask for (the design queries of Sec. 5.1: permeability against
 * radius and carrier density, one independent channel each).  A batch holds
 * contexts with the same lattice, storage precision, wall kind (TUBE or
 * planar) and thermal-noise form in member slots; sizes, tau, force,
 * friction, kT and noise seed may differ.  One launch per time step
 * advances a group of members over a work list of 64-lane items laid out in
 * whole workgroups that never share a column (wall columns first); runs of
 * 64 steps are replayed from captured hipGraphs.  Members are cut into
 * groups whose state fits the last-level cache (128 MiB by default, 96 MiB
 * for F16S storage, see lbm_batch_set_group_bytes); a call to lbm_batch_step
 * runs each group 64 steps at a time, so a group's populations stay cached
 * between its steps.  Groups are dealt round-robin to two streams by default
 * (see lbm_batch_set_streams): the batch stream and streams the batch
 * creates at the default priority, which wait for the batch stream's earlier
 * work and are joined back into it, so every call stays ordered on the batch
 * stream.  Members keep their own buffers, parameters and step counters,
 * and a member advanced in a batch is bit-for-bit the same as the member
 * advanced alone.  Their lbm_get_*, lbm_invariants and lbm_get_state calls
 * stay valid between batch calls; a member stepped, restored or transferred
 * outside the batch is taken up at its current step by the next batch call
 * (if its stream is not the batch stream, the caller orders the two).
 * Members join (lbm_batch_add) and leave (lbm_batch_remove) while the batch
 * runs: only the groups they touch get new work lists and graphs.  Members
 * must outlive their membership.  The members of a batch share the noise
 * form, the kind of x ends (all periodic or all open; each its own end
 * densities) and electron lines (on all or none; each its own line
 * parameters, and phonon lines or not; a step runs the group's line steps,
 * then its water step).  Batches refuse MASKED members (LBM_EINVAL);
 * lbm_batch_step refuses a member whose noise form, kind of ends or
 * electron lines changed after it joined, and takes up a changed kT, seed,
 * noise closure, end densities or line parameters. */
typedef struct lbm_batch lbm_batch; /* opaque */

/* Capacity of a batch made empty (lbm_batch_create_spec): the kind of its
 * members and the most members, work items and fluid columns it holds at
 * once (lbm_batch_member_cost gives a context's items and columns). */
typedef struct {
  int lattice;     /* lbm_lattice */
  int precision;   /* lbm_precision */
  int tube;        /* 1: TUBE members (interpolated walls), 0: SLAB / DUCT */
  int noise;       /* thermal-noise form of every member: 0 none, LBM_NOISE_* */
  int open_ends;   /* 1: every member has open x ends (lbm_set_open_ends), 0: periodic */
  int electrons;   /* 1: every member has electron lines (lbm_set_electrons), 0: none */
  int max_members;
  int64_t max_items, max_columns;
} lbm_batch_spec;
/* Work items (the most over every workgroup shape) and fluid columns a
 * context takes up in a batch; either pointer may be NULL. */
lbm_status lbm_batch_member_cost(const lbm_ctx *ctx, int64_t *items, int64_t *columns);
/* Device bytes of a batch of this capacity (member table, work list, column
 * ids, the reduction's per-item partials). */
lbm_status lbm_batch_spec_footprint(const lbm_batch_spec *spec, size_t *bytes);
/* An empty batch of that capacity.  arena: device, >= footprint bytes,
 * 256-byte aligned, owned by the caller (borrowed, never freed).
 * Synchronous. */
lbm_status lbm_batch_create_spec(const lbm_batch_spec *spec, void *arena, size_t arena_bytes,
                                 void *hip_stream, lbm_batch **out);
/* Device bytes a batch of exactly these contexts needs. */
lbm_status lbm_batch_footprint(lbm_ctx *const *ctxs, int n, size_t *bytes);
/* A batch of these n contexts in slots 0..n-1 (capacity for exactly them).
 * Synchronous.  LBM_EINVAL if the members differ in kind (see above) or one
 * appears twice. */
lbm_status lbm_batch_create(lbm_ctx *const *ctxs, int n, void *arena, size_t arena_bytes,
                            void *hip_stream, lbm_batch **out);
void lbm_batch_destroy(lbm_batch *b);  /* members and arena untouched */
/* Take ctx in, at its current step and state, into the lowest free slot
 * (*slot, may be NULL): it joins the first group with room for its state or
 * a new group, whose work list and graph are rebuilt; the other groups keep
 * theirs.  Synchronous (waits for the batch's queued steps).  LBM_EINVAL: a
 * member already, or of another kind; LBM_ENOMEM: no free slot or no room in
 * the work list (nothing changed). */
lbm_status lbm_batch_add(lbm_batch *b, lbm_ctx *ctx, int *slot);
/* Let ctx leave after the batch's queued steps (synchronous); its slot is
 * free again, its group's work list is rebuilt.  LBM_EINVAL if not a
 * member.  The context is untouched and may be stepped alone or join again. */
lbm_status lbm_batch_remove(lbm_batch *b, lbm_ctx *ctx);
/* Members now, and slots in use (the highest taken slot + 1); either may be
 * NULL. */
lbm_status lbm_batch_size(const lbm_batch *b, int *members, int *slots);
lbm_status lbm_batch_items(const lbm_batch *b, int64_t *nitems);
/* Advance every member nsteps steps (asynchronous, on the batch stream). */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps);
/* Per slot s < slots: out[3s] flux, out[3s+1] mass, out[3s+2] mass
 * deviation, as lbm_invariants (NaN for a free slot).  Deterministic FP64
 * reductions.  Synchronous. */
lbm_status lbm_batch_invariants(lbm_batch *b, double *out);

/* Autotuner settings: workgroup shape (waves per workgroup), group size in
 * bytes of state, streams; the timed step of the chosen setting and of the
 * default one (4 waves, default group size, 2 streams), in microseconds. */
typedef struct {
  int waves_per_group;
  size_t group_bytes;
  int streams;
  double us_per_step;          /* 0 when not timed (taken from the cache) */
  double us_per_step_default;  /* 0 when not timed */
  int cached;                  /* 1: taken from the process-wide cache */
  int64_t repacks;             /* lbm_batch_settings: times every group was laid out anew */
} lbm_batch_tuning;
/* Autotuner: for this kind of batch (lattice, storage, wall kind, noise
 * form, and a size bucket: log2 of its fluid cells and of its members) take
 * the setting a previous search chose in this process, else search: every
 * combination of 2, 4 or 8 waves per workgroup, groups of 64, 96, 128 or
 * 192 MiB of state and 1, 2 or 3 streams is laid out and timed on this
 * batch, the fastest kept and cached (the default, 4 waves, 128 MiB or 96
 * MiB for F16S, 2 streams, unless another is more than 1 % faster).
 * flags LBM_TUNE_RETIME: search even if
 * cached.  The timed launches write only the buffers the next step
 * overwrites: no state or counter changes, and no setting changes results.
 * *chosen may be NULL.  Synchronous. */
lbm_status lbm_batch_tune(lbm_batch *b, int flags, lbm_batch_tuning *chosen);
/* The current setting (us_* and cached zero). */
lbm_status lbm_batch_settings(const lbm_batch *b, lbm_batch_tuning *now);
/* Set the workgroup shape directly (1, 2, 4 or 8 waves; 4 at creation);
 * rebuilds the work list, synchronous. */
lbm_status lbm_batch_set_shape(lbm_batch *b, int waves_per_group);
/* Largest state (both buffers of every member) of one group, in bytes; a
 * member larger than that forms a group of its own; 0 puts every member in
 * one group (all members advance step by step together).  Regroups the
 * members in slot order and rewrites the work list; synchronous.  Results do
 * not depend on the grouping. */
lbm_status lbm_batch_set_group_bytes(lbm_batch *b, size_t bytes);
lbm_status lbm_batch_groups(const lbm_batch *b, int *ngroups);
/* Number of streams (1..4) the groups are dealt to; results do not depend
 * on it. */
lbm_status lbm_batch_set_streams(lbm_batch *b, int nstreams);
const char *lbm_batch_last_error(const lbm_batch *b);

/* Plain streaming device-to-device copy of `bytes` (a multiple of 16, both
 * pointers 16-byte aligned) on hip_stream, asynchronous.  Not part of the
 * method: it measures the copy-bandwidth ceiling the stream-collide kernel is
 * compared with, and calibrates the memory-traffic counters. */
lbm_status lbm_copy_probe(const void *src, void *dst, size_t bytes, void *hip_stream);
lbm_status lbm_sync(lbm_ctx *ctx);               /* waits, surfaces errors */
const char *lbm_last_error(const lbm_ctx *ctx);  /* owned by ctx */

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */

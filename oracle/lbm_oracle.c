/*
 * oracle/lbm_oracle.c -- plain, slow, obviously-correct CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header,
 * table or constant with the GPU library; it is written from the paper and the
 * readings listed in the design notes, in plain scalar loops, and computes in
 * `real` = double (or x87 long double when built with ORACLE_LONG_DOUBLE, to
 * bound its own rounding floor).
 *
 * What it computes (Keldysh-lattice-Boltzmann paper, arXiv 2403.15768):
 *
 *  - Water as one lattice-Boltzmann population set (Sec. 4, "one set of
 *    discrete distributions per species"; Eqs. 1-2 are the continuity and
 *    momentum equations it reproduces, inertia kept).  Lattices: D2Q9 with the
 *    velocity numbering the paper gives beside Eqs. 19-21 (0 = rest, 1 = +x,
 *    2 = +y, 3 = -x, 4 = -y, 5 = (+,+), 6 = (-,+), 7 = (-,-), 8 = (+,-)), and
 *    D3Q19 (0 rest; 1..6 = +x,-x,+y,-y,+z,-z; then (+,+,0),(-,-,0),(+,-,0),
 *    (-,+,0),(+,0,+),(-,0,-),(+,0,-),(-,0,+),(0,+,+),(0,-,-),(0,+,-),(0,-,+)).
 *  - Collision: single-relaxation-time BGK with the second-order equilibrium;
 *    body force (the pressure-gradient-like bulk force F of Eq. 2) by Guo's
 *    scheme.  The paper only says "well established procedures" (Sec. 4).
 *  - State: post-collision populations stored as deviations from the rest
 *    equilibrium, g_i = f_i - w_i rho0 ("shifted" storage).  Algebraically the
 *    textbook scheme; it only changes rounding.
 *  - Walls (Sec. 4.2): the paper's bounce-back rule for no-slip outer walls and
 *    its free-slip rule at the liquid/solid interface are mixed per wall node
 *    with weight r = 3 lambda / (1 + 3 lambda), lambda being the interfacial
 *    friction coefficient of the linear drag law (Eq. 5 and the appendix
 *    result F_kl = gamma_kl (u_k - u_l), Eq. 27) in lattice units.  The slip
 *    half is the same-node transverse reversal (c_x, -c_y, -c_z).  Bounce-back
 *    is half-way on planar walls and Bouzidi-Firdaouss-Lallemand linear
 *    interpolation on the circular tube.  Inlet/outlet are periodic in x (the
 *    first option of Sec. 4.2), or open (its Neumann-like option: ghost
 *    nodes rebuilt from the boundary node at a prescribed density, see
 *    open_ghost; a masked wall continues past an open end as that end's row
 *    of the mask).  Walls that vary along x (a solid mask in
 *    the (x, y) plane: corrugated, wrinkled or stepped walls) take the slip
 *    half from a pairing of the node's wall links (pair_slip_links) that
 *    keeps mass exact.
 *  - Friction quadrature: a (q, omega) midpoint sum of the imaginary parts of
 *    a Drude solid response and a Lorentzian liquid response with a thermal
 *    factor, optionally divided by the coupling denominator
 *    |1 - g_s g_l e^{-2qd}|^2 and with a q-dependent liquid mode; the paper
 *    states only that the Keldysh analysis yields linear friction
 *    coefficients (appendix, Eq. 27), so the spectra here are synthetic
 *    stand-ins of that form.
 *
 * Step n -> n+1, for every fluid cell x (no blocking, no fusion):
 *   1. pull:   df_i = g_i(x - c_i), periodic in x (and z for the slab);
 *              if x - c_i is solid, the wall rule gives df_i instead;
 *   2. moments: rho = rho0 + sum df_i;  rho u = sum df_i c_i + F/2;
 *   3. dfeq_i = w_i [ (rho - rho0) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u) ],
 *      with rho - rho0 taken as the summed deviation sum df_i;
 *   4. g_i(x, n+1) = df_i - (df_i - dfeq_i)/tau
 *                    + (1 - 1/(2 tau)) w_i [ 3 (c_i - u) + 9 (c_i.u) c_i ].F
 *   Reported rho, u "after n steps" are the moments of step 2 built from g(n).
 *
 * Thermal fluctuations (optional, Sec. 3.2 Eq. 6 and Sec. 4 Eq. 17): the
 * classical fluctuation-dissipation theorem fixes the random momentum flux,
 * and the fluctuating LB equation adds it as a local source in the stress
 * directions w_i (c_ia c_ib - c_s^2 delta_ab).  With a lattice temperature kT
 * (lattice units, equipartition reads <rho u_a^2> = kT per site), step 4
 * gains a zero-mean Gaussian term xi_i; see thermal_noise() below for the two
 * forms (the paper's stress source alone, or every non-conserved direction).
 * Electron wind (optional, SLAB): the solid's electrons as a second
 * population set on one sheet per wall, coupled to the water by the
 * relative-velocity drag (Sec. 3.3, Eq. 5, Eq. 27); see electron_step().
 * Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), a
 * counter-based generator, keyed by the seed and counted by (cell, step,
 * block), with Box-Muller (1958) normals.
 *
 * Parity pins: exact discrete slip-Poiseuille and Couette profiles, exact
 * mass conservation, free-slip plug acceleration, Hagen-Poiseuille
 * convergence in the tube, long-double self-floor; quadrature pinned by
 * complex-arithmetic brute force on tiny grids, the f-sum rule, the closed
 * form of the q integral and an adaptive integrator; thermal noise pinned by
 * numpy's Philox4x64-10, the normal distribution, exact conservation, the
 * paper's stress form and the stationarity of the equilibrium Gaussian
 * measure; electron wind pinned by exact per-step momentum bookkeeping and
 * exact coupled steady states (see tests/).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_LONG_DOUBLE
typedef long double real;
#define R_SQRT sqrtl
#define R_EXP expl
#define R_SINH sinhl
#define R_ISFINITE(v) isfinite(v)
#else
typedef double real;
#define R_SQRT sqrt
#define R_EXP exp
#define R_SINH sinh
#define R_ISFINITE(v) isfinite(v)
#endif

#define ORA_OK 0
#define ORA_EINVAL -1
#define ORA_ENOMEM -2

enum { ORA_SLAB = 0, ORA_DUCT = 1, ORA_TUBE = 2, ORA_MASKED = 3 };

/* Same field order as the GPU library's parameter struct, but declared here
 * independently: only the layout of plain numbers is common. */
typedef struct {
  int lattice;  /* 9 or 19 */
  int precision; /* ignored by the oracle (always real) */
  int geometry; /* ORA_SLAB / ORA_DUCT / ORA_TUBE / ORA_MASKED */
  int nx, ny, nz;
  double tube_radius, tube_cy, tube_cz;
  double tau, rho0;
  double force[3];
  double wall_velocity_top; /* moving top wall (y = ny - 1/2), slab/duct only */
  /* ORA_MASKED: solid points of the (x, y) plane, nx*ny bytes, x fastest,
   * nonzero = solid, the same for every z; read at creation only */
  const unsigned char *solid;
} ora_params;

typedef struct {
  ora_params p;
  int q;
  int c[19][3];
  real w[19];
  int opp[19];  /* c_opp = -c */
  int sig[19];  /* c_sig = (c_x, -c_y, -c_z) */
  long ncell;   /* nx*ny*nz */
  unsigned char *fluid;
  long *wall_id; /* canonical wall-node index or -1 */
  long nwall;
  long nfluid;
  real *r;     /* per cell (wall nodes only) */
  real *qlink; /* per cell * 19: Bouzidi fraction of wall links (0 if none) */
  unsigned char *mask;  /* ORA_MASKED: copy of the (x, y) solid mask */
  signed char *partner; /* ORA_MASKED: per cell * 19, slip partner of wall link i */
  real *g, *gn;
  long step;
  double kT;     /* lattice temperature; 0 = no fluctuations */
  int noise;     /* 1 = stress directions only, 2 = all non-conserved */
  /* open x ends (Neumann-like inlet and outlet): prescribed densities */
  int open;
  double rho_in, rho_out;
  uint64_t seed; /* key of the thermal random numbers */
  /* one-point closure of the quantum noise: square roots of the factors
   * m_c by which the stress components' variances are scaled, in the order
   * xx, yy, zz, xy, xz, yz (1 = classical) */
  real qfac[6];
  /* electron shells (SLAB, DUCT and TUBE): the solid columns next to the
   * water, each with an electron line along x, D1Q3 (see shell_of); TUBE:
   * their number and the shell of each column of the box (-1: none) */
  long tube_nsh;
  long *tube_shell;
  int elec;
  double tau_e, rho_e0, gamma_e, force_e;
  real *e, *en; /* shifted populations [i][shell][x], i = 0, +x, -x */
  real *ue;     /* electron velocity of the last step, [shell][x] */
  /* phonon lines beside the electron lines (Sec. 3.4), same layout */
  int phon;
  double tau_p, rho_p0, gamma_pc, gamma_ep;
  real *ph, *phn, *up;
} ora_ctx;

/* ---------------------------------------------------------------- lattice */

static void set_lattice(ora_ctx *o) {
  static const int d2q9[9][2] = {{0, 0}, {1, 0},  {0, 1},   {-1, 0}, {0, -1},
                                 {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
  static const int d3q19[19][3] = {
      {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
      {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
      {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
      {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  int i, k;
  o->q = o->p.lattice;
  for (i = 0; i < o->q; i++) {
    if (o->q == 9) {
      o->c[i][0] = d2q9[i][0];
      o->c[i][1] = d2q9[i][1];
      o->c[i][2] = 0;
    } else {
      o->c[i][0] = d3q19[i][0];
      o->c[i][1] = d3q19[i][1];
      o->c[i][2] = d3q19[i][2];
    }
  }
  /* weights from |c|^2: D2Q9 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36 */
  for (i = 0; i < o->q; i++) {
    int c2 = o->c[i][0] * o->c[i][0] + o->c[i][1] * o->c[i][1] +
             o->c[i][2] * o->c[i][2];
    if (o->q == 9)
      o->w[i] = c2 == 0 ? (real)4 / 9 : (c2 == 1 ? (real)1 / 9 : (real)1 / 36);
    else
      o->w[i] = c2 == 0 ? (real)1 / 3 : (c2 == 1 ? (real)1 / 18 : (real)1 / 36);
  }
  /* opposite and transverse reversal found by search over the velocity set */
  for (i = 0; i < o->q; i++) {
    o->opp[i] = -1;
    o->sig[i] = -1;
    for (k = 0; k < o->q; k++) {
      if (o->c[k][0] == -o->c[i][0] && o->c[k][1] == -o->c[i][1] &&
          o->c[k][2] == -o->c[i][2])
        o->opp[i] = k;
      if (o->c[k][0] == o->c[i][0] && o->c[k][1] == -o->c[i][1] &&
          o->c[k][2] == -o->c[i][2])
        o->sig[i] = k;
    }
  }
}

/* --------------------------------------------------------------- geometry */

static long cell(const ora_ctx *o, int x, int y, int z) {
  return (long)x + (long)o->p.nx * ((long)y + (long)o->p.ny * (long)z);
}

/* Electron shells: the solid columns next to the water that carry an
 * electron line along x.  Numbering: y = -1 (z = 0..nz-1), then y = ny,
 * then (DUCT only) z = -1 (y = 0..ny-1), then z = nz.  TUBE: the solid
 * columns of the box with a fluid column next to them along +-y or +-z (the
 * only transverse steps of the links that cross x), in increasing y + ny z.
 * -1 if (ys, zs) is none of them. */
static long nshell(const ora_ctx *o) {
  if (o->p.geometry == ORA_TUBE) return o->tube_nsh;
  return 2L * o->p.nz + (o->p.geometry == ORA_DUCT ? 2L * o->p.ny : 0);
}
static long shell_of(const ora_ctx *o, int ys, int zs) {
  if (o->p.geometry == ORA_TUBE) {
    if (ys < 0 || ys >= o->p.ny || zs < 0 || zs >= o->p.nz) return -1;
    return o->tube_shell[(long)ys + (long)o->p.ny * zs];
  }
  if (zs >= 0 && zs < o->p.nz) {
    if (ys == -1) return zs;
    if (ys == o->p.ny) return o->p.nz + zs;
  }
  if (o->p.geometry == ORA_DUCT && ys >= 0 && ys < o->p.ny) {
    if (zs == -1) return 2L * o->p.nz + ys;
    if (zs == o->p.nz) return 2L * o->p.nz + o->p.ny + ys;
  }
  return -1;
}
/* the shell's solid column (ys, zs) */
static void shell_column(const ora_ctx *o, long s, int *ys, int *zs) {
  long nz = o->p.nz, ny = o->p.ny;
  if (o->p.geometry == ORA_TUBE) {
    long c;
    for (c = 0; c < ny * nz; c++)
      if (o->tube_shell[c] == s) {
        *ys = (int)(c % ny);
        *zs = (int)(c / ny);
        return;
      }
  }
  if (s < 2 * nz) {
    *ys = s < nz ? -1 : (int)ny;
    *zs = (int)(s % nz);
  } else {
    s -= 2 * nz;
    *zs = s < ny ? -1 : (int)nz;
    *ys = (int)(s % ny);
  }
}

/* Is the lattice point (x, y, z) -- already wrapped in the periodic
 * directions -- a solid point? */
static int is_solid(const ora_ctx *o, int x, int y, int z) {
  if (y < 0 || y >= o->p.ny || z < 0 || z >= o->p.nz) return 1;
  if (o->p.geometry == ORA_MASKED) return o->mask[(long)x + (long)o->p.nx * y] != 0;
  if (o->p.geometry == ORA_TUBE) {
    double dy = (double)y - o->p.tube_cy, dz = (double)z - o->p.tube_cz;
    return !(dy * dy + dz * dz < o->p.tube_radius * o->p.tube_radius);
  }
  return 0;
}

/* upstream point of link i at (x, y, z): x - c_i with periodic wrap */
static void upstream(const ora_ctx *o, int x, int y, int z, int i, int *sx,
                     int *sy, int *sz) {
  *sx = ((x - o->c[i][0]) % o->p.nx + o->p.nx) % o->p.nx;
  *sy = y - o->c[i][1];
  *sz = z - o->c[i][2];
  if (o->p.geometry == ORA_SLAB || o->p.geometry == ORA_MASKED)
    *sz = ((*sz) % o->p.nz + o->p.nz) % o->p.nz;
}

/* Bouzidi fraction: distance from the fluid node P to the circular wall
 * along -c (in units of |c|, transverse plane only since the tube axis is x).
 * Solves |P - s C|^2 = R^2 for the root s in (0, 1]. */
static real bouzidi_q(const ora_ctx *o, int y, int z, int i) {
  real py = (real)y - (real)o->p.tube_cy, pz = (real)z - (real)o->p.tube_cz;
  real cy = (real)o->c[i][1], cz = (real)o->c[i][2];
  real a = cy * cy + cz * cz;
  real b = -2 * (py * cy + pz * cz);
  real cc = py * py + pz * pz - (real)o->p.tube_radius * (real)o->p.tube_radius;
  return (-b + R_SQRT(b * b - 4 * a * cc)) / (2 * a);
}

/* Slip partners on a masked wall (corrugated or stepped walls, Sec. 4.2 and
 * the wall-design remark of Sec. 5.1).  At a wall node the links whose
 * upstream point is solid (set J) and the links pointing into the solid (set
 * K = the opposites of J) have equal counts.  The slip half of the wall rule
 * hands each j in J the node's own population of one link k in K; when every
 * k is handed out exactly once, the weights r and 1 - r of every into-wall
 * population sum to one and mass is conserved exactly.  The pairing below
 * picks, in this order of preference and each time over j in increasing
 * direction index, among the links of K not yet handed out:
 *   1. the reflection about a wall normal to y, (c_x, -c_y, -c_z) -- the
 *      transverse reversal of the planar walls, so flat stretches of the
 *      mask behave exactly as the slab;
 *   2. the reflection about a wall normal to x, (-c_x, c_y, -c_z) -- step
 *      faces, where the slip keeps the flow along the face;
 *   3. the opposite -c_j (plain bounce-back);
 *   4. the lowest-numbered link of K still free.
 * Each pass maps distinct j to distinct k, so passes 1-3 commute with the
 * mirror images x -> -x and y -> -y of the geometry. */
static int find_dir(const ora_ctx *o, int cx, int cy, int cz) {
  int k;
  for (k = 0; k < o->q; k++)
    if (o->c[k][0] == cx && o->c[k][1] == cy && o->c[k][2] == cz) return k;
  return -1;
}
static void pair_slip_links(ora_ctx *o, int x, int y, int z, signed char *pt) {
  int inJ[19], inK[19], taken[19], i, pass, k;
  for (i = 0; i < 19; i++) {
    inJ[i] = inK[i] = taken[i] = 0;
    pt[i] = -1;
  }
  for (i = 1; i < o->q; i++) {
    int sx, sy, sz;
    upstream(o, x, y, z, i, &sx, &sy, &sz);
    if (is_solid(o, sx, sy, sz)) {
      inJ[i] = 1;
      inK[o->opp[i]] = 1;
    }
  }
  for (pass = 1; pass <= 4; pass++)
    for (i = 1; i < o->q; i++) {
      if (!inJ[i] || pt[i] >= 0) continue;
      if (pass == 1) k = find_dir(o, o->c[i][0], -o->c[i][1], -o->c[i][2]);
      else if (pass == 2) k = find_dir(o, -o->c[i][0], o->c[i][1], -o->c[i][2]);
      else if (pass == 3) k = o->opp[i];
      else
        for (k = 1; k < o->q && !(inK[k] && !taken[k]); k++) {
        }
      if (k >= 0 && k < o->q && inK[k] && !taken[k]) {
        pt[i] = (signed char)k;
        taken[k] = 1;
      }
    }
}

/* ------------------------------------------------------------- life cycle */

void ora_destroy(ora_ctx *o);

int ora_create(const ora_params *p, ora_ctx **out) {
  ora_ctx *o;
  int x, y, z, i;
  *out = NULL;
  if (!(p->lattice == 9 || p->lattice == 19)) return ORA_EINVAL;
  if (p->geometry < 0 || p->geometry > 3) return ORA_EINVAL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return ORA_EINVAL;
  if (p->lattice == 9 &&
      (p->nz != 1 || (p->geometry != ORA_SLAB && p->geometry != ORA_MASKED)))
    return ORA_EINVAL;
  if (!(p->tau > 0.5)) return ORA_EINVAL;
  if (p->wall_velocity_top != 0.0 && (p->geometry == ORA_TUBE || p->geometry == ORA_MASKED))
    return ORA_EINVAL;
  if (p->geometry == ORA_MASKED && !p->solid) return ORA_EINVAL;
  o = (ora_ctx *)calloc(1, sizeof(ora_ctx));
  if (!o) return ORA_ENOMEM;
  o->p = *p;
  for (i = 0; i < 6; i++) o->qfac[i] = 1;
  set_lattice(o);
  o->ncell = (long)p->nx * p->ny * p->nz;
  o->fluid = (unsigned char *)calloc(o->ncell, 1);
  o->wall_id = (long *)malloc(sizeof(long) * o->ncell);
  o->r = (real *)calloc(o->ncell, sizeof(real));
  o->qlink = (real *)calloc(o->ncell * 19, sizeof(real));
  o->g = (real *)calloc(o->ncell * o->q, sizeof(real));
  o->gn = (real *)calloc(o->ncell * o->q, sizeof(real));
  if (p->geometry == ORA_MASKED) {
    o->mask = (unsigned char *)malloc((size_t)p->nx * p->ny);
    o->partner = (signed char *)malloc((size_t)o->ncell * 19);
    if (o->mask) memcpy(o->mask, p->solid, (size_t)p->nx * p->ny);
  }
  o->p.solid = NULL; /* the caller's array is not kept */
  if (!o->fluid || !o->wall_id || !o->r || !o->qlink || !o->g || !o->gn ||
      (p->geometry == ORA_MASKED && (!o->mask || !o->partner))) {
    ora_destroy(o);
    return ORA_ENOMEM;
  }
  /* classify cells and wall links; wall nodes numbered by increasing linear
   * index x + nx (y + ny z) */
  o->nwall = 0;
  o->nfluid = 0;
  for (z = 0; z < p->nz; z++)
    for (y = 0; y < p->ny; y++)
      for (x = 0; x < p->nx; x++) {
        long n = cell(o, x, y, z);
        int is_wall = 0;
        o->wall_id[n] = -1;
        if (is_solid(o, x, y, z)) continue;
        o->fluid[n] = 1;
        o->nfluid++;
        for (i = 0; i < o->q; i++) {
          int sx, sy, sz;
          upstream(o, x, y, z, i, &sx, &sy, &sz);
          if (is_solid(o, sx, sy, sz)) {
            is_wall = 1;
            o->qlink[n * 19 + i] =
                p->geometry == ORA_TUBE ? bouzidi_q(o, y, z, i) : (real)0.5;
          }
        }
        if (is_wall) {
          o->wall_id[n] = o->nwall++;
          o->r[n] = 1; /* default: no-slip bounce-back */
        }
        if (p->geometry == ORA_MASKED) pair_slip_links(o, x, y, z, o->partner + n * 19);
      }
  if (p->geometry == ORA_MASKED && o->nfluid == 0) {
    ora_destroy(o);
    return ORA_EINVAL;
  }
  if (p->geometry == ORA_TUBE) {
    o->tube_shell = (long *)malloc(sizeof(long) * p->ny * p->nz);
    if (!o->tube_shell) {
      ora_destroy(o);
      return ORA_ENOMEM;
    }
    o->tube_nsh = 0;
    for (z = 0; z < p->nz; z++)
      for (y = 0; y < p->ny; y++) {
        long c = (long)y + (long)p->ny * z;
        o->tube_shell[c] = -1;
        if (!is_solid(o, 0, y, z)) continue;
        if (!is_solid(o, 0, y - 1, z) || !is_solid(o, 0, y + 1, z) ||
            !is_solid(o, 0, y, z - 1) || !is_solid(o, 0, y, z + 1))
          o->tube_shell[c] = o->tube_nsh++;
      }
  }
  *out = o;
  return ORA_OK;
}

void ora_destroy(ora_ctx *o) {
  if (!o) return;
  free(o->e);
  free(o->en);
  free(o->ue);
  free(o->ph);
  free(o->phn);
  free(o->up);
  free(o->tube_shell);
  free(o->fluid);
  free(o->wall_id);
  free(o->r);
  free(o->qlink);
  free(o->mask);
  free(o->partner);
  free(o->g);
  free(o->gn);
  free(o);
}

long ora_wall_count(const ora_ctx *o) { return o->nwall; }
long ora_fluid_count(const ora_ctx *o) { return o->nfluid; }
long ora_step_count(const ora_ctx *o) { return o->step; }

/* xyz: 3*nwall ints (x, y, z) in canonical order */
void ora_wall_coords(const ora_ctx *o, int32_t *xyz) {
  int x, y, z;
  for (z = 0; z < o->p.nz; z++)
    for (y = 0; y < o->p.ny; y++)
      for (x = 0; x < o->p.nx; x++) {
        long k = o->wall_id[cell(o, x, y, z)];
        if (k >= 0) {
          xyz[3 * k] = x;
          xyz[3 * k + 1] = y;
          xyz[3 * k + 2] = z;
        }
      }
}

/* Bouzidi fractions of the wall links: out[k*19 + i] for wall node k */
void ora_wall_links(const ora_ctx *o, double *out) {
  long n;
  int i;
  for (n = 0; n < o->ncell; n++) {
    long k = o->wall_id[n];
    if (k < 0) continue;
    for (i = 0; i < 19; i++) out[k * 19 + i] = (double)o->qlink[n * 19 + i];
  }
}

/* lambda in lattice units per wall node (canonical order); +inf = no slip.
 * r = 3 lambda / (1 + 3 lambda) makes the slip length nu / lambda. */
int ora_set_friction(ora_ctx *o, const double *lambda) {
  long n;
  for (n = 0; n < o->ncell; n++) {
    long k = o->wall_id[n];
    if (k < 0) continue;
    if (!(lambda[k] >= 0)) return ORA_EINVAL; /* rejects NaN and < 0 */
  }
  for (n = 0; n < o->ncell; n++) {
    long k = o->wall_id[n];
    real l;
    if (k < 0) continue;
    l = (real)lambda[k];
    o->r[n] = isinf(lambda[k]) ? (real)1 : 3 * l / (1 + 3 * l);
  }
  return ORA_OK;
}

/* ------------------------------------------------------------ the update */

/* Value of the incoming population i at fluid cell (x,y,z) whose upstream
 * point is solid: the Navier-slip wall rule. */
static real open_ghost(const ora_ctx *o, const real *g, int xb, int yb, int zb,
                       int i, double rho_bc);

static real wall_value(const ora_ctx *o, const real *g, int x, int y, int z,
                       int i, int sy) {
  long n = cell(o, x, y, z);
  int ib = o->opp[i];
  real bb, qv, mw;
  /* moving top wall (Couette check): bounce-back plus the momentum the wall
   * hands over, 6 w_i rho0 (c_i . U) with U along x */
  if (o->p.wall_velocity_top != 0.0 && sy >= o->p.ny)
    return g[(long)ib * o->ncell + n] +
           6 * o->w[i] * (real)o->p.rho0 * (real)o->c[i][0] *
               (real)o->p.wall_velocity_top;
  qv = o->qlink[n * 19 + i];
  mw = 1; /* weight of the moving-wall term in bb */
  if (o->p.geometry != ORA_TUBE) {
    bb = g[(long)ib * o->ncell + n]; /* half-way bounce-back */
  } else if (qv < (real)0.5) {
    /* wall closer than half a link: interpolate between this node's and the
     * next node's (along +c_i) populations heading into the wall; with open
     * ends, a next node beyond x = 0 or x = nx - 1 is a ghost node, whose
     * population is the open_ghost of the boundary node of its column */
    int xr = x + o->c[i][0];
    int xn = (xr % o->p.nx + o->p.nx) % o->p.nx;
    int yn = y + o->c[i][1], zn = z + o->c[i][2];
    if (is_solid(o, xn, yn, zn)) {
      bb = g[(long)ib * o->ncell + n];
    } else {
      real behind;
      if (o->open && (xr < 0 || xr >= o->p.nx))
        behind = open_ghost(o, g, x, yn, zn, ib, xr < 0 ? o->rho_in : o->rho_out);
      else
        behind = g[(long)ib * o->ncell + cell(o, xn, yn, zn)];
      bb = 2 * qv * g[(long)ib * o->ncell + n] + (1 - 2 * qv) * behind;
    }
  } else {
    /* wall farther than half a link: interpolate between the bounced
     * population and this node's own outgoing population i; a moving wall's
     * term is divided by 2q as well (Bouzidi, Firdaouss and Lallemand), so
     * that a uniform flow at the wall's velocity stays exact */
    bb = g[(long)ib * o->ncell + n] / (2 * qv) +
         (2 * qv - 1) / (2 * qv) * g[(long)i * o->ncell + n];
    mw = 1 / (2 * qv);
  }
  if (o->elec && o->c[i][0] != 0) {
    /* the wall moves with the electrons of the solid point x - c_i */
    int xs = ((x - o->c[i][0]) % o->p.nx + o->p.nx) % o->p.nx;
    int zs = z - o->c[i][2];
    if (o->p.geometry == ORA_SLAB) zs = (zs % o->p.nz + o->p.nz) % o->p.nz;
    bb += mw * 6 * o->w[i] * (real)o->p.rho0 * (real)o->c[i][0] *
          o->ue[shell_of(o, sy, zs) * o->p.nx + xs];
  }
  if (o->p.geometry == ORA_MASKED)
    return o->r[n] * bb + (1 - o->r[n]) * g[(long)o->partner[n * 19 + i] * o->ncell + n];
  return o->r[n] * bb + (1 - o->r[n]) * g[(long)o->sig[i] * o->ncell + n];
}

/* Open x ends (the Neumann-like option for inlet and outlet, Sec. 4.2).
 * A link that pulls from beyond the box in x (x - c_i outside 0..nx-1) reads
 * a ghost node just outside the end.  The ghost copies the populations of
 * its neighbour inside the box, the boundary node b in the ghost's own
 * column (zero normal gradient of velocity and of the non-equilibrium part),
 * moved along the local equilibrium to the density prescribed at that end:
 *   ghost_i = g_i(b) + w_i (rho_bc - rho_b) (1 + 3 c_i.u_b + 4.5 (c_i.u_b)^2
 *                                             - 1.5 u_b.u_b),
 * with rho_b = rho0 + sum_k g_k(b) and u_b = sum_k g_k(b) c_k / rho_b the
 * moments of b's stored populations.  rho_bc is rho_in at x = -1 and rho_out
 * at x = nx; the pressure c_s^2 rho_bc is the drive. */
/* Masked walls continue past each open end as that end's row of the mask;
 * with equal first and last rows this continuation and the periodic one
 * give every node the same wall links (and slip pairs). */
static int mask_ends_equal(const ora_ctx *o) {
  int y;
  for (y = 0; y < o->p.ny; y++)
    if ((o->mask[(long)o->p.nx * y] != 0) != (o->mask[(long)o->p.nx * y + o->p.nx - 1] != 0))
      return 0;
  return 1;
}

int ora_set_open_ends(ora_ctx *o, int open, double rho_in, double rho_out) {
  if (open && ((o->p.geometry == ORA_MASKED && !mask_ends_equal(o)) || o->elec ||
               o->p.nx < 2 || !(rho_in > 0) || !(rho_out > 0) || !isfinite(rho_in) ||
               !isfinite(rho_out)))
    return ORA_EINVAL;
  o->open = open ? 1 : 0;
  o->rho_in = rho_in;
  o->rho_out = rho_out;
  return ORA_OK;
}

static real open_ghost(const ora_ctx *o, const real *g, int xb, int yb, int zb,
                       int i, double rho_bc) {
  long nb = cell(o, xb, yb, zb);
  real drho = 0, j[3] = {0, 0, 0}, rho, u[3], cu, usq;
  int k, a;
  for (k = 0; k < o->q; k++) {
    real v = g[(long)k * o->ncell + nb];
    drho += v;
    for (a = 0; a < 3; a++) j[a] += (real)o->c[k][a] * v;
  }
  rho = (real)o->p.rho0 + drho;
  for (a = 0; a < 3; a++) u[a] = j[a] / rho;
  cu = (real)o->c[i][0] * u[0] + (real)o->c[i][1] * u[1] + (real)o->c[i][2] * u[2];
  usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return g[(long)i * o->ncell + nb] +
         o->w[i] * (((real)rho_bc - (real)o->p.rho0) - drho) *
             (1 + 3 * cu + (real)4.5 * cu * cu - (real)1.5 * usq);
}

/* steps 1 and 2: gather the populations a collision at (x,y,z) sees */
static void gather(const ora_ctx *o, const real *g, int x, int y, int z,
                   real *df) {
  int i;
  for (i = 0; i < o->q; i++) {
    int sx, sy, sz, xr = x - o->c[i][0];
    upstream(o, x, y, z, i, &sx, &sy, &sz);
    if (is_solid(o, sx, sy, sz))
      df[i] = wall_value(o, g, x, y, z, i, sy);
    else if (o->open && (xr < 0 || xr >= o->p.nx))
      df[i] = open_ghost(o, g, x, sy, sz, i, xr < 0 ? o->rho_in : o->rho_out);
    else
      df[i] = g[(long)i * o->ncell + cell(o, sx, sy, sz)];
  }
}

/* drho = sum df is the density deviation rho - rho0 itself; it is kept as
 * summed rather than recovered as (rho0 + drho) - rho0, which would round it
 * to the spacing of numbers near rho0 and undo the point of storing
 * deviations. */
static void moments(const ora_ctx *o, const real *df, real *drho, real *rho,
                    real u[3], real j[3]) {
  int i, a;
  *drho = 0;
  for (a = 0; a < 3; a++) j[a] = 0;
  for (i = 0; i < o->q; i++) {
    *drho += df[i];
    for (a = 0; a < 3; a++) j[a] += df[i] * (real)o->c[i][a];
  }
  for (a = 0; a < 3; a++) j[a] += (real)o->p.force[a] / 2;
  *rho = (real)o->p.rho0 + *drho;
  for (a = 0; a < 3; a++) u[a] = j[a] / *rho;
}

/* ------------------------------------------------ thermal fluctuations */

/* kT >= 0 (0 switches the noise off); mode 1 or 2 when kT > 0. */
int ora_set_thermal(ora_ctx *o, double kT, int mode, uint64_t seed) {
  if (!(kT >= 0) || isinf(kT)) return ORA_EINVAL;
  if (kT > 0 && mode != 1 && mode != 2) return ORA_EINVAL;
  o->kT = kT;
  o->noise = kT > 0 ? mode : 0;
  o->seed = seed;
  return ORA_OK;
}

/* One-point closure of the quantum fluctuations (Sec. 4, Eq. 18): the
 * two-point quantum correlator (Eq. 7), whose lag dependence Gamma_ab the
 * Keldysh analysis would supply, is averaged over spatial lags r and time
 * lags s with weights W_x(r), W_t(s) into a one-point tensor,
 *   m_ab = sum_r sum_s W_x(r) W_t(s) Gamma_ab(r, s),
 * which here scales the variance of each component of the random stress of
 * the stress-source noise (Eq. 17): P_ab -> sqrt(m_ab) P_ab.  gamma holds
 * Gamma for the six components xx, yy, zz, xy, xz, yz, each an nr x ns table
 * (component-major, then r, then s); a 2-D lattice ignores zz, xz, yz.  Every
 * m must come out finite and >= 0.  gamma == NULL restores the classical
 * noise (m = 1). */
int ora_set_noise_closure(ora_ctx *o, const double *gamma, int nr, int ns,
                          const double *wx, const double *wt) {
  real m[6];
  int c, r, t;
  if (!gamma) {
    for (c = 0; c < 6; c++) o->qfac[c] = 1;
    return ORA_OK;
  }
  if (nr < 1 || ns < 1 || !wx || !wt) return ORA_EINVAL;
  for (c = 0; c < 6; c++) {
    m[c] = 0;
    for (r = 0; r < nr; r++)
      for (t = 0; t < ns; t++)
        m[c] += (real)wx[r] * (real)wt[t] * (real)gamma[((long)c * nr + r) * ns + t];
    if (!(m[c] >= 0) || !R_ISFINITE(m[c])) return ORA_EINVAL;
  }
  for (c = 0; c < 6; c++) o->qfac[c] = R_SQRT(m[c]);
  return ORA_OK;
}

/* Philox4x64 with 10 rounds: each round multiplies words 0 and 2 by two
 * fixed odd constants, forms the new words from the high halves xor the
 * other words xor the round key and from the low halves, and the key grows by
 * two Weyl constants (golden ratio and sqrt(3) - 1, scaled to 64 bits)
 * between rounds. */
void ora_philox4x64(const uint64_t ctr[4], const uint64_t key[2],
                    uint64_t out[4]) {
  const uint64_t m0 = 0xD2E7470EE14C6C93ULL, m1 = 0xCA5A826395121157ULL;
  const uint64_t w0 = 0x9E3779B97F4A7C15ULL, w1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  int r;
  for (r = 0; r < 10; r++) {
    unsigned __int128 p0 = (unsigned __int128)m0 * x0;
    unsigned __int128 p1 = (unsigned __int128)m1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
    k0 += w0;
    k1 += w1;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* The first `count` standard normals of cell `cell` at step `step`.
 * Block b of the counter (cell, step, b, 0) gives four 64-bit words; word w
 * gives normals 8b + 2w and 8b + 2w + 1.  From the word's low and high 32-bit
 * halves take the top 23 bits each, u = (k + 1/2) / 2^23 (exact in binary32
 * as well, and never 0 or 1), and apply Box-Muller:
 *   z = sqrt(-2 ln u_low) cos(2 pi u_high),  z' = sqrt(-2 ln u_low) sin(2 pi u_high).
 * The largest |z| is sqrt(48 ln 2) = 5.77. */
void ora_thermal_normals(uint64_t seed, long cell, long step, int count,
                         double *z) {
  int k;
  uint64_t word[4] = {0, 0, 0, 0};
  for (k = 0; k < count; k++) {
    int b = k / 8, w = (k % 8) / 2;
    double ul, uh, rad, ang;
    if (k % 8 == 0) {
      uint64_t ctr[4], key[2];
      ctr[0] = (uint64_t)cell;
      ctr[1] = (uint64_t)step;
      ctr[2] = (uint64_t)b;
      ctr[3] = 0;
      key[0] = seed;
      key[1] = 0;
      ora_philox4x64(ctr, key, word);
    }
    ul = ((double)((uint32_t)word[w] >> 9) + 0.5) / 8388608.0;
    uh = ((double)((uint32_t)(word[w] >> 32) >> 9) + 0.5) / 8388608.0;
    rad = sqrt(-2.0 * log(ul));
    ang = 2.0 * 3.14159265358979323846 * uh;
    z[k] = k % 2 == 0 ? rad * cos(ang) : rad * sin(ang);
  }
}

/* Thermal term xi_i added to the post-collision population of cell n.
 *
 * Every non-conserved direction relaxes by the factor gamma = 1 - 1/tau per
 * step; a direction kept at variance mu (in the coordinates where the
 * equilibrium covariance is mu w_i delta_ij) needs added noise of variance
 * mu (1 - gamma^2): the fluctuation-dissipation balance of one linear
 * relaxation step.  mu = rho0 kT / c_s^2 gives <j_a^2> = rho0 kT, i.e.
 * equipartition.  A = sqrt(mu (1 - gamma^2)).
 *
 *  mode 1 (the paper's source, Eq. 17): xi_i = w_i / (2 c_s^4) P_ab
 *    (c_ia c_ib - c_s^2 delta_ab), P symmetric Gaussian with
 *    <P_ab P_cd> = A^2 c_s^4 (delta_ac delta_bd + delta_ad delta_bc):
 *    P_aa = sqrt(2) c_s^2 A z, P_ab = c_s^2 A z (a < b), one normal each in
 *    the order xx, yy, (zz,) xy, (xz, yz).
 *  mode 2 (stress and kinetic directions): v_i = sqrt(w_i) z_i for every i,
 *    then the mass and momentum parts are removed,
 *    xi_i = A (v_i - w_i sum_k v_k - 3 w_i c_i . sum_k v_k c_k). */
static void thermal_noise(const ora_ctx *o, long n, long step, real *xi) {
  const real cs2 = (real)1 / 3;
  real gam = 1 - 1 / (real)o->p.tau;
  real mu = (real)o->p.rho0 * (real)o->kT / cs2;
  real A = sqrt((double)(mu * (1 - gam * gam)));
  int d = o->q == 9 ? 2 : 3;
  int i, a, b;
  double z[19];
  if (o->noise == 1) {
    real P[3][3];
    int k = 0;
    ora_thermal_normals(o->seed, n, step, d * (d + 1) / 2, z);
    for (a = 0; a < 3; a++)
      for (b = 0; b < 3; b++) P[a][b] = 0;
    for (a = 0; a < d; a++) P[a][a] = sqrt(2.0) * cs2 * A * o->qfac[a] * (real)z[k++];
    for (a = 0; a < d; a++)
      for (b = a + 1; b < d; b++) {
        /* xy -> 3, xz -> 4, yz -> 5 */
        P[a][b] = cs2 * A * o->qfac[a == 0 ? 2 + b : 5] * (real)z[k++];
        P[b][a] = P[a][b];
      }
    for (i = 0; i < o->q; i++) {
      real s = 0;
      for (a = 0; a < 3; a++)
        for (b = 0; b < 3; b++)
          s += P[a][b] * ((real)(o->c[i][a] * o->c[i][b]) - (a == b ? cs2 : 0));
      xi[i] = o->w[i] / (2 * cs2 * cs2) * s;
    }
  } else {
    real v[19], sv = 0, sc[3] = {0, 0, 0};
    ora_thermal_normals(o->seed, n, step, o->q, z);
    for (i = 0; i < o->q; i++) {
      v[i] = sqrt((double)o->w[i]) * (real)z[i];
      sv += v[i];
      for (a = 0; a < 3; a++) sc[a] += v[i] * (real)o->c[i][a];
    }
    for (i = 0; i < o->q; i++) {
      real cdot = 0;
      for (a = 0; a < 3; a++) cdot += (real)o->c[i][a] * sc[a];
      xi[i] = A * (v[i] - o->w[i] * sv - 3 * o->w[i] * cdot);
    }
  }
}

/* ------------------------------------------------------ electron wind */

/* The solid's electrons as a second population set (Sec. 3.3, Sec. 4: one
 * set of distributions per species), coupled to the water by the
 * relative-velocity drag of Eq. 5 / Eq. 27 (F_kl = -F_lk): the bounce-back
 * half of the wall rule reflects off a wall moving with the electrons, and
 * the electrons take back exactly the axial momentum the water gains there.
 *
 * Every solid column next to the water on a SLAB or DUCT wall (the shells,
 * see shell_of) carries one electron line along x (the flow axis;
 * transverse transport in the sheet is not modelled), D1Q3 (c = 0, +1, -1,
 * w = 2/3, 1/6, 1/6), periodic in x; BGK with tau_e around rho_e0, Guo
 * forcing with F = force_e (the field drive) + F_wall - gamma_e rho u_e
 * (drag on the lattice, Eq. 13's F^{fr,eC}).  The interface rules of
 * Eqs. 22-24 keep the electrons in the solid: here they never leave their
 * line.  Requires wall_velocity_top == 0.  Off after creation. */
int ora_set_electrons(ora_ctx *o, double tau_e, double rho_e0, double gamma_e,
                      double force_e) {
  long n = nshell(o) * o->p.nx;
  if (o->p.geometry == ORA_MASKED || o->p.wall_velocity_top != 0.0 || o->open)
    return ORA_EINVAL;
  if (o->p.geometry == ORA_TUBE) {
    /* every wall link that crosses x must pull from a shell in the box */
    int y, z, i;
    for (z = 0; z < o->p.nz; z++)
      for (y = 0; y < o->p.ny; y++) {
        if (is_solid(o, 0, y, z)) continue;
        for (i = 0; i < o->q; i++)
          if (o->c[i][0] != 0 && is_solid(o, 0, y - o->c[i][1], z - o->c[i][2]) &&
              shell_of(o, y - o->c[i][1], z - o->c[i][2]) < 0)
            return ORA_EINVAL;
      }
  }
  if (!(tau_e > 0.5) || !(rho_e0 > 0) || !(gamma_e >= 0) || !isfinite(force_e) ||
      !isfinite(tau_e) || !isfinite(rho_e0) || !isfinite(gamma_e))
    return ORA_EINVAL;
  if (!o->e) {
    o->e = (real *)calloc(3 * n, sizeof(real));
    o->en = (real *)calloc(3 * n, sizeof(real));
    o->ue = (real *)calloc(n, sizeof(real));
    if (!o->e || !o->en || !o->ue) return ORA_ENOMEM;
  }
  memset(o->e, 0, 3 * n * sizeof(real));
  memset(o->ue, 0, n * sizeof(real));
  o->elec = 1;
  o->phon = 0; /* switching the electrons on resets them without phonons */
  o->tau_e = tau_e;
  o->rho_e0 = rho_e0;
  o->gamma_e = gamma_e;
  o->force_e = force_e;
  return ORA_OK;
}

/* One electron step from the water state g (both at step n).  Per shell
 * node s, the water links that leave s and land on a fluid node x_f = s + c_k
 * with c_kx != 0 carry the axial exchange (one fluid column per shell, two
 * directions): the water at x_f gains
 *   r(x_f) (2 g_opp(k)(x_f) + 6 w_k rho0 c_kx u_e(s)) c_kx
 * (its wall rule; the free-slip half exchanges no axial momentum), so
 *   F_wall(s) = F0 - K u_e,  F0 = -sum 2 r g_opp(k) c_kx,  K = 6 rho0 sum r w_k.
 * With the drag and Guo's half-force the velocity solves
 *   rho u = j + (force_e + F0 - K u - gamma rho u) / 2. */
static void electron_step(ora_ctx *o) {
  const int cd[3] = {0, 1, -1};
  const real wd[3] = {(real)2 / 3, (real)1 / 6, (real)1 / 6};
  int x, i, k, ys, zs;
  long sh;
  real tau = (real)o->tau_e, gam = (real)o->gamma_e;
  long n = nshell(o) * o->p.nx;
  for (sh = 0; sh < nshell(o); sh++) {
    shell_column(o, sh, &ys, &zs);
    for (x = 0; x < o->p.nx; x++) {
      long s = sh * o->p.nx + x;
      real de[3], drho = 0, j = 0, rho, u, F0 = 0, K = 0, F;
      for (i = 0; i < 3; i++) {
        int xs = ((x - cd[i]) % o->p.nx + o->p.nx) % o->p.nx;
        de[i] = o->e[(long)i * n + sh * o->p.nx + xs];
        drho += de[i];
        j += de[i] * (real)cd[i];
      }
      rho = (real)o->rho_e0 + drho;
      for (k = 0; k < o->q; k++) {
        long cf;
        int xf, yf = ys + o->c[k][1], zf = zs + o->c[k][2];
        real gob, term, mw = 1;
        if (o->c[k][0] == 0) continue;
        if (o->p.geometry == ORA_SLAB) zf = (zf % o->p.nz + o->p.nz) % o->p.nz;
        if (yf < 0 || yf >= o->p.ny || zf < 0 || zf >= o->p.nz) continue;
        xf = ((x + o->c[k][0]) % o->p.nx + o->p.nx) % o->p.nx;
        cf = cell(o, xf, yf, zf);
        if (!o->fluid[cf]) continue;
        /* the axial momentum the water at cf gains through its wall link k
         * (pulling from this shell node): r c_kx (bb_k + g_opp(k)) summed
         * over the node's links (the slip half cancels within the node, the
         * transverse reversal pairing each wall link with an into-wall one
         * of the same c_x); bb_k's moving-wall part is mw 6 w_k rho0 c_kx u */
        gob = o->g[(long)o->opp[k] * o->ncell + cf];
        term = 2 * gob;
        if (o->p.geometry == ORA_TUBE) {
          real qv = o->qlink[cf * 19 + k];
          if (qv < (real)0.5) {
            int xb = ((xf + o->c[k][0]) % o->p.nx + o->p.nx) % o->p.nx;
            int yb = yf + o->c[k][1], zb = zf + o->c[k][2];
            if (!is_solid(o, xb, yb, zb))
              term += (1 - 2 * qv) * (o->g[(long)o->opp[k] * o->ncell + cell(o, xb, yb, zb)] - gob);
          } else {
            term += (2 * qv - 1) / (2 * qv) * (o->g[(long)k * o->ncell + cf] - gob);
            mw = 1 / (2 * qv);
          }
        }
        F0 -= o->r[cf] * term * (real)o->c[k][0];
        K += 6 * (real)o->p.rho0 * o->r[cf] * o->w[k] * mw;
      }
      if (!o->phon) {
        u = (j + ((real)o->force_e + F0) / 2) / (rho * (1 + gam / 2) + K / 2);
        F = (real)o->force_e + F0 - K * u - gam * rho * u;
      } else {
        /* phonons: the electron-phonon drag -G (u - u_p) on the electrons and
         * +G (u - u_p) on the phonons (Sec. 3.4; equal and opposite, Eq. 27),
         * G = gamma_ep rho, and the crystal drag -gamma_pc rho_p u_p on the
         * phonons; with Guo's half-forces both velocities solve
         *   rho u     = j   + (force_e + F0 - K u - gam rho u - G (u - u_p)) / 2
         *   rho_p u_p = j_p + (-gamma_pc rho_p u_p + G (u - u_p)) / 2 */
        const real taup = (real)o->tau_p, gp = (real)o->gamma_pc;
        real dp[3], drp = 0, jp = 0, rp, G, a11, a22, b1, det, Fp, upv;
        for (i = 0; i < 3; i++) {
          int xs = ((x - cd[i]) % o->p.nx + o->p.nx) % o->p.nx;
          dp[i] = o->ph[(long)i * n + sh * o->p.nx + xs];
          drp += dp[i];
          jp += dp[i] * (real)cd[i];
        }
        rp = (real)o->rho_p0 + drp;
        G = (real)o->gamma_ep * rho;
        a11 = rho * (1 + gam / 2) + K / 2 + G / 2;
        a22 = rp * (1 + gp / 2) + G / 2;
        b1 = j + ((real)o->force_e + F0) / 2;
        det = a11 * a22 - G * G / 4;
        u = (b1 * a22 + G / 2 * jp) / det;
        upv = (a11 * jp + G / 2 * b1) / det;
        F = (real)o->force_e + F0 - K * u - gam * rho * u - G * (u - upv);
        Fp = -gp * rp * upv + G * (u - upv);
        for (i = 0; i < 3; i++) {
          real c = (real)cd[i];
          real eq = wd[i] * (drp + rp * (3 * c * upv + (real)4.5 * c * c * upv * upv -
                                        (real)1.5 * upv * upv));
          real src = (1 - 1 / (2 * taup)) * wd[i] * (3 * (c - upv) + 9 * c * upv * c) * Fp;
          o->phn[(long)i * n + s] = dp[i] - (dp[i] - eq) / taup + src;
        }
        o->up[s] = upv;
      }
      for (i = 0; i < 3; i++) {
        real c = (real)cd[i];
        real eq = wd[i] * (drho + rho * (3 * c * u + (real)4.5 * c * c * u * u -
                                         (real)1.5 * u * u));
        real src = (1 - 1 / (2 * tau)) * wd[i] * (3 * (c - u) + 9 * c * u * c) * F;
        o->en[(long)i * n + s] = de[i] - (de[i] - eq) / tau + src;
      }
      o->ue[s] = u;
    }
  }
  {
    real *t = o->e;
    o->e = o->en;
    o->en = t;
  }
  if (o->phon) {
    real *t = o->ph;
    o->ph = o->phn;
    o->phn = t;
  }
}

/* Phonon lines (Sec. 3.4): a third population set, one D1Q3 line beside
 * every electron line, BGK with tau_p around rho_p0, driven only by the
 * electron-phonon drag of Sec. 3.4 (equal and opposite on the two, Eq. 27;
 * coefficient gamma_ep rho_e) and damped by the crystal, -gamma_pc rho_p u_p;
 * they do not touch the water.  Requires the electron lines on; resets the
 * phonons to rest; tau_p == 0 switches them off. */
int ora_set_phonons(ora_ctx *o, double tau_p, double rho_p0, double gamma_pc, double gamma_ep) {
  long n = nshell(o) * o->p.nx;
  if (tau_p == 0) {
    o->phon = 0;
    return ORA_OK;
  }
  if (!o->elec || !(tau_p > 0.5) || !(rho_p0 > 0) || !(gamma_pc >= 0) || !(gamma_ep >= 0) ||
      !isfinite(tau_p) || !isfinite(rho_p0) || !isfinite(gamma_pc) || !isfinite(gamma_ep))
    return ORA_EINVAL;
  if (!o->ph) {
    o->ph = (real *)calloc(3 * n, sizeof(real));
    o->phn = (real *)calloc(3 * n, sizeof(real));
    o->up = (real *)calloc(n, sizeof(real));
    if (!o->ph || !o->phn || !o->up) return ORA_ENOMEM;
  }
  memset(o->ph, 0, 3 * n * sizeof(real));
  memset(o->up, 0, n * sizeof(real));
  o->phon = 1;
  o->tau_p = tau_p;
  o->rho_p0 = rho_p0;
  o->gamma_pc = gamma_pc;
  o->gamma_ep = gamma_ep;
  return ORA_OK;
}

/* phonon velocity of the last step [shell][x] and populations [i][shell][x] */
void ora_get_phonons(const ora_ctx *o, double *up, double *pops) {
  long k, n = nshell(o) * o->p.nx;
  if (!o->phon) return;
  for (k = 0; k < n; k++)
    if (up) up[k] = (double)o->up[k];
  if (pops)
    for (k = 0; k < 3 * n; k++) pops[k] = (double)o->ph[k];
}

/* electron velocity of the last step [shell][x] and the shifted populations
 * [i][shell][x] of the current state (either may be NULL) */
long ora_shell_count(const ora_ctx *o) { return nshell(o); }

/* Replace the electron populations (shifted, [i][shell][x], 3 nshell nx
 * values) of a context whose electron lines are on. */
int ora_set_electron_populations(ora_ctx *o, const double *pops) {
  long k, n = nshell(o) * o->p.nx;
  if (!o->elec || !pops) return ORA_EINVAL;
  for (k = 0; k < 3 * n; k++) o->e[k] = (real)pops[k];
  return ORA_OK;
}

void ora_get_electrons(const ora_ctx *o, double *ue, double *pops) {
  long k, n = nshell(o) * o->p.nx;
  if (!o->e) return;
  for (k = 0; k < n; k++) {
    if (ue) ue[k] = (double)o->ue[k];
  }
  if (pops)
    for (k = 0; k < 3 * n; k++) pops[k] = (double)o->e[k];
}

void ora_step(ora_ctx *o, long nsteps) {
  long s;
  int x, y, z, i, a;
  real tau = (real)o->p.tau;
  real F[3];
  for (a = 0; a < 3; a++) F[a] = (real)o->p.force[a];
  for (s = 0; s < nsteps; s++) {
    if (o->elec) electron_step(o); /* reads g at step n, sets u_e of step n */
    for (z = 0; z < o->p.nz; z++)
      for (y = 0; y < o->p.ny; y++)
        for (x = 0; x < o->p.nx; x++) {
          long n = cell(o, x, y, z);
          real df[19], drho, rho, u[3], j[3], usq, uF, xi[19];
          if (!o->fluid[n]) continue;
          for (i = 0; i < o->q; i++) xi[i] = 0;
          if (o->noise) thermal_noise(o, n, o->step, xi);
          gather(o, o->g, x, y, z, df);
          moments(o, df, &drho, &rho, u, j);
          usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
          uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
          for (i = 0; i < o->q; i++) {
            real cu = 0, cF = 0, feq, src;
            for (a = 0; a < 3; a++) {
              cu += (real)o->c[i][a] * u[a];
              cF += (real)o->c[i][a] * F[a];
            }
            feq = o->w[i] *
                  (drho + rho * (3 * cu + (real)4.5 * cu * cu -
                                         (real)1.5 * usq));
            src = (1 - 1 / (2 * tau)) * o->w[i] * (3 * (cF - uF) + 9 * cu * cF);
            o->gn[(long)i * o->ncell + n] =
                df[i] - (df[i] - feq) / tau + src + xi[i];
          }
        }
    {
      real *t = o->g;
      o->g = o->gn;
      o->gn = t;
    }
    o->step++;
  }
}

/* Fields after the current step: rho, ux, uy, uz per cell (dense box, zero
 * on solid cells).  Any pointer may be NULL. */
void ora_fields(const ora_ctx *o, double *rho, double *ux, double *uy,
                double *uz) {
  int x, y, z;
  for (z = 0; z < o->p.nz; z++)
    for (y = 0; y < o->p.ny; y++)
      for (x = 0; x < o->p.nx; x++) {
        long n = cell(o, x, y, z);
        real df[19], dr, r, u[3], j[3];
        if (!o->fluid[n]) {
          if (rho) rho[n] = 0;
          if (ux) ux[n] = 0;
          if (uy) uy[n] = 0;
          if (uz) uz[n] = 0;
          continue;
        }
        gather(o, o->g, x, y, z, df);
        moments(o, df, &dr, &r, u, j);
        if (rho) rho[n] = (double)r;
        if (ux) ux[n] = (double)u[0];
        if (uy) uy[n] = (double)u[1];
        if (uz) uz[n] = (double)u[2];
      }
}

/* out[0] = flux Q = (1/nx) sum_fluid rho u_x ; out[1] = mass M = sum rho ;
 * out[2] = sum (rho - rho0), the mass deviation, summed on its own so that
 * drift is visible below the rounding of M itself. */
void ora_invariants(const ora_ctx *o, double *out) {
  int x, y, z;
  real q = 0, dm = 0;
  for (z = 0; z < o->p.nz; z++)
    for (y = 0; y < o->p.ny; y++)
      for (x = 0; x < o->p.nx; x++) {
        long n = cell(o, x, y, z);
        real df[19], dr, r, u[3], j[3];
        if (!o->fluid[n]) continue;
        gather(o, o->g, x, y, z, df);
        moments(o, df, &dr, &r, u, j);
        q += j[0];
        dm += dr;
      }
  out[0] = (double)(q / (real)o->p.nx);
  out[1] = (double)((real)o->nfluid * (real)o->p.rho0 + dm);
  out[2] = (double)dm;
}

/* populations g_i (shifted, post-collision) of the current state, dense box,
 * layout [i][z][y][x] in double */
void ora_get_populations(const ora_ctx *o, double *out) {
  long k, n = o->ncell * o->q;
  for (k = 0; k < n; k++) out[k] = (double)o->g[k];
}

void ora_set_populations(ora_ctx *o, const double *in, long step) {
  long k, n = o->ncell * o->q;
  for (k = 0; k < n; k++) o->g[k] = (real)in[k];
  o->step = step;
}

/* ------------------------------------------------- friction quadrature */

/* Spectral parameters (units hbar = k_B = 1, lengths in units of the gap) */
typedef struct {
  double T, omega0, gamma_s, omega_l, gamma_l, a_l, d;
  int nq, nw;
  double q_max, w_max;
  double lambda_target;
  int dispersion; /* 1: omega_p^2 = Omega^2 q d ; 0: omega_p^2 = Omega^2 */
  int coupling;   /* 1: divide by |1 - g_s g_l e^{-2qd}|^2 ; 0: leave it out */
  double v_l;     /* liquid mode: omega_l(q)^2 = omega_l^2 + v_l^2 q^2 */
} ora_spectral;

/* imaginary part of the Lorentzian liquid response at frequency w (q = 0) */
double ora_img_l(const ora_spectral *s, double w) {
  real wl2 = (real)s->omega_l * (real)s->omega_l, ww = (real)w;
  real den = (wl2 - ww * ww) * (wl2 - ww * ww) +
             (real)s->gamma_l * (real)s->gamma_l * ww * ww;
  return (double)((real)s->a_l * wl2 * (real)s->gamma_l * ww / den);
}

/* imaginary part of the Drude-like solid response with plasmon frequency
 * omega_p(q)^2 = Omega^2 q d (2-D plasmon dispersion) at wavevector q */
double ora_img_s(const ora_spectral *s, double Omega, double q, double w) {
  real wp2 = (real)Omega * (real)Omega *
             (s->dispersion ? (real)q * (real)s->d : (real)1);
  real ww = (real)w;
  real den = (wp2 - ww * ww) * (wp2 - ww * ww) +
             (real)s->gamma_s * (real)s->gamma_s * ww * ww;
  return (double)(wp2 * (real)s->gamma_s * ww / den);
}

/* The complex surface responses at (q, w), each a damped oscillator
 * A W / (W - w^2 - i gamma w):
 *   solid  g_s: A = 1,   W = omega_p(q)^2 (as in ora_img_s), gamma_s;
 *   liquid g_l: A = a_l, W = omega_l^2 + v_l^2 q^2, gamma_l.
 * out = (Re g_s, Im g_s, Re g_l, Im g_l). */
static void responses(const ora_spectral *s, real Omega, real q, real w,
                      real out[4]) {
  real Ws = Omega * Omega * (s->dispersion ? q * (real)s->d : (real)1);
  real Wl = (real)s->omega_l * (real)s->omega_l +
            (real)s->v_l * (real)s->v_l * q * q;
  real ds = Ws - w * w, es = (real)s->gamma_s * w;
  real dl = Wl - w * w, el = (real)s->gamma_l * w;
  real ns = Ws / (ds * ds + es * es);
  real nl = (real)s->a_l * Wl / (dl * dl + el * el);
  /* A W / (d - i e) = A W (d + i e) / (d^2 + e^2) */
  out[0] = ns * ds;
  out[1] = ns * es;
  out[2] = nl * dl;
  out[3] = nl * el;
}

void ora_response(const ora_spectral *s, double Omega, double q, double w,
                  double *out) {
  real r[4];
  int k;
  responses(s, (real)Omega, (real)q, (real)w, r);
  for (k = 0; k < 4; k++) out[k] = (double)r[k];
}

/* raw friction sum for one plasmon frequency Omega:
 *   C sum_a sum_b dq dw q^3 e^{-2 q d} Im g_s Im g_l
 *       / (sinh^2(w / 2T) |1 - g_s g_l e^{-2 q d}|^2),
 *   C = 1 / (8 pi^2 T), midpoint grids on (0, q_max) and (0, w_max).
 * The denominator (the two surfaces' repeated mutual screening) is 1 when
 * coupling = 0; with v_l = 0 the liquid response does not depend on q. */
double ora_friction_raw(const ora_spectral *s, double Omega) {
  real pi = (real)3.14159265358979323846264338327950288L;
  real C = 1 / (8 * pi * pi * (real)s->T);
  real dq = (real)s->q_max / s->nq, dw = (real)s->w_max / s->nw;
  real sum = 0;
  int a, b;
  for (a = 0; a < s->nq; a++) {
    real q = ((real)a + (real)0.5) * dq;
    real e = R_EXP(-2 * q * (real)s->d);
    real kq = q * q * q * e;
    for (b = 0; b < s->nw; b++) {
      real w = ((real)b + (real)0.5) * dw;
      real sh = R_SINH(w / (2 * (real)s->T));
      real g[4], den = 1;
      responses(s, (real)Omega, q, w, g);
      if (s->coupling) {
        /* z = e g_s g_l ; |1 - z|^2 */
        real zr = e * (g[0] * g[2] - g[1] * g[3]);
        real zi = e * (g[0] * g[3] + g[1] * g[2]);
        den = (1 - zr) * (1 - zr) + zi * zi;
      }
      sum += dq * dw * kq * g[1] * g[3] / (sh * sh * den);
    }
  }
  return (double)(C * sum);
}

/* per wall node: raw[k] (may be NULL) and lattice friction
 *   lambda_k = lambda_target * raw(Omega_k) / raw(omega0) */
void ora_friction(const ora_spectral *s, const double *Omega, long n,
                  double *raw, double *lambda_lat) {
  double ref = ora_friction_raw(s, s->omega0);
  long k;
  for (k = 0; k < n; k++) {
    double v = ora_friction_raw(s, Omega[k]);
    if (raw) raw[k] = v;
    if (lambda_lat) lambda_lat[k] = (double)((real)s->lambda_target * (real)v / (real)ref);
  }
}

int ora_sizeof_real(void) { return (int)sizeof(real); }

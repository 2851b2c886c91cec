// lbm_kernels.hip -- HIP kernels for gfx950 (MI355X) and their launchers.
//
//  k_step           fused pull stream + Navier-slip wall + BGK/Guo collide,
//                   one thread per fluid cell, ping-pong buffers; TH = 1, 2
//                   adds thermal noise of that form (fluctuating LB)
//  k_moments        moments of the current state (the populations the next
//                   collision sees), per-block FP64 partials of the flux and
//                   the mass deviation, optional dense field output
//  k_reduce_final   fixed-order FP64 sum of the per-block partials
//  k_friction_raw   (q, omega) friction quadrature, omega table tiled
//                   through LDS, FP64 sums, wavefront + block reduction
//  k_friction_full  the same with the screening denominator |1 - g_s g_l e^{-2qd}|^2
//                   and a dispersive liquid mode (complex responses)
//  k_friction_lat   normalisation lambda_k = lambda_target raw_k / raw_ref
//  k_set_r          lambda -> wall mixing weight r = 3 lambda / (1 + 3 lambda)
//  k_copy           plain 16-byte streaming copy (measured bandwidth ceiling)
//  k_set_step, k_add_step   device-resident step base read by graph-launched steps
//  k_batch_step     k_step over the work list of a group of channels of a
//                   batch, one 64-lane item per wave
//  k_batch_moments, k_batch_reduce   per-member flux and mass of a batch
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "lbm_device.h"
#include "lbm_launch.h"

namespace lbm {

// ------------------------------------------------------------ stream-collide
// One lane's cell of the step kernel (x < nxp).  With CHECK the lane also
// returns, in FP64, j_x (with the half-force) and rho - rho0 of the
// populations its collision sees, as k_moments forms them (0 on padding
// lanes).
template <class L, typename S, typename M, bool BOUZ, int TH, bool ELEC, bool OPEN, bool CHECK,
          bool NT = false>
__device__ __forceinline__ void step_cell(const S* __restrict__ src, S* __restrict__ dst,
                                          const StepArgs& a, int slot, int x, double* jx_c,
                                          double* dr_c) {
  // Lanes on the padding of an x-line (nx <= x < nxp) recompute cell nx - 1
  // and store it into the padding, so every cache line of the output is
  // written whole (a partly written line costs HBM a read-modify-write).
  // Nothing reads the padding.
  const int xc = x < a.nx ? x : a.nx - 1;
  const LBM_GLOBAL ColSlot& cs = gbl(a.slots)[slot];
  const int col = uniform(cs.col);
  ColInfo info;
  info.wallcol = uniform(cs.wallcol);
  info.mask = (uint32_t)uniform((int)cs.mask);
  const int64_t step = (a.dstep ? uniform64(*gbl(a.dstep)) : 0) + a.step_off;
  M df[L::Q];
  // the thermal term depends only on (cell, step): drawn before the gather,
  // it holds fewer registers than while the gathered values are live
  M xi[L::Q];
  if constexpr (TH != 0)
    thermal_noise<L, M, TH, NormalT<S>>(a, (uint32_t)col * (uint32_t)a.nx + (uint32_t)x, step, xi);
  gather<L, S, M, M, BOUZ, ELEC, OPEN>(src, a, col, xc, info, df);
  if constexpr (OPEN) open_correct<L, M, BOUZ>(a, a.bmom, col, xc, info, df);
  if constexpr (CHECK) {
    if (x < a.nx) {
      double dr = 0, jx = 0;
#pragma unroll
      for (int i = 0; i < L::Q; i++) {
        dr += static_cast<double>(df[i]);
        jx += L::cx[i] * static_cast<double>(df[i]);
      }
      *jx_c = jx + a.F[0] / 2;
      *dr_c = dr;
    }
  }
  M rec[4];
  collide_store<L, M, S, TH, OPEN, NT>(df, a, gbl(dst) + (int64_t)col * a.sC, (unsigned)x,
                                       (uint32_t)col * (uint32_t)a.nx + (uint32_t)x, step, xi,
                                       rec);
  // open ends: the end nodes leave the record of what they stored (the same
  // sums end_record forms) for the ghosts of the next step
  if constexpr (OPEN)
    if (x == xc && (x == 0 || x == a.nx - 1)) {
      LBM_GLOBAL double* o =
          gbl(a.bmom_out) + ((x == 0 ? 0 : (int64_t)a.ny * a.nz) + col) * 4;
      const M rho = static_cast<M>(a.rho0) + rec[0];
      o[0] = static_cast<double>(rec[0]);
      o[1] = static_cast<double>(rec[1] / rho);
      o[2] = static_cast<double>(rec[2] / rho);
      o[3] = static_cast<double>(rec[3] / rho);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Per-block partial sums (s0, s1) over a block of the step or moments grid:
// a fixed butterfly within each wave, then the waves in order (deterministic).
__device__ __forceinline__ void block_partials(double s0, double s1, double* __restrict__ out) {
  __shared__ double red[2][8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (lane == 0) {
    red[0][wv] = s0;
    red[1][wv] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double t0 = 0, t1 = 0;
    for (int k = 0; k < nw; k++) {
      t0 += red[0][k];
      t1 += red[1][k];
    }
    out[0] = t0;
    out[1] = t1;
  }
}

template <class L, typename S, typename M, bool BOUZ, int TH, bool ELEC, bool OPEN,
          bool CHECK = false, bool NT = false>
__device__ __forceinline__ void step_cells(const S* __restrict__ src, S* __restrict__ dst,
                                           const StepArgs& a) {
  // grid (fluid columns, segments per x-line).  Wall columns go first (their
  // blocks do more work and would otherwise form the tail of the grid).  The
  // rest are visited in one order when reading one buffer and in the reverse
  // order when reading the other: a step then starts on the columns the
  // previous step wrote last, which are still in the last-level cache.
  int slot = blockIdx.x;
  if (a.rev && slot >= a.nwallcols) slot = a.nactive - 1 - slot + a.nwallcols;
  const int x = blockIdx.y * a.bx + threadIdx.x;
  if constexpr (CHECK) {
    // a checked step (the last of a chunk) also sums the flux and mass
    // deviation of the populations its collision sees -- the invariants of
    // the state before the step -- per block, indexed like k_moments' blocks
    // (slot, segment), so the two agree bit for bit where the arithmetic is
    // double
    double jx_c = 0.0, dr_c = 0.0;
    if (x < a.nxp)
      step_cell<L, S, M, BOUZ, TH, ELEC, OPEN, true>(src, dst, a, slot, x, &jx_c, &dr_c);
    block_partials(jx_c, dr_c, a.partials + 2 * ((int64_t)slot * a.segs + blockIdx.y));
    return;
  }
  if (x >= a.nxp) return;
  step_cell<L, S, M, BOUZ, TH, ELEC, OPEN, false, NT>(src, dst, a, slot, x, nullptr, nullptr);
}

template <class L, typename S, typename M, bool BOUZ, int TH, bool ELEC = false,
          bool CHECK = false, bool NT = false>
__global__ void __launch_bounds__(512) k_step(const S* __restrict__ src, S* __restrict__ dst,
                                              StepArgs a) {
  step_cells<L, S, M, BOUZ, TH, ELEC, false, CHECK, NT>(src, dst, a);
}

// Open x ends: the same update with the ghost pulls at both ends of every
// x-line (the end-node records hold a few more registers: four waves per
// SIMD instead of five; asking for five makes the compiler spill).  BOUZ:
// tubes, whose interpolated wall links at the ends also read ghosts.
template <class L, typename S, typename M, bool BOUZ, int TH>
__global__ void __launch_bounds__(512) k_step_open(const S* __restrict__ src,
                                                      S* __restrict__ dst, StepArgs a) {
  step_cells<L, S, M, BOUZ, TH, false, true>(src, dst, a);
}

// Masked walls: the same update on every fluid point of the columns that
// hold one.  Columns with wall nodes come first (slot mask != 0); their
// lanes take the row's non-solid points from a packed list (solid points
// are neither computed nor stored: nothing reads them), and the class of
// each point (interior or wall node) comes from a table of the (x, y)
// plane, so a wave may hold both.  The other columns are wholly interior
// and only pull.  Their order alternates as in k_step.  OPEN: open x
// ends (the mask's first and last rows are equal, so the wall links are
// those of the periodic channel): the ghost pulls and the end-node records as
// in the open step kernel.
template <class L, typename S, typename M, int TH, bool OPEN = false>
__global__ void __launch_bounds__(512) k_step_masked(const S* __restrict__ src,
                                                     S* __restrict__ dst, StepArgs a) {
  int slot = blockIdx.x;
  if (a.rev && slot >= a.nwallcols) slot = a.nactive - 1 - slot + a.nwallcols;
  const LBM_GLOBAL ColSlot& cs = gbl(a.slots)[slot];
  const int col = uniform(cs.col);
  const bool wallcol = uniform((int)cs.mask) != 0;
  const int z = col / a.ny;
  const int y = col - z * a.ny;
  // a column of a wall row takes its points from the row's packed list, so
  // that its solid points hold no lanes (whole waves past the list leave)
  int x = blockIdx.y * a.bx + threadIdx.x;
  if (wallcol) {
    const LBM_GLOBAL int32_t* rx = gbl(a.rowx) + (int64_t)y * (a.nxp + 1);
    if (x >= uniform(rx[0])) return;
    x = rx[1 + x];
  } else if (x >= a.nxp) {
    return;
  }
  const int xc = x < a.nx ? x : a.nx - 1;  // padding lanes: cell nx - 1 again
  const int cw = wallcol ? gbl(a.cellw)[xc + (int64_t)a.nx * y] : kCellInterior;
  if (cw == kCellSolid) return;
  const int64_t step = (a.dstep ? uniform64(*gbl(a.dstep)) : 0) + a.step_off;
  M df[L::Q];
  M xi[L::Q];
  if constexpr (TH != 0)
    thermal_noise<L, M, TH, NormalT<S>>(a, (uint32_t)col * (uint32_t)a.nx + (uint32_t)x, step, xi);
  uint32_t wl = 0u;
  if (wallcol)
    gather_masked<L, S, M, M, OPEN>(src, a, col, z, xc, cw, df, &wl);
  else
    gather_masked_interior<L, S, M, OPEN>(src, a, col, z, xc, df);
  if constexpr (OPEN) {
    ColInfo info;
    info.wallcol = 0;
    info.mask = wl;
    open_correct<L, M>(a, a.bmom, col, xc, info, df);
  }
  M rec[4];
  collide_store<L, M, S, TH, OPEN>(df, a, gbl(dst) + (int64_t)col * a.sC, (unsigned)x,
                                   (uint32_t)col * (uint32_t)a.nx + (uint32_t)x, step, xi, rec);
  if constexpr (OPEN)
    if (x == xc && (x == 0 || x == a.nx - 1)) {
      LBM_GLOBAL double* o =
          gbl(a.bmom_out) + ((x == 0 ? 0 : (int64_t)a.ny * a.nz) + col) * 4;
      const M rho = static_cast<M>(a.rho0) + rec[0];
      o[0] = static_cast<double>(rec[0]);
      o[1] = static_cast<double>(rec[1] / rho);
      o[2] = static_cast<double>(rec[2] / rho);
      o[3] = static_cast<double>(rec[3] / rho);
    }
}

// Open x ends: the records (sum g, u) of the first and last node of every
// fluid column of src ([side][column][4]) where no step has left them (after
// the state was set from outside).  One lane per (column, side).
template <class L, typename S, typename M>
__global__ void __launch_bounds__(256) k_open_moments(const S* __restrict__ src, StepArgs a,
                                                      double* __restrict__ bmom) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * (int64_t)a.nactive) return;
  const int side = (int)(t & 1);
  const int col = gbl(a.slots)[t >> 1].col;
  const unsigned x = side ? (unsigned)a.nx - 1u : 0u;
  end_record<L, S, M>(gbl(src) + (int64_t)col * a.sC, a, x,
                      gbl(bmom) + ((int64_t)side * a.ny * a.nz + col) * 4);
}

// ------------------------------------------------------------ electron sheets
// One electron step per shell node (lines along x, D1Q3: c = 0, +1, -1,
// w = 2/3, 1/6, 1/6, shifted populations [i][shell][x] in double):
//   pull along the line (periodic); the water links from this node to the
//   fluid column next to it (c_kx != 0) give the axial force the
//   water's wall rule takes from the sheet, F_wall = F0 - K u,
//     F0 = -sum 2 r g_opp(k)(x + c_kx) c_kx,  K = 6 rho0 sum r w_k;
//   with the field force and the drag -gamma rho u, Guo's half-force makes
//     rho u = j + (force + F0 - K u - gamma rho u) / 2
//   linear in u; then BGK + Guo with F = force + F0 - K u - gamma rho u.
template <class L, typename S, typename W>
__device__ __forceinline__ void electron_node(const S* __restrict__ g,
                                              const double* __restrict__ es,
                                              double* __restrict__ ed, double* __restrict__ ue,
                                              const ElecArgs& ea, int64_t s) {
  const int64_t n = (int64_t)ea.nshell * ea.nx;
  const int64_t sh = s / ea.nx;  // shell
  const int x = (int)(s - sh * ea.nx);
  const int64_t line = sh * ea.nx;
  const int xm = x == 0 ? ea.nx - 1 : x - 1, xp = x == ea.nx - 1 ? 0 : x + 1;
  const double d0 = es[s], d1 = es[n + line + xm], d2 = es[2 * n + line + xp];
  const double drho = d0 + d1 + d2, j = d1 - d2;
  const double rho = ea.rho_e0 + drho;
  double F0 = 0.0, K = 0.0;
  if (ea.tube) {
    // a tube: up to four fluid columns next to the shell (at -y, +y, -z,
    // +z); through each link k from the shell into one of them the water
    // gains r c_kx (bb_k + g_opp(k)) of axial momentum, bb_k the interpolated
    // bounce-back (coefficients cb on the node behind, cc on g_k) whose
    // moving-wall part is (1 - cc) 6 w_k rho0 c_kx u
    const LBM_GLOBAL int32_t* ts = gbl(ea.swc) + sh * 8;
    const LBM_GLOBAL W* rwall = gbl(static_cast<const W*>(ea.rwall));
    const LBM_GLOBAL W* bz = gbl(static_cast<const W*>(ea.bz));
    const LBM_GLOBAL S* gg = gbl(g);
#pragma unroll
    for (int d = 0; d < 4; d++) {
      const int fc = ts[2 * d], wc = ts[2 * d + 1];
      if (fc < 0) continue;
      const int dy = d == 0 ? -1 : (d == 1 ? 1 : 0), dz = d == 2 ? -1 : (d == 3 ? 1 : 0);
#pragma unroll
      for (int k = 0; k < L::Q; k++) {
        if (L::cx[k] == 0 || L::cy[k] != dy || L::cz[k] != dz) continue;
        const int xf = L::cx[k] > 0 ? xp : xm;
        const double r = static_cast<double>(rwall[(int64_t)wc * ea.nx + xf]);
        const double gob =
            dec<S, double>(gg[(int64_t)fc * ea.sC + L::row[L::opp[k]] * ea.sI + xf]);
        const double cbz = static_cast<double>(bz[((int64_t)wc * L::Q + k) * 2]);
        const double ccz = static_cast<double>(bz[((int64_t)wc * L::Q + k) * 2 + 1]);
        double term = 2.0 * gob;
        if (cbz != 0.0) {  // the node behind, x_f + c_k, in the column beyond
          const int xb = L::cx[k] > 0 ? (xf == ea.nx - 1 ? 0 : xf + 1)
                                      : (xf == 0 ? ea.nx - 1 : xf - 1);
          const int64_t cbk = (int64_t)fc + dy + (int64_t)ea.ny * dz;
          term += cbz * (dec<S, double>(gg[cbk * ea.sC + L::row[L::opp[k]] * ea.sI + xb]) - gob);
        }
        if (ccz != 0.0)
          term += ccz * (dec<S, double>(gg[(int64_t)fc * ea.sC + L::row[k] * ea.sI + xf]) - gob);
        F0 -= r * term * L::cx[k];
        K += 6.0 * ea.rho0 * r * L::w[k] * (1.0 - ccz);
      }
    }
  } else {
    // the fluid column next to the shell and the (c_y, c_z) of the links to it
    int cy, cz;
    int64_t col;
    if (sh < 2LL * ea.nz) {
      const bool low = sh < ea.nz;
      cy = low ? 1 : -1;
      cz = 0;
      col = (low ? 0 : ea.ny - 1) + (int64_t)ea.ny * (sh % ea.nz);
    } else {
      const int64_t t = sh - 2LL * ea.nz;
      const bool low = t < ea.ny;
      cy = 0;
      cz = low ? 1 : -1;
      col = t % ea.ny + (int64_t)ea.ny * (low ? 0 : ea.nz - 1);
    }
    const LBM_GLOBAL W* rw = gbl(static_cast<const W*>(ea.rwall)) + (int64_t)ea.swc[sh] * ea.nx;
#pragma unroll
    for (int k = 0; k < L::Q; k++) {
      if (L::cx[k] == 0 || (L::cy[k] == 0 && L::cz[k] == 0)) continue;
      if (L::cy[k] != cy || L::cz[k] != cz) continue;
      const int xf = L::cx[k] > 0 ? xp : xm;
      const double r = static_cast<double>(rw[xf]);
      const double go = dec<S, double>(gbl(g)[col * ea.sC + L::row[L::opp[k]] * ea.sI + xf]);
      F0 -= 2.0 * r * go * L::cx[k];
      K += 6.0 * ea.rho0 * r * L::w[k];
    }
  }
  const double gam = ea.gamma_e;
  const double c[3] = {0.0, 1.0, -1.0}, w[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
  double u, F;
  if (!ea.phon) {
    u = (j + 0.5 * (ea.force_e + F0)) / (rho * (1.0 + 0.5 * gam) + 0.5 * K);
    F = ea.force_e + F0 - K * u - gam * rho * u;
  } else {
    // phonon line beside it: the electron-phonon drag G (u - u_p), G =
    // gamma_ep rho, on both (opposite signs) and the crystal drag on the
    // phonons; with the half-forces a 2 x 2 linear system in (u, u_p)
    const double p0 = es[3 * n + s], p1 = es[4 * n + line + xm], p2 = es[5 * n + line + xp];
    const double drp = p0 + p1 + p2, jp = p1 - p2;
    const double rp = ea.rho_p0 + drp, gp = ea.gamma_pc;
    const double G = ea.gamma_ep * rho;
    const double a11 = rho * (1.0 + 0.5 * gam) + 0.5 * K + 0.5 * G;
    const double a22 = rp * (1.0 + 0.5 * gp) + 0.5 * G;
    const double b1 = j + 0.5 * (ea.force_e + F0);
    const double det = a11 * a22 - 0.25 * G * G;
    u = (b1 * a22 + 0.5 * G * jp) / det;
    const double up = (a11 * jp + 0.5 * G * b1) / det;
    F = ea.force_e + F0 - K * u - gam * rho * u - G * (u - up);
    const double Fp = -gp * rp * up + G * (u - up);
    const double omp = ea.omega_p, Ap = 1.0 - 0.5 * omp;
    const double dp[3] = {p0, p1, p2};
#pragma unroll
    for (int i = 0; i < 3; i++) {
      const double eq =
          w[i] * (drp + rp * (3.0 * c[i] * up + 4.5 * c[i] * c[i] * up * up - 1.5 * up * up));
      const double src = Ap * w[i] * (3.0 * (c[i] - up) + 9.0 * c[i] * up * c[i]) * Fp;
      ed[(3 + i) * n + s] = dp[i] - omp * (dp[i] - eq) + src;
    }
    ue[n + s] = up;
  }
  const double om = ea.omega_e, A = 1.0 - 0.5 * om;
  const double d[3] = {d0, d1, d2};
#pragma unroll
  for (int i = 0; i < 3; i++) {
    const double eq = w[i] * (drho + rho * (3.0 * c[i] * u + 4.5 * c[i] * c[i] * u * u - 1.5 * u * u));
    const double src = A * w[i] * (3.0 * (c[i] - u) + 9.0 * c[i] * u * c[i]) * F;
    ed[i * n + s] = d[i] - om * (d[i] - eq) + src;
  }
  ue[s] = u;
}

template <class L, typename S, typename W>
__global__ void __launch_bounds__(256) k_electron_step(const S* __restrict__ g,
                                                       const double* __restrict__ es,
                                                       double* __restrict__ ed,
                                                       double* __restrict__ ue, ElecArgs ea) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (int64_t)ea.nshell * ea.nx) return;
  electron_node<L, S, W>(g, es, ed, ue, ea, s);
}

// The electron step of up to kEGroupMax members of a batch group (blockIdx.y
// picks the member, blockIdx.x a block of its line nodes), each from the
// water state and line buffer of its current parity, before the group's
// water step: as k_electron_step for each member alone.
template <class L, typename S, typename W>
__global__ void __launch_bounds__(256) k_batch_electrons(const MemberDesc* __restrict__ md,
                                                         EGroup eg,
                                                         const int64_t* __restrict__ bstep,
                                                         int64_t step_off) {
  if ((int)blockIdx.y >= eg.n) return;
  const MemberDesc& d = md[eg.slot[blockIdx.y]];
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (int64_t)d.ea.nshell * d.ea.nx) return;
  const int64_t k = *bstep + step_off;
  const int odd = (int)((d.cur_base + k) & 1);
  electron_node<L, S, W>(static_cast<const S*>(d.pop[odd]), d.eline[odd], d.eline[1 - odd], d.uel,
                         d.ea, s);
}

// ------------------------------------------------------------ moments

template <class L, typename S, typename W, bool BOUZ, bool ELEC = false, bool MASKED = false>
__global__ void __launch_bounds__(512) k_moments(const S* __restrict__ src, StepArgs a,
                                                 int which, double* __restrict__ field,
                                                 double* __restrict__ partials) {
  const int slot = blockIdx.x / a.segs;
  const int seg = blockIdx.x - slot * a.segs;
  const int x = seg * a.bx + threadIdx.x;
  double jx_cell = 0.0, drho_cell = 0.0;
  const LBM_GLOBAL ColSlot& cs = gbl(a.slots)[slot];
  const int col = uniform(cs.col);
  // masked walls: solid points contribute nothing (their field stays zero)
  const int cw = MASKED && x < a.nx ? gbl(a.cellw)[x + (int64_t)a.nx * (col % a.ny)] : 0;
  if (x < a.nx && !(MASKED && cw == kCellSolid)) {
    double df[L::Q];
    if constexpr (MASKED) {
      const int z = col / a.ny;
      if (a.open) {  // reads clamped at the ends, then the ghosts
        uint32_t wl = 0u;
        if (cw >= 0)
          gather_masked<L, S, double, W, true>(src, a, col, z, x, cw, df, &wl);
        else
          gather_masked_interior<L, S, double, true>(src, a, col, z, x, df);
        ColInfo info;
        info.wallcol = 0;
        info.mask = wl | ((L::Q == 19 && (z == 0 || z == a.nz - 1)) ? kWrapColumn : 0u);
        open_patch<L, S, double>(src, a, col, x, info, df);
      } else {
        gather_masked<L, S, double, W>(src, a, col, z, x, cw, df);
      }
    } else {
      ColInfo info;
      info.wallcol = uniform(cs.wallcol);
      info.mask = (uint32_t)uniform((int)cs.mask);
      // with electron sheets the wall moves with u_e of the last step
      if (a.open) {  // reads clamped at the ends, then the ghosts
        gather<L, S, double, W, BOUZ, ELEC, true>(src, a, col, x, info, df);
        open_patch<L, S, double, BOUZ, W>(src, a, col, x, info, df);
      } else {
        gather<L, S, double, W, BOUZ, ELEC>(src, a, col, x, info, df);
      }
    }
    double drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
      drho += df[i];
      jx += L::cx[i] * df[i];
      jy += L::cy[i] * df[i];
      jz += L::cz[i] * df[i];
    }
    jx += a.F[0] / 2;
    jy += a.F[1] / 2;
    jz += a.F[2] / 2;
    const double rho = a.rho0 + drho;
    jx_cell = jx;
    drho_cell = drho;
    if (field) {
      double v = which == 0 ? rho : (which == 1 ? jx / rho : (which == 2 ? jy / rho : jz / rho));
      field[(int64_t)col * a.nx + x] = v;
    }
  }
  // deterministic block reduction (the checked step kernel forms the same)
  block_partials(jx_cell, drho_cell, partials + 2 * (int64_t)blockIdx.x);
}

// Fixed-order FP64 sum of the (j_x, rho - rho0) partials of nblocks blocks:
// thread t adds blocks t, t + 1024, ... in order (loads unrolled so that
// several are in flight), then a fixed butterfly in each wave and the 16
// waves in order.  out: the two sums, then the invariants they give, flux
// = sum j_x / nx, mass = nfluid rho0 + sum (rho - rho0), mass deviation.
constexpr int kReduceThreads = 1024;
__global__ void __launch_bounds__(kReduceThreads) k_reduce_final(const double* __restrict__ partials,
                                                                 int64_t nblocks,
                                                                 double* __restrict__ out, int nx,
                                                                 double mass0,
                                                                 double* __restrict__ out_host) {
  __shared__ double red[2][kReduceThreads / 64];
  const double2* p2 = reinterpret_cast<const double2*>(partials);
  double t0 = 0, t1 = 0;
#pragma unroll 8
  for (int64_t b = threadIdx.x; b < nblocks; b += kReduceThreads) {
    const double2 v = p2[b];
    t0 += v.x;
    t1 += v.y;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  t0 = wave_sum(t0);
  t1 = wave_sum(t1);
  if (lane == 0) {
    red[0][wv] = t0;
    red[1][wv] = t1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0, s1 = 0;
    for (int k = 0; k < kReduceThreads / 64; k++) {
      s0 += red[0][k];
      s1 += red[1][k];
    }
    const double v[5] = {s0, s1, s0 / nx, mass0 + s1, s1};
    for (int k = 0; k < 5; k++) {
      out[k] = v[k];
      if (out_host) out_host[k] = v[k];  // pinned host memory: no copy needed
    }
  }
}

// ------------------------------------------------------------ friction quadrature
constexpr int kQuadThreads = 256;
constexpr int kQuadNodes = 4;     // wall nodes per workgroup (share the LDS tile)
constexpr int kQuadTile = 1024;   // omega points per LDS tile

struct OmegaEntry {
  double s, t, v, pad;  // w^2, gamma_s^2 w^2, gamma_s w Im g_l(w) / sinh^2(w/2T)
};

// 1/d for the integrands' denominators (positive, far inside the normal
// range: at least gamma_s^2 (dw/2)^2): the hardware reciprocal refined by
// two Newton-Raphson steps r <- r + r (1 - d r), each of which squares the
// relative error, so the result is within about an ulp of 1/d.  Four fused
// multiply-adds and one reciprocal instead of the scaled, fixed-up IEEE
// division; the sums it feeds hold positive terms, so their relative error
// stays at that level.
__device__ __forceinline__ double recip_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}

// raw[k] for k < n uses omega[k]; raw[n] is the reference at omega0.
__global__ void __launch_bounds__(kQuadThreads) k_friction_raw(SpecArgs s,
                                                               const double* __restrict__ omega,
                                                               int64_t n,
                                                               double* __restrict__ raw) {
  __shared__ OmegaEntry tab[kQuadTile];
  __shared__ double red[kQuadNodes][kQuadThreads / 64];
  const int tid = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * kQuadNodes;
  double om2[kQuadNodes];
#pragma unroll
  for (int j = 0; j < kQuadNodes; j++) {
    const int64_t k = k0 + j;
    const double o = k < n ? omega[k] : s.omega0;  // k >= n: reference (k == n) or padding
    om2[j] = o * o;
  }
  const double dq = s.q_max / s.nq, dw = s.w_max / s.nw;
  const double gs2 = s.gamma_s * s.gamma_s, wl2 = s.omega_l * s.omega_l;
  const double gl2 = s.gamma_l * s.gamma_l;
  double acc[kQuadNodes];
#pragma unroll
  for (int j = 0; j < kQuadNodes; j++) acc[j] = 0.0;

  for (int b0 = 0; b0 < s.nw; b0 += kQuadTile) {
    const int nb = min(kQuadTile, s.nw - b0);
    __syncthreads();
    for (int b = tid; b < nb; b += kQuadThreads) {
      const double w = ((double)(b0 + b) + 0.5) * dw;
      const double w2 = w * w;
      const double sh = sinh(w / (2.0 * s.T));
      const double dl = wl2 - w2;
      const double iml = s.a_l * wl2 * s.gamma_l * w / (dl * dl + gl2 * w2);
      OmegaEntry e;
      e.s = w2;
      e.t = gs2 * w2;
      e.v = s.gamma_s * w * iml / (sh * sh);
      e.pad = 0.0;
      tab[b] = e;
    }
    __syncthreads();
    for (int ai = tid; ai < s.nq; ai += kQuadThreads) {
      const double q = ((double)ai + 0.5) * dq;
      const double kq = q * q * q * exp(-2.0 * q * s.d);
      const double qd = s.dispersion ? q * s.d : 1.0;
      double P[kQuadNodes], S[kQuadNodes];
#pragma unroll
      for (int j = 0; j < kQuadNodes; j++) {
        P[j] = om2[j] * qd;
        S[j] = 0.0;
      }
      for (int b = 0; b < nb; b++) {
        const OmegaEntry e = tab[b];  // same b for every lane: LDS broadcast
#pragma unroll
        for (int j = 0; j < kQuadNodes; j++) {
          const double dd = P[j] - e.s;
          S[j] = __builtin_fma(e.v, recip_nr(dd * dd + e.t), S[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < kQuadNodes; j++) acc[j] += kq * P[j] * S[j];
    }
  }
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int j = 0; j < kQuadNodes; j++) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) red[j][wv] = v;
  }
  __syncthreads();
  if (tid < kQuadNodes) {
    const int64_t k = k0 + tid;
    if (k <= n) {
      double t = 0;
      for (int w = 0; w < kQuadThreads / 64; w++) t += red[tid][w];
      const double C = 1.0 / (8.0 * M_PI * M_PI * s.T);
      raw[k] = C * dq * dw * t;
    }
  }
}

// The screened form: complex responses g_s = P (d_s + i gamma_s w) / D,
// d_s = P - w^2, D = d_s^2 + gamma_s^2 w^2, and g_l = a_l W (d_l + i gamma_l w)
// / (d_l^2 + gamma_l^2 w^2), W = omega_l^2 + v_l^2 q^2, d_l = W - w^2; with
// z = e^{-2qd} g_s g_l = (e P / D)(a + i b), a = d_s Re g_l - gamma_s w Im g_l,
// b = d_s Im g_l + gamma_s w Re g_l, the term
//   q^3 e^{-2qd} Im g_s Im g_l / (sinh^2 |1 - z|^2)
//   = q^3 e^{-2qd} P (gamma_s w / sinh^2) Im g_l D / ((D - e P a)^2 + (e P b)^2)
// takes one divide (SCREEN = false: the unscreened term with a dispersive
// liquid, q^3 e^{-2qd} P (gamma_s w / sinh^2) Im g_l / D).
constexpr int kFullTile = 512;

struct OmegaEntryFull {
  double w2, gw, t, v, glw, gl2w2, pad0, pad1;  // w^2, gamma_s w, gamma_s^2 w^2,
                                                // gamma_s w / sinh^2, gamma_l w, (gamma_l w)^2
};

template <bool SCREEN>
__global__ void __launch_bounds__(kQuadThreads) k_friction_full(SpecArgs s,
                                                                const double* __restrict__ omega,
                                                                int64_t n,
                                                                double* __restrict__ raw) {
  __shared__ OmegaEntryFull tab[kFullTile];
  __shared__ double red[kQuadNodes][kQuadThreads / 64];
  const int tid = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * kQuadNodes;
  double om2[kQuadNodes];
#pragma unroll
  for (int j = 0; j < kQuadNodes; j++) {
    const int64_t k = k0 + j;
    const double o = k < n ? omega[k] : s.omega0;  // k >= n: reference (k == n) or padding
    om2[j] = o * o;
  }
  const double dq = s.q_max / s.nq, dw = s.w_max / s.nw;
  double acc[kQuadNodes];
#pragma unroll
  for (int j = 0; j < kQuadNodes; j++) acc[j] = 0.0;

  for (int b0 = 0; b0 < s.nw; b0 += kFullTile) {
    const int nb = min(kFullTile, s.nw - b0);
    __syncthreads();
    for (int b = tid; b < nb; b += kQuadThreads) {
      const double w = ((double)(b0 + b) + 0.5) * dw;
      const double sh = sinh(w / (2.0 * s.T));
      OmegaEntryFull e;
      e.w2 = w * w;
      e.gw = s.gamma_s * w;
      e.t = e.gw * e.gw;
      e.v = e.gw / (sh * sh);
      e.glw = s.gamma_l * w;
      e.gl2w2 = e.glw * e.glw;
      e.pad0 = e.pad1 = 0.0;
      tab[b] = e;
    }
    __syncthreads();
    for (int ai = tid; ai < s.nq; ai += kQuadThreads) {
      const double q = ((double)ai + 0.5) * dq;
      const double ex = exp(-2.0 * q * s.d);
      const double kq = q * q * q * ex;
      const double qd = s.dispersion ? q * s.d : 1.0;
      const double Wl = s.omega_l * s.omega_l + s.v_l * s.v_l * q * q;
      const double Al = s.a_l * Wl;
      double P[kQuadNodes], eP[kQuadNodes], S[kQuadNodes];
#pragma unroll
      for (int j = 0; j < kQuadNodes; j++) {
        P[j] = om2[j] * qd;
        eP[j] = ex * P[j];
        S[j] = 0.0;
      }
      for (int b = 0; b < nb; b++) {
        const OmegaEntryFull e = tab[b];  // same b for every lane: LDS broadcast
        const double dl = Wl - e.w2;
        const double inv = Al / (dl * dl + e.gl2w2);
        const double Rl = inv * dl, Il = inv * e.glw;
        const double vI = e.v * Il;
        const double c1 = e.gw * Il, c2 = e.gw * Rl;
#pragma unroll
        for (int j = 0; j < kQuadNodes; j++) {
          const double dd = P[j] - e.w2;
          const double D = dd * dd + e.t;
          if constexpr (SCREEN) {
            const double a = dd * Rl - c1, bb = dd * Il + c2;
            const double A = D - eP[j] * a, B = eP[j] * bb;
            S[j] = __builtin_fma(vI * D, recip_nr(A * A + B * B), S[j]);
          } else {
            S[j] = __builtin_fma(vI, recip_nr(D), S[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < kQuadNodes; j++) acc[j] += kq * P[j] * S[j];
    }
  }
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int j = 0; j < kQuadNodes; j++) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) red[j][wv] = v;
  }
  __syncthreads();
  if (tid < kQuadNodes) {
    const int64_t k = k0 + tid;
    if (k <= n) {
      double t = 0;
      for (int w = 0; w < kQuadThreads / 64; w++) t += red[tid][w];
      const double C = 1.0 / (8.0 * M_PI * M_PI * s.T);
      raw[k] = C * dq * dw * t;
    }
  }
}

__global__ void k_friction_lat(const double* __restrict__ raw, int64_t n, double target,
                               double* __restrict__ lambda) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) lambda[k] = target * raw[k] / raw[n];
}

template <typename W>
__global__ void k_set_r(const double* __restrict__ lambda, int64_t n, W* __restrict__ r,
                        int* __restrict__ bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double l = lambda[k];
  if (!(l >= 0.0)) {
    *bad = 1;  // every writer stores the same value
    return;
  }
  r[k] = static_cast<W>(isinf(l) ? 1.0 : 3.0 * l / (1.0 + 3.0 * l));
}

// ------------------------------------------------------------ copy probe
__global__ void __launch_bounds__(256) k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                              int64_t n16) {
  // one 16-byte element per thread: measured faster than a grid-stride loop
  // (1 GiB: 6.2 against 4.8 TB/s)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

// ------------------------------------------------------------ precision change
// rows x-lines of nx values, nxp_in / nxp_out elements apart; the output's
// padding is cleared
template <typename A, typename B>
__global__ void __launch_bounds__(256) k_convert(const A* __restrict__ in, int nxp_in,
                                                 B* __restrict__ out, int nxp_out, int64_t rows,
                                                 int nx) {
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const A* src = in + r * nxp_in;
    B* dst = out + r * nxp_out;
    for (int x = threadIdx.x; x < nxp_out; x += blockDim.x) {
      const double v = x < nx ? dec<A, double>(src[x]) : 0.0;
      if constexpr (sizeof(B) == 2)
        dst[x] = (B)(float)(v * kHalfScale);
      else
        dst[x] = (B)v;
    }
  }
}

// ------------------------------------------------------------ batches
// The lane's cell of a batch item: column, x, and the index shift from the
// item's first column (colA); false for an idle lane.  colA..colC are the
// item's first three run columns, loaded uniformly by the caller.
struct LaneCell {
  int col, x;
  unsigned dl;
};
__device__ __forceinline__ bool lane_cell(const WorkItem& item, const StepArgs& a, int colA,
                                          int colB, int colC, int lane, LaneCell* c) {
  int x = item.xs + lane, j = 0;
  if (item.ncols > 1) {
    // nxp >= 32: 64 lanes cross at most two column ends
    if (x >= a.nxp) {
      x -= a.nxp;
      j = 1;
      if (x >= a.nxp) {
        x -= a.nxp;
        j = 2;
      }
    }
    if (item.c0 + j >= item.ncols) return false;
  } else if (x >= a.nxp) {
    return false;
  }
  c->col = j == 0 ? colA : (j == 1 ? colB : colC);
  c->x = x;
  c->dl = (unsigned)((int64_t)(c->col - colA) * a.sC);
  return true;
}

// the first three column ids of an item's run from its first column on
__device__ __forceinline__ void run_cols(const int32_t* cols, const WorkItem& item, int* ca,
                                         int* cb, int* cc) {
  const LBM_GLOBAL int32_t* cl = gbl(cols) + item.cbase + item.c0;
  *ca = uniform(cl[0]);
  *cb = item.c0 + 1 < item.ncols ? uniform(cl[1]) : *ca;
  *cc = item.c0 + 2 < item.ncols ? uniform(cl[2]) : *ca;
}

template <class L, typename S, typename M, bool BOUZ, int TH = 0, bool OPEN = false,
          bool ELEC = false>
__global__ void __launch_bounds__(512) k_batch_step(const MemberDesc* __restrict__ md,
                                                    const WorkItem* __restrict__ items,
                                                    const int32_t* __restrict__ cols,
                                                    int64_t first, int64_t nwall, int64_t last,
                                                    const int64_t* __restrict__ bstep,
                                                    int64_t step_off, int wpb) {
  // items [first, last) of one group of members, general-path items
  // [first, nwall) first; on odd step_off the others are taken in reverse
  // order (whole workgroups: both ranges are multiples of wpb), so that
  // consecutive steps of a group meet its most recently written lines first.
  // The wave index is in a scalar register: item and member are wave-uniform.
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  int64_t it = first + (int64_t)blockIdx.x * wpb + wv;
  if (it >= last) return;
  if ((step_off & 1) && it >= nwall) it = last - 1 - (it - nwall);
  const WorkItem item = items[it];
  if (item.member < 0) return;
  const MemberDesc& d = md[item.member];
  const int64_t k = uniform64(*gbl(bstep)) + step_off;  // steps since the batch was built
  const StepArgs& a = d.a;
  int colA, colB, colC;
  run_cols(cols, item, &colA, &colB, &colC);
  LaneCell c;
  if (!lane_cell(item, a, colA, colB, colC, (int)(threadIdx.x & 63), &c)) return;
  const int xc = c.x < a.nx ? c.x : a.nx - 1;  // padding lanes: as in k_step
  // both pointers loaded up front, then selected: no load waits on the parity
  const void* p0 = d.pop[0];
  const void* p1 = d.pop[1];
  const bool odd = ((d.cur_base + k) & 1) != 0;
  const S* src = static_cast<const S*>(odd ? p1 : p0);
  S* dst = static_cast<S*>(const_cast<void*>(odd ? p0 : p1));
  ColInfo info;
  info.wallcol = item.wallcol;
  info.mask = item.mask;
  M df[L::Q];
  // thermal term of the member's cell and step (each member its own kT and
  // seed), drawn before the gather as in k_step
  M xi[L::Q];
  if constexpr (TH != 0)
    thermal_noise<L, M, TH, NormalT<S>>(a, (uint32_t)c.col * (uint32_t)a.nx + (uint32_t)c.x, d.base_step + k,
                            xi);
  gather<L, S, M, M, BOUZ, ELEC, OPEN>(src, a, colA, xc, info, df, c.dl);
  // open ends: the ghosts from the records of the buffer read (the lane's own
  // column: runs of plain columns have no wall links or z wrap)
  if constexpr (OPEN) open_correct<L, M, BOUZ>(a, d.bmom[odd ? 1 : 0], c.col, xc, info, df);
  M rec[4];
  collide_store<L, M, S, TH, OPEN>(df, a, gbl(dst) + (int64_t)colA * a.sC, c.dl + (unsigned)c.x,
                                   (uint32_t)c.col * (uint32_t)a.nx + (uint32_t)c.x,
                                   d.base_step + k, xi, rec);
  if constexpr (OPEN)
    if (c.x == xc && (c.x == 0 || c.x == a.nx - 1)) {
      LBM_GLOBAL double* o = gbl(d.bmom[odd ? 0 : 1]) +
                             ((c.x == 0 ? 0 : (int64_t)a.ny * a.nz) + c.col) * 4;
      const M rho = static_cast<M>(a.rho0) + rec[0];
      o[0] = static_cast<double>(rec[0]);
      o[1] = static_cast<double>(rec[1] / rho);
      o[2] = static_cast<double>(rec[2] / rho);
      o[3] = static_cast<double>(rec[3] / rho);
    }
}

// per-item partial sums of (j_x, rho - rho0) of items [first, first + count);
// one wave per item, partials at the item's index
template <class L, typename S, typename W, bool BOUZ>
__global__ void __launch_bounds__(256) k_batch_moments(const MemberDesc* __restrict__ md,
                                                       const WorkItem* __restrict__ items,
                                                       const int32_t* __restrict__ cols,
                                                       int64_t first, int64_t count,
                                                       const int64_t* __restrict__ bstep,
                                                       double* __restrict__ partials) {
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t j = (int64_t)blockIdx.x * 4 + wv;
  if (j >= count) return;
  const int64_t it = first + j;
  const WorkItem item = items[it];
  if (item.member < 0) return;  // empty items are in no member's reduction
  const MemberDesc& d = md[item.member];
  const StepArgs& a = d.a;
  int colA, colB, colC;
  run_cols(cols, item, &colA, &colB, &colC);
  LaneCell c;
  double jx = 0.0, dr = 0.0;
  if (lane_cell(item, a, colA, colB, colC, (int)(threadIdx.x & 63), &c) && c.x < a.nx) {
    const int par = (int)((d.cur_base + uniform64(*gbl(bstep))) & 1);
    const S* src = static_cast<const S*>(d.pop[par]);
    ColInfo info;
    info.wallcol = item.wallcol;
    info.mask = item.mask;
    double df[L::Q];
    if (a.open) {  // reads clamped at the ends, then the ghosts
      gather<L, S, double, W, BOUZ, false, true>(src, a, colA, c.x, info, df, c.dl);
      open_patch<L, S, double, BOUZ, W>(src, a, c.col, c.x, info, df);
    } else if (a.ue) {  // walls moving with the electron lines of the last step
      gather<L, S, double, W, BOUZ, true>(src, a, colA, c.x, info, df, c.dl);
    } else {
      gather<L, S, double, W, BOUZ>(src, a, colA, c.x, info, df, c.dl);
    }
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
      dr += df[i];
      jx += L::cx[i] * df[i];
    }
    jx += a.F[0] / 2;
  }
  jx = wave_sum(jx);
  dr = wave_sum(dr);
  if ((threadIdx.x & 63) == 0) {
    partials[2 * it] = jx;
    partials[2 * it + 1] = dr;
  }
}

// one block per member slot m: the partials of its items, listed in
// order[mstart[m] .. mstart[m] + mcount[m]) (a free slot has none: zeros)
__global__ void __launch_bounds__(256) k_batch_reduce(const double* __restrict__ partials,
                                                      const int32_t* __restrict__ order,
                                                      const int64_t* __restrict__ mstart,
                                                      const int64_t* __restrict__ mcount,
                                                      double* __restrict__ out) {
  __shared__ double red[2][256];
  const int m = blockIdx.x;
  double t0 = 0, t1 = 0;
  const int64_t k0 = mstart[m], k1 = mstart[m] + mcount[m];
  for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
    const int64_t it = order[k];
    t0 += partials[2 * it];
    t1 += partials[2 * it + 1];
  }
  red[0][threadIdx.x] = t0;
  red[1][threadIdx.x] = t1;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if ((int)threadIdx.x < s2) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s2];
      red[1][threadIdx.x] += red[1][threadIdx.x + s2];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * m] = red[0][0];
    out[2 * m + 1] = red[1][0];
  }
}

// ------------------------------------------------------------ step base
__global__ void k_set_step(int64_t* __restrict__ d, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *d = v;
}
__global__ void k_add_step(int64_t* __restrict__ d, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *d += v;
}

// ------------------------------------------------------------ launchers
hipError_t launch_set_step(int64_t* d, int64_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, st, d, v);
  return hipGetLastError();
}
const void* add_step_kernel_ptr() { return reinterpret_cast<const void*>(&k_add_step); }

template <class L, typename S, typename M>
static const void* batch_kernel_t(bool bouz, int th, bool open, bool elec) {
  if (elec && bouz) {
    if (th == 1) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, true, 1, false, true>);
    if (th == 2) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, true, 2, false, true>);
    return reinterpret_cast<const void*>(&k_batch_step<L, S, M, true, 0, false, true>);
  }
  if (elec) {
    if (th == 1) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, false, 1, false, true>);
    if (th == 2) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, false, 2, false, true>);
    return reinterpret_cast<const void*>(&k_batch_step<L, S, M, false, 0, false, true>);
  }
  if (open && bouz) {
    if (th == 1) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, true, 1, true>);
    if (th == 2) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, true, 2, true>);
    return reinterpret_cast<const void*>(&k_batch_step<L, S, M, true, 0, true>);
  }
  if (open) {
    if (th == 1) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, false, 1, true>);
    if (th == 2) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, false, 2, true>);
    return reinterpret_cast<const void*>(&k_batch_step<L, S, M, false, 0, true>);
  }
  if (bouz) {
    if (th == 1) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, true, 1>);
    if (th == 2) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, true, 2>);
    return reinterpret_cast<const void*>(&k_batch_step<L, S, M, true, 0>);
  }
  if (th == 1) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, false, 1>);
  if (th == 2) return reinterpret_cast<const void*>(&k_batch_step<L, S, M, false, 2>);
  return reinterpret_cast<const void*>(&k_batch_step<L, S, M, false, 0>);
}
const void* batch_step_kernel_ptr(int q, int prec, bool bouz, int th, bool open, bool elec) {
  if (q == 9) {
    if (prec == 0) return batch_kernel_t<D2Q9, double, double>(bouz, th, open, elec);
    if (prec == 1) return batch_kernel_t<D2Q9, float, double>(bouz, th, open, elec);
    return batch_kernel_t<D2Q9, _Float16, float>(bouz, th, open, elec);
  }
  if (prec == 0) return batch_kernel_t<D3Q19, double, double>(bouz, th, open, elec);
  if (prec == 1) return batch_kernel_t<D3Q19, float, double>(bouz, th, open, elec);
  return batch_kernel_t<D3Q19, _Float16, float>(bouz, th, open, elec);
}

const void* batch_electron_kernel_ptr(int q, int prec) {
  if (q == 9) {
    if (prec == 0) return reinterpret_cast<const void*>(&k_batch_electrons<D2Q9, double, double>);
    if (prec == 1) return reinterpret_cast<const void*>(&k_batch_electrons<D2Q9, float, double>);
    return reinterpret_cast<const void*>(&k_batch_electrons<D2Q9, _Float16, float>);
  }
  if (prec == 0) return reinterpret_cast<const void*>(&k_batch_electrons<D3Q19, double, double>);
  if (prec == 1) return reinterpret_cast<const void*>(&k_batch_electrons<D3Q19, float, double>);
  return reinterpret_cast<const void*>(&k_batch_electrons<D3Q19, _Float16, float>);
}

template <class L, typename S, typename W>
static hipError_t batch_moments_t(const MemberDesc* md, const WorkItem* items, const int32_t* cols,
                                  int64_t first, int64_t count, const int64_t* bstep,
                                  double* partials, bool bouz, hipStream_t st) {
  const dim3 grid((unsigned)((count + 3) / 4)), block(256);
  if (bouz)
    hipLaunchKernelGGL((k_batch_moments<L, S, W, true>), grid, block, 0, st, md, items, cols,
                       first, count, bstep, partials);
  else
    hipLaunchKernelGGL((k_batch_moments<L, S, W, false>), grid, block, 0, st, md, items, cols,
                       first, count, bstep, partials);
  return hipGetLastError();
}
hipError_t launch_batch_moments(int q, int prec, const MemberDesc* md, const WorkItem* items,
                                const int32_t* cols, int64_t first, int64_t count,
                                const int64_t* bstep, double* partials, bool bouz,
                                hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if ((count + 3) / 4 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
#define BM(L, S, W) \
  batch_moments_t<L, S, W>(md, items, cols, first, count, bstep, partials, bouz, st)
  if (q == 9)
    return prec == 0 ? BM(D2Q9, double, double) : prec == 1 ? BM(D2Q9, float, double)
                                                 : BM(D2Q9, _Float16, float);
  return prec == 0 ? BM(D3Q19, double, double) : prec == 1 ? BM(D3Q19, float, double)
                                                : BM(D3Q19, _Float16, float);
#undef BM
}
hipError_t launch_batch_reduce(const double* partials, const int32_t* order, const int64_t* mstart,
                               const int64_t* mcount, int nslots, double* out, hipStream_t st) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_reduce, dim3(nslots), dim3(256), 0, st, partials, order, mstart,
                     mcount, out);
  return hipGetLastError();
}

template <typename A>
static hipError_t convert_from(const void* in, int nxp_in, int pout, void* out, int nxp_out,
                               int64_t rows, int nx, hipStream_t st) {
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(rows, 16384));
  const A* src = static_cast<const A*>(in);
  if (pout == 0)
    hipLaunchKernelGGL((k_convert<A, double>), dim3(blocks), dim3(256), 0, st, src, nxp_in,
                       (double*)out, nxp_out, rows, nx);
  else if (pout == 1)
    hipLaunchKernelGGL((k_convert<A, float>), dim3(blocks), dim3(256), 0, st, src, nxp_in,
                       (float*)out, nxp_out, rows, nx);
  else
    hipLaunchKernelGGL((k_convert<A, _Float16>), dim3(blocks), dim3(256), 0, st, src, nxp_in,
                       (_Float16*)out, nxp_out, rows, nx);
  return hipGetLastError();
}
hipError_t launch_convert(int pin, const void* in, int nxp_in, int pout, void* out, int nxp_out,
                          int64_t rows, int nx, hipStream_t st) {
  if (pin == 0) return convert_from<double>(in, nxp_in, pout, out, nxp_out, rows, nx, st);
  if (pin == 1) return convert_from<float>(in, nxp_in, pout, out, nxp_out, rows, nx, st);
  return convert_from<_Float16>(in, nxp_in, pout, out, nxp_out, rows, nx, st);
}

hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t st) {
  const int64_t n16 = bytes / 16;
  const int64_t blocks = (n16 + 255) / 256;
  if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, st,
                     (const uint4*)src, (uint4*)dst, n16);
  return hipGetLastError();
}

// the step kernel for a wall kind and a noise form (0: none)
// nt: nontemporal stores (plain steps of states far beyond the last-level
// cache, no noise or sheets)
template <class L, typename S, typename M>
static const void* step_kernel_t(bool bouz, int th_mode, bool elec, bool masked, bool open,
                                 bool nt) {
  if (masked && open) {
    if (th_mode == 1) return reinterpret_cast<const void*>(&k_step_masked<L, S, M, 1, true>);
    if (th_mode == 2) return reinterpret_cast<const void*>(&k_step_masked<L, S, M, 2, true>);
    return reinterpret_cast<const void*>(&k_step_masked<L, S, M, 0, true>);
  }
  if (masked) {
    if (th_mode == 1) return reinterpret_cast<const void*>(&k_step_masked<L, S, M, 1>);
    if (th_mode == 2) return reinterpret_cast<const void*>(&k_step_masked<L, S, M, 2>);
    return reinterpret_cast<const void*>(&k_step_masked<L, S, M, 0>);
  }
  if (open && bouz) {
    if (th_mode == 1) return reinterpret_cast<const void*>(&k_step_open<L, S, M, true, 1>);
    if (th_mode == 2) return reinterpret_cast<const void*>(&k_step_open<L, S, M, true, 2>);
    return reinterpret_cast<const void*>(&k_step_open<L, S, M, true, 0>);
  }
  if (open) {
    if (th_mode == 1) return reinterpret_cast<const void*>(&k_step_open<L, S, M, false, 1>);
    if (th_mode == 2) return reinterpret_cast<const void*>(&k_step_open<L, S, M, false, 2>);
    return reinterpret_cast<const void*>(&k_step_open<L, S, M, false, 0>);
  }
  if (elec && bouz) {
    if (th_mode == 1) return reinterpret_cast<const void*>(&k_step<L, S, M, true, 1, true>);
    if (th_mode == 2) return reinterpret_cast<const void*>(&k_step<L, S, M, true, 2, true>);
    return reinterpret_cast<const void*>(&k_step<L, S, M, true, 0, true>);
  }
  if (elec) {
    if (th_mode == 1) return reinterpret_cast<const void*>(&k_step<L, S, M, false, 1, true>);
    if (th_mode == 2) return reinterpret_cast<const void*>(&k_step<L, S, M, false, 2, true>);
    return reinterpret_cast<const void*>(&k_step<L, S, M, false, 0, true>);
  }
  if (bouz) {
    if (th_mode == 1) return reinterpret_cast<const void*>(&k_step<L, S, M, true, 1>);
    if (th_mode == 2) return reinterpret_cast<const void*>(&k_step<L, S, M, true, 2>);
    if (nt) return reinterpret_cast<const void*>(&k_step<L, S, M, true, 0, false, false, true>);
    return reinterpret_cast<const void*>(&k_step<L, S, M, true, 0>);
  }
  if (th_mode == 1) return reinterpret_cast<const void*>(&k_step<L, S, M, false, 1>);
  if (th_mode == 2) return reinterpret_cast<const void*>(&k_step<L, S, M, false, 2>);
  if (nt) return reinterpret_cast<const void*>(&k_step<L, S, M, false, 0, false, false, true>);
  return reinterpret_cast<const void*>(&k_step<L, S, M, false, 0>);
}

template <class L, typename S, typename M>
static hipError_t launch_step_t(const void* src, void* dst, const StepArgs& a, bool bouz,
                                hipStream_t st) {
  const dim3 grid((unsigned)a.nactive, (unsigned)a.segs), block(a.bx);
  const S* s = static_cast<const S*>(src);
  S* d = static_cast<S*>(dst);
  StepArgs args = a;
  void* kargs[3] = {(void*)&s, (void*)&d, (void*)&args};
  return hipLaunchKernel(
      step_kernel_t<L, S, M>(bouz, a.th_mode, a.ue != nullptr, a.cellw != nullptr, a.open != 0,
                             a.ntstore != 0),
      grid, block, kargs, 0, st);
}

// the checked step: planar or tube walls, no noise, sheets, mask or open ends
template <class L, typename S, typename M>
static hipError_t launch_step_checked_t(const void* src, void* dst, const StepArgs& a, bool bouz,
                                        hipStream_t st) {
  const dim3 grid((unsigned)a.nactive, (unsigned)a.segs), block(a.bx);
  const S* s = static_cast<const S*>(src);
  S* d = static_cast<S*>(dst);
  StepArgs args = a;
  void* kargs[3] = {(void*)&s, (void*)&d, (void*)&args};
  const void* fn = bouz ? reinterpret_cast<const void*>(&k_step<L, S, M, true, 0, false, true>)
                        : reinterpret_cast<const void*>(&k_step<L, S, M, false, 0, false, true>);
  return hipLaunchKernel(fn, grid, block, kargs, 0, st);
}

hipError_t launch_step_checked(int q, int prec, const void* src, void* dst, const StepArgs& a,
                               bool bouz, hipStream_t st) {
  if (!a.partials || a.th_mode != 0 || a.ue || a.cellw || a.open) return hipErrorInvalidValue;
  if (q == 9) {
    if (prec == 0) return launch_step_checked_t<D2Q9, double, double>(src, dst, a, bouz, st);
    if (prec == 1) return launch_step_checked_t<D2Q9, float, double>(src, dst, a, bouz, st);
    return launch_step_checked_t<D2Q9, _Float16, float>(src, dst, a, bouz, st);
  }
  if (prec == 0) return launch_step_checked_t<D3Q19, double, double>(src, dst, a, bouz, st);
  if (prec == 1) return launch_step_checked_t<D3Q19, float, double>(src, dst, a, bouz, st);
  return launch_step_checked_t<D3Q19, _Float16, float>(src, dst, a, bouz, st);
}

hipError_t launch_step(int q, int prec, const void* src, void* dst, const StepArgs& a, bool bouz,
                       hipStream_t st) {
  if (q == 9) {
    if (prec == 0) return launch_step_t<D2Q9, double, double>(src, dst, a, bouz, st);
    if (prec == 1) return launch_step_t<D2Q9, float, double>(src, dst, a, bouz, st);
    return launch_step_t<D2Q9, _Float16, float>(src, dst, a, bouz, st);
  }
  if (prec == 0) return launch_step_t<D3Q19, double, double>(src, dst, a, bouz, st);
  if (prec == 1) return launch_step_t<D3Q19, float, double>(src, dst, a, bouz, st);
  return launch_step_t<D3Q19, _Float16, float>(src, dst, a, bouz, st);
}

const void* step_kernel_ptr(int q, int prec, bool bouz, int th_mode, bool elec, bool masked,
                            bool open, bool nt) {
#define KP(L, S, M) step_kernel_t<L, S, M>(bouz, th_mode, elec, masked, open, nt)
  if (q == 9) {
    if (prec == 0) return KP(D2Q9, double, double);
    if (prec == 1) return KP(D2Q9, float, double);
    return KP(D2Q9, _Float16, float);
  }
  if (prec == 0) return KP(D3Q19, double, double);
  if (prec == 1) return KP(D3Q19, float, double);
  return KP(D3Q19, _Float16, float);
#undef KP
}

const void* open_moments_kernel_ptr(int q, int prec) {
  if (q == 9) {
    if (prec == 0) return reinterpret_cast<const void*>(&k_open_moments<D2Q9, double, double>);
    if (prec == 1) return reinterpret_cast<const void*>(&k_open_moments<D2Q9, float, double>);
    return reinterpret_cast<const void*>(&k_open_moments<D2Q9, _Float16, float>);
  }
  if (prec == 0) return reinterpret_cast<const void*>(&k_open_moments<D3Q19, double, double>);
  if (prec == 1) return reinterpret_cast<const void*>(&k_open_moments<D3Q19, float, double>);
  return reinterpret_cast<const void*>(&k_open_moments<D3Q19, _Float16, float>);
}

hipError_t launch_open_moments(int q, int prec, const void* src, const StepArgs& a, double* bmom,
                               hipStream_t st) {
  const int64_t n = 2 * (int64_t)a.nactive;
  if (n <= 0 || (n + 255) / 256 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  StepArgs args = a;
  void* kargs[3] = {(void*)&src, (void*)&args, (void*)&bmom};
  return hipLaunchKernel(open_moments_kernel_ptr(q, prec), dim3((unsigned)((n + 255) / 256)),
                         dim3(256), kargs, 0, st);
}

const void* electron_kernel_ptr(int q, int prec) {
  if (q == 9) {
    if (prec == 0) return reinterpret_cast<const void*>(&k_electron_step<D2Q9, double, double>);
    if (prec == 1) return reinterpret_cast<const void*>(&k_electron_step<D2Q9, float, double>);
    return reinterpret_cast<const void*>(&k_electron_step<D2Q9, _Float16, float>);
  }
  if (prec == 0) return reinterpret_cast<const void*>(&k_electron_step<D3Q19, double, double>);
  if (prec == 1) return reinterpret_cast<const void*>(&k_electron_step<D3Q19, float, double>);
  return reinterpret_cast<const void*>(&k_electron_step<D3Q19, _Float16, float>);
}

hipError_t launch_electron_step(int q, int prec, const void* g, const double* e_src,
                                double* e_dst, double* ue, const ElecArgs& ea, hipStream_t st) {
  const int64_t n = (int64_t)ea.nshell * ea.nx;
  if (n <= 0 || (n + 255) / 256 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  ElecArgs args = ea;
  void* kargs[5] = {(void*)&g, (void*)&e_src, (void*)&e_dst, (void*)&ue, (void*)&args};
  return hipLaunchKernel(electron_kernel_ptr(q, prec), dim3((unsigned)((n + 255) / 256)), dim3(256),
                         kargs, 0, st);
}

template <class L, typename S, typename W>
static hipError_t launch_moments_t(const void* src, const StepArgs& a, bool bouz, int which,
                                   double* field, double* partials, hipStream_t st) {
  const dim3 grid((unsigned)((int64_t)a.nactive * a.segs)), block(a.bx);
  if (a.cellw)
    hipLaunchKernelGGL((k_moments<L, S, W, false, false, true>), grid, block, 0, st,
                       (const S*)src, a, which, field, partials);
  else if (bouz && a.ue)
    hipLaunchKernelGGL((k_moments<L, S, W, true, true>), grid, block, 0, st, (const S*)src, a,
                       which, field, partials);
  else if (bouz)
    hipLaunchKernelGGL((k_moments<L, S, W, true>), grid, block, 0, st, (const S*)src, a, which,
                       field, partials);
  else if (a.ue)
    hipLaunchKernelGGL((k_moments<L, S, W, false, true>), grid, block, 0, st, (const S*)src, a,
                       which, field, partials);
  else
    hipLaunchKernelGGL((k_moments<L, S, W, false>), grid, block, 0, st, (const S*)src, a, which,
                       field, partials);
  return hipGetLastError();
}

hipError_t launch_moments(int q, int prec, const void* src, const StepArgs& a, bool bouz,
                          int which, double* field, double* partials, hipStream_t st) {
  if (q == 9) {
    if (prec == 0) return launch_moments_t<D2Q9, double, double>(src, a, bouz, which, field, partials, st);
    if (prec == 1) return launch_moments_t<D2Q9, float, double>(src, a, bouz, which, field, partials, st);
    return launch_moments_t<D2Q9, _Float16, float>(src, a, bouz, which, field, partials, st);
  }
  if (prec == 0) return launch_moments_t<D3Q19, double, double>(src, a, bouz, which, field, partials, st);
  if (prec == 1) return launch_moments_t<D3Q19, float, double>(src, a, bouz, which, field, partials, st);
  return launch_moments_t<D3Q19, _Float16, float>(src, a, bouz, which, field, partials, st);
}

hipError_t launch_reduce_final(const double* partials, int64_t nblocks, double* out, int nx,
                               double mass0, hipStream_t st, double* out_host) {
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kReduceThreads), 0, st, partials, nblocks, out,
                     nx, mass0, out_host);
  return hipGetLastError();
}

hipError_t launch_friction(const SpecArgs& s, const double* omega, int64_t n, double* raw,
                           double* lambda, hipStream_t st) {
  const int64_t nodes = n + 1;
  const unsigned blocks = (unsigned)((nodes + kQuadNodes - 1) / kQuadNodes);
  if (s.coupling)
    hipLaunchKernelGGL(k_friction_full<true>, dim3(blocks), dim3(kQuadThreads), 0, st, s, omega, n,
                       raw);
  else if (s.v_l != 0.0)
    hipLaunchKernelGGL(k_friction_full<false>, dim3(blocks), dim3(kQuadThreads), 0, st, s, omega,
                       n, raw);
  else
    hipLaunchKernelGGL(k_friction_raw, dim3(blocks), dim3(kQuadThreads), 0, st, s, omega, n, raw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n > 0)
    hipLaunchKernelGGL(k_friction_lat, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, raw, n,
                       s.lambda_target, lambda);
  return hipGetLastError();
}

hipError_t launch_set_r(int prec, const double* lambda, int64_t n, void* r, int* bad,
                        hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (prec != 2)
    hipLaunchKernelGGL(k_set_r<double>, grid, block, 0, st, lambda, n, (double*)r, bad);
  else
    hipLaunchKernelGGL(k_set_r<float>, grid, block, 0, st, lambda, n, (float*)r, bad);
  return hipGetLastError();
}

}  // namespace lbm

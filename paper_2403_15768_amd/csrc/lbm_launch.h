// lbm_launch.h -- host-side launchers of the kernels in lbm_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"

namespace lbm {

// Spectral parameters as the quadrature kernel takes them (mirrors
// lbm_spectral of the public header).
struct SpecArgs {
  double T, omega0, gamma_s, omega_l, gamma_l, a_l, d;
  int nq, nw;
  double q_max, w_max;
  double lambda_target;
  int dispersion;
  int coupling;  // 1: screening denominator
  double v_l;    // liquid mode dispersion
};


// q: 9 or 19; prec: 0 F64, 1 F32, 2 F16S
hipError_t launch_step(int q, int prec, const void* src, void* dst, const StepArgs& a, bool bouz,
                       hipStream_t st);  // a.ue: electron-sheet walls; a.cellw: masked walls
// one step that also leaves the per-block FP64 (j_x, rho - rho0) partials of
// the populations its collision sees in a.partials (k_moments' blocks and
// order); planar or tube walls without noise, sheets, mask or open ends
hipError_t launch_step_checked(int q, int prec, const void* src, void* dst, const StepArgs& a,
                               bool bouz, hipStream_t st);
const void* step_kernel_ptr(int q, int prec, bool bouz, int th_mode, bool elec,
                            bool masked, bool open, bool nt);
// one electron step from the water state g (step n): e_src -> e_dst, u_e of
// step n -> ue; the water step of step n then reads ue
hipError_t launch_electron_step(int q, int prec, const void* g, const double* e_src,
                                double* e_dst, double* ue, const ElecArgs& ea, hipStream_t st);
const void* electron_kernel_ptr(int q, int prec);
// open x ends: the moments of the first and last node of every column of
// src ([side][column][4] doubles), before the step that reads src
hipError_t launch_open_moments(int q, int prec, const void* src, const StepArgs& a, double* bmom,
                               hipStream_t st);
const void* open_moments_kernel_ptr(int q, int prec);  // (src, StepArgs, bmom)
hipError_t launch_moments(int q, int prec, const void* src, const StepArgs& a, bool bouz,
                          int which, double* field, double* partials, hipStream_t st);
// out[0..4]: sum j_x, sum (rho - rho0), then flux (sum j_x / nx), mass
// (mass0 + sum (rho - rho0)) and the mass deviation; out_host (pinned host
// memory, device pointer) receives the same if not null
hipError_t launch_reduce_final(const double* partials, int64_t nblocks, double* out, int nx,
                               double mass0, hipStream_t st, double* out_host = nullptr);
hipError_t launch_friction(const SpecArgs& s, const double* omega, int64_t n, double* raw,
                           double* lambda, hipStream_t st);
hipError_t launch_set_step(int64_t* d, int64_t v, hipStream_t st);
const void* add_step_kernel_ptr();  // k_add_step(int64_t* d, int64_t v)
// storage-precision change (0 F64, 1 F32, 2 F16S) of `rows` x-lines of nx
// populations, nxp_in / nxp_out elements apart
hipError_t launch_convert(int pin, const void* in, int nxp_in, int pout, void* out, int nxp_out,
                          int64_t rows, int nx, hipStream_t st);
// batches
const void* batch_step_kernel_ptr(int q, int prec, bool bouz, int th, bool open,
                                  bool elec);  // th: noise form; open: open x ends
// k_batch_electrons: grid (blocks of 256 line nodes of the largest member,
// members), arguments (md, EGroup, bstep, step_off)
const void* batch_electron_kernel_ptr(int q, int prec);
// k_batch_step(const MemberDesc*, const WorkItem*, const int32_t* cols, int64_t first,
//              int64_t nwall, int64_t last, const int64_t* bstep, int64_t step_off, int wpb)
// per-item partials of the flux and mass of items [first, first + count)
hipError_t launch_batch_moments(int q, int prec, const MemberDesc* md, const WorkItem* items,
                                const int32_t* cols, int64_t first, int64_t count,
                                const int64_t* bstep, double* partials, bool bouz,
                                hipStream_t st);
// per member slot m < nslots: out[2m..2m+1] = sum of the partials of the
// items order[mstart[m] .. mstart[m] + mcount[m])
hipError_t launch_batch_reduce(const double* partials, const int32_t* order, const int64_t* mstart,
                               const int64_t* mcount, int nslots, double* out, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t st);
hipError_t launch_set_r(int prec, const double* lambda, int64_t n, void* r, int* bad,
                        hipStream_t st);

}  // namespace lbm

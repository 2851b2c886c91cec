// lbm_internal.h -- host-side context and plan shared by the API files.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_launch.h"

namespace lbm_host {

using lbm::ColInfo;
using lbm::StepArgs;

constexpr size_t kAlign = 256;
constexpr int kGraphSteps = 64;  // steps per captured graph (even: keeps buffer parity)
constexpr uint32_t kSeed = 0x2403157u;  // stochastic-rounding stream (same for every context)

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Plan {
  int Q = 0, prec = 0;
  size_t ssize = 0, wsize = 0;  // storage bytes, wall-table bytes per value
  int nx = 0, nxp = 0, ny = 0, nz = 0;
  int64_t ncolbox = 0, sI = 0, sC = 0;  // layout g[col][i][x]: col * sC + i * sI + x
  std::vector<lbm::ColSlot> slots;  // fluid columns: wall columns, then interior ones
  std::vector<ColInfo> colinfo;     // per box column (host only)
  std::vector<int32_t> wallcols;   // column id of each wall column, increasing
  std::vector<double> linkq;       // [wallcol][Q] wall fraction (0: no wall link)
  std::vector<double> bzc;         // [wallcol][Q][2] interpolation coefficients b, c (TUBE)
  int64_t nfluid = 0, nwall = 0;
  int bx = 0, segs = 0;
  int64_t nblocks = 0;
  bool bouz = false;
  // MASKED: per point of the (x, y) plane its 2-D wall-node index, or
  // kCellInterior / kCellSolid; per 2-D wall node and link the storage row of
  // the slip partner (kNoLink: the upstream point is fluid); the 2-D wall
  // nodes' x + nx y in increasing order
  bool masked = false;
  std::vector<unsigned char> solid;  // [x + nx y]
  std::vector<int32_t> cellw;
  std::vector<uint8_t> ptab;
  std::vector<int32_t> w2d;
  int64_t nw2d = 0;
  int pstride = 0;         // partner-table bytes per 2-D wall node (whole words)
  int64_t nwallslots = 0;  // leading slots whose columns hold wall nodes
  std::vector<int32_t> rowx;  // per wall row: count, then the x of its points ([y][nxp + 1])
  size_t off_cellw = 0, off_ptab = 0, off_rowx = 0;
  size_t off_bmom = 0;  // open ends: [side][column][4] moments of the end nodes
  int64_t nsheet = 0;               // electron shell nodes (nshell nx)
  // per shell: the wall column of the fluid column next to it (SLAB, DUCT);
  // TUBE: for the fluid columns at -y, +y, -z, +z of it, (column, wall
  // column) or (-1, -1)
  std::vector<int32_t> sheet_wc;
  std::vector<int32_t> shellof;     // TUBE: shell of each box column (-1: none)
  bool shells_whole = true;         // every wall link crossing x pulls from a shell
  // arena offsets
  size_t off_pop[2] = {0, 0}, pop_bytes = 0;
  size_t off_slots = 0, off_r = 0, off_bz = 0, off_lambda = 0, off_raw = 0,
         off_partials = 0, off_out = 0, off_flag = 0, off_step = 0, total = 0;
  size_t off_e[2] = {0, 0}, off_ue = 0, off_swc = 0, off_shellof = 0;  // electron shells
};

}  // namespace lbm_host

struct lbm_ctx {
  lbm_params p{};
  lbm_host::Plan pl;
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  void* pop[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t step = 0;
  lbm::StepArgs args{};
  std::string err;
  bool have_raw = false;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  bool graphs_ok = true;
  int64_t dstep_value = 0;  // value the device step base holds after enqueued work
  double kT = 0.0;          // lattice temperature of the thermal noise (0: none)
  bool elec = false;        // electron sheets on (SLAB)
  bool bmom_ok = false;     // open ends: end-node records of pop[cur] are current
  int64_t checked_step = -1;  // step whose invariants' partials the arena holds (-1: none)
  // 8 doubles of pinned host memory the reduce kernel writes the invariants
  // to, through fin_host_dev (null if none could be had)
  double* fin_host = nullptr;
  double* fin_host_dev = nullptr;
  int step_bx = 0;  // threads per block of the plain step launches (0: the plan's default)
  lbm::ElecArgs ea{};

  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(arena + off);
  }
  lbm_status fail(lbm_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return s;
  }
  lbm_status hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return LBM_OK;
    return fail(LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  }
};

#define HIPCHK(ctx, call)                                    \
  do {                                                       \
    lbm_status _s = (ctx)->hip((call), #call);               \
    if (_s != LBM_OK) return _s;                             \
  } while (0)


namespace lbm_host {
// the spectral parameters the quadrature accepts (finite, positive scales,
// coupling 0 or 1, v_l >= 0)
inline bool spectral_valid(const lbm_spectral* sp) {
  return sp && sp->T > 0 && sp->d > 0 && sp->gamma_s > 0 && sp->gamma_l > 0 && sp->omega_l > 0 &&
         sp->a_l > 0 && sp->q_max > 0 && sp->w_max > 0 && sp->omega0 > 0 && sp->nq >= 1 &&
         sp->nw >= 1 && sp->lambda_target >= 0 && (sp->coupling == 0 || sp->coupling == 1) &&
         sp->v_l >= 0 &&
         std::isfinite(sp->T + sp->d + sp->gamma_s + sp->gamma_l + sp->omega_l + sp->a_l +
                       sp->q_max + sp->w_max + sp->omega0 + sp->lambda_target + sp->v_l);
}
inline lbm::SpecArgs spec_args(const lbm_spectral* sp) {
  return lbm::SpecArgs{sp->T,     sp->omega0, sp->gamma_s,       sp->omega_l,    sp->gamma_l,
                       sp->a_l,   sp->d,      sp->nq,            sp->nw,         sp->q_max,
                       sp->w_max, sp->lambda_target, sp->dispersion, sp->coupling, sp->v_l};
}
lbm_status sync(lbm_ctx* c);
// open ends: the end-node records ([side][column][4]) of population buffer b
inline double* end_records(lbm_ctx* c, int b) {
  return c->at<double>(c->pl.off_bmom) + (size_t)b * 2 * c->pl.ncolbox * 4;
}
// rebuild the records of the current buffer if no step has left them
// (asynchronous, on the context's stream)
lbm_status ensure_end_records(lbm_ctx* c);
// one plain step launch; check: the step also leaves the per-block partials
// of the invariants of the state it reads (see lbm_step_checked)
lbm_status launch_one_step(lbm_ctx* c, bool check = false);
// the step arguments of the plain (unchecked) step launches: the context's,
// with the block width the autotuner chose (the moments kernel and the
// checked step keep the plan's, so that reductions do not depend on it)
inline lbm::StepArgs step_args(const lbm_ctx* c) {
  lbm::StepArgs a = c->args;
  if (c->step_bx > 0) {
    a.bx = c->step_bx;
    a.segs = (c->pl.nxp + c->step_bx - 1) / c->step_bx;
  }
  return a;
}
}  // namespace lbm_host

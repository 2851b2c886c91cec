// lbm_api.hip -- host side of the C ABI declared in include/lbm.h.
//
// Owns no device memory: every buffer is carved out of the caller's arena.
// Geometry set-up (which cells are fluid, which links end on the wall, the
// interpolated bounce-back coefficients) runs once per context on the host;
// everything per step runs in the kernels of lbm_kernels.hip on the
// context's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lbm_internal.h"

using lbm::ColInfo;
using lbm::StepArgs;
using namespace lbm_host;

namespace {

int lat_c(int Q, int i, int a) {
  if (Q == 9) return a == 0 ? lbm::D2Q9::cx[i] : (a == 1 ? lbm::D2Q9::cy[i] : 0);
  return a == 0 ? lbm::D3Q19::cx[i] : (a == 1 ? lbm::D3Q19::cy[i] : lbm::D3Q19::cz[i]);
}

// storage row of direction i within a column
int lat_row(int Q, int i) { return Q == 9 ? lbm::D2Q9::row[i] : lbm::D3Q19::row[i]; }
int lat_opp(int Q, int i) { return Q == 9 ? lbm::D2Q9::opp[i] : lbm::D3Q19::opp[i]; }
int lat_dir(int Q, int cx, int cy, int cz) {
  for (int k = 0; k < Q; k++)
    if (lat_c(Q, k, 0) == cx && lat_c(Q, k, 1) == cy && lat_c(Q, k, 2) == cz) return k;
  return -1;
}

// Slip partners at one node of a masked wall.  from_solid[i]: link i pulls
// from a solid point (set J); the links pointing into the solid are their
// opposites (set K, as many).  Each i in J gets one k in K and each k serves
// one i, so the wall rule's weights r and 1 - r of every into-wall population
// sum to one (exact mass).  Candidates in order of preference, each pass over
// i in increasing index and among the k not yet taken: the reflection about a
// y-normal wall (c_x, -c_y, -c_z), about an x-normal face (-c_x, c_y, -c_z),
// the opposite, the lowest free k.  Within a pass distinct i have distinct
// candidates, so the result does not depend on the order inside a pass.
void slip_partners(int Q, const bool* from_solid, int* partner) {
  bool into[19] = {}, taken[19] = {};
  for (int i = 0; i < Q; i++) {
    partner[i] = -1;
    if (from_solid[i]) into[lat_opp(Q, i)] = true;
  }
  for (int pass = 0; pass < 4; pass++)
    for (int i = 1; i < Q; i++) {
      if (!from_solid[i] || partner[i] >= 0) continue;
      const int cx = lat_c(Q, i, 0), cy = lat_c(Q, i, 1), cz = lat_c(Q, i, 2);
      int k = -1;
      if (pass == 0) k = lat_dir(Q, cx, -cy, -cz);
      else if (pass == 1) k = lat_dir(Q, -cx, cy, -cz);
      else if (pass == 2) k = lat_opp(Q, i);
      else
        for (int t = 1; t < Q && k < 0; t++)
          if (into[t] && !taken[t]) k = t;
      if (k > 0 && into[k] && !taken[k]) {
        partner[i] = k;
        taken[k] = true;
      }
    }
}

// Positive root s of |P - s C|^2 = R^2 with P inside and P - C outside the
// circle (the fraction of the link from the fluid node to the wall).
double wall_fraction(double py, double pz, double cy, double cz, double R) {
  const double a = cy * cy + cz * cz;
  const double b = -2.0 * (py * cy + pz * cz);
  const double c = py * py + pz * pz - R * R;  // < 0
  const double disc = std::sqrt(b * b - 4.0 * a * c);
  return b >= 0.0 ? (2.0 * c) / (-b - disc) : (-b + disc) / (2.0 * a);
}

lbm_status validate(const lbm_params* p, std::string* err) {
  auto fail = [&](const char* m) {
    if (err) *err = m;
    return LBM_EINVAL;
  };
  if (!p) return fail("null parameters");
  if (p->lattice != 9 && p->lattice != 19) return fail("lattice must be 9 or 19");
  if (p->precision < 0 || p->precision > 2) return fail("bad precision");
  if (p->geometry < 0 || p->geometry > 3) return fail("bad geometry");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail("sizes must be >= 1");
  if ((int64_t)p->ny * p->nz > (int64_t)1 << 28 || p->nx > (1 << 24)) return fail("box too large");
  if (p->lattice == 9 && (p->nz != 1 || (p->geometry != LBM_SLAB && p->geometry != LBM_MASKED)))
    return fail("D2Q9 needs SLAB or MASKED geometry with nz = 1");
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail("tau must be finite and > 0.5");
  if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return fail("rho0 must be finite and > 0");
  for (int a = 0; a < 3; a++)
    if (!std::isfinite(p->force[a])) return fail("force must be finite");
  if (!std::isfinite(p->wall_velocity_top)) return fail("wall velocity must be finite");
  if (p->wall_velocity_top != 0.0 && (p->geometry == LBM_TUBE || p->geometry == LBM_MASKED))
    return fail("moving top wall needs SLAB or DUCT");
  if (p->geometry == LBM_MASKED && !p->solid) return fail("MASKED needs a solid mask");
  if (p->geometry == LBM_TUBE &&
      (!(p->tube_radius > 0.0) || !std::isfinite(p->tube_cy) || !std::isfinite(p->tube_cz)))
    return fail("tube needs radius > 0 and a finite centre");
  return LBM_OK;
}

lbm_status make_plan(const lbm_params* p, Plan* P, std::string* err) {
  lbm_status s = validate(p, err);
  if (s != LBM_OK) return s;
  Plan& pl = *P;
  pl.Q = p->lattice;
  pl.prec = p->precision;
  pl.ssize = p->precision == LBM_F64 ? 8 : (p->precision == LBM_F32 ? 4 : 2);
  // wall tables in the arithmetic type: double for F64 and F32 (FP32 storage,
  // FP64 arithmetic), float for F16S
  pl.wsize = p->precision == LBM_F16S ? 4 : 8;
  pl.nx = p->nx;
  // x-lines of up to 128 cells are stored back to back (a column's Q lines
  // are written by one workgroup, so the cache lines they share are
  // completed in one L2); longer ones are padded to whole 128-byte cache
  // lines (32 floats or doubles, 64 halves) and the kernels write the
  // padding too, so no line is written in part by two workgroups
  const int pad = p->precision == LBM_F16S ? 64 : 32;
  pl.nxp = p->nx <= 128 ? p->nx : (p->nx + pad - 1) / pad * pad;
  pl.ny = p->ny;
  pl.nz = p->nz;
  pl.ncolbox = (int64_t)p->ny * p->nz;
  pl.sI = pl.nxp;
  pl.sC = (int64_t)pl.Q * pl.nxp;
  pl.bouz = p->geometry == LBM_TUBE;
  pl.masked = p->geometry == LBM_MASKED;
  // z periodic
  const bool slab = p->geometry == LBM_SLAB || pl.masked;

  std::vector<unsigned char> fluid(pl.ncolbox, 1);
  if (pl.masked) {
    // a column (y, z) holds storage when some x of its row is fluid
    pl.solid.assign((size_t)p->nx * p->ny, 0);
    for (int64_t k = 0; k < (int64_t)p->nx * p->ny; k++) pl.solid[k] = p->solid[k] != 0;
    for (int z = 0; z < p->nz; z++)
      for (int y = 0; y < p->ny; y++) {
        bool any = false;
        for (int x = 0; x < p->nx && !any; x++) any = !pl.solid[x + (int64_t)p->nx * y];
        fluid[y + (int64_t)p->ny * z] = any ? 1 : 0;
      }
  }
  if (p->geometry == LBM_TUBE) {
    const double R2 = p->tube_radius * p->tube_radius;
    for (int z = 0; z < p->nz; z++)
      for (int y = 0; y < p->ny; y++) {
        const double dy = y - p->tube_cy, dz = z - p->tube_cz;
        fluid[y + (int64_t)p->ny * z] = (dy * dy + dz * dz < R2) ? 1 : 0;
      }
  }
  auto fluid_at = [&](int y, int z) {
    if (slab) z = ((z % p->nz) + p->nz) % p->nz;
    if (y < 0 || y >= p->ny || z < 0 || z >= p->nz) return false;
    return fluid[y + (int64_t)p->ny * z] != 0;
  };

  pl.colinfo.assign(pl.ncolbox, ColInfo{-1, lbm::kSolidColumn});
  pl.slots.clear();
  pl.wallcols.clear();
  std::vector<int32_t> interior;
  for (int z = 0; z < p->nz; z++)
    for (int y = 0; y < p->ny; y++) {
      const int64_t col = y + (int64_t)p->ny * z;
      if (!fluid[col]) continue;
      uint32_t mask = 0;
      // masked walls: no column-wide wall links (the kernel classifies cells)
      for (int i = 1; i < pl.Q && !pl.masked; i++)
        if (!fluid_at(y - lat_c(pl.Q, i, 1), z - lat_c(pl.Q, i, 2))) mask |= 1u << i;
      ColInfo ci{-1, mask};
      if (mask) {
        ci.wallcol = (int32_t)pl.wallcols.size();
        pl.wallcols.push_back((int32_t)col);
      } else {
        interior.push_back((int32_t)col);
      }
      // pulls across the periodic z boundary take the general path
      if (slab && pl.Q == 19 && (z == 0 || z == p->nz - 1)) ci.mask |= lbm::kWrapColumn;
      pl.colinfo[col] = ci;
    }
  // wall columns first: their blocks do more work, so they start early
  // instead of forming the tail of the grid
  for (int32_t col : pl.wallcols)
    pl.slots.push_back(lbm::ColSlot{col, pl.colinfo[col].wallcol, pl.colinfo[col].mask, 0});
  for (int32_t col : interior) pl.slots.push_back(lbm::ColSlot{col, -1, pl.colinfo[col].mask, 0});
  const int64_t nwc = (int64_t)pl.wallcols.size();
  pl.linkq.assign(nwc * pl.Q, 0.0);
  if (pl.bouz) pl.bzc.assign(nwc * pl.Q * 2, 0.0);
  for (int64_t k = 0; k < nwc; k++) {
    const int col = pl.wallcols[k];
    const int y = col % p->ny, z = col / p->ny;
    const uint32_t mask = pl.colinfo[col].mask;
    for (int i = 0; i < pl.Q; i++) {
      if (!(mask & (1u << i))) continue;
      double q = 0.5;
      if (pl.bouz)
        q = wall_fraction(y - p->tube_cy, z - p->tube_cz, lat_c(pl.Q, i, 1), lat_c(pl.Q, i, 2),
                          p->tube_radius);
      pl.linkq[k * pl.Q + i] = q;
      if (pl.bouz) {
        // BB = a g_opp(x) + b g_opp(x + c_i) + c g_i(x) with a = 1 - b - c:
        // q < 1/2: a = 2q, b = 1 - 2q; q >= 1/2: a = 1/(2q), c = (2q - 1)/(2q);
        // q < 1/2 with no fluid node behind the link: half-way (b = c = 0)
        double* co = &pl.bzc[(k * pl.Q + i) * 2];
        if (q < 0.5 && fluid_at(y + lat_c(pl.Q, i, 1), z + lat_c(pl.Q, i, 2))) {
          co[0] = 1.0 - 2.0 * q;
          co[1] = 0.0;
        } else if (q < 0.5) {
          co[0] = 0.0;
          co[1] = 0.0;
        } else {
          co[0] = 0.0;
          co[1] = (2.0 * q - 1.0) / (2.0 * q);
        }
      }
    }
  }
  if (pl.slots.empty()) {
    if (err) *err = "geometry has no fluid cell";
    return LBM_EINVAL;
  }
  pl.nfluid = (int64_t)pl.slots.size() * pl.nx;
  pl.nwall = nwc * pl.nx;
  if (pl.masked) {
    // classify the points of the (x, y) plane; 2-D wall nodes in increasing
    // x + nx y, so that node (k, z) of the 3-D numbering is z nw2d + k
    const int nx = p->nx, ny = p->ny;
    auto solid_at = [&](int x, int y) {
      if (y < 0 || y >= ny) return true;
      x = ((x % nx) + nx) % nx;
      return pl.solid[x + (int64_t)nx * y] != 0;
    };
    pl.cellw.assign((size_t)nx * ny, lbm::kCellSolid);
    pl.pstride = (pl.Q + 3) / 4 * 4;  // whole 32-bit words per node
    pl.ptab.clear();
    pl.w2d.clear();
    int64_t nf2 = 0;
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        if (solid_at(x, y)) continue;
        nf2++;
        bool from_solid[19] = {};
        bool wall = false;
        for (int i = 1; i < pl.Q; i++) {
          from_solid[i] = solid_at(x - lat_c(pl.Q, i, 0), y - lat_c(pl.Q, i, 1));
          wall = wall || from_solid[i];
        }
        if (!wall) {
          pl.cellw[x + (int64_t)nx * y] = lbm::kCellInterior;
          continue;
        }
        int partner[19];
        slip_partners(pl.Q, from_solid, partner);
        for (int i = 0; i < pl.pstride; i++) {
          if (i < pl.Q && from_solid[i] && partner[i] < 0) {
            if (err) *err = "internal: unpaired wall link";
            return LBM_EINVAL;
          }
          pl.ptab.push_back(i < pl.Q && from_solid[i] ? (uint8_t)lat_row(pl.Q, partner[i])
                                                      : lbm::kNoLink);
        }
        pl.cellw[x + (int64_t)nx * y] = (int32_t)pl.w2d.size();
        pl.w2d.push_back((int32_t)(x + nx * y));
      }
    pl.nw2d = (int64_t)pl.w2d.size();
    pl.nfluid = nf2 * pl.nz;
    pl.nwall = pl.nw2d * pl.nz;
    // columns whose row holds a wall node first, flagged (mask 1): only their
    // blocks classify points; every other column is wholly interior (a row
    // with both fluid and solid points has wall nodes)
    std::vector<char> wallrow(ny, 0);
    for (int32_t w : pl.w2d) wallrow[w / nx] = 1;
    std::vector<lbm::ColSlot> first, rest;
    for (lbm::ColSlot cs : pl.slots) {
      const int y = cs.col % ny;
      cs.mask = wallrow[y] ? 1u : 0u;
      (wallrow[y] ? first : rest).push_back(cs);
    }
    pl.nwallslots = (int64_t)first.size();
    pl.slots = first;
    pl.slots.insert(pl.slots.end(), rest.begin(), rest.end());
    // the points a wall row's columns compute, packed to the front of the
    // column's lanes (the waves past them have nothing to do and leave):
    // the non-solid x, then the padding lanes (x >= nx, computing cell
    // nx - 1 again) where that cell is fluid
    const int64_t rs = (int64_t)pl.nxp + 1;
    pl.rowx.assign((size_t)(ny * rs), 0);
    for (int y = 0; y < ny; y++) {
      if (!wallrow[y]) continue;
      int32_t* r = pl.rowx.data() + y * rs;  // r[0]: count, r[1..]: the points' x
      for (int x = 0; x < pl.nxp; x++) {
        const int xc = x < nx ? x : nx - 1;
        if (pl.cellw[xc + (int64_t)nx * y] == lbm::kCellSolid) continue;
        r[1 + r[0]] = x;
        r[0]++;
      }
    }
  }
  pl.bx = std::min((pl.nx + 63) / 64 * 64, 512);
  pl.segs = (pl.nx + pl.bx - 1) / pl.bx;
  pl.nblocks = (int64_t)pl.slots.size() * pl.segs;
  if (pl.nblocks >= ((int64_t)1 << 31)) {
    if (err) *err = "grid too large";
    return LBM_EINVAL;
  }

  // every load the step kernel issues must land on a fluid column of the box
  // (masked walls: on a fluid point, by the classification above)
  for (const lbm::ColSlot& cs : pl.slots) {
    if (pl.masked) break;
    const int col = cs.col;
    const int y = col % p->ny, z = col / p->ny;
    const ColInfo ci{cs.wallcol, cs.mask};
    for (int i = 0; i < pl.Q; i++) {
      const bool wall = ci.mask & (1u << i);
      if (!wall && !fluid_at(y - lat_c(pl.Q, i, 1), z - lat_c(pl.Q, i, 2))) {
        if (err) *err = "internal: fluid link to a solid column";
        return LBM_EINVAL;
      }
      const int zs = z - lat_c(pl.Q, i, 2);
      if (!wall && !(ci.mask & lbm::kWrapColumn) && (zs < 0 || zs >= p->nz)) {
        if (err) *err = "internal: unflagged periodic pull";
        return LBM_EINVAL;
      }
      if (wall && pl.bouz && pl.bzc[((int64_t)ci.wallcol * pl.Q + i) * 2] != 0.0 &&
          !fluid_at(y + lat_c(pl.Q, i, 1), z + lat_c(pl.Q, i, 2))) {
        if (err) *err = "internal: interpolation node is solid";
        return LBM_EINVAL;
      }
    }
  }

  if (p->geometry == LBM_SLAB || p->geometry == LBM_DUCT) {
    // electron shells: the solid columns next to the water, y = -1 and y = ny
    // (by z), then for a duct z = -1 and z = nz (by y); each couples to one
    // fluid column, whose wall column is recorded
    const int64_t nshell = 2LL * pl.nz + (p->geometry == LBM_DUCT ? 2LL * pl.ny : 0);
    pl.nsheet = nshell * pl.nx;
    pl.sheet_wc.assign((size_t)nshell, -1);
    for (int64_t sh = 0; sh < nshell; sh++) {
      int64_t col;
      if (sh < 2LL * pl.nz)
        col = (sh < pl.nz ? 0 : pl.ny - 1) + (int64_t)pl.ny * (sh % pl.nz);
      else {
        const int64_t t = sh - 2LL * pl.nz;
        col = t % pl.ny + (int64_t)pl.ny * (t < pl.ny ? 0 : pl.nz - 1);
      }
      pl.sheet_wc[(size_t)sh] = pl.colinfo[col].wallcol;
      if (pl.colinfo[col].wallcol < 0) {
        if (err) *err = "internal: wall row without wall links";
        return LBM_EINVAL;
      }
    }
  } else if (p->geometry == LBM_TUBE) {
    // electron shells: the solid columns with a fluid column next to them
    // along y or z (the transverse steps of the links that cross x), in
    // increasing column index; each records its fluid neighbours
    pl.shellof.assign(pl.ncolbox, -1);
    pl.sheet_wc.clear();
    int64_t nshell = 0;
    const int dy[4] = {-1, 1, 0, 0}, dz[4] = {0, 0, -1, 1};
    for (int z = 0; z < p->nz; z++)
      for (int y = 0; y < p->ny; y++) {
        if (fluid_at(y, z)) continue;
        int32_t nb[8];
        bool any = false;
        for (int d = 0; d < 4; d++) {
          const int yf = y + dy[d], zf = z + dz[d];
          nb[2 * d] = nb[2 * d + 1] = -1;
          if (!fluid_at(yf, zf)) continue;
          const int64_t cf = yf + (int64_t)p->ny * zf;
          if (pl.colinfo[cf].wallcol < 0) {
            if (err) *err = "internal: fluid column next to the wall without wall links";
            return LBM_EINVAL;
          }
          nb[2 * d] = (int32_t)cf;
          nb[2 * d + 1] = pl.colinfo[cf].wallcol;
          any = true;
        }
        if (!any) continue;
        pl.shellof[y + (int64_t)p->ny * z] = (int32_t)nshell++;
        pl.sheet_wc.insert(pl.sheet_wc.end(), nb, nb + 8);
      }
    pl.nsheet = nshell * pl.nx;
    // electron lines need every wall link that crosses x to pull from a
    // shell inside the box (a tube touching the box's edge has none there)
    for (const lbm::ColSlot& cs : pl.slots) {
      if (cs.wallcol < 0) continue;
      const int y = cs.col % p->ny, z = cs.col / p->ny;
      for (int i = 0; i < pl.Q; i++) {
        if (!(cs.mask & (1u << i)) || lat_c(pl.Q, i, 0) == 0) continue;
        const int ys = y - lat_c(pl.Q, i, 1), zs = z - lat_c(pl.Q, i, 2);
        if (ys < 0 || ys >= p->ny || zs < 0 || zs >= p->nz ||
            pl.shellof[ys + (int64_t)p->ny * zs] < 0)
          pl.shells_whole = false;
      }
    }
  }

  size_t off = 0;
  pl.pop_bytes = (size_t)pl.ncolbox * pl.sC * pl.ssize;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  pl.off_pop[0] = take(pl.pop_bytes);
  pl.off_pop[1] = take(pl.pop_bytes);
  pl.off_slots = take(pl.slots.size() * sizeof(lbm::ColSlot));
  pl.off_r = take((size_t)pl.nwall * pl.wsize);
  pl.off_bz = take(pl.bouz ? (size_t)nwc * pl.Q * 2 * pl.wsize : 0);
  pl.off_lambda = take((size_t)pl.nwall * sizeof(double));
  pl.off_raw = take((size_t)(pl.nwall + 1) * sizeof(double));
  pl.off_partials = take((size_t)pl.nblocks * 2 * sizeof(double));
  pl.off_out = take(8 * sizeof(double));
  pl.off_flag = take(4 * sizeof(int));
  pl.off_step = take(sizeof(int64_t));
  // electron lines: rows 0..2 electrons, 3..5 phonons; velocities u_e then u_p
  pl.off_e[0] = take((size_t)pl.nsheet * 6 * sizeof(double));
  pl.off_e[1] = take((size_t)pl.nsheet * 6 * sizeof(double));
  pl.off_ue = take((size_t)pl.nsheet * 2 * sizeof(double));
  pl.off_swc = take(pl.sheet_wc.size() * sizeof(int32_t));
  pl.off_shellof = take(pl.shellof.size() * sizeof(int32_t));
  pl.off_cellw = take(pl.cellw.size() * sizeof(int32_t));
  pl.off_rowx = take(pl.rowx.size() * sizeof(int32_t));
  // open ends: per population buffer, [side][column][4] records of the end nodes
  pl.off_bmom = take((size_t)2 * 2 * pl.ncolbox * 4 * sizeof(double));
  pl.off_ptab = take(pl.ptab.size());
  pl.total = off;
  return LBM_OK;
}

}  // namespace

namespace {

lbm_status upload(lbm_ctx* c, size_t off, const void* host, size_t bytes) {
  if (bytes == 0) return LBM_OK;
  HIPCHK(c, hipMemcpyAsync(c->arena + off, host, bytes, hipMemcpyHostToDevice, c->stream));
  return LBM_OK;
}

}  // namespace

lbm_status lbm_host::sync(lbm_ctx* c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipGetLastError());
  return LBM_OK;
}

namespace {

void fill_args(lbm_ctx* c) {
  const Plan& pl = c->pl;
  StepArgs& a = c->args;
  a.nx = pl.nx;
  a.nxp = pl.nxp;
  a.ny = pl.ny;
  a.nz = pl.nz;
  a.sI = pl.sI;
  a.sC = pl.sC;
  a.nactive = (int)pl.slots.size();
  a.nwallcols = pl.masked ? (int)pl.nwallslots : (int)pl.wallcols.size();
  a.rev = 0;
  a.bx = pl.bx;
  a.segs = pl.segs;
  a.slab = c->p.geometry == LBM_SLAB;
  a.slots = c->at<lbm::ColSlot>(pl.off_slots);
  a.rwall = c->at<void>(pl.off_r);
  a.bz = pl.bouz ? c->at<void>(pl.off_bz) : nullptr;
  a.rho0 = c->p.rho0;
  a.omega = 1.0 / c->p.tau;
  for (int i = 0; i < 3; i++) a.F[i] = c->p.force[i];
  a.rho0_f = (float)a.rho0;
  a.omega_f = (float)a.omega;
  for (int i = 0; i < 3; i++) a.F_f[i] = (float)a.F[i];
  a.utop = c->p.wall_velocity_top;
  a.dstep = nullptr;
  a.step_off = 0;
  a.seed = kSeed;
  a.th_amp = 0.0;
  a.th_mode = 0;
  a.th_seed = 0;
  for (int k = 0; k < 6; k++) a.th_fac[k] = 1.0;
  a.ue = nullptr;
  a.shellof = pl.shellof.empty() ? nullptr : c->at<int32_t>(pl.off_shellof);
  a.cellw = pl.masked ? c->at<int32_t>(pl.off_cellw) : nullptr;
  a.rowx = pl.masked ? c->at<int32_t>(pl.off_rowx) : nullptr;
  a.ptab = pl.masked ? c->at<uint8_t>(pl.off_ptab) : nullptr;
  a.nw2d = pl.nw2d;
  a.open = 0;
  a.drho_in = 0.0;
  a.drho_out = 0.0;
  a.bmom = nullptr;  // set per launch (open ends)
  a.bmom_out = nullptr;
  a.partials = nullptr;  // set for a checked step only
  // a state (both buffers) of twice the last-level cache or more goes out
  // with nontemporal stores
  a.ntstore = 2 * pl.pop_bytes >= ((size_t)512 << 20) ? 1 : 0;
  for (int i = 0; i < 19; i++)
    a.nboff[i] = i < pl.Q ? (int64_t)lat_row(pl.Q, i) * pl.sI - lat_c(pl.Q, i, 1) * pl.sC -
                                lat_c(pl.Q, i, 2) * (int64_t)pl.ny * pl.sC
                          : 0;
}

template <typename W>
std::vector<W> convert(const std::vector<double>& v) {
  return std::vector<W>(v.begin(), v.end());
}

lbm_status upload_wall_r(lbm_ctx* c, const double* lambda_dev, int64_t n) {
  int* flag = c->at<int>(c->pl.off_flag);
  HIPCHK(c, hipMemsetAsync(flag, 0, sizeof(int), c->stream));
  HIPCHK(c, lbm::launch_set_r(c->pl.prec, lambda_dev, n, c->at<void>(c->pl.off_r), flag, c->stream));
  int h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  lbm_status s = sync(c);
  if (s != LBM_OK) return s;
  if (h) return c->fail(LBM_EINVAL, "friction must be >= 0 (NaN rejected)");
  return LBM_OK;
}

}  // namespace

namespace {

double* bmom_buf(lbm_ctx* c, int b) { return lbm_host::end_records(c, b); }

}  // namespace

// Open ends: the step kernels leave the end-node records of the buffer they
// write; after the state was set from outside, rebuild them for the current
// buffer once.
lbm_status lbm_host::ensure_end_records(lbm_ctx* c) {
  if (c->bmom_ok) return LBM_OK;
  HIPCHK(c, lbm::launch_open_moments(c->pl.Q, c->pl.prec, c->pop[c->cur], c->args,
                                     bmom_buf(c, c->cur), c->stream));
  c->bmom_ok = true;
  return LBM_OK;
}

lbm_status lbm_host::launch_one_step(lbm_ctx* c, bool check) {
  StepArgs a = c->args;
  a.step_off = c->step;  // plain launch: the step travels as an argument
  a.rev = c->cur;
  if (check) {  // the step also leaves the invariants' partials of its input state
    a.partials = c->at<double>(c->pl.off_partials);
    HIPCHK(c, lbm::launch_step_checked(c->pl.Q, c->pl.prec, c->pop[c->cur], c->pop[1 - c->cur], a,
                                       c->pl.bouz, c->stream));
    c->cur = 1 - c->cur;
    c->step++;
    return LBM_OK;
  }
  a = step_args(c);
  a.step_off = c->step;
  a.rev = c->cur;
  if (c->elec)  // the electrons of step n first: the water step reads their velocity
    HIPCHK(c, lbm::launch_electron_step(c->pl.Q, c->pl.prec, c->pop[c->cur],
                                        c->at<double>(c->pl.off_e[c->cur]),
                                        c->at<double>(c->pl.off_e[1 - c->cur]),
                                        c->at<double>(c->pl.off_ue), c->ea, c->stream));
  if (a.open) {  // the ghosts read the end-node records of the buffer the step reads
    lbm_status s = ensure_end_records(c);
    if (s != LBM_OK) return s;
    a.bmom = bmom_buf(c, c->cur);
    a.bmom_out = bmom_buf(c, 1 - c->cur);
  }
  HIPCHK(c, lbm::launch_step(c->pl.Q, c->pl.prec, c->pop[c->cur], c->pop[1 - c->cur], a,
                             c->pl.bouz, c->stream));
  c->cur = 1 - c->cur;
  c->step++;
  return LBM_OK;
}

namespace {

// A graph of kGraphSteps chained step kernels starting from buffer `parity`.
lbm_status build_graph(lbm_ctx* c, int parity) {
  hipGraph_t g = nullptr;
  HIPCHK(c, hipGraphCreate(&g, 0));
  const void* fn = lbm::step_kernel_ptr(c->pl.Q, c->pl.prec, c->pl.bouz, c->args.th_mode,
                                        c->elec, c->pl.masked, c->args.open != 0,
                                        c->args.ntstore != 0);
  const void* fe = c->elec ? lbm::electron_kernel_ptr(c->pl.Q, c->pl.prec) : nullptr;
  double* bm[2] = {bmom_buf(c, parity), bmom_buf(c, 1 - parity)};
  const double* esrc[2] = {c->at<double>(c->pl.off_e[parity]), c->at<double>(c->pl.off_e[1 - parity])};
  double* edst[2] = {c->at<double>(c->pl.off_e[1 - parity]), c->at<double>(c->pl.off_e[parity])};
  double* uep = c->at<double>(c->pl.off_ue);
  lbm::ElecArgs eargs = c->ea;
  hipGraphNode_t prev = nullptr;
  // kernel arguments must outlive instantiation only; keep them on the stack
  const void* srcs[2] = {c->pop[parity], c->pop[1 - parity]};
  void* dsts[2] = {c->pop[1 - parity], c->pop[parity]};
  // node k runs step (*d_step + k); a last node advances *d_step
  StepArgs args[kGraphSteps];
  int64_t* dstep = c->at<int64_t>(c->pl.off_step);
  const StepArgs base = step_args(c);
  for (int k = 0; k < kGraphSteps; k++) {
    args[k] = base;
    args[k].dstep = dstep;
    args[k].step_off = k;
    args[k].rev = (parity + k) & 1;
    if (fe) {  // the electron step of step k, before the water step that reads u_e
      void* eargv[5] = {(void*)&srcs[k & 1], (void*)&esrc[k & 1], (void*)&edst[k & 1], (void*)&uep,
                        (void*)&eargs};
      hipKernelNodeParams ep{};
      ep.func = const_cast<void*>(fe);
      ep.gridDim = dim3((unsigned)((c->pl.nsheet + 255) / 256));
      ep.blockDim = dim3(256);
      ep.kernelParams = eargv;
      hipGraphNode_t enode = nullptr;
      hipError_t e = hipGraphAddKernelNode(&enode, g, prev ? &prev : nullptr, prev ? 1 : 0, &ep);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return c->hip(e, "hipGraphAddKernelNode");
      }
      prev = enode;
    }
    if (args[k].open) {  // end-node records: read those of the source buffer
      args[k].bmom = bm[k & 1];
      args[k].bmom_out = bm[(k + 1) & 1];
    }
    void* kargs[3] = {(void*)&srcs[k & 1], (void*)&dsts[k & 1], (void*)&args[k]};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(fn);
    kp.gridDim = dim3((unsigned)c->pl.slots.size(), (unsigned)base.segs);
    kp.blockDim = dim3(base.bx);
    kp.sharedMemBytes = 0;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return c->hip(e, "hipGraphAddKernelNode");
    }
    prev = node;
  }
  {
    int64_t inc = kGraphSteps;
    void* kargs[2] = {(void*)&dstep, (void*)&inc};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(lbm::add_step_kernel_ptr());
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(64);
    kp.kernelParams = kargs;
    hipGraphNode_t node = nullptr;
    hipError_t e = hipGraphAddKernelNode(&node, g, &prev, 1, &kp);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return c->hip(e, "hipGraphAddKernelNode");
    }
  }
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return c->hip(e, "hipGraphInstantiate");
  }
  c->graph[parity] = g;
  c->gexec[parity] = ex;
  return LBM_OK;
}

lbm_status do_steps(lbm_ctx* c, int64_t n) {
  while (n >= kGraphSteps && c->graphs_ok) {
    if (!c->gexec[c->cur]) {
      lbm_status s = build_graph(c, c->cur);
      if (s != LBM_OK) {
        c->graphs_ok = false;  // fall back to plain launches
        c->err.clear();
        (void)hipGetLastError();
        break;
      }
    }
    if (c->dstep_value != c->step) {
      HIPCHK(c, lbm::launch_set_step(c->at<int64_t>(c->pl.off_step), c->step, c->stream));
      c->dstep_value = c->step;
    }
    if (c->args.open) {
      lbm_status s = ensure_end_records(c);
      if (s != LBM_OK) return s;
    }
    HIPCHK(c, hipGraphLaunch(c->gexec[c->cur], c->stream));
    c->step += kGraphSteps;  // even count: buffer parity unchanged
    c->dstep_value += kGraphSteps;
    n -= kGraphSteps;
  }
  for (; n > 0; n--) {
    lbm_status s = launch_one_step(c);
    if (s != LBM_OK) return s;
  }
  return LBM_OK;
}

// the fixed-order reduction of the per-block partials in the arena; the
// device out slot (and with to_host the context's pinned host buffer) then
// holds (sums, flux, mass, mass deviation)
lbm_status launch_reduce(lbm_ctx* c, bool to_host = false) {
  HIPCHK(c, lbm::launch_reduce_final(c->at<double>(c->pl.off_partials), c->pl.nblocks,
                                     c->at<double>(c->pl.off_out), c->pl.nx,
                                     (double)c->pl.nfluid * c->p.rho0, c->stream,
                                     to_host ? c->fin_host_dev : nullptr));
  return LBM_OK;
}

// The per-block partials in the arena -> (flux, mass, mass deviation):
// fixed-order reduction, synchronise; the reduce kernel writes the result
// straight into pinned host memory (else it is copied from the device).
lbm_status reduce_partials(lbm_ctx* c, double out[3]) {
  lbm_status s = launch_reduce(c, c->fin_host != nullptr);
  if (s != LBM_OK) return s;
  if (c->fin_host) {
    if ((s = sync(c)) != LBM_OK) return s;
    std::copy(c->fin_host + 2, c->fin_host + 5, out);
  } else {
    HIPCHK(c, hipMemcpyAsync(out, c->at<double>(c->pl.off_out) + 2, 3 * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    if ((s = sync(c)) != LBM_OK) return s;
  }
  if (!std::isfinite(out[0]) || !std::isfinite(out[1]))
    return c->fail(LBM_EDIVERGED, "flux or mass is not finite");
  return LBM_OK;
}

// the moments of the current state into the per-block partials (asynchronous)
lbm_status moments_partials(lbm_ctx* c) {
  HIPCHK(c, lbm::launch_moments(c->pl.Q, c->pl.prec, c->pop[c->cur], c->args, c->pl.bouz, -1,
                                nullptr, c->at<double>(c->pl.off_partials), c->stream));
  return LBM_OK;
}

lbm_status invariants(lbm_ctx* c, double out[3]) {
  c->checked_step = -1;  // the partials are about to hold the current state's
  lbm_status s = moments_partials(c);
  if (s != LBM_OK) return s;
  return reduce_partials(c, out);
}

// nsteps >= 1 steps; the partials are left holding the invariants of the
// state before the last step (fused into that step where the step kernel
// can: planar or tube walls without noise, sheets, mask or open ends).
lbm_status steps_checked(lbm_ctx* c, int64_t nsteps) {
  lbm_status s = do_steps(c, nsteps - 1);
  if (s != LBM_OK) return s;
  c->checked_step = -1;
  const bool fused = !c->elec && !c->args.open && !c->pl.masked && c->args.th_mode == 0;
  if (!fused && (s = moments_partials(c)) != LBM_OK) return s;
  if ((s = launch_one_step(c, fused)) != LBM_OK) return s;
  c->checked_step = c->step - 1;
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_footprint(const lbm_params* p, size_t* bytes) {
  if (!bytes) return LBM_EINVAL;
  Plan pl;
  lbm_status s = make_plan(p, &pl, nullptr);
  if (s != LBM_OK) return s;
  *bytes = pl.total;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_params* p, void* arena, size_t arena_bytes, void* hip_stream,
                      lbm_ctx** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ENOMEM;
  lbm_status s = make_plan(p, &c->pl, &c->err);
  if (s != LBM_OK) {
    delete c;
    return s;
  }
  if (!arena || (reinterpret_cast<uintptr_t>(arena) % kAlign) != 0) {
    delete c;
    return LBM_EINVAL;
  }
  if (arena_bytes < c->pl.total) {
    delete c;
    return LBM_ENOMEM;
  }
  c->p = *p;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->arena = static_cast<char*>(arena);
  c->pop[0] = c->arena + c->pl.off_pop[0];
  c->pop[1] = c->arena + c->pl.off_pop[1];
  fill_args(c);
  const Plan& pl = c->pl;
  lbm_status st = LBM_OK;
  do {
    if ((st = c->hip(hipMemsetAsync(c->arena, 0, pl.total, c->stream), "hipMemsetAsync")) != LBM_OK) break;
    if ((st = upload(c, pl.off_slots, pl.slots.data(), pl.slots.size() * sizeof(lbm::ColSlot))) != LBM_OK) break;
    if (!pl.sheet_wc.empty() &&
        (st = upload(c, pl.off_swc, pl.sheet_wc.data(), pl.sheet_wc.size() * sizeof(int32_t))) != LBM_OK)
      break;
    if (!pl.shellof.empty() &&
        (st = upload(c, pl.off_shellof, pl.shellof.data(), pl.shellof.size() * sizeof(int32_t))) != LBM_OK)
      break;
    if (pl.masked &&
        ((st = upload(c, pl.off_cellw, pl.cellw.data(), pl.cellw.size() * sizeof(int32_t))) != LBM_OK ||
         (st = upload(c, pl.off_rowx, pl.rowx.data(), pl.rowx.size() * sizeof(int32_t))) != LBM_OK ||
         (st = upload(c, pl.off_ptab, pl.ptab.data(), pl.ptab.size())) != LBM_OK))
      break;
    std::vector<double> inf(pl.nwall, INFINITY);
    std::vector<double> ones(pl.nwall, 1.0);
    if ((st = upload(c, pl.off_lambda, inf.data(), inf.size() * sizeof(double))) != LBM_OK) break;
    if (pl.wsize == 8) {
      if ((st = upload(c, pl.off_r, ones.data(), ones.size() * 8)) != LBM_OK) break;
      if (pl.bouz && (st = upload(c, pl.off_bz, pl.bzc.data(), pl.bzc.size() * 8)) != LBM_OK) break;
      if ((st = sync(c)) != LBM_OK) break;
    } else {
      std::vector<float> onesf = convert<float>(ones), bzf = convert<float>(pl.bzc);
      if ((st = upload(c, pl.off_r, onesf.data(), onesf.size() * 4)) != LBM_OK) break;
      if (pl.bouz && (st = upload(c, pl.off_bz, bzf.data(), bzf.size() * 4)) != LBM_OK) break;
      if ((st = sync(c)) != LBM_OK) break;
    }
  } while (0);
  if (st != LBM_OK) {
    lbm_destroy(c);
    return st;
  }
  // pinned host memory the reduce kernel writes its result to; without it
  // the result is copied from the device
  void* h = nullptr;
  if (hipHostMalloc(&h, 8 * sizeof(double), hipHostMallocDefault) == hipSuccess && h) {
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) == hipSuccess && d) {
      c->fin_host = static_cast<double*>(h);
      c->fin_host_dev = static_cast<double*>(d);
    } else {
      (void)hipHostFree(h);
    }
  }
  (void)hipGetLastError();
  *out = c;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->fin_host) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipHostFree(c->fin_host);
  }
  for (int k = 0; k < 2; k++) {
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
  }
  delete c;
}

lbm_status lbm_fluid_count(const lbm_ctx* c, size_t* n) {
  if (!c || !n) return LBM_EINVAL;
  *n = (size_t)c->pl.nfluid;
  return LBM_OK;
}

lbm_status lbm_wall_count(const lbm_ctx* c, size_t* n) {
  if (!c || !n) return LBM_EINVAL;
  *n = (size_t)c->pl.nwall;
  return LBM_OK;
}

lbm_status lbm_wall_coords(const lbm_ctx* c, int32_t* xyz) {
  if (!c || (!xyz && c->pl.nwall)) return LBM_EINVAL;
  const Plan& pl = c->pl;
  int64_t k = 0;
  if (pl.masked) {
    for (int z = 0; z < pl.nz; z++)
      for (int64_t w = 0; w < pl.nw2d; w++, k++) {
        xyz[3 * k] = pl.w2d[w] % pl.nx;
        xyz[3 * k + 1] = pl.w2d[w] / pl.nx;
        xyz[3 * k + 2] = z;
      }
    return LBM_OK;
  }
  for (size_t w = 0; w < pl.wallcols.size(); w++) {
    const int col = pl.wallcols[w];
    for (int x = 0; x < pl.nx; x++, k++) {
      xyz[3 * k] = x;
      xyz[3 * k + 1] = col % pl.ny;
      xyz[3 * k + 2] = col / pl.ny;
    }
  }
  return LBM_OK;
}

lbm_status lbm_wall_links(const lbm_ctx* c, double* links) {
  if (!c || (!links && c->pl.nwall)) return LBM_EINVAL;
  const Plan& pl = c->pl;
  int64_t k = 0;
  if (pl.masked) {  // half-way bounce-back on every wall link
    for (int z = 0; z < pl.nz; z++)
      for (int64_t w = 0; w < pl.nw2d; w++, k++)
        for (int i = 0; i < pl.Q; i++)
          links[k * pl.Q + i] = pl.ptab[w * pl.pstride + i] != lbm::kNoLink ? 0.5 : 0.0;
    return LBM_OK;
  }
  for (size_t w = 0; w < pl.wallcols.size(); w++)
    for (int x = 0; x < pl.nx; x++, k++)
      for (int i = 0; i < pl.Q; i++) links[k * pl.Q + i] = pl.linkq[w * pl.Q + i];
  return LBM_OK;
}

lbm_status lbm_set_friction(lbm_ctx* c, const double* lambda, size_t n, int on_device) {
  if (!c) return LBM_EINVAL;
  if (n != (size_t)c->pl.nwall) return c->fail(LBM_EINVAL, "expected %lld friction values", (long long)c->pl.nwall);
  if (n == 0) return LBM_OK;
  if (!lambda) return c->fail(LBM_EINVAL, "null friction array");
  std::vector<double> h;
  const double* src = lambda;
  if (on_device) {
    h.resize(n);
    HIPCHK(c, hipMemcpyAsync(h.data(), lambda, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    lbm_status s = sync(c);
    if (s != LBM_OK) return s;
    src = h.data();
  }
  for (size_t k = 0; k < n; k++)
    if (!(src[k] >= 0.0)) return c->fail(LBM_EINVAL, "friction[%zu] must be >= 0 (inf allowed)", k);
  double* dl = c->at<double>(c->pl.off_lambda);
  HIPCHK(c, hipMemcpyAsync(dl, lambda, n * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  c->have_raw = false;
  return upload_wall_r(c, dl, (int64_t)n);
}

lbm_status lbm_set_friction_spectral(lbm_ctx* c, const lbm_spectral* sp, const double* omega,
                                     size_t n, int on_device) {
  if (!c || !sp) return LBM_EINVAL;
  if (n != (size_t)c->pl.nwall) return c->fail(LBM_EINVAL, "expected %lld plasmon frequencies", (long long)c->pl.nwall);
  if (!spectral_valid(sp)) return c->fail(LBM_EINVAL, "bad spectral parameters");
  std::vector<double> h;
  const double* hsrc = omega;
  if (n && !omega) return c->fail(LBM_EINVAL, "null omega array");
  if (n && on_device) {
    h.resize(n);
    HIPCHK(c, hipMemcpyAsync(h.data(), omega, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    lbm_status s = sync(c);
    if (s != LBM_OK) return s;
    hsrc = h.data();
  }
  for (size_t k = 0; k < n; k++)
    if (!(hsrc[k] >= 0.0) || !std::isfinite(hsrc[k]))
      return c->fail(LBM_EINVAL, "omega[%zu] must be finite and >= 0", k);
  // the lambda buffer holds Omega until the quadrature has read it
  double* dl = c->at<double>(c->pl.off_lambda);
  double* draw = c->at<double>(c->pl.off_raw);
  if (n)
    HIPCHK(c, hipMemcpyAsync(dl, omega, n * sizeof(double),
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, lbm::launch_friction(spec_args(sp), dl, (int64_t)n, draw, dl, c->stream));
  c->have_raw = true;
  return upload_wall_r(c, dl, (int64_t)n);
}

lbm_status lbm_get_friction(lbm_ctx* c, double* lambda, double* raw) {
  if (!c) return LBM_EINVAL;
  const size_t n = (size_t)c->pl.nwall;
  if (lambda && n)
    HIPCHK(c, hipMemcpyAsync(lambda, c->at<double>(c->pl.off_lambda), n * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
  if (raw) {
    if (!c->have_raw) return c->fail(LBM_ESTATE, "no spectral friction has been set");
    HIPCHK(c, hipMemcpyAsync(raw, c->at<double>(c->pl.off_raw), (n + 1) * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
  }
  return sync(c);
}

lbm_status lbm_set_thermal(lbm_ctx* c, double kT, int mode, uint64_t seed) {
  if (!c) return LBM_EINVAL;
  if (!(kT >= 0.0) || std::isinf(kT)) return c->fail(LBM_EINVAL, "kT must be finite and >= 0");
  if (kT > 0.0 && mode != LBM_NOISE_STRESS && mode != LBM_NOISE_ALL)
    return c->fail(LBM_EINVAL, "noise form must be LBM_NOISE_STRESS or LBM_NOISE_ALL");
  // the step graphs hold the step arguments: finish queued work, rebuild later
  lbm_status s = sync(c);
  if (s != LBM_OK) return s;
  for (int k = 0; k < 2; k++) {
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->gexec[k] = nullptr;
    c->graph[k] = nullptr;
  }
  // every non-conserved direction relaxes by gamma = 1 - 1/tau per step; the
  // added variance mu (1 - gamma^2), mu = rho0 kT / c_s^2, holds it at mu w_i
  const double gam = 1.0 - 1.0 / c->p.tau;
  c->args.th_amp = kT > 0.0 ? std::sqrt(3.0 * c->p.rho0 * kT * (1.0 - gam * gam)) : 0.0;
  c->args.th_mode = kT > 0.0 ? mode : 0;
  c->args.th_seed = seed;
  c->kT = kT;
  return LBM_OK;
}

lbm_status lbm_set_noise_closure(lbm_ctx* c, const double* gamma, int nr, int ns,
                                 const double* wx, const double* wt) {
  if (!c) return LBM_EINVAL;
  double fac[6] = {1, 1, 1, 1, 1, 1};
  if (gamma) {
    if (nr < 1 || ns < 1 || !wx || !wt) return c->fail(LBM_EINVAL, "need nr, ns >= 1 and weights");
    for (int k = 0; k < 6; k++) {
      // the lag average of component k: sum_r sum_s W_x(r) W_t(s) Gamma_k(r, s)
      double m = 0.0;
      for (int r = 0; r < nr; r++)
        for (int t = 0; t < ns; t++) m += wx[r] * wt[t] * gamma[((int64_t)k * nr + r) * ns + t];
      if (!(m >= 0.0) || !std::isfinite(m))
        return c->fail(LBM_EINVAL, "closure factor %d is %g: must be finite and >= 0", k, m);
      fac[k] = std::sqrt(m);
    }
  }
  lbm_status s = sync(c);
  if (s != LBM_OK) return s;
  for (int k = 0; k < 2; k++) {  // the step graphs hold the step arguments
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->gexec[k] = nullptr;
    c->graph[k] = nullptr;
  }
  for (int k = 0; k < 6; k++) c->args.th_fac[k] = fac[k];
  return LBM_OK;
}

lbm_status lbm_set_open_ends(lbm_ctx* c, int open, double rho_in, double rho_out) {
  if (!c) return LBM_EINVAL;
  if (open) {
    if (c->p.geometry == LBM_MASKED) {
      // the wall continues past each end as that end's row of the mask; with
      // equal first and last rows it has the periodic channel's wall links
      const std::vector<unsigned char>& m = c->pl.solid;
      for (int y = 0; y < c->pl.ny; y++)
        if ((m[(size_t)c->pl.nx * y] != 0) != (m[(size_t)c->pl.nx * y + c->pl.nx - 1] != 0))
          return c->fail(LBM_EINVAL, "open ends on masked walls need equal first and last rows");
    }
    if (c->elec) return c->fail(LBM_EINVAL, "open ends need the electron sheets off");
    if (c->pl.nx < 2) return c->fail(LBM_EINVAL, "open ends need nx >= 2");
    if (!(rho_in > 0.0) || !(rho_out > 0.0) || !std::isfinite(rho_in) || !std::isfinite(rho_out))
      return c->fail(LBM_EINVAL, "densities must be finite and > 0");
  }
  lbm_status s = sync(c);
  if (s != LBM_OK) return s;
  for (int k = 0; k < 2; k++) {  // the step graphs hold the kernels and their arguments
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->gexec[k] = nullptr;
    c->graph[k] = nullptr;
  }
  c->args.open = open ? 1 : 0;
  c->args.drho_in = open ? rho_in - c->p.rho0 : 0.0;
  c->args.drho_out = open ? rho_out - c->p.rho0 : 0.0;
  c->bmom_ok = false;
  return LBM_OK;
}

lbm_status lbm_set_electrons(lbm_ctx* c, double tau_e, double rho_e0, double gamma_e,
                             double force_e) {
  if (!c) return LBM_EINVAL;
  const bool on = tau_e != 0.0;
  if (on) {
    if (c->p.geometry == LBM_MASKED || c->p.wall_velocity_top != 0.0)
      return c->fail(LBM_EINVAL, "electron sheets need a SLAB, DUCT or TUBE without a moving wall");
    if (c->pl.nsheet <= 0 || !c->pl.shells_whole)
      return c->fail(LBM_EINVAL, "electron lines need solid columns around the wall inside the box");
    if (c->args.open) return c->fail(LBM_EINVAL, "electron sheets need periodic x ends");
    if (!(tau_e > 0.5) || !(rho_e0 > 0.0) || !(gamma_e >= 0.0) || !std::isfinite(tau_e) ||
        !std::isfinite(rho_e0) || !std::isfinite(gamma_e) || !std::isfinite(force_e))
      return c->fail(LBM_EINVAL, "need tau_e > 1/2, rho_e0 > 0, gamma_e >= 0, finite values");
  }
  lbm_status s = sync(c);
  if (s != LBM_OK) return s;
  for (int k = 0; k < 2; k++) {  // the step graphs hold the kernels and their arguments
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->gexec[k] = nullptr;
    c->graph[k] = nullptr;
  }
  c->elec = on;
  c->args.ue = on ? c->at<double>(c->pl.off_ue) : nullptr;
  if (!on) return LBM_OK;
  const Plan& pl = c->pl;
  lbm::ElecArgs& ea = c->ea;
  ea.nx = pl.nx;
  ea.ny = pl.ny;
  ea.nz = pl.nz;
  ea.sI = pl.sI;
  ea.sC = pl.sC;
  ea.nshell = (int)(pl.nsheet / pl.nx);
  ea.rwall = c->at<void>(pl.off_r);
  ea.swc = c->at<int32_t>(pl.off_swc);
  ea.tube = pl.bouz ? 1 : 0;
  ea.bz = pl.bouz ? c->at<void>(pl.off_bz) : nullptr;
  ea.rho0 = c->p.rho0;
  ea.omega_e = 1.0 / tau_e;
  ea.rho_e0 = rho_e0;
  ea.gamma_e = gamma_e;
  ea.force_e = force_e;
  ea.phon = 0;  // switching the electrons on resets them without phonons
  // electrons at rest
  for (int k = 0; k < 2; k++)
    HIPCHK(c, hipMemsetAsync(c->at<void>(pl.off_e[k]), 0, (size_t)pl.nsheet * 6 * sizeof(double),
                             c->stream));
  HIPCHK(c, hipMemsetAsync(c->at<void>(pl.off_ue), 0, (size_t)pl.nsheet * 2 * sizeof(double),
                           c->stream));
  return sync(c);
}

lbm_status lbm_shell_count(const lbm_ctx* c, size_t* n) {
  if (!c || !n) return LBM_EINVAL;
  *n = c->pl.nx > 0 ? (size_t)(c->pl.nsheet / c->pl.nx) : 0;
  return LBM_OK;
}

lbm_status lbm_set_phonons(lbm_ctx* c, double tau_p, double rho_p0, double gamma_pc,
                           double gamma_ep) {
  if (!c) return LBM_EINVAL;
  const bool on = tau_p != 0.0;
  if (on) {
    if (!c->elec) return c->fail(LBM_EINVAL, "phonon lines need the electron lines on");
    if (!(tau_p > 0.5) || !(rho_p0 > 0.0) || !(gamma_pc >= 0.0) || !(gamma_ep >= 0.0) ||
        !std::isfinite(tau_p) || !std::isfinite(rho_p0) || !std::isfinite(gamma_pc) ||
        !std::isfinite(gamma_ep))
      return c->fail(LBM_EINVAL, "need tau_p > 1/2, rho_p0 > 0, gamma_pc, gamma_ep >= 0, finite");
  }
  lbm_status s = sync(c);
  if (s != LBM_OK) return s;
  for (int k = 0; k < 2; k++) {  // the step graphs hold the electron arguments
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->gexec[k] = nullptr;
    c->graph[k] = nullptr;
  }
  lbm::ElecArgs& ea = c->ea;
  ea.phon = on ? 1 : 0;
  if (!on) return LBM_OK;
  ea.omega_p = 1.0 / tau_p;
  ea.rho_p0 = rho_p0;
  ea.gamma_pc = gamma_pc;
  ea.gamma_ep = gamma_ep;
  const Plan& pl = c->pl;
  for (int k = 0; k < 2; k++)  // phonons at rest
    HIPCHK(c, hipMemsetAsync(c->at<double>(pl.off_e[k]) + 3 * pl.nsheet, 0,
                             (size_t)pl.nsheet * 3 * sizeof(double), c->stream));
  HIPCHK(c, hipMemsetAsync(c->at<double>(pl.off_ue) + pl.nsheet, 0, (size_t)pl.nsheet * sizeof(double),
                           c->stream));
  return sync(c);
}

lbm_status lbm_get_phonons(lbm_ctx* c, double* up, double* pops) {
  if (!c) return LBM_EINVAL;
  if (!c->elec || !c->ea.phon) return c->fail(LBM_ESTATE, "phonon lines are off");
  const Plan& pl = c->pl;
  if (up)
    HIPCHK(c, hipMemcpyAsync(up, c->at<double>(pl.off_ue) + pl.nsheet,
                             (size_t)pl.nsheet * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (pops)
    HIPCHK(c, hipMemcpyAsync(pops, c->at<double>(pl.off_e[c->cur]) + 3 * pl.nsheet,
                             (size_t)pl.nsheet * 3 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
  return sync(c);
}

lbm_status lbm_get_electrons(lbm_ctx* c, double* ue, double* pops) {
  if (!c) return LBM_EINVAL;
  if (!c->elec) return c->fail(LBM_ESTATE, "electron sheets are off");
  const Plan& pl = c->pl;
  if (ue)
    HIPCHK(c, hipMemcpyAsync(ue, c->at<double>(pl.off_ue), (size_t)pl.nsheet * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
  if (pops)
    HIPCHK(c, hipMemcpyAsync(pops, c->at<double>(pl.off_e[c->cur]),
                             (size_t)pl.nsheet * 3 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
  return sync(c);
}

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps) {
  if (!c || nsteps < 0) return LBM_EINVAL;
  return do_steps(c, nsteps);
}

lbm_status lbm_run_to_steady(lbm_ctx* c, double rel_tol, int64_t check_every, int64_t max_steps,
                             int64_t* steps_taken) {
  if (!c || !(rel_tol > 0) || check_every < 1 || max_steps < 0) return LBM_EINVAL;
  if (steps_taken) *steps_taken = 0;
  double inv[3];
  lbm_status s = invariants(c, inv);
  if (s != LBM_OK) return s;
  double prev = inv[0];
  int64_t taken = 0;
  // each chunk's last step also reduces the flux of the state it reads, so a
  // check costs no extra pass over the populations: the flux compared is
  // that of the step before each chunk's end (check_every steps apart, the
  // first chunk's one step fewer from the starting state)
  while (taken < max_steps) {
    const int64_t k = std::min(check_every, max_steps - taken);
    if ((s = steps_checked(c, k)) != LBM_OK) return s;
    taken += k;
    if (steps_taken) *steps_taken = taken;
    if ((s = reduce_partials(c, inv)) != LBM_OK) return s;
    if (std::fabs(inv[0] - prev) < rel_tol * std::fabs(inv[0])) return LBM_OK;
    prev = inv[0];
  }
  return c->fail(LBM_ENOTCONV, "no steady state after %lld steps", (long long)taken);
}

lbm_status lbm_invariants_async(lbm_ctx* c, double* host_out) {
  if (!c || !host_out) return LBM_EINVAL;
  c->checked_step = -1;  // the partials are about to hold the current state's
  lbm_status s = moments_partials(c);
  if (s == LBM_OK) s = launch_reduce(c);
  if (s != LBM_OK) return s;
  HIPCHK(c, hipMemcpyAsync(host_out, c->at<double>(c->pl.off_out) + 2, 3 * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  return LBM_OK;
}

}  // extern "C"

namespace {

void drop_step_graphs(lbm_ctx* c) {
  for (int k = 0; k < 2; k++) {
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->gexec[k] = nullptr;
    c->graph[k] = nullptr;
  }
}

// Block widths the step kernels may take: whole waves, at most 512 threads,
// no wider than the x-line (rounded up to a wave).
bool block_ok(const lbm_ctx* c, int bx) {
  return bx >= 64 && bx <= 512 && bx % 64 == 0 && bx <= (c->pl.nxp + 63) / 64 * 64;
}

// The autotuner's choices per kind of channel: lattice, storage, geometry,
// noise form, electron lines, open ends, and size bucket (log2 of nx and of
// the fluid columns).  Shared by every context of the process.
struct StepKey {
  int Q, prec, geom, th, elec, open, nx_log2, cols_log2;
  bool operator<(const StepKey& o) const {
    const int a[8] = {Q, prec, geom, th, elec, open, nx_log2, cols_log2};
    const int b[8] = {o.Q, o.prec, o.geom, o.th, o.elec, o.open, o.nx_log2, o.cols_log2};
    return std::lexicographical_compare(a, a + 8, b, b + 8);
  }
};
std::mutex g_step_mu;
std::map<StepKey, int> g_step_tune;

int log2i(int64_t v) {
  int r = 0;
  while (v > 1) {
    v >>= 1;
    r++;
  }
  return r;
}

// Time `reps` real steps (an even number, after two untimed ones, so the
// buffer parity comes back) with block width bx: the alternating column
// order and the cache contents between steps are those of a run.  The steps
// advance the state; the caller restores it from a checkpoint.
lbm_status time_step_kernel(lbm_ctx* c, int bx, int reps, hipEvent_t e0, hipEvent_t e1,
                            double* us) {
  const int saved = c->step_bx;
  c->step_bx = bx;
  lbm_status s = LBM_OK;
  for (int r = 0; r < reps + 2 && s == LBM_OK; r++) {
    if (r == 2 && hipEventRecord(e0, c->stream) != hipSuccess)
      s = c->fail(LBM_EDEVICE, "hipEventRecord failed");
    if (s == LBM_OK) s = launch_one_step(c);
  }
  c->step_bx = saved;
  if (s != LBM_OK) return s;
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipEventSynchronize(e1));
  float ms = 0;
  HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
  *us = 1e3 * ms / reps;
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_set_block(lbm_ctx* c, int bx) {
  if (!c) return LBM_EINVAL;
  if (bx != 0 && !block_ok(c, bx)) return c->fail(LBM_EINVAL, "block width %d not allowed", bx);
  lbm_status s = sync(c);
  if (s != LBM_OK) return s;
  if ((bx ? bx : c->pl.bx) != (c->step_bx ? c->step_bx : c->pl.bx)) drop_step_graphs(c);
  c->step_bx = bx;
  return LBM_OK;
}

lbm_status lbm_tune(lbm_ctx* c, int flags, int* bx_out, double* us_out) {
  if (!c) return LBM_EINVAL;
  const StepKey key{c->pl.Q, c->pl.prec, c->p.geometry, c->args.th_mode, c->elec ? 1 : 0,
                    c->args.open ? 1 : 0, log2i(c->pl.nx), log2i((int64_t)c->pl.slots.size())};
  int pick = 0;
  double best = 0.0;
  if (!(flags & LBM_TUNE_RETIME)) {
    std::lock_guard<std::mutex> lock(g_step_mu);
    auto it = g_step_tune.find(key);
    if (it != g_step_tune.end()) pick = it->second;
  }
  if (!pick || !block_ok(c, pick)) {
    // the candidates are timed over real steps from a host copy of the
    // checkpoint, which is put back afterwards (state, lines, step count)
    std::vector<char> ck;
    size_t nbytes = 0;
    (void)lbm_state_bytes(c, &nbytes);
    try {
      ck.resize(nbytes);
    } catch (const std::bad_alloc&) {
      return c->fail(LBM_ENOMEM, "no host memory for the tuner's checkpoint");
    }
    int64_t step0 = 0;
    const int cur0 = c->cur;
    const int64_t checked0 = c->checked_step;
    lbm_status s = lbm_get_state(c, ck.data(), ck.size(), &step0);
    if (s != LBM_OK) return s;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return c->fail(LBM_EDEVICE, "hipEventCreate failed");
    }
    // the plan's width is timed first and kept unless another is faster by
    // more than kTuneMargin (run-to-run spread of twenty steps is ~0.5 %)
    constexpr double kTuneMargin = 0.01;
    constexpr int kTuneSteps = 20;
    pick = c->pl.bx;
    if ((s = time_step_kernel(c, pick, kTuneSteps, e0, e1, &best)) == LBM_OK) {
      const double keep = best * (1.0 - kTuneMargin);
      for (int bx : {64, 128, 256, 512}) {
        if (bx == c->pl.bx || !block_ok(c, bx)) continue;
        double us = 0;
        if ((s = time_step_kernel(c, bx, kTuneSteps, e0, e1, &us)) != LBM_OK) break;
        if (us < keep && us < best) {
          best = us;
          pick = bx;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != LBM_OK) return s;
    c->cur = cur0;  // every candidate took an even number of steps
    if ((s = lbm_set_state(c, ck.data(), ck.size(), step0)) != LBM_OK) return s;
    c->checked_step = checked0;  // plain steps leave the partials alone
    std::lock_guard<std::mutex> lock(g_step_mu);
    g_step_tune[key] = pick;
  }
  lbm_status s = lbm_set_block(c, pick == c->pl.bx ? 0 : pick);
  if (s != LBM_OK) return s;
  if (bx_out) *bx_out = pick;
  if (us_out) *us_out = best;
  return LBM_OK;
}

lbm_status lbm_step_checked(lbm_ctx* c, int64_t nsteps) {
  if (!c || nsteps < 1) return LBM_EINVAL;
  return steps_checked(c, nsteps);
}

lbm_status lbm_checked_invariants(lbm_ctx* c, double out[3], int64_t* at_step) {
  if (!c || !out) return LBM_EINVAL;
  if (c->checked_step < 0) return c->fail(LBM_ESTATE, "no checked step since the last reduction");
  const int64_t at = c->checked_step;
  lbm_status s = reduce_partials(c, out);
  if (s == LBM_OK && at_step) *at_step = at;
  return s;
}

lbm_status lbm_invariants(lbm_ctx* c, double out[3]) {
  if (!c || !out) return LBM_EINVAL;
  return invariants(c, out);
}

lbm_status lbm_flux(lbm_ctx* c, double* q) {
  if (!c || !q) return LBM_EINVAL;
  double inv[3];
  lbm_status s = invariants(c, inv);
  if (s == LBM_OK) *q = inv[0];
  return s;
}

lbm_status lbm_mass(lbm_ctx* c, double* m) {
  if (!c || !m) return LBM_EINVAL;
  double inv[3];
  lbm_status s = invariants(c, inv);
  if (s == LBM_OK) *m = inv[1];
  return s;
}

lbm_status lbm_get_field(lbm_ctx* c, int which, double* host_out) {
  if (!c || !host_out || which < 0 || which > 3) return LBM_EINVAL;
  // the buffer the next step overwrites serves as scratch (>= 8 B per cell)
  double* scratch = static_cast<double*>(c->pop[1 - c->cur]);
  const size_t bytes = (size_t)c->pl.ncolbox * c->pl.nx * sizeof(double);
  HIPCHK(c, hipMemsetAsync(scratch, 0, bytes, c->stream));
  c->checked_step = -1;  // the moments kernel writes the partials too
  HIPCHK(c, lbm::launch_moments(c->pl.Q, c->pl.prec, c->pop[c->cur], c->args, c->pl.bouz, which,
                                scratch, c->at<double>(c->pl.off_partials), c->stream));
  HIPCHK(c, hipMemcpyAsync(host_out, scratch, bytes, hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

lbm_status lbm_get_populations(lbm_ctx* c, double* host_out) {
  if (!c || !host_out) return LBM_EINVAL;
  const Plan& pl = c->pl;
  std::vector<unsigned char> raw(pl.pop_bytes);
  HIPCHK(c, hipMemcpyAsync(raw.data(), c->pop[c->cur], pl.pop_bytes, hipMemcpyDeviceToHost, c->stream));
  lbm_status s = sync(c);
  if (s != LBM_OK) return s;
  for (int i = 0; i < pl.Q; i++)
    for (int64_t col = 0; col < pl.ncolbox; col++) {
      const bool solid = pl.colinfo[col].mask & lbm::kSolidColumn;
      const int y = (int)(col % pl.ny);
      for (int x = 0; x < pl.nx; x++) {
        const int64_t src = col * pl.sC + lat_row(pl.Q, i) * pl.sI + x;
        double v = 0.0;
        if (!solid && !(pl.masked && pl.solid[x + (int64_t)pl.nx * y])) {
          if (pl.prec == LBM_F64) v = reinterpret_cast<const double*>(raw.data())[src];
          else if (pl.prec == LBM_F32) v = reinterpret_cast<const float*>(raw.data())[src];
          else v = (double)(float)reinterpret_cast<const _Float16*>(raw.data())[src] / 4096.0;
        }
        host_out[((int64_t)i * pl.ncolbox + col) * pl.nx + x] = v;
      }
    }
  return LBM_OK;
}

lbm_status lbm_set_populations(lbm_ctx* c, const double* host_in, int64_t step) {
  if (!c || !host_in || step < 0) return LBM_EINVAL;
  const Plan& pl = c->pl;
  // largest |g| each storage holds (half: scaled by 2^12 below 65504)
  const double vmax = pl.prec == LBM_F64 ? 1.7976931348623157e308
                      : pl.prec == LBM_F32 ? 3.4028234663852886e38 : 65504.0 / 4096.0;
  for (int i = 0; i < pl.Q; i++)
    for (int64_t col = 0; col < pl.ncolbox; col++) {
      if (pl.colinfo[col].mask & lbm::kSolidColumn) continue;
      for (int x = 0; x < pl.nx; x++) {
        if (pl.masked && pl.solid[x + (int64_t)pl.nx * (col % pl.ny)]) continue;
        const double v = host_in[((int64_t)i * pl.ncolbox + col) * pl.nx + x];
        if (!(std::fabs(v) <= vmax))
          return c->fail(LBM_EINVAL, "population %d at column %lld, x %d is %g: NaN or beyond "
                                     "the storage range", i, (long long)col, x, v);
      }
    }
  std::vector<unsigned char> raw(pl.pop_bytes, 0);
  for (int i = 0; i < pl.Q; i++)
    for (int64_t col = 0; col < pl.ncolbox; col++) {
      if (pl.colinfo[col].mask & lbm::kSolidColumn) continue;
      for (int x = 0; x < pl.nxp; x++) {
        // padding lanes take the value of cell nx - 1, as the step writes them
        const int xs = x < pl.nx ? x : pl.nx - 1;
        // solid points of masked walls hold zero (nothing reads them)
        const double v = pl.masked && pl.solid[xs + (int64_t)pl.nx * (col % pl.ny)]
                             ? 0.0
                             : host_in[((int64_t)i * pl.ncolbox + col) * pl.nx + xs];
        const int64_t dst = col * pl.sC + lat_row(pl.Q, i) * pl.sI + x;
        if (pl.prec == LBM_F64) reinterpret_cast<double*>(raw.data())[dst] = v;
        else if (pl.prec == LBM_F32) reinterpret_cast<float*>(raw.data())[dst] = (float)v;
        else reinterpret_cast<_Float16*>(raw.data())[dst] = (_Float16)(float)(v * 4096.0);
      }
    }
  HIPCHK(c, hipMemcpyAsync(c->pop[c->cur], raw.data(), pl.pop_bytes, hipMemcpyHostToDevice, c->stream));
  lbm_status s = sync(c);
  if (s == LBM_OK) c->step = step;
  c->bmom_ok = false;
  c->checked_step = -1;
  return s;
}

}  // extern "C"

namespace {

// The checkpoint: the water populations in storage precision, then, with
// electron lines on, their populations (electron and phonon rows of the
// current buffer) and the velocities of the last step, u_e then u_p.
size_t line_bytes(const lbm_ctx* c) {
  return c->elec ? (size_t)c->pl.nsheet * (6 + 2) * sizeof(double) : 0;
}
size_t state_bytes(const lbm_ctx* c) { return c->pl.pop_bytes + line_bytes(c); }

}  // namespace

extern "C" {

lbm_status lbm_state_bytes(const lbm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return LBM_EINVAL;
  *bytes = state_bytes(c);
  return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx* c, void* host_buf, size_t bytes, int64_t* step) {
  if (!c || !host_buf) return LBM_EINVAL;
  if (bytes != state_bytes(c))
    return c->fail(LBM_EINVAL, "state holds %zu bytes", state_bytes(c));
  char* h = static_cast<char*>(host_buf);
  const Plan& pl = c->pl;
  HIPCHK(c, hipMemcpyAsync(h, c->pop[c->cur], pl.pop_bytes, hipMemcpyDeviceToHost, c->stream));
  if (c->elec) {
    const size_t eb = (size_t)pl.nsheet * 6 * sizeof(double);
    HIPCHK(c, hipMemcpyAsync(h + pl.pop_bytes, c->at<double>(pl.off_e[c->cur]), eb,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(h + pl.pop_bytes + eb, c->at<double>(pl.off_ue),
                             (size_t)pl.nsheet * 2 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
  }
  lbm_status s = sync(c);
  if (s == LBM_OK && step) *step = c->step;
  return s;
}

lbm_status lbm_set_state(lbm_ctx* c, const void* host_buf, size_t bytes, int64_t step) {
  if (!c || !host_buf || step < 0) return LBM_EINVAL;
  if (bytes != state_bytes(c))
    return c->fail(LBM_EINVAL, "state holds %zu bytes (electron lines %s)", state_bytes(c),
                   c->elec ? "on" : "off");
  const char* h = static_cast<const char*>(host_buf);
  const Plan& pl = c->pl;
  HIPCHK(c, hipMemcpyAsync(c->pop[c->cur], h, pl.pop_bytes, hipMemcpyHostToDevice, c->stream));
  if (c->elec) {
    const size_t eb = (size_t)pl.nsheet * 6 * sizeof(double);
    HIPCHK(c, hipMemcpyAsync(c->at<double>(pl.off_e[c->cur]), h + pl.pop_bytes, eb,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->at<double>(pl.off_ue), h + pl.pop_bytes + eb,
                             (size_t)pl.nsheet * 2 * sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
  }
  lbm_status s = sync(c);
  if (s == LBM_OK) c->step = step;
  c->bmom_ok = false;
  c->checked_step = -1;
  return s;
}

lbm_status lbm_step_count(const lbm_ctx* c, int64_t* step) {
  if (!c || !step) return LBM_EINVAL;
  *step = c->step;
  return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  return sync(c);
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : "null context"; }

lbm_status lbm_transfer_state(lbm_ctx* dst, lbm_ctx* src) {
  if (!dst || !src || dst == src) return LBM_EINVAL;
  const lbm_params &a = dst->p, &b = src->p;
  if (a.lattice != b.lattice || a.geometry != b.geometry || a.nx != b.nx || a.ny != b.ny ||
      a.nz != b.nz || a.tube_radius != b.tube_radius || a.tube_cy != b.tube_cy ||
      a.tube_cz != b.tube_cz)
    return dst->fail(LBM_EINVAL, "transfer needs the same lattice and geometry");
  if (dst->pl.masked && dst->pl.solid != src->pl.solid)
    return dst->fail(LBM_EINVAL, "transfer needs the same solid mask");
  lbm_status s = sync(src);
  if (s != LBM_OK) return s;
  const Plan &pd = dst->pl, &ps = src->pl;
  HIPCHK(dst, lbm::launch_convert(ps.prec, src->pop[src->cur], ps.nxp, pd.prec, dst->pop[dst->cur],
                                  pd.nxp, ps.ncolbox * ps.Q, ps.nx, dst->stream));
  const size_t nw = (size_t)pd.nwall;
  if (nw) {
    HIPCHK(dst, hipMemcpyAsync(dst->at<double>(pd.off_lambda), src->at<double>(ps.off_lambda),
                               nw * sizeof(double), hipMemcpyDeviceToDevice, dst->stream));
    HIPCHK(dst, hipMemcpyAsync(dst->at<double>(pd.off_raw), src->at<double>(ps.off_raw),
                               (nw + 1) * sizeof(double), hipMemcpyDeviceToDevice, dst->stream));
  }
  dst->have_raw = src->have_raw;
  dst->step = src->step;
  dst->bmom_ok = false;
  dst->checked_step = -1;
  s = upload_wall_r(dst, dst->at<double>(pd.off_lambda), (int64_t)nw);
  return s;
}

lbm_status lbm_copy_probe(const void* src, void* dst, size_t bytes, void* hip_stream) {
  if (!src || !dst || bytes == 0 || bytes % 16 ||
      (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
    return LBM_EINVAL;
  return lbm::launch_copy(src, dst, (int64_t)bytes, reinterpret_cast<hipStream_t>(hip_stream)) ==
                 hipSuccess
             ? LBM_OK
             : LBM_EDEVICE;
}

}  // extern "C"

// lbm_device.h -- device-side building blocks of the stream-collide update.
//
// Lattice tables, the pull gather with the Navier-slip wall rule, and the
// BGK + Guo collision, shared by the step kernel, the moments kernel and the
// batched kernel.  Follows the paper's LB procedure (Sec. 4: one population
// set for the water, local equilibria, forcing as a source; Sec. 4.2: the
// boundary rules at liquid/solid sites, periodic inlet/outlet).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

// ------------------------------------------------------------------ lattices
// D2Q9 in the paper's numbering (Sec. 4.2, beside Eqs. 19-21).
struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  // transverse reversal (c_x, -c_y)
  static constexpr int sig[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};
  static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  // storage row of direction i within a column (see the layout note below)
  static constexpr int row[9] = {0, 1, 3, 2, 6, 4, 5, 7, 8};
};

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  // transverse reversal (c_x, -c_y, -c_z)
  static constexpr int sig[19] = {0, 1, 2, 4, 3, 6, 5, 9, 10, 7, 8, 13, 14, 11, 12, 16, 15, 18, 17};
  static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                   1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  // storage row of direction i within a column (see the layout note below)
  static constexpr int row[19] = {8, 9, 10, 11, 5, 15, 1, 12, 6, 7, 13, 16, 2, 3, 17, 18, 0, 4, 14};
};

// ------------------------------------------------------------------ layout
// Populations live in a dense box of "columns" (y, z), col = y + ny z.  A
// column holds its Q x-lines back to back, each nxp elements long:
// g[col][row(i)][x] (address col * sC + row(i) * sI + x, sI = nxp,
// sC = Q nxp), so the block that updates a column writes one contiguous
// Q * nxp run.  The rows are ordered by the column that pulls them: the
// x-lines with the same (c_y, c_z) are adjacent, so one destination column
// reads them as one contiguous run and, when x-lines are not padded to whole
// cache lines, the lines they share are fetched once.  The runs themselves
// go by destination, z-1 before z before z+1 and within each y-1, y, y+1
// (D3Q19: 16, {6,12,13}, 17, {4,8,9}, {0,1,2}, {3,7,10}, 18, {5,11,14}, 15;
// D2Q9: {0,1,3}, {2,5,6}, {4,7,8}): a cache line that two runs share is
// then mostly wanted by two destinations next to each other in y, which
// the same workgroup (or the next) updates, so the line is used whole while
// it is in that L2.  Every geometry here is x-invariant: a column is
// entirely fluid or entirely solid and its wall links are the same for
// every x.

constexpr uint32_t kSolidColumn = 0x80000000u;
// a fluid column whose pulls wrap around the periodic z boundary (slab)
constexpr uint32_t kWrapColumn = 0x40000000u;
constexpr uint32_t kLinkBits = 0x000fffffu;
// masked walls: cell classes of the (x, y) plane (>= 0: 2-D wall-node index)
// and the partner-table entry of a link whose upstream point is fluid
constexpr int32_t kCellInterior = -1;
constexpr int32_t kCellSolid = -2;
constexpr uint8_t kNoLink = 0xff;

struct ColInfo {
  int32_t wallcol;  // index among wall columns, -1 for columns without wall links
  uint32_t mask;    // bit i: link i pulls from a solid point; kWrapColumn; kSolidColumn
};

// One fluid column as the kernels see it: everything a wave needs about its
// column in one 16-byte record (one scalar load, no dependent lookups).
struct ColSlot {
  int32_t col;
  int32_t wallcol;
  uint32_t mask;
  int32_t pad;
};

struct StepArgs {
  int nx, nxp, ny, nz;
  int64_t sI;         // elements between the x-lines of two directions (nxp)
  int64_t sC;         // elements between two columns (Q nxp)
  int nactive;        // number of fluid columns
  int nwallcols;      // the first nwallcols of them have wall links
  int rev;            // visit the other columns in reverse order (see k_step)
  int bx;             // threads per block along x
  int segs;           // blocks per column = ceil(nx / bx)
  int slab;           // z periodic
  const ColSlot* slots;     // fluid columns, wall columns first
  const void* rwall;        // [wallcol][nx] wall mixing weight r (arithmetic type)
  const void* bz;           // [wallcol][Q][2] interpolated bounce-back coefs (b, c) or null
  double rho0, omega;       // omega = 1/tau
  double F[3];
  double utop;              // moving top wall speed (0: none)
  // time step of this launch, for the stochastic-rounding bits:
  // (dstep ? *dstep : 0) + step_off
  const int64_t* dstep;
  int64_t step_off;
  uint32_t seed;
  // thermal fluctuations (see thermal_noise): amplitude A (0: none), form
  // (1: stress source, 2: every non-conserved direction), random-number key
  double th_amp;
  int th_mode;
  uint64_t th_seed;
  // one-point closure of the quantum noise (form 1): factors on the random
  // stress components xx, yy, zz, xy, xz, yz (1: classical)
  double th_fac[6];
  // electron shells: x velocity of each shell node in the step being taken,
  // [shell][x]; slab and duct: shells y = -1, y = ny (by z), then for a duct
  // z = -1, z = nz (by y); tube: shellof[y + ny z] is the shell of a solid
  // column (-1: none)
  const double* ue;
  const int32_t* shellof;
  // masked walls (walls that vary along x; null for the other geometries):
  // cellw[x + nx y] is the class of the point (kCellSolid, kCellInterior or
  // the 2-D wall-node index k), ptab[k Q + i] the storage row of the slip
  // partner of wall link i (kNoLink if the link pulls from a fluid point),
  // and the wall weight of node (k, z) is rwall[z nw2d + k]
  const int32_t* cellw;
  const uint8_t* ptab;
  int64_t nw2d;
  // open x ends (0: periodic): prescribed density deviations rho - rho0 of
  // the ghost planes x = -1 (inlet) and x = nx (outlet); records
  // (sum g, u_x, u_y, u_z) of the stored populations of the first and the
  // last node of every column, [side][column][4], of the buffer the step
  // reads (bmom) and of the one it writes (bmom_out)
  int open;
  double drho_in, drho_out;
  const double* bmom;
  double* bmom_out;
  // a checked step (the last step of a chunk of run-to-steady): per-block
  // FP64 sums (j_x, rho - rho0) of the populations the step's collision
  // sees, [slot * segs + segment][2]; null otherwise
  double* partials;
  // nonzero: the state is far larger than the last-level cache; the plain
  // step then stores with nontemporal stores (see store_pop)
  int ntstore;
  // element offset, from the start of a column, of the x-line of g_i in the
  // column the pull of link i reads: row(i) sI - c_iy sC - c_iz ny sC (no wrap)
  int64_t nboff[19];
  // rho0, omega and F rounded to float (the float arithmetic's parameters)
  float rho0_f, omega_f, F_f[3];
  // masked walls: per row y of the (x, y) plane that holds wall nodes, its
  // count of points to compute and their x, packed: rowx[y (nxp + 1)] is
  // the count, rowx[y (nxp + 1) + 1 + k] the k-th x (the non-solid points
  // in increasing x, then the padding lanes if the last point is fluid)
  const int32_t* rowx;
};

// ------------------------------------------------------------------ uniformity
// Values that are the same for every lane of a wave but were loaded through a
// pointer the compiler cannot prove uniform: move them to scalar registers so
// that everything derived from them (column, buffer, line bases) stays scalar.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ------------------------------------------------------------------ electron lines
// Electron shells (the solid columns next to the water, one line along x
// each, D1Q3): slab and duct y = -1 and y = ny (by z), then for a duct
// z = -1 and z = nz (by y); tube: the solid columns with a fluid column next
// to them along y or z, by increasing column index
struct ElecArgs {
  int nx, ny, nz, nshell;
  int64_t sI, sC;        // water layout
  const void* rwall;     // water wall weights r [wallcol][nx] (double, float for F16S)
  // slab and duct: [shell] the wall column of the fluid column next to the
  // shell; tube: [shell][8] (column, wall column) of the fluid columns at
  // -y, +y, -z, +z of the shell, -1 where solid
  const int32_t* swc;
  int tube;              // interpolated walls: bz holds their coefficients
  const void* bz;        // [wallcol][Q][2] (double, float for F16S)
  double rho0;           // water reference density
  double omega_e, rho_e0, gamma_e, force_e;
  // phonon lines beside the electron lines (rows 3..5 of the state, their
  // velocity after the electrons'): on/off, 1/tau_p, rho_p0, crystal drag,
  // electron-phonon drag coefficient
  int phon;
  double omega_p, rho_p0, gamma_pc, gamma_ep;
};

// ------------------------------------------------------------------ batches
// The members of a batch group whose electron lines one launch steps.
constexpr int kEGroupMax = 32;
struct EGroup {
  int n;
  int slot[kEGroupMax];
};

// One member of a batch: its step arguments, its two population buffers,
// its step and current buffer when the batch was built.  With k the steps
// the batch has taken since (one device counter for the whole batch), the
// member is at step base_step + k and its state is in pop[(cur_base + k) & 1].
struct MemberDesc {
  StepArgs a;
  const void* pop[2];
  double* bmom[2];  // open ends: the end-node records of pop[0] and pop[1]
  // electron lines: their arguments, populations beside pop[0] and pop[1]
  // (electron rows 0..2, phonon rows 3..5) and the velocities of the last
  // step (u_e, then u_p)
  ElecArgs ea;
  double* eline[2];
  double* uel;
  int64_t base_step;
  int32_t cur_base;
  int32_t pad;
};

// A batch work item: the 64 lanes of one wave over one member.  The wave
// covers cells xs .. xs+63 of the run of ncols columns whose ids are
// cols[cbase], cols[cbase+1], ... starting in the run's column c0; lanes
// past the end of a column continue in the next column of the run (runs of
// plain columns only), lanes past the run (or past nxp for a single column)
// are idle.  Items with member < 0 are empty.  wallcol and mask describe the
// column of single-column items (mask 0 for plain columns).
struct WorkItem {
  int32_t member, cbase, ncols, c0, xs;
  int32_t wallcol;
  uint32_t mask;
  int32_t pad;
};

// ------------------------------------------------------------------ storage
// Device arrays are addressed through global-address-space pointers (plain
// pointers read from a descriptor would be accessed with flat instructions),
// and every population access is (uniform line base) + (32-bit lane index).
// The byte offset is formed in 32-bit unsigned arithmetic so that the
// compiler can address with a scalar base and a 32-bit vector offset instead
// of one 64-bit vector address per access (x < nxp <= 2^24: no wrap).
#define LBM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const LBM_GLOBAL T* gbl(const T* p) {
  return (const LBM_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ LBM_GLOBAL T* gbl(T* p) {
  return (LBM_GLOBAL T*)p;
}
template <typename S>
__device__ __forceinline__ const LBM_GLOBAL S* at(const LBM_GLOBAL S* line, unsigned i) {
  return (const LBM_GLOBAL S*)((const LBM_GLOBAL char*)line + i * (unsigned)sizeof(S));
}
template <typename S>
__device__ __forceinline__ LBM_GLOBAL S* at(LBM_GLOBAL S* line, unsigned i) {
  return (LBM_GLOBAL S*)((LBM_GLOBAL char*)line + i * (unsigned)sizeof(S));
}
// A wave-uniform line pointer pinned to scalar registers: without it the
// compiler folds the lane offset into the base once and then forms every
// store address with 64-bit vector arithmetic.
template <typename T>
__device__ __forceinline__ LBM_GLOBAL T* sbase(LBM_GLOBAL T* p) {
  return (LBM_GLOBAL T*)uniform64((int64_t)(uintptr_t)p);
}
template <typename S, typename M>
__device__ __forceinline__ M ld(const LBM_GLOBAL S* line, unsigned i);  // defined after dec()
// ------------------------------------------------------------------ rounding
// Storage below the arithmetic precision is rounded stochastically: rounding
// to nearest stalls once the per-step change of a population falls below
// half a unit in the last place, and near steady state that bias is the
// same every step, so it accumulates over the slowest viscous time (measured
// 2e-5..7e-5 of the flux for float storage in a CPU emulation, 1e-7 with
// stochastic rounding).  The random bits are counter-based (a function of
// seed, step and cell only), so results are reproducible bit for bit.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// 16 random bits per population of one cell and step: the MurmurHash3
// finaliser of (seed, step, cell) seeds a Marsaglia xorshift32 stream, one
// 32-bit word per two populations (shifts and xors only), drawn as needed.
struct RoundBits {
  uint32_t x;
  __device__ __forceinline__ RoundBits(uint32_t seed, int64_t step, uint32_t cell)
      : x(fmix32(cell ^ fmix32(seed ^ fmix32((uint32_t)step ^ (uint32_t)(step >> 32)))) | 1u) {}
  // the next 32-bit word (xorshift32 must not start at zero: hence the | 1)
  __device__ __forceinline__ uint32_t next() {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
  }
};

// Half-precision deviations are stored scaled by 2^12 so that the values of
// interest (1e-8 .. 1e-2) sit in the normal half range.
constexpr float kHalfScale = 4096.0f;
constexpr float kHalfUnscale = 1.0f / 4096.0f;

// double -> float, stochastic: add 16 random bits at the top of the 29
// discarded mantissa bits and truncate (carries into the exponent are what
// the integer add does; exact for results in the normal float range)
__device__ __forceinline__ float sr_float(double v, uint32_t r16) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  b = (b + ((uint64_t)r16 << 13)) & ~((1ull << 29) - 1ull);
  return (float)__longlong_as_double((long long)b);
}
// float -> half, stochastic: gfx950's conversion with a stochastic-rounding
// operand adds the top 13 bits of r (bits 19..31) to the 13 discarded
// mantissa bits and truncates (checked bit for bit against that rule on
// random inputs over the normal half range; results in the subnormal half
// range are rounded stochastically at the subnormal spacing).  It writes
// one half of a register and keeps the other; the register of the value
// itself is passed as the kept one (no register has to be cleared first).
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ _Float16 sr_half(float s, uint32_t r) {
  return __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(half2_t, s), s, r, false)[0];
}

// Store<S, M>: kScale is the factor between a population and what is stored
// (2^12 for half storage); the collision forms its results already scaled
// (every scaled term is a power-of-two multiple of the unscaled one, so
// this is exact), and enc(v, bits) / enc2 (a pair from one random word)
// round the scaled values to the storage type.
template <typename S, typename M>
struct Store {  // same precision: plain store
  static constexpr bool kRandom = false;
  static constexpr float kScale = 1.0f;
  __device__ __forceinline__ static S enc(M v, uint32_t) { return static_cast<S>(v); }
  __device__ __forceinline__ static void enc2(M vi, M vo, uint32_t, S* ei, S* eo) {
    *ei = static_cast<S>(vi);
    *eo = static_cast<S>(vo);
  }
};
template <>
struct Store<float, double> {  // 16 bits each: the low and the high half of the word
  static constexpr bool kRandom = true;
  static constexpr float kScale = 1.0f;
  __device__ __forceinline__ static float enc(double v, uint32_t w) {
    return sr_float(v, w & 0xffffu);
  }
  __device__ __forceinline__ static void enc2(double vi, double vo, uint32_t w, float* ei,
                                              float* eo) {
    *ei = sr_float(vi, w & 0xffffu);
    *eo = sr_float(vo, w >> 16);
  }
};
template <>
struct Store<_Float16, float> {
  static constexpr bool kRandom = true;
  static constexpr float kScale = kHalfScale;
  __device__ __forceinline__ static _Float16 enc(float s, uint32_t w) { return sr_half(s, w); }
  // the word and the word rotated by 16: bits 19..31 and 3..15 of the
  // word; both results in the halves of one register
  __device__ __forceinline__ static void enc2(float si, float so, uint32_t w, _Float16* ei,
                                              _Float16* eo) {
    half2_t p = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(half2_t, si), si, w, false);
    p = __builtin_amdgcn_cvt_sr_f16_f32(p, so, __builtin_amdgcn_alignbit(w, w, 16), true);
    *ei = p[0];
    *eo = p[1];
  }
};
// a parameter in the arithmetic type: float arithmetic takes the float copy
template <typename M>
__device__ __forceinline__ M par(double d, float) {
  return static_cast<M>(d);
}
template <>
__device__ __forceinline__ float par<float>(double, float f) {
  return f;
}
template <typename S, typename M>
__device__ __forceinline__ M dec(S v) {
  return static_cast<M>(v);
}
// -0.0f in a register the compiler cannot see into (a constant -0 addend
// would be folded away, and with it the one-instruction decode below)
__device__ __forceinline__ float opaque_neg_zero() {
  float z;
  asm("v_mov_b32 %0, 0x80000000" : "=v"(z));
  return z;
}
// v * 2^-12 + (-0) is v * 2^-12 exactly (the product is exact and adding -0
// keeps every value, the sign of zero included); in this form the
// conversion and the scaling are one mixed-precision multiply-add
template <>
__device__ __forceinline__ float dec<_Float16, float>(_Float16 v) {
  return __builtin_fmaf(static_cast<float>(v), kHalfUnscale, opaque_neg_zero());
}
template <>
__device__ __forceinline__ double dec<_Float16, double>(_Float16 v) {
  return static_cast<double>(static_cast<float>(v) * kHalfUnscale);
}
template <typename S, typename M>
__device__ __forceinline__ M ld(const LBM_GLOBAL S* line, unsigned i) {
  return dec<S, M>(*at(line, i));
}

// element offset, from the start of column (y, z), of the x-line of g_i in
// the column the pull of link i reads (sZ = ny sC); with wrap, z is periodic
template <class L>
__device__ __forceinline__ int64_t src_off(const StepArgs& a, int i, int z, bool wrap) {
  int64_t off = a.nboff[i];
  if (L::cz[i] != 0 && wrap) {
    const int64_t sZ = (int64_t)a.ny * a.sC;
    const int zs = z - L::cz[i];
    if (zs < 0) off += (int64_t)a.nz * sZ;
    if (zs >= a.nz) off -= (int64_t)a.nz * sZ;
  }
  return off;
}

// Pull gather: df_i = g_i(x - c_i), periodic in x; a link whose upstream
// point is solid takes the wall rule
//   df_i = r BB_i + (1 - r) g_sig(i)(x),
// BB_i = g_opp(i)(x) (half-way) or the interpolated bounce-back
//   a g_opp(i)(x) + b g_opp(i)(x + c_i) + c g_i(x),  a + b + c = 1,
// and on a moving top wall BB_i = g_opp(i)(x) + 6 w_i rho0 c_ix U.
// Mixtures are evaluated as g + r (bb - g) and gb + b (gnb - gb) + c (gi - gb)
// so that their weights sum to one exactly in the working precision (a
// rounded 1 - r would multiply the wall populations by 1 + eps every step).
//
// dl (interior columns only) is added to every lane index: a lane working on
// column col + k takes the lines of column col shifted by dl = k sC, which is
// the same shift for every source column away from periodic wrap in z.
//
// With ELEC (walls with electron shells) the bounce-back half reflects off a
// wall moving with the electrons of the solid point x - c_i:
//   BB_i = g_opp(i)(x) + 6 w_i rho0 c_ix u_e(x - c_i)
// (a wall link with c_ix != 0 crosses a y wall or a z wall, never both); on
// a tube the term is scaled by 1 - cc (1 / 2q where the wall lies farther
// than half a link), so that a uniform flow at the wall's velocity stays
// exact.
//
// With OPEN (open x ends) the pulls of the first and last node that would
// wrap around x read the node itself instead (x - c_i clamped into the box):
// the ghost's own population g_i(b); open_correct adds the rest of the ghost.
template <class L, typename S, typename M, typename W, bool BOUZ, bool ELEC = false,
          bool OPEN = false>
__device__ __forceinline__ void gather(const S* __restrict__ g0, const StepArgs& a, int col,
                                       int x, ColInfo info, M* df, unsigned dl = 0u) {
  const LBM_GLOBAL S* g = gbl(g0);
  const int64_t sI = a.sI, sC = a.sC;
  const unsigned ux = (unsigned)x;
  const unsigned xm = (x == 0) ? (OPEN ? 0u : (unsigned)a.nx - 1u) : ux - 1u;
  const unsigned xp = (x == a.nx - 1) ? (OPEN ? ux : 0u) : ux + 1u;
  const uint32_t mask = info.mask;
  const LBM_GLOBAL S* gown = g + (int64_t)col * sC;
  if (mask == 0u) {
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
      const LBM_GLOBAL S* line = gown + a.nboff[i];  // uniform
      df[i] = ld<S, M>(sbase(line), dl + (L::cx[i] > 0 ? xm : (L::cx[i] < 0 ? xp : ux)));
    }
    return;
  }
  // Wall column: issue every load first (the mask is uniform over the block,
  // so these are uniform branches around loads only), then combine.
  //   pv[i]: the pulled value of a fluid link, or for an interpolated wall
  //          link the node behind it, g_opp(i)(x + c_i);
  //   ow[k]: this node's own g_k, for every k pointing into the wall (and
  //          for wall links that interpolate with g_i(x)).
  const int z = col / a.ny;
  const int y = col - z * a.ny;
  const LBM_GLOBAL W* cw =
      BOUZ ? gbl(static_cast<const W*>(a.bz)) + (int64_t)info.wallcol * L::Q * 2 : nullptr;
  S pv[L::Q], ow[L::Q];
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    const bool wall = mask & (1u << i);
    if (!wall) {
      const LBM_GLOBAL S* line = gown + src_off<L>(a, i, z, (mask & kWrapColumn) != 0u);
      pv[i] = *at(sbase(line), L::cx[i] > 0 ? xm : (L::cx[i] < 0 ? xp : ux));
    } else if (BOUZ && cw[2 * i] != W(0)) {
      const int nc = (y + L::cy[i]) + a.ny * (z + L::cz[i]);
      const LBM_GLOBAL S* line = g + (int64_t)nc * sC + L::row[L::opp[i]] * sI;
      pv[i] = *at(sbase(line), L::cx[i] > 0 ? xp : (L::cx[i] < 0 ? xm : ux));
    }
    if ((mask & (1u << L::opp[i])) || (BOUZ && wall && cw[2 * i + 1] != W(0)))
      ow[i] = *at(sbase(gown + L::row[i] * sI), ux);
  }
  if ((mask & kLinkBits) == 0u) {  // a wrapping column without wall links
#pragma unroll
    for (int i = 0; i < L::Q; i++) df[i] = dec<S, M>(pv[i]);
    return;
  }
  const M r = static_cast<M>(gbl(static_cast<const W*>(a.rwall))[(int64_t)info.wallcol * a.nx + x]);
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    if (!(mask & (1u << i))) {
      df[i] = dec<S, M>(pv[i]);
      continue;
    }
    const M gb = dec<S, M>(ow[L::opp[i]]);
    if (a.utop != 0.0 && L::cy[i] == -1 && y == a.ny - 1) {
      df[i] = gb + static_cast<M>(6.0 * L::w[i] * a.rho0 * L::cx[i] * a.utop);
      continue;
    }
    M bb = gb;
    if (ELEC && L::cx[i] != 0) {
      int64_t shell;
      if constexpr (BOUZ)  // a tube: the shell of the solid column the link pulls from
        shell = gbl(a.shellof)[(int64_t)(y - L::cy[i]) + (int64_t)a.ny * (z - L::cz[i])];
      else
        shell = L::cy[i] != 0 ? (int64_t)(L::cy[i] > 0 ? 0 : a.nz) + z
                              : 2LL * a.nz + (L::cz[i] > 0 ? 0 : a.ny) + y;
      const int64_t sn = shell * a.nx + (L::cx[i] > 0 ? xm : xp);
      M mv = static_cast<M>(6.0 * L::w[i] * a.rho0 * L::cx[i]) * static_cast<M>(gbl(a.ue)[sn]);
      // interpolated walls: where the wall lies farther than half a link the
      // moving wall's term is divided by 2q, i.e. scaled by 1 - cc
      if constexpr (BOUZ) mv *= M(1) - static_cast<M>(cw[2 * i + 1]);
      bb += mv;
    }
    if (BOUZ) {
      const M cb = static_cast<M>(cw[2 * i]), cc = static_cast<M>(cw[2 * i + 1]);
      if (cb != M(0)) bb += cb * (dec<S, M>(pv[i]) - gb);
      if (cc != M(0)) bb += cc * (dec<S, M>(ow[i]) - gb);
    }
    const M gs = dec<S, M>(ow[L::sig[i]]);
    df[i] = gs + r * (bb - gs);
  }
}

// Masked walls (walls that vary along x).  The class of each point of the
// (x, y) plane (cellw) is kCellSolid, kCellInterior or its 2-D wall-node
// index k; a wall node's partner table holds, per link i, the storage row of
// i's slip partner (kNoLink where the upstream point is fluid), padded to
// whole 32-bit words.
template <class L>
constexpr int ptab_words() {
  return (L::Q + 3) / 4;
}

// Pulls only: a column none of whose points is a wall node (all of them
// interior; the block's branch is uniform).  z is periodic.  OPEN: the pulls
// that would wrap around x read the node itself (as gather<OPEN>).
template <class L, typename S, typename M, bool OPEN = false>
__device__ __forceinline__ void gather_masked_interior(const S* __restrict__ g0, const StepArgs& a,
                                                       int col, int z, int x, M* df) {
  const LBM_GLOBAL S* gown = gbl(g0) + (int64_t)col * a.sC;
  const unsigned ux = (unsigned)x;
  const unsigned xm = (x == 0) ? (OPEN ? 0u : (unsigned)a.nx - 1u) : ux - 1u;
  const unsigned xp = (x == a.nx - 1) ? (OPEN ? ux : 0u) : ux + 1u;
  const bool wrap = L::Q == 19 && (z == 0 || z == a.nz - 1);
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    const LBM_GLOBAL S* line = gown + src_off<L>(a, i, z, wrap);
    df[i] = ld<S, M>(sbase(line), L::cx[i] > 0 ? xm : (L::cx[i] < 0 ? xp : ux));
  }
}

// Any non-solid point (cw >= 0: a wall node, kCellInterior otherwise).  A
// link whose upstream point is solid takes
//   df_i = r BB_i + (1 - r) g_p(i)(x),   BB_i = g_opp(i)(x) (half-way),
// p(i) its slip partner, evaluated as g + r (bb - g) like the column-wide
// rule.  Lanes of one wave may be wall nodes or not: every lane issues one
// load per link (its pull, or its partner's own population) and wall lanes
// one more (the bounced population), all before any is combined.  OPEN:
// the pulls that would wrap around x read the node itself (as gather<OPEN>).
// *wlinks (if given) receives the lane's wall links (bit i: upstream solid).
template <class L, typename S, typename M, typename W, bool OPEN = false>
__device__ __forceinline__ void gather_masked(const S* __restrict__ g0, const StepArgs& a,
                                              int col, int z, int x, int cw, M* df,
                                              uint32_t* wlinks = nullptr) {
  const LBM_GLOBAL S* gown = gbl(g0) + (int64_t)col * a.sC;
  const int64_t sI = a.sI;
  const unsigned ux = (unsigned)x;
  const unsigned xm = (x == 0) ? (OPEN ? 0u : (unsigned)a.nx - 1u) : ux - 1u;
  const unsigned xp = (x == a.nx - 1) ? (OPEN ? ux : 0u) : ux + 1u;
  const bool wrap = L::Q == 19 && (z == 0 || z == a.nz - 1);
  const bool wall = cw >= 0;
  constexpr int kWords = ptab_words<L>();
  uint32_t pw[kWords];
  const LBM_GLOBAL uint32_t* pt =
      reinterpret_cast<const LBM_GLOBAL uint32_t*>(gbl(a.ptab)) + (int64_t)(wall ? cw : 0) * kWords;
#pragma unroll
  for (int w = 0; w < kWords; w++) pw[w] = wall ? pt[w] : 0xffffffffu;
  const M r = wall ? static_cast<M>(gbl(static_cast<const W*>(a.rwall))[(int64_t)z * a.nw2d + cw])
                   : M(0);
  S A[L::Q], B[L::Q];
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    const unsigned prow = (pw[i >> 2] >> (8 * (i & 3))) & 0xffu;
    const bool wl = prow != kNoLink;
    const LBM_GLOBAL S* pull =
        at(gown + src_off<L>(a, i, z, wrap), L::cx[i] > 0 ? xm : (L::cx[i] < 0 ? xp : ux));
    const LBM_GLOBAL S* own = at(gown + (int64_t)(wl ? prow : 0u) * sI, ux);
    A[i] = *(wl ? own : pull);
    if (wl) B[i] = *at(gown + L::row[L::opp[i]] * sI, ux);
  }
  uint32_t links = 0u;
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    const unsigned prow = (pw[i >> 2] >> (8 * (i & 3))) & 0xffu;
    const M gs = dec<S, M>(A[i]);
    if (prow != kNoLink) {
      const M bb = dec<S, M>(B[i]);
      df[i] = gs + r * (bb - gs);
      links |= 1u << i;
    } else {
      df[i] = gs;
    }
  }
  if (wlinks) *wlinks = links;
}

// Weights of the terms linear in c_i (3 w_i), chosen so that
// sum_i t_i c_ia c_ib = delta_ab holds exactly in the working precision:
// with 3 w_i rounded independently the equilibrium's momentum would come out
// as (1 + eps) rho u and every collision would add eps omega rho u, a
// systematic anti-friction that grows to eps omega / (nu k^2) relative.
template <class L, typename M>
__device__ __forceinline__ M lin_weight(int i) {
  const int c2 = L::cx[i] * L::cx[i] + L::cy[i] * L::cy[i] + L::cz[i] * L::cz[i];
  if (c2 == 0) return M(0);
  if (L::Q == 19) {  // 2 t1 + 8 t2 = 1
    const M t2 = M(1) / M(12);
    return c2 == 2 ? t2 : (M(1) - M(8) * t2) * M(0.5);
  }
  const M t1 = M(1) / M(3);  // D2Q9: 2 t1 + 4 t2 = 1
  return c2 == 1 ? t1 : (M(1) - M(2) * t1) * M(0.25);
}

// c_i . (vx, vy, vz) from the nonzero components of c_i only: a product with
// a literal zero cannot be dropped under IEEE rules, so it is never formed
template <class L, typename M>
__device__ __forceinline__ M cdot(int i, M vx, M vy, M vz) {
  M r = M(0);
  bool any = false;
  if (L::cx[i]) {
    r = L::cx[i] > 0 ? vx : -vx;
    any = true;
  }
  if (L::cy[i]) {
    const M t = L::cy[i] > 0 ? vy : -vy;
    r = any ? r + t : t;
    any = true;
  }
  if (L::cz[i]) {
    const M t = L::cz[i] > 0 ? vz : -vz;
    r = any ? r + t : t;
  }
  return r;
}

// Open x ends: a fluid link of the first (last) node of an x-line that
// pulls from x = -1 (x = nx) reads a ghost.  The ghost copies the boundary
// node b of its own column (the column the pull reads, at the same x),
// moved along the local equilibrium to the prescribed density:
//   ghost_i = g_i(b) + w_i (drho_bc - drho_b) (1 + 3 c_i.u_b + 4.5 (c_i.u_b)^2
//                                               - 1.5 u_b.u_b),
// drho_b = sum_k g_k(b), u_b = sum_k g_k(b) c_k / (rho0 + drho_b).  Replaces
// df_i of those links after the gather, which must be the OPEN one (reads
// clamped at the ends); x is the lane's cell, the column is uniform.  On a
// tube (BOUZ) an interpolated wall link whose node behind lies beyond the
// end reads that ghost too.
template <class L, typename S, typename M, bool BOUZ = false, typename W = M>
__device__ __forceinline__ void open_patch(const S* __restrict__ g0, const StepArgs& a, int col,
                                           int x, ColInfo info, M* df) {
  const bool in = x == 0, out = x == a.nx - 1;
  if (!in && !out) return;
  const uint32_t mask = info.mask;
  const LBM_GLOBAL S* g = gbl(g0);
  const LBM_GLOBAL S* gown = g + (int64_t)col * a.sC;
  const int z = col / a.ny;
  const bool wrap = (mask & kWrapColumn) != 0u;
  const unsigned ux = (unsigned)x;
  // the ghost value of population k of a ghost next to the end node of the
  // column whose base is cb (the end of this lane's x).  Per-lane pointers:
  // the lanes of a batch work item may sit in different columns.
  auto ghost_shift = [&](const LBM_GLOBAL S* cb, int k, bool at_in, M* gk) {
    M drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int m = 0; m < L::Q; m++) {
      const M v = ld<S, M>(cb + L::row[m] * a.sI, ux);
      drho += v;
      if (L::cx[m]) jx += L::cx[m] > 0 ? v : -v;
      if (L::cy[m]) jy += L::cy[m] > 0 ? v : -v;
      if (L::cz[m]) jz += L::cz[m] > 0 ? v : -v;
      if (m == k) *gk = v;
    }
    const M rho = static_cast<M>(a.rho0) + drho;
    const M ux_ = jx / rho, uy_ = jy / rho, uz_ = jz / rho;
    const M cu = cdot<L, M>(k, ux_, uy_, uz_);
    const M usq = ux_ * ux_ + uy_ * uy_ + uz_ * uz_;
    const M dbc = static_cast<M>(at_in ? a.drho_in : a.drho_out);
    return static_cast<M>(L::w[k]) * (dbc - drho) *
           (M(1) + M(3) * cu + M(4.5) * cu * cu - M(1.5) * usq);
  };
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    if (L::cx[i] == 0 || (mask & (1u << i))) continue;
    if (!((L::cx[i] > 0 && in) || (L::cx[i] < 0 && out))) continue;
    // the source column of link i
    const LBM_GLOBAL S* cb = gown + src_off<L>(a, i, z, wrap) - L::row[i] * a.sI;
    M gi = 0;
    const M sh = ghost_shift(cb, i, in, &gi);
    df[i] = gi + sh;
  }
  if constexpr (BOUZ) {
    // interpolated wall links whose node behind, x + c_i, lies beyond this
    // end: the gather (clamped at the ends) read g_opp(i) of the boundary
    // node of that column; the ghost adds its shift, weighted as the gather
    // weighted the value (r times the interpolation coefficient)
    if ((mask & kLinkBits) == 0u) return;
    const int y = col - z * a.ny;
    const LBM_GLOBAL W* cw = gbl(static_cast<const W*>(a.bz)) + (int64_t)info.wallcol * L::Q * 2;
    const M r = static_cast<M>(gbl(static_cast<const W*>(a.rwall))[(int64_t)info.wallcol * a.nx + x]);
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
      if (L::cx[i] == 0 || !(mask & (1u << i))) continue;
      if (!((L::cx[i] > 0 && out) || (L::cx[i] < 0 && in))) continue;
      const M cbz = static_cast<M>(cw[2 * i]);
      if (cbz == M(0)) continue;
      const int nc = (y + L::cy[i]) + a.ny * (z + L::cz[i]);
      M gk = 0;
      const M sh = ghost_shift(g + (int64_t)nc * a.sC, L::opp[i], in, &gk);
      df[i] += r * cbz * sh;
    }
  }
}

// Record of one end node for the open-end ghosts: drho = sum_k g_k and
// u = sum_k g_k c_k / (rho0 + drho) of its stored populations (gc: the
// column's base, x its cell), written to o[0..3].  Summed in the order the
// step kernel's collide_store<REC> sums what it stores (rest, then each
// opposite pair), so that a state set from outside continues bit for bit.
template <class L, typename S, typename M>
__device__ __forceinline__ void end_record(const LBM_GLOBAL S* gc, const StepArgs& a, unsigned x,
                                           LBM_GLOBAL double* o) {
  M r0 = ld<S, M>(gc + L::row[0] * a.sI, x), jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 1; i < L::Q; i++) {
    const int op = L::opp[i];
    if (op < i) continue;
    const M di = ld<S, M>(gc + L::row[i] * a.sI, x), d_o = ld<S, M>(gc + L::row[op] * a.sI, x);
    const M dd = di - d_o;
    r0 += di + d_o;
    if (L::cx[i]) jx += L::cx[i] > 0 ? dd : -dd;
    if (L::cy[i]) jy += L::cy[i] > 0 ? dd : -dd;
    if (L::cz[i]) jz += L::cz[i] > 0 ? dd : -dd;
  }
  const M rho = static_cast<M>(a.rho0) + r0;
  o[0] = static_cast<double>(r0);
  o[1] = static_cast<double>(jx / rho);
  o[2] = static_cast<double>(jy / rho);
  o[3] = static_cast<double>(jz / rho);
}

// The rest of the ghost for the step kernel (whose OPEN gather already
// read g_i(b)): for the first (last) node of an x-line, each fluid link that
// would pull from x = -1 (x = nx) gains
//   w_i (drho_bc - drho_b) (1 + 3 c_i.u_b + 4.5 (c_i.u_b)^2 - 1.5 u_b.u_b)
// from b's record (bmom: the records of the buffer the step reads,
// [side][column][4]).  Lanes inside the line return at once.
template <class L, typename M, bool BOUZ = false>
__device__ __forceinline__ void open_correct(const StepArgs& a, const double* bmom, int col, int x,
                                             ColInfo info, M* df) {
  const bool in = x == 0, out = x == a.nx - 1;
  if (!in && !out) return;
  const uint32_t mask = info.mask;
  const int z = col / a.ny;
  const int y = col - z * a.ny;
  const LBM_GLOBAL double* bm_in = gbl(bmom);
  const LBM_GLOBAL double* bm_out = bm_in + (int64_t)a.ny * a.nz * 4;
  // w_k (drho_bc - drho_b) (1 + 3 c_k.u_b + 4.5 (c_k.u_b)^2 - 1.5 u_b.u_b)
  auto shift = [&](const LBM_GLOBAL double* r, int k, bool at_in) {
    const M drho = static_cast<M>(r[0]);
    const M ux_ = static_cast<M>(r[1]), uy_ = static_cast<M>(r[2]), uz_ = static_cast<M>(r[3]);
    const M cu = cdot<L, M>(k, ux_, uy_, uz_);
    const M usq = ux_ * ux_ + uy_ * uy_ + uz_ * uz_;
    const M dbc = static_cast<M>(at_in ? a.drho_in : a.drho_out);
    return static_cast<M>(L::w[k]) * (dbc - drho) *
           (M(1) + M(3) * cu + M(4.5) * cu * cu - M(1.5) * usq);
  };
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    if (L::cx[i] == 0 || (mask & (1u << i))) continue;
    if (!((L::cx[i] > 0 && in) || (L::cx[i] < 0 && out))) continue;
    int zb = z - L::cz[i];
    if (zb < 0) zb += a.nz;  // z periodic (slab; a duct or tube never pulls across z)
    if (zb >= a.nz) zb -= a.nz;
    const LBM_GLOBAL double* r = (in ? bm_in : bm_out) +
                                 ((int64_t)(y - L::cy[i]) + (int64_t)a.ny * zb) * 4;
    df[i] += shift(r, i, in);
  }
  if constexpr (BOUZ) {
    // interpolated wall links whose node behind, x + c_i, lies beyond this
    // end (the OPEN gather read g_opp(i) of the boundary node of that
    // column): the ghost's shift, weighted as the gather weighted the value
    if ((mask & kLinkBits) == 0u) return;
    const LBM_GLOBAL M* cw = gbl(static_cast<const M*>(a.bz)) + (int64_t)info.wallcol * L::Q * 2;
    const M rw = gbl(static_cast<const M*>(a.rwall))[(int64_t)info.wallcol * a.nx + x];
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
      if (L::cx[i] == 0 || !(mask & (1u << i))) continue;
      if (!((L::cx[i] > 0 && out) || (L::cx[i] < 0 && in))) continue;
      const M cbz = cw[2 * i];
      if (cbz == M(0)) continue;
      const int64_t nc = (int64_t)(y + L::cy[i]) + (int64_t)a.ny * (z + L::cz[i]);
      df[i] += rw * cbz * shift((in ? bm_in : bm_out) + nc * 4, L::opp[i], in);
    }
  }
}

// ------------------------------------------------------------------ thermal noise
// Fluctuating LB (Sec. 3.2, Eq. 6: the classical fluctuation-dissipation
// theorem for the random momentum flux; Sec. 4, Eq. 17: the fluctuating LB
// equation adds it as a local source along w_i (c_ia c_ib - c_s^2 delta_ab)).
//
// Random numbers: Philox4x64 with ten rounds (Salmon, Moraes, Dror & Shaw,
// SC'11), counter (cell, step, block, 0), key (seed, 0).  A round multiplies
// words 0 and 2 by two odd 64-bit constants; the next words are the high
// product halves xored with words 1 and 3 and the round key, and the low
// halves; the key advances by two 64-bit Weyl increments.
struct Philox4 {
  uint64_t w[4];
};

// 64 x 64 -> 128-bit product from four 32 x 32 + 64 multiply-adds: with
// m = m1 2^32 + m0, v = v1 2^32 + v0, the middle sums cannot overflow
// ((2^32 - 1)^2 + 2 (2^32 - 1) = 2^64 - 1)
__device__ __forceinline__ void mulhilo64(uint64_t m, uint64_t v, uint64_t* hi, uint64_t* lo) {
  const uint32_t m0 = (uint32_t)m, m1 = (uint32_t)(m >> 32);
  const uint32_t v0 = (uint32_t)v, v1 = (uint32_t)(v >> 32);
  const uint64_t p00 = (uint64_t)m0 * v0;
  const uint64_t t = (uint64_t)m1 * v0 + (p00 >> 32);
  const uint64_t u = (uint64_t)m0 * v1 + (uint32_t)t;
  *hi = (uint64_t)m1 * v1 + (t >> 32) + (u >> 32);
  *lo = (u << 32) | (uint32_t)p00;
}
__device__ __forceinline__ Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                 uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = c0, x1 = c1, x2 = c2, x3 = 0;
#pragma unroll
  for (int r = 0; r < 10; r++) {
    uint64_t h0, l0, h1, l1;
    mulhilo64(kM0, x0, &h0, &l0);
    mulhilo64(kM1, x2, &h1, &l1);
    x0 = h1 ^ x1 ^ k0;
    x1 = l1;
    x2 = h0 ^ x3 ^ k1;
    x3 = l0;
    k0 += kW0;
    k1 += kW1;
  }
  return Philox4{{x0, x1, x2, x3}};
}

// Two standard normals from one 64-bit word (Box-Muller): the top 23 bits of
// each 32-bit half give u = (k + 1/2) 2^-23, exact in binary32 and never 0
// or 1; z = sqrt(-2 ln u_lo) (cos, sin)(2 pi u_hi).  |z| <= sqrt(48 ln 2).
// Binary32 form (float and half storage): over all 2^23 such u the hardware
// log2 gives the radius within 5.3e-7 and the hardware sin / cos (argument
// in revolutions) are within 1.3e-7 of binary64 (measured), so
// |dz| < 1.3e-6.
__device__ __forceinline__ void normal_pair(uint64_t word, float* z0, float* z1) {
  const float ul = (static_cast<float>(static_cast<uint32_t>(word) >> 9) + 0.5f) * 0x1p-23f;
  const float uh = (static_cast<float>(static_cast<uint32_t>(word >> 32) >> 9) + 0.5f) * 0x1p-23f;
  // hardware log2 and sin / cos of 2 pi t (argument in revolutions)
  const float rad = sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(ul));
  *z0 = rad * __builtin_amdgcn_cosf(uh);
  *z1 = rad * __builtin_amdgcn_sinf(uh);
}
// Binary64 form (double storage, the reference precision): the same
// uniforms, the transform in double with the device library's log, sqrt and
// sincos (each within an ulp or two), so a normal agrees with a binary64
// evaluation of the same formula to a few units in the last place.
__device__ __forceinline__ void normal_pair(uint64_t word, double* z0, double* z1) {
  const double ul = (static_cast<double>(static_cast<uint32_t>(word) >> 9) + 0.5) * 0x1p-23;
  const double uh = (static_cast<double>(static_cast<uint32_t>(word >> 32) >> 9) + 0.5) * 0x1p-23;
  const double rad = sqrt(-2.0 * log(ul));
  double sn, cs;
  sincos(6.28318530717958647692 * uh, &sn, &cs);
  *z0 = rad * cs;
  *z1 = rad * sn;
}

// the type the thermal normals of a storage type are drawn in
template <typename S>
using NormalT = typename std::conditional<sizeof(S) == 8, double, float>::type;

// sqrt(w_i) from the weight class (|c|^2 and the lattice)
template <class L, typename M>
__device__ __forceinline__ constexpr M sqrt_w(int i) {
  return L::Q == 9 ? (i == 0 ? M(2.0 / 3) : (i < 5 ? M(1.0 / 3) : M(1.0 / 6)))
                   : (i == 0 ? M(0.57735026918962576451) : (i < 7 ? M(0.23570226039551584147) : M(1.0 / 6)));
}

// Thermal term xi_i added to the post-collision population of a cell.  Each
// non-conserved direction relaxes by gamma = 1 - omega per step; holding it at
// the equilibrium variance mu w_i (mu = rho0 kT / c_s^2, which gives
// <j_a^2> = rho0 kT) takes added variance mu (1 - gamma^2): A^2 (host side).
// The normals z_k come in the order block k/8, word (k mod 8)/2, cos then sin.
//  th_mode 1 (the stress source): P_aa = sqrt(2) c_s^2 A z, P_ab = c_s^2 A z
//    (order xx, yy, [zz,] xy, [xz, yz]), xi_i = w_i/(2 c_s^4) P:(c_i c_i - c_s^2 I),
//    i.e. xi_i = w_i [1.5 sqrt(2) A sum_a z_aa (c_ia^2 - 1/3) + 3 A sum_a<b z_ab c_ia c_ib];
//  th_mode 2: v_i = sqrt(w_i) z_i for every i, mass and momentum removed:
//    xi_i = A (v_i - w_i sum v - 3 w_i c_i . sum v c).
// Z is the type the normals are drawn in: double for double storage,
// float (the hardware transcendentals) for float and half storage.
template <class L, typename M, int MODE, typename Z = float>
__device__ __forceinline__ void thermal_noise(const StepArgs& a, uint32_t cell, int64_t step,
                                              M* xi) {
  static_assert(MODE == 1 || MODE == 2, "noise form");
  const M A = static_cast<M>(a.th_amp);
  const uint64_t key = a.th_seed;
  if constexpr (MODE == 1) {
    Z z[6] = {0, 0, 0, 0, 0, 0};
    const Philox4 r = philox4x64_10(cell, (uint64_t)step, 0, key, 0);
    normal_pair(r.w[0], &z[0], &z[1]);
    normal_pair(r.w[1], &z[2], &z[3]);
    if (L::Q == 19) normal_pair(r.w[2], &z[4], &z[5]);
    const M sd = M(2.12132034355964257320) * A, so = M(3) * A;
    // 2-D: xx, yy, xy; 3-D: xx, yy, zz, xy, xz, yz; each component scaled by
    // its closure factor (exactly 1 for the classical noise)
    const M pxx = (sd * static_cast<M>(a.th_fac[0])) * z[0];
    const M pyy = (sd * static_cast<M>(a.th_fac[1])) * z[1];
    const M pzz = L::Q == 19 ? (sd * static_cast<M>(a.th_fac[2])) * z[2] : M(0);
    const M pxy = (so * static_cast<M>(a.th_fac[3])) * (L::Q == 19 ? z[3] : z[2]);
    const M pxz = L::Q == 19 ? (so * static_cast<M>(a.th_fac[4])) * z[4] : M(0);
    const M pyz = L::Q == 19 ? (so * static_cast<M>(a.th_fac[5])) * z[5] : M(0);
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
      const M t = M(1) / M(3);
      const M s = pxx * (M(L::cx[i] * L::cx[i]) - t) + pyy * (M(L::cy[i] * L::cy[i]) - t) +
                  (L::Q == 19 ? pzz * (M(L::cz[i] * L::cz[i]) - t) : M(0)) +
                  pxy * M(L::cx[i] * L::cy[i]) + pxz * M(L::cx[i] * L::cz[i]) +
                  pyz * M(L::cy[i] * L::cz[i]);
      xi[i] = static_cast<M>(L::w[i]) * s;
    }
    return;
  } else {
    Z z[L::Q];
    constexpr int kBlocks = (L::Q + 7) / 8;
#pragma unroll
    for (int b = 0; b < kBlocks; b++) {
      const Philox4 r = philox4x64_10(cell, (uint64_t)step, (uint64_t)b, key, 0);
#pragma unroll
      for (int w = 0; w < 4; w++) {
        const int k = 8 * b + 2 * w;
        if (k >= L::Q) break;
        Z z0, z1;
        normal_pair(r.w[w], &z0, &z1);
        z[k] = z0;
        if (k + 1 < L::Q) z[k + 1] = z1;
      }
    }
    M v[L::Q], sv = 0, sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
      v[i] = sqrt_w<L, M>(i) * static_cast<M>(z[i]);
      sv += v[i];
      if (L::cx[i]) sx += L::cx[i] > 0 ? v[i] : -v[i];
      if (L::cy[i]) sy += L::cy[i] > 0 ? v[i] : -v[i];
      if (L::cz[i]) sz += L::cz[i] > 0 ? v[i] : -v[i];
    }
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
      const M wi = static_cast<M>(L::w[i]);
      const M cs = M(L::cx[i]) * sx + M(L::cy[i]) * sy + M(L::cz[i]) * sz;
      xi[i] = A * (v[i] - wi * sv - M(3) * wi * cs);
    }
  }
}

// BGK relaxation with Guo forcing on shifted populations; each result is
// stored as soon as it is computed (out_col: the column's base, uniform):
//   rho = rho0 + sum df, j = rho u = sum df c + F/2,
//   dfeq_i = w_i [(rho - rho0) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)],
//   df_i <- df_i - omega (df_i - dfeq_i) + (1 - omega/2) w_i [3 (c_i - u) + 9 (c_i.u) c_i].F
// with rho (3 c.u) written as t_i (c.j) (t_i = 3 w_i, see lin_weight).  Per
// cell the terms common to all directions are gathered first:
//   C0 = omega (drho - 1.5 rho u.u) - 3 A u.F,      A = 1 - omega/2,
//   U  = 4.5 omega rho u + 9 A F,  J = omega j + A F,
// so that  df_i <- (1 - omega) df_i + E_i + O_i  with the even part
// E_i = w_i (C0 + (c.u)(c.U)) and the odd part O_i = t_i (c.J).  Opposite
// directions share E and take O with its sign flipped, so each pair is
// computed once and the odd parts cancel exactly in the next moments.
// With TH = 1 or 2, xi holds the cell's thermal term of that form
// (thermal_noise), added to every result.
//
// With REC the moments of the values as stored (decoded back: sum g,
// sum g c) are summed into rec[0..3] (the open ends' end-node records).
// Store of one new population.  A state far larger than the 256 MB
// last-level cache cannot be kept there from one step to the next, and
// writing it through that cache only evicts lines the step still reads: it
// then goes out with nontemporal stores (NT; measured on the 637 MB FP64
// duct: 114.5 -> 107.7 us per step; on the 319 MB FP32 duct, whose
// alternating column order reuses the cache, they cost 3 %).  A compile-time
// choice: a uniform run-time flag is folded into plain stores.
template <bool NT, typename S>
__device__ __forceinline__ void store_pop(LBM_GLOBAL S* p, S v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

template <class L, typename M, typename S, int TH = 0, bool REC = false, bool NT = false>
__device__ __forceinline__ void collide_store(const M* df, const StepArgs& a, LBM_GLOBAL S* out_col,
                                              unsigned x, uint32_t cell, int64_t step,
                                              const M* xi = nullptr, M* rec = nullptr) {
  constexpr bool THERM = TH != 0;
  M drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    drho += df[i];
    if (L::cx[i]) jx += L::cx[i] > 0 ? df[i] : -df[i];
    if (L::cy[i]) jy += L::cy[i] > 0 ? df[i] : -df[i];
    if (L::cz[i]) jz += L::cz[i] > 0 ? df[i] : -df[i];
  }
  const M Fx = par<M>(a.F[0], a.F_f[0]), Fy = par<M>(a.F[1], a.F_f[1]),
          Fz = par<M>(a.F[2], a.F_f[2]);
  jx += Fx * M(0.5);
  jy += Fy * M(0.5);
  jz += Fz * M(0.5);
  const M rho = par<M>(a.rho0, a.rho0_f) + drho;
  const M irho = M(1) / rho;
  const M ux = jx * irho, uy = jy * irho, uz = jz * irho;
  const M om = par<M>(a.omega, a.omega_f);
  const M A = M(1) - M(0.5) * om;
  const M usq15 = M(1.5) * (ux * ux + uy * uy + uz * uz);
  const M uF3 = M(3) * (ux * Fx + uy * Fy + uz * Fz);
  // the terms of the new populations, each times the storage scale sc
  constexpr M sc = static_cast<M>(Store<S, M>::kScale);
  const M C0 = (om * (drho - rho * usq15) - A * uF3) * sc;
  const M k45 = M(4.5) * om * rho * sc, a9 = M(9) * A * sc;
  const M Ux = k45 * ux + a9 * Fx, Uy = k45 * uy + a9 * Fy, Uz = k45 * uz + a9 * Fz;
  const M oms = om * sc, As = A * sc;
  const M Jx = oms * jx + As * Fx, Jy = oms * jy + As * Fy, Jz = oms * jz + As * Fz;
  const M keep = (M(1) - om) * sc;
  // rounding bits: one 32-bit word for the rest population, then one per
  // opposite pair (low half for the first direction, high half for its opposite)
  RoundBits rb(a.seed, step, Store<S, M>::kRandom ? cell : 0u);
  {
    const uint32_t w0 = Store<S, M>::kRandom ? rb.next() : 0u;
    M v = keep * df[0] + static_cast<M>(L::w[0]) * C0;
    if constexpr (THERM) v += xi[0] * sc;
    const S e = Store<S, M>::enc(v, w0);
    store_pop<NT>(at(sbase(out_col + L::row[0] * a.sI), x), e);
    if constexpr (REC) {
      rec[0] = dec<S, M>(e);
      rec[1] = rec[2] = rec[3] = M(0);
    }
  }
#pragma unroll
  for (int i = 1; i < L::Q; i++) {
    const int o = L::opp[i];
    if (o < i) continue;  // each pair once, from its first direction
    const M wi = static_cast<M>(L::w[i]);
    const M cu = cdot<L, M>(i, ux, uy, uz);
    const M cU = cdot<L, M>(i, Ux, Uy, Uz);
    const M cJ = cdot<L, M>(i, Jx, Jy, Jz);
    const M E = (wi * cu) * cU + wi * C0;
    const M O = lin_weight<L, M>(i) * cJ;
    M vi = (keep * df[i] + E) + O;
    M vo = (keep * df[o] + E) - O;
    if constexpr (THERM) {
      vi += xi[i] * sc;
      vo += xi[o] * sc;
    }
    const uint32_t word = Store<S, M>::kRandom ? rb.next() : 0u;
    S ei, eo;
    Store<S, M>::enc2(vi, vo, word, &ei, &eo);
    store_pop<NT>(at(sbase(out_col + L::row[i] * a.sI), x), ei);
    store_pop<NT>(at(sbase(out_col + L::row[o] * a.sI), x), eo);
    if constexpr (REC) {  // c_o = -c_i
      const M di = dec<S, M>(ei), dd = di - dec<S, M>(eo);
      rec[0] += di + dec<S, M>(eo);
      if (L::cx[i]) rec[1] += L::cx[i] > 0 ? dd : -dd;
      if (L::cy[i]) rec[2] += L::cy[i] > 0 ? dd : -dd;
      if (L::cz[i]) rec[3] += L::cz[i] > 0 ? dd : -dd;
    }
  }
}

}  // namespace lbm

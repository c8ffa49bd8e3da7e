// stage_common.hpp -- launch arguments, index conventions and buffer-resource
// helpers shared by the RK-stage kernel (stage_kernel.hpp) and the host ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chemora {

// ---- grid-function numbering and symmetric-tensor packing ----------------
// packed symmetric index: xx xy xz yy yz zz
__device__ __forceinline__ constexpr int S(int i, int j) {
  return (i == 0) ? j : (j == 0 ? i : (i == 1 ? (j == 1 ? 3 : 4) : (j == 1 ? 4 : 5)));
}
// weight of a packed slot in a full double sum over (i, j)
__device__ __forceinline__ constexpr double W(int s) { return (s == 1 || s == 2 || s == 4) ? 2.0 : 1.0; }
// row / column of a packed slot
__device__ __forceinline__ constexpr int SI(int s) { return s < 3 ? 0 : (s < 5 ? 1 : 2); }
__device__ __forceinline__ constexpr int SJ(int s) { return s < 3 ? s : (s < 5 ? s - 2 : 2); }

// storage order of the 24 grid functions (the chemora.h GF layout)
enum : int { gCHI = 0, gGT = 1, gK = 7, gAT = 8, gXT = 14, gALPHA = 17, gBETA = 18, gB = 21 };

struct Gauge {
  int lapse;   // 0 1+log, 1 harmonic, 2 frozen
  int shift;   // 0 Gamma-driver, 1 frozen
  double eta;
};

// ---- launch arguments ----------------------------------------------------
// Geometry of a patch (all strides in elements).
struct Geo {
  int nx, ny, nz, g;
  int64_t sy, sz, sf;
};

struct Scales {
  double d1;    // 1 / (D1 h)
  double d2;    // 1 / (D2 h^2)
  double d11;   // 1 / (D1 h)^2
  double up;    // 1 / (DU h)
  double ko;    // 2^(-2r) * (eps / h)
  double kow[5];  // Kreiss-Oliger weights of s_1 .. s_5 for radius ko_r, zero past it
  int ko_r;
};

// What the kernel does with the right-hand side k it computed (HAM: nothing;
// it stores the Hamiltonian constraint into out, one GF with the patch's
// strides, instead), with
// Y = yin[point] and U = un[point] read at every point in every mode, and
// out = cu U + cyo Y + cs k formed as fma(cs, k, fma(cyo, Y, cu U)):
//   RHS     out = k                             (cu = cyo = 0, cs = 1)
//   STAGE1  y = Y + cy k,   out = U + cs k      (yin = un = u_n; RK4)
//   STAGE23 y = Y + cy k,   out = U + cs k      (yin = y, un = u_n; RK4)
//   STAGE4  out = U + cs k                      (un = yin = accumulator, cs = cy; RK4)
//   RK3     out = cu U + cyo Y + cs k           (un = u_n, yin = the stage input; RK3)
// Pointers a mode does not need are set to an array the stage reads anyway
// (in / u_n / the accumulator), so the unconditional reads cost no HBM
// traffic and keep the kernel free of mode-dependent loads.
enum Mode : int { MODE_RHS = 0, MODE_STAGE1 = 1, MODE_STAGE23 = 2, MODE_STAGE4 = 4, MODE_HAM = 8, MODE_RK3 = 16 };

struct StageArgs {
  const double* __restrict__ in;   // stencil input of this stage
  const double* un;                // U operand (see Mode)
  const double* yin;               // Y operand (see Mode)
  double* y;                       // RK accumulator written by stages 1-3
  double* out;                     // rhs (MODE_RHS), next stage input, or u (stage 4)
  Geo geo;
  Scales sc;
  Gauge gauge;
  double cy;                       // weight of k in the accumulator update
  double cs;                       // weight of k in out
  double cu;                       // weight of U in out (0 for the bare right-hand side)
  double cyo;                      // weight of Y in out (RK3 stages 2 and 3, else 0)
  double chi_split;                // split precision: FP64 chi phase where chi < chi_split
  int tiles_x, tiles_y;            // tile grid of the launch's tile variant
  int mode;                        // a Mode
};

constexpr int NXCD = 8;

// Batched form: all tiles of all patches of a plan.  ntiles == 0 selects the
// single-patch form (the StageArgs kernel argument, one tile per work-group).
// queue == nullptr: one work-group per tile.  Otherwise the launch is
// persistent (a few work-groups per CU) and its work-groups pull tiles from
// NXCD queues -- queue x hands out the x-th contiguous eighth of the tile
// list, a work-group pulls from its own XCD's queue first and then from the
// others -- and queue[NXCD] counts the work-groups that have finished: the
// last one returns every counter to zero for the next launch.  The counters
// must be zero when the launch starts.
constexpr int QUEUE_INTS = 16;   // ints per launch: NXCD heads, the finished count, padding
struct BatchTable {
  const StageArgs* args;     // one per patch (device memory)
  const int* tile_start;     // prefix sums of tiles per patch, npatch + 1 entries
  int* queue;                // persistent form: QUEUE_INTS zeroed counters
  int npatch;
  int ntiles;
};

// ---- device helpers ------------------------------------------------------
// Materialises a value in registers at this point.  Without it the compiler
// sinks the arithmetic of an accumulator to its last use near the end of the
// kernel while the stencil reads feeding it stay early (stores intervene),
// which keeps every tap live across the kernel.
__device__ __forceinline__ void keep(double& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void keep(float& x) { asm volatile("" : "+v"(x)); }
template <class V, int N>
__device__ __forceinline__ void keep(V (&x)[N]) {
#pragma unroll
  for (int n = 0; n < N; ++n) keep(x[n]);
}
template <class V, int N, int M>
__device__ __forceinline__ void keep(V (&x)[N][M]) {
#pragma unroll
  for (int n = 0; n < N; ++n) keep(x[n]);
}

// Raw buffer access (gfx9 descriptor word 3 = 0x00020000).  Each state
// buffer (24 GFs) is one buffer resource whose base sits XB elements before
// the array, and an access is
//   base + voffset (per lane) + soffset (uniform: GF, plane, tile) + imm,
// so per-point offsets stay in one register and GF / plane offsets are
// scalar arithmetic.  Offsets are 32-bit: the host rejects patches whose
// 24-GF state exceeds 4 GiB.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
constexpr int XB = 8;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t state_rsrc(const double* base, int64_t sf) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)(base - XB), (short)0, (int)((24 * sf + XB) * 8), 0x00020000);
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)voff, (int)soff, 0);
}

// Work-groups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap the hardware block id so that each XCD receives a contiguous
// range of tiles (neighbours share halos in that XCD's L2).
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  const int full = (nblocks / NXCD) * NXCD;
  if (bid >= full) return bid;
  return (bid % NXCD) * (nblocks / NXCD) + bid / NXCD;
}

// Values loaded from the plan tables are the same in every lane, but the
// compiler cannot prove it (the kernel also writes global memory), and a
// buffer descriptor held in vector registers turns every access into a
// waterfall loop.  Broadcasting lane 0 puts them in scalar registers.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The plan tables are written by the host only, so they are read through
// the constant address space: the compiler may then use scalar loads even
// after the kernel's own stores (the persistent form's tile loop).
typedef const __attribute__((address_space(4))) int* const_int_ptr;
__device__ __forceinline__ int table_load(const int* p, int i) { return ((const_int_ptr)p)[i]; }

__device__ __forceinline__ StageArgs uniform_args(const StageArgs* p) {
  constexpr int N = (int)(sizeof(StageArgs) / 4);
  static_assert(sizeof(StageArgs) % 4 == 0, "StageArgs is a whole number of words");
  int w[N];
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = table_load((const int*)p, i);
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  StageArgs a;
  __builtin_memcpy(&a, w, sizeof(StageArgs));
  return a;
}

// The XCD a work-group runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ int xcd_id() { return __builtin_amdgcn_s_getreg(0xf814) & (NXCD - 1); }

// Persistent form: the next tile for a work-group on XCD x, or -1 when every
// queue is empty.  Queue q hands out tiles [q n / NXCD, (q + 1) n / NXCD) in
// order; each atomic increment hands out one index exactly once, so a tile
// is taken by exactly one work-group whichever queues the work-groups try.
__device__ __forceinline__ int pull_tile(const BatchTable& bt, int x) {
  for (int s = 0; s < NXCD; ++s) {
    const int q = (x + s) & (NXCD - 1);
    const int lo = (int)((int64_t)q * bt.ntiles / NXCD), hi = (int)((int64_t)(q + 1) * bt.ntiles / NXCD);
    if (hi <= lo || __atomic_load_n(bt.queue + q, __ATOMIC_RELAXED) >= hi - lo) continue;
    const int i = atomicAdd(bt.queue + q, 1);
    if (i < hi - lo) return lo + i;
  }
  return -1;
}

// patch of global tile t (binary search over the prefix sums)
__device__ __forceinline__ int batch_patch(const BatchTable& bt, int t) {
  int lo = 0, hi = bt.npatch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (uniform(table_load(bt.tile_start, mid)) <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---- tile variants: the launch shapes the tuner chooses among -----------
// TX columns x WPG waves per work-group over TZ planes (a wave covers
// 64 / TX rows of one plane): tiles of TX x TY x TZ points.
struct TileVariant {
  int tx, wpg, tz;
};
constexpr int NVARIANT = 6;
constexpr TileVariant VARIANTS[NVARIANT] = {{64, 4, 1}, {64, 8, 1}, {32, 4, 1}, {32, 8, 1}, {32, 8, 2}, {32, 8, 4}};
inline int variant_ty(int v) { return VARIANTS[v].wpg / VARIANTS[v].tz * 64 / VARIANTS[v].tx; }
inline int variant_tz(int v) { return VARIANTS[v].tz; }
// order 8's staged neighbourhood is too large for the 8-wave shapes
inline bool variant_supported(int order, int v) {
  return v >= 0 && v < NVARIANT && (order == 4 || (VARIANTS[v].wpg == 4 && VARIANTS[v].tz == 1));
}

// ---- host-side launchers, one per order (stage_o4.hip / stage_o8.hip) ----
// Single-patch form: bt.ntiles == 0, grid = tiles of a.  Batched form: a is
// unused, grid = bt.ntiles (one work-group per tile of the plan) or, with
// persist (bt.queue set), any grid >= 1.  The tile counts in a / the plan
// tables must be those of `variant`.  wgs != nullptr: nothing is launched;
// *wgs receives how many work-groups of that kernel fit one CU (0 if the
// query fails).  Each (precision, persist) part is its own object file.
// split: FP32 stencil combinations and algebra (order 4 only)
template <bool SPLIT, bool PERSIST>
void launch_stage_o4_part(int variant, bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt, int grid,
                          hipStream_t s, int* wgs);
template <bool PERSIST>
void launch_stage_o8_part(int variant, bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt, int grid,
                          hipStream_t s, int* wgs);
#define CHEMORA_DECLARE_O4_PART(SP, PE)                                                                          \
  template <>                                                                                                     \
  void launch_stage_o4_part<SP, PE>(int variant, bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt, \
                                    int grid, hipStream_t s, int* wgs);
CHEMORA_DECLARE_O4_PART(false, false)
CHEMORA_DECLARE_O4_PART(false, true)
CHEMORA_DECLARE_O4_PART(true, false)
CHEMORA_DECLARE_O4_PART(true, true)
#undef CHEMORA_DECLARE_O4_PART
template <>
void launch_stage_o8_part<false>(int variant, bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt,
                                 int grid, hipStream_t s, int* wgs);
template <>
void launch_stage_o8_part<true>(int variant, bool upwind, int ko_r, const StageArgs& a, const BatchTable& bt,
                                int grid, hipStream_t s, int* wgs);

inline void launch_stage_o4(int variant, bool split, bool persist, bool upwind, int ko_r, const StageArgs& a,
                            const BatchTable& bt, int grid, hipStream_t s, int* wgs = nullptr) {
  if (split)
    persist ? launch_stage_o4_part<true, true>(variant, upwind, ko_r, a, bt, grid, s, wgs)
            : launch_stage_o4_part<true, false>(variant, upwind, ko_r, a, bt, grid, s, wgs);
  else
    persist ? launch_stage_o4_part<false, true>(variant, upwind, ko_r, a, bt, grid, s, wgs)
            : launch_stage_o4_part<false, false>(variant, upwind, ko_r, a, bt, grid, s, wgs);
}
inline void launch_stage_o8(int variant, bool persist, bool upwind, int ko_r, const StageArgs& a,
                            const BatchTable& bt, int grid, hipStream_t s, int* wgs = nullptr) {
  persist ? launch_stage_o8_part<true>(variant, upwind, ko_r, a, bt, grid, s, wgs)
          : launch_stage_o8_part<false>(variant, upwind, ko_r, a, bt, grid, s, wgs);
}

}  // namespace chemora

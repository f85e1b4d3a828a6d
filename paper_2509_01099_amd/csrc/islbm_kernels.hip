// HIP kernels of the ISLBM time step for gfx950 (MI355X).
//
// One launch of step_kernel advances every fluid node by one time step
// (Sec. 2.1-2.3): the post-collision populations of the previous step are
// pull-streamed by tensor-product quadratic interpolation at the departure
// points x - e_i dt (Sec. 2.2; weights precomputed per axis on the host), the
// half-way bounce-back / anti-bounce-back rules replace links that leave the
// fluid (Sec. 2.3), then the MRT collision of f and g runs in registers and
// the new post-collision populations are stored.  Optionally the same launch
// accumulates the Nusselt / Reynolds / mass reductions in FP64.
//
// Memory design: each buffer (f or g) holds, for every (z, y) row of the mesh,
// the rows of its Q populations one after another ([z][y][pop][x], padded
// row pitch).  The 2Q read and write streams of a tile then lie in a few
// DRAM pages rather than in 2Q planes gigabytes apart; a plain copy with the
// step's pattern runs about 20 % faster this way.  Every workgroup stages a
// TX x TY x TZ tile of each moving population
// plus the halo that population's stencil needs (only along the axes it is
// shifted on) into LDS with coalesced row loads, so every interpolation tap
// is an LDS read.  Workgroups are remapped so that consecutive tiles land on
// the same XCD (blocks are dealt round-robin over the 8 XCDs), which keeps
// halo re-reads inside one L2.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "islbm_lattice.hpp"
#include "islbm_launch.hpp"

namespace islbm {

// ---------------------------------------------------------------------------
// Storage conversion
// ---------------------------------------------------------------------------
template <typename S>
struct Store;
// st_nt: streaming store for working sets larger than the last-level cache
// (the output of a step is not re-read until the next launch).
template <>
struct Store<float> {
  using R = float;
  static constexpr bool kDither = false;
  __device__ static float ld(const float* p) { return *p; }
  __device__ static void st(float* p, float v) { *p = v; }
  __device__ static void st_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Store<double> {
  using R = double;
  static constexpr bool kDither = false;
  __device__ static double ld(const double* p) { return *p; }
  __device__ static void st(double* p, double v) { *p = v; }
  __device__ static void st_nt(double* p, double v) { __builtin_nontemporal_store(v, p); }
};
// FP16 holds the deviations scaled by 2^12 (an exact power of two): deviations
// down to ~1.5e-8 stay normal numbers; |f - w| and |g| up to 16 are
// representable.  BF16 has the FP32 exponent range and needs no scale.
//
// The time step stores 2-byte values with stochastic rounding (st_dither):
// the FP32 result is rounded up with probability equal to its distance from
// the lower neighbour in units of the spacing.  gfx950 does this in one
// instruction (v_cvt_sr_f16_f32 / v_cvt_sr_bf16_f32) from a 32-bit random
// word; measured on MI355X, the mean over random words of the rounded value
// equals the FP32 value to sampling accuracy whichever 13 or 16 of the word's
// bits are random, i.e. the rounding is unbiased.  With round-to-nearest, a
// change smaller than half a spacing is lost every step and slowly driven
// states stall; stochastic rounding keeps the expected stored value equal to
// the FP32 one.  Other writers (initialisation, uploads) round to nearest.
typedef __fp16 f16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
template <>
struct Store<__half> {
  using R = float;
  static constexpr bool kDither = true;
  static constexpr float kScale = 4096.0f, kInv = 1.0f / 4096.0f;
  __device__ static float ld(const __half* p) { return __half2float(*p) * kInv; }
  // two x-neighbours loaded as one 4-byte word (lower address in the low half)
  __device__ static void unpack(unsigned w, float& lo, float& hi) {
    lo = __half2float(__ushort_as_half((unsigned short)(w & 0xFFFFu))) * kInv;
    hi = __half2float(__ushort_as_half((unsigned short)(w >> 16))) * kInv;
  }
  __device__ static void st(__half* p, float v) { *p = __float2half_rn(v * kScale); }
  __device__ static void st_nt(__half* p, float v) { st(p, v); }
  // the convert writes the low half of its destination and keeps the high
  // half, which is never stored: seeding it with the input's own bits lets
  // the destination reuse the input register (no copy per store)
  __device__ static void st_dither(__half* p, float v, unsigned bits) {
    const float x = v * kScale;
    f16x2_t h = __builtin_bit_cast(f16x2_t, x);
    h = __builtin_amdgcn_cvt_sr_f16_f32(h, x, bits, false);
    *reinterpret_cast<__fp16*>(p) = h.x;
  }
};
template <>
struct Store<__hip_bfloat16> {
  using R = float;
  static constexpr bool kDither = true;
  __device__ static float ld(const __hip_bfloat16* p) { return __bfloat162float(*p); }
  // a bfloat16 is the upper half of the float with the same bits
  __device__ static void unpack(unsigned w, float& lo, float& hi) {
    lo = __uint_as_float(w << 16);
    hi = __uint_as_float(w & 0xFFFF0000u);
  }
  __device__ static void st(__hip_bfloat16* p, float v) { *p = __float2bfloat16(v); }
  __device__ static void st_nt(__hip_bfloat16* p, float v) { st(p, v); }
  __device__ static void st_dither(__hip_bfloat16* p, float v, unsigned bits) {
    bf16x2_t h = __builtin_bit_cast(bf16x2_t, v);  // high half unused, as for FP16
    h = __builtin_amdgcn_cvt_sr_bf16_f32(h, v, bits, false);
    *reinterpret_cast<__bf16*>(p) = h.x;
  }
};

// FP32 storage with FP64 arithmetic: the same 4-byte deviations as FP32,
// loaded into double, updated in double, and written back with stochastic
// rounding from double (29 random bits below the kept float mantissa), so
// that changes far below a float ulp are kept in expectation.
struct f32s {
  float x;
};
template <>
struct Store<f32s> {
  using R = double;
  static constexpr bool kDither = true;
  __device__ static double ld(const f32s* p) { return double(p->x); }
  __device__ static void st(f32s* p, double v) { p->x = float(v); }
  __device__ static void st_nt(f32s* p, double v) { __builtin_nontemporal_store(float(v), &p->x); }
  __device__ static void st_dither(f32s* p, double v, unsigned bits) {
    unsigned long long u = __double_as_longlong(v);
    u = (u + ((unsigned long long)bits >> 3)) & ~0x1FFFFFFFull;  // exact in float across its normal range
    p->x = float(__longlong_as_double(u));
  }
};

// 32-bit integer hash "lowbias32" (C. Wellons, "Prospecting for hash
// functions", 2018) of node and device-side step counter; the bits of
// population i are the top bits of that hash times a distinct odd constant
// (multiply-shift hashing), which st_dither takes from the high end.
__device__ __forceinline__ unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Store of population i of a node whose hash is h0.  The rounding bits of
// population i are the low 32 bits of the product of h0's low 24 bits and a
// distinct odd 24-bit constant (a full-rate 24-bit multiply); st_dither takes
// them from the high end, where every bit of the multiplicand contributes.
template <typename S, bool NTS>
__device__ __forceinline__ void store_pop(S* p, typename Store<S>::R v, unsigned h0, int i) {
  if constexpr (Store<S>::kDither)
    Store<S>::st_dither(p, v, __umul24(h0, (unsigned(2 * i + 1) * 0x9E3779B1u) & 0xFFFFFFu));
  else if constexpr (NTS) Store<S>::st_nt(p, v);
  else Store<S>::st(p, v);
}

template <typename R>
struct KArgs {
  int n[3];
  int pitch;            // elements of one population row (>= n[0])
  long long ps;         // elements between the rows of two populations (= pitch)
  long long rsf, rsg;   // elements between consecutive rows of one population (Q pitch)
  int tiles[3];
  int nblocks;
  Rates<R> k;
  R omega, Thot, Tcold;
  int collide;
  const R* wtab[3];
  // reductions
  double* partials;
  const double* red;
  long long red_vol[3], red_mw[3], red_chot, red_ccold, red_cmv, red_cmd;
  double inv_uf, inv_dT, T0;
  // step counters of the stochastic rounding: a launch reads rctr[rpar] and
  // its block 0 writes rctr[rpar ^ 1] = rctr[rpar] + 1 for the next launch
  unsigned int* rctr;
  int rpar;
};

template <typename R>
static KArgs<R> make_args(const DevState& s) {
  KArgs<R> a{};
  for (int i = 0; i < 3; ++i) a.n[i] = s.n[i];
  a.pitch = s.pitch;
  a.ps = s.ps;
  a.rsf = s.rsf;
  a.rsg = s.rsg;
  a.k.s_e = R(s.s_e);
  a.k.s_eps = R(s.s_eps);
  a.k.s_q = R(s.s_q);
  a.k.s_nu = R(s.s_nu);
  a.k.s_pi = R(s.s_pi);
  a.k.s_m = R(s.s_m);
  a.k.q_j = R(s.q_j);
  a.k.q_e = R(s.q_e);
  a.k.q_nu = R(s.q_nu);
  a.k.aT = R(s.aT);
  a.k.gbeta = R(s.gbeta);
  a.k.T0 = R(s.T0);
  a.omega = R(s.omega);
  a.Thot = R(s.Thot);
  a.Tcold = R(s.Tcold);
  a.collide = s.collide;
  for (int i = 0; i < 3; ++i) a.wtab[i] = static_cast<const R*>(s.wtab[i]);
  a.red = s.red;
  for (int i = 0; i < 3; ++i) {
    a.red_vol[i] = s.red_vol[i];
    a.red_mw[i] = s.red_mw[i];
  }
  a.red_chot = s.red_chot;
  a.red_ccold = s.red_ccold;
  a.red_cmv = s.red_cmv;
  a.red_cmd = s.red_cmd;
  a.inv_uf = s.inv_uf;
  a.inv_dT = s.inv_dT;
  a.T0 = s.T0;
  a.rctr = s.rctr;
  a.rpar = s.rpar;
  return a;
}

// Per-launch key of the stochastic rounding (2-byte storage only).
template <typename S, typename R>
__device__ __forceinline__ unsigned dither_key(const KArgs<R>& a) {
  if constexpr (Store<S>::kDither) {
    const unsigned base = a.rctr[a.rpar];
    if (blockIdx.x == 0 && threadIdx.x == 0) a.rctr[a.rpar ^ 1] = base + 1u;
    return mix32(base * 0x85EBCA77u + 0x165667B1u);
  } else {
    return 0u;
  }
}

// ---------------------------------------------------------------------------
// Tile geometry and LDS slots (one per moving population)
// ---------------------------------------------------------------------------
// XH: x extent added to the tile by the halo of an x-shifted population: 2
// (one node each side), or 4 for 2-byte storage, whose staged boxes start at
// an even x so that they are loaded as 4-byte x pairs.
template <int TX_, int TY_, int TZ_, int NR_, int XH_ = 2>
struct Tile {
  static constexpr int TX = TX_, TY = TY_, TZ = TZ_, NR = NR_, XH = XH_;
  static constexpr int ROWS = TY * TZ;       // (y,z) rows of a tile
  static constexpr int RS = ROWS / NR;       // rows covered by one pass of the block
  static constexpr int NT = TX * RS;         // threads per block
  static_assert(ROWS % NR == 0, "rows per thread must divide the tile");
  static_assert(XH == 2 || (XH == 4 && TX % 2 == 0), "paired staging needs an even tile width");
  __host__ __device__ static constexpr int ext(int a) { return a == 0 ? TX : (a == 1 ? TY : TZ); }
};

template <int D, class T>
struct Slots {
  using LF = typename Pair<D>::F;
  using LG = typename Pair<D>::G;
  static constexpr int NF = LF::Q - 1, NG = LG::Q - 1, N = NF + NG;
  __host__ __device__ static constexpr bool isg(int s) { return s >= NF; }
  __host__ __device__ static constexpr int pop(int s) { return s < NF ? s + 1 : s - NF + 1; }
  __host__ __device__ static constexpr int e(int s, int a) {
    return isg(s) ? LG::e(pop(s), a) : LF::e(pop(s), a);
  }
  __host__ __device__ static constexpr int ext(int s, int a) {
    return T::ext(a) + (e(s, a) != 0 ? (a == 0 ? T::XH : 2) : 0);
  }
  __host__ __device__ static constexpr int size(int s) { return ext(s, 0) * ext(s, 1) * ext(s, 2); }
  __host__ __device__ static constexpr int off(int s) {
    int o = 0;
    for (int k = 0; k < s; ++k) o += size(k);
    return o;
  }
  // slot of the opposite population (same set)
  __host__ __device__ static constexpr int opps(int s) {
    return isg(s) ? NF + opp<LG>(pop(s)) - 1 : opp<LF>(pop(s)) - 1;
  }
  static constexpr int total = off(N);
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Geometry of the block's tile: tile origin t0 and halo origin lo per axis.
struct TileOrigin {
  int t0[3];
  int lo[3];
};

template <class T>
__device__ __forceinline__ TileOrigin tile_origin(const int* n, const int* tiles, int nblocks) {
  // Workgroups are dealt round-robin over the 8 XCDs; give each XCD a
  // contiguous range of tiles so that neighbouring tiles share its L2.
  const int b = blockIdx.x;
  const int xcd = b & 7, loc = b >> 3;
  const int per = nblocks >> 3, rem = nblocks & 7;
  const int lb = xcd * per + (xcd < rem ? xcd : rem) + loc;
  const int bx = lb % tiles[0];
  const int byz = lb / tiles[0];
  const int by = byz % tiles[1];
  const int bz = byz / tiles[1];
  TileOrigin o;
  o.t0[0] = bx * T::TX;
  o.t0[1] = by * T::TY;
  o.t0[2] = bz * T::TZ;
#pragma unroll
  for (int a = 0; a < 3; ++a) o.lo[a] = n[a] >= 3 ? clampi(o.t0[a] - 1, 0, n[a] - 3) : o.t0[a];
  if constexpr (T::XH == 4) o.lo[0] &= ~1;  // paired staging: boxes start at an even x
  return o;
}

// Staging of the tiles into LDS.
// The box a slot stages depends only on the axes its population is shifted
// along (its "shape": a bit per axis), so every slot of one shape and one
// population set has the same per-thread element offsets.  A thread forms
// those offsets once per shape (plan_shape: byte offsets relative to the
// tile's first halo row R0, 32 bits), and each slot's loads are then a
// workgroup-uniform base address plus these offsets, with no per-element index
// arithmetic.  2-byte storage stages x pairs: one 4-byte load per two
// elements, boxes starting at an even x.  Every thread first issues all of
// its global loads into registers, and only then writes them to LDS, so that
// a workgroup has its whole tile in flight at once.
template <int D, class T>
struct Shapes {
  using SL = Slots<D, T>;
  static constexpr int U = T::XH == 4 ? 2 : 1;  // elements per load unit
  __host__ __device__ static constexpr int of(int s) {
    return (SL::e(s, 0) != 0 ? 1 : 0) | (SL::e(s, 1) != 0 ? 2 : 0) | (SL::e(s, 2) != 0 ? 4 : 0);
  }
  __host__ __device__ static constexpr int ext(int m, int a) {
    return T::ext(a) + (((m >> a) & 1) ? (a == 0 ? T::XH : 2) : 0);
  }
  __host__ __device__ static constexpr int units(int m) { return ext(m, 0) / U * ext(m, 1) * ext(m, 2); }
  __host__ __device__ static constexpr int iters(int m) { return (units(m) + T::NT - 1) / T::NT; }
  // shape m is staged by some slot of the thermal (g) or flow (!g) set
  __host__ __device__ static constexpr bool used(int m, bool g) {
    for (int s = 0; s < SL::N; ++s)
      if (SL::isg(s) == g && of(s) == m) return true;
    return false;
  }
  // first offset of shape m in the set's offset array, and their number
  __host__ __device__ static constexpr int ooff(int m, bool g) {
    int o = 0;
    for (int k = 0; k < m; ++k)
      if (used(k, g)) o += iters(k);
    return o;
  }
  __host__ __device__ static constexpr int noff(bool g) { return ooff(8, g) > 0 ? ooff(8, g) : 1; }
  // staging registers of slot s (one per load unit)
  __host__ __device__ static constexpr int roff(int s) {
    int o = 0;
    for (int k = 0; k < s; ++k) o += iters(of(k));
    return o;
  }
  static constexpr int total = roff(SL::N);
};

// Element type of the LDS tiles.  In 3-D, 2-byte storage keeps its raw
// stored values in LDS (FP16 halves scaled by 2^12, BF16 unscaled): half the
// LDS of an FP32 tile, so four workgroups fit a CU instead of two, and no
// conversion at the commit; the FP16 pulls read a half and a float weight in
// one mixed-precision FMA and scale the interpolated value once, the BF16
// pulls widen each tap by a shift (exact, so the results are unchanged).
// Measured on 384^3: FP16 +18 %, BF16 +7.5 %; in 2-D, where LDS does not
// limit the occupancy, the 16-bit LDS reads cost 10 % on 1024^2, so 2-D
// tiles and every other storage type keep the arithmetic type in LDS.
template <int D, typename S>
struct Lds {
  using type = typename Store<S>::R;
  static constexpr bool kScaled = false;
};
template <>
struct Lds<3, __half> {
  using type = __half;
  static constexpr bool kScaled = true;
};
template <>
struct Lds<3, __hip_bfloat16> {
  using type = __hip_bfloat16;
  static constexpr bool kScaled = false;
};
template <typename R, typename L>
__device__ __forceinline__ R lv(L v) {
  if constexpr (std::is_same_v<L, __half>) return __half2float(v);
  else return R(v);
}
// w * value of an LDS entry: for FP16 tiles written as an FMA with zero so
// that it becomes one mixed-precision FMA (the sign of an exact zero is the
// only difference, and it does not survive the sums it feeds)
template <typename R, typename L>
__device__ __forceinline__ R lw(R w, L v) {
  if constexpr (std::is_same_v<L, __half>) return __builtin_fmaf(w, __half2float(v), 0.0f);
  else return w * R(v);
}

// byte address base + off (off a 32-bit byte offset): with a workgroup-uniform
// base the access takes a scalar base and a 32-bit vector offset
__device__ __forceinline__ const char* atb(const char* base, unsigned off) { return base + off; }
__device__ __forceinline__ char* atb(char* base, unsigned off) { return base + off; }

template <int D, class T, typename S, typename R, int m>
__device__ __forceinline__ void plan_shape(unsigned* offf, unsigned* offg, const KArgs<R>& a,
                                           const TileOrigin& o, unsigned R0) {
  using SH = Shapes<D, T>;
  constexpr bool UF = SH::used(m, false), UG = SH::used(m, true);
  if constexpr (UF || UG) {
    constexpr int U = SH::U, W = SH::ext(m, 0) / U, H = SH::ext(m, 1), V = SH::units(m);
    const int ox = (m & 1) ? o.lo[0] : o.t0[0];
    const int oy = (m & 2) ? o.lo[1] : o.t0[1];
    const int oz = (m & 4) ? o.lo[2] : o.t0[2];
    // last load unit of a row: a pair never starts beyond the last even x
    // (its second element then lies in the row padding, or is the last node)
    const int xmax = U == 2 ? ((a.n[0] - 1) & ~1) : a.n[0] - 1;
#pragma unroll
    for (int k = 0; k < SH::iters(m); ++k) {
      // Branch-free: positions beyond the box or the mesh are clamped to a
      // valid node; those LDS entries are never read by a pull.
      int idx = threadIdx.x + k * T::NT;
      if (V % T::NT != 0 && k + 1 == SH::iters(m)) idx = idx < V ? idx : V - 1;
      const int lz = idx / (W * H);
      const int rem = idx - lz * (W * H);
      const int ly = rem / W;
      const int lx = rem - ly * W;
      const unsigned gx = unsigned(min(ox + lx * U, xmax));
      const unsigned gy = unsigned(min(oy + ly, a.n[1] - 1));
      const unsigned gz = unsigned(min(oz + lz, a.n[2] - 1));
      // 24-bit multiplies (full rate): node counts per axis, rows of a tile's
      // span and row strides are all below 2^24
      const unsigned row = __umul24(gz, unsigned(a.n[1])) + gy - R0;
      if constexpr (UF) offf[SH::ooff(m, false) + k] = (__umul24(row, unsigned(a.rsf)) + gx) * unsigned(sizeof(S));
      if constexpr (UG) offg[SH::ooff(m, true) + k] = (__umul24(row, unsigned(a.rsg)) + gx) * unsigned(sizeof(S));
    }
  }
}

// One load unit: the stored value (converted), or for paired staging the raw
// 4 bytes of two x-neighbours.
template <typename S, bool PAIR>
struct Unit {
  using type = std::conditional_t<PAIR, unsigned, typename Store<S>::R>;
  __device__ static type ld(const char* p) {
    if constexpr (PAIR) return *reinterpret_cast<const unsigned*>(p);
    else return Store<S>::ld(reinterpret_cast<const S*>(p));
  }
};

template <int D, class T, int s, typename S, typename W, typename R>
__device__ __forceinline__ void issue_slot(W* regs, const char* fb, const char* gb, const unsigned* offf,
                                           const unsigned* offg, const KArgs<R>& a) {
  using SL = Slots<D, T>;
  using SH = Shapes<D, T>;
  constexpr int m = SH::of(s);
  constexpr bool g = SL::isg(s);
  const char* base = (g ? gb : fb) + (long long)SL::pop(s) * a.ps * (long long)sizeof(S);
  const unsigned* off = (g ? offg : offf) + SH::ooff(m, g);
#pragma unroll
  for (int k = 0; k < SH::iters(m); ++k)
    regs[SH::roff(s) + k] = Unit<S, (T::XH == 4)>::ld(atb(base, off[k]));
}

template <int D, class T, int s, typename S, typename W, typename L>
__device__ __forceinline__ void commit_slot(L* lds, const W* regs) {
  using SL = Slots<D, T>;
  using SH = Shapes<D, T>;
  constexpr int m = SH::of(s), V = SH::units(m);
  L* dst = lds + SL::off(s);
#pragma unroll
  for (int k = 0; k < SH::iters(m); ++k) {
    const int idx = threadIdx.x + k * T::NT;
    if (V % T::NT == 0 || k + 1 < SH::iters(m) || idx < V) {
      if constexpr (sizeof(L) == 2) {
        reinterpret_cast<unsigned*>(dst)[idx] = regs[SH::roff(s) + k];  // the raw pair
      } else if constexpr (T::XH == 4) {
        L lo, hi;
        Store<S>::unpack(regs[SH::roff(s) + k], lo, hi);
        reinterpret_cast<float2*>(dst)[idx] = make_float2(lo, hi);
      } else {
        dst[idx] = regs[SH::roff(s) + k];
      }
    }
  }
}

// Per-node geometry used by the pulls.
template <typename R>
struct NodeGeo {
  int g[3];       // global node
  int own[3];     // own node in an unshifted frame (g - t0)
  int ownh[3];    // own node in a shifted frame (g - lo)
  int base[3];    // clamped stencil base in the shifted frame
  R wp[3][3];     // weights, direction +1, per axis
  R wm[3][3];     // weights, direction -1, per axis
  int dep[3][2];  // uniform mesh: departure node x - e (+1, -1) in the shifted frame,
                  // clamped into the frame for links that leave the fluid
};

// Interpolated (or, on a uniform mesh, shifted) pull of one moving
// population.  Links that leave the fluid have all-zero weights and are
// overwritten by wall_slot afterwards.
template <int D, class T, int s, bool UNI, typename R, typename L>
__device__ __forceinline__ R pull_slot(const L* lds, const NodeGeo<R>& q) {
  using SL = Slots<D, T>;
  constexpr int ex = SL::e(s, 0), ey = SL::e(s, 1), ez = SL::e(s, 2);
  constexpr int W = SL::ext(s, 0), H = SL::ext(s, 1);
  constexpr int sy = W, sz = W * H;
  const L* Ls = lds + SL::off(s);
  if constexpr (UNI) {
    // departure node x - e (the clamped index keeps wall links in range)
    const int ix = ex ? q.dep[0][ex > 0 ? 0 : 1] : q.own[0];
    const int iy = ey ? q.dep[1][ey > 0 ? 0 : 1] : q.own[1];
    const int iz = ez ? q.dep[2][ez > 0 ? 0 : 1] : q.own[2];
    return lv<R>(Ls[ix + iy * sy + iz * sz]);
  } else {
    const int ix = ex ? q.base[0] : q.own[0];
    const int iy = ey ? q.base[1] : q.own[1];
    const int iz = ez ? q.base[2] : q.own[2];
    const L* P = Ls + ix + iy * sy + iz * sz;
    const R* wx = ex > 0 ? q.wp[0] : q.wm[0];
    const R* wy = ey > 0 ? q.wp[1] : q.wm[1];
    const R* wz = ez > 0 ? q.wp[2] : q.wm[2];
    constexpr int nsh = (ex != 0) + (ey != 0) + (ez != 0);
    if constexpr (nsh == 1) {
      constexpr int st = ex ? 1 : (ey ? sy : sz);
      const R* w = ex ? wx : (ey ? wy : wz);
      return lw(w[0], P[0]) + w[1] * lv<R>(P[st]) + w[2] * lv<R>(P[2 * st]);
    } else {
      // two shifted axes: first along the inner axis (virtual nodes), then
      // along the outer one (Fig. 1 two-stage construction)
      constexpr int s1 = ex ? 1 : sy;
      constexpr int s2 = ez ? sz : sy;
      const R* w1 = ex ? wx : wy;
      const R* w2 = ez ? wz : wy;
      R acc = R(0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const L* Pb = P + b * s2;
        const R v = lw(w1[0], Pb[0]) + w1[1] * lv<R>(Pb[s1]) + w1[2] * lv<R>(Pb[2 * s1]);
        acc = b == 0 ? w2[0] * v : acc + w2[b] * v;
      }
      return acc;
    }
  }
}

// Half-way wall rules for a link that leaves the fluid (Sec. 2.3):
// bounce-back for f and for g on adiabatic walls, anti-bounce-back for g on
// the isothermal x walls.
template <int D, class T, int s, typename R, typename L>
__device__ __forceinline__ void wall_slot(const L* lds, const NodeGeo<R>& q, const KArgs<R>& a, R lscale,
                                          R& val) {
  using SL = Slots<D, T>;
  constexpr int ex = SL::e(s, 0), ey = SL::e(s, 1), ez = SL::e(s, 2);
  constexpr int W = SL::ext(s, 0), H = SL::ext(s, 1);
  const bool wall = (ex == 1 && q.g[0] == 0) || (ex == -1 && q.g[0] == a.n[0] - 1) ||
                    (ey == 1 && q.g[1] == 0) || (ey == -1 && q.g[1] == a.n[1] - 1) ||
                    (ez == 1 && q.g[2] == 0) || (ez == -1 && q.g[2] == a.n[2] - 1);
  if (!wall) return;
  constexpr int so = SL::opps(s);
  const L* Lo = lds + SL::off(so);
  const int ix = ex ? q.ownh[0] : q.own[0];
  const int iy = ey ? q.ownh[1] : q.own[1];
  const int iz = ez ? q.ownh[2] : q.own[2];
  const R back = lv<R>(Lo[ix + iy * W + iz * W * H]) * lscale;
  if constexpr (SL::isg(s) && ex != 0) {
    const R Tw = (ex == 1) ? a.Thot : a.Tcold;
    val = -back + a.omega * Tw;
  } else {
    val = back;
  }
}

// lscale: factor from LDS units to values (kInv for FP16 tiles, else 1)
template <int D, class T, bool UNI, typename R, typename L, int... SS>
__device__ __forceinline__ void pull_all(const L* lds, const NodeGeo<R>& q, const KArgs<R>& a, R lscale,
                                         R* d, R* g, std::integer_sequence<int, SS...>) {
  using SL = Slots<D, T>;
  ((SL::isg(SS) ? (g[SL::pop(SS)] = pull_slot<D, T, SS, UNI>(lds, q) * lscale)
                : (d[SL::pop(SS)] = pull_slot<D, T, SS, UNI>(lds, q) * lscale)),
   ...);
  // one branch per node: only nodes next to a wall take the wall rules
  bool edge = q.g[0] == 0 || q.g[0] == a.n[0] - 1 || q.g[1] == 0 || q.g[1] == a.n[1] - 1;
  if constexpr (D == 3) edge = edge || q.g[2] == 0 || q.g[2] == a.n[2] - 1;
  if (edge) (wall_slot<D, T, SS>(lds, q, a, lscale, SL::isg(SS) ? g[SL::pop(SS)] : d[SL::pop(SS)]), ...);
}

// ---------------------------------------------------------------------------
// Reductions: per-thread accumulators, wave reductions, one partial record
// per workgroup (record slots: 0-7 and 12 FP64 sums, 8-10 maxima of |u*|,
// 11 the count of non-finite nodes).
// ---------------------------------------------------------------------------
template <typename R>
struct RedAcc {
  double v[kRedSlots];  // the sums (maxima and count slots unused here)
  R umax[3];            // max |u_a| in lattice units, in the arithmetic type
  unsigned bad;         // non-finite nodes
};

template <typename R>
__device__ __forceinline__ void red_init(RedAcc<R>& r) {
#pragma unroll
  for (int i = 0; i < kRedSlots; ++i) r.v[i] = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) r.umax[i] = R(0);
  r.bad = 0u;
}

template <typename R>
__device__ __forceinline__ void red_node(RedAcc<R>& r, const KArgs<R>& a, const int* g, const Macro<R>& m) {
  const double* red = a.red;
  const double A = red[a.red_vol[1] + g[1]] * red[a.red_vol[2] + g[2]];
  const double W = red[a.red_vol[0] + g[0]] * A;
  const double Mw = red[a.red_mw[0] + g[0]] * red[a.red_mw[1] + g[1]] * red[a.red_mw[2] + g[2]];
  const double rho = double(m.rho);
  const double us = double(m.u[0]) * a.inv_uf, vs = double(m.u[1]) * a.inv_uf,
               ws = double(m.u[2]) * a.inv_uf;
  const double Ts = (double(m.T) - a.T0) * a.inv_dT;
  r.v[0] += W * us * Ts;
  r.v[1] += W * sqrt(us * us + vs * vs + ws * ws);
  r.v[2] += W * sqrt(us * us + vs * vs);
  r.v[3] += Mw * rho;
  r.v[4] += rho;
  r.v[5] += A * red[a.red_chot + g[0]] * Ts;
  r.v[6] += A * red[a.red_ccold + g[0]] * Ts;
  r.v[7] += A * (red[a.red_cmv + g[0]] * us * Ts + red[a.red_cmd + g[0]] * Ts);
  // max |u*| = (max |u|) / u_f exactly: scaling by a positive constant and
  // rounding are both monotonic
#pragma unroll
  for (int i = 0; i < 3; ++i) r.umax[i] = fmax(r.umax[i], fabs(m.u[i]));
  const bool bad = !(isfinite(rho) && isfinite(us) && isfinite(vs) && isfinite(ws) && isfinite(Ts));
  r.bad += bad ? 1u : 0u;
  r.v[12] += W * (us * us + vs * vs + ws * ws);
}

// Cross-lane moves within rows of 16 lanes (DPP; no LDS traffic):
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
  return unsigned(__builtin_amdgcn_update_dpp(0, int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = dpp_u32<CTRL>(unsigned(b)), hi = dpp_u32<CTRL>(unsigned(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __uint_as_float(dpp_u32<CTRL>(__float_as_uint(v)));
}
template <int CTRL>
__device__ __forceinline__ unsigned dpp(unsigned v) {
  return dpp_u32<CTRL>(v);
}

// Wave-wide sum or maximum in a fixed order, the result in every lane: the
// four in-row levels by DPP moves, the two cross-row levels by shuffles.
// Each level combines a lane's value with its partner's, and x + y == y + x
// exactly, so the lanes of a pair hold the same value after every level.
template <bool MAX, typename V>
__device__ __forceinline__ V wave_reduce(V v) {
  auto op = [](V x, V y) { return MAX ? V(fmax(x, y)) : V(x + y); };
  v = op(v, dpp<kDppXor1>(v));
  v = op(v, dpp<kDppXor2>(v));
  v = op(v, dpp<kDppHalfMirror>(v));
  v = op(v, dpp<kDppMirror>(v));
  v = op(v, __shfl_xor(v, 16, 64));
  v = op(v, __shfl_xor(v, 32, 64));
  return v;
}

template <int NT, typename R>
__device__ __forceinline__ void red_block(RedAcc<R>& r, double inv_uf, double* out) {
  constexpr int NW = NT / 64;
  __shared__ double sh[NW][kRedSlots];
  double w[kRedSlots];
  w[0] = wave_reduce<false>(r.v[0]);
  w[1] = wave_reduce<false>(r.v[1]);
  w[2] = wave_reduce<false>(r.v[2]);
  w[3] = wave_reduce<false>(r.v[3]);
  w[4] = wave_reduce<false>(r.v[4]);
  w[12] = wave_reduce<false>(r.v[12]);
  // slots 5-7 are non-zero only next to the walls and the mid-plane: waves
  // with no such node skip them (a wave-uniform branch)
#pragma unroll
  for (int i = 5; i <= 7; ++i)
    w[i] = __ballot(r.v[i] != 0.0) ? wave_reduce<false>(r.v[i]) : 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) w[8 + i] = double(wave_reduce<true>(r.umax[i])) * inv_uf;
  w[11] = __ballot(r.bad != 0u) ? double(wave_reduce<false>(r.bad)) : 0.0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < kRedSlots; ++i) sh[wid][i] = w[i];
  __syncthreads();
  if (threadIdx.x < kRedSlots) {
    const int i = threadIdx.x;
    double v = sh[0][i];
    for (int k = 1; k < NW; ++k) v = (i >= 8 && i <= 10) ? fmax(v, sh[k][i]) : v + sh[k][i];
    out[i] = v;
  }
}

// ---------------------------------------------------------------------------
// The fused time step
// ---------------------------------------------------------------------------
// Per-axis weights of node j: the three weights of direction +1 (table row j)
// and of direction -1 (row n + j), each row padded to four entries, so one
// 16-byte (FP32) or two 16-byte (FP64) loads per row.
template <typename R>
__device__ __forceinline__ void load_weights(const R* tab, int n, int j, R* wp, R* wm) {
  if constexpr (std::is_same_v<R, float>) {
    const float4 p = reinterpret_cast<const float4*>(tab)[j];
    const float4 m = reinterpret_cast<const float4*>(tab)[n + j];
    wp[0] = p.x, wp[1] = p.y, wp[2] = p.z;
    wm[0] = m.x, wm[1] = m.y, wm[2] = m.z;
  } else {
    const double2* t = reinterpret_cast<const double2*>(tab);
    const double2 p0 = t[2 * j], p1 = t[2 * j + 1], m0 = t[2 * (n + j)], m1 = t[2 * (n + j) + 1];
    wp[0] = p0.x, wp[1] = p0.y, wp[2] = p1.x;
    wm[0] = m0.x, wm[1] = m0.y, wm[2] = m1.x;
  }
}

template <int D, class T, typename S, bool UNI, bool REDUCE, bool COLLIDE, bool NTS>
__global__ void __launch_bounds__(T::NT) step_kernel(const S* __restrict__ fin, const S* __restrict__ gin,
                                                     S* __restrict__ fout, S* __restrict__ gout,
                                                     KArgs<typename Store<S>::R> a) {
  using R = typename Store<S>::R;
  using SL = Slots<D, T>;
  using SH = Shapes<D, T>;
  using LF = typename SL::LF;
  using LG = typename SL::LG;
  using W = typename Unit<S, (T::XH == 4)>::type;
  using L = typename Lds<D, S>::type;
  __shared__ __align__(16) L lds[SL::total];
  // LDS units to values: 3-D FP16 tiles hold the stored (scaled) halves
  const R lscale = Lds<D, S>::kScaled ? R(1.0 / 4096.0) : R(1);
  const unsigned dkey = dither_key<S>(a);

  const TileOrigin o = tile_origin<T>(a.n, a.tiles, a.nblocks);
  // Every global address of the launch is a workgroup-uniform base at the
  // tile's first halo row R0 plus a 32-bit byte offset (the library checks
  // at create that a tile's span of rows fits 32-bit offsets).
  const unsigned R0 = unsigned(o.lo[2]) * unsigned(a.n[1]) + unsigned(o.lo[1]);
  constexpr long long SB = sizeof(S);
  const char* fb = reinterpret_cast<const char*>(fin) + (long long)R0 * a.rsf * SB;
  const char* gb = reinterpret_cast<const char*>(gin) + (long long)R0 * a.rsg * SB;

  // 1. staging offsets, once per shape; then every global load of the tile
  //    (moving populations into staging registers, rest populations and
  //    weights directly)
  unsigned offf[SH::noff(false)], offg[SH::noff(true)];
  [&]<int... MM>(std::integer_sequence<int, MM...>) {
    (plan_shape<D, T, S, R, MM>(offf, offg, a, o, R0), ...);
  }(std::make_integer_sequence<int, 8>{});
  W regs[SH::total];
  [&]<int... SS>(std::integer_sequence<int, SS...>) {
    (issue_slot<D, T, SS, S>(regs, fb, gb, offf, offg, a), ...);
  }(std::make_integer_sequence<int, SL::N>{});

  const int lx = threadIdx.x % T::TX;
  const int r0 = threadIdx.x / T::TX;
  NodeGeo<R> q;
  q.g[0] = o.t0[0] + lx;
  q.own[0] = lx;
  q.ownh[0] = q.g[0] - o.lo[0];
  const bool xin = q.g[0] < a.n[0];
  if (UNI) {
    q.dep[0][0] = q.g[0] == 0 ? q.ownh[0] : q.ownh[0] - 1;
    q.dep[0][1] = q.g[0] == a.n[0] - 1 ? q.ownh[0] : q.ownh[0] + 1;
  }
  if (!UNI && xin) {
    q.base[0] = clampi(q.g[0] - 1, 0, a.n[0] - 3) - o.lo[0];
    load_weights(a.wtab[0], a.n[0], q.g[0], q.wp[0], q.wm[0]);
  }
  // byte offset of node (x, row (ly, lz) of the tile) from R0 in a set with
  // row stride rs
  auto noff = [&](int ly, int lz, long long rs) {
    const unsigned row = __umul24(unsigned(o.t0[2] + lz), unsigned(a.n[1])) + unsigned(o.t0[1] + ly) - R0;
    return (__umul24(row, unsigned(rs)) + unsigned(q.g[0])) * unsigned(SB);
  };
  R rest_f[T::NR], rest_g[T::NR];
#pragma unroll
  for (int k = 0; k < T::NR; ++k) {
    const int row = r0 + k * T::RS;
    const int ly = row % T::TY, lz = row / T::TY;
    const int gy = o.t0[1] + ly, gz = o.t0[2] + lz;
    rest_f[k] = R(0);
    rest_g[k] = R(0);
    if (xin && gy < a.n[1] && gz < a.n[2]) {
      rest_f[k] = Store<S>::ld(reinterpret_cast<const S*>(atb(fb, noff(ly, lz, a.rsf))));
      rest_g[k] = Store<S>::ld(reinterpret_cast<const S*>(atb(gb, noff(ly, lz, a.rsg))));
    }
  }
  // 2. write the staged tiles to LDS
  [&]<int... SS>(std::integer_sequence<int, SS...>) {
    (commit_slot<D, T, SS, S>(lds, regs), ...);
  }(std::make_integer_sequence<int, SL::N>{});
  __syncthreads();

  RedAcc<R> acc;
  if constexpr (REDUCE) red_init(acc);
  char* fo = reinterpret_cast<char*>(fout) + (long long)R0 * a.rsf * SB;
  char* go = reinterpret_cast<char*>(gout) + (long long)R0 * a.rsg * SB;

#pragma unroll 1
  for (int k = 0; k < T::NR; ++k) {
    const int row = r0 + k * T::RS;
    const int ly = row % T::TY, lz = row / T::TY;
    q.g[1] = o.t0[1] + ly;
    q.g[2] = o.t0[2] + lz;
    if (!xin || q.g[1] >= a.n[1] || q.g[2] >= a.n[2]) continue;
    q.own[1] = ly;
    q.own[2] = lz;
    q.ownh[1] = q.g[1] - o.lo[1];
    q.ownh[2] = q.g[2] - o.lo[2];
    if constexpr (UNI) {
#pragma unroll
      for (int ax = 1; ax < D; ++ax) {
        q.dep[ax][0] = q.g[ax] == 0 ? q.ownh[ax] : q.ownh[ax] - 1;
        q.dep[ax][1] = q.g[ax] == a.n[ax] - 1 ? q.ownh[ax] : q.ownh[ax] + 1;
      }
    } else {
#pragma unroll
      for (int ax = 1; ax < D; ++ax) {
        q.base[ax] = clampi(q.g[ax] - 1, 0, a.n[ax] - 3) - o.lo[ax];
        load_weights(a.wtab[ax], a.n[ax], q.g[ax], q.wp[ax], q.wm[ax]);
      }
    }
    R d[LF::Q], g[LG::Q];
    d[0] = rest_f[k];
    g[0] = rest_g[k];
    pull_all<D, T, UNI>(lds, q, a, lscale, d, g, std::make_integer_sequence<int, SL::N>{});

    Macro<R> m;
    if constexpr (COLLIDE) {
      collide<D>(d, g, a.k, m);
    } else {
      // stream-only: the statistics describe the streamed (pre-collision) state
      if constexpr (REDUCE) macro_post<D>(d, g, a.k, m);
    }
    const long long mrow = (long long)q.g[2] * a.n[1] + q.g[1];
    // rounding bits keyed by the node (its index in a row-pitched mesh)
    const unsigned h0 = Store<S>::kDither ? mix32(unsigned(mrow * a.pitch + q.g[0]) ^ dkey) : 0u;
    // population i lies i rows of ps elements further (a few MB at most, so
    // the whole offset stays a 32-bit vector offset from the uniform base)
    const unsigned cf = noff(ly, lz, a.rsf), cg = noff(ly, lz, a.rsg);
    const unsigned prow = unsigned(a.ps) * unsigned(SB);
#pragma unroll
    for (int i = 0; i < LF::Q; ++i)
      store_pop<S, NTS>(reinterpret_cast<S*>(atb(fo, cf + unsigned(i) * prow)), d[i], h0, i);
#pragma unroll
    for (int i = 0; i < LG::Q; ++i)
      store_pop<S, NTS>(reinterpret_cast<S*>(atb(go, cg + unsigned(i) * prow)), g[i], h0, 32 + i);
    // after the stores, so that the FP64 statistics do not hold registers
    // while the populations are still live
    if constexpr (REDUCE) red_node(acc, a, q.g, m);
  }
  if constexpr (REDUCE) {
    const int lb = blockIdx.x;
    red_block<T::NT>(acc, a.inv_uf, a.partials + (long long)lb * kRedSlots);
  }
}

// ---------------------------------------------------------------------------
// Geometry of the 3-D z-march (imarch3d_kernel below).  A workgroup owns a
// TX x TY column of the mesh and walks along z through a segment of ZS
// planes, one node per thread per plane.  Populations without a z component
// keep one plane (plus their x/y halo) in LDS; populations with a z
// component keep a ring of three planes.
// ---------------------------------------------------------------------------
template <int TX_, int TY_, int ZS_, int XH_ = 2>
struct March {
  static constexpr int TX = TX_, TY = TY_, ZS = ZS_, NT = TX * TY;
  // slot geometry: z-shifted slots hold 3 planes; XH = 4 for 2-byte storage
  // (x-shifted boxes start at an even x and are staged as 4-byte x pairs)
  using T = Tile<TX, TY, 1, 1, XH_>;
  static constexpr int U = XH_ == 4 ? 2 : 1;  // elements per 4-byte load unit
};

template <class M>
struct MStage {
  using SL = Slots<3, typename M::T>;
  __host__ __device__ static constexpr int plane(int s) { return SL::ext(s, 0) * SL::ext(s, 1); }
};

// In-plane staging offsets of the marching kernel: a slot's plane box depends
// only on whether its population is shifted along x and along y (in-plane
// shape m = x bit | y bit), so a thread forms its 32-bit byte offsets within
// a z-plane once per shape and set (they do not change along the march);
// each plane's loads are then a workgroup-uniform plane base plus these
// offsets.  Every load moves one 4-byte unit (one element, or an x pair of
// 2-byte elements).
template <class M>
struct MShapes {
  using SL = Slots<3, typename M::T>;
  __host__ __device__ static constexpr int of(int s) { return (SL::e(s, 0) != 0 ? 1 : 0) | (SL::e(s, 1) != 0 ? 2 : 0); }
  __host__ __device__ static constexpr int w(int m) { return M::TX + ((m & 1) ? M::T::XH : 0); }
  __host__ __device__ static constexpr int h(int m) { return M::TY + ((m & 2) ? 2 : 0); }
  __host__ __device__ static constexpr int units(int m) { return w(m) / M::U * h(m); }
  __host__ __device__ static constexpr int iters(int m) { return (units(m) + M::NT - 1) / M::NT; }
  __host__ __device__ static constexpr int ooff(int m) {
    int o = 0;
    for (int k = 0; k < m; ++k) o += iters(k);
    return o;
  }
  static constexpr int total = ooff(4);
};

template <class M, typename S, typename R>
__device__ __forceinline__ void mplan(unsigned* offf, unsigned* offg, const KArgs<R>& a, const TileOrigin& o) {
  using MSH = MShapes<M>;
  constexpr int U = M::U;
  // last load unit of a row: a pair never starts beyond the last even x
  const int xmax = U == 2 ? ((a.n[0] - 1) & ~1) : a.n[0] - 1;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int W = MSH::w(m) / U, V = MSH::units(m);
    const int ox = (m & 1) ? o.lo[0] : o.t0[0];
    const int oy = (m & 2) ? o.lo[1] : o.t0[1];
#pragma unroll
    for (int k = 0; k < MSH::iters(m); ++k) {
      int idx = threadIdx.x + k * M::NT;
      idx = idx < V ? idx : V - 1;
      const int ly = idx / W;
      const int lx = idx - ly * W;
      const unsigned gx = unsigned(min(ox + lx * U, xmax));
      const unsigned gy = unsigned(min(oy + ly, a.n[1] - 1));
      offf[MSH::ooff(m) + k] = (__umul24(gy, unsigned(a.rsf)) + gx) * unsigned(sizeof(S));
      offg[MSH::ooff(m) + k] = (__umul24(gy, unsigned(a.rsg)) + gx) * unsigned(sizeof(S));
    }
  }
}

// ---------------------------------------------------------------------------
// 3-D marching kernel (plain launches; FP32 storage, and 2-byte storage on
// uniform meshes): the column and plane ring above, with the interpolated
// pulls of step_kernel (or, on a uniform mesh, the shift by one node).
// The ring already holds the three stencil planes zb .. zb + 2 of plane z
// (zb = clamp(z - 1, 0, nz - 3)), so z halos are read once per column.  The
// planes are staged with direct global -> LDS loads (lane l of a wave writes
// the wave's LDS base + 4 l), which need no staging registers: after the
// pulls of plane z (and a barrier) the next plane's loads are issued into the
// freed slots and land while plane z collides and is stored.  Measured on
// 256^3 / 384^3 tanh meshes: 22.9k / 22.6k MLUPS against 20.6k / 20.2k for
// step_kernel's 32 x 4 x 4 tiles.
// ---------------------------------------------------------------------------
// A workgroup-uniform plane base made opaque to the optimiser (kept in
// scalar registers): otherwise it splits base + z * stride + offset and
// hoists base + offset out of the z loop as one 64-bit vector address per
// population and load unit, far more registers than the march can hold.
// (The value must be the same in every lane: it is read from the first
// active one.)  The rebuilt pointer is marked as global memory, so that its
// loads and stores stay global ones (scalar base + 32-bit vector offset)
// rather than flat ones with a 64-bit vector address each.
template <typename P>
__device__ __forceinline__ P opaque_base(P p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(v));
  const unsigned hi = __builtin_amdgcn_readfirstlane(unsigned(v >> 32));
  using G = __attribute__((address_space(1))) char*;
  const G g = reinterpret_cast<G>((static_cast<unsigned long long>(hi) << 32) | lo);
  return (P)((char*)g);
}

typedef __attribute__((address_space(4))) const float CFloat;  // constant (scalar-cache) memory

struct IGeo {
  int g[3];
  int own[2];       // own node in an unshifted x/y frame
  int ownh[2];      // own node in a shifted x/y frame
  int base[2];      // clamped x/y stencil base in the shifted frame
  float wp[3][3];   // weights, direction +1, per axis (z: of the current plane)
  float wm[3][3];   // weights, direction -1
  int ring[3];      // ring slots of the stencil planes zb, zb + 1, zb + 2
  int ringown;      // ring slot of plane z
  int dep[2][2];    // uniform mesh: departure node x - e (+1, -1) in the shifted x/y frame,
                    // clamped into the frame for links that leave the fluid
  int ringdep[2];   // uniform mesh: ring slot of plane z - 1 (+1) and z + 1 (-1), clamped
};

// L: the LDS element type (float, or the raw stored values of 2-byte storage,
// read through lv / lw as in step_kernel; the caller applies the scale)
template <class M, int s, bool UNI, typename L>
__device__ __forceinline__ float ipull_slot(const L* lds, const IGeo& q) {
  using SL = Slots<3, typename M::T>;
  constexpr int ex = SL::e(s, 0), ey = SL::e(s, 1), ez = SL::e(s, 2);
  constexpr int W = SL::ext(s, 0), P = MStage<M>::plane(s);
  if constexpr (UNI) {
    // departure node x - e (the clamped indices keep wall links in range)
    const int ix = ex ? q.dep[0][ex > 0 ? 0 : 1] : q.own[0];
    const int iy = ey ? q.dep[1][ey > 0 ? 0 : 1] : q.own[1];
    const int iz = ez ? q.ringdep[ez > 0 ? 0 : 1] : 0;
    return lv<float>(lds[SL::off(s) + ix + iy * W + iz * P]);
  }
  const int ix = ex ? q.base[0] : q.own[0];
  const int iy = ey ? q.base[1] : q.own[1];
  const L* Pxy = lds + SL::off(s) + ix + iy * W;
  const float* wx = ex > 0 ? q.wp[0] : q.wm[0];
  const float* wy = ey > 0 ? q.wp[1] : q.wm[1];
  const float* wz = ez > 0 ? q.wp[2] : q.wm[2];
  constexpr int nsh = (ex != 0) + (ey != 0) + (ez != 0);
  if constexpr (nsh == 1 && ez == 0) {
    constexpr int st = ex ? 1 : W;
    const float* w = ex ? wx : wy;
    return lw(w[0], Pxy[0]) + w[1] * lv<float>(Pxy[st]) + w[2] * lv<float>(Pxy[2 * st]);
  } else if constexpr (nsh == 1) {
    return lw(wz[0], Pxy[q.ring[0] * P]) + wz[1] * lv<float>(Pxy[q.ring[1] * P]) +
           wz[2] * lv<float>(Pxy[q.ring[2] * P]);
  } else if constexpr (ez == 0) {
    // x and y: inner axis x, outer y (as in step_kernel)
    float acc = 0.0f;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const L* Pb = Pxy + b * W;
      const float v = lw(wx[0], Pb[0]) + wx[1] * lv<float>(Pb[1]) + wx[2] * lv<float>(Pb[2]);
      acc = b == 0 ? wy[0] * v : acc + wy[b] * v;
    }
    return acc;
  } else {
    // x or y with z: the in-plane axis first, then z across the ring
    constexpr int s1 = ex ? 1 : W;
    const float* w1 = ex ? wx : wy;
    float acc = 0.0f;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const L* Pb = Pxy + q.ring[b] * P;
      const float v = lw(w1[0], Pb[0]) + w1[1] * lv<float>(Pb[s1]) + w1[2] * lv<float>(Pb[2 * s1]);
      acc = b == 0 ? wz[0] * v : acc + wz[b] * v;
    }
    return acc;
  }
}

template <class M, int s, typename L>
__device__ __forceinline__ void iwall_slot(const L* lds, const IGeo& q, const KArgs<float>& a, float lscale,
                                           float& val) {
  using SL = Slots<3, typename M::T>;
  constexpr int ex = SL::e(s, 0), ey = SL::e(s, 1), ez = SL::e(s, 2);
  const bool wall = (ex == 1 && q.g[0] == 0) || (ex == -1 && q.g[0] == a.n[0] - 1) ||
                    (ey == 1 && q.g[1] == 0) || (ey == -1 && q.g[1] == a.n[1] - 1) ||
                    (ez == 1 && q.g[2] == 0) || (ez == -1 && q.g[2] == a.n[2] - 1);
  if (!wall) return;
  constexpr int so = SL::opps(s);
  constexpr int W = SL::ext(so, 0), P = MStage<M>::plane(so);
  const int ix = ex ? q.ownh[0] : q.own[0];
  const int iy = ey ? q.ownh[1] : q.own[1];
  const int iz = ez ? q.ringown : 0;
  const float back = lv<float>(lds[SL::off(so) + ix + iy * W + iz * P]) * lscale;
  if constexpr (SL::isg(s) && ex != 0) {
    const float Tw = (ex == 1) ? a.Thot : a.Tcold;
    val = -back + a.omega * Tw;
  } else {
    val = back;
  }
}

template <class M, bool UNI, typename L, int... SS>
__device__ __forceinline__ void ipull_all(const L* lds, const IGeo& q, const KArgs<float>& a, float lscale,
                                          float* d, float* g, std::integer_sequence<int, SS...>) {
  using SL = Slots<3, typename M::T>;
  ((SL::isg(SS) ? (g[SL::pop(SS)] = ipull_slot<M, SS, UNI>(lds, q) * lscale)
                : (d[SL::pop(SS)] = ipull_slot<M, SS, UNI>(lds, q) * lscale)),
   ...);
  const bool edge = q.g[0] == 0 || q.g[0] == a.n[0] - 1 || q.g[1] == 0 || q.g[1] == a.n[1] - 1 ||
                    q.g[2] == 0 || q.g[2] == a.n[2] - 1;
  if (edge) (iwall_slot<M, SS>(lds, q, a, lscale, SL::isg(SS) ? g[SL::pop(SS)] : d[SL::pop(SS)]), ...);
}

// Direct global -> LDS staging of one slot's plane gz into ring slot `ring`
// (slots without a z component have one plane).  Lanes past the plane box
// stay idle; a wave's 64 lanes write 64 consecutive LDS entries.
template <class M, int s, typename S, typename L>
__device__ __forceinline__ void dma_plane(L* lds, const S* __restrict__ fin, const S* __restrict__ gin,
                                          const unsigned* offf, const unsigned* offg, const KArgs<float>& a,
                                          int gz, int ring) {
  using SL = Slots<3, typename M::T>;
  using MS = MStage<M>;
  using MSH = MShapes<M>;
  constexpr int m = MSH::of(s), V = MSH::units(m);
  const bool g = SL::isg(s);
  const long long rs = g ? a.rsg : a.rsf;
  const char* base = opaque_base(reinterpret_cast<const char*>((g ? gin : fin) + (long long)SL::pop(s) * a.ps +
                                                               (long long)gz * a.n[1] * rs));
  const unsigned* off = (g ? offg : offf) + MSH::ooff(m);
  // 4-byte load units of this slot's plane (one element, or an x pair)
  unsigned* dst = reinterpret_cast<unsigned*>(lds + SL::off(s) + (SL::e(s, 2) != 0 ? ring * MS::plane(s) : 0)) +
                  (threadIdx.x & ~63);
#pragma unroll
  for (int k = 0; k < MSH::iters(m); ++k) {
    const int idx = threadIdx.x + k * M::NT;
    if (V % M::NT == 0 || k + 1 < MSH::iters(m) || idx < V)
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(atb(base, off[k])), dst + k * M::NT, 4, 0,
                                       0);
  }
}

template <class M, bool ZC, typename S, typename L, int... SS>
__device__ __forceinline__ void dma_class(L* lds, const S* fin, const S* gin, const unsigned* offf,
                                          const unsigned* offg, const KArgs<float>& a, int gz, int ring,
                                          std::integer_sequence<int, SS...>) {
  using SL = Slots<3, typename M::T>;
  ([&] {
    if constexpr ((SL::e(SS, 2) != 0) == ZC) dma_plane<M, SS>(lds, fin, gin, offf, offg, a, gz, ring);
  }(), ...);
}

// wait for this thread's direct-to-LDS loads (vmcnt(0)); the barrier that
// follows makes every wave's loads visible
__device__ __forceinline__ void dma_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

template <class M, typename S, bool UNI, bool NTS>
__global__ void __launch_bounds__(M::NT) imarch3d_kernel(const S* __restrict__ fin, const S* __restrict__ gin,
                                                         S* __restrict__ fout, S* __restrict__ gout,
                                                         KArgs<float> a) {
  using R = float;
  static_assert(std::is_same_v<typename Store<S>::R, float>, "FP32 arithmetic");
  // LDS holds the stored values unchanged: float, or the raw 2-byte values
  // (FP16 scaled by 2^12, BF16 unscaled), converted at each pull
  using L = std::conditional_t<sizeof(S) == 2, S, typename Store<S>::R>;
  static_assert(sizeof(L) == sizeof(S), "the plane loads copy stored values into LDS unchanged");
  static_assert((M::U == 2) == (sizeof(S) == 2), "2-byte storage is staged in x pairs");
  const R lscale = Lds<3, S>::kScaled ? R(1.0 / 4096.0) : R(1);
  using SL = Slots<3, typename M::T>;
  using LF = typename SL::LF;
  using LG = typename SL::LG;
  __shared__ __attribute__((aligned(16))) L lds[SL::total];
  const unsigned dkey = dither_key<S>(a);
  constexpr auto slots = std::make_integer_sequence<int, SL::N>{};

  // column and z segment of this workgroup (XCD-aware numbering as in step_kernel)
  const int b = blockIdx.x;
  const int xcd = b & 7, loc = b >> 3;
  const int per = a.nblocks >> 3, rem = a.nblocks & 7;
  const int lb = xcd * per + (xcd < rem ? xcd : rem) + loc;
  const int cols = a.tiles[0] * a.tiles[1];
  const int col = lb % cols, seg = lb / cols;
  TileOrigin o;
  o.t0[0] = (col % a.tiles[0]) * M::TX;
  o.t0[1] = (col / a.tiles[0]) * M::TY;
  o.t0[2] = 0;
  o.lo[0] = clampi(o.t0[0] - 1, 0, a.n[0] - 3);
  if constexpr (M::U == 2) o.lo[0] &= ~1;  // paired staging: boxes start at an even x
  o.lo[1] = clampi(o.t0[1] - 1, 0, a.n[1] - 3);
  o.lo[2] = 0;
  const int nz = a.n[2];
  const int z0 = seg * M::ZS;
  const int z1 = min(nz, z0 + M::ZS);

  IGeo q;
  const int lx = threadIdx.x % M::TX, ly = threadIdx.x / M::TX;
  q.g[0] = o.t0[0] + lx;
  q.g[1] = o.t0[1] + ly;
  q.own[0] = lx;
  q.own[1] = ly;
  q.ownh[0] = q.g[0] - o.lo[0];
  q.ownh[1] = q.g[1] - o.lo[1];
  const bool in = q.g[0] < a.n[0] && q.g[1] < a.n[1];
  if (in) {
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
      if constexpr (UNI) {
        q.dep[ax][0] = q.g[ax] == 0 ? q.ownh[ax] : q.ownh[ax] - 1;
        q.dep[ax][1] = q.g[ax] == a.n[ax] - 1 ? q.ownh[ax] : q.ownh[ax] + 1;
      } else {
        q.base[ax] = clampi(q.g[ax] - 1, 0, a.n[ax] - 3) - o.lo[ax];
        load_weights(a.wtab[ax], a.n[ax], q.g[ax], q.wp[ax], q.wm[ax]);
      }
    }
  }
  // every global access is a workgroup-uniform base (plane z of one
  // population, in scalar registers) plus the thread's 32-bit in-plane byte
  // offset, so no per-population 64-bit address stays live across the march
  const unsigned gy0 = in ? unsigned(q.g[1]) : 0u, gx0 = in ? unsigned(q.g[0]) : 0u;
  constexpr unsigned SB = sizeof(S);
  unsigned cxyf = (__umul24(gy0, unsigned(a.rsf)) + gx0) * SB, cxyg = (__umul24(gy0, unsigned(a.rsg)) + gx0) * SB;
  const long long zsf = (long long)a.n[1] * a.rsf * SB, zsg = (long long)a.n[1] * a.rsg * SB;
  const long long ps4 = (long long)a.ps * SB;
  const char* const fi = reinterpret_cast<const char*>(fin);
  const char* const gi = reinterpret_cast<const char*>(gin);
  char* const fo = reinterpret_cast<char*>(fout);
  char* const go = reinterpret_cast<char*>(gout);

  // in-plane staging offsets (once), then the prologue: the three stencil
  // planes of z0 and the x/y planes of z0
  unsigned offf[MShapes<M>::total], offg[MShapes<M>::total];
  mplan<M, S, R>(offf, offg, a, o);
  const int zb0 = clampi(z0 - 1, 0, nz - 3);
#pragma unroll 1
  for (int p = 0; p < 3; ++p) dma_class<M, true>(lds, fin, gin, offf, offg, a, zb0 + p, (zb0 + p) % 3, slots);
  dma_class<M, false>(lds, fin, gin, offf, offg, a, z0, 0, slots);
  R rf = Store<S>::ld(reinterpret_cast<const S*>(atb(opaque_base(fi + z0 * zsf), cxyf)));
  R rg = Store<S>::ld(reinterpret_cast<const S*>(atb(opaque_base(gi + z0 * zsg), cxyg)));
  dma_wait();
  __syncthreads();

#pragma unroll 1
  for (int z = z0; z < z1; ++z) {
    const bool more = z + 1 < z1;
    const int zb = clampi(z - 1, 0, nz - 3);
    const int zbn = clampi(z, 0, nz - 3);
    const bool newz = more && zbn > zb;
    // the 32-bit in-plane offsets are redefined (unchanged) each plane, so
    // that their 64-bit extensions are not hoisted out of the loop: every
    // access then keeps the scalar-base + 32-bit-offset form
    asm volatile("" : "+v"(cxyf), "+v"(cxyg));
#pragma unroll
    for (int k = 0; k < MShapes<M>::total; ++k) asm volatile("" : "+v"(offf[k]), "+v"(offg[k]));
    R d[LF::Q], g[LG::Q];
    // z weights of the plane: uniform, read through the scalar cache (a
    // vector load here would make its wait also wait for the previous
    // plane's stores, which complete in order with it)
    if constexpr (!UNI) {
      const CFloat* wz = (const CFloat*)(opaque_base(a.wtab[2]));  // 4 floats per node and direction
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        q.wp[2][i] = wz[4 * z + i];
        q.wm[2][i] = wz[4 * (nz + z) + i];
      }
    }
    if (in) {
      q.g[2] = z;
      q.ringown = z % 3;
#pragma unroll
      for (int i = 0; i < 3; ++i) q.ring[i] = (zb + i) % 3;
      q.ringdep[0] = z == 0 ? q.ringown : (z - 1) % 3;
      q.ringdep[1] = z == nz - 1 ? q.ringown : (z + 1) % 3;
      d[0] = rf;
      g[0] = rg;
      // an opaque zero added to the LDS base each plane keeps the compiler
      // from hoisting plane-invariant tap addresses out of the z loop (about
      // 20 fewer VGPRs)
      int zero = 0;
      asm volatile("" : "+v"(zero));
      ipull_all<M, UNI>(lds + zero, q, a, lscale, d, g, slots);
    }
    // the rest populations of the next plane come straight to registers
    R nf = R(0), ng = R(0);
    if (more) {
      nf = Store<S>::ld(reinterpret_cast<const S*>(atb(opaque_base(fi + (z + 1) * zsf), cxyf)));
      ng = Store<S>::ld(reinterpret_cast<const S*>(atb(opaque_base(gi + (z + 1) * zsg), cxyg)));
    }
    __syncthreads();  // every pull of plane z has read the slots refilled next
    if (more) dma_class<M, false>(lds, fin, gin, offf, offg, a, z + 1, 0, slots);
    if (newz) dma_class<M, true>(lds, fin, gin, offf, offg, a, zbn + 2, (zbn + 2) % 3, slots);
    if (in) {
      Macro<R> m;
      collide<3>(d, g, a.k, m);
      char* const fz = opaque_base(fo + z * zsf);
      char* const gz = opaque_base(go + z * zsg);
      // rounding bits keyed by the node (its index in a row-pitched mesh), as in step_kernel
      const unsigned h0 =
          Store<S>::kDither ? mix32(unsigned(((long long)z * a.n[1] + q.g[1]) * a.pitch + q.g[0]) ^ dkey) : 0u;
#pragma unroll
      for (int i = 0; i < LF::Q; ++i)
        store_pop<S, NTS>(reinterpret_cast<S*>(atb(fz + i * ps4, cxyf)), d[i], h0, i);
#pragma unroll
      for (int i = 0; i < LG::Q; ++i)
        store_pop<S, NTS>(reinterpret_cast<S*>(atb(gz + i * ps4, cxyg)), g[i], h0, 32 + i);
    }
    rf = nf;
    rg = ng;
    dma_wait();
    __syncthreads();
  }
}

// Tile shapes per lattice, arithmetic width and working-set class (TX x TY x
// TZ nodes, NR nodes per thread).  "Large" means the two population buffers
// do not fit the 256 MB last-level cache: those launches use larger 2-D
// tiles with two rows per thread (fewer halo re-reads) and streaming stores;
// cache-resident meshes use small tiles (more workgroups per CU) and
// ordinary stores.  Shapes are from sweeps on MI355X.
template <int D, typename R, bool LARGE>
struct TileFor;
template <>
struct TileFor<2, float, false> {
  using T = Tile<64, 4, 1, 1>;
};
template <>
struct TileFor<2, float, true> {
  using T = Tile<128, 4, 1, 2>;
};
template <bool L>
struct TileFor<2, double, L> {
  using T = Tile<64, 4, 1, 1>;
};
template <bool L>
struct TileFor<3, float, L> {
  using T = Tile<32, 4, 4, 1>;
};
template <bool L>
struct TileFor<3, double, L> {
  using T = Tile<16, 4, 4, 1>;
};

template <int D, class T>
static int grid_of(const DevState& s, int* tiles) {
  tiles[0] = (s.n[0] + T::TX - 1) / T::TX;
  tiles[1] = (s.n[1] + T::TY - 1) / T::TY;
  tiles[2] = (s.n[2] + T::TZ - 1) / T::TZ;
  return tiles[0] * tiles[1] * tiles[2];
}

// 2-byte storage stages x pairs (Tile XH = 4) and in 2-D keeps the short
// 64 x 4 tiles also for large meshes (measured 13 % faster there than 64 x 8
// tiles with two rows per thread).  In 3-D its LDS tiles hold the raw 2-byte
// values, and wide flat 64 x 2 x 2 tiles (256 threads, 27 KB of LDS) beat
// the FP32 shape: FP16 32.8k / 34.2k MLUPS on 256^3 / 384^3 tanh meshes
// against 30.3k / 31.2k in 32 x 4 x 4 (BF16 31.0k against 28.3k on 384^3;
// 64 x 2 x 4 31.8k / 32.9k, 64 x 4 x 2 31.5k / 32.3k, 128 x 2 x 2 29.6k /
// 31.0k, 32 x 4 x 2 28.8k / 29.4k); on the 400^3 erf mesh 30.3k against
// 29.8k.
template <class T>
struct Paired;
template <int TX, int TY, int TZ, int NR, int XH>
struct Paired<Tile<TX, TY, TZ, NR, XH>> {
  using type = Tile<TX, TY, TZ, NR, 4>;
};
template <int D, typename S, bool LARGE>
struct TileSel {
  using T0 = typename TileFor<D, typename Store<S>::R, LARGE>::T;
  using T = std::conditional_t<sizeof(S) == 2, typename Paired<T0>::type, T0>;
};
template <bool L>
struct TileSel<2, __half, L> {
  using T = Tile<64, 4, 1, 1, 4>;
};
template <bool L>
struct TileSel<2, __hip_bfloat16, L> {
  using T = Tile<64, 4, 1, 1, 4>;
};
using Tile3Pair = Tile<64, 2, 2, 1, 4>;
template <bool L>
struct TileSel<3, __half, L> {
  using T = Tile3Pair;
};
template <bool L>
struct TileSel<3, __hip_bfloat16, L> {
  using T = Tile3Pair;
};

template <int D, typename S, bool LARGE, bool UNI, bool RED, bool COL>
static hipError_t launch_step_t(const DevState& s, const void* fin, const void* gin, void* fout,
                                void* gout, double* partials, hipStream_t st) {
  using R = typename Store<S>::R;
  using T = typename TileSel<D, S, LARGE>::T;
  KArgs<R> a = make_args<R>(s);
  const int nb = grid_of<D, T>(s, a.tiles);
  a.nblocks = nb;
  a.partials = partials;
  hipLaunchKernelGGL((step_kernel<D, T, S, UNI, RED, COL, LARGE>), dim3(nb), dim3(T::NT), 0, st,
                     static_cast<const S*>(fin), static_cast<const S*>(gin), static_cast<S*>(fout),
                     static_cast<S*>(gout), a);
  return hipGetLastError();
}

template <int D, typename S, bool LARGE>
static hipError_t dispatch_step(const DevState& s, const void* fin, const void* gin, void* fout,
                                void* gout, bool reduce, double* partials, hipStream_t st) {
  const bool uni = s.uniform != 0, col = s.collide != 0;
  if (col) {
    if (uni)
      return reduce ? launch_step_t<D, S, LARGE, true, true, true>(s, fin, gin, fout, gout, partials, st)
                    : launch_step_t<D, S, LARGE, true, false, true>(s, fin, gin, fout, gout, partials, st);
    return reduce ? launch_step_t<D, S, LARGE, false, true, true>(s, fin, gin, fout, gout, partials, st)
                  : launch_step_t<D, S, LARGE, false, false, true>(s, fin, gin, fout, gout, partials, st);
  }
  return reduce ? launch_step_t<D, S, LARGE, false, true, false>(s, fin, gin, fout, gout, partials, st)
                : launch_step_t<D, S, LARGE, false, false, false>(s, fin, gin, fout, gout, partials, st);
}

// 3-D meshes with collision use the marching kernel for their plain launches
// with FP32 storage, and with FP16 or BF16 storage on uniform meshes (below);
// the FP64-arithmetic modes keep the tile kernel.  64 x 8 columns, 32
// planes per segment, one 512-thread workgroup per CU (110 KB of LDS for
// FP32).  Measured on 256^3 / 384^3 tanh meshes (MLUPS; FETCH_SIZE
// over the algorithmic reads on 256^3): 64 x 8 x 32 22.9k / 22.6k, 1.04x;
// 32 x 8 x 32 20.6k / 22.1k, 1.32x; 32 x 16 x 32 20.6k / 21.3k, 1.14x;
// 32 x 8 x 64 19.9k / 21.5k; 32 x 4 x 32 20.3k / 21.9k.  Wider rows leave
// fewer x-halo cache lines and y-halo rows to fetch beyond L2.
using IMarch3 = March<64, 8, 32>;

template <class M>
static int imarch_grid(const DevState& s, int* tiles) {
  tiles[0] = (s.n[0] + M::TX - 1) / M::TX;
  tiles[1] = (s.n[1] + M::TY - 1) / M::TY;
  tiles[2] = (s.n[2] + M::ZS - 1) / M::ZS;
  return tiles[0] * tiles[1] * tiles[2];
}

// 2-byte storage marches on uniform meshes only, in 64 x 4 columns (raw
// stored pairs staged into 2-byte LDS; 30 KB of LDS and about 80 VGPRs, five
// workgroups per CU).  FP16: 38.2k / 42.5k MLUPS on 256^3 / 384^3 against
// 36.7k / 39.1k in 64 x 8 columns and 31.3k / 32.4k for the tile kernel;
// BF16: 38.2k / 42.9k against 28.8k / 29.2k for the tile kernel (then with
// float LDS tiles).  The interpolating FP16 form ran 30.7k / 31.7k on tanh
// meshes in 64 x 8 columns (107 VGPRs once the pulls were fenced in groups
// of slots, 220 without) and 16.4k / 17.3k in 64 x 4, against 30.6k / 31.1k
// for the tile kernel, which stretched 2-byte meshes keep.
static bool use_imarch(const DevState& s) {
  return s.dim == 3 && s.collide != 0 && (s.storage == 0 || ((s.storage == 2 || s.storage == 3) && s.uniform != 0));
}

// Plain launches only: the statistics of the reducing launch would hold 13
// FP64 accumulators across the march and push it beyond 256 VGPRs, so that
// launch stays with step_kernel (once per call).
template <typename S>
using IMarchFor = std::conditional_t<sizeof(S) == 2, March<64, 4, 32, 4>, IMarch3>;

// FP32 on uniform meshes marches in 128 x 4 columns of 64 planes where they
// pad x no further than 64-wide columns (bitwise the same result): 25.7k /
// 25.1k MLUPS on 256^3 / 384^3 against 23.9k / 24.8k in 64 x 8 x 32; on 400^3
// (x padded to 512 instead of 448) 21.2k against 23.3k.
using IMarchU = March<128, 4, 64>;
static bool wide_columns(const DevState& s) {
  return (s.n[0] + 127) / 128 * 128 <= (s.n[0] + 63) / 64 * 64;
}

template <class M, typename S, bool UNI, bool LARGE>
static hipError_t launch_march_as(const DevState& s, const void* fin, const void* gin, void* fout, void* gout,
                                  hipStream_t st) {
  KArgs<float> a = make_args<float>(s);
  a.nblocks = imarch_grid<M>(s, a.tiles);
  hipLaunchKernelGGL((imarch3d_kernel<M, S, UNI, LARGE>), dim3(a.nblocks), dim3(M::NT), 0, st,
                     static_cast<const S*>(fin), static_cast<const S*>(gin), static_cast<S*>(fout),
                     static_cast<S*>(gout), a);
  return hipGetLastError();
}

template <typename S, bool LARGE>
static hipError_t launch_imarch(const DevState& s, const void* fin, const void* gin, void* fout, void* gout,
                                hipStream_t st) {
  using M = IMarchFor<S>;
  if (s.uniform) {
    if constexpr (sizeof(S) == 4)
      if (wide_columns(s)) return launch_march_as<IMarchU, S, true, LARGE>(s, fin, gin, fout, gout, st);
    return launch_march_as<M, S, true, LARGE>(s, fin, gin, fout, gout, st);
  }
  if constexpr (sizeof(S) == 4) return launch_march_as<M, S, false, LARGE>(s, fin, gin, fout, gout, st);
  return hipErrorInvalidValue;  // not dispatched: use_imarch takes 2-byte storage on uniform meshes only
}

template <typename Fn>
static hipError_t by_storage(int storage, int dim, Fn&& fn) {
  (void)dim;
  switch (storage) {
    case 0: return fn(float{});
    case 1: return fn(double{});
    case 2: return fn(__half{});
    case 3: return fn(__hip_bfloat16{});
    case 4: return fn(f32s{});
    default: return hipErrorInvalidValue;
  }
}

template <int D, typename R, bool LARGE>
static int blocks_for(const DevState& s) {
  int tiles[3];
  return grid_of<D, typename TileFor<D, R, LARGE>::T>(s, tiles);
}

int step_blocks(const DevState& s) {
  const bool dbl = s.storage == 1 || s.storage == 4, lg = s.large != 0;
  if (s.dim == 2) {
    if (dbl) return blocks_for<2, double, false>(s);
    if (lg && (s.storage == 2 || s.storage == 3)) {
      int tiles[3];
      return grid_of<2, typename TileSel<2, __half, true>::T>(s, tiles);
    }
    return lg ? blocks_for<2, float, true>(s) : blocks_for<2, float, false>(s);
  }
  if (dbl) return blocks_for<3, double, false>(s);
  if (s.storage == 2 || s.storage == 3) {
    int tiles[3];
    return grid_of<3, Tile3Pair>(s, tiles);
  }
  return lg ? blocks_for<3, float, true>(s) : blocks_for<3, float, false>(s);
}

hipError_t launch_step(const DevState& s, const void* fin, const void* gin, void* fout, void* gout,
                       bool reduce, double* partials, hipStream_t st) {
  return by_storage(s.storage, s.dim, [&](auto tag) {
    using S = decltype(tag);
    if constexpr (std::is_same_v<typename Store<S>::R, double>) {
      // FP64 arithmetic: same tiles in both classes; streaming stores only
      // for working sets far beyond the cache (just beyond it they cost 36 %
      // at 1024^2, above 1 GB they gain 2-6 %)
      if (s.large >= 2)
        return s.dim == 2 ? dispatch_step<2, S, true>(s, fin, gin, fout, gout, reduce, partials, st)
                          : dispatch_step<3, S, true>(s, fin, gin, fout, gout, reduce, partials, st);
      return s.dim == 2 ? dispatch_step<2, S, false>(s, fin, gin, fout, gout, reduce, partials, st)
                        : dispatch_step<3, S, false>(s, fin, gin, fout, gout, reduce, partials, st);
    } else {
      if constexpr (std::is_same_v<S, float> || std::is_same_v<S, __half> || std::is_same_v<S, __hip_bfloat16>)
        if (use_imarch(s) && !reduce)
          return s.large ? launch_imarch<S, true>(s, fin, gin, fout, gout, st)
                         : launch_imarch<S, false>(s, fin, gin, fout, gout, st);
      if (s.dim == 3)
        return s.large ? dispatch_step<3, S, true>(s, fin, gin, fout, gout, reduce, partials, st)
                       : dispatch_step<3, S, false>(s, fin, gin, fout, gout, reduce, partials, st);
      return s.large ? dispatch_step<2, S, true>(s, fin, gin, fout, gout, reduce, partials, st)
                     : dispatch_step<2, S, false>(s, fin, gin, fout, gout, reduce, partials, st);
    }
  });
}

// ---------------------------------------------------------------------------
// Per-node helper kernels (set-up, I/O, statistics of a stored state)
// ---------------------------------------------------------------------------
// Element of node `node` (x fastest) in the row of population 0, for a
// buffer whose rows of one population are `rs` elements apart.
__device__ __forceinline__ long long pitched(long long node, const int* n, long long rs) {
  const long long x = node % n[0];
  const long long yz = node / n[0];
  return yz * rs + x;
}

__global__ void fill_zero_kernel(unsigned int* p, size_t words) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t words = bytes / 4;
  const int nb = (int)((words + 255) / 256 < 65536 ? (words + 255) / 256 : 65536);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(nb > 0 ? nb : 1), dim3(256), 0, st,
                     static_cast<unsigned int*>(p), words);
  return hipGetLastError();
}

// Plain device copy (a measured bandwidth ceiling for streaming kernels; not
// part of the step): one 16-byte vector per thread, non-temporal load and
// store, 256-thread workgroups over the whole range.  Of the variants timed
// on MI355X for 1 GiB (one, two, four or eight vectors per thread, grid-stride
// loops, 256-1024 threads), this one moved the most bytes (6.5 TB/s read +
// write; 6.2 TB/s with ordinary loads and stores).
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) copy16_kernel(u32x4_t* __restrict__ dst, const u32x4_t* __restrict__ src,
                                                     size_t n) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  const size_t nb = (n + 255) / 256;
  if (nb > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy16_kernel, dim3((unsigned)nb), dim3(256), 0, st, static_cast<u32x4_t*>(dst),
                     static_cast<const u32x4_t*>(src), n);
  return hipGetLastError();
}

template <int D>
__host__ __device__ double flow_weight(int i) {
  return D == 2 ? D2Q9::w(i) : D3Q19::w(i);
}

template <int D, typename S>
__global__ void convert_in_kernel(const double* __restrict__ src, S* __restrict__ dst, int pop, int flow,
                                  KArgs<typename Store<S>::R> a) {
  const long long nn = (long long)a.n[0] * a.n[1] * a.n[2];
  const double w = flow ? flow_weight<D>(pop) : 0.0;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x)
    Store<S>::st(dst + pitched(k, a.n, flow ? a.rsf : a.rsg), typename Store<S>::R(src[k] - w));
}

template <int D, typename S>
__global__ void convert_out_kernel(const S* __restrict__ src, double* __restrict__ dst, int pop, int flow,
                                   KArgs<typename Store<S>::R> a) {
  const long long nn = (long long)a.n[0] * a.n[1] * a.n[2];
  const double w = flow ? flow_weight<D>(pop) : 0.0;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x)
    dst[k] = double(Store<S>::ld(src + pitched(k, a.n, flow ? a.rsf : a.rsg))) + w;
}

static int node_blocks(const DevState& s) {
  const long long nn = (long long)s.n[0] * s.n[1] * s.n[2];
  long long nb = (nn + 255) / 256;
  return (int)(nb < 8192 ? (nb > 0 ? nb : 1) : 8192);
}

hipError_t launch_convert_in(const DevState& s, const double* src, void* dst, int pop, int flow,
                             hipStream_t st) {
  return by_storage(s.storage, s.dim, [&](auto tag) {
    using S = decltype(tag);
    using R = typename Store<S>::R;
    KArgs<R> a = make_args<R>(s);
    if (s.dim == 2)
      hipLaunchKernelGGL((convert_in_kernel<2, S>), dim3(node_blocks(s)), dim3(256), 0, st, src,
                         static_cast<S*>(dst), pop, flow, a);
    else
      hipLaunchKernelGGL((convert_in_kernel<3, S>), dim3(node_blocks(s)), dim3(256), 0, st, src,
                         static_cast<S*>(dst), pop, flow, a);
    return hipGetLastError();
  });
}

hipError_t launch_convert_out(const DevState& s, const void* src, double* dst, int pop, int flow,
                              hipStream_t st) {
  return by_storage(s.storage, s.dim, [&](auto tag) {
    using S = decltype(tag);
    using R = typename Store<S>::R;
    KArgs<R> a = make_args<R>(s);
    if (s.dim == 2)
      hipLaunchKernelGGL((convert_out_kernel<2, S>), dim3(node_blocks(s)), dim3(256), 0, st,
                         static_cast<const S*>(src), dst, pop, flow, a);
    else
      hipLaunchKernelGGL((convert_out_kernel<3, S>), dim3(node_blocks(s)), dim3(256), 0, st,
                         static_cast<const S*>(src), dst, pop, flow, a);
    return hipGetLastError();
  });
}

// Collision only (pre-collision state in, post-collision state out).
template <int D, typename S>
__global__ void collide_only_kernel(const S* __restrict__ fin, const S* __restrict__ gin, S* __restrict__ fout,
                                    S* __restrict__ gout, KArgs<typename Store<S>::R> a) {
  using R = typename Store<S>::R;
  using LF = typename Pair<D>::F;
  using LG = typename Pair<D>::G;
  const long long nn = (long long)a.n[0] * a.n[1] * a.n[2];
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x) {
    const long long cf = pitched(k, a.n, a.rsf), cg = pitched(k, a.n, a.rsg);
    R d[LF::Q], g[LG::Q];
#pragma unroll
    for (int i = 0; i < LF::Q; ++i) d[i] = Store<S>::ld(fin + i * a.ps + cf);
#pragma unroll
    for (int i = 0; i < LG::Q; ++i) g[i] = Store<S>::ld(gin + i * a.ps + cg);
    Macro<R> m;
    if (a.collide) collide<D>(d, g, a.k, m);
#pragma unroll
    for (int i = 0; i < LF::Q; ++i) Store<S>::st(fout + i * a.ps + cf, d[i]);
#pragma unroll
    for (int i = 0; i < LG::Q; ++i) Store<S>::st(gout + i * a.ps + cg, g[i]);
  }
}

hipError_t launch_collide_only(const DevState& s, const void* fin, const void* gin, void* fout,
                               void* gout, hipStream_t st) {
  return by_storage(s.storage, s.dim, [&](auto tag) {
    using S = decltype(tag);
    using R = typename Store<S>::R;
    KArgs<R> a = make_args<R>(s);
    if (s.dim == 2)
      hipLaunchKernelGGL((collide_only_kernel<2, S>), dim3(node_blocks(s)), dim3(256), 0, st,
                         static_cast<const S*>(fin), static_cast<const S*>(gin), static_cast<S*>(fout),
                         static_cast<S*>(gout), a);
    else
      hipLaunchKernelGGL((collide_only_kernel<3, S>), dim3(node_blocks(s)), dim3(256), 0, st,
                         static_cast<const S*>(fin), static_cast<const S*>(gin), static_cast<S*>(fout),
                         static_cast<S*>(gout), a);
    return hipGetLastError();
  });
}

// Equilibrium state from (u, T) with rho = 1, collided once.
template <int D, typename S>
__global__ void init_eq_kernel(const double* __restrict__ ux, const double* __restrict__ uy,
                               const double* __restrict__ uz, const double* __restrict__ Tf,
                               S* __restrict__ fout, S* __restrict__ gout, KArgs<typename Store<S>::R> a) {
  using R = typename Store<S>::R;
  using LF = typename Pair<D>::F;
  using LG = typename Pair<D>::G;
  const long long nn = (long long)a.n[0] * a.n[1] * a.n[2];
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x) {
    const R u = R(ux[k]), v = R(uy[k]), w = (D == 3 && uz) ? R(uz[k]) : R(0), T = R(Tf[k]);
    R m[LF::Q], n[LG::Q];
    for (int r = 0; r < LF::Q; ++r) m[r] = R(0);
    for (int r = 0; r < LG::Q; ++r) n[r] = R(0);
    if constexpr (D == 2) {
      const R u2 = u * u + v * v;
      m[1] = R(3) * u2;
      m[2] = R(-3) * u2;
      m[3] = u;
      m[4] = -u;
      m[5] = v;
      m[6] = -v;
      m[7] = u * u - v * v;
      m[8] = u * v;
      n[0] = T;
      n[1] = u * T;
      n[2] = v * T;
      n[3] = a.k.aT * T;
    } else {
      const R u2 = u * u + v * v + w * w;
      const R c23 = R(2.0 / 3.0);
      const R pxx = R(2) * u * u - v * v - w * w, pww = v * v - w * w;
      m[1] = R(19) * u2;
      m[2] = R(-5.5) * u2;
      m[3] = u;
      m[4] = -c23 * u;
      m[5] = v;
      m[6] = -c23 * v;
      m[7] = w;
      m[8] = -c23 * w;
      m[9] = pxx;
      m[10] = R(-0.5) * pxx;
      m[11] = pww;
      m[12] = R(-0.5) * pww;
      m[13] = u * v;
      m[14] = v * w;
      m[15] = u * w;
      n[0] = T;
      n[1] = u * T;
      n[2] = v * T;
      n[3] = w * T;
      n[4] = a.k.aT * T;
    }
    R d[LF::Q], g[LG::Q];
    from_moments<LF>(m, d);
    from_moments<LG>(n, g);
    Macro<R> mm;
    if (a.collide) collide<D>(d, g, a.k, mm);
    const long long cf = pitched(k, a.n, a.rsf), cg = pitched(k, a.n, a.rsg);
#pragma unroll
    for (int i = 0; i < LF::Q; ++i) Store<S>::st(fout + i * a.ps + cf, d[i]);
#pragma unroll
    for (int i = 0; i < LG::Q; ++i) Store<S>::st(gout + i * a.ps + cg, g[i]);
  }
}

hipError_t launch_init_eq(const DevState& s, const double* ux, const double* uy, const double* uz,
                          const double* T, void* fout, void* gout, hipStream_t st) {
  return by_storage(s.storage, s.dim, [&](auto tag) {
    using S = decltype(tag);
    using R = typename Store<S>::R;
    KArgs<R> a = make_args<R>(s);
    if (s.dim == 2)
      hipLaunchKernelGGL((init_eq_kernel<2, S>), dim3(node_blocks(s)), dim3(256), 0, st, ux, uy, uz, T,
                         static_cast<S*>(fout), static_cast<S*>(gout), a);
    else
      hipLaunchKernelGGL((init_eq_kernel<3, S>), dim3(node_blocks(s)), dim3(256), 0, st, ux, uy, uz, T,
                         static_cast<S*>(fout), static_cast<S*>(gout), a);
    return hipGetLastError();
  });
}

template <int D, typename S>
__device__ __forceinline__ void load_node(const S* f, const S* g, long long k, const KArgs<typename Store<S>::R>& a,
                                          typename Store<S>::R* d, typename Store<S>::R* gg) {
  using LF = typename Pair<D>::F;
  using LG = typename Pair<D>::G;
  const long long cf = pitched(k, a.n, a.rsf), cg = pitched(k, a.n, a.rsg);
#pragma unroll
  for (int i = 0; i < LF::Q; ++i) d[i] = Store<S>::ld(f + i * a.ps + cf);
#pragma unroll
  for (int i = 0; i < LG::Q; ++i) gg[i] = Store<S>::ld(g + i * a.ps + cg);
}

template <int D, typename S>
__global__ void fields_kernel(const S* __restrict__ f, const S* __restrict__ g, double* rho, double* ux,
                              double* uy, double* uz, double* T, KArgs<typename Store<S>::R> a) {
  using R = typename Store<S>::R;
  const long long nn = (long long)a.n[0] * a.n[1] * a.n[2];
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x) {
    R d[Pair<D>::F::Q], gg[Pair<D>::G::Q];
    load_node<D, S>(f, g, k, a, d, gg);
    Macro<R> m;
    macro_post<D>(d, gg, a.k, m);
    if (rho) rho[k] = double(m.rho);
    if (ux) ux[k] = double(m.u[0]);
    if (uy) uy[k] = double(m.u[1]);
    if (uz && D == 3) uz[k] = double(m.u[2]);
    if (T) T[k] = double(m.T);
  }
}

hipError_t launch_fields(const DevState& s, const void* f, const void* g, double* rho, double* ux,
                         double* uy, double* uz, double* T, hipStream_t st) {
  return by_storage(s.storage, s.dim, [&](auto tag) {
    using S = decltype(tag);
    using R = typename Store<S>::R;
    KArgs<R> a = make_args<R>(s);
    if (s.dim == 2)
      hipLaunchKernelGGL((fields_kernel<2, S>), dim3(node_blocks(s)), dim3(256), 0, st,
                         static_cast<const S*>(f), static_cast<const S*>(g), rho, ux, uy, uz, T, a);
    else
      hipLaunchKernelGGL((fields_kernel<3, S>), dim3(node_blocks(s)), dim3(256), 0, st,
                         static_cast<const S*>(f), static_cast<const S*>(g), rho, ux, uy, uz, T, a);
    return hipGetLastError();
  });
}

// Statistics of the stored post-collision state (no time step).
template <int D, typename S>
__global__ void __launch_bounds__(256) reduce_state_kernel(const S* __restrict__ f, const S* __restrict__ g,
                                                           KArgs<typename Store<S>::R> a) {
  using R = typename Store<S>::R;
  const long long nn = (long long)a.n[0] * a.n[1] * a.n[2];
  RedAcc<R> acc;
  red_init(acc);
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x) {
    R d[Pair<D>::F::Q], gg[Pair<D>::G::Q];
    load_node<D, S>(f, g, k, a, d, gg);
    Macro<R> m;
    macro_post<D>(d, gg, a.k, m);
    int gi[3];
    gi[0] = (int)(k % a.n[0]);
    gi[1] = (int)((k / a.n[0]) % a.n[1]);
    gi[2] = (int)(k / ((long long)a.n[0] * a.n[1]));
    red_node(acc, a, gi, m);
  }
  red_block<256>(acc, a.inv_uf, a.partials + (long long)blockIdx.x * kRedSlots);
}

int reduce_state_blocks(const DevState& s) {
  const int nb = node_blocks(s);
  return nb < 1024 ? nb : 1024;
}

hipError_t launch_reduce_state(const DevState& s, const void* f, const void* g, double* partials,
                               hipStream_t st) {
  return by_storage(s.storage, s.dim, [&](auto tag) {
    using S = decltype(tag);
    using R = typename Store<S>::R;
    KArgs<R> a = make_args<R>(s);
    a.partials = partials;
    const int nb = reduce_state_blocks(s);
    if (s.dim == 2)
      hipLaunchKernelGGL((reduce_state_kernel<2, S>), dim3(nb), dim3(256), 0, st,
                         static_cast<const S*>(f), static_cast<const S*>(g), a);
    else
      hipLaunchKernelGGL((reduce_state_kernel<3, S>), dim3(nb), dim3(256), 0, st,
                         static_cast<const S*>(f), static_cast<const S*>(g), a);
    return hipGetLastError();
  });
}

// Change of the velocity and temperature fields against a snapshot u', T'
// taken earlier (the steady-state measure of Sec. 3): per workgroup, sums of
// |u - u'|_2, |u'|_2, |T - T'| and |T'| in FP64; the snapshot is then
// overwritten with the current fields (snap holds ux, uy, uz, T planes of nn
// doubles each).
template <int D, typename S>
__global__ void __launch_bounds__(256) steady_change_kernel(const S* __restrict__ f, const S* __restrict__ g,
                                                            double* __restrict__ snap, int first,
                                                            double* __restrict__ partials,
                                                            KArgs<typename Store<S>::R> a) {
  using R = typename Store<S>::R;
  const long long nn = (long long)a.n[0] * a.n[1] * a.n[2];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x) {
    R d[Pair<D>::F::Q], gg[Pair<D>::G::Q];
    load_node<D, S>(f, g, k, a, d, gg);
    Macro<R> m;
    macro_post<D>(d, gg, a.k, m);
    const double u0 = double(m.u[0]), u1 = double(m.u[1]), u2 = D == 3 ? double(m.u[2]) : 0.0;
    const double T = double(m.T);
    if (!first) {
      const double p0 = snap[k], p1 = snap[nn + k], p2 = snap[2 * nn + k], pT = snap[3 * nn + k];
      const double e0 = u0 - p0, e1 = u1 - p1, e2 = u2 - p2;
      acc[0] += sqrt(e0 * e0 + e1 * e1 + e2 * e2);
      acc[1] += sqrt(p0 * p0 + p1 * p1 + p2 * p2);
      acc[2] += fabs(T - pT);
      acc[3] += fabs(pT);
    }
    snap[k] = u0;
    snap[nn + k] = u1;
    snap[2 * nn + k] = u2;
    snap[3 * nn + k] = T;
  }
  __shared__ double sh[4][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double v = acc[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) sh[wid][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int i = threadIdx.x;
    partials[(long long)blockIdx.x * 4 + i] = ((sh[0][i] + sh[1][i]) + sh[2][i]) + sh[3][i];
  }
}

hipError_t launch_steady_change(const DevState& s, const void* f, const void* g, double* snap, int first,
                                double* partials, hipStream_t st) {
  return by_storage(s.storage, s.dim, [&](auto tag) {
    using S = decltype(tag);
    using R = typename Store<S>::R;
    KArgs<R> a = make_args<R>(s);
    const int nb = reduce_state_blocks(s);
    if (s.dim == 2)
      hipLaunchKernelGGL((steady_change_kernel<2, S>), dim3(nb), dim3(256), 0, st, static_cast<const S*>(f),
                         static_cast<const S*>(g), snap, first, partials, a);
    else
      hipLaunchKernelGGL((steady_change_kernel<3, S>), dim3(nb), dim3(256), 0, st, static_cast<const S*>(f),
                         static_cast<const S*>(g), snap, first, partials, a);
    return hipGetLastError();
  });
}

// Fixed-order sum of the per-workgroup partial records.
__global__ void __launch_bounds__(256) finish_kernel(const double* __restrict__ partials, int nblocks,
                                                     double* __restrict__ out) {
  __shared__ double sh[256];
  for (int i = 0; i < kRedSlots; ++i) {
    const bool mx = i >= 8 && i <= 10;
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
      const double p = partials[(long long)b * kRedSlots + i];
      v = mx ? fmax(v, p) : v + p;
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) sh[threadIdx.x] = mx ? fmax(sh[threadIdx.x], sh[threadIdx.x + w])
                                                : sh[threadIdx.x] + sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = sh[0];
    __syncthreads();
  }
}

hipError_t launch_finish(const double* partials, int nblocks, double* out, hipStream_t st) {
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, st, partials, nblocks, out);
  return hipGetLastError();
}

}  // namespace islbm

// Persistent PDHG solve kernel for gfx950 (CDNA4).
//
// Method (the paper fixes the problem, not the iteration): a restarted, reflected
// Halpern PDHG on the splitting described in include/ffolio.h, in diagonally scaled
// variables xs = W / dc, ys = Y / dr.  One iteration computes T(z) for z = (xs, ys):
//
//   x+ = prox_{tau g}(xs - tau K~^T ys)      per asset: weighted L1-ball solve with a
//                                            global multiplier mu_t per period
//   y+ = prox_{sigma h~*}(ys + sigma K~ (2 x+ - xs))
//
// then z <- (k+1)/(k+2) ((1+rho) T(z) - rho z) + 1/(k+2) z0 (Halpern anchoring with
// reflection), with adaptive restarts on the fixed-point residual and a primal weight
// omega (tau = eta/omega, sigma = eta*omega, eta = safety/||K~|| from a power
// iteration run at the start of the kernel).
//
// Work split: workgroup w owns a contiguous slice of assets for every period.  Its
// slice of the constraint rows and its per-asset state stay in LDS when they fit (else
// in device memory, touched only by this workgroup); the exposure and factor duals
// (P x (m+k) numbers) are replicated in every workgroup and updated redundantly from
// the same exchanged totals, so all workgroups hold bit-identical copies and take
// identical control decisions.
//
// Exchange: each workgroup publishes partial sums with device-scope (sc1) stores or
// atomic adds, then arrives at a counter barrier; readers fetch totals with
// device-scope loads.  No L2 writeback/invalidate fences are needed because every
// exchanged word is accessed only through device-coherent operations.  Every wait is
// bounded (spin_limit): on expiry the kernel records DS_BARRIER and all workgroups exit.
//
// The L1-ball multiplier mu_t is exact.  Speculative mode (one period): a predicted
// bracket [lo, hi] is tested in the same exchange that carries the two affine pieces
// of K~ x_bar(mu); if the root lies in the bracket and no breakpoint |b_i| falls
// inside it, mu and K~ x_bar follow in closed form (one exchange per iteration).
// Two-phase mode (many periods): a small exchange settles mu_t, a second one carries
// K~ x_bar.  Misses fall back to a 32-candidate multisection that isolates a
// breakpoint-free piece.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include <type_traits>
#include "internal.h"
#include "cost_math.h"

namespace ffo {
namespace {

#ifndef FFO_TB
#define FFO_TB 256
#endif
constexpr int TB = FFO_TB;       // threads per workgroup (one workgroup per CU)
constexpr int NWAVE = TB / 64;
constexpr int MSC = 32;          // multisection candidates per round
constexpr int MS_ROUNDS = 40;
constexpr int NC = 8;            // bracket candidates per period
constexpr int STW = 2 + 3 * NC;  // published statistics per period
constexpr int RED_OUT = TB, RED_MAX = TB + 64, RED_LEN = TB + 64 + 16;
static_assert(TB == 256 || TB == 512, "workgroup size");

__device__ __forceinline__ double ldd(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void std_(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void addd(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }

// Cross-lane moves of a double through DPP (two 32-bit halves; every source lane valid
// for the controls used here: quad_perm and the row mirrors).
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
constexpr int DPP_SWAP1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int DPP_SWAP2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141; // lane i <- 7 - i within each 8-lane half-row
constexpr int DPP_MIRROR = 0x140;      // lane i <- 15 - i within each 16-lane row

// Sums over aligned groups of 4, 8 and 16 lanes; every lane of the group gets the sum.
__device__ __forceinline__ double sum4(double x) { x += dpp<DPP_SWAP1>(x); return x + dpp<DPP_SWAP2>(x); }
__device__ __forceinline__ double sum8(double x) { x = sum4(x); return x + dpp<DPP_HALF_MIRROR>(x); }
__device__ __forceinline__ double sum16(double x) { x = sum8(x); return x + dpp<DPP_MIRROR>(x); }
__device__ __forceinline__ double max8(double x) {
  x = fmax(x, dpp<DPP_SWAP1>(x));
  x = fmax(x, dpp<DPP_SWAP2>(x));
  return fmax(x, dpp<DPP_HALF_MIRROR>(x));
}
__device__ __forceinline__ double max16(double x) { x = max8(x); return fmax(x, dpp<DPP_MIRROR>(x)); }
template <int L>
__device__ __forceinline__ double sum_lanes(double x) {
  static_assert(L == 8 || L == 16, "lane group");
  if constexpr (L == 8) return sum8(x);
  else return sum16(x);
}
__device__ __forceinline__ double lane_of(double x, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// Wave-wide sum / max (fixed order), uniform across the wave.
__device__ __forceinline__ double wave_sum(double x) {
  x = sum16(x);
  return (lane_of(x, 15) + lane_of(x, 31)) + (lane_of(x, 47) + lane_of(x, 63));
}
__device__ __forceinline__ double wave_max(double x) {
  x = max16(x);
  return fmax(fmax(lane_of(x, 15), lane_of(x, 31)), fmax(lane_of(x, 47), lane_of(x, 63)));
}

// LDS-qualified element types: indexing through these compiles to ds_read/ds_write
// instead of generic (flat) memory instructions.
typedef __attribute__((address_space(3))) double ldbl;
typedef __attribute__((address_space(3))) int lint;
// Device-memory pointers in the global address space: their loads count only against
// vmcnt (generic FLAT loads also count against lgkmcnt, so every LDS wait would drain them).
template <class T>
using gmem_t = __attribute__((address_space(1))) T;
template <class R>
using lds_t = __attribute__((address_space(3))) R;

// Per-(t, li) array view: element (t, li) at b[t * ld + off + li]; SL selects LDS
// (true) or device memory (false) at compile time, R the stored type.
template <bool SL, class R = double>
struct Arr {
  using P = typename std::conditional<SL, lds_t<R>*, R*>::type;
  P b;
  int ld, off;
  __device__ __forceinline__ auto& operator()(int t, int li) const { return b[(size_t)t * ld + off + li]; }
};

// ---------------------------------------------------------------------------------
// Workgroup context and the exchange primitive
// ---------------------------------------------------------------------------------
struct Ctx {
  int wg, nwg, tid;
  int i0, nwa;            // owned assets [i0, i0 + nwa)
  unsigned long long epoch;
  double* xbuf;
  unsigned long long* bar;  // [0]: arrivals of groups; [XGSTRIDE * (1 + g)]: arrivals in group g;
                            // [XGSTRIDE * (1 + XG_MAX + g)]: release of group g (last epoch)
  int vmax, xmode, P;
  int ng, grp, gsize;     // atomic mode: copies of the exchange slot, this workgroup's copy, its users
  int mx_lo, mx_hi;       // exchange indices lo + STW*t + 1 in [mx_lo, mx_hi) combine by max
  uint32_t spin_limit;
  ldbl* tot;              // LDS [vmax]
  ldbl* red;              // LDS reduction scratch [RED_LEN]
  ldbl* lslot;            // LDS [3][vmax] exchange slots of a single-workgroup team (XM_LOCAL)
  lint* flag;             // LDS flag word
  long long t_wait;       // device-clock ticks spent waiting (thread 0)
  long long t_pre;        // ticks from exchange entry to barrier arrival (store completion)
  long long t_read;       // ticks reading totals after the barrier
};

// Contribution j of this workgroup to the current exchange.  In gather mode every
// index in [0, V) must be written each exchange; in atomic mode zeros may be skipped.
__device__ __forceinline__ void put(const Ctx& c, int j, double v) {
  if (c.xmode == XM_LOCAL) {
    if (v != 0.0)
      __hip_atomic_fetch_add(&c.lslot[(size_t)(c.epoch % 3) * c.vmax + j], v, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
  } else if (c.xmode == XM_GATHER) {
    std_(&c.xbuf[((size_t)(c.epoch & 1) * c.nwg + c.wg) * c.vmax + j], v);
  } else if (v != 0.0) {
    addd(&c.xbuf[((size_t)(c.epoch % 3) * c.ng + c.grp) * c.vmax + j], v);
  }
}

// Contribution j (a max-combined index, see Ctx::mx_lo) of a non-negative value.  In
// atomic mode the maximum is taken on the bit patterns, which order non-negative
// doubles like their values.
__device__ __forceinline__ void put_max(const Ctx& c, int j, double v) {
  if (c.xmode == XM_LOCAL) {
    if (v > 0.0) {
      typedef __attribute__((address_space(3))) unsigned long long lu64;
      __hip_atomic_fetch_max((lu64*)&c.lslot[(size_t)(c.epoch % 3) * c.vmax + j],
                             (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  } else if (c.xmode == XM_GATHER) {
    std_(&c.xbuf[((size_t)(c.epoch & 1) * c.nwg + c.wg) * c.vmax + j], v);
  } else if (v > 0.0) {
    unsigned long long* a = (unsigned long long*)&c.xbuf[((size_t)(c.epoch % 3) * c.ng + c.grp) * c.vmax + j];
    __hip_atomic_fetch_max(a, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Destination of this workgroup's contributions to the current exchange, for code that
// runs out of line (no Ctx): put_at(put_to(c), j, v) does what put(c, j, v) does.
struct PutTo {
  double* g;   // device slot (gather: this workgroup's; atomic: the shared one)
  ldbl* l;     // LDS slot of a single-workgroup team
  int mode;
};

__device__ __forceinline__ PutTo put_to(const Ctx& c) {
  PutTo q;
  q.mode = c.xmode;
  q.l = c.lslot ? c.lslot + (size_t)(c.epoch % 3) * c.vmax : nullptr;
  q.g = c.xmode == XM_GATHER ? c.xbuf + ((size_t)(c.epoch & 1) * c.nwg + c.wg) * c.vmax
                             : c.xbuf + ((size_t)(c.epoch % 3) * c.ng + c.grp) * c.vmax;
  return q;
}

__device__ __forceinline__ void put_at(const PutTo& q, int j, double v) {
  if (q.mode == XM_LOCAL) {
    if (v != 0.0) __hip_atomic_fetch_add(&q.l[j], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  } else if (q.mode == XM_GATHER) {
    std_(&q.g[j], v);
  } else if (v != 0.0) {
    addd(&q.g[j], v);
  }
}

// Barrier + reduction of the V published values into c.tot (LDS).  Returns false when
// the bounded wait expired.
__device__ __forceinline__ bool xsync(Ctx& c, int V) {
  if (c.xmode == XM_LOCAL) {   // one workgroup: the slot already holds the totals
    __builtin_amdgcn_s_waitcnt(0);   // device-memory stores of this exchange (lists) are complete
    __syncthreads();
    const ldbl* cur = c.lslot + (size_t)(c.epoch % 3) * c.vmax;
    ldbl* nxt = c.lslot + (size_t)((c.epoch + 2) % 3) * c.vmax;
    for (int j = c.tid; j < c.vmax; j += TB) {
      if (j < V) c.tot[j] = cur[j];
      nxt[j] = 0.0;
    }
    __syncthreads();
    c.epoch++;
    c.mx_lo = c.mx_hi = 0;
    return true;
  }
  const long long tp0 = wall_clock64();
  __builtin_amdgcn_s_waitcnt(0);  // this wave's device-scope stores/atomics are complete
  __syncthreads();
  if (c.tid == 0) {
    const long long t0 = wall_clock64();
    c.t_pre += t0 - tp0;
    unsigned long long target;
    const unsigned long long* poll = c.bar;
    if (c.ng > 1) {
      // two-level arrival: the last workgroup of each group arrives for the group, so
      // at most max(group size, groups) read-modify-writes meet on one counter; the
      // last group's arrival releases every group through its own flag, so each flag
      // is polled by one group only
      target = c.epoch + 1;
      const unsigned long long gt = (c.epoch + 1) * (unsigned long long)c.gsize;
      if (__hip_atomic_fetch_add(c.bar + XGSTRIDE * (1 + c.grp), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) +
              1 == gt) {
        if (__hip_atomic_fetch_add(c.bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 ==
            (c.epoch + 1) * (unsigned long long)c.ng)
          for (int g = 0; g < c.ng; ++g)
            __hip_atomic_store(c.bar + XGSTRIDE * (1 + XG_MAX + g), c.epoch + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
      poll = c.bar + XGSTRIDE * (1 + XG_MAX + c.grp);
    } else {
      target = (c.epoch + 1) * (unsigned long long)c.nwg;
      __hip_atomic_fetch_add(c.bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t spins = 0;
    int ok = 1;
    while (__hip_atomic_load(poll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > c.spin_limit) { ok = 0; break; }
    }
    *c.flag = ok;
    c.t_wait += wall_clock64() - t0;
  }
  __syncthreads();
  if (!*c.flag) return false;
  const long long tr0 = wall_clock64();
  if (c.xmode == XM_GATHER) {
    const double* base = c.xbuf + (size_t)(c.epoch & 1) * c.nwg * c.vmax;
    for (int j = c.tid; j < V; j += TB) {
      double s = 0.0;
      if (j >= c.mx_lo && j < c.mx_hi && (j - c.mx_lo) % STW == 1)
        for (int w = 0; w < c.nwg; ++w) s = fmax(s, ldd(&base[(size_t)w * c.vmax + j]));
      else
        for (int w = 0; w < c.nwg; ++w) s += ldd(&base[(size_t)w * c.vmax + j]);
      c.tot[j] = s;
    }
  } else {
    const double* base = c.xbuf + (size_t)(c.epoch % 3) * c.ng * c.vmax;
    if (c.ng == 1) {
      // four loads in flight per thread
      for (int j = c.tid; j < V; j += 4 * TB) {
        double u[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) u[r] = j + r * TB < V ? ldd(&base[j + r * TB]) : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (j + r * TB < V) c.tot[j + r * TB] = u[r];
      }
    } else {
      // the copies combine in a fixed order (sum, or max for the max-combined entries);
      // two totals per thread and step, every copy's load issued before the first use
      for (int j = c.tid; j < V; j += 2 * TB) {
        double u[2][XG_MAX];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int g = 0; g < XG_MAX; ++g)
            u[r][g] = (g < c.ng && j + r * TB < V) ? ldd(&base[(size_t)g * c.vmax + j + r * TB]) : 0.0;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const int jj = j + r * TB;
          double t = u[r][0];
          if (jj >= c.mx_lo && jj < c.mx_hi && (jj - c.mx_lo) % STW == 1) {
#pragma unroll
            for (int g = 1; g < XG_MAX; ++g) t = fmax(t, u[r][g]);
          } else {
#pragma unroll
            for (int g = 1; g < XG_MAX; ++g) t += u[r][g];
          }
          if (jj < V) c.tot[jj] = t;
        }
      }
    }
    // clear the slot used two exchanges from now (its last readers passed this barrier)
    double* z = c.xbuf + (size_t)((c.epoch + 2) % 3) * c.ng * c.vmax;
    const int zl = c.ng * c.vmax;
    const int per = (zl + c.nwg - 1) / c.nwg;
    const int j0 = c.wg * per, j1 = min(zl, j0 + per);
    for (int j = j0 + c.tid; j < j1; j += TB) std_(&z[j], 0.0);
  }
  __syncthreads();
  if (c.tid == 0) c.t_read += wall_clock64() - tr0;
  c.epoch++;
  c.mx_lo = c.mx_hi = 0;
  return true;
}

// Fixed-order workgroup sum of NV per-thread values; result in red[RED_OUT + q] (LDS),
// valid for every thread after the call.  Uses red[0 .. NWAVE*NV), NWAVE*NV <= RED_OUT.
template <int NV>
__device__ __forceinline__ void wg_sum(const Ctx& c, double (&v)[NV]) {
  static_assert(NWAVE * NV <= RED_OUT && NV <= RED_MAX - RED_OUT, "reduction scratch");
  ldbl* out = c.red + RED_OUT;
  const int lane = c.tid & 63, wave = c.tid >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double x = wave_sum(v[q]);
    if (lane == 0) c.red[wave * NV + q] = x;
  }
  __syncthreads();
  if (c.tid < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) s += c.red[w * NV + c.tid];
    out[c.tid] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ double wg_max(const Ctx& c, double x) {
  x = wave_max(x);
  if ((c.tid & 63) == 0) c.red[RED_MAX + (c.tid >> 6)] = x;
  __syncthreads();
  double m = 0.0;
  for (int w = 0; w < NWAVE; ++w) m = fmax(m, c.red[RED_MAX + w]);
  __syncthreads();
  return m;
}

// ---------------------------------------------------------------------------------
// Per-workgroup problem and state views
// ---------------------------------------------------------------------------------
// A per-asset iterate: the value itself (R = double) or a float offset from the FP64
// restart anchor z0 (R = float).  Offsets keep the rounding of each stored update
// proportional to the distance moved since the last restart, not to the size of the
// iterate (rounding errors that do not shrink would accumulate through the Halpern
// anchoring).
template <bool SL, class R>
struct Iter {
  static constexpr bool OFF = !std::is_same<R, double>::value;
  Arr<SL, double> z0;
  Arr<SL, R> d;
  __device__ __forceinline__ double operator()(int t, int li) const {
    if constexpr (OFF) return z0(t, li) + (double)d(t, li);
    else return d(t, li);
  }
  __device__ __forceinline__ void set(int t, int li, double v) const {
    if constexpr (OFF) d(t, li) = (R)(v - z0(t, li));
    else d(t, li) = v;
  }
};

// A bfloat16 bit pattern in device memory (rows of the FP32_BF16K form); widening to
// double is exact.
struct bf16 {
  uint16_t b;
  __device__ __forceinline__ explicit operator double() const { return (double)__uint_as_float((uint32_t)b << 16); }
};

// Row element loaded through a global-address pointer.
template <class T>
__device__ __forceinline__ T gload(const gmem_t<T>* p) { return *p; }
template <>
__device__ __forceinline__ bf16 gload<bf16>(const gmem_t<bf16>* p) {
  bf16 r;
  r.b = *(const gmem_t<uint16_t>*)p;
  return r;
}

// Element type of the rows read from device memory: double in the FP64 form, float in
// the FP32 form (bf16 is chosen explicitly).
template <class R>
struct default_kg {
  using type = typename std::conditional<std::is_same<R, float>::value, float, double>::type;
};

// R: stored type of the per-asset iterates and of the LDS copies (double in the FP64
// form, float in the FP32 form); every expression evaluates in double.
template <bool KL, bool SL, class R = double, class KGT = typename default_kg<R>::type>
struct S {
  using RC = typename std::conditional<SL, R, double>::type;   // constants: LDS copies or FP64 inputs
  static constexpr bool KLDS = KL;
  using KG = KGT;
  const DevProblem* p;
  const lds_t<R>* Kl;   // LDS slice [nr][ldl] (KL) ...
  const KG* Kg;         // ... or the rows in device memory, times the LDS row scale ks
  const ldbl* ks;
  int nw, ldl, i0;
  // state: anchors and per-iteration scratch in FP64, iterates through Iter views
  Arr<SL, double> x0s, bb, aa, xb;          // [P] anchor, prox input b, 1/a, xbar
  Iter<SL, R> xs, Txs;                      // [P]
  Arr<SL, double> ys0C;                     // [Tp]
  Iter<SL, R> ysC, TysC;                    // [Tp]
  // constants: the ones that define a trade (column scale, trade-row scale, w0, w_T and
  // the risk centre) stay float64 in every form, so the fixed point trades to the exact
  // w0 (a float copy of w0 shifts the cost kinks by ~1e-10, which large cost weights turn
  // into a relative gap of ~1e-4); the others are LDS copies of type RC
  Arr<SL, RC> alpha;                        // [P]
  Arr<SL, RC> ca, cb;                       // [Tp]
  Arr<SL, double> drC;                      // [Tp]
  Arr<SL, RC> arisk;                        // [1]
  Arr<SL, double> dc, cvec, w0, wT;         // [1]
  __device__ __forceinline__ double Kat(int j, int li) const {
    if constexpr (KL) return (double)Kl[j * ldl + li];
    else return (double)Kg[(size_t)j * p->ldk + i0 + li] * ks[j];
  }
};

// sum_{j0 <= j < j1} K~[j][li] y[j] with four independent accumulators.
template <class SV>
__device__ __forceinline__ double kcol_dot(const SV& v, const ldbl* y, int li, int j0, int j1) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = j0;
  for (; j + 4 <= j1; j += 4) {
    s0 = fma(v.Kat(j, li), y[j], s0);
    s1 = fma(v.Kat(j + 1, li), y[j + 1], s1);
    s2 = fma(v.Kat(j + 2, li), y[j + 2], s2);
    s3 = fma(v.Kat(j + 3, li), y[j + 3], s3);
  }
  for (; j < j1; ++j) s0 = fma(v.Kat(j, li), y[j], s0);
  return (s0 + s1) + (s2 + s3);
}

// (K~^T y) over the exposure and factor rows for every owned (t, li), into out[t*nw + li]
// (LDS).  Small slices split the rows over 2 or 4 thread groups with partials in
// red[0, TB).  All threads call; synchronised on return.
// The same with the rows in device memory (K~[j][li] = K[j*ldk + i0 + li] ks[j]).
template <int AW, class KG>
__device__ __forceinline__ void kty_dev(const KG* K, int ldk, int i0, const ldbl* ks, const ldbl* y, int P, int nr,
                                     int nw, int nwa, ldbl* red, ldbl* out) {
  const int tid = threadIdx.x, ne = P * nwa;
  auto dot = [&](const ldbl* yt, int li, int j0, int j1) {
    const gmem_t<KG>* col = (const gmem_t<KG>*)(K + i0 + li);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int j = j0;
    for (; j + 8 <= j1; j += 8) {   // eight loads in flight, summed as two steps of four
      KG kr[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) kr[u] = gload(col + (size_t)(j + u) * ldk);
      __builtin_amdgcn_sched_barrier(0);
      s0 = fma((double)kr[0] * ks[j], yt[j], s0);
      s1 = fma((double)kr[1] * ks[j + 1], yt[j + 1], s1);
      s2 = fma((double)kr[2] * ks[j + 2], yt[j + 2], s2);
      s3 = fma((double)kr[3] * ks[j + 3], yt[j + 3], s3);
      s0 = fma((double)kr[4] * ks[j + 4], yt[j + 4], s0);
      s1 = fma((double)kr[5] * ks[j + 5], yt[j + 5], s1);
      s2 = fma((double)kr[6] * ks[j + 6], yt[j + 6], s2);
      s3 = fma((double)kr[7] * ks[j + 7], yt[j + 7], s3);
    }
    for (; j + 4 <= j1; j += 4) {
      const KG k0 = gload(col + (size_t)j * ldk), k1 = gload(col + (size_t)(j + 1) * ldk);
      const KG k2 = gload(col + (size_t)(j + 2) * ldk), k3 = gload(col + (size_t)(j + 3) * ldk);
      __builtin_amdgcn_sched_barrier(0);   // the four loads in flight together
      s0 = fma((double)k0 * ks[j], yt[j], s0);
      s1 = fma((double)k1 * ks[j + 1], yt[j + 1], s1);
      s2 = fma((double)k2 * ks[j + 2], yt[j + 2], s2);
      s3 = fma((double)k3 * ks[j + 3], yt[j + 3], s3);
    }
    for (; j < j1; ++j) s0 = fma((double)gload(col + (size_t)j * ldk) * ks[j], yt[j], s0);
    return (s0 + s1) + (s2 + s3);
  };
  if (ne == 0) { __syncthreads(); return; }
  const int G = ne <= TB / 4 ? 4 : (ne <= TB / 2 ? 2 : 1);
  if (G > 1) {
    const int per = TB / G, g = tid / per, e = tid - g * per;
    double r = 0.0;
    if (e < ne) {
      const int t = e / nwa, li = e - t * nwa;
      r = dot(y + t * nr, li, g * nr / G, (g + 1) * nr / G);
    }
    red[tid] = r;
    __syncthreads();
    if (tid < ne) {
      const int t = tid / nwa, li = tid - t * nwa;
      double a = 0.0;
      for (int gg = 0; gg < G; ++gg) a += red[gg * per + tid];
      out[t * nw + li] = a;
    }
  } else if (AW > 1 && nr >= 8) {
    // AW assets per thread and step: 8 AW row loads in flight per lane (the plain
    // kernel's long slices; the batched kernel's register budget keeps one asset)
    int e = tid;
    for (; e + (AW - 1) * TB < ne; e += AW * TB) {
      const gmem_t<KG>* col[AW];
      const ldbl* yy[AW];
      double acc[AW][2];
#pragma unroll
      for (int a = 0; a < AW; ++a) {
        const int f = e + a * TB, t = f / nwa, l = f - t * nwa;
        col[a] = (const gmem_t<KG>*)(K + i0 + l);
        yy[a] = y + t * nr;
        acc[a][0] = acc[a][1] = 0.0;
      }
      int j = 0;
      for (; j + 8 <= nr; j += 8) {
        KG kr[AW][8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int a = 0; a < AW; ++a) kr[a][u] = gload(col[a] + (size_t)(j + u) * ldk);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int a = 0; a < AW; ++a) acc[a][u & 1] = fma((double)kr[a][u] * ks[j + u], yy[a][j + u], acc[a][u & 1]);
      }
      for (; j < nr; ++j)
#pragma unroll
        for (int a = 0; a < AW; ++a) acc[a][0] = fma((double)gload(col[a] + (size_t)j * ldk) * ks[j], yy[a][j], acc[a][0]);
#pragma unroll
      for (int a = 0; a < AW; ++a) {
        const int f = e + a * TB, t = f / nwa, l = f - t * nwa;
        out[t * nw + l] = acc[a][0] + acc[a][1];
      }
    }
    for (; e < ne; e += TB) {
      const int t = e / nwa, li = e - t * nwa;
      out[t * nw + li] = dot(y + t * nr, li, 0, nr);
    }
  } else {
    for (int e = tid; e < ne; e += TB) {
      const int t = e / nwa, li = e - t * nwa;
      out[t * nw + li] = dot(y + t * nr, li, 0, nr);
    }
  }
  __syncthreads();
}

template <int AW = 1, class SV>
__device__ __forceinline__ void kty_all(const Ctx& c, const SV& v, const ldbl* y, int P, int nr, int nw, ldbl* out) {
  if constexpr (!SV::KLDS) {
    kty_dev<AW>(v.Kg, v.p->ldk, v.i0, v.ks, y, P, nr, nw, c.nwa, c.red, out);
    return;
  }
  const int ne = P * c.nwa;
  if (ne == 0) { __syncthreads(); return; }
  // as many thread groups over the rows as the workgroup holds copies of the slice's
  // (t, li) pairs: short slices keep every thread busy on a shorter chain
  const int G = ne <= TB / 16 ? 16 : (ne <= TB / 8 ? 8 : (ne <= TB / 4 ? 4 : (ne <= TB / 2 ? 2 : 1)));
  if (G > 1) {
    const int per = TB / G, g = c.tid / per, e = c.tid - g * per;
    double r = 0.0;
    if (e < ne) {
      const int t = e / c.nwa, li = e - t * c.nwa;
      r = kcol_dot(v, y + t * nr, li, g * nr / G, (g + 1) * nr / G);
    }
    c.red[c.tid] = r;
    __syncthreads();
    if (c.tid < ne) {
      const int t = c.tid / c.nwa, li = c.tid - t * c.nwa;
      double a = 0.0;
      for (int gg = 0; gg < G; ++gg) a += c.red[gg * per + c.tid];
      out[t * nw + li] = a;
    }
  } else {
    for (int e = c.tid; e < ne; e += TB) {
      const int t = e / c.nwa, li = e - t * c.nwa;
      out[t * nw + li] = kcol_dot(v, y + t * nr, li, 0, nr);
    }
  }
  __syncthreads();
}

// Row products for long asset slices with the rows in device memory: lanes run over
// assets (coalesced loads), each wave takes RB rows at a time and reduces them with wave
// sums; the sums go to the exchange: put_at(q, off1 + e, K~x1) and, when NX = 2,
// put_at(q, off2 + e, K~x2) for every e = t*nr + j.  All threads call; no synchronisation.
template <int NX, class KG>
__device__ __forceinline__ void rows_dev(const KG* K, int ldk, int i0, const ldbl* ks, const ldbl* x1, const ldbl* x2,
                                      int nw, int nwa, int P, int nr, PutTo q, int off1, int off2) {
  constexpr int RB = 6;   // 70 rows: three steps with every wave busy (8 would leave one wave alone)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, ntot = P * nr;
  for (int base = wave * RB; base < ntot; base += NWAVE * RB) {
    double a[RB][NX];
    int jr[RB], tr[RB];
    const gmem_t<KG>* rp[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int e = min(base + r, ntot - 1);
      tr[r] = e / nr;
      jr[r] = e - tr[r] * nr;
      rp[r] = (const gmem_t<KG>*)(K + (size_t)jr[r] * ldk + i0);
#pragma unroll
      for (int u = 0; u < NX; ++u) a[r][u] = 0.0;
    }
    if (tr[0] == tr[RB - 1]) {   // all RB rows in one period: one x value per asset
      const ldbl* y1 = x1 + tr[0] * nw;
      const ldbl* y2 = x2 + tr[0] * nw;
      // four assets per lane and step (li, li + 64, li + 128, li + 192: the order of a
      // one-asset loop), so 4 RB loads are in flight per lane; past the end of the slice
      // a load repeats li and its product is skipped
      for (int li = lane; li < nwa; li += 256) {
        int lk[4];
        bool in[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) { lk[h] = li + 64 * h; in[h] = lk[h] < nwa; }
        KG kr[4][RB];
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
          for (int r = 0; r < RB; ++r) kr[h][r] = gload(rp[r] + (in[h] ? lk[h] : li));
        __builtin_amdgcn_sched_barrier(0);   // keep the conversions behind the loads
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          if (in[h]) {
            const double v1 = y1[lk[h]], v2 = NX > 1 ? (double)y2[lk[h]] : 0.0;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
              const double kv = (double)kr[h][r];
              a[r][0] = fma(kv, v1, a[r][0]);
              if (NX > 1) a[r][NX - 1] = fma(kv, v2, a[r][NX - 1]);
            }
          }
        }
      }
    } else {
      for (int li = lane; li < nwa; li += 64) {
        KG kr[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) kr[r] = gload(rp[r] + li);
        __builtin_amdgcn_sched_barrier(0);
        double kv[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) kv[r] = (double)kr[r];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          a[r][0] = fma(kv[r], x1[tr[r] * nw + li], a[r][0]);
          if (NX > 1) a[r][NX - 1] = fma(kv[r], x2[tr[r] * nw + li], a[r][NX - 1]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
#pragma unroll
      for (int u = 0; u < NX; ++u) {
        const double sum = wave_sum(a[r][u] * ks[jr[r]]);
        if (lane == 0 && base + r < ntot) put_at(q, (u == 0 ? off1 : off2) + base + r, sum);
      }
    }
  }
}

// Row products over the owned assets with four lanes per row: for every e = t*nr + j,
// emit(e, a) with a[q] = sum_li K~[j][li] xq[t*nw + li] (x1, and x2 when NX = 2; LDS).
// All threads call (the lane shuffles need full waves).
template <int NX, int LPR, class SV, class F>
__device__ __forceinline__ void rows_prod_lds_l(const Ctx& c, const SV& v, const ldbl* x1, const ldbl* x2, int nw, int P,
                                                int nr, F emit) {
  const int q = c.tid & (LPR - 1), ntot = P * nr;
  for (int base = 0; base < ntot; base += TB / LPR) {
    const int e = base + c.tid / LPR;
    double a[NX];
#pragma unroll
    for (int u = 0; u < NX; ++u) a[u] = 0.0;
    if (e < ntot) {
      const int t = e / nr, j = e - t * nr;
      const ldbl* xa = x1 + t * nw;
      const ldbl* xb = (NX > 1 ? x2 : x1) + t * nw;
#pragma unroll 4
      for (int li = q; li < c.nwa; li += LPR) {
        const double kv = v.Kat(j, li);
        a[0] = fma(kv, xa[li], a[0]);
        if (NX > 1) a[NX - 1] = fma(kv, xb[li], a[NX - 1]);
      }
    }
    if constexpr (LPR == 4) {
#pragma unroll
      for (int u = 0; u < NX; ++u) a[u] = sum4(a[u]);
    }
    if (q == 0 && e < ntot) emit(e, a);
  }
}

// Lanes per row: one for slices of up to 32 assets (every lane owns a row, so a pass
// covers 256 rows with no lane reduction), else four with a DPP quad sum.
template <int NX, class SV, class F>
__device__ __forceinline__ void rows_prod_lds(const Ctx& c, const SV& v, const ldbl* x1, const ldbl* x2, int nw, int P, int nr,
                              F emit) {
  if (c.nwa <= 32) rows_prod_lds_l<NX, 1>(c, v, x1, x2, nw, P, nr, emit);
  else rows_prod_lds_l<NX, 4>(c, v, x1, x2, nw, P, nr, emit);
}

// Short slices (the usual case, rows in LDS or not): four lanes per row.  Long slices
// of rows in device memory (batched teams, very large n): the coalesced wide form,
// whose per-row wave reductions pay off once each lane has several assets.
template <int NX, class SV>
__device__ __forceinline__ void rows_prod(const Ctx& c, const SV& v, const ldbl* x1, const ldbl* x2, int nw, int P,
                                          int nr, int off1, int off2 = 0) {
  if constexpr (!SV::KLDS) {
    if (c.nwa > 512) {
      rows_dev<NX>(v.Kg, v.p->ldk, v.i0, v.ks, x1, x2, nw, c.nwa, P, nr, put_to(c), off1, off2);
      return;
    }
  }
  rows_prod_lds<NX>(c, v, x1, x2, nw, P, nr, [&](int e, const double* a) {
    put(c, off1 + e, a[0]);
    if (NX > 1) put(c, off2 + e, a[NX - 1]);
  });
}

// Trade-row adjoint for asset li, period t: dc (drC_t yC_t - drC_{t+1} yC_{t+1}).
template <class SV, class A>
__device__ __forceinline__ double kty_trade(const SV& v, const A& yC, int t, int li) {
  double r = v.drC(t, li) * yC(t, li);
  if (v.p->multi) r -= v.drC(t + 1, li) * yC(t + 1, li);
  return v.dc(0, li) * r;
}

// Trade row t of K~ applied to a scaled primal x for asset li.
template <class SV, class A>
__device__ __forceinline__ double kx_trade(const SV& v, const A& x, int t, int li) {
  double d;
  if (!v.p->multi || t == 0) d = x(0, li);
  else if (t == v.p->P) d = -x(v.p->P - 1, li);
  else d = x(t, li) - x(t - 1, li);
  return v.drC(t, li) * v.dc(0, li) * d;
}

// Offset b_C of trade row t: w0 for the first trade, -w_T for the last (multi-period).
template <class SV>
__device__ __forceinline__ double trade_offset(const SV& v, int t, int li) {
  if (t == 0) return v.w0(0, li);
  if (v.p->multi && t == v.p->P) return -v.wT(0, li);
  return 0.0;
}

// Unscaled trade u_t of W = dc * x for asset li.
template <class SV, class A>
__device__ __forceinline__ double trade_of(const SV& v, const A& x, int t, int li) {
  const double dci = v.dc(0, li);
  if (!v.p->multi || t == 0) return dci * x(0, li) - v.w0(0, li);
  if (t == v.p->P) return v.wT(0, li) - dci * x(v.p->P - 1, li);
  return dci * (x(t, li) - x(t - 1, li));
}

// ---------------------------------------------------------------------------------
// Exact L1-budget multiplier
// ---------------------------------------------------------------------------------
// S_t(mu) = sum_i max(|b_ti| - mu, 0) / a_ti with signed b in bb and 1/a in aa.

// Bracket candidates for period t: cen + f_q * hw, f = (-64, -16, -4, -1, 1, 4, 16, 64),
// clamped at 0.  The central pair (q = 3, 4) is the predicted bracket [lo, hi].
__device__ __forceinline__ double cand(double cen, double hw, int q) {
  const double f = (q < 4 ? -1.0 : 1.0) * (double)(1 << (2 * (q < 4 ? 3 - q : q - 4)));
  return fmax(cen + f * hw, 0.0);
}

// Statistics of S_t at the bracket candidates for every period t, published at
// off0 + STW*t: [S(0), max |b|, (S(c_q), A0(c_q), cnt(c_q)) for q < NC] with
// A0(c) = sum_{|b| > c} 1/a and cnt(c) = #{|b| > c}.  absb/inva: LDS [P][nw] with |b|
// and 1/a of the owned assets.  One wave per period, eight lanes per candidate.  The
// caller sets the max-combined range and synchronises before the exchange.
__device__ __forceinline__ void period_stats(Ctx& c, const ldbl* absb, const ldbl* inva, int nw, const ldbl* cen,
                             const ldbl* hw, int off0) {
  const int lane = c.tid & 63, wave = c.tid >> 6, g = lane >> 3, sub = lane & 7;
  // waves per period: all of them share one period's assets when there are few periods
  // and many assets; one period of at most 64 assets stays in wave 0 (a few elements per
  // lane, and no combine through LDS with its two barriers)
  const int WP = (c.P >= NWAVE || (c.P == 1 && c.nwa <= 64)) ? 1 : (c.P >= NWAVE / 2 ? 2 : NWAVE);
  const int pw = wave % WP, tw = wave / WP, groups = NWAVE / WP;
  static_assert(NWAVE * 32 <= RED_OUT, "reduction scratch");
  for (int t0 = 0; t0 < c.P; t0 += groups) {
    const int t = t0 + tw;
    const bool act = tw < groups && t < c.P;
    double S = 0.0, A0 = 0.0, N = 0.0, S0 = 0.0, mx = 0.0;
    if (act) {
      const double cq = cand(cen[t], hw[t], g);
      for (int li = pw * 8 + sub; li < c.nwa; li += 8 * WP) {
        const double ab = absb[t * nw + li], ia = inva[t * nw + li];
        S0 = fma(ab, ia, S0);
        mx = fmax(mx, ab);
        if (ab > cq) { S = fma(ab - cq, ia, S); A0 += ia; N += 1.0; }
      }
    }
    S = sum8(S); A0 = sum8(A0); N = sum8(N); S0 = sum8(S0); mx = max8(mx);
    if (WP == 1) {
      if (act) {
        const int off = off0 + STW * t;
        if (sub == 0) { put(c, off + 2 + 3 * g, S); put(c, off + 3 + 3 * g, A0); put(c, off + 4 + 3 * g, N); }
        if (lane == 0) { put(c, off, S0); put_max(c, off + 1, mx); }
      }
    } else {
      // combine the WP waves of each period through LDS (fixed order)
      // per wave: [4g, 4g+3) candidate g's (S, A0, cnt); slot 3 = S(0), slot 7 = max |b|
      if (sub == 0) {
        ldbl* r = c.red + wave * 32 + 4 * g;
        r[0] = S; r[1] = A0; r[2] = N;
        if (g == 0) r[3] = S0;
        if (g == 1) r[3] = mx;
      }
      __syncthreads();
      if (pw == 0 && act && sub == 0) {
        double s3[3] = {0.0, 0.0, 0.0}, s0 = 0.0, m0 = 0.0;
        for (int w = wave; w < wave + WP; ++w) {
          const ldbl* r = c.red + w * 32 + 4 * g;
          s3[0] += r[0]; s3[1] += r[1]; s3[2] += r[2];
          s0 += c.red[w * 32 + 3];
          m0 = fmax(m0, (double)c.red[w * 32 + 7]);
        }
        const int off = off0 + STW * t;
        put(c, off + 2 + 3 * g, s3[0]); put(c, off + 3 + 3 * g, s3[1]); put(c, off + 4 + 3 * g, s3[2]);
        if (g == 0) { put(c, off, s0); put_max(c, off + 1, m0); }
      }
      __syncthreads();
    }
  }
}

// Decision from the exchanged statistics st[STW] and the global max |b|:
// st = the period's exchanged statistics (st[1] = max |b| over all assets):
//   1 = mu exact from the central pair (the speculative K~ xbar is valid),
//   4 = mu exact from another breakpoint-free candidate interval,
//   2 = mu = 0 while the central pair was not [0, 0],
//   0 = multisection needed, root in the central pair (breakpoints inside it),
//   3 = multisection needed, root outside the central pair.
// For 0 and 3, lo/hi receive a bracket with S(lo) >= 1 >= S(hi), and bits 4 and up of the
// result hold qs + 1, where lo = c_qs is the bracket's lower candidate (qs = -1: lo is 0 or
// the bracket is [0, max |b|]).
// Called by a whole wave (uniform arguments; the candidate tests use one lane each).
__device__ int bracket_decide(const ldbl* st, double cen, double hw, double& lo, double& hi, double& mu) {
  const double S0 = st[0], maxb = st[1];
  if (S0 <= 1.0) { mu = 0.0; return (cen + hw <= 0.0) ? 1 : 2; }
  const int lane = threadIdx.x & 63;
  const unsigned long long ge = __ballot(lane < NC && st[2 + 3 * (lane < NC ? lane : 0)] >= 1.0);
  int qs = ge ? 63 - __clzll((long long)ge) : -1;   // S is non-increasing: {q : S(c_q) >= 1} = [0, qs]
  double a, b;
  if (qs < 0) { a = 0.0; b = cand(cen, hw, 0); }
  else if (qs == NC - 1) { a = cand(cen, hw, NC - 1); b = maxb; }
  else { a = cand(cen, hw, qs); b = cand(cen, hw, qs + 1); }
  if (qs >= 0 && qs < NC - 1 && st[4 + 3 * qs] == st[4 + 3 * (qs + 1)] && st[3 + 3 * qs] > 0.0) {
    mu = fmin(fmax(a + (st[2 + 3 * qs] - 1.0) / st[3 + 3 * qs], a), b);
    return qs == 3 ? 1 : 4;
  }
  if (!(b >= a)) { a = 0.0; b = maxb; qs = -1; }
  lo = a;
  hi = b;
  return (qs == 3 ? 0 : 3) | ((qs + 1) << 4);
}

// The same decision with eight lanes per period (lane & 7 = candidate, lane >> 3 = group),
// so one wave decides eight periods at once.  Called by the eight lanes of each group that
// has a period; the lanes of a group receive the same results.
__device__ __forceinline__ int bracket_decide8(const ldbl* st, double cen, double hw, double& lo, double& hi,
                                               double& mu) {
  static_assert(NC == 8, "one lane per candidate");
  const double S0 = st[0], maxb = st[1];
  if (S0 <= 1.0) { mu = 0.0; return (cen + hw <= 0.0) ? 1 : 2; }
  const int lane = threadIdx.x & 63, sub = lane & 7, grp = lane >> 3;
  const unsigned long long all = __ballot(st[2 + 3 * sub] >= 1.0);
  const unsigned ge = (unsigned)((all >> (8 * grp)) & 0xFFull);
  int qs = ge ? 31 - __clz(ge) : -1;   // S is non-increasing: {q : S(c_q) >= 1} = [0, qs]
  double a, b;
  if (qs < 0) { a = 0.0; b = cand(cen, hw, 0); }
  else if (qs == NC - 1) { a = cand(cen, hw, NC - 1); b = maxb; }
  else { a = cand(cen, hw, qs); b = cand(cen, hw, qs + 1); }
  if (qs >= 0 && qs < NC - 1 && st[4 + 3 * qs] == st[4 + 3 * (qs + 1)] && st[3 + 3 * qs] > 0.0) {
    mu = fmin(fmax(a + (st[2 + 3 * qs] - 1.0) / st[3 + 3 * qs], a), b);
    return qs == 3 ? 1 : 4;
  }
  if (!(b >= a)) { a = 0.0; b = maxb; qs = -1; }
  lo = a;
  hi = b;
  return (qs == 3 ? 0 : 3) | ((qs + 1) << 4);
}

// Multisection for the periods with need[t] != 0 (caller synchronised; S(lo) >= 1 >= S(hi)):
// MSC candidates per round, TB / MSC lanes per candidate.  absb/inva as in period_stats.
__device__ __forceinline__ bool multisect(Ctx& c, int P, const ldbl* absb, const ldbl* inva, int nw, lint* need, ldbl* lo,
                          ldbl* hi, ldbl* mu, lint* rounds_out) {
  constexpr int MSL = TB / MSC;   // lanes per candidate
  const int q = c.tid / MSL, sub = c.tid % MSL;
  for (int round = 0; round < MS_ROUNDS; ++round) {
    int any = 0;
    for (int t = 0; t < P; ++t) any |= need[t];
    if (!any) return true;
    if (c.tid == 0) ++*rounds_out;
    for (int t = 0; t < P; ++t) {
      if (!need[t]) continue;
      const double cq = lo[t] + (hi[t] - lo[t]) * (double)q / (double)(MSC - 1);
      double S = 0.0, A0 = 0.0, N = 0.0;
      for (int li = sub; li < c.nwa; li += MSL) {
        const double ab = absb[t * nw + li];
        if (ab > cq) { const double ia = inva[t * nw + li]; S = fma(ab - cq, ia, S); A0 += ia; N += 1.0; }
      }
      S = sum_lanes<MSL>(S); A0 = sum_lanes<MSL>(A0); N = sum_lanes<MSL>(N);
      if (sub == 0) {
        const int e = t * MSC + q;
        put(c, 3 * e + 0, S);
        put(c, 3 * e + 1, A0);
        put(c, 3 * e + 2, N);
      }
    }
    if (!xsync(c, 3 * P * MSC)) return false;
    {
      const int lane = c.tid & 63, wave = c.tid >> 6;
      for (int t = wave; t < P; t += NWAVE) {   // one wave per period
        if (!need[t]) continue;
        const ldbl* T0 = c.tot + 3 * t * MSC;
        const unsigned long long ge = __ballot(lane < MSC && T0[3 * (lane < MSC ? lane : 0)] >= 1.0);
        const int qs = ge ? 63 - __clzll((long long)ge) : 0;
        const double l = lo[t], h = hi[t];
        const double cq = l + (h - l) * (double)qs / (double)(MSC - 1);
        const double cn = l + (h - l) * (double)(qs + 1) / (double)(MSC - 1);
        const bool top = qs == MSC - 1;
        const bool linear = !top && T0[3 * qs + 2] == T0[3 * (qs + 1) + 2];
        const bool tiny = (cn - cq) <= 4.0 * 2.220446049250313e-16 * fabs(cn);
        const double m_ = T0[3 * qs + 1] > 0.0 ? cq + (T0[3 * qs] - 1.0) / T0[3 * qs + 1] : cq;
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
          if (top) { mu[t] = h; need[t] = 0; }
          else if (linear || tiny || round == MS_ROUNDS - 1) { mu[t] = fmin(fmax(m_, cq), cn); need[t] = 0; }
          else { lo[t] = cq; hi[t] = cn; }
        }
      }
    }
    __syncthreads();
  }
  return true;
}

// Out-of-line forms of the exchange, the statistics and the multisection.  The solve body
// inlines them when it runs alone on the device (its hot loops then keep the workgroup
// context in registers); the batched kernel calls them, which leaves its long
// device-memory loops enough registers to keep their loads in flight.
__device__ __noinline__ bool xsync_call(Ctx& c, int V) { return xsync(c, V); }
__device__ __noinline__ void period_stats_call(Ctx& c, const ldbl* absb, const ldbl* inva, int nw, const ldbl* cen,
                                               const ldbl* hw, int off0) {
  period_stats(c, absb, inva, nw, cen, hw, off0);
}
__device__ __noinline__ bool multisect_call(Ctx& c, int P, const ldbl* absb, const ldbl* inva, int nw, lint* need,
                                            ldbl* lo, ldbl* hi, ldbl* mu, lint* rounds_out) {
  return multisect(c, P, absb, inva, nw, need, lo, hi, mu, rounds_out);
}
template <bool INL>
__device__ __forceinline__ bool xsync_x(Ctx& c, int V) {
  if constexpr (INL) return xsync(c, V);
  else return xsync_call(c, V);
}
template <bool INL>
__device__ __forceinline__ void period_stats_x(Ctx& c, const ldbl* absb, const ldbl* inva, int nw, const ldbl* cen,
                                               const ldbl* hw, int off0) {
  if constexpr (INL) period_stats(c, absb, inva, nw, cen, hw, off0);
  else period_stats_call(c, absb, inva, nw, cen, hw, off0);
}
template <bool INL>
__device__ __forceinline__ bool multisect_x(Ctx& c, int P, const ldbl* absb, const ldbl* inva, int nw, lint* need,
                                            ldbl* lo, ldbl* hi, ldbl* mu, lint* rounds_out) {
  if constexpr (INL) return multisect(c, P, absb, inva, nw, need, lo, hi, mu, rounds_out);
  else return multisect_call(c, P, absb, inva, nw, need, lo, hi, mu, rounds_out);
}

// ---------------------------------------------------------------------------------
// Breakpoint lists
// ---------------------------------------------------------------------------------
// While it forms the prox inputs, every workgroup publishes, for each period, the owned
// assets whose |b| lies in the window (c_2, c_5] around the prediction (at most LIST_CAP
// of them, and the true count).  When the root falls inside the window, the lists hold
// every breakpoint between the bracket ends, so each workgroup finishes the multiplier
// exactly from them after the statistics barrier (and, in speculative mode, corrects the
// affine K~ xbar with the few columns whose state differs between c_4 and mu) instead of
// spending further exchanges.  Every workgroup reads the same lists and sorts them the
// same way, so all of them reach bit-identical results.
constexpr int NPOOL = TB;    // listed breakpoints gathered per iteration (all periods)

__device__ __forceinline__ double* list_at(const double* blist, int par, int nwg, int P, int w, int t) {
  return (double*)blist + (((size_t)par * nwg + w) * P + t) * LIST_W;
}

// Gathers the lists of every period t with gneed[t] > 0 into pool[NPOOL][4] = (|b|, 1/a,
// asset, sign(b)/(a dc)), period t in the entries [poff[t], poff[t] + ptot[t]), sorted by
// (|b|, asset).  Periods take pool space in order; a period whose lists overflowed, or
// that (with all the needing periods before it) does not fit, gets gneed[t] = -1.  Every
// decision here depends only on the published counts, never on the order of the
// appends, so all workgroups agree.  Whole workgroup; ptot is zero on entry and returned
// holding the entry counts.
__device__ __noinline__ void gather_pool(const double* blist, int par, int nwg, int P, lint* gneed, lint* ptot,
                                            lint* poff, lint* pfill, lint* nidx, ldbl* pool, lint* psrc,
                                            lint* pper) {
  constexpr int U = 8;   // pairs per thread with loads in flight together
  const int tid = threadIdx.x;
  // the periods that want their lists, in increasing order, in nidx[0, nidx[P]) (wave 0):
  // the (period, workgroup) pairs below run over those periods only
  if (tid < 64) {
    int carry = 0;
    for (int t0 = 0; t0 < P; t0 += 64) {
      const int t = t0 + tid;
      const bool nd = t < P && gneed[t] > 0;
      const unsigned long long bal = __ballot(nd);
      if (nd) nidx[carry + __popcll(bal & ((1ull << tid) - 1ull))] = t;
      carry += __popcll(bal);
    }
    if (tid == 0) nidx[P] = carry;
  }
  __syncthreads();
  const int npair = nidx[P] * nwg;
  const bool held = npair <= TB * U;   // one pass covers every pair: the counts stay in registers
  double cn[U];
  // pass 1: per-period entry counts
  for (int base = tid; base < npair; base += TB * U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * TB, r = idx / nwg, w = idx - r * nwg;
      cn[u] = idx < npair ? ldd(list_at(blist, par, nwg, P, w, nidx[r])) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!(cn[u] > 0.0)) continue;
      const int t = nidx[(base + u * TB) / nwg], cnt = (int)cn[u];
      if (cnt > LIST_CAP) gneed[t] = -1;
      __hip_atomic_fetch_add(&ptot[t], min(cnt, LIST_CAP), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
  __syncthreads();
  // pool offsets: exclusive prefix over the needing periods (wave 0, one lane per period)
  if (tid < 64) {
    int carry = 0;
    for (int t0 = 0; t0 < P; t0 += 64) {
      const int t = t0 + tid;
      const int g = t < P ? (int)gneed[t] : 0;
      const int v = g > 0 ? (int)ptot[t] : 0;
      int incl = v;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(incl, d);
        if (tid >= d) incl += o;
      }
      const int excl = carry + incl - v;
      if (t < P) {
        const bool fits = g > 0 && excl + v <= NPOOL;
        if (g > 0 && !fits) gneed[t] = -1;
        ptot[t] = fits ? v : 0;
        poff[t] = excl;
        pfill[t] = 0;
      }
      carry += __shfl(incl, 63);
    }
  }
  __syncthreads();
  // pass 2: every listed entry gets its pool position and source (list slot, entry) in
  // LDS, then one thread per entry loads it: one round trip for the whole pool
  for (int base = tid; base < npair; base += TB * U) {
    if (!held) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * TB, r = idx / nwg, w = idx - r * nwg;
        cn[u] = (idx < npair && gneed[nidx[r]] > 0) ? ldd(list_at(blist, par, nwg, P, w, nidx[r])) : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * TB, r = idx / nwg, w = idx - r * nwg;
      if (idx >= npair) continue;
      const int t = nidx[r];
      if (!(cn[u] > 0.0) || gneed[t] <= 0) continue;
      const int kmax = min((int)cn[u], LIST_CAP);
      const int pos = poff[t] + __hip_atomic_fetch_add(&pfill[t], kmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      for (int k = 0; k < kmax; ++k) {
        psrc[pos + k] = (w * LIST_CAP + k);
        pper[pos + k] = t;
      }
    }
  }
  __syncthreads();
  // the pool's extent: the last needing period's offset plus its entries
  int total = 0;
  for (int r = 0; r < nidx[P]; ++r) {
    const int t = nidx[r];
    if (gneed[t] > 0) total = max(total, (int)poff[t] + (int)ptot[t]);
  }
  double e0 = 0.0, e1 = 0.0, e2 = 0.0, e3 = 0.0;
  const int i = tid;   // NPOOL == TB: one entry per thread
  int t = -1;
  if (i < total) {
    t = pper[i];
    const int src = psrc[i], w = src / LIST_CAP, k = src - w * LIST_CAP;
    const double* L = list_at(blist, par, nwg, P, w, t) + 1 + 4 * k;
    e0 = ldd(L); e1 = ldd(L + 1); e2 = ldd(L + 2); e3 = ldd(L + 3);
    ldbl* q = pool + 4 * i;
    q[0] = e0; q[1] = e1; q[2] = e2; q[3] = e3;
  }
  __syncthreads();
  // sort each period's entries in place by (|b|, asset): entry i takes its rank among its
  // period's entries (four comparisons per step)
  int dst = -1;
  if (t >= 0) {
    const int j0 = poff[t], j1 = j0 + ptot[t];
    int r0 = 0, r1 = 0, r2 = 0, r3 = 0;
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
      const double v0 = pool[4 * j], v1 = pool[4 * j + 4], v2 = pool[4 * j + 8], v3 = pool[4 * j + 12];
      const double g0 = pool[4 * j + 2], g1 = pool[4 * j + 6], g2 = pool[4 * j + 10], g3 = pool[4 * j + 14];
      r0 += (v0 < e0 || (v0 == e0 && g0 < e2)) ? 1 : 0;
      r1 += (v1 < e0 || (v1 == e0 && g1 < e2)) ? 1 : 0;
      r2 += (v2 < e0 || (v2 == e0 && g2 < e2)) ? 1 : 0;
      r3 += (v3 < e0 || (v3 == e0 && g3 < e2)) ? 1 : 0;
    }
    for (; j < j1; ++j) {
      const double vj = pool[4 * j], gj = pool[4 * j + 2];
      r0 += (vj < e0 || (vj == e0 && gj < e2)) ? 1 : 0;
    }
    dst = j0 + (r0 + r1) + (r2 + r3);
  }
  __syncthreads();
  if (dst >= 0) {
    ldbl* q = pool + 4 * dst;
    q[0] = e0; q[1] = e1; q[2] = e2; q[3] = e3;
  }
}

// Index range [k0, k1) of the sorted entries pool[a, a + cnt) with |b| in (lo, hi] (one
// whole wave; uniform result).
__device__ __forceinline__ void pool_range(const ldbl* pool, int a, int cnt, double lo, double hi, int& k0, int& k1) {
  const int lane = threadIdx.x & 63;
  int nb = 0, nu = 0;
  for (int j0 = 0; j0 < cnt; j0 += 64) {
    const int j = j0 + lane;
    const double v = j < cnt ? (double)pool[4 * (a + j)] : INFINITY;
    nb += __popcll(__ballot(v <= lo));
    nu += __popcll(__ballot(v <= hi));
  }
  k0 = a + nb;
  k1 = a + nu;
}

// Exact root of S(mu) = 1 on [lo, hi] from S(lo), A0(lo) and the sorted breakpoints in
// (lo, hi] (one whole wave; uniform result).  Between breakpoints S is affine:
// S(v_k) = S(lo) - (v_k - lo) A0(lo) + sum_{j<k} (v_k - v_j)/a_j, slope -(A0(lo) - sum_{j<=k} 1/a_j).
__device__ double solve_from_list(const ldbl* buf, int n, double lo, double hi, double Slo, double Alo) {
  const int lane = threadIdx.x & 63;
  double Sk = 0.0, slope_after = 0.0;
  if (lane < n) {
    const double v = buf[lane * 4];
    double acc = Slo - (v - lo) * Alo, iasum = 0.0;
    for (int j = 0; j < lane; ++j) acc = fma(v - buf[j * 4], buf[j * 4 + 1], acc);
    for (int j = 0; j <= lane; ++j) iasum += buf[j * 4 + 1];
    Sk = acc;
    slope_after = Alo - iasum;
  }
  const unsigned long long ge = __ballot(lane < n && Sk >= 1.0);
  double mu;
  if (!ge) {
    const double nxt = n > 0 ? (double)buf[0] : hi;
    mu = Alo > 0.0 ? lo + (Slo - 1.0) / Alo : lo;
    mu = fmin(fmax(mu, lo), nxt);
  } else {
    const int k = 63 - __clzll((long long)ge);
    const double vk = buf[k * 4];
    const double Skk = lane_of(Sk, k), sl = lane_of(slope_after, k);
    const double nxt = k + 1 < n ? (double)buf[(k + 1) * 4] : hi;
    mu = sl > 0.0 ? vk + (Skk - 1.0) / sl : vk;
    mu = fmin(fmax(mu, vk), nxt);
  }
  return mu;
}

// Relative half-width policy after a decision r (see bracket_decide): kept on a hit,
// shrunk when breakpoints fell inside the central pair, grown when the root was outside.
__device__ __forceinline__ double adapt_width(int r, double w) {
  if (r == 1 || r == 2) return w;
  if (r == 0) return fmax(w * 0.7, 1e-13);
  return fmin(w * 1.6, 0.25);   // r = 3, 4: the root fell outside the central pair
}

// Next prediction: centre at the trend mu + (mu - mu_prev), half-width w * mu.
__device__ __forceinline__ void next_bracket(double mu, double mprev, double w, ldbl& cen, ldbl& hw) {
  if (mu <= 0.0) { cen = 0.0; hw = 0.0; return; }
  cen = fmax(mu + (mu - mprev), 0.5 * mu);
  hw = w * mu;
}

// ---------------------------------------------------------------------------------
// The kernel
// ---------------------------------------------------------------------------------
struct Scal {   // uniform scalars kept in LDS (identical in every workgroup)
  double omega, eta, r0, rprev;
  long long it, kk, restarts, spec_miss, checks, miss_in, miss_out;
  int done, status, restart, ms_rounds;
};

extern __shared__ double g_lds[];

// Doubles of LDS taken by `count` elements of type R (every array starts 8-byte aligned).
template <class R>
__host__ __device__ constexpr size_t lds_doubles(size_t count) { return (count * sizeof(R) + 7) / 8; }

// One solve by a team of nwg workgroups; this workgroup is rank wg of the team.
// Elementwise pass over e in [0, ne) with two elements per thread and step, for per-asset
// state in device memory: both elements' loads are issued before the first store.  With
// one element per step every element waits a full memory round trip, because the compiler
// cannot move a load above a store that may alias it.  Elements are taken in the order
// of a one-element loop.
template <class L, class W>
__device__ __forceinline__ void each2(int tid, int ne, L load, W work) {
  for (int e = tid; e < ne; e += 2 * TB) {
    const int e1 = e + TB;
    const bool two = e1 < ne;
    const auto a = load(e);
    const auto b = load(two ? e1 : e);
    work(a);
    if (two) work(b);
  }
}

template <bool KL, bool SL, class R, bool LS, class KGT = typename default_kg<R>::type>
__device__ __forceinline__ void solve_body(const DevProblem& p, const DevState& s, const DevControl& ctl, int wg,
                                           int nwg) {
  ldbl* lds = (ldbl*)g_lds;
  const int P = p.P, nr = p.nr, n = p.n, Tp = p.Tp, nw = ctl.nw;
  Ctx c;
  c.wg = wg;
  c.nwg = nwg;
  c.tid = threadIdx.x;
  c.i0 = c.wg * nw;
  c.nwa = max(0, min(nw, n - c.i0));
  c.epoch = 0;
  c.xbuf = s.xbuf;
  c.bar = s.bar;
  c.vmax = ctl.vmax;
  c.xmode = ctl.xmode;
  c.ng = ctl.xmode == XM_ATOMIC ? max(1, min(ctl.xgroups, min(XG_MAX, nwg))) : 1;
  c.grp = wg % c.ng;
  c.gsize = (nwg - c.grp + c.ng - 1) / c.ng;
  c.P = P;
  c.spin_limit = ctl.spin_limit;
  c.mx_lo = c.mx_hi = 0;
  c.t_wait = 0;
  c.t_pre = 0;
  c.t_read = 0;
  long long t_phA = 0, t_phB = 0, t_phC = 0, t_phD = 0, t_b1 = 0, t_b2 = 0, t_b3 = 0, t_b1s = 0, t_gather = 0;
  long long n_gather = 0;

  // LDS layout (doubles); must match solve_lds_bytes
  ldbl* ptr = lds;
  lds_t<R>* Kl = nullptr;
  const int ldl = nw | 1;   // odd row stride: row-parallel reads spread over the LDS banks
  if (KL) { Kl = (lds_t<R>*)ptr; ptr += lds_doubles<R>((size_t)nr * ldl); }
  ldbl* ys = ptr;   ptr += P * nr;
  ldbl* ys0 = ptr;  ptr += P * nr;          // anchor (= last restart point)
  ldbl* Tys = ptr;  ptr += P * nr;
  ldbl* Kx = ptr;   ptr += P * nr;          // K~ xbar rows (exchanged)
  ldbl* xv1 = ptr;  ptr += P * nw;          // staging
  ldbl* xv2 = ptr;  ptr += P * nw;          // staging
  ldbl* xv3 = ptr;  ptr += P * nw;          // |b| of the current multiplier problem
  ldbl* xv4 = ptr;  ptr += P * nw;          // 1/a of the current multiplier problem
  ldbl* tot = ptr;  ptr += ctl.vmax;
  ldbl* red = ptr;  ptr += RED_LEN;
  ldbl* ks = ptr;   ptr += nr;              // row scale applied to rows read from device memory
  ldbl* lslot = nullptr;
  if (ctl.xmode == XM_LOCAL) { lslot = ptr; ptr += 3 * (size_t)ctl.vmax; }
  ldbl* cen = ptr;  ptr += P;               // predicted multiplier (centre) ...
  ldbl* hw = ptr;   ptr += P;               // ... and half-width of the central pair
  ldbl* lo = ptr;   ptr += P;               // multisection bracket
  ldbl* hi = ptr;   ptr += P;
  ldbl* mu = ptr;   ptr += P;
  ldbl* mpv = ptr;  ptr += P;               // previous mu (trend)
  ldbl* wid = ptr;  ptr += P;               // relative half-width
  ldbl* dcen = ptr; ptr += P;               // the same for the dual inner problem
  ldbl* dhw = ptr;  ptr += P;
  ldbl* dlo = ptr;  ptr += P;
  ldbl* dhi = ptr;  ptr += P;
  ldbl* dmu = ptr;  ptr += P;
  ldbl* dmp = ptr;  ptr += P;
  ldbl* dwd = ptr;  ptr += P;
  const bool lists = LS && ctl.lists;       // breakpoint lists (single-team launches only)
  ldbl* pool = nullptr;                     // gathered breakpoint lists (sorted)
  lint* psrc = nullptr;                     // per pool entry: its list slot and entry, its period
  lint* pper = nullptr;
  if (lists) {
    pool = ptr; ptr += NPOOL * 4;
    psrc = (lint*)ptr; ptr += NPOOL / 2;
    pper = (lint*)ptr; ptr += NPOOL / 2;
  }
  using SV = S<KL, SL, R, KGT>;
  SV V;
  V.p = &p;
  V.nw = nw;
  V.ldl = ldl;
  V.i0 = c.i0;
  if constexpr (SL) {
    auto take = [&](auto tag, int rows) {
      using E = decltype(tag);
      Arr<SL, E> r{(lds_t<E>*)ptr, nw, 0};
      ptr += lds_doubles<E>((size_t)rows * nw);
      return r;
    };
    const double fd = 0.0;
    const R fr = 0;
    const typename SV::RC fc = 0;
    V.x0s = take(fd, P); V.bb = take(fd, P); V.aa = take(fd, P); V.xb = take(fd, P);
    V.xs = {V.x0s, take(fr, P)}; V.Txs = {V.x0s, take(fr, P)};
    V.ys0C = take(fd, Tp);
    V.ysC = {V.ys0C, take(fr, Tp)}; V.TysC = {V.ys0C, take(fr, Tp)};
    V.alpha = take(fc, P); V.ca = take(fc, Tp); V.cb = take(fc, Tp); V.drC = take(fd, Tp);
    V.dc = take(fd, 1); V.arisk = take(fc, 1); V.cvec = take(fd, 1); V.w0 = take(fd, 1); V.wT = take(fd, 1);
  } else {
    // state buffers hold [P or Tp][n] elements (iterates of type R); constants are the
    // FP64 inputs
    auto gs = [&](const double* b) { return Arr<SL, R>{(R*)b, n, c.i0}; };
    auto g = [&](const double* b) { return Arr<SL, double>{(double*)b, n, c.i0}; };
    V.x0s = g(s.x0s); V.bb = g(s.bb); V.aa = g(s.aa); V.xb = g(s.vpow);
    V.xs = {V.x0s, gs(s.xs)}; V.Txs = {V.x0s, gs(s.Txs)};
    V.ys0C = g(s.ys0C);
    V.ysC = {V.ys0C, gs(s.ysC)}; V.TysC = {V.ys0C, gs(s.TysC)};
    V.alpha = g(p.alpha); V.ca = g(p.ca); V.cb = g(p.cb); V.drC = g(p.drC);
    V.dc = g(p.dc); V.arisk = g(p.arisk); V.cvec = g(p.cvec); V.w0 = g(p.w0);
    V.wT = g(p.wT ? p.wT : p.w0);
  }
  // FP64 view of the problem (device-memory rows and constants) for the checks of the
  // FP32 form; the FP64 form checks with the same view it iterates with.
  S<false, false, double> G;
  {
    auto g = [&](const double* b) { return Arr<false, double>{(double*)b, n, c.i0}; };
    G.p = &p; G.Kl = nullptr; G.Kg = p.K; G.ks = ks; G.nw = nw; G.ldl = ldl; G.i0 = c.i0;
    G.alpha = g(p.alpha); G.ca = g(p.ca); G.cb = g(p.cb); G.drC = g(p.drC);
    G.dc = g(p.dc); G.arisk = g(p.arisk); G.cvec = g(p.cvec); G.w0 = g(p.w0);
    G.wT = g(p.wT ? p.wT : p.w0);
  }
  auto& Vc = [&]() -> auto& {
    if constexpr (std::is_same<R, double>::value) return V;
    else return G;
  }();
  __attribute__((address_space(3))) Scal* sc = (__attribute__((address_space(3))) Scal*)ptr;
  ptr += (sizeof(Scal) + 7) / 8;
  lint* iflag = (lint*)ptr; ptr += 2;       // [0] exchange status, [1] fallback, [2] miss, [3] spare
  lint* fbflag = iflag + 1;
  lint* msflag = iflag + 2;
  lint* need = (lint*)ptr;
  lint* ncor = need + P;                    // per period: list corrections of K~ xbar (-1: none) ...
  lint* ncs = ncor + P;                     // ... starting at this pool entry
  lint* gneed = ncs + P;                    // per period: lists wanted (1 solve, 2 correction), -1 overflow
  lint* ldec = gneed + P;                   // per period: bracket decision
  lint* lcnt = ldec + P;                    // per period: entries published by this workgroup
  lint* ptot = lcnt + P;                    // per period: gathered entries, their first pool
  lint* poff = ptot + P;                    // entry, and the fill counter
  lint* pfill = poff + P;
  lint* nidx = pfill + P;                   // [P + 1]: periods gathering lists, their count
  c.tot = tot;
  c.red = red;
  c.flag = iflag;
  c.lslot = lslot;
  V.Kl = Kl;
  if constexpr (std::is_same<typename SV::KG, bf16>::value) V.Kg = (const bf16*)p.Kb;
  else if constexpr (std::is_same<typename SV::KG, float>::value) V.Kg = p.Kf;
  else V.Kg = p.K;
  V.ks = ks;

  for (int j = c.tid; j < nr; j += TB) ks[j] = p.kscaled ? 1.0 : p.dr[j];
  if (lslot)
    for (int e = c.tid; e < 3 * ctl.vmax; e += TB) lslot[e] = 0.0;
  __syncthreads();
  if (KL) {
    for (int e = c.tid; e < nr * nw; e += TB) {
      const int j = e / nw, li = e % nw;
      Kl[j * ldl + li] = li < c.nwa ? p.K[(size_t)j * p.ldk + c.i0 + li] * ks[j] : 0.0;
    }
  }
  if (SL) {
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      V.alpha(t, li) = p.alpha[(size_t)t * n + c.i0 + li];
    }
    for (int e = c.tid; e < Tp * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const size_t ix = (size_t)t * n + c.i0 + li;
      V.ca(t, li) = p.ca[ix]; V.cb(t, li) = p.cb[ix]; V.drC(t, li) = p.drC[ix];
    }
    for (int li = c.tid; li < c.nwa; li += TB) {
      const int i = c.i0 + li;
      V.dc(0, li) = p.dc[i]; V.arisk(0, li) = p.arisk[i]; V.cvec(0, li) = p.cvec[i];
      V.w0(0, li) = p.w0[i]; V.wT(0, li) = p.wT ? p.wT[i] : 0.0;
    }
  }
  // starting duals: zero, or the caller's (unscaled, y_out layout) divided by the row scales
  for (int e = c.tid; e < P * nr; e += TB) {
    double y = 0.0;
    if (s.y_init) {
      const int t = e / nr, j = e % nr;
      const double yu = j < p.m ? s.y_init[(size_t)t * p.m + j] : s.y_init[(size_t)P * p.m + (size_t)t * p.k + (j - p.m)];
      y = yu / p.dr[j];
    }
    ys[e] = y; ys0[e] = y; Tys[e] = y; Kx[e] = 0.0;
  }
  if (c.tid == 0) {
    sc->omega = ctl.omega0 > 0.0 ? ctl.omega0 : 1.0; sc->it = 0; sc->kk = 0; sc->restarts = 0; sc->spec_miss = 0; sc->checks = 0;
    sc->miss_in = 0; sc->miss_out = 0;
    sc->r0 = -1.0; sc->rprev = INFINITY; sc->done = 0; sc->status = DS_RUNNING; sc->restart = 0;
    sc->ms_rounds = 0;
    fbflag[0] = 0;
    msflag[0] = 0;
    for (int t = 0; t < P; ++t) {
      cen[t] = 0.0; hw[t] = 0.0; lo[t] = 0.0; hi[t] = 0.0; mu[t] = 0.0; mpv[t] = 0.0; wid[t] = 1e-3;
      dcen[t] = 0.0; dhw[t] = 0.0; dlo[t] = 0.0; dhi[t] = 0.0; dmu[t] = 0.0; dmp[t] = 0.0; dwd[t] = 1e-3;
      need[t] = 0;
      ncor[t] = -1; ncs[t] = 0; gneed[t] = 0; ldec[t] = 0; lcnt[t] = 0;
      ptot[t] = 0; poff[t] = 0; pfill[t] = 0;
    }
  }
  __syncthreads();
  // initial primal point: w0 in every period (paper Section 4.1), or the caller's warm
  // start; trade duals zero or the caller's.  Scaled coordinates: x = w / dc, y = y_u / dr.
  for (int e = c.tid; e < P * c.nwa; e += TB) {
    const int t = e / c.nwa, li = e % c.nwa, i = c.i0 + li;
    const double x = s.w_init ? s.w_init[(size_t)t * n + i] / p.dc[i] : V.w0(0, li) / V.dc(0, li);
    V.x0s(t, li) = x; V.xs.set(t, li, x); V.Txs.set(t, li, x);
    V.xb(t, li) = 1.0 + 0.25 * (double)((i * 7919 + t * 104729) % 1000) / 1000.0;   // power vector
  }
  for (int e = c.tid; e < Tp * c.nwa; e += TB) {
    const int t = e / c.nwa, li = e % c.nwa;
    const size_t ix = (size_t)t * n + c.i0 + li;
    const double y = s.y_init ? s.y_init[(size_t)P * nr + ix] / p.drC[ix] : 0.0;
    V.ys0C(t, li) = y; V.ysC.set(t, li, y); V.TysC.set(t, li, y);
  }
  __syncthreads();
  const long long t_start = wall_clock64();
  long long t_check = 0;
  long long t_loop = t_start;
  int lpar = 0;   // list buffer of this iteration (alternates)

  // ------------------------------------------------------------- power iteration
  // lambda ~ ||K~ v||^2 / ||v||^2 ; v <- K~^T K~ v / (lambda ||v||)  (v kept in xb)
  double lam = 0.0;
  for (int pw = 0; pw < ctl.npow; ++pw) {
    double loc[2] = {0.0, 0.0};
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double x = V.xb(t, li);
      xv1[t * nw + li] = x;
      loc[0] = fma(x, x, loc[0]);
    }
    for (int e = c.tid; e < Tp * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double u = kx_trade(V, V.xb, t, li);
      loc[1] = fma(u, u, loc[1]);
    }
    wg_sum<2>(c, loc);
    if (c.tid == 0) { put(c, 0, red[RED_OUT]); put(c, 1, red[RED_OUT + 1]); }
    __syncthreads();
    rows_prod<1>(c, V, xv1, xv1, nw, P, nr, 2);
    if (!xsync_x<LS>(c, 2 + P * nr)) goto barrier_fail;
    {
      const double vv = tot[0];
      double kv = tot[1];
      for (int e = 0; e < P * nr; ++e) kv = fma(tot[2 + e], tot[2 + e], kv);
      lam = vv > 0.0 ? kv / vv : 0.0;
      const double scale = (lam > 0.0 && vv > 0.0) ? 1.0 / (lam * sqrt(vv)) : 1.0;
      kty_all(c, V, tot + 2, P, nr, nw, xv2);
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double r = xv2[t * nw + li];
        double uc = kx_trade(V, V.xb, t, li) * V.drC(t, li) * V.dc(0, li);
        if (p.multi) uc -= kx_trade(V, V.xb, t + 1, li) * V.drC(t + 1, li) * V.dc(0, li);
        xv2[t * nw + li] = (r + uc) * scale;
      }
      __syncthreads();
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        V.xb(t, li) = xv2[t * nw + li];
      }
      __syncthreads();
    }
  }
  if (c.tid == 0) sc->eta = ctl.eta_safety / sqrt(fmax(lam, 1e-300));
  __syncthreads();
  t_loop = wall_clock64();

  // ------------------------------------------------------------- main loop
  while (true) {
    const double omega = sc->omega, eta = sc->eta;
    const double tau = eta / omega, sigma = eta * omega;
    const bool check = ((sc->it + 1) % ctl.check_every == 0) || (sc->it + 1 >= ctl.max_iter);

    const long long ta0 = wall_clock64();
    // Phase A: prox inputs (signed b and 1/a) for owned (t, li).
    kty_all<LS ? 2 : 1>(c, V, ys, P, nr, nw, xv1);
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double Ry = xv1[t * nw + li] + kty_trade(V, V.ysC, t, li);
      const double v = V.xs(t, li) - tau * Ry;
      const double dci = V.dc(0, li);
      const double a = 1.0 / (tau * dci * dci) + V.arisk(0, li);
      const double b = v / (tau * dci) + V.alpha(t, li) + V.arisk(0, li) * V.cvec(0, li);
      V.bb(t, li) = b;
      V.aa(t, li) = 1.0 / a;
      xv3[t * nw + li] = fabs(b);
      xv4[t * nw + li] = 1.0 / a;
      if (lists) {
        const double ab = fabs(b);
        if (ab > cand(cen[t], hw[t], 2) && ab <= cand(cen[t], hw[t], 5)) {
          const int pos = __hip_atomic_fetch_add(&lcnt[t], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (pos < LIST_CAP) {
            double* L = list_at(s.blist, lpar, nwg, P, c.wg, t) + 1 + 4 * pos;
            std_(L, ab);
            std_(L + 1, 1.0 / a);
            std_(L + 2, (double)(c.i0 + li));
            std_(L + 3, sgn(b) / (a * dci));
          }
        }
      }
    }
    __syncthreads();
    if (lists)
      for (int t = c.tid; t < P; t += TB) {
        std_(list_at(s.blist, lpar, nwg, P, c.wg, t), (double)lcnt[t]);
        lcnt[t] = 0;
      }
    const long long tb0 = wall_clock64();
    t_phA += tb0 - ta0;

    // Phase B: the multiplier mu_t and K~ xbar.
    {
      const int oP1 = STW * P, oP2 = oP1 + P * nr;
      const int VE1 = ctl.spec ? oP2 + P * nr : STW * P;
      period_stats_x<LS>(c, xv3, xv4, nw, cen, hw, 0);
      t_b1s += wall_clock64() - tb0;
      if (ctl.spec) {
        // affine pieces at hi: P1 = K~ (2 xhat_s(hi) - xs), P2 = K~ d xhat_s / d mu
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double b = V.bb(t, li), ab = fabs(b), ia = V.aa(t, li), dci = V.dc(0, li);
          const double h = cand(cen[t], hw[t], 4);
          const double xh = ab > h ? sgn(b) * (ab - h) * ia / dci : 0.0;
          xv1[t * nw + li] = 2.0 * xh - V.xs(t, li);
          xv2[t * nw + li] = ab > h ? -sgn(b) * ia / dci : 0.0;
        }
        __syncthreads();
        rows_prod<2>(c, V, xv1, xv2, nw, P, nr, oP1, oP2);
      }
      const long long tb1 = wall_clock64();
      t_b1 += tb1 - tb0;
      c.mx_lo = 0;
      c.mx_hi = STW * P;
      if (!xsync_x<LS>(c, VE1)) goto barrier_fail;
      const long long tb2 = wall_clock64();
      if constexpr (!LS) {
        const int lane = c.tid & 63, wave = c.tid >> 6;
        for (int t = wave; t < P; t += NWAVE) {   // one wave per period
          double l = 0.0, h = 0.0, m_ = 0.0;
          const int r = bracket_decide(tot + STW * t, cen[t], hw[t], l, h, m_) & 15;
          if (lane == 0) {
            wid[t] = adapt_width(r, wid[t]);
            mpv[t] = mu[t];
            if (r == 1) {
              mu[t] = m_;
              need[t] = 0;
            } else if (r == 2 || r == 4) {
              mu[t] = m_;
              need[t] = 0;
              __hip_atomic_fetch_or(fbflag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
              lo[t] = l; hi[t] = h;
              need[t] = 1;
              __hip_atomic_fetch_or(fbflag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
              __hip_atomic_fetch_or(msflag, r == 0 ? 1 : 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
          }
        }
      } else {
        {
          const int lane = c.tid & 63, wave = c.tid >> 6, grp = lane >> 3, sub = lane & 7;
          for (int t0 = wave * 8; t0 < P; t0 += NWAVE * 8) {   // eight periods per wave
            const int t = t0 + grp;
            if (t >= P) continue;
            double l = 0.0, h = 0.0, m_ = 0.0;
            const int rq = bracket_decide8(tot + STW * t, cen[t], hw[t], l, h, m_);
            if (sub == 0) {
              const int r0 = rq & 15, qs = (rq >> 4) - 1;
              int g = 0;
              if (lists && r0 != 1) {
                const double c2 = cand(cen[t], hw[t], 2), c5 = cand(cen[t], hw[t], 5);
                if ((r0 == 0 || r0 == 3) && qs >= 2 && qs <= 4 && l >= c2 && h <= c5) g = 1;   // solve from lists
                else if (ctl.spec && (r0 == 2 || r0 == 4) && m_ >= c2 && m_ <= c5) g = 2;       // correct K~ xbar
              }
              gneed[t] = g;
              ldec[t] = rq;
              lo[t] = l; hi[t] = h;
              wid[t] = adapt_width(r0, wid[t]);
              mpv[t] = mu[t];
              if (r0 != 0 && r0 != 3) mu[t] = m_;
            }
          }
        }
        __syncthreads();
        if (lists) {
          int anyg = 0;
          for (int t = 0; t < P; ++t) anyg |= gneed[t];
          if (anyg) {
            const long long tg0 = wall_clock64();
            gather_pool(s.blist, lpar, nwg, P, gneed, ptot, poff, pfill, nidx, pool, psrc, pper);
            __syncthreads();
            t_gather += wall_clock64() - tg0;
            ++n_gather;
          }
        }
        {
          const int lane = c.tid & 63, wave = c.tid >> 6;
          for (int t = wave; t < P; t += NWAVE) {   // one wave per period
            const int rq = ldec[t], r0 = rq & 15, qs = (rq >> 4) - 1, g = gneed[t];
            const double l = lo[t], h = hi[t];
            double m_ = mu[t];
            int r = r0, nc = -1, k0 = 0;
            if (g > 0) {
              if (g == 1) {
                int k1;
                pool_range(pool, poff[t], ptot[t], l, h, k0, k1);
                if (k1 - k0 <= 64) {
                  const ldbl* st = tot + STW * t;
                  m_ = solve_from_list(pool + 4 * k0, k1 - k0, l, h, st[2 + 3 * qs], st[3 + 3 * qs]);
                  r = 4;
                }
              }
              const double c4 = cand(cen[t], hw[t], 4);
              if (ctl.spec && r != 0 && r != 3 && m_ >= cand(cen[t], hw[t], 2) && m_ <= cand(cen[t], hw[t], 5)) {
                int k1;
                pool_range(pool, poff[t], ptot[t], fmin(m_, c4), fmax(m_, c4), k0, k1);
                nc = k1 - k0;
              }
            }
            if (lane == 0) {
              ncor[t] = nc;
              ncs[t] = k0;
              if (r == 1) {
                need[t] = 0;
              } else if (r == 2 || r == 4) {
                mu[t] = m_;
                need[t] = 0;
                if (nc < 0) __hip_atomic_fetch_or(fbflag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
              } else {
                need[t] = 1;
                __hip_atomic_fetch_or(fbflag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_or(msflag, r == 0 ? 1 : 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
              }
            }
          }
        }
      }
      __syncthreads();
      if (c.tid == 0) {
        const int anyfb = *fbflag, anymiss = *msflag;
        // speculative mode recomputes K~ xbar after any miss; two-phase always does
        *iflag = ctl.spec ? anyfb : 1;
        if (anymiss || (ctl.spec && anyfb)) sc->spec_miss++;
        if (anymiss & 1) sc->miss_in++;
        if (anymiss & 2) sc->miss_out++;
        *fbflag = 0;
        *msflag = 0;
        if constexpr (LS)
          for (int t = 0; t < P; ++t) ptot[t] = 0;
      }
      __syncthreads();
      const long long tb3 = wall_clock64();
      t_b2 += tb3 - tb2;
      const int redo = *iflag;
      if (!redo) {
        for (int e = c.tid; e < P * nr; e += TB) {
          const int t = e / nr, j = e - t * nr;
          const double c4 = cand(cen[t], hw[t], 4), m_ = mu[t];
          double v = tot[oP1 + e] + 2.0 * (m_ - c4) * tot[oP2 + e];
          const int nc = LS ? (int)ncor[t] : -1;
          if (nc > 0) {
            // x_hat(mu) - (affine piece at c_4) = sgn(b)/(a dc) (|b| - mu) ([|b| > mu] - [|b| > c_4])
            const ldbl* lb = pool + 4 * ncs[t];
            const double* Kr = p.K + (size_t)j * p.ldk;
            double corr = 0.0;
            for (int k = 0; k < nc; ++k) {
              const double vk = lb[4 * k], cf = lb[4 * k + 3];
              const int g = (int)lb[4 * k + 2];
              const double dx = cf * (vk - m_) * ((vk > m_ ? 1.0 : 0.0) - (vk > c4 ? 1.0 : 0.0));
              corr = fma(Kr[g], dx, corr);
            }
            v = fma(2.0 * ks[j], corr, v);
          }
          Kx[e] = v;
        }
        __syncthreads();
      } else {
        int any = 0;
        for (int t = 0; t < P; ++t) any |= need[t];
        if (any && !multisect_x<LS>(c, P, xv3, xv4, nw, need, lo, hi, mu, &sc->ms_rounds)) goto barrier_fail;
        // exact K~ xbar for every period
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double b = V.bb(t, li), ab = fabs(b);
          const double xh = ab > mu[t] ? sgn(b) * (ab - mu[t]) * V.aa(t, li) / V.dc(0, li) : 0.0;
          xv1[t * nw + li] = 2.0 * xh - V.xs(t, li);
        }
        __syncthreads();
        rows_prod<1>(c, V, xv1, xv1, nw, P, nr, 0);
        if (!xsync_x<LS>(c, P * nr)) goto barrier_fail;
        for (int e = c.tid; e < P * nr; e += TB) Kx[e] = tot[e];
        __syncthreads();
      }
      for (int t = c.tid; t < P; t += TB) next_bracket(mu[t], mpv[t], wid[t], cen[t], hw[t]);
      lpar ^= 1;
      __syncthreads();
      t_b3 += wall_clock64() - tb3;
    }

    const long long tcc0 = wall_clock64();
    t_phB += tcc0 - tb0;
    // Phase C: T(z).  Primal: xhat; trades and rows: dual prox.
    // The plain kernel keeps one element per step: two per step reshuffled its registers and
    // slowed the multi-period solve (state in device memory) by ~4%.
    if constexpr (SL || LS) {
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double b = V.bb(t, li), ab = fabs(b);
        const double xh = ab > mu[t] ? sgn(b) * (ab - mu[t]) * V.aa(t, li) / V.dc(0, li) : 0.0;
        V.xb(t, li) = 2.0 * xh - V.xs(t, li);
        V.Txs.set(t, li, xh);
      }
      __syncthreads();
      for (int e = c.tid; e < Tp * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double kc = kx_trade(V, V.xb, t, li);
        const double vs = V.ysC(t, li) + sigma * kc;
        const double drc = V.drC(t, li);
        const double bc = trade_offset(V, t, li);
        const double z = vs / (sigma * drc) - bc;
        const double pr = prox_cost(z, 1.0 / (sigma * drc * drc), V.ca(t, li), V.cb(t, li), p.d);
        V.TysC.set(t, li, vs - sigma * drc * bc - sigma * drc * pr);
      }
    } else {   // the same arithmetic, two elements per step
      struct InX { double b, ia, dci, x; int t, li; };
      each2(c.tid, P * c.nwa,
            [&](int e) {
              InX r;
              r.t = e / c.nwa;
              r.li = e - r.t * c.nwa;
              r.b = V.bb(r.t, r.li);
              r.ia = V.aa(r.t, r.li);
              r.dci = V.dc(0, r.li);
              r.x = V.xs(r.t, r.li);
              return r;
            },
            [&](const InX& r) {
              const double ab = fabs(r.b);
              const double xh = ab > mu[r.t] ? sgn(r.b) * (ab - mu[r.t]) * r.ia / r.dci : 0.0;
              V.xb(r.t, r.li) = 2.0 * xh - r.x;
              V.Txs.set(r.t, r.li, xh);
            });
      __syncthreads();
      struct InC { double kc, ys, drc, bc, ca, cb; int t, li; };
      each2(c.tid, Tp * c.nwa,
            [&](int e) {
              InC r;
              r.t = e / c.nwa;
              r.li = e - r.t * c.nwa;
              r.kc = kx_trade(V, V.xb, r.t, r.li);
              r.ys = V.ysC(r.t, r.li);
              r.drc = V.drC(r.t, r.li);
              r.bc = trade_offset(V, r.t, r.li);
              r.ca = V.ca(r.t, r.li);
              r.cb = V.cb(r.t, r.li);
              return r;
            },
            [&](const InC& r) {
              const double vs = r.ys + sigma * r.kc;
              const double z = vs / (sigma * r.drc) - r.bc;
              const double pr = prox_cost(z, 1.0 / (sigma * r.drc * r.drc), r.ca, r.cb, p.d);
              V.TysC.set(r.t, r.li, vs - sigma * r.drc * r.bc - sigma * r.drc * pr);
            });
    }
    for (int e = c.tid; e < P * nr; e += TB) {
      const int j = e % nr;
      const double vs = ys[e] + sigma * Kx[e];
      double ny;
      if (j < p.m) {
        const double sd = sigma * p.dr[j];
        ny = vs - sd * fmin(fmax(vs / sd, p.L[j]), p.U[j]);
        // an infinite bound side forces the dual's sign exactly (rounding of
        // vs - sd (vs / sd) must not leave the conjugate's domain)
        if (isinf(p.U[j]) && ny > 0.0) ny = 0.0;
        if (isinf(p.L[j]) && ny < 0.0) ny = 0.0;
      } else {
        const double drj = p.dr[j];
        ny = 2.0 * p.g1 * (vs - sigma * drj * p.bF[j - p.m]) / (sigma * drj * drj + 2.0 * p.g1);
      }
      Tys[e] = ny;
    }
    __syncthreads();
    t_phC += wall_clock64() - tcc0;

    // Checks (FP64): fixed-point residual, relative KKT at T(z), restart decisions.
    if (check) {
      const long long tc0 = wall_clock64();
      // C1 = [16 scalars][P budgets][P*nr K~ Txs][STW*P dual-inner stats]
      const int oB = 16, oR = 16 + P, oD = oR + P * nr, VC1 = oD + STW * P;
      double v[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double tx = V.Txs(t, li), dx = V.xs(t, li) - tx, dl = tx - V.x0s(t, li);
        v[0] = fma(omega * dx, dx, v[0]);
        v[1] = fma(dl, dl, v[1]);
        const double w = Vc.dc(0, li) * tx, wc = w - Vc.cvec(0, li);
        v[3] += -Vc.alpha(t, li) * w + 0.5 * Vc.arisk(0, li) * wc * wc;
        if (!isfinite(tx)) v[9] += 1.0;
        xv1[t * nw + li] = tx;
      }
      for (int e = c.tid; e < Tp * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double ty = V.TysC(t, li), dy = V.ysC(t, li) - ty, dl = ty - V.ys0C(t, li);
        v[0] = fma(dy / omega, dy, v[0]);
        v[2] = fma(dl, dl, v[2]);
        const double au = fabs(trade_of(Vc, V.Txs, t, li));
        const double ca = Vc.ca(t, li), cb = Vc.cb(t, li);
        v[4] += ca * au + cb * pow(au, p.d);
        const double yc = Vc.drC(t, li) * ty;   // unscaled trade dual
        v[5] += conj_cost(yc, ca, cb, p.d);
        if (t == 0) v[6] += yc * Vc.w0(0, li);
        if (p.multi && t == P) v[6] -= yc * Vc.wT(0, li);
        v[7] = fma(yc, yc, v[7]);
        if (cb <= 0.0 && fabs(yc) > ca) { const double ex = fabs(yc) - ca; v[10] = fma(ex, ex, v[10]); }
        if (!isfinite(ty)) v[9] += 1.0;
      }
      if (c.wg == 0) {   // replicated row duals enter the sums once
        for (int e = c.tid; e < P * nr; e += TB) {
          const int j = e % nr;
          const double dy = ys[e] - Tys[e], dl = Tys[e] - ys0[e];
          v[0] = fma(dy / omega, dy, v[0]);
          v[2] = fma(dl, dl, v[2]);
          const double yu = p.dr[j] * Tys[e];
          v[7] = fma(yu, yu, v[7]);
          if (j < p.m) {
            if (isinf(p.L[j]) && yu < 0.0) v[10] = fma(yu, yu, v[10]);
            if (isinf(p.U[j]) && yu > 0.0) v[10] = fma(yu, yu, v[10]);
          }
        }
        if (c.tid == 0) {
          const double el = (double)(wall_clock64() - t_start) / ctl.wall_hz;
          v[8] = el > ctl.time_limit_s ? 1.0 : 0.0;
        }
      }
      wg_sum<12>(c, v);
      if (c.tid < 12) put(c, c.tid, red[RED_OUT + c.tid]);
      {
        const int lane = c.tid & 63, wave = c.tid >> 6;
        for (int t = wave; t < P; t += NWAVE) {   // L1 norms of T(x), one wave per period
          double b = 0.0;
          for (int li = lane; li < c.nwa; li += 64) b += fabs(Vc.dc(0, li) * xv1[t * nw + li]);
          b = wave_sum(b);
          if (lane == 0) put(c, oB + t, b);
        }
      }
      rows_prod<1>(c, Vc, xv1, xv1, nw, P, nr, oR);
      // dual inner problem: b' = alpha + arisk c - R' (signed, in bb), 1/a' in aa,
      // R' = unscaled K^T Y at T(y).
      kty_all(c, Vc, Tys, P, nr, nw, xv2);
      for (int e = c.tid; e < P * c.nwa; e += TB) {   // xv2: signed b', xv3: |b'|, xv4: 1/a'
        const int t = e / c.nwa, li = e % c.nwa;
        const double Ry = (xv2[t * nw + li] + kty_trade(Vc, V.TysC, t, li)) / Vc.dc(0, li);
        const double b = Vc.alpha(t, li) + Vc.arisk(0, li) * Vc.cvec(0, li) - Ry;
        xv2[t * nw + li] = b;
        xv3[t * nw + li] = fabs(b);
        xv4[t * nw + li] = 1.0 / Vc.arisk(0, li);
      }
      __syncthreads();
      period_stats_x<LS>(c, xv3, xv4, nw, dcen, dhw, oD);
      c.mx_lo = oD;
      c.mx_hi = oD + STW * P;
      if (!xsync_x<LS>(c, VC1)) goto barrier_fail;
      double c1s[16];
      for (int q = 0; q < 16; ++q) c1s[q] = tot[q];
      // row terms, spread over the threads: primal residual, clip norm, factor risk, and
      // the row part of the dual objective
      double rv[4] = {0.0, 0.0, 0.0, 0.0};
      for (int e = c.tid; e < P * nr; e += TB) {
        const int j = e % nr;
        const double drj = p.dr[j];
        const double val = tot[oR + e] / drj;   // unscaled (A W)_j or (G^T W)_l
        const double yu = drj * Tys[e];
        if (j < p.m) {
          const double Lj = p.L[j], Uj = p.U[j];
          const double cl = fmin(fmax(val, Lj), Uj);
          rv[0] = fma(val - cl, val - cl, rv[0]);
          rv[1] = fma(cl, cl, rv[1]);
          if (yu > 0.0) rv[3] -= (isinf(Uj) ? INFINITY : Uj * yu);
          else if (yu < 0.0) rv[3] -= (isinf(Lj) ? INFINITY : Lj * yu);
        } else {
          const double bf = p.bF[j - p.m];
          const double g = val - bf;
          rv[2] = fma(p.g1 * g, g, rv[2]);
          rv[3] -= yu * bf + yu * yu / (4.0 * p.g1);
        }
      }
      wg_sum<4>(c, rv);
      double pres2 = red[RED_OUT], clip2 = red[RED_OUT + 1];
      const double phi = c1s[3] + c1s[4] + red[RED_OUT + 2];
      const double psi_rows = red[RED_OUT + 3];
      for (int t = 0; t < P; ++t) {
        const double ex = fmax(tot[oB + t] - 1.0, 0.0);
        pres2 += ex * ex;
      }
      __syncthreads();
      {
        const int lane = c.tid & 63, wave = c.tid >> 6;
        for (int t = wave; t < P; t += NWAVE) {   // one wave per period
          double l = 0.0, h = 0.0, m_ = 0.0;
          const int r = bracket_decide(tot + oD + STW * t, dcen[t], dhw[t], l, h, m_) & 15;
          if (lane == 0) {
            dwd[t] = adapt_width(r, dwd[t]);
            dmp[t] = dmu[t];
            if (r == 1 || r == 2 || r == 4) { dmu[t] = m_; need[t] = 0; }
            else {
              dlo[t] = l; dhi[t] = h; need[t] = 1;
              __hip_atomic_fetch_or(fbflag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
          }
        }
      }
      __syncthreads();
      if (c.tid == 0) { *iflag = *fbflag; *fbflag = 0; }
      __syncthreads();
      if (*iflag && !multisect_x<LS>(c, P, xv3, xv4, nw, need, dlo, dhi, dmu, &sc->ms_rounds)) goto barrier_fail;
      for (int t = c.tid; t < P; t += TB) next_bracket(dmu[t], dmp[t], dwd[t], dcen[t], dhw[t]);
      __syncthreads();
      // C2: inner value sum (a'/2 w^2 - b' w), w = sign(b') max(|b'| - mu', 0) / a'.
      // With exposure rows it also carries, per period, max_i |(A^T d)_i| for the
      // infeasibility test below (d = T(y_A) - y_A, unscaled; staged in Kx, which is not
      // read again before the next iteration recomputes it).
      const bool inf_test = ctl.infeas && p.m > 0;
      {
        double iv[1] = {0.0};
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double b = xv2[t * nw + li], ab = fabs(b), ia = xv4[t * nw + li];
          const double w = ab > dmu[t] ? sgn(b) * (ab - dmu[t]) * ia : 0.0;
          iv[0] += 0.5 * w * w / ia - b * w;
        }
        wg_sum<1>(c, iv);
        const double ivs = red[RED_OUT];
        __syncthreads();
        int V2 = 1;
        if (inf_test) {
          for (int e = c.tid; e < P * nr; e += TB) {
            const int j = e % nr;
            Kx[e] = j < p.m ? Tys[e] - ys[e] : 0.0;
          }
          __syncthreads();
          kty_all(c, Vc, Kx, P, nr, nw, xv1);   // xv1[t][li] = dc_i (A^T d_u)_i
          const int lane = c.tid & 63, wave = c.tid >> 6;
          for (int t = wave; t < P; t += NWAVE) {
            double mx = 0.0;
            for (int li = lane; li < c.nwa; li += 64) mx = fmax(mx, fabs(xv1[t * nw + li] / Vc.dc(0, li)));
            mx = wave_max(mx);
            if (lane == 0) put_max(c, 1 + STW * t, mx);
          }
          V2 = 2 + STW * (P - 1);
          if (c.xmode == XM_GATHER)   // gather mode: every index of the exchange is written
            for (int j = c.tid; j < V2; j += TB)
              if (j > 0 && j % STW != 1) put(c, j, 0.0);
          c.mx_lo = 0;
          c.mx_hi = V2;
        }
        if (c.tid == 0) put(c, 0, ivs);
        if (!xsync_x<LS>(c, V2)) goto barrier_fail;
      }
      // Infeasibility (a Farkas certificate for one period's feasible set, which is the
      // same in every period): for any y in R^m and feasible w, y^T A w lies between
      // -||A^T y||_inf (the budget ||w||_1 <= 1) and sum_j max(U_j y_j, L_j y_j) (the box),
      // so sum_j max(U_j y_j, L_j y_j) + ||A^T y||_inf < 0 proves that no w is feasible.
      // When the box and the budget do not intersect the exposure duals diverge and
      // their displacement T(y_A) - y_A tends to such a y.
      bool infeasible = false;
      if (inf_test) {
        lint* infl = iflag + 3;
        if (c.tid == 0) *infl = 0;
        __syncthreads();
        const int lane = c.tid & 63, wave = c.tid >> 6;
        for (int t = wave; t < P; t += NWAVE) {
          double sup = 0.0, mag = 0.0;
          for (int j = lane; j < p.m; j += 64) {
            const double du = p.dr[j] * Kx[t * nr + j];
            double term = 0.0;
            if (du > 0.0) term = isinf(p.U[j]) ? INFINITY : p.U[j] * du;
            else if (du < 0.0) term = isinf(p.L[j]) ? INFINITY : p.L[j] * du;
            sup += term;
            mag += fabs(term);
          }
          sup = wave_sum(sup);
          mag = wave_sum(mag);
          const double amax = tot[1 + STW * t];
          if (lane == 0 && amax + mag > 0.0 && sup + amax < -1e-9 * (mag + amax))
            __hip_atomic_fetch_or(infl, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
        infeasible = *infl != 0;
        __syncthreads();
      }
      const double psi = tot[0] + (double)P * p.crisk[0] - c1s[6] - c1s[5] + psi_rows;
      const double rel_pri = sqrt(pres2) / (1.0 + sqrt(clip2));
      const double rel_dual = sqrt(c1s[10]) / (1.0 + sqrt(c1s[7]));
      const double den = fabs(phi) + fabs(psi);
      const double rel_gap = den > 0.0 ? fabs(phi - psi) / den : 0.0;
      const double relkkt = fmax(rel_pri, fmax(rel_dual, rel_gap));
      const double fpr = sqrt(c1s[0]);
      // (fmax drops a NaN operand, so the gap and both objectives are tested themselves)
      const bool nonfinite = c1s[9] > 0.0 || !isfinite(phi) || !isfinite(psi) || !isfinite(rel_gap) ||
                             !isfinite(relkkt);
      if (c.tid == 0) {
        sc->checks++;
        sc->restart = 0;
        if (c.wg == 0) {
          s.info[IX_RELKKT] = relkkt; s.info[IX_RELPRI] = rel_pri; s.info[IX_RELDUAL] = rel_dual;
          s.info[IX_RELGAP] = rel_gap; s.info[IX_FPR] = fpr; s.info[IX_POBJ] = phi; s.info[IX_DOBJ] = psi;
          if (ctl.verbose >= 2)
            printf("[ffo] it %lld kkt %.3e pri %.3e gap %.3e fpr %.3e omega %.3e restarts %lld miss %lld\n",
                   sc->it + 1, relkkt, rel_pri, rel_gap, fpr, omega, sc->restarts, sc->spec_miss);
        }
        if (nonfinite) { sc->done = 1; sc->status = DS_NUMERIC; }
        else if (infeasible) { sc->done = 1; sc->status = DS_INFEASIBLE; }
        else if (relkkt <= ctl.tol) { sc->done = 1; sc->status = DS_OK; }
        else if (c1s[8] > 0.0) { sc->done = 1; sc->status = DS_TIMEOUT; }
        else if (sc->it + 1 >= ctl.max_iter) { sc->done = 1; sc->status = DS_NOT_CONVERGED; }
        else {
          if (sc->r0 < 0.0) sc->r0 = fpr;
          const bool rs = (fpr <= ctl.r_suff * sc->r0) ||
                          (fpr <= ctl.r_nec * sc->r0 && fpr > sc->rprev) ||
                          ((double)(sc->kk + 1) >= ctl.r_art * (double)(sc->it + 1));
          sc->rprev = fpr;
          if (rs) {
            const double dxn = sqrt(c1s[1]), dyn = sqrt(c1s[2]);
            if (dxn > 1e-300 && dyn > 1e-300)
              sc->omega = exp(0.5 * log(dyn / dxn) + 0.5 * log(sc->omega));
            sc->r0 = fpr;
            sc->rprev = INFINITY;
            sc->restarts++;
            sc->restart = 1;
            // a restart jumps the iterate: drop the multiplier trend
            for (int t = 0; t < P; ++t) { mpv[t] = mu[t]; next_bracket(mu[t], mu[t], wid[t], cen[t], hw[t]); }
          }
        }
      }
      __syncthreads();
      t_check += wall_clock64() - tc0;
      if (sc->done) {
        const bool bad = sc->status == DS_NUMERIC;
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          s.w_out[(size_t)t * n + c.i0 + li] = Vc.dc(0, li) * (bad ? V.x0s(t, li) : V.Txs(t, li));
        }
        if (s.y_out) {
          double* yA = s.y_out;
          double* yF = s.y_out + (size_t)P * p.m;
          double* yC = s.y_out + (size_t)P * nr;
          // infeasible: the exposure part holds the certificate direction d of the test
          const bool cert = sc->status == DS_INFEASIBLE;
          if (c.wg == 0)
            for (int e = c.tid; e < P * nr; e += TB) {
              const int t = e / nr, j = e % nr;
              const double yu = p.dr[j] * (bad ? ys0[e] : (cert && j < p.m ? Kx[e] : Tys[e]));
              if (j < p.m) yA[(size_t)t * p.m + j] = yu; else yF[(size_t)t * p.k + (j - p.m)] = yu;
            }
          for (int e = c.tid; e < Tp * c.nwa; e += TB) {
            const int t = e / c.nwa, li = e % c.nwa;
            yC[(size_t)t * n + c.i0 + li] = Vc.drC(t, li) * (bad ? V.ys0C(t, li) : V.TysC(t, li));
          }
        }
        if (c.tid == 0) sc->it++;
        break;
      }
      if (sc->restart) {
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double x = V.Txs(t, li);
          V.x0s(t, li) = x; V.xs.set(t, li, x); V.Txs.set(t, li, x);
        }
        for (int e = c.tid; e < Tp * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double y = V.TysC(t, li);
          V.ys0C(t, li) = y; V.ysC.set(t, li, y); V.TysC.set(t, li, y);
        }
        for (int e = c.tid; e < P * nr; e += TB) { const double y = Tys[e]; ys[e] = y; ys0[e] = y; }
        __syncthreads();
        if (c.tid == 0) { sc->kk = 0; sc->it++; }
        __syncthreads();
        continue;
      }
    }

    // Phase D: reflected Halpern step
    const long long td0 = wall_clock64();
    {
      const double kk = (double)sc->kk;
      const double a1 = (kk + 1.0) / (kk + 2.0), a0 = 1.0 / (kk + 2.0), rho = ctl.rho;
      if constexpr (SL || LS) {
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          V.xs.set(t, li, a1 * ((1.0 + rho) * V.Txs(t, li) - rho * V.xs(t, li)) + a0 * V.x0s(t, li));
        }
        for (int e = c.tid; e < Tp * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          V.ysC.set(t, li, a1 * ((1.0 + rho) * V.TysC(t, li) - rho * V.ysC(t, li)) + a0 * V.ys0C(t, li));
        }
      } else {   // the same arithmetic, two elements per step
        struct InH { double tz, z, z0; int t, li; };
        each2(c.tid, P * c.nwa,
              [&](int e) {
                InH r;
                r.t = e / c.nwa;
                r.li = e - r.t * c.nwa;
                r.tz = V.Txs(r.t, r.li);
                r.z = V.xs(r.t, r.li);
                r.z0 = V.x0s(r.t, r.li);
                return r;
              },
              [&](const InH& r) { V.xs.set(r.t, r.li, a1 * ((1.0 + rho) * r.tz - rho * r.z) + a0 * r.z0); });
        each2(c.tid, Tp * c.nwa,
              [&](int e) {
                InH r;
                r.t = e / c.nwa;
                r.li = e - r.t * c.nwa;
                r.tz = V.TysC(r.t, r.li);
                r.z = V.ysC(r.t, r.li);
                r.z0 = V.ys0C(r.t, r.li);
                return r;
              },
              [&](const InH& r) { V.ysC.set(r.t, r.li, a1 * ((1.0 + rho) * r.tz - rho * r.z) + a0 * r.z0); });
      }
      for (int e = c.tid; e < P * nr; e += TB) ys[e] = a1 * ((1.0 + rho) * Tys[e] - rho * ys[e]) + a0 * ys0[e];
      __syncthreads();
      if (c.tid == 0) { sc->kk++; sc->it++; }
      __syncthreads();
    }
    t_phD += wall_clock64() - td0;
  }

  if (c.wg == 0 && c.tid == 0) {
    const long long t_end = wall_clock64();
    s.info[IX_ITERS] = (double)sc->it;
    s.info[IX_RESTARTS] = (double)sc->restarts;
    s.info[IX_OMEGA] = sc->omega;
    s.info[IX_ETA] = sc->eta;
    s.info[IX_NORMK] = ctl.eta_safety / sc->eta;
    s.info[IX_SPEC_MISS] = (double)sc->spec_miss;
    s.info[IX_EXCHANGES] = (double)c.epoch;
    s.info[IX_CHECKS] = (double)sc->checks;
    s.info[IX_T_WAIT] = (double)c.t_wait / ctl.wall_hz;
    s.info[IX_T_ITER] = (double)(t_end - t_loop) / ctl.wall_hz;
    s.info[IX_T_CHECK] = (double)t_check / ctl.wall_hz;
    s.info[IX_T_POWER] = (double)(t_loop - t_start) / ctl.wall_hz;
    s.info[IX_MS_ROUNDS] = (double)sc->ms_rounds;
    s.info[IX_T_PHA] = (double)t_phA / ctl.wall_hz;
    s.info[IX_T_PHB] = (double)t_phB / ctl.wall_hz;
    s.info[IX_T_PHC] = (double)t_phC / ctl.wall_hz;
    s.info[IX_T_PHD] = (double)t_phD / ctl.wall_hz;
    s.info[IX_T_PRE] = (double)c.t_pre / ctl.wall_hz;
    s.info[IX_T_READ] = (double)c.t_read / ctl.wall_hz;
    s.info[IX_T_B1] = (double)t_b1 / ctl.wall_hz;
    s.info[IX_T_B2] = (double)t_b2 / ctl.wall_hz;
    s.info[IX_T_B3] = (double)t_b3 / ctl.wall_hz;
    s.info[IX_T_B1S] = (double)t_b1s / ctl.wall_hz;
    s.info[IX_MISS_IN] = (double)sc->miss_in;
    s.info[IX_MISS_OUT] = (double)sc->miss_out;
    s.info[IX_T_GATHER] = (double)t_gather / ctl.wall_hz;
    s.info[IX_GATHERS] = (double)n_gather;
    s.status[0] = sc->status;
  }
  return;

barrier_fail:
  if (c.tid == 0) __hip_atomic_store(s.status, (int32_t)DS_BARRIER, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return;
}

template <bool KL, bool SL, class R>
__global__ __launch_bounds__(TB) void k_solve(DevProblem p, DevState s, DevControl ctl) {
  solve_body<KL, SL, R, true>(p, s, ctl, blockIdx.x, gridDim.x);
}

// Batched: every team solves its own instance; teams never wait for each other.
template <bool KL, bool SL, class R, class KGT = typename default_kg<R>::type>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(2))) void k_solve_batch(const DevProblem* __restrict__ dp, const DevState* __restrict__ ds,
                                                    const DevControl* __restrict__ dcl, const int* __restrict__ wg_team,
                                                    const int* __restrict__ wg_rank) {
  const int team = wg_team[blockIdx.x];
  const DevControl ctl = dcl[team];
  solve_body<KL, SL, R, false, KGT>(dp[team], ds[team], ctl, wg_rank[blockIdx.x], ctl.nwg);
}

// ---------------------------------------------------------------------------------
// Adjoint: fixed-point implicit differentiation of the solve operator
// ---------------------------------------------------------------------------------
// At a solution z* = T(z*) of the iteration above, a loss l of W* = dc x* has
// dl/dtheta = lambda^T dT/dtheta with lambda = J^T lambda + g, J = dT/dz at z*, g = (dc dl/dW, 0).
// J is the linearisation of one step with every nonsmooth piece frozen as T(z*) finds it:
// the budget support S_t and whether mu_t > 0 (primal prox: per period
// dw/db = diag(1{S}/a) - s s^T / c_S with s = 1{S} sign(b)/a, c_S = sum_S 1/a, when mu_t > 0),
// the clipped exposure rows (dual prox derivative 1, else 0), the factor rows
// (2 g1 / (sigma dr^2 + 2 g1)) and the trade rows (1 - prox'(z), prox' = 0 in the dead
// zone of the spread term, 1 / (1 + t' b d (d-1) rho^(d-2)) outside it).  Transposing one
// step in reverse order gives, with mu_y = N lambda_y, q = lambda_x + 2 sigma K~^T mu_y,
// nu = dw/db (q / dc):
//   J^T lambda = ( nu / (tau dc) - sigma K~^T mu_y ,  mu_y - K~ (nu / dc) ),
// and nu is the gradient with respect to alpha.  One exchange per iteration carries the
// row sums of K~ (1{S}/a q / dc^2) and s^T (q / dc) per period (K~ s / dc is fixed).  The
// iteration is the same restarted reflected Halpern scheme as the solve.  At the end:
//   dl/ds   = lambda_yC g2 sign(z) prox'(z) / drC,
//   dl/dG_il = dr_j (sum_t sigma mu_y,tj w*_ti - y*_tj nu_ti) - [multi-period] sigma dr_j c_i sum_t mu_y,tj
// for the factor row j = m + l (dK~_ji / dG_il = dr_j dc_i; the scaling is held fixed, which
// leaves the solution map unchanged), and dl/dF = dl/dG C^T follows in launch_grad_F.
struct AScal {
  double omega, eta, tau, sigma, r0, rprev, gnorm;
  long long it, kk, restarts, checks;
  int done, status, restart;
};

template <bool KL>
__global__ __launch_bounds__(TB) void k_adjoint(DevProblem p, AdjState a, DevControl ctl, double omega_in) {
  ldbl* lds = (ldbl*)g_lds;
  const int P = p.P, nr = p.nr, n = p.n, Tp = p.Tp, nw = ctl.nw, m = p.m;
  Ctx c;
  c.wg = blockIdx.x;
  c.nwg = gridDim.x;
  c.tid = threadIdx.x;
  c.i0 = c.wg * nw;
  c.nwa = max(0, min(nw, n - c.i0));
  c.epoch = 0;
  c.xbuf = a.xbuf;
  c.bar = a.bar;
  c.vmax = ctl.vmax;
  c.xmode = ctl.xmode;
  c.ng = ctl.xmode == XM_ATOMIC ? max(1, min(ctl.xgroups, min(XG_MAX, (int)gridDim.x))) : 1;
  c.grp = c.wg % c.ng;
  c.gsize = (c.nwg - c.grp + c.ng - 1) / c.ng;
  c.P = P;
  c.spin_limit = ctl.spin_limit;
  c.mx_lo = c.mx_hi = 0;
  c.t_wait = c.t_pre = c.t_read = 0;

  // LDS layout (doubles); must match adjoint_lds_bytes
  ldbl* ptr = lds;
  ldbl* Kl = nullptr;
  const int ldl = nw | 1;
  if (KL) { Kl = ptr; ptr += (size_t)nr * ldl; }
  ldbl* ks = ptr;   ptr += nr;
  ldbl* ys = ptr;   ptr += P * nr;     // y* (scaled rows)
  ldbl* nR = ptr;   ptr += P * nr;     // row prox derivatives
  ldbl* Kr = ptr;   ptr += P * nr;     // K~ (s / dc), fixed
  ldbl* ly = ptr;   ptr += P * nr;     // adjoint row part, anchor, image
  ldbl* ly0 = ptr;  ptr += P * nr;
  ldbl* Tly = ptr;  ptr += P * nr;
  ldbl* muy = ptr;  ptr += P * nr;     // N lambda_y (rows)
  ldbl* KDu = ptr;  ptr += P * nr;     // exchanged row sums
  ldbl* xv1 = ptr;  ptr += P * nw;
  ldbl* xv2 = ptr;  ptr += P * nw;
  ldbl* xv3 = ptr;  ptr += P * nw;
  ldbl* xv4 = ptr;  ptr += P * nw;
  ldbl* mC = ptr;   ptr += Tp * nw;    // N lambda_yC of the owned assets
  ldbl* tot = ptr;  ptr += ctl.vmax;
  ldbl* red = ptr;  ptr += RED_LEN;
  ldbl* cen = ptr;  ptr += P;
  ldbl* hw = ptr;   ptr += P;
  ldbl* lo = ptr;   ptr += P;
  ldbl* hi = ptr;   ptr += P;
  ldbl* mu = ptr;   ptr += P;
  ldbl* cS = ptr;   ptr += P;
  ldbl* stu = ptr;  ptr += P;
  __attribute__((address_space(3))) AScal* sc = (__attribute__((address_space(3))) AScal*)ptr;
  ptr += (sizeof(AScal) + 7) / 8;
  lint* iflag = (lint*)ptr; ptr += 2;
  lint* fbflag = iflag + 1;
  lint* need = (lint*)ptr;
  c.tot = tot;
  c.red = red;
  c.flag = iflag;
  c.lslot = nullptr;

  S<KL, false, double> V;
  {
    auto g = [&](const double* b) { return Arr<false, double>{(double*)b, n, c.i0}; };
    V.p = &p; V.Kl = Kl; V.Kg = p.K; V.ks = ks; V.nw = nw; V.ldl = ldl; V.i0 = c.i0;
    V.alpha = g(p.alpha); V.ca = g(p.ca); V.cb = g(p.cb); V.drC = g(p.drC);
    V.dc = g(p.dc); V.arisk = g(p.arisk); V.cvec = g(p.cvec); V.w0 = g(p.w0);
    V.wT = g(p.wT ? p.wT : p.w0);
  }
  auto G = [&](double* b) { return Arr<false, double>{b, n, c.i0}; };
  const auto xs = G(a.xs), xbar = G(a.xbar), bb = G(a.bb), sx = G(a.sx);
  const auto lx = G(a.lx), lx0 = G(a.lx0), Tlx = G(a.Tlx);
  const auto ysC = G(a.ysC), lyC = G(a.lyC), lyC0 = G(a.lyC0), TlyC = G(a.TlyC), nC = G(a.nC), gsf = G(a.gsf);
  const auto tsg = G(a.tsg), trho = G(a.trho);
  const Arr<true, double> mCv{mC, nw, 0}, nbv{xv4, nw, 0};

  for (int j = c.tid; j < nr; j += TB) ks[j] = p.kscaled ? 1.0 : p.dr[j];
  __syncthreads();
  if (KL)
    for (int e = c.tid; e < nr * nw; e += TB) {
      const int j = e / nw, li = e % nw;
      Kl[j * ldl + li] = li < c.nwa ? p.K[(size_t)j * p.ldk + c.i0 + li] * ks[j] : 0.0;
    }
  // the solution in scaled variables
  for (int e = c.tid; e < P * c.nwa; e += TB) {
    const int t = e / c.nwa, li = e % c.nwa;
    xs(t, li) = a.w_star[(size_t)t * n + c.i0 + li] / V.dc(0, li);
    xbar(t, li) = 1.0 + 0.25 * (double)(((c.i0 + li) * 7919 + t * 104729) % 1000) / 1000.0;   // power vector
  }
  {
    const double* yC = a.y_star + (size_t)P * nr;
    for (int e = c.tid; e < Tp * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      ysC(t, li) = yC[(size_t)t * n + c.i0 + li] / V.drC(t, li);
    }
  }
  for (int e = c.tid; e < P * nr; e += TB) {
    const int t = e / nr, j = e % nr;
    const double yu = j < m ? a.y_star[(size_t)t * m + j] : a.y_star[(size_t)P * m + (size_t)t * p.k + (j - m)];
    ys[e] = yu / p.dr[j];
    ly[e] = 0.0; ly0[e] = 0.0; Tly[e] = 0.0;
  }
  if (c.tid == 0) {
    sc->omega = omega_in; sc->it = 0; sc->kk = 0; sc->restarts = 0; sc->checks = 0;
    sc->r0 = -1.0; sc->rprev = INFINITY; sc->done = 0; sc->status = DS_RUNNING; sc->restart = 0;
    fbflag[0] = 0;
    for (int t = 0; t < P; ++t) { cen[t] = 0.0; hw[t] = 0.0; mu[t] = 0.0; need[t] = 0; }
  }
  __syncthreads();
  const long long t_start = wall_clock64();

  // ---- power iteration for ||K~|| (same recipe as the solve)
  double lam = 0.0;
  for (int pw = 0; pw < ctl.npow; ++pw) {
    double loc[2] = {0.0, 0.0};
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double x = xbar(t, li);
      xv1[t * nw + li] = x;
      loc[0] = fma(x, x, loc[0]);
    }
    for (int e = c.tid; e < Tp * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double u = kx_trade(V, xbar, t, li);
      loc[1] = fma(u, u, loc[1]);
    }
    wg_sum<2>(c, loc);
    if (c.tid == 0) { put(c, 0, red[RED_OUT]); put(c, 1, red[RED_OUT + 1]); }
    __syncthreads();
    rows_prod<1>(c, V, xv1, xv1, nw, P, nr, 2);
    if (!xsync(c, 2 + P * nr)) goto adj_fail;
    {
      const double vv = tot[0];
      double kv = tot[1];
      for (int e = 0; e < P * nr; ++e) kv = fma(tot[2 + e], tot[2 + e], kv);
      lam = vv > 0.0 ? kv / vv : 0.0;
      const double scale = (lam > 0.0 && vv > 0.0) ? 1.0 / (lam * sqrt(vv)) : 1.0;
      kty_all(c, V, tot + 2, P, nr, nw, xv2);
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        double uc = kx_trade(V, xbar, t, li) * V.drC(t, li) * V.dc(0, li);
        if (p.multi) uc -= kx_trade(V, xbar, t + 1, li) * V.drC(t + 1, li) * V.dc(0, li);
        xv2[t * nw + li] = (xv2[t * nw + li] + uc) * scale;
      }
      __syncthreads();
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        xbar(t, li) = xv2[t * nw + li];
      }
      __syncthreads();
    }
  }
  if (c.tid == 0) {
    sc->eta = ctl.eta_safety / sqrt(fmax(lam, 1e-300));
    sc->tau = sc->eta / sc->omega;
    sc->sigma = sc->eta * sc->omega;
  }
  __syncthreads();

  {
    double tau = sc->tau, sigma = sc->sigma;
    // ---- one step T(z*): the pieces the linearisation freezes
    kty_all(c, V, ys, P, nr, nw, xv1);
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double Ry = xv1[t * nw + li] + kty_trade(V, ysC, t, li);
      const double v = xs(t, li) - tau * Ry;
      const double dci = V.dc(0, li);
      const double ia = 1.0 / (1.0 / (tau * dci * dci) + V.arisk(0, li));
      const double b = v / (tau * dci) + V.alpha(t, li) + V.arisk(0, li) * V.cvec(0, li);
      bb(t, li) = b;
      xv3[t * nw + li] = fabs(b);
      xv4[t * nw + li] = ia;
    }
    __syncthreads();
    period_stats(c, xv3, xv4, nw, cen, hw, 0);
    c.mx_lo = 0;
    c.mx_hi = STW * P;
    if (!xsync(c, STW * P)) goto adj_fail;
    {
      const int lane = c.tid & 63, wave = c.tid >> 6;
      for (int t = wave; t < P; t += NWAVE) {
        double l = 0.0, h = 0.0, m_ = 0.0;
        const int r = bracket_decide(tot + STW * t, 0.0, 0.0, l, h, m_) & 15;
        if (lane == 0) {
          if (r == 0 || r == 3) { lo[t] = l; hi[t] = h; need[t] = 1; fbflag[0] = 1; }
          else { mu[t] = m_; need[t] = 0; }
        }
      }
    }
    __syncthreads();
    if (*fbflag && !multisect(c, P, xv3, xv4, nw, need, lo, hi, mu, iflag + 3)) goto adj_fail;
    // support, x^+, xbar; rows of K~ xbar, sum_S 1/a, K~ (s / dc) in one exchange
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      const double b = bb(t, li), ab = fabs(b), ia = xv4[t * nw + li], dci = V.dc(0, li);
      const bool in = ab > mu[t];
      const double xp = in ? sgn(b) * (ab - mu[t]) * ia / dci : 0.0;
      const double xb = 2.0 * xp - xs(t, li);
      xbar(t, li) = xb;
      bb(t, li) = in ? sgn(b) : 0.0;     // frozen support and signs
      xv1[t * nw + li] = xb;
    }
    __syncthreads();
    rows_prod<1>(c, V, xv1, xv1, nw, P, nr, 0);
    if (!xsync(c, P * nr)) goto adj_fail;
    for (int e = c.tid; e < P * nr; e += TB) {   // frozen clipped exposure rows
      const int j = e % nr;
      const double vs = ys[e] + sigma * tot[e];
      if (j < m) {
        const double sd = sigma * p.dr[j], z = vs / sd;
        nR[e] = (z > p.L[j] && z < p.U[j]) ? 0.0 : 1.0;
      }
    }
    for (int e = c.tid; e < Tp * c.nwa; e += TB) {   // frozen dead zones and trade sizes
      const int t = e / c.nwa, li = e % c.nwa;
      const double kc = kx_trade(V, xbar, t, li);
      const double vs = ysC(t, li) + sigma * kc;
      const double drc = V.drC(t, li);
      const double z = vs / (sigma * drc) - trade_offset(V, t, li);
      const double tp = 1.0 / (sigma * drc * drc);
      const double ca = V.ca(t, li), cb = V.cb(t, li);
      const bool live = fabs(z) - tp * ca > 0.0;
      tsg(t, li) = live ? sgn(z) : 0.0;
      trho(t, li) = live ? fabs(prox_cost(z, tp, ca, cb, p.d)) : 0.0;
      lyC(t, li) = 0.0; lyC0(t, li) = 0.0; TlyC(t, li) = 0.0;
    }
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      lx(t, li) = 0.0; lx0(t, li) = 0.0; Tlx(t, li) = 0.0;
    }
    __syncthreads();

    // Step-size dependent factors of J for the current (tau, sigma), the pieces held
    // fixed: sx = 1{S} sign(b) / a, c_S = sum_S 1/a, K~ (sx / dc), the factor-row and
    // trade-row prox derivatives.  One exchange.
    auto refactor = [&]() -> bool {
      tau = sc->tau;
      sigma = sc->sigma;
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double dci = V.dc(0, li);
        const double ia = 1.0 / (1.0 / (tau * dci * dci) + V.arisk(0, li));
        const double sv = bb(t, li) * ia;
        sx(t, li) = sv;
        xv2[t * nw + li] = sv / dci;
        xv3[t * nw + li] = fabs(sv);
      }
      __syncthreads();
      {
        const int lane = c.tid & 63, wave = c.tid >> 6;
        for (int t = wave; t < P; t += NWAVE) {
          double v = 0.0;
          for (int li = lane; li < c.nwa; li += 64) v += xv3[t * nw + li];
          v = wave_sum(v);
          if (lane == 0) put(c, P * nr + t, v);
        }
      }
      rows_prod<1>(c, V, xv2, xv2, nw, P, nr, 0);
      if (!xsync(c, P * nr + P)) return false;
      for (int e = c.tid; e < P * nr; e += TB) {
        const int j = e % nr;
        Kr[e] = tot[e];
        if (j >= m) {
          const double drj = p.dr[j];
          nR[e] = 2.0 * p.g1 / (sigma * drj * drj + 2.0 * p.g1);
        }
      }
      for (int t = c.tid; t < P; t += TB) cS[t] = tot[P * nr + t];
      for (int e = c.tid; e < Tp * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double drc = V.drC(t, li), tp = 1.0 / (sigma * drc * drc), cb = V.cb(t, li);
        const double rho = trho(t, li), sg = tsg(t, li);
        double dp = 0.0;
        if (sg != 0.0) {
          if (p.d == 2.0) dp = 1.0 / (1.0 + 2.0 * tp * cb);
          else if (rho > 0.0) dp = 1.0 / (1.0 + tp * cb * p.d * (p.d - 1.0) * pow(rho, p.d - 2.0));
        }
        nC(t, li) = 1.0 - dp;
        gsf(t, li) = p.g2 * sg * dp / drc;
      }
      __syncthreads();
      return true;
    };
    if (!refactor()) goto adj_fail;

    // ---- adjoint iteration
    // one application of lambda -> J^T lambda + g; leaves nu in xv3 (per owned (t, i)), mu_y
    // in muy / mC, K~^T mu_y in xv1.  Returns false when a bounded wait expired.
    auto apply = [&]() -> bool {
      for (int e = c.tid; e < P * nr; e += TB) muy[e] = nR[e] * ly[e];
      for (int e = c.tid; e < Tp * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        mC[t * nw + li] = nC(t, li) * lyC(t, li);
      }
      __syncthreads();
      kty_all(c, V, muy, P, nr, nw, xv1);
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double Kt = xv1[t * nw + li] + kty_trade(V, mCv, t, li);
        xv1[t * nw + li] = Kt;
        const double dci = V.dc(0, li);
        const double u = (lx(t, li) + 2.0 * sigma * Kt) / dci;
        const double ia = fabs(sx(t, li));
        xv2[t * nw + li] = ia * u / dci;     // (1{S}/a) u / dc
        xv3[t * nw + li] = u;
      }
      __syncthreads();
      {
        const int lane = c.tid & 63, wave = c.tid >> 6;
        for (int t = wave; t < P; t += NWAVE) {
          double v = 0.0;
          for (int li = lane; li < c.nwa; li += 64) v = fma(sx(t, li), xv3[t * nw + li], v);
          v = wave_sum(v);
          if (lane == 0) put(c, P * nr + t, v);
        }
      }
      rows_prod<1>(c, V, xv2, xv2, nw, P, nr, 0);
      if (!xsync(c, P * nr + P)) return false;
      for (int t = c.tid; t < P; t += TB) stu[t] = (mu[t] > 0.0 && cS[t] > 0.0) ? tot[P * nr + t] / cS[t] : 0.0;
      __syncthreads();
      for (int e = c.tid; e < P * nr; e += TB) {
        const int t = e / nr;
        Tly[e] = muy[e] - (tot[e] - stu[t] * Kr[e]);
      }
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double ia = fabs(sx(t, li));
        const double nu = ia * xv3[t * nw + li] - sx(t, li) * stu[t];
        const double dci = V.dc(0, li);
        xv3[t * nw + li] = nu;
        xv4[t * nw + li] = nu / dci;
        Tlx(t, li) = nu / (tau * dci) - sigma * xv1[t * nw + li] + dci * a.grad_w[(size_t)t * n + c.i0 + li];
      }
      __syncthreads();
      for (int e = c.tid; e < Tp * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        TlyC(t, li) = mC[t * nw + li] - kx_trade(V, nbv, t, li);
      }
      __syncthreads();
      return true;
    };

    // |g| for the relative residual
    {
      double gv[1] = {0.0};
      for (int e = c.tid; e < P * c.nwa; e += TB) {
        const int t = e / c.nwa, li = e % c.nwa;
        const double gx = V.dc(0, li) * a.grad_w[(size_t)t * n + c.i0 + li];
        gv[0] = fma(gx, gx, gv[0]);
      }
      wg_sum<1>(c, gv);
      if (c.tid == 0) put(c, 0, red[RED_OUT]);
      if (!xsync(c, 1)) goto adj_fail;
      if (c.tid == 0) sc->gnorm = sqrt(tot[0]);
      __syncthreads();
    }
    while (true) {
      if (!apply()) goto adj_fail;
      const bool check = ((sc->it + 1) % ctl.check_every == 0) || (sc->it + 1 >= ctl.max_iter);
      if (check) {
        // [residual^2, non-finite count, |T lambda_x - anchor|^2, |T lambda_y - anchor|^2]
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double d = Tlx(t, li) - lx(t, li), dl = Tlx(t, li) - lx0(t, li);
          v[0] = fma(d, d, v[0]);
          v[2] = fma(dl, dl, v[2]);
          if (!isfinite(d)) v[1] += 1.0;
        }
        for (int e = c.tid; e < Tp * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          const double d = TlyC(t, li) - lyC(t, li), dl = TlyC(t, li) - lyC0(t, li);
          v[0] = fma(d, d, v[0]);
          v[3] = fma(dl, dl, v[3]);
          if (!isfinite(d)) v[1] += 1.0;
        }
        if (c.wg == 0)
          for (int e = c.tid; e < P * nr; e += TB) {
            const double d = Tly[e] - ly[e], dl = Tly[e] - ly0[e];
            v[0] = fma(d, d, v[0]);
            v[3] = fma(dl, dl, v[3]);
          }
        wg_sum<4>(c, v);
        if (c.tid < 4) put(c, c.tid, red[RED_OUT + c.tid]);
        if (c.wg == 0 && c.tid == 0) {
          const double el = (double)(wall_clock64() - t_start) / ctl.wall_hz;
          put(c, 4, el > ctl.time_limit_s ? 1.0 : 0.0);
        }
        if (!xsync(c, 5)) goto adj_fail;
        const double res = sqrt(tot[0]) / fmax(sc->gnorm, 1e-300);
        if (c.tid == 0) {
          sc->checks++;
          sc->restart = 0;
          if (c.wg == 0) {
            a.info[IX_RELKKT] = res;
            a.info[IX_FPR] = res;
            if (ctl.verbose >= 2)
              printf("[ffo adjoint] it %lld res %.3e omega %.3e |dlx| %.3e |dly| %.3e restarts %lld\n", sc->it + 1, res,
                     sc->omega, sqrt(tot[2]), sqrt(tot[3]), sc->restarts);
          }
          if (tot[1] > 0.0 || !isfinite(res)) { sc->done = 1; sc->status = DS_NUMERIC; }
          else if (res <= ctl.tol) { sc->done = 1; sc->status = DS_OK; }
          else if (tot[4] > 0.0) { sc->done = 1; sc->status = DS_TIMEOUT; }
          else if (sc->it + 1 >= ctl.max_iter) { sc->done = 1; sc->status = DS_NOT_CONVERGED; }
          else {
            if (sc->r0 < 0.0) sc->r0 = res;
            const bool rs = (res <= ctl.r_suff * sc->r0) || (res <= ctl.r_nec * sc->r0 && res > sc->rprev) ||
                            ((double)(sc->kk + 1) >= ctl.r_art * (double)(sc->it + 1));
            sc->rprev = res;
            // the weight stays fixed: unlike the solve's, this fixed point moves with
            // (tau, sigma), so a new weight would discard the progress made
            if (rs) { sc->r0 = res; sc->rprev = INFINITY; sc->restarts++; sc->restart = 1; }
          }
        }
        __syncthreads();
        if (sc->done) break;
        if (sc->restart) {
          for (int e = c.tid; e < P * c.nwa; e += TB) {
            const int t = e / c.nwa, li = e % c.nwa;
            const double x = Tlx(t, li);
            lx(t, li) = x; lx0(t, li) = x;
          }
          for (int e = c.tid; e < Tp * c.nwa; e += TB) {
            const int t = e / c.nwa, li = e % c.nwa;
            const double y = TlyC(t, li);
            lyC(t, li) = y; lyC0(t, li) = y;
          }
          for (int e = c.tid; e < P * nr; e += TB) { ly[e] = Tly[e]; ly0[e] = Tly[e]; }
          __syncthreads();
          if (c.tid == 0) { sc->kk = 0; sc->it++; }
          __syncthreads();
          continue;
        }
      }
      {
        const double kk = (double)sc->kk;
        const double a1 = (kk + 1.0) / (kk + 2.0), a0 = 1.0 / (kk + 2.0), rho = ctl.rho;
        for (int e = c.tid; e < P * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          lx(t, li) = a1 * ((1.0 + rho) * Tlx(t, li) - rho * lx(t, li)) + a0 * lx0(t, li);
        }
        for (int e = c.tid; e < Tp * c.nwa; e += TB) {
          const int t = e / c.nwa, li = e % c.nwa;
          lyC(t, li) = a1 * ((1.0 + rho) * TlyC(t, li) - rho * lyC(t, li)) + a0 * lyC0(t, li);
        }
        for (int e = c.tid; e < P * nr; e += TB) ly[e] = a1 * ((1.0 + rho) * Tly[e] - rho * ly[e]) + a0 * ly0[e];
        __syncthreads();
        if (c.tid == 0) { sc->kk++; sc->it++; }
        __syncthreads();
      }
    }
    // ---- gradients at the final lambda (one more application gives nu, mu_y)
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      lx(t, li) = Tlx(t, li);
    }
    for (int e = c.tid; e < Tp * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      lyC(t, li) = TlyC(t, li);
    }
    for (int e = c.tid; e < P * nr; e += TB) ly[e] = Tly[e];
    __syncthreads();
    if (!apply()) goto adj_fail;
    for (int e = c.tid; e < P * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      a.grad_alpha[(size_t)t * n + c.i0 + li] = xv3[t * nw + li];
    }
    for (int e = c.tid; e < Tp * c.nwa; e += TB) {
      const int t = e / c.nwa, li = e % c.nwa;
      a.grad_s[(size_t)t * n + c.i0 + li] = lyC(t, li) * gsf(t, li);
    }
    for (int e = c.tid; e < c.nwa * p.k; e += TB) {
      const int li = e / p.k, l = e % p.k, j = m + l;
      const double dci = V.dc(0, li), drj = p.dr[j];
      double gsum = 0.0, msum = 0.0;
      for (int t = 0; t < P; ++t) {
        const double wst = dci * xs(t, li);
        gsum += sigma * muy[t * nr + j] * wst - ys[t * nr + j] * xv3[t * nw + li];
        msum += muy[t * nr + j];
      }
      double g = drj * gsum;
      if (p.multi) g -= sigma * drj * V.cvec(0, li) * msum;
      a.grad_G[(size_t)(c.i0 + li) * p.k + l] = g;
    }
  }
  if (c.wg == 0 && c.tid == 0) {
    a.info[IX_ITERS] = (double)sc->it;
    a.info[IX_RESTARTS] = (double)sc->restarts;
    a.info[IX_OMEGA] = sc->omega;
    a.info[IX_ETA] = sc->eta;
    a.info[IX_CHECKS] = (double)sc->checks;
    a.info[IX_EXCHANGES] = (double)c.epoch;
    a.status[0] = sc->status;
  }
  return;

adj_fail:
  if (c.tid == 0) __hip_atomic_store(a.status, (int32_t)DS_BARRIER, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return;
}

// grad_F[i][p] = sum_l grad_G[i][l] C[p][l]
__global__ __launch_bounds__(TB) void k_grad_F(int n, int k, const double* __restrict__ gG, const double* __restrict__ C,
                                              double* __restrict__ gF) {
  const int64_t e = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (e >= (int64_t)n * k) return;
  const int i = (int)(e / k), pp = (int)(e % k);
  double s = 0.0;
  for (int l = 0; l < k; ++l) s = fma(gG[(size_t)i * k + l], C[(size_t)pp * k + l], s);
  gF[e] = s;
}

}  // namespace

int solve_vmax(const DevProblem& p) {
  const int P = p.P, nr = p.nr;
  int v = STW * P + 2 * P * nr;                   // speculative exchange
  v = std::max(v, 16 + P + P * nr + STW * P);     // check exchange
  v = std::max(v, 3 * P * MSC);                   // multisection round
  v = std::max(v, 2 + P * nr);                    // power iteration
  return (v + 63) / 64 * 64;
}

// LDS doubles of the per-asset state (the arrays the kernel takes when it holds the
// state in LDS, in the same order and rounding).
template <class R>
static size_t state_lds_doubles(size_t P, size_t Tp, size_t nw) {
  return 4 * P * nw + 2 * lds_doubles<R>(P * nw) + Tp * nw + 2 * lds_doubles<R>(Tp * nw) +
         lds_doubles<R>(P * nw) + 2 * lds_doubles<R>(Tp * nw) + Tp * nw + lds_doubles<R>(nw) + 4 * nw;
}

size_t solve_lds_bytes(const DevProblem& p, const DevControl& c) {
  const size_t P = p.P, Tp = p.Tp, nr = p.nr, nw = c.nw;
  const bool f32 = c.prec != PREC_FP64;
  size_t d = 0;
  if (c.lds_k) d += f32 ? lds_doubles<float>(nr * (nw | 1)) : lds_doubles<double>(nr * (nw | 1));
  d += 4 * P * nr + 4 * P * nw + (size_t)c.vmax + RED_LEN + 14 * P + nr;
  if (c.xmode == XM_LOCAL) d += 3 * (size_t)c.vmax;
  if (c.lds_state) d += f32 ? state_lds_doubles<float>(P, Tp, nw) : state_lds_doubles<double>(P, Tp, nw);
  if (c.lists) d += NPOOL * 4 + NPOOL;   // pool, and two ints per pool entry
  d += (sizeof(Scal) + 7) / 8 + 2 + 5 * P + 1;   // flags, nine per-period integer arrays and nidx[P + 1]
  return d * sizeof(double);
}

int launch_solve(const DevProblem& p, const DevState& s, const DevControl& c, void* stream, size_t lds) {
  void* args[] = {(void*)&p, (void*)&s, (void*)&c};
  const void* fn;
  if (c.prec == PREC_FP32)
    fn = c.lds_k ? (c.lds_state ? (const void*)k_solve<true, true, float> : (const void*)k_solve<true, false, float>)
                 : (c.lds_state ? (const void*)k_solve<false, true, float> : (const void*)k_solve<false, false, float>);
  else
    fn = c.lds_k ? (c.lds_state ? (const void*)k_solve<true, true, double> : (const void*)k_solve<true, false, double>)
                 : (c.lds_state ? (const void*)k_solve<false, true, double> : (const void*)k_solve<false, false, double>);
  hipError_t e = hipLaunchCooperativeKernel(fn, dim3(c.nwg), dim3(TB), args, (unsigned int)lds, (hipStream_t)stream);
  return e == hipSuccess ? 0 : (int)e;
}

static const void* batch_fn(int kl, int sl, int prec) {
  // the batched kernel reads its rows from device memory: no LDS slice in the bf16 form
  if (prec == PREC_BF16K) return kl ? nullptr : (sl ? (const void*)k_solve_batch<false, true, float, bf16>
                                                      : (const void*)k_solve_batch<false, false, float, bf16>);
  if (prec == PREC_FP32)
    return kl ? (sl ? (const void*)k_solve_batch<true, true, float> : (const void*)k_solve_batch<true, false, float>)
              : (sl ? (const void*)k_solve_batch<false, true, float> : (const void*)k_solve_batch<false, false, float>);
  return kl ? (sl ? (const void*)k_solve_batch<true, true, double> : (const void*)k_solve_batch<true, false, double>)
            : (sl ? (const void*)k_solve_batch<false, true, double> : (const void*)k_solve_batch<false, false, double>);
}

int launch_solve_batch(const DevProblem* dp, const DevState* ds, const DevControl* dc, const int* wg_team,
                       const int* wg_rank, int nblocks, int kl, int sl, int prec, void* stream, size_t lds) {
  void* args[] = {(void*)&dp, (void*)&ds, (void*)&dc, (void*)&wg_team, (void*)&wg_rank};
  const void* fn = batch_fn(kl, sl, prec);
  if (!fn) return (int)hipErrorInvalidValue;
  hipError_t e = hipLaunchCooperativeKernel(fn, dim3(nblocks), dim3(TB), args,
                                            (unsigned int)lds, (hipStream_t)stream);
  return e == hipSuccess ? 0 : (int)e;
}

int solve_batch_occupancy(int kl, int sl, int prec, size_t lds) {
  int blocks = 0;
  const void* fn = batch_fn(kl, sl, prec);
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, TB, lds) != hipSuccess) return 0;
  return blocks;
}

int adjoint_vmax(const DevProblem& p) {
  const int P = p.P, nr = p.nr;
  int v = STW * P;
  v = std::max(v, 3 * P * MSC);
  v = std::max(v, P * nr + P);
  v = std::max(v, 2 + P * nr);
  v = std::max(v, 8);
  return (v + 63) / 64 * 64;
}

size_t adjoint_lds_bytes(const DevProblem& p, const DevControl& c) {
  const size_t P = p.P, Tp = p.Tp, nr = p.nr, nw = c.nw;
  size_t d = 0;
  if (c.lds_k) d += nr * (nw | 1);
  d += nr + 8 * P * nr + 4 * P * nw + Tp * nw + (size_t)c.vmax + RED_LEN + 7 * P;
  d += (sizeof(AScal) + 7) / 8 + 2 + (P + 1) / 2 + 1;
  return d * sizeof(double);
}

int launch_adjoint(const DevProblem& p, const AdjState& a, const DevControl& c, double omega, void* stream,
                   size_t lds) {
  void* args[] = {(void*)&p, (void*)&a, (void*)&c, (void*)&omega};
  const void* fn = c.lds_k ? (const void*)k_adjoint<true> : (const void*)k_adjoint<false>;
  hipError_t e = hipLaunchCooperativeKernel(fn, dim3(c.nwg), dim3(TB), args, (unsigned int)lds, (hipStream_t)stream);
  return e == hipSuccess ? 0 : (int)e;
}

int launch_grad_F(int n, int k, const double* gG, const double* C, double* gF, void* stream) {
  const int64_t tot = (int64_t)n * k;
  if (tot == 0) return 0;
  hipLaunchKernelGGL(k_grad_F, dim3((unsigned)((tot + TB - 1) / TB)), dim3(TB), 0, (hipStream_t)stream, n, k, gG, C, gF);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace ffo

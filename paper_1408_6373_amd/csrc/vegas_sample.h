// vegas_sample.h -- the Vegas DoSample kernel (a1-a6) and the
// per-coordinate helpers it shares with the points kernel.
//
// The kernel template is instantiated per precision and histogram type in
// its own translation unit (vegas_sample_*.hip), so that the instances build
// in parallel; vegas.hip dispatches to them.
#pragma once
#ifndef CCUBA_RTC  // the run-time compiled build has no C++ library headers
#include <cstddef>
#include <vector>
#else
#define offsetof(type, member) __builtin_offsetof(type, member)
#endif

#include "engine.h"
#include "genz.h"
#include "philox.h"
#include "vegas.h"

namespace ccuba {

// ---------------------------------------------------------------------------
// Descriptors read as one word per lane: a single vector load brings a whole
// VJob (or VState) into the wavefront, where field-by-field scalar loads are
// issued as each field is first needed and can each cost a round trip to
// memory.  Lanes past the descriptor's last word read nothing.
constexpr int kJobWords = (int)(sizeof(VJob) / 4);
constexpr int kStateWords = (int)(sizeof(VState) / 4);
static_assert(sizeof(VJob) % 8 == 0 && kJobWords <= 64, "a VJob fits one wavefront");
static_assert(sizeof(VState) % 8 == 0 && kStateWords <= 64, "a VState fits one wavefront");

template <int NW>
__device__ __forceinline__ uint32_t load_words(const void *p, int lane) {
  return lane < NW ? ((const __attribute__((address_space(1))) uint32_t *)p)[lane] : 0u;
}

// The field at byte offset OFF of the descriptor whose words the wavefront
// holds (a wave-uniform value).
template <typename F, int OFF>
__device__ __forceinline__ F word_field(uint32_t w) {
  static_assert(OFF % 4 == 0 && (sizeof(F) == 4 || sizeof(F) == 8), "word-aligned field");
  if constexpr (sizeof(F) == 4) {
    const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)w, OFF / 4);
    F r;
    __builtin_memcpy(&r, &v, 4);
    return r;
  } else {
    const unsigned long long v =
        (unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)w, OFF / 4) |
        ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)w, OFF / 4 + 1) << 32);
    F r;
    __builtin_memcpy(&r, &v, 8);
    return r;
  }
}
#define JOB_FIELD(w, f) (word_field<decltype(VJob::f), (int)offsetof(VJob, f)>(w))

// The whole descriptor from the words the wavefront holds (the reads of
// fields the caller never uses are dropped).
template <typename S>
__device__ __forceinline__ S from_words(uint32_t w) {
  constexpr int n = (int)(sizeof(S) / 4);
  uint32_t words[n];
#pragma unroll
  for (int i = 0; i < n; ++i) words[i] = (uint32_t)__builtin_amdgcn_readlane((int)w, i);
  S r;
  __builtin_memcpy(&r, words, sizeof(S));
  return r;
}

// A device pointer taken from a descriptor word is a generic pointer, and
// loads through it are flat loads, which also count against the scalar
// memory counter: a wait for any scalar load then waits for them too.
// Loads through the global-address-space view are global loads.
template <typename T>
using gbl = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ const gbl<T> *gload(const T *p) {
  return (const gbl<T> *)p;
}
template <typename T>
__device__ __forceinline__ gbl<T> *gstore(T *p) {
  return (gbl<T> *)p;
}

// The value lane l of the wavefront holds (l wave-uniform).
__device__ __forceinline__ double lane_value(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// a3: the grid as staged in LDS.  Cell k of dimension j sits at [j * N + k]
// and holds its lower edge and its span in the working precision: the width
// E[k+1] - E[k] for a general N, and N times the width when N = 2^L.  Both
// are formed once per tile from the two converted edges, exactly as they
// would be formed per point (scaling by 2^L is exact), so staging changes no
// value.  One LDS read per coordinate fetches both.

template <typename T>
struct alignas(2 * sizeof(T)) Cell {
  T lo, span;
};

// Each thread loads the edges of kStageCells cells before it stores any, so
// that the whole grid of a typical integral (up to kStageCells * blockDim
// cells) arrives in one round trip to memory.  Indices past the end are
// clamped to the last cell: their loads stay in range and nothing is stored.
constexpr int kStageCells = 4;

template <typename T, bool POW2>
__device__ __forceinline__ void stage_cells(const double *__restrict__ E, int d, int N,
                                            Cell<T> *sC) {
  const int row = N + 1, dN = d * N, bs = blockDim.x;
  const T Nt = (T)N;
  const gbl<double> *Eg = gload(E);
  auto batch = [&](int e0) {
    double lo[kStageCells], hi[kStageCells];
#pragma unroll
    for (int b = 0; b < kStageCells; ++b) {
      const int e = min(e0 + b * bs, dN - 1), j = e / N, k = e - j * N;
      lo[b] = Eg[j * row + k];
      hi[b] = Eg[j * row + k + 1];
    }
#pragma unroll
    for (int b = 0; b < kStageCells; ++b) {
      const int e = e0 + b * bs;
      const T l = (T)lo[b], h = (T)hi[b];
      if (e < dN) sC[e] = Cell<T>{l, POW2 ? Nt * (h - l) : h - l};
    }
  };
  // the first batch outside the loop: a loop head would wait for every load
  // in flight (the caller's too) before reusing the batch's registers
  batch(threadIdx.x);
  for (int e0 = threadIdx.x + kStageCells * bs; e0 < dN; e0 += kStageCells * bs) batch(e0);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}


template <typename T>
__device__ __forceinline__ const T *param_ptr(const VJob &J, int which);
template <>
__device__ __forceinline__ const double *param_ptr<double>(const VJob &J, int which) {
  return J.p64 + which * kParamRow;
}
template <>
__device__ __forceinline__ const float *param_ptr<float>(const VJob &J, int which) {
  return J.p32 + which * kParamRow;
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }

// Bin and fractional position of one coordinate (a2 + the first half of
// a3).  General N: z = y N, k = min(floor z, N - 1), frac = z - k, then
// x = fma(frac, width, lo) and w *= N width.
// N = 2^L: the bin is the top L bits of the word and the fraction the bits
// below them, which is exactly what the floating-point formula gives (every
// step there is exact).  These helpers return fs = frac / N (exact), so that
// with the staged span s = N width, x = fma(fs, s, lo) has the same exact
// product fs s = frac width and rounds to the same x, and w *= s is the same
// product as before: one multiply fewer per coordinate.
__device__ __forceinline__ void bin_frac_pow2(uint32_t r, int L, double scale, double &fs,
                                              int &k) {
  k = (int)(r >> (32 - L));
  const uint32_t m = (r << L) | (1u << (L - 1));  // (r N mod 2^32) + N/2
  fs = (double)m * scale;                         // scale = 2^(-32-L)
}
__device__ __forceinline__ void bin_frac_pow2(uint32_t r, int L, float scale, float &fs,
                                              int &k) {
  k = (int)(r >> (32 - L));
  // the 23 - L bits of r >> 9 below the bin index, then the half-step bit
  // 2^(L-1), as the mantissa M of a float with exponent -L: that float is
  // 2^-L (1 + M 2^-23), and removing 2^-L (= scale) leaves M 2^(-23-L)
  // = frac / N exactly.  (x & mask) | c is one three-input bit operation
  // (truth table 0xEA).
  static_assert(kMaxBins <= 512, "the shift below needs L <= 9");
  const uint32_t mask = 0x7FFFFFu & ~((1u << L) - 1u);
  const uint32_t c = ((uint32_t)(127 - L) << 23) | (1u << (L - 1));
  const uint32_t bits = (uint32_t)__builtin_amdgcn_bitop3_b32(r >> (9 - L), mask, c, 0xEA);
  fs = __uint_as_float(bits) - scale;
}
__device__ __forceinline__ void bin_frac_any(uint32_t r, int N, double Nd, double &frac, int &k) {
  const double y = (double)r * 0x1p-32 + 0x1p-33;
  const double z = y * Nd;
  int kk = (int)z;
  kk = kk > N - 1 ? N - 1 : kk;
  frac = z - (double)kk;
  k = kk;
}
__device__ __forceinline__ void bin_frac_any(uint32_t r, int N, float Nf, float &frac, int &k) {
  const float y = (float)(r >> 9) * 0x1p-23f + 0x1p-24f;
  const float z = y * Nf;
  int kk = (int)z;
  kk = kk > N - 1 ? N - 1 : kk;
  frac = z - (float)kk;
  k = kk;
}

// 2^-L (FP32) or 2^(-32-L) (FP64): the scale of the power-of-two fraction.
template <typename T>
__device__ __forceinline__ T pow2_scale(int L);
template <>
__device__ __forceinline__ float pow2_scale<float>(int L) {
  return __uint_as_float((uint32_t)(127 - L) << 23);
}
template <>
__device__ __forceinline__ double pow2_scale<double>(int L) {
  return __longlong_as_double((long long)(1023 - 32 - L) << 52);
}

// ---------------------------------------------------------------------------
// a6: the histogram in 64-bit fixed point, exactly.
//
// LDS integer adds are several times cheaper than FP64 adds on gfx950 (and
// FP32 LDS atomics far slower still).  With FP32 evaluation every v^2 has a
// 24-bit mantissa, so a v^2 that is a whole multiple of a unit 2^(E-62) goes
// into an unsigned 64-bit sum without any rounding; 2^E bounds the tile's
// total of every bin, so the sums cannot overflow, and integer sums do not
// depend on the order of the adds.  Every other v^2 -- too small to be a
// whole multiple of the unit, above the cap, or not finite -- goes to a
// second, FP64 histogram, as on the FP64 path.  The two are added when the
// tile is written, so the tile's histogram is the FP64 one up to rounding
// order: the split changes speed, not results.
//
// The bound is 2^E >= 4 cnt c for the tile's cnt points and a cap c on the
// v^2 that may enter the fixed-point sums.  In an integral's first
// iteration c is a true bound from the staged grid and the integrand's
// maximum: w <= prod_j max_k (N width_jk), and f <= 1 for every family except
// the product peak, where f <= 1 / prod_j a_j^-2 (the FP32 products are
// formed in the order the point's own products are, so rounding keeps them
// bounds).  Once the grid adapts that bound grows far beyond the values that
// occur (it takes every dimension's widest bin), so later iterations take
// c = 1024 times the mean v^2 of the previous one (at most 1 in 1024 of the
// v^2 exceed that).
//
// With FP64 evaluation v^2 has a 53-bit mantissa M, v^2 = M 2^(e - 1075) for
// the biased exponent e.  In units U = 2^(E - 91) it is the integer
// X = M 2^s, s = e - 984 - E, whenever s >= 0, and X < 2^90: its low 32 bits
// and X >> 32 go to two 64-bit sums (below 2^46 and 2^57 for a tile of any
// size), so the FP64 histogram too is exact and does not depend on the order
// of the adds, for two integer LDS adds that cost about what one FP64 LDS
// add does.  Every other v^2 goes to the FP64 histogram beside them.

template <typename HT>
struct FixedHist {
  static constexpr bool value = false;
};
template <>
struct FixedHist<unsigned long long> {
  static constexpr bool value = true;
};

// Sample the points [i0, i0 + cnt) of one tile; lane sums of v - shift and
// (v - shift)^2 go to S1, S2.
// NB = ceil(d/4) Philox blocks per point is a template argument so that the
// per-dimension loop is fully unrolled with only the last block guarded, and
// FULL (d = 4 NB) drops that guard too.
// Each lane carries ILP independent points per trip (q, q + blockDim, ...),
// so that several Philox chains are in flight; a point past the tile end is
// computed (its LDS reads stay in range) but contributes nothing.  A trip's
// histogram updates are issued at its end, so that the LDS works through
// them while the next trip's Philox rounds run; the next trip's wait for its
// grid reads then finds them done.  (Updates deferred to after the next
// trip's grid reads made every such wait also wait for the updates.)
template <typename T, typename HT, int FAM, int NB, int ILP, bool POW2, bool FULL>
__device__ __forceinline__ void sample_tile(const VJob &J, int t, long long i0, int cnt,
                                            const Cell<T> *__restrict__ sC, HT *sH,
                                            const T (&pp0)[4 * NB], const T (&pp1)[4 * NB],
                                            int E, float cap, double shift,
                                            double *sHx, double &S1, double &S2) {
  constexpr int ND = 4 * NB;
  const int d = J.ndim, N = J.nbins;
  const T Nt = (T)N;
  const int L = POW2 ? 31 - __clz(N) : 0;
  const T scale = pow2_scale<T>(L);
  const uint32_t c1 = (uint32_t)t << 8;
  const uint32_t sid = J.sid, k0 = J.key0, k1 = J.key1;
#ifndef CCUBA_RTC
  const T phase0 = pp1[0];
#endif
  const int bs = blockDim.x;
  // an assembly comment naming the family, so that the per-point loop that
  // follows can be found in the assembly listing (it emits no instruction)
  asm volatile("; ccuba sample_tile family %0" ::"n"(FAM));
  for (int q0 = threadIdx.x; q0 < cnt; q0 += ILP * bs) {
    T fr[ILP][ND], lo[ILP][ND], sp[ILP][ND];
    int idx[ILP][ND];
    // words, bins and the grid cells they select
#pragma unroll
    for (int e = 0; e < ILP; ++e) {
      const uint32_t i = (uint32_t)(i0 + q0 + e * bs);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const U4 r = philox4x32_10(U4{i, c1 | (uint32_t)b, sid, 0u}, k0, k1);
        const uint32_t rr[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int j = 4 * b + c;
          if (FULL || b < NB - 1 || j < d) {
            int k;
            if (POW2)
              bin_frac_pow2(rr[c], L, scale, fr[e][j], k);
            else
              bin_frac_any(rr[c], N, Nt, fr[e][j], k);
            idx[e][j] = j * N + k;
            const Cell<T> cell = sC[j * N + k];
            lo[e][j] = cell.lo;
            sp[e][j] = cell.span;
          }
        }
      }
    }
    // weights, integrand, sums, histogram updates
#pragma unroll
    for (int e = 0; e < ILP; ++e) {
      T w = (T)1;
#ifdef CCUBA_RTC
      // a caller's function of the whole point, compiled with this kernel:
      // T ccuba_user(const T *x, int ndim, const T *a, const T *u)
      T xs[ND];
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        if (FULL || j < 4 * (NB - 1) || j < d) {
          xs[j] = fma_t(fr[e][j], sp[e][j], lo[e][j]);
          w = POW2 ? w * sp[e][j] : w * (Nt * sp[e][j]);
        } else {
          xs[j] = (T)0;
        }
      }
      const T v = w * ccuba_user(xs, d, pp0, pp1);
#else
      T acc = Genz<T, FAM>::init(phase0);
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        if (FULL || j < 4 * (NB - 1) || j < d) {
          const T x = fma_t(fr[e][j], sp[e][j], lo[e][j]);
          w = POW2 ? w * sp[e][j] : w * (Nt * sp[e][j]);
          acc = Genz<T, FAM>::step(acc, x, pp0[j], pp1[j]);
        }
      }
      const T v = w * Genz<T, FAM>::finish(acc, d);
#endif
      if (q0 + e * bs < cnt) {
        const double dv = (double)v - shift;
        S1 += dv;
        S2 = fma(dv, dv, S2);
        if constexpr (FixedHist<HT>::value && sizeof(T) == 8) {
          const double v2 = v * v;
          const unsigned long long b = (unsigned long long)__double_as_longlong(v2);
          const int eb = (int)(b >> 52);
          const int s = eb - (984 + E);  // v2 = M 2^s units; s <= 37 below the cap
          if (v2 <= (double)cap && s >= 0 && eb >= 1) {
            const unsigned long long M = (b & 0xFFFFFFFFFFFFFull) | (1ull << 52);
            const unsigned long long xlo = (M << s) & 0xFFFFFFFFull;
            const unsigned long long xhi = (M << 11) >> (43 - s);  // floor(M 2^(s-32))
            HT *sHh = sH + d * N;
#pragma unroll
            for (int j = 0; j < ND; ++j)
              if (FULL || j < 4 * (NB - 1) || j < d) {
                atomicAdd(&sH[idx[e][j]], xlo);
                atomicAdd(&sHh[idx[e][j]], xhi);
              }
          } else {  // not a normal whole multiple of the unit, above the cap, or not finite
#pragma unroll
            for (int j = 0; j < ND; ++j)
              if (FULL || j < 4 * (NB - 1) || j < d) unsafeAtomicAdd(&sHx[idx[e][j]], v2);
          }
        } else if constexpr (FixedHist<HT>::value) {
          const float v2f = (float)(v * v);
          const uint32_t b = __float_as_uint(v2f);
          const int sh = (int)(b >> 23) - (88 + E);  // v2 = m 2^sh units
          if (v2f <= cap && sh >= 0 && b >= 0x800000u) {  // (zeros and subnormals: below)
            const unsigned long long v2 = (unsigned long long)((b & 0x7FFFFFu) | 0x800000u)
                                          << sh;
#pragma unroll
            for (int j = 0; j < ND; ++j)
              if (FULL || j < 4 * (NB - 1) || j < d) atomicAdd(&sH[idx[e][j]], v2);
          } else {  // not a normal whole multiple of the unit, above the cap, or not finite
            const double v2 = (double)v2f;
#pragma unroll
            for (int j = 0; j < ND; ++j)
              if (FULL || j < 4 * (NB - 1) || j < d) unsafeAtomicAdd(&sHx[idx[e][j]], v2);
          }
        } else {
          const HT v2 = (HT)(v * v);
#pragma unroll
          for (int j = 0; j < ND; ++j)
            if (FULL || j < 4 * (NB - 1) || j < d) unsafeAtomicAdd(&sH[idx[e][j]], v2);
        }
      }
    }
  }
}

// One kernel per (precision, histogram type, ILP, NB, power-of-two bins,
// d = 4 NB): every instance only holds the registers and the tests its own
// class needs.  A launch walks the slice [tile_first, tile_first +
// tile_count) of the tile list, which holds the tiles of the jobs of that
// class.
template <typename T, typename HT, int ILP, int NB, bool POW2, bool FULL>
__global__ void __launch_bounds__(256) vegas_dosample_kernel(VegasArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[2][4];
  __shared__ uint32_t smax[kMaxDim + 2];  // fixed-point histogram: per-dimension maxima, E, cap
  Cell<T> *sC = (Cell<T> *)smem;
  HT *sH = (HT *)(smem + A.lds_hist_byte_off);
  const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63, wid = tid >> 6;
  const int myprec = sizeof(T) == 8 ? FP64 : FP32;

  const int tend = A.tile_first + A.tile_count;
  for (int tt = A.tile_first + blockIdx.x; tt < tend; tt += gridDim.x) {
    // the descriptor as one vector load (a word per lane); with one job in
    // the launch its index needs no lookup
    const int jb = A.njobs == 1 ? 0 : A.tile_job[tt];
    const VJob J = from_words<VJob>(load_words<kJobWords>(A.jobs + jb, lane));
    if (J.prec != myprec || ((J.ndim + 3) >> 2) != NB ||
        ((J.nbins & (J.nbins - 1)) == 0) != POW2 || (J.ndim == 4 * NB) != FULL)
      continue;
    const int d = J.ndim, N = J.nbins, dN = d * N;
    // One round trip to memory for: the state (a word per lane), the
    // integrand's parameters (rows zero-padded to 16) and the grid cells
    // (staged into LDS whether or not the integral turns out to be done).
    uint32_t sw = load_words<kStateWords>(J.state, lane);
    constexpr int ND = 4 * NB;
    T pp0[ND], pp1[ND];
    {
      const gbl<T> *p0 = gload(param_ptr<T>(J, 0)), *p1 = gload(param_ptr<T>(J, 1));
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        pp0[j] = p0[j];
        pp1[j] = p1[j];
      }
    }
    stage_cells<T, POW2>(J.grid, d, N, sC);
    // the state words are first used here, after the cells' loads are issued
    // (without this the compiler waits for them before issuing those loads)
    asm volatile("" : "+v"(sw)::"memory");
    const VState st = from_words<VState>(sw);
    if (st.done) continue;  // the same for the whole block: nothing read the cells yet
    const int lt = tt - J.tile0;
    const long long n_t = J.nstart + (long long)st.T * J.nincrease;
    const long long i0 = (long long)lt * J.tile_pts;
    long long c = n_t - i0;
    c = c < 0 ? 0 : (c > J.tile_pts ? J.tile_pts : c);
    const int cnt = (int)c;

    // fixed point: the integer sums (two per bin with FP64 evaluation), then
    // the FP64 histogram of the rest
    constexpr int kFixWords = (FixedHist<HT>::value && sizeof(T) == 8) ? 2 : 1;
    for (int e = tid; e < kFixWords * dN; e += bs) sH[e] = (HT)0;
    double *sHx = (double *)(sH + kFixWords * dN);
    if constexpr (FixedHist<HT>::value) {
      for (int e = tid; e < dN; e += bs) sHx[e] = 0.0;
      if (tid <= kMaxDim) smax[tid] = 0u;
    }
    __syncthreads();

    int E = 0;
    float cap = 0.0f;
    if constexpr (FixedHist<HT>::value) {
      const float prev = st.hcap;
      if (!(prev > 0.0f)) {
        // first iteration: per dimension the largest weight factor
        // (positive floats order as their bit patterns)
        const T Nt = (T)N;
        for (int e = tid; e < dN; e += bs) {
          const T f = POW2 ? sC[e].span : Nt * sC[e].span;
          atomicMax(&smax[e / N], __float_as_uint((float)f));
        }
        __syncthreads();
      }
      if (tid == 0) {
        float cv;
        if (prev > 0.0f) {
          cv = prev;
        } else {
          float w = 1.0f, q = 1.0f;
          for (int j = 0; j < d; ++j) w = w * __uint_as_float(smax[j]);
          if (J.family == PRODUCT_PEAK) {
            for (int j = 0; j < d; ++j) q = q * (float)pp0[j];
            q = 1.0f / q;
          }
          const float v = w * q;
          cv = v * v;
        }
        // a cap that is not finite or too large for the sums' exponent range
        // (an integrand far above 1) sends every value to the FP64 histogram
        if (!(cv <= 0x1p100f)) cv = 0.0f;
        // 2^E >= 4 cnt c bounds the fixed-point total of every bin
        const double B = 4.0 * (double)cv * (double)(cnt > 0 ? cnt : 1);
        int ex = 0;
        (void)frexp(B, &ex);
        smax[kMaxDim] = (uint32_t)ex;
        smax[kMaxDim + 1] = __float_as_uint(cv);
      }
      __syncthreads();
      E = (int)smax[kMaxDim];
      cap = __uint_as_float(smax[kMaxDim + 1]);
    }
    double S1 = 0.0, S2 = 0.0;
#ifdef CCUBA_RTC
    sample_tile<T, HT, USER, NB, ILP, POW2, FULL>(J, st.T, i0, cnt, sC, sH, pp0, pp1, E, cap, st.shift, sHx, S1, S2);
#else
    switch (J.family) {
      case GAUSSIAN: sample_tile<T, HT, GAUSSIAN, NB, ILP, POW2, FULL>(J, st.T, i0, cnt, sC, sH, pp0, pp1, E, cap, st.shift, sHx, S1, S2); break;
      case OSCILLATORY: sample_tile<T, HT, OSCILLATORY, NB, ILP, POW2, FULL>(J, st.T, i0, cnt, sC, sH, pp0, pp1, E, cap, st.shift, sHx, S1, S2); break;
      case PRODUCT_PEAK: sample_tile<T, HT, PRODUCT_PEAK, NB, ILP, POW2, FULL>(J, st.T, i0, cnt, sC, sH, pp0, pp1, E, cap, st.shift, sHx, S1, S2); break;
      case CORNER_PEAK: sample_tile<T, HT, CORNER_PEAK, NB, ILP, POW2, FULL>(J, st.T, i0, cnt, sC, sH, pp0, pp1, E, cap, st.shift, sHx, S1, S2); break;
      default: sample_tile<T, HT, C0, NB, ILP, POW2, FULL>(J, st.T, i0, cnt, sC, sH, pp0, pp1, E, cap, st.shift, sHx, S1, S2); break;
    }
#endif
    S1 = wave_sum(S1);
    S2 = wave_sum(S2);
    if (lane == 0) {
      red[0][wid] = S1;
      red[1][wid] = S2;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int q = 0; q < (bs >> 6); ++q) {
        a += red[0][q];
        b += red[1][q];
      }
      J.tsums[2 * lt] = a;
      J.tsums[2 * lt + 1] = b;
    }
    double *th = J.thist + (long long)lt * dN;
    if constexpr (FixedHist<HT>::value && sizeof(T) == 8) {
      for (int e = tid; e < dN; e += bs)
        th[e] = ldexp((double)sH[dN + e], E - 59) + ldexp((double)sH[e], E - 91) + sHx[e];
    } else if constexpr (FixedHist<HT>::value) {
      for (int e = tid; e < dN; e += bs) th[e] = ldexp((double)sH[e], E - 62) + sHx[e];
    } else {
      for (int e = tid; e < dN; e += bs) th[e] = (double)sH[e];
    }

    __syncthreads();
  }
}

#ifndef CCUBA_RTC
// ---------------------------------------------------------------------------
// launchers of the instances of one (precision, histogram type)

template <typename T, typename HT, int ILP, int NB>
static void launch_dosample_cls(const VegasArgs &A, bool pow2, bool full, int grid, int block,
                                size_t lds, hipStream_t s) {
  if (pow2) {
    if (full)
      hipLaunchKernelGGL((vegas_dosample_kernel<T, HT, ILP, NB, true, true>), dim3(grid),
                         dim3(block), lds, s, A);
    else
      hipLaunchKernelGGL((vegas_dosample_kernel<T, HT, ILP, NB, true, false>), dim3(grid),
                         dim3(block), lds, s, A);
  } else {
    if (full)
      hipLaunchKernelGGL((vegas_dosample_kernel<T, HT, ILP, NB, false, true>), dim3(grid),
                         dim3(block), lds, s, A);
    else
      hipLaunchKernelGGL((vegas_dosample_kernel<T, HT, ILP, NB, false, false>), dim3(grid),
                         dim3(block), lds, s, A);
  }
}

template <typename T, typename HT, int ILP>
static void launch_dosample_ilp(const VegasArgs &A, int nb, bool pow2, bool full, int grid,
                                int block, size_t lds, hipStream_t s) {
  switch (nb) {
    case 1: launch_dosample_cls<T, HT, ILP, 1>(A, pow2, full, grid, block, lds, s); break;
    case 2: launch_dosample_cls<T, HT, ILP, 2>(A, pow2, full, grid, block, lds, s); break;
    case 3: launch_dosample_cls<T, HT, ILP, 3>(A, pow2, full, grid, block, lds, s); break;
    default: launch_dosample_cls<T, HT, ILP, 4>(A, pow2, full, grid, block, lds, s); break;
  }
}

template <typename T, typename HT>
static hipError_t launch_dosample_t(const VegasArgs &A, int nb, bool pow2, bool full, int grid,
                                    int block, size_t lds, hipStream_t s) {
  if (A.ilp == 2)
    launch_dosample_ilp<T, HT, 2>(A, nb, pow2, full, grid, block, lds, s);
  else
    launch_dosample_ilp<T, HT, 1>(A, nb, pow2, full, grid, block, lds, s);
  return hipGetLastError();
}

template <typename T, typename HT, int ILP, int NB>
static void dosample_fns_cls(std::vector<const void *> &fns) {
  fns.push_back((const void *)vegas_dosample_kernel<T, HT, ILP, NB, true, true>);
  fns.push_back((const void *)vegas_dosample_kernel<T, HT, ILP, NB, true, false>);
  fns.push_back((const void *)vegas_dosample_kernel<T, HT, ILP, NB, false, true>);
  fns.push_back((const void *)vegas_dosample_kernel<T, HT, ILP, NB, false, false>);
}

template <typename T, typename HT>
static void dosample_fns_t(std::vector<const void *> &fns) {
  dosample_fns_cls<T, HT, 1, 1>(fns);
  dosample_fns_cls<T, HT, 1, 2>(fns);
  dosample_fns_cls<T, HT, 1, 3>(fns);
  dosample_fns_cls<T, HT, 1, 4>(fns);
  dosample_fns_cls<T, HT, 2, 1>(fns);
  dosample_fns_cls<T, HT, 2, 2>(fns);
  dosample_fns_cls<T, HT, 2, 3>(fns);
  dosample_fns_cls<T, HT, 2, 4>(fns);
}

#endif  // CCUBA_RTC

}  // namespace ccuba

// Workgroup-resident negacyclic NTT for one polynomial of n = 2^LOGN words.
//
// The transform is the one of the scheme: entry i of the forward transform of
// a(X) mod q is a(psi^(2 brv(i) + 1)), psi the smallest primitive 2n-th root.
// It is evaluated as Cooley-Tukey stages s = 0..LOGN-1 (stage s: 2^s groups,
// butterfly distance n / 2^(s+1), twiddle psi^brv(2^s + group)) with lazy
// reduction (paper §7.1): the twiddle product t = W Y mod q uses a Shoup
// quotient without its low partial products (t in [0, 4q), shoup4), and the
// forward butterfly X' = X + t, Y' = X + 4q - t does no other reduction, so a
// bound B on the inputs grows to B + 4q per stage.  With q < 2^54 and inputs
// below 2q, all 13 stages of an n = 8192 transform stay below 54q < 2^60, and
// the outputs are reduced once.
// The inverse runs Gentleman-Sande butterflies of the same stages in reverse
// order, keeping values in [0, 4q): X' = X + Y (minus 4q when above),
// Y' = W (X - Y + 4q) with the same quotient.
//
// Layout on gfx950: T = n/E threads, E = 2^LOGE elements per thread in
// registers.  Stages are grouped in passes of LOGE (radix E) done entirely in
// registers; between passes the polynomial goes through LDS (n words plus
// padding).  Element e of thread tid in the pass starting at stage S0
// (window of RW stages, combos of 2^RW elements) has index
//     idx = (high << (LOGN - S0)) | (w << LOWB) | low,
//     e = c * 2^RW + w, combo = tid + T * c, high = combo >> LOWB,
//     low = combo mod 2^LOWB, LOWB = LOGN - S0 - RW.
// The first pass is the natural order (idx = (e << (LOGN-LOGE)) | tid: lanes
// read consecutive words), the last pass leaves each thread with contiguous
// elements of the transform.
#pragma once
#include "arith.h"

namespace wally {

template <int LOGN, int LOGE>
struct NttShape {
  static constexpr int N = 1 << LOGN;
  static constexpr int E = 1 << LOGE;
  static constexpr int T = N / E;
  static constexpr int NPASS = (LOGN + LOGE - 1) / LOGE;
  static constexpr int LAST_S0 = LOGE * (NPASS - 1);
  static constexpr int LDS_WORDS = N + N / 32;
  __device__ static __forceinline__ int lds(int idx) { return idx + (idx >> 5); }
};

template <int LOGN, int LOGE, int S0>
struct PassMap {
  static constexpr int RW = (LOGN - S0) < LOGE ? (LOGN - S0) : LOGE;
  static constexpr int LOWB = LOGN - S0 - RW;
  static constexpr int COMBOS = (1 << LOGE) >> RW;
  static constexpr int T = NttShape<LOGN, LOGE>::T;
  // index of register e of thread tid
  __host__ __device__ static constexpr uint32_t idx_c(int tid, int e) {
    const uint32_t c = (uint32_t)e >> RW, w = (uint32_t)e & ((1u << RW) - 1);
    const uint32_t combo = (uint32_t)tid + T * c;
    const uint32_t high = combo >> LOWB, low = combo & ((1u << LOWB) - 1);
    return (high << (LOGN - S0)) | (w << LOWB) | low;
  }
  __device__ static __forceinline__ uint32_t idx(int tid, int e) { return idx_c(tid, e); }
};

// The index of a map is a thread part OR an element part on disjoint bits
// (combo = tid + T c puts tid below c), and the padded LDS offset idx +
// idx / 32 of such a sum splits the same way (no carry crosses bit 5).  So an
// exchange needs one per-thread base and compile-time element offsets, which
// become the immediate offsets of the LDS instructions.
template <int LOGN, int LOGE, class MAP>
__device__ __forceinline__ int lds_base(int tid) {
  return NttShape<LOGN, LOGE>::lds(MAP::idx(tid, 0));
}
template <int LOGN, int LOGE, class MAP>
__host__ __device__ constexpr int lds_off(int e) {
  return (int)(MAP::idx_c(0, e) + (MAP::idx_c(0, e) >> 5));
}
template <int LOGN, int LOGE, class MAP>
constexpr bool lds_split_holds() {
  constexpr int T = NttShape<LOGN, LOGE>::T, E = 1 << LOGE;
  for (int tid = 0; tid < T; ++tid)
    for (int e = 0; e < E; ++e) {
      const uint32_t i = MAP::idx_c(tid, e), i0 = MAP::idx_c(tid, 0), ie = MAP::idx_c(0, e);
      if ((i0 & ie) != 0 || (i0 | ie) != i) return false;
      if (i + (i >> 5) != i0 + (i0 >> 5) + ie + (ie >> 5)) return false;
    }
  return true;
}

template <int LOGN, int LOGE>
using FirstMap = PassMap<LOGN, LOGE, 0>;
template <int LOGN, int LOGE>
using LastMap = PassMap<LOGN, LOGE, NttShape<LOGN, LOGE>::LAST_S0>;

// Cooley-Tukey butterfly without reduction: inputs below B, outputs below B + 4q
// (q4 = 4q).
__device__ __forceinline__ void ct_bfly(uint64_t& X, uint64_t& Y, ulonglong2 W, uint64_t q, uint64_t q4) {
  const uint64_t t = shoup4(Y, W.x, W.y, 0 - q);
  Y = X + q4 - t;
  X = X + t;
}

// Gentleman-Sande butterfly, inputs and outputs in [0, 4q) (q4 = 4q).
__device__ __forceinline__ void gs_bfly(uint64_t& X, uint64_t& Y, ulonglong2 W, uint64_t q, uint64_t q4) {
  const uint64_t u = X + Y;
  const uint64_t v = X - Y + q4;
  X = csub(u, q4);
  Y = shoup4(v, W.x, W.y, 0 - q);
}

// Group index of combination c of thread tid in pass S0.  When the pass's low
// bits cover every thread index (the first forward pass, the last inverse
// pass) it does not depend on tid: written as a constant, the twiddles of the
// pass become uniform loads.
template <int LOGN, int LOGE, int S0>
__device__ __forceinline__ uint32_t pass_high(int tid, int c) {
  using M = PassMap<LOGN, LOGE, S0>;
  constexpr int LOGT = LOGN - LOGE;
  if constexpr (M::LOWB >= LOGT) return (uint32_t)c >> (M::LOWB - LOGT);
  else return ((uint32_t)tid + M::T * (uint32_t)c) >> M::LOWB;
}

template <int LOGN, int LOGE, int S0>
__device__ __forceinline__ void ct_pass(uint64_t (&x)[1 << LOGE], const ulonglong2* __restrict__ tw, uint64_t q,
                                        uint64_t q4, int tid) {
  using M = PassMap<LOGN, LOGE, S0>;
#pragma unroll
  for (int c = 0; c < M::COMBOS; ++c) {
    const uint32_t high = pass_high<LOGN, LOGE, S0>(tid, c);
#pragma unroll
    for (int ls = 0; ls < M::RW; ++ls) {
      const int half = 1 << (M::RW - 1 - ls);
#pragma unroll
      for (int w = 0; w < (1 << M::RW); ++w) {
        if (w & half) continue;
        const uint32_t grp = ((high << M::RW) | (uint32_t)w) >> (M::RW - ls);
        const ulonglong2 W = tw[(1u << (S0 + ls)) + grp];
        ct_bfly(x[c * (1 << M::RW) + w], x[c * (1 << M::RW) + w + half], W, q, q4);
      }
    }
  }
}

template <int LOGN, int LOGE, int S0>
__device__ __forceinline__ void gs_pass(uint64_t (&x)[1 << LOGE], const ulonglong2* __restrict__ itw, uint64_t q,
                                        uint64_t q4, int tid) {
  using M = PassMap<LOGN, LOGE, S0>;
#pragma unroll
  for (int c = 0; c < M::COMBOS; ++c) {
    const uint32_t high = pass_high<LOGN, LOGE, S0>(tid, c);
#pragma unroll
    for (int ls = M::RW - 1; ls >= 0; --ls) {
      const int half = 1 << (M::RW - 1 - ls);
#pragma unroll
      for (int w = 0; w < (1 << M::RW); ++w) {
        if (w & half) continue;
        const uint32_t grp = ((high << M::RW) | (uint32_t)w) >> (M::RW - ls);
        const ulonglong2 W = itw[(1u << (S0 + ls)) + grp];
        gs_bfly(x[c * (1 << M::RW) + w], x[c * (1 << M::RW) + w + half], W, q, q4);
      }
    }
  }
}

// Move the polynomial from the register mapping of pass A to that of pass B.
// Ends with a barrier so the buffer can be reused right away.
template <int LOGN, int LOGE, int SA, int SB>
__device__ __forceinline__ void exchange(uint64_t (&x)[1 << LOGE], uint64_t* lds, int tid) {
  using S = NttShape<LOGN, LOGE>;
  using MA = PassMap<LOGN, LOGE, SA>;
  using MB = PassMap<LOGN, LOGE, SB>;
  static_assert(lds_split_holds<LOGN, LOGE, MA>() && lds_split_holds<LOGN, LOGE, MB>(), "padded offsets split");
  uint64_t* wa = lds + lds_base<LOGN, LOGE, MA>(tid);
#pragma unroll
  for (int e = 0; e < S::E; ++e) wa[lds_off<LOGN, LOGE, MA>(e)] = x[e];
  __syncthreads();
  const uint64_t* rb = lds + lds_base<LOGN, LOGE, MB>(tid);
#pragma unroll
  for (int e = 0; e < S::E; ++e) x[e] = rb[lds_off<LOGN, LOGE, MB>(e)];
  __syncthreads();
}

// The same move through half the LDS: the low 32-bit halves of the words
// first, then the high halves (N + N/32 32-bit words; four barriers).
template <int LOGN, int LOGE, int SA, int SB>
__device__ __forceinline__ void exchange_split(uint64_t (&x)[1 << LOGE], uint64_t* lds, int tid) {
  using S = NttShape<LOGN, LOGE>;
  using MA = PassMap<LOGN, LOGE, SA>;
  using MB = PassMap<LOGN, LOGE, SB>;
  static_assert(lds_split_holds<LOGN, LOGE, MA>() && lds_split_holds<LOGN, LOGE, MB>(), "padded offsets split");
  uint32_t* l32 = (uint32_t*)lds;
  uint32_t* wa = l32 + lds_base<LOGN, LOGE, MA>(tid);
  const uint32_t* rb = l32 + lds_base<LOGN, LOGE, MB>(tid);
  uint32_t lo[S::E];
#pragma unroll
  for (int e = 0; e < S::E; ++e) wa[lds_off<LOGN, LOGE, MA>(e)] = (uint32_t)x[e];
  __syncthreads();
#pragma unroll
  for (int e = 0; e < S::E; ++e) lo[e] = rb[lds_off<LOGN, LOGE, MB>(e)];
  __syncthreads();
#pragma unroll
  for (int e = 0; e < S::E; ++e) wa[lds_off<LOGN, LOGE, MA>(e)] = (uint32_t)(x[e] >> 32);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < S::E; ++e) x[e] = ((uint64_t)rb[lds_off<LOGN, LOGE, MB>(e)] << 32) | lo[e];
  __syncthreads();
}

template <int LOGN, int LOGE, int P, bool SPLIT = false>
__device__ __forceinline__ void fwd_passes(uint64_t (&x)[1 << LOGE], uint64_t* lds, const ulonglong2* tw, uint64_t q,
                                           uint64_t q4, int tid) {
  constexpr int S0 = LOGE * P;
  if constexpr (S0 < LOGN) {
    if constexpr (P > 0) {
      if constexpr (SPLIT) exchange_split<LOGN, LOGE, LOGE * (P - 1), S0>(x, lds, tid);
      else exchange<LOGN, LOGE, LOGE * (P - 1), S0>(x, lds, tid);
    }
    ct_pass<LOGN, LOGE, S0>(x, tw, q, q4, tid);
    fwd_passes<LOGN, LOGE, P + 1, SPLIT>(x, lds, tw, q, q4, tid);
  }
}

template <int LOGN, int LOGE, int P, bool SPLIT = false>
__device__ __forceinline__ void inv_passes(uint64_t (&x)[1 << LOGE], uint64_t* lds, const ulonglong2* itw, uint64_t q,
                                           uint64_t q4, int tid) {
  if constexpr (P >= 0) {
    constexpr int S0 = LOGE * P;
    if constexpr (P < NttShape<LOGN, LOGE>::NPASS - 1) {
      if constexpr (SPLIT) exchange_split<LOGN, LOGE, LOGE * (P + 1), S0>(x, lds, tid);
      else exchange<LOGN, LOGE, LOGE * (P + 1), S0>(x, lds, tid);
    }
    gs_pass<LOGN, LOGE, S0>(x, itw, q, q4, tid);
    inv_passes<LOGN, LOGE, P - 1, SPLIT>(x, lds, itw, q, q4, tid);
  }
}

// Forward transform.  In: FirstMap order, values < 2q.  Out: LastMap order,
// values below (2 + 4 LOGN) q (reduce with reduce_lazy).
template <int LOGN, int LOGE, bool SPLIT = false>
__device__ __forceinline__ void ntt_fwd(uint64_t (&x)[1 << LOGE], uint64_t* lds, const ulonglong2* tw, uint64_t q,
                                        int tid) {
  fwd_passes<LOGN, LOGE, 0, SPLIT>(x, lds, tw, q, 4 * q, tid);
}

// Inverse transform without the n^-1 factor.  In: LastMap order, values < 4q.
// Out: FirstMap order, [0, 4q).
template <int LOGN, int LOGE, bool SPLIT = false>
__device__ __forceinline__ void ntt_inv(uint64_t (&x)[1 << LOGE], uint64_t* lds, const ulonglong2* itw, uint64_t q,
                                        int tid) {
  inv_passes<LOGN, LOGE, NttShape<LOGN, LOGE>::NPASS - 1, SPLIT>(x, lds, itw, q, 4 * q, tid);
}

// Forward transform with natural-order I/O: in and out in FirstMap order
// (lane-consecutive words for every register); same bounds as ntt_fwd.
template <int LOGN, int LOGE>
__device__ __forceinline__ void ntt_fwd_nat(uint64_t (&x)[1 << LOGE], uint64_t* lds, const ulonglong2* tw, uint64_t q,
                                            int tid) {
  fwd_passes<LOGN, LOGE, 0>(x, lds, tw, q, 4 * q, tid);
  exchange<LOGN, LOGE, NttShape<LOGN, LOGE>::LAST_S0, 0>(x, lds, tid);
}

// Inverse transform (no n^-1) with natural-order I/O: in and out in FirstMap
// order, in < 4q, out in [0, 4q).
template <int LOGN, int LOGE>
__device__ __forceinline__ void ntt_inv_nat(uint64_t (&x)[1 << LOGE], uint64_t* lds, const ulonglong2* itw, uint64_t q,
                                            int tid) {
  exchange<LOGN, LOGE, 0, NttShape<LOGN, LOGE>::LAST_S0>(x, lds, tid);
  inv_passes<LOGN, LOGE, NttShape<LOGN, LOGE>::NPASS - 1>(x, lds, itw, q, 4 * q, tid);
}

// Source index of NTT entry i under X -> X^gal: entry i holds a(psi^(2 brv(i)+1)),
// so sigma(a) at i is a at psi^(gal (2 brv(i) + 1)).
template <int LOGN>
__device__ __forceinline__ uint32_t galois_src(uint32_t i, uint32_t gal) {
  const uint32_t mask2n = (2u << LOGN) - 1;
  const uint32_t e = 2u * (__brev(i) >> (32 - LOGN)) + 1u;
  const uint32_t f = (e * gal) & mask2n;
  return __brev((f - 1u) >> 1) >> (32 - LOGN);
}

}  // namespace wally

// HIP kernels of the encrypted scoring path (gfx950).
//
// Ciphertexts are [2][L][n] words in NTT form (entry i of limb l holds the
// polynomial at psi_l^(2 brv(i)+1) mod q_l); Galois keys are [L digits][2][L+1
// moduli][n] with the special prime P last; plaintexts of a cluster chunk are
// [d_pad][L][n].  One workgroup transforms one polynomial (see ntt.h).
//
// Key switching for CtRotate (paper §2.1) follows the hybrid RNS method of
// paper §7.1 with one digit per ciphertext limb and one special prime P:
//   ks_digits : x_i = INTT_{q_i}(sigma(c1)_i)                         (L per item)
//   ks_extend : D[m][i] = NTT_m(x_i mod m), m in {q_0..q_{L-1}, P} \ {q_i}   (L^2 per item)
//   ks_inner  : u_t[m] = sum_i D[m][i] * key[i][t][m]               (elementwise)
//               D[m][m] = sigma(c1)_m read from the input row
//   ks_pinv   : y_t = INTT_P(u_t[P])                                (2 per item)
//   ks_moddown: out_t[j] = (u_t[j] - NTT_j([y_t]_centred mod q_j)) * P^-1
//               (+ sigma(c0)_j for t = 0) (+ acc_i)                (2L per item)
// In the fused form ks_inner covers m = P alone and k_ks_moddown forms the
// u_t[j] of the q_j rows itself; in the stored form ks_inner covers every m
// and k_ks_moddown_u reads them (the host picks per launch).
// Each transform kernel does one NTT per workgroup, with coalesced row I/O
// (lane-consecutive words, or lane-consecutive word pairs where a row is in
// the last pass's order), so the compute-bound transforms stay light on
// registers and the memory-bound inner product runs at full occupancy.  The giant-step sums
// acc_i = sum_j PT[g i + j] * ct'_j (Server Computation algorithm, paper §5)
// are computed for all i by one tiled kernel; a Horner step
// R <- acc_i + Rot(R, g) adds acc_i inside ks_moddown.
//
// Rows that a launch touches once (keys, extended digits, key inner products,
// sigma's source rows, acc_i, the sums' rotated copies) are read and, for the
// extended digits and inner products, written with non-temporal accesses: a
// launch streams hundreds of MB of them, and as ordinary accesses they would
// displace the rows that are re-read from the caches (digits, P parts,
// plaintexts, twiddles).
#include "kernels.h"
#include "ntt.h"

namespace wally {

// Pointers read from descriptors in memory are generic to the compiler, which
// then emits flat loads and stores (also counted by the LDS wait counter, so
// the transforms' LDS waits would wait for them).  They always address device
// global memory, so every access goes through a pointer typed with the global
// address space.
#define WALLY_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ WALLY_GLOBAL T* gmem(T* p) {
  return (WALLY_GLOBAL T*)p;
}
// two words in one 16-byte access (a builtin vector type, usable in any
// address space)
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// The selector is uniform; the chosen field is read straight from the item in
// global memory (a dynamic pick from a register copy of the item would be
// lowered to a stack array in scratch memory).
__device__ __forceinline__ WALLY_GLOBAL const uint64_t* sel_in(const KsItem* it, int sel, uint64_t off) {
  const uint64_t* r;
  switch (sel) {
    case 0: r = it->buf0; break;
    case 1: r = it->buf1; break;
    case 2: r = it->fin; break;
    default: r = it->acc; break;
  }
  return gmem(r) + off;
}
__device__ __forceinline__ WALLY_GLOBAL uint64_t* sel_out(const KsItem* it, int sel, uint64_t off) {
  uint64_t* r;
  switch (sel) {
    case 0: r = it->buf0; break;
    case 1: r = it->buf1; break;
    default: r = it->fin; break;
  }
  return gmem(r) + off;
}

// Rows in LastMap order.  The last pass has LOWB = 0, so registers 2c and
// 2c + 1 of a thread hold adjacent words and lanes hold consecutive pairs:
// a row moves with one coalesced 16-byte access per pair, and a transform
// whose output (forward) or input (inverse) is in this order needs no
// exchange to or from the natural order.  Rows live in global memory (the
// pointer may be generic or global-typed).
template <int LOGN, int LOGE, bool NT = false, class PTR>
__device__ __forceinline__ void load_last(uint64_t (&x)[1 << LOGE], PTR src, int tid) {
  using LM = LastMap<LOGN, LOGE>;
  static_assert(LM::LOWB == 0 && LM::RW >= 1, "pairs of the last pass are adjacent words");
#pragma unroll
  for (int c = 0; c < (1 << LOGE) / 2; ++c) {
    WALLY_GLOBAL const u64x2* p = (WALLY_GLOBAL const u64x2*)(src + LM::idx(tid, 2 * c));
    const u64x2 v = NT ? __builtin_nontemporal_load(p) : *p;
    x[2 * c] = v.x;
    x[2 * c + 1] = v.y;
  }
}

template <int LOGN, int LOGE, bool NT = false, class PTR>
__device__ __forceinline__ void store_last(PTR dst, const uint64_t (&x)[1 << LOGE], int tid) {
  using LM = LastMap<LOGN, LOGE>;
  static_assert(LM::LOWB == 0 && LM::RW >= 1, "pairs of the last pass are adjacent words");
#pragma unroll
  for (int c = 0; c < (1 << LOGE) / 2; ++c)
  {
    WALLY_GLOBAL u64x2* p = (WALLY_GLOBAL u64x2*)(dst + LM::idx(tid, 2 * c));
    if (NT)
      __builtin_nontemporal_store(u64x2{x[2 * c], x[2 * c + 1]}, p);
    else
      *p = u64x2{x[2 * c], x[2 * c + 1]};
  }
}

// x <- sigma_gal(src) in LastMap order, read straight from global memory.
// Entry i of an NTT row holds a(psi^(2 brv(i) + 1)); under X -> X^gal (gal
// odd) the top bits of the source index depend only on the top bits of i,
// so an aligned pair (i, i + 1) comes from an aligned pair (possibly
// swapped), and the 128 consecutive entries a wave holds for one register
// pair come from 8 whole 128-byte lines: the loads use every byte they fetch,
// as a coalesced read does, and need no LDS staging.
template <int LOGN, int LOGE, class PTR>
__device__ __forceinline__ void load_galois_last(uint64_t (&x)[1 << LOGE], PTR src, uint32_t gal, int tid) {
  using LM = LastMap<LOGN, LOGE>;
  static_assert(LM::LOWB == 0 && LM::RW >= 1, "pairs of the last pass are adjacent words");
#pragma unroll
  for (int c = 0; c < (1 << LOGE) / 2; ++c) {
    const uint32_t sidx = galois_src<LOGN>(LM::idx(tid, 2 * c), gal);
    const u64x2 v = __builtin_nontemporal_load((WALLY_GLOBAL const u64x2*)(src + (sidx & ~1u)));
    const bool odd = sidx & 1u;
    x[2 * c] = odd ? v.y : v.x;
    x[2 * c + 1] = odd ? v.x : v.y;
  }
}

// XCD-aware placement. The work-groups of a launch go to the eight XCDs round
// robin (block id mod 8) and each XCD has its own L2. Where a launch has groups
// of `per` blocks that read the same input row, a group's members get ids that
// are congruent mod 8 and consecutive on that XCD, id = 8 (per s + k) + x for
// member k of group 8 s + x, so the row comes from HBM once and from L2 after.
constexpr uint32_t kXcds = 8;
struct GroupSlot {
  uint32_t group, member;
};
__device__ __forceinline__ GroupSlot xcd_group(uint32_t id, uint32_t per) {
  const uint32_t x = id % kXcds, r = id / kXcds;
  return {(r / per) * kXcds + x, r % per};
}
inline uint32_t xcd_blocks(uint32_t groups, uint32_t per) { return (groups + kXcds - 1) / kXcds * kXcds * per; }

// ---------------------------------------------------------------------------
// key switching, step 1: digits.  The extended digit D[i][i] (digit i in its
// own modulus) is sigma(c1)_i itself: it is not stored, the inner product
// reads it from the input row.
// Held at eight waves per SIMD (64 VGPRs, four workgroups per CU; it spills
// two registers).
// grid (items, L); block T
template <int LOGN, int LOGE>
__global__ __launch_bounds__((NttShape<LOGN, LOGE>::T)) __attribute__((amdgpu_waves_per_eu(8))) void k_ks_digits(
    const KsItem* __restrict__ items, KsArgs a, DevModuli M) {
  using S = NttShape<LOGN, LOGE>;
  using FM = FirstMap<LOGN, LOGE>;
  __shared__ uint64_t lds[(S::LDS_WORDS + 1) / 2];  // 32-bit exchanges
  const int tid = threadIdx.x;
  const int b = blockIdx.x, i = blockIdx.y;
  const auto c1 = sel_in(items + b, a.in_sel, a.in_off) + ((uint64_t)a.L + i) * S::N;
  const uint64_t q = M.q[i];
  uint64_t x[S::E];
  load_galois_last<LOGN, LOGE>(x, c1, a.gal, tid);  // sigma(c1)_i, INTT input order
  ntt_inv<LOGN, LOGE, true>(x, lds, M.inv[i], q, tid);
  uint64_t* X = a.X + ((uint64_t)b * a.L + i) * S::N;
#pragma unroll
  for (int e = 0; e < S::E; ++e) X[FM::idx(tid, e)] = csub(shoup(x[e], M.ninv[i], M.ninvp[i], q), q);
}

// ---------------------------------------------------------------------------
// key switching, step 2: extended digits D[m][i] = NTT_m(x_i mod m) for the
// L moduli m != i of Q P (D[i][i] = sigma(c1)_i is read by the inner product
// from the input row).
// 1-D grid of xcd_blocks(items * L, L): group (b, i) reads digit x_i of item
// b, its L members are the target moduli m; block T
template <int LOGN, int LOGE>
__global__ __launch_bounds__((NttShape<LOGN, LOGE>::T)) void k_ks_extend(const KsItem* __restrict__ items, KsArgs a,
                                                                         int n_items, DevModuli M) {
  using S = NttShape<LOGN, LOGE>;
  using FM = FirstMap<LOGN, LOGE>;
  __shared__ uint64_t lds[(S::LDS_WORDS + 1) / 2];  // 32-bit exchanges
  const int tid = threadIdx.x;
  const int L = a.L;
  const GroupSlot gs = xcd_group(blockIdx.x, L);
  if (gs.group >= (uint32_t)(n_items * L)) return;  // padding block (whole block, before any barrier)
  const int b = gs.group / L, i = gs.group % L;
  const int m = (int)gs.member < i ? (int)gs.member : (int)gs.member + 1;  // the moduli of Q P other than q_i
  uint64_t* D = a.D + (((uint64_t)b * (L + 1) + m) * L + i) * S::N;
  uint64_t d[S::E];
  const uint64_t q = M.q[m];
  const uint64_t* X = a.X + ((uint64_t)b * L + i) * S::N;
#pragma unroll
  for (int e = 0; e < S::E; ++e) d[e] = X[FM::idx(tid, e)];  // < q_i < 2 q_m: a valid lazy input
  ntt_fwd<LOGN, LOGE, true>(d, lds, M.fwd[m], q, tid);  // out < 54 q, LastMap order
  // stored unreduced: the inner product's 128-bit sums take words below 54 q
  // (up to eight products of them with key words stay below 2^117) and
  // reduce once
  store_last<LOGN, LOGE, true>(D, d, tid);
}

// ---------------------------------------------------------------------------
// key switching, step 3: key inner product u_t[m] = sum_i D[m][i] * key[i][t][m]
// for the rows m = m0 .. L, with one 128-bit lazy sum per output word
// (elementwise, memory bound; two words per thread through 16-byte loads).
// D words are below 54 q (the forward transform's lazy bound), key words
// below q.  D[m][m] (m < L) is sigma(c1)_m, read from the input row as
// load_galois_last does: the aligned pair of words a thread takes comes from
// an aligned pair there.  m0 = L (the P rows alone) when k_ks_moddown forms
// the others, m0 = 0 when k_ks_moddown_u reads them.
// grid (n / 512, L + 1 - m0, items); block 256
template <int L>
__global__ __launch_bounds__(256) void k_ks_inner(const KsItem* __restrict__ items, KsArgs a, int m0, DevModuli M) {
  constexpr int MM = L + 1;
  const int m = m0 + blockIdx.y, b = blockIdx.z;
  const uint64_t n = 1ull << a.log_n;
  const uint64_t p = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * 2;
  WALLY_GLOBAL const uint64_t* key = a.key_fold ? gmem(items[b].key_fold) + a.key_off : gmem(items[b].key);
  const uint64_t* D = a.D + ((uint64_t)b * MM + m) * L * n + p;
  const ModConst mc = M.mc[m];
  // source of sigma(c1)_m at p (and p + 1): entry p holds a(psi^(2 brv(p) + 1))
  const uint32_t mask2n = (2u << a.log_n) - 1;
  const uint32_t ep = 2u * (__brev((uint32_t)p) >> (32 - a.log_n)) + 1u;
  const uint32_t sidx = __brev((((ep * a.gal) & mask2n) - 1u) >> 1) >> (32 - a.log_n);
  // all 3L loads of a thread are issued before the first product (L is a
  // compile-time constant), so each thread keeps 48 L bytes in flight
  u64x2 d[L], k0[L], k1[L];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    if (i == m) {
      const u64x2 v = __builtin_nontemporal_load(
          (WALLY_GLOBAL const u64x2*)(sel_in(items + b, a.in_sel, a.in_off) + ((uint64_t)L + m) * n + (sidx & ~1u)));
      d[i] = (sidx & 1u) ? u64x2{v.y, v.x} : v;
    } else {
      d[i] = __builtin_nontemporal_load((WALLY_GLOBAL const u64x2*)(D + (uint64_t)i * n));
    }
    k0[i] = __builtin_nontemporal_load((WALLY_GLOBAL const u64x2*)(key + (((uint64_t)i * 2 + 0) * MM + m) * n + p));
    k1[i] = __builtin_nontemporal_load((WALLY_GLOBAL const u64x2*)(key + (((uint64_t)i * 2 + 1) * MM + m) * n + p));
  }
  u128w a00{0, 0}, a01{0, 0}, a10{0, 0}, a11{0, 0};  // [t][word]
#pragma unroll
  for (int i = 0; i < L; ++i) {
    mac128(a00, d[i].x, k0[i].x);
    mac128(a01, d[i].y, k0[i].y);
    mac128(a10, d[i].x, k1[i].x);
    mac128(a11, d[i].y, k1[i].y);
  }
  uint64_t* U = a.U + ((uint64_t)b * 2 * MM + m) * n + p;  // U[b][t][m], m = L is the P part
  __builtin_nontemporal_store(u64x2{reduce128(a00, mc.q, mc.r64, mc.r64p, mc.onep), reduce128(a01, mc.q, mc.r64, mc.r64p, mc.onep)},
                              (WALLY_GLOBAL u64x2*)U);
  __builtin_nontemporal_store(u64x2{reduce128(a10, mc.q, mc.r64, mc.r64p, mc.onep), reduce128(a11, mc.q, mc.r64, mc.r64p, mc.onep)},
                              (WALLY_GLOBAL u64x2*)(U + (uint64_t)MM * n));
}

// ---------------------------------------------------------------------------
// key switching, step 4: y_t = INTT_P(u_t[P]), kept in [0, P) (centred by
// the consumer).  grid (items, 2); block T
template <int LOGN, int LOGE>
__global__ __launch_bounds__((NttShape<LOGN, LOGE>::T)) void k_ks_pinv(KsArgs a, DevModuli M) {
  using S = NttShape<LOGN, LOGE>;
  using FM = FirstMap<LOGN, LOGE>;
  __shared__ uint64_t lds[(S::LDS_WORDS + 1) / 2];  // 32-bit exchanges
  const int tid = threadIdx.x;
  const int b = blockIdx.x, t = blockIdx.y;
  const int L = a.L, MM = a.L + 1;
  const uint64_t P = M.q[L];
  const uint64_t* U = a.U + (((uint64_t)b * 2 + t) * MM + L) * S::N;
  uint64_t y[S::E];
  load_last<LOGN, LOGE, true>(y, U, tid);
  ntt_inv<LOGN, LOGE, true>(y, lds, M.inv[L], P, tid);  // out FirstMap order
  uint64_t* Y = a.Y + ((uint64_t)b * 2 + t) * S::N;
#pragma unroll
  for (int e = 0; e < S::E; ++e) Y[FM::idx(tid, e)] = csub(shoup(y[e], M.ninv[L], M.ninvp[L], P), P);
}

// ---------------------------------------------------------------------------
// key switching, step 5: division by P and the rest of CtRotate:
//   out_t[j] = (u_t[j] - NTT_j([y_t]_centred mod q_j)) * P^-1
//              (+ sigma(c0)_j for t = 0) (+ acc_i in a Horner step)
// Two kernels share the transform and the additions: k_ks_moddown forms the
// key inner products u_t[j] itself, k_ks_moddown_u reads them from U (where
// the inner-product kernel wrote every row); the host picks by launch size.

// z = NTT_j([Y_t]_centred mod q_j), LastMap order, below (2 + 4 LOGN) q_j
template <int LOGN, int LOGE>
__device__ __forceinline__ void moddown_transform(uint64_t (&z)[1 << LOGE], uint64_t* lds, const KsArgs& a, const DevModuli& M,
                                                  int b, int t, int j, int tid) {
  using S = NttShape<LOGN, LOGE>;
  using FM = FirstMap<LOGN, LOGE>;
  const uint64_t q = M.q[j];
  const uint64_t P = M.q[a.L];
  const uint64_t halfP = (P - 1) / 2;
  const uint64_t* Y = a.Y + ((uint64_t)b * 2 + t) * S::N;
#pragma unroll
  for (int e = 0; e < S::E; ++e) {
    const uint64_t y = Y[FM::idx(tid, e)];
    z[e] = y > halfP ? y + (q - P) : y;  // centred lift, then mod q_j (P < q_j)
  }
  ntt_fwd<LOGN, LOGE, true>(z, lds, M.fwd[j], q, tid);
}

// z = (u + zb - z) P^-1 mod q_j for one pair of words: u - z taken as
// u + zb - z with zb the transform's output bound (below 2^60, which the
// Shoup product by P^-1 accepts unreduced)
template <int LOGN>
__device__ __forceinline__ void moddown_div(uint64_t& z0, uint64_t& z1, uint64_t u0, uint64_t u1, const DevModuli& M,
                                            int j) {
  const uint64_t q = M.q[j];
  const uint64_t zb = (2 + 4 * LOGN) * q;
  z0 = csub(shoup(u0 + zb - z0, M.pinv[j], M.pinvp[j], q), q);
  z1 = csub(shoup(u1 + zb - z1, M.pinv[j], M.pinvp[j], q), q);
}

// + sigma(c0)_j (t = 0), + the input itself (fold step), + acc_i (Horner
// step), then the store of out_t[j]
template <int LOGN, int LOGE>
__device__ __forceinline__ void moddown_finish(uint64_t (&z)[1 << LOGE], const KsItem* __restrict__ items, const KsArgs& a,
                                               int b, int t, int j, uint64_t q, int tid) {
  using S = NttShape<LOGN, LOGE>;
  using LM = LastMap<LOGN, LOGE>;
  const int L = a.L;
  if (t == 0) {  // + sigma(c0)_j
    uint64_t v[S::E];
    load_galois_last<LOGN, LOGE>(v, sel_in(items + b, a.in_sel, a.in_off) + (uint64_t)j * S::N, a.gal, tid);
#pragma unroll
    for (int e = 0; e < S::E; ++e) z[e] = addmod(z[e], v[e], q);
  }
  const uint64_t toff = ((uint64_t)t * L + j) * S::N;
  if (a.add_in) {  // fold step: + the input itself, unpermuted (R + Rot(R))
    WALLY_GLOBAL const uint64_t* r = sel_in(items + b, a.in_sel, a.in_off) + toff;
#pragma unroll
    for (int c = 0; c < S::E / 2; ++c) {
      const u64x2 v = *(WALLY_GLOBAL const u64x2*)(r + LM::idx(tid, 2 * c));
      z[2 * c] = addmod(z[2 * c], v.x, q);
      z[2 * c + 1] = addmod(z[2 * c + 1], v.y, q);
    }
  }
  if (a.giant >= 0) {  // Horner step: + acc_i
    WALLY_GLOBAL const uint64_t* acc = gmem(items[b].acc) + (uint64_t)a.giant * 2 * L * S::N + toff;
#pragma unroll
    for (int c = 0; c < S::E / 2; ++c) {
      const u64x2 v = __builtin_nontemporal_load((WALLY_GLOBAL const u64x2*)(acc + LM::idx(tid, 2 * c)));
      z[2 * c] = addmod(z[2 * c], v.x, q);
      z[2 * c + 1] = addmod(z[2 * c + 1], v.y, q);
    }
  }
  store_last<LOGN, LOGE>(sel_out(items + b, a.out_sel, a.out_off) + toff, z, tid);
}

// The key inner product u_t[j] = sum_i D[j][i] * key[i][t][j] is formed here,
// one pair of words at a time with 128-bit lazy sums (D[j][j] = sigma(c1)_j
// straight from the input row), so that it is neither stored nor read back.
// Uncapped, the kernel takes 128 VGPRs (two workgroups per CU); held lower it
// spills.
// 1-D grid of xcd_blocks(items, 2 L): group b is item b; its 2 L members
// (j, t) are consecutive on one XCD, so the two parts of limb j read D[j][*]
// and the members of part t read Y_t from that XCD's L2; block T
template <int LOGN, int LOGE>
__global__ __launch_bounds__((NttShape<LOGN, LOGE>::T)) void k_ks_moddown(
    const KsItem* __restrict__ items, KsArgs a, int n_items, DevModuli M) {
  using S = NttShape<LOGN, LOGE>;
  using LM = LastMap<LOGN, LOGE>;
  __shared__ uint64_t lds[(S::LDS_WORDS + 1) / 2];  // 32-bit exchanges
  const int tid = threadIdx.x;
  const int L = a.L, MM = a.L + 1;
  const GroupSlot gs = xcd_group(blockIdx.x, 2 * L);
  if (gs.group >= (uint32_t)n_items) return;  // padding block (whole block, before any barrier)
  const int b = gs.group, t = gs.member & 1, j = gs.member >> 1;
  uint64_t z[S::E];
  moddown_transform<LOGN, LOGE>(z, lds, a, M, b, t, j, tid);
  // u_t[j] = sum_i D[j][i] key[i][t][j], D[j][j] = sigma(c1)_j from the input row
  WALLY_GLOBAL const uint64_t* key = a.key_fold ? gmem(items[b].key_fold) + a.key_off : gmem(items[b].key);
  const uint64_t* Dj = a.D + ((uint64_t)b * MM + j) * L * S::N;
  WALLY_GLOBAL const uint64_t* c1j = sel_in(items + b, a.in_sel, a.in_off) + ((uint64_t)L + j) * S::N;
  const ModConst mc = M.mc[j];
#pragma unroll
  for (int c = 0; c < S::E / 2; ++c) {
    const uint32_t p = LM::idx(tid, 2 * c);
    u128w s0{0, 0}, s1{0, 0};
#pragma unroll 1
    for (int i = 0; i < L; ++i) {
      u64x2 d;
      if (i == j) {
        const uint32_t sidx = galois_src<LOGN>(p, a.gal);
        const u64x2 v = __builtin_nontemporal_load((WALLY_GLOBAL const u64x2*)(c1j + (sidx & ~1u)));
        d = (sidx & 1u) ? u64x2{v.y, v.x} : v;
      } else {
        d = *(WALLY_GLOBAL const u64x2*)(Dj + (uint64_t)i * S::N + p);
      }
      const u64x2 k = __builtin_nontemporal_load((WALLY_GLOBAL const u64x2*)(key + (((uint64_t)i * 2 + t) * MM + j) * S::N + p));
      mac128(s0, d.x, k.x);
      mac128(s1, d.y, k.y);
    }
    moddown_div<LOGN>(z[2 * c], z[2 * c + 1], reduce128(s0, mc.q, mc.r64, mc.r64p, mc.onep),
                      reduce128(s1, mc.q, mc.r64, mc.r64p, mc.onep), M, j);
  }
  moddown_finish<LOGN, LOGE>(z, items, a, b, t, j, M.q[j], tid);
}

// The same with u_t[j] read from U (the inner-product kernel wrote every
// row): for launches of few items, where the inner products spread over many
// small workgroups and this kernel, at 68 VGPRs, holds three workgroups per
// CU.
// 1-D grid of xcd_blocks(items * 2, L): group (b, t) reads Y_t of item b, its
// L members are the target limbs j; block T
template <int LOGN, int LOGE>
__global__ __launch_bounds__((NttShape<LOGN, LOGE>::T)) __attribute__((amdgpu_waves_per_eu(6))) void k_ks_moddown_u(
    const KsItem* __restrict__ items, KsArgs a, int n_items, DevModuli M) {
  using S = NttShape<LOGN, LOGE>;
  using LM = LastMap<LOGN, LOGE>;
  __shared__ uint64_t lds[(S::LDS_WORDS + 1) / 2];  // 32-bit exchanges
  const int tid = threadIdx.x;
  const int L = a.L, MM = a.L + 1;
  const GroupSlot gs = xcd_group(blockIdx.x, L);
  if (gs.group >= (uint32_t)(n_items * 2)) return;  // padding block (whole block, before any barrier)
  const int b = gs.group >> 1, t = gs.group & 1, j = gs.member;
  uint64_t z[S::E];
  moddown_transform<LOGN, LOGE>(z, lds, a, M, b, t, j, tid);
  const uint64_t* U = a.U + (((uint64_t)b * 2 + t) * MM + j) * S::N;
#pragma unroll
  for (int c = 0; c < S::E / 2; ++c) {
    const u64x2 u = __builtin_nontemporal_load((WALLY_GLOBAL const u64x2*)(U + LM::idx(tid, 2 * c)));
    moddown_div<LOGN>(z[2 * c], z[2 * c + 1], u.x, u.y, M, j);
  }
  moddown_finish<LOGN, LOGE>(z, items, a, b, t, j, M.q[j], tid);
}

// ---------------------------------------------------------------------------
// giant-step sums (Server Computation algorithm, paper §5: for each giant
// step i, the g products of a plaintext with a rotated query copy, summed):
//   acc_i[t][l][x] = sum_{j<g} PT[g i + j][l][x] * ct'_j[t][l][x]  for all i < h.
// Per coefficient this is a (queries x g) by (g x h) product over Z_q; the
// items of a tile share one plaintext chunk, so PT is read once per tile while
// each item's g rotated copies are read once into registers.
// Exact lazy accumulation: both factors (< 2^54) are split into 27-bit halves,
// a = a1 2^27 + a0, so a*b = a0 b0 + (a0 b1 + a1 b0) 2^27 + a1 b1 2^54 and the
// three partial sums of g <= 32 products stay below 2^60 in 64-bit words (one
// v_mad_u64_u32 per partial product, no carries); they are reduced once.
__device__ __forceinline__ uint64_t fold27(uint64_t s0, uint64_t s1, uint64_t s2, const ModConst& mc,
                                           uint64_t c27, uint64_t c27p) {
  const uint64_t q = mc.q;
  // ((s2 2^27 mod q) + s1) 2^27 + s0  (mod q); each Shoup result is below 2q
  const uint64_t u = shoup(s2, c27, c27p, q) + s1;        // < 2q + 2^60
  const uint64_t v = shoup(u, c27, c27p, q) + s0;         // < 2q + 2^59
  return csub(v - mulhi64(v, mc.onep) * q, q);            // v mod q
}

// grid (n / 64, L, tiles); block 256 = 64 coefficients x 4 thread rows.  TP
// ciphertext parts per thread: with TP = 2 a thread keeps both parts of one
// item's g rotated copies in registers (4g 27-bit halves) and each plaintext
// word it loads feeds two products, so the loads (served by L1/L2: every item
// of the tile streams the same plaintext) are halved; the 4 rows take 4 items
// at a time.  With TP = 1 (g = 32, where both parts would not fit in
// registers) the rows are 2 parts x 2 items.
template <int G, int TP>
__global__ __launch_bounds__(256) void k_mac_tiles(const KsItem* __restrict__ items, const MacTile* __restrict__ tiles,
                                                   KsArgs a, int h, DevModuli M) {
  static_assert(TP == 1 || TP == 2, "one or both ciphertext parts per thread");
  constexpr int LANES = TP == 2 ? 4 : 2;  // items in flight per block
  const MacTile tl = tiles[blockIdx.z];
  const int j = blockIdx.y;
  const int L = a.L;
  const uint64_t n = 1ull << a.log_n;
  const uint64_t x = (uint64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int row = threadIdx.x >> 6;
  const int t0 = TP == 2 ? 0 : (row & 1);
  const int lane = TP == 2 ? row : (row >> 1);
  const ModConst mc = M.mc[j];
  const uint64_t c27 = M.c27[j], c27p = M.c27p[j];
  const uint64_t ctw = 2ull * L * n;
  WALLY_GLOBAL const uint64_t* pt = gmem(items[tl.first].pt) + (uint64_t)j * n + x;  // PT[m][j][x] at m * L * n
  const uint64_t M27 = (1ull << 27) - 1;
  for (uint32_t k = lane; k < tl.count; k += LANES) {
    const KsItem& it = items[tl.first + k];
    uint32_t cl[TP][G], ch[TP][G];
#pragma unroll
    for (int p = 0; p < TP; ++p) {
      WALLY_GLOBAL const uint64_t* ctp = gmem(it.ctp) + ((uint64_t)(t0 + p) * L + j) * n + x;
#pragma unroll
      for (int jj = 0; jj < G; ++jj) {
        const uint64_t v = __builtin_nontemporal_load(&ctp[jj * ctw]);
        cl[p][jj] = (uint32_t)(v & M27);
        ch[p][jj] = (uint32_t)(v >> 27);
      }
    }
    WALLY_GLOBAL uint64_t* acc = gmem(it.acc) + ((uint64_t)t0 * L + j) * n + x;
    for (int i = 0; i < h; ++i) {
      uint64_t s0[TP], s1[TP], s2[TP];
#pragma unroll
      for (int p = 0; p < TP; ++p) s0[p] = s1[p] = s2[p] = 0;
#pragma unroll
      for (int jj = 0; jj < G; ++jj) {
        const uint64_t w = pt[(uint64_t)(G * i + jj) * L * n];
        const uint32_t wl = (uint32_t)(w & M27), wh = (uint32_t)(w >> 27);
#pragma unroll
        for (int p = 0; p < TP; ++p) {
          s0[p] += (uint64_t)wl * cl[p][jj];
          s1[p] += (uint64_t)wl * ch[p][jj] + (uint64_t)wh * cl[p][jj];
          s2[p] += (uint64_t)wh * ch[p][jj];
        }
      }
#pragma unroll
      for (int p = 0; p < TP; ++p) acc[(uint64_t)i * ctw + (uint64_t)p * L * n] = fold27(s0[p], s1[p], s2[p], mc, c27, c27p);
    }
  }
}

// copy each item's source ciphertext into slot 0 of its rotated-copies buffer
// grid (items); block 256
__global__ __launch_bounds__(256) void k_copy_ct(const CopyItem* __restrict__ items, uint64_t words) {
  const CopyItem it = items[blockIdx.x];
  WALLY_GLOBAL const u64x2* src = (WALLY_GLOBAL const u64x2*)gmem(it.src);
  WALLY_GLOBAL u64x2* dst = (WALLY_GLOBAL u64x2*)gmem(it.dst);
  for (uint64_t k = threadIdx.x; k < words / 2; k += blockDim.x) dst[k] = src[k];
}

// ---------------------------------------------------------------------------
// cluster encoding (Server Initialization algorithm, paper §5; diagonal
// packing, paper §4.1).  One workgroup makes plaintext m of one chunk:
//   slot s of the chunk belongs to entry base + s; diagonal m holds coordinate
//   ((s mod d_pad) + m) mod d_pad of that entry (0 past the cluster or past d);
//   plaintext g*i + j is that diagonal rotated right by g*i within each row;
//   with a fold factor B (folded layout, not in the paper) the chunk has
//   D = d_pad / B diagonals and slot s = W d_pad + u (window W, u < d_pad)
//   belongs to entry W D + (u mod D), so an entry spreads its coordinates
//   over B slots (B = 1 is the paper's layout);
//   slots -> polynomial mod t (inverse NTT mod t after placing slot s at the
//   NTT index holding it); centred lift; NTT in every ciphertext limb.
// grid (jobs, d_pad); block T
template <int LOGN>
__global__ __launch_bounds__((NttShape<LOGN, 4>::T)) void k_encode(const EncodeJob* __restrict__ jobs, EncodeArgs a,
                                                                 DevModuli M) {
  using S = NttShape<LOGN, 4>;
  __shared__ uint64_t lds[S::LDS_WORDS];
  const int tid = threadIdx.x;
  const EncodeJob jb = jobs[blockIdx.x];
  const uint32_t m = blockIdx.y;
  const uint32_t half = S::N / 2;
  const uint32_t dp = a.d_pad, d = a.d;
  const uint32_t nd = a.d_pad / jb.fold;  // diagonals of this chunk
  if (m >= nd) return;                     // whole block, before any barrier
  const uint32_t rot = (jb.g * (m / jb.g)) % half;
  const int it = a.L + 1;  // index of t in the modulus tables
  const uint64_t t = M.q[it];
  uint64_t x[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const uint32_t pos = LastMap<LOGN, 4>::idx(tid, e);
    const uint32_t s = a.slot_of[pos];  // slot whose value sits at NTT index pos
    const uint32_t row = s / half, c = s % half;
    const uint32_t s2 = row * half + (c + half - rot) % half;  // pre-rotation (right by g*i)
    const uint32_t u = s2 % dp;
    const uint64_t entry = (uint64_t)(s2 / dp) * nd + u % nd;
    const uint32_t coord = (u + m) % dp;
    int v = 0;
    if (entry < jb.n_entries && coord < d)
      v = a.wide ? gmem((const int16_t*)jb.emb)[entry * d + coord] : gmem((const int8_t*)jb.emb)[entry * d + coord];
    x[e] = v < 0 ? (uint64_t)((int64_t)t + v) : (uint64_t)v;
  }
  ntt_inv<LOGN, 4>(x, lds, M.inv[it], t, tid);
  int64_t cc[16];
  const uint64_t halft = (t - 1) / 2;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const uint64_t v = csub(shoup(x[e], M.ninv[it], M.ninvp[it], t), t);
    cc[e] = v > halft ? (int64_t)v - (int64_t)t : (int64_t)v;
  }
  for (int l = 0; l < a.L; ++l) {
    const uint64_t q = M.q[l];
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = cc[e] < 0 ? (uint64_t)((int64_t)q + cc[e]) : (uint64_t)cc[e];
    ntt_fwd_nat<LOGN, 4>(x, lds, M.fwd[l], q, tid);
    WALLY_GLOBAL uint64_t* out = gmem(jb.out) + ((uint64_t)m * a.L + l) * S::N;
#pragma unroll
    for (int e = 0; e < 16; ++e) out[FirstMap<LOGN, 4>::idx(tid, e)] = reduce_lazy(x[e], q, M.mc[l].onep);
  }
}

// ---------------------------------------------------------------------------
// Index PIR (paper §4.2, MulPIR).  Coefficient-encoded plaintexts: values in
// [0, t) lifted centred to each limb, then put in NTT form.  grid (plaintexts, L)
template <int LOGN>
__global__ __launch_bounds__((NttShape<LOGN, 4>::T)) void k_pir_encode(const uint32_t* __restrict__ coeffs,
                                                                     uint64_t* __restrict__ out, int L, DevModuli M) {
  using S = NttShape<LOGN, 4>;
  __shared__ uint64_t lds[S::LDS_WORDS];
  const int tid = threadIdx.x;
  const uint64_t p = blockIdx.x;
  const int l = blockIdx.y;
  const uint64_t q = M.q[l], t = M.q[L + 1];
  const uint64_t halft = (t - 1) / 2;
  WALLY_GLOBAL const uint32_t* src = gmem(coeffs) + p * S::N;
  uint64_t x[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const uint64_t v = src[FirstMap<LOGN, 4>::idx(tid, e)];
    x[e] = v > halft ? v + (q - t) : v;  // centred lift (t < q)
  }
  ntt_fwd_nat<LOGN, 4>(x, lds, M.fwd[l], q, tid);
  WALLY_GLOBAL uint64_t* dst = gmem(out) + (p * L + l) * S::N;
#pragma unroll
  for (int e = 0; e < 16; ++e) dst[FirstMap<LOGN, 4>::idx(tid, e)] = reduce_lazy(x[e], q, M.mc[l].onep);
}

// one expansion level after its substitutions: grid (n / 256, 2 L, items); block 256
__global__ __launch_bounds__(256) void k_pir_split(PirSplitArgs a, DevModuli M) {
  const uint64_t n = 1ull << a.log_n;
  const uint32_t i = blockIdx.z;
  const uint32_t qi = i / a.half, b = i % a.half;
  const int tl = blockIdx.y, l = tl % a.L;
  const uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t ctw = 2ull * a.L * n;
  const uint64_t off = (uint64_t)tl * n + x;
  const uint64_t q = M.q[l];
  const uint64_t base = (uint64_t)qi * a.stride + b;
  if (a.e3 != nullptr) {  // linearised last level: its linearised pairs are k_pir_lin_split's
    if (!((b >= a.col_lo && b < a.col_hi) || (b + a.half >= a.col_lo && b + a.half < a.col_hi))) return;
    if (tl >= a.L) {  // the other pairs get no third part
      WALLY_GLOBAL uint64_t* e3 = gmem(a.e3) + (base * a.L + l) * n + x;
      e3[0] = 0;
      e3[(uint64_t)a.half * a.L * n] = 0;
    }
  }
  const uint64_t xv = gmem(a.cur)[base * ctw + off];
  const uint64_t yv = gmem(a.ybuf)[((uint64_t)qi * a.ystride + b) * ctw + off];
  const u64x2 w = *((WALLY_GLOBAL const u64x2*)a.w + (uint64_t)l * n + x);  // (value, Shoup factor)
  gmem(a.next)[base * ctw + off] = addmod(xv, yv, q);
  gmem(a.next)[(base + a.half) * ctw + off] = csub(shoup(xv + q - yv, w.x, w.y, q), q);
}

// The linearised pairs of the last expansion level (PirSplitArgs): the
// automorphism z = x(X^g) without key switching, which in NTT form permutes
// the entries of every row the same way, and the pair's outputs
//   b: (x0 + z0, x1 | z1),  b + half: ((x0 - z0) w, x1 w | -z1 w).
// A row of x is read with coalesced loads into LDS; z's words come from
// their source entries there.  Item fields: buf0 = x, buf1 = output b in
// the next list, fin = its third part (output b + half is half ciphertexts,
// half third parts further on).  grid (2 L, items); block 256
template <int LOGN>
__global__ __launch_bounds__(256) void k_pir_lin_split(const KsItem* __restrict__ items, PirSplitArgs a, uint32_t gal,
                                                       DevModuli M) {
  constexpr int N = 1 << LOGN;
  __shared__ uint64_t lds[N];
  const int tl = blockIdx.x, l = tl % a.L;
  const uint64_t q = M.q[l];
  const KsItem it = items[blockIdx.y];
  WALLY_GLOBAL const uint64_t* src = gmem(it.buf0) + (uint64_t)tl * N;
  for (int k = threadIdx.x; k < N; k += 256) lds[k] = src[k];
  __syncthreads();
  const uint64_t ctw = 2ull * a.L * N;
  WALLY_GLOBAL uint64_t* nb = gmem(it.buf1) + (uint64_t)tl * N;
  WALLY_GLOBAL uint64_t* nh = nb + (uint64_t)a.half * ctw;
  WALLY_GLOBAL const u64x2* w = (WALLY_GLOBAL const u64x2*)a.w + (uint64_t)l * N;  // (value, Shoup factor)
  if (tl < a.L) {
    for (int k = threadIdx.x; k < N; k += 256) {
      const uint64_t xv = lds[k], zv = lds[galois_src<LOGN>((uint32_t)k, gal)];
      const u64x2 wk = w[k];
      nb[k] = addmod(xv, zv, q);
      nh[k] = csub(shoup(xv + q - zv, wk.x, wk.y, q), q);
    }
  } else {
    WALLY_GLOBAL uint64_t* eb = gmem(it.fin) + (uint64_t)l * N;
    WALLY_GLOBAL uint64_t* eh = eb + (uint64_t)a.half * a.L * N;
    for (int k = threadIdx.x; k < N; k += 256) {
      const uint64_t xv = lds[k], zv = lds[galois_src<LOGN>((uint32_t)k, gal)];
      const u64x2 wk = w[k];
      nb[k] = xv;
      eb[k] = zv;
      nh[k] = csub(shoup(xv, wk.x, wk.y, q), q);
      eh[k] = csub(shoup(q - zv, wk.x, wk.y, q), q);
    }
  }
}

// first dimension: grid (n / 512, L, column pairs x query pairs); block 256.
// A thread takes two adjacent coefficients (16-byte loads) of two columns and
// two queries, all TP ciphertext parts: per row r it loads 2 plaintext pairs
// and 2 TP ciphertext pairs and does 8 TP products into 128-bit lazy sums
// (d1 <= 2048 products of words below 2^54 stay below 2^119), reduced once at
// the end.  TP = 3 for a linearised expansion (the third parts from E3).
template <int TP>
__global__ __launch_bounds__(256) void k_pir_dot(PirDotArgs a, DevModuli M) {
  const uint64_t n = 1ull << a.log_n;
  const uint64_t x = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * 2;
  const int l = blockIdx.y;
  const uint32_t kpairs = (a.d2 + 1) / 2;
  const uint32_t k0 = (blockIdx.z % kpairs) * 2, q0 = (blockIdx.z / kpairs) * 2;
  const bool k1v = k0 + 1 < a.d2, q1v = q0 + 1 < a.nq;
  const ModConst mc = M.mc[l];
  const uint64_t ctw = 2ull * a.L * n, ptw = (uint64_t)a.L * n;
  WALLY_GLOBAL const uint64_t* pt0 = gmem(a.pt) + (uint64_t)k0 * a.d1 * ptw + (uint64_t)l * n + x;
  WALLY_GLOBAL const uint64_t* pt1 = pt0 + (k1v ? (uint64_t)a.d1 * ptw : 0);
  WALLY_GLOBAL const uint64_t* e0 = gmem(a.E) + (uint64_t)q0 * a.stride * ctw + (uint64_t)l * n + x;
  WALLY_GLOBAL const uint64_t* e1 = e0 + (q1v ? (uint64_t)a.stride * ctw : 0);
  WALLY_GLOBAL const uint64_t* f0 = nullptr;
  WALLY_GLOBAL const uint64_t* f1 = nullptr;
  if constexpr (TP == 3) {
    f0 = gmem(a.E3) + (uint64_t)q0 * a.stride * ptw + (uint64_t)l * n + x;
    f1 = f0 + (q1v ? (uint64_t)a.stride * ptw : 0);
  }
  u128w acc[2][2][TP][2] = {};  // [column][query][part][coefficient]
  for (uint32_t r = 0; r < a.d1; ++r) {
    const u64x2 w[2] = {*(WALLY_GLOBAL const u64x2*)(pt0 + (uint64_t)r * ptw),
                        *(WALLY_GLOBAL const u64x2*)(pt1 + (uint64_t)r * ptw)};
    u64x2 v[2][TP];
#pragma unroll
    for (int tp = 0; tp < 2; ++tp) {
      v[0][tp] = *(WALLY_GLOBAL const u64x2*)(e0 + (uint64_t)r * ctw + (uint64_t)tp * ptw);
      v[1][tp] = *(WALLY_GLOBAL const u64x2*)(e1 + (uint64_t)r * ctw + (uint64_t)tp * ptw);
    }
    if constexpr (TP == 3) {
      v[0][2] = *(WALLY_GLOBAL const u64x2*)(f0 + (uint64_t)r * ptw);
      v[1][2] = *(WALLY_GLOBAL const u64x2*)(f1 + (uint64_t)r * ptw);
    }
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int qq = 0; qq < 2; ++qq)
#pragma unroll
        for (int tp = 0; tp < TP; ++tp) {
          mac128(acc[kk][qq][tp][0], w[kk].x, v[qq][tp].x);
          mac128(acc[kk][qq][tp][1], w[kk].y, v[qq][tp].y);
        }
  }
  // column layout: [U0][U1] (TP = 2), [U0][U2][0][U1] (TP = 3)
  constexpr int kSlot[3] = {0, TP == 3 ? 3 : 1, 1};
  const uint64_t colw = TP == 3 ? 4 * ptw : ctw;
#pragma unroll
  for (int kk = 0; kk < 2; ++kk)
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {
      if ((kk && !k1v) || (qq && !q1v)) continue;
      WALLY_GLOBAL uint64_t* o = gmem(a.out[q0 + qq]) + (uint64_t)(k0 + kk) * colw + (uint64_t)l * n + x;
#pragma unroll
      for (int tp = 0; tp < TP; ++tp)
        *(WALLY_GLOBAL u64x2*)(o + (uint64_t)kSlot[tp] * ptw) =
            u64x2{reduce128(acc[kk][qq][tp][0], mc.q, mc.r64, mc.r64p, mc.onep),
                  reduce128(acc[kk][qq][tp][1], mc.q, mc.r64, mc.r64p, mc.onep)};
      if constexpr (TP == 3) *(WALLY_GLOBAL u64x2*)(o + 2 * ptw) = u64x2{0, 0};
    }
}

// ---------------------------------------------------------------------------
// diagnostics: in-place NTT / INTT of rows (canonical order) mod modulus `mi`
template <int LOGN>
__global__ __launch_bounds__((NttShape<LOGN, 4>::T)) void k_ntt_rows(uint64_t* data, int mi, int inverse, DevModuli M) {
  using S = NttShape<LOGN, 4>;
  __shared__ uint64_t lds[S::LDS_WORDS];
  const int tid = threadIdx.x;
  uint64_t* row = data + (uint64_t)blockIdx.x * S::N;
  const uint64_t q = M.q[mi];
  uint64_t x[16];
  if (!inverse) {
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = row[FirstMap<LOGN, 4>::idx(tid, e)];
    ntt_fwd_nat<LOGN, 4>(x, lds, M.fwd[mi], q, tid);
#pragma unroll
    for (int e = 0; e < 16; ++e) row[FirstMap<LOGN, 4>::idx(tid, e)] = reduce_lazy(x[e], q, M.mc[mi].onep);
  } else {
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = row[FirstMap<LOGN, 4>::idx(tid, e)];
    ntt_inv_nat<LOGN, 4>(x, lds, M.inv[mi], q, tid);
#pragma unroll
    for (int e = 0; e < 16; ++e) row[FirstMap<LOGN, 4>::idx(tid, e)] = csub(shoup(x[e], M.ninv[mi], M.ninvp[mi], q), q);
  }
}

// ---------------------------------------------------------------------------
// Index PIR, second dimension (paper §4.2, step 3): the sum over columns k of
// the BFV products of column k with the second indicator entry d1 + k, the
// tensor products summed as integers in the extended basis and scaled once
// (§7.1), then relinearized by the key-switching kernels.

// acc (kMaxConvWords words) += y * m (m zero padded to kMaxConvWords words)
__device__ __forceinline__ void mw_mac_full(uint64_t (&acc)[kMaxConvWords], uint64_t y, const uint64_t* m) {
  uint64_t carry = 0;
#pragma unroll
  for (int w = 0; w < kMaxConvWords; ++w) {
    const uint64_t mw = m[w];
    const uint64_t lo = y * mw, hi = __umul64hi(y, mw);
    uint64_t s = acc[w] + lo;
    uint64_t c = s < lo;
    s += carry;
    c += s < carry;
    acc[w] = s;
    carry = hi + c;
  }
}

// acc >= m (multi-word)
__device__ __forceinline__ bool mw_geq(const uint64_t (&acc)[kMaxConvWords], const uint64_t* m) {
  bool gt = false, lt = false;
#pragma unroll
  for (int w = kMaxConvWords - 1; w >= 0; --w) {
    const uint64_t mw = m[w];
    const bool undecided = !gt && !lt;
    gt = gt || (undecided && acc[w] > mw);
    lt = lt || (undecided && acc[w] < mw);
  }
  return !lt;
}

__device__ __forceinline__ void mw_sub(uint64_t (&acc)[kMaxConvWords], const uint64_t* m) {
  uint64_t borrow = 0;
#pragma unroll
  for (int w = 0; w < kMaxConvWords; ++w) {
    const uint64_t mw = m[w];
    const uint64_t d = acc[w] - mw;
    const uint64_t b1 = acc[w] < mw;
    const uint64_t d2 = d - borrow;
    const uint64_t b2 = d < borrow;
    acc[w] = d2;
    borrow = b1 | b2;
  }
}

// out[j] = v mod t_j for the integer v with residues r[i] modulo the source
// primes: v in [0, S), or its centred lift in (-S/2, S/2] (see BaseConv).
// The multi-word sum has at most ns S < 2^(64 kMaxConvWords).
__device__ void base_conv(const BaseConv* __restrict__ C, const uint64_t* r, uint64_t* out, bool centred) {
  const uint32_t ns = C->ns, nt = C->nt;
  uint64_t y[kMaxBase];
  uint64_t acc[kMaxConvWords];
#pragma unroll
  for (int w = 0; w < kMaxConvWords; ++w) acc[w] = 0;
#pragma unroll
  for (int i = 0; i < kMaxBase; ++i) {
    if ((uint32_t)i < ns) {
      const uint64_t si = C->s[i];
      y[i] = csub(shoup(r[i], C->inv[i], C->invp[i], si), si);
      mw_mac_full(acc, y[i], C->hat[i]);
    } else {
      y[i] = 0;
    }
  }
  uint32_t alpha = 0;
  for (uint32_t it = 0; it < ns; ++it) {  // the sum is below ns S
    if (!mw_geq(acc, C->S)) break;
    mw_sub(acc, C->S);
    ++alpha;
  }
  if (centred) {
    // v > floor(S/2): the centred lift is v - S
    uint64_t h1[kMaxConvWords];
#pragma unroll
    for (int w = 0; w < kMaxConvWords; ++w) h1[w] = C->half[w];
    // acc > half  <=>  acc >= half + 1
    uint64_t carry = 1;
#pragma unroll
    for (int w = 0; w < kMaxConvWords; ++w) {
      const uint64_t v = h1[w] + carry;
      carry = v < carry;
      h1[w] = v;
    }
    if (mw_geq(acc, h1)) ++alpha;
  }
  for (uint32_t j = 0; j < nt; ++j) {
    const uint64_t tj = C->t[j];
    uint64_t sum = 0;  // ns terms below 2 t_j each (t_j < 2^55, ns <= 20): below 2^61
#pragma unroll
    for (int i = 0; i < kMaxBase; ++i)
      if ((uint32_t)i < ns) sum += shoup(y[i], C->hat_t[i][j], C->hat_tp[i][j], tj);
    sum = sum % tj;
    const uint64_t sub = csub(shoup((uint64_t)alpha, C->S_t[j], C->S_tp[j], tj), tj);
    out[j] = submod(sum, sub, tj);
  }
}

// INTT of the column and indicator rows of the pass: one row per workgroup,
// row r = (((q kc + k) 2 + which) 2 + part) L + limb; output in [0, q_limb).
template <int LOGN>
__global__ __launch_bounds__((NttShape<LOGN, 4>::T)) void k_pir2_coef(Pir2Args a, DevModuli M) {
  using S = NttShape<LOGN, 4>;
  using FM = FirstMap<LOGN, 4>;
  __shared__ uint64_t lds[S::LDS_WORDS];
  const int tid = threadIdx.x;
  const uint32_t L = (uint32_t)a.L;
  uint32_t r = blockIdx.x;
  const uint32_t limb = r % L;
  r /= L;
  const uint32_t part = r & 1;
  r >>= 1;
  const uint32_t which = r & 1;
  r >>= 1;
  const uint32_t k = r % a.kc, qq = r / a.kc;
  const uint64_t ctw = 2ull * L * S::N;
  const uint64_t* src = which ? a.E + ((uint64_t)qq * a.stride + a.d1 + a.k0 + k) * ctw
                              : a.col + ((uint64_t)qq * a.d2 + a.k0 + k) * ctw;
  src += ((uint64_t)part * L + limb) * S::N;
  const uint64_t q = M.q[limb];
  uint64_t x[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) x[e] = gmem(src)[FM::idx(tid, e)];
  ntt_inv_nat<LOGN, 4>(x, lds, M.inv[limb], q, tid);
  WALLY_GLOBAL uint64_t* dst = gmem(a.cf) + (uint64_t)blockIdx.x * S::N;
#pragma unroll
  for (int e = 0; e < 16; ++e) dst[FM::idx(tid, e)] = csub(shoup(x[e], M.ninv[limb], M.ninvp[limb], q), q);
}

// centred lift of every coefficient of the pass's rows (mod Q) to the
// auxiliary primes: grid (n / 256, polys = nq kc 4); block 256
__global__ __launch_bounds__(256) void k_pir2_extend(Pir2Args a) {
  const uint64_t n = 1ull << a.log_n;
  const uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t p = blockIdx.y;
  const Pir2Consts* K = a.K;
  uint64_t r[kMaxBase], v[kMaxBase];
#pragma unroll
  for (int i = 0; i < kMaxBase; ++i) r[i] = i < a.L ? gmem(a.cf)[(p * a.L + i) * n + x] : 0;
  base_conv(&K->q_to_b, r, v, true);
  for (int b = 0; b < a.Lb; ++b) gmem(a.ext)[(p * a.Lb + b) * n + x] = v[b];
}

// in-place transform of rows modulo K->mod[m0 + r % period]; natural order
// in and out, results in [0, m)
template <int LOGN>
__global__ __launch_bounds__((NttShape<LOGN, 4>::T)) void k_rows_ntt(uint64_t* data, const Pir2Consts* K, int m0,
                                                                  int period, int inverse) {
  using S = NttShape<LOGN, 4>;
  using FM = FirstMap<LOGN, 4>;
  __shared__ uint64_t lds[S::LDS_WORDS];
  const int tid = threadIdx.x;
  const RowMod md = K->mod[m0 + (int)(blockIdx.x % (uint32_t)period)];
  WALLY_GLOBAL uint64_t* row = gmem(data) + (uint64_t)blockIdx.x * S::N;
  uint64_t x[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) x[e] = row[FM::idx(tid, e)];
  if (inverse) {
    ntt_inv_nat<LOGN, 4>(x, lds, md.inv, md.q, tid);
#pragma unroll
    for (int e = 0; e < 16; ++e) row[FM::idx(tid, e)] = csub(shoup(x[e], md.ninv, md.ninvp, md.q), md.q);
  } else {
    ntt_fwd_nat<LOGN, 4>(x, lds, md.fwd, md.q, tid);
#pragma unroll
    for (int e = 0; e < 16; ++e) row[FM::idx(tid, e)] = reduce_lazy(x[e], md.q, md.onep);
  }
}

// tensor sums of the pass's columns in every modulus of the extended basis
// (NTT form): X0 = sum a0 b0, X1 = sum (a0 b1 + a1 b0), X2 = sum a1 b1 with
// 128-bit lazy sums (2 kc <= 32 products below 2^108).  Ciphertext primes read
// the NTT-form rows themselves, auxiliary primes the extended rows.
// grid (n / 256, L + Lb, nq); block 256
__global__ __launch_bounds__(256) void k_pir2_tensor(Pir2Args a) {
  const uint64_t n = 1ull << a.log_n;
  const uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const int m = blockIdx.y;
  const uint64_t qq = blockIdx.z;
  const RowMod md = a.K->mod[m];
  const uint64_t ctw = 2ull * a.L * n;
  const int MB = a.L + a.Lb;
  u128w s0{0, 0}, s1{0, 0}, s2{0, 0};
  for (uint32_t k = 0; k < a.kc; ++k) {
    uint64_t av[2], bv[2];
    if (m < a.L) {
      WALLY_GLOBAL const uint64_t* ca = gmem(a.col) + (qq * a.d2 + a.k0 + k) * ctw + (uint64_t)m * n + x;
      WALLY_GLOBAL const uint64_t* cb = gmem(a.E) + (qq * a.stride + a.d1 + a.k0 + k) * ctw + (uint64_t)m * n + x;
      av[0] = ca[0];
      av[1] = ca[(uint64_t)a.L * n];
      bv[0] = cb[0];
      bv[1] = cb[(uint64_t)a.L * n];
    } else {
      const uint64_t base = ((qq * a.kc + k) * 4) * a.Lb + (uint64_t)(m - a.L);
      WALLY_GLOBAL const uint64_t* e = gmem(a.ext) + base * n + x;
      const uint64_t stride = (uint64_t)a.Lb * n;  // next part; two parts per ciphertext
      av[0] = e[0];
      av[1] = e[stride];
      bv[0] = e[2 * stride];
      bv[1] = e[3 * stride];
    }
    mac128(s0, av[0], bv[0]);
    mac128(s1, av[0], bv[1]);
    mac128(s1, av[1], bv[0]);
    mac128(s2, av[1], bv[1]);
  }
  WALLY_GLOBAL uint64_t* o = gmem(a.x3) + (qq * 3 * MB + m) * n + x;
  const u128w sums[3] = {s0, s1, s2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    uint64_t v = reduce128(sums[c], md.q, md.r64, md.r64p, md.onep);
    if (a.accumulate) v = addmod(v, o[(uint64_t)c * MB * n], md.q);
    o[(uint64_t)c * MB * n] = v;
  }
}

// scaling: per coefficient of each tensor sum x (residues in the extended
// basis, coefficient form), y = round(t x / Q) = (t x + floor(Q/2) - r) / Q
// with r = (t x + floor(Q/2)) mod Q: r is carried from Q to the auxiliary
// primes exactly, y is formed there (|y| < B / 2) and carried back to the
// ciphertext primes with its centred lift.  Output slots (c0, c2, 0, c1).
// grid (n / 256, 3, nq); block 256
__global__ __launch_bounds__(256) void k_pir2_scale(Pir2Args a) {
  const uint64_t n = 1ull << a.log_n;
  const uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  const uint64_t qq = blockIdx.z;
  const Pir2Consts* K = a.K;
  const int L = a.L, Lb = a.Lb, MB = L + Lb;
  WALLY_GLOBAL const uint64_t* xin = gmem(a.x3) + (qq * 3 + c) * MB * n + x;
  uint64_t r[kMaxBase], rb[kMaxBase], yb[kMaxBase], yq[kMaxBase];
#pragma unroll
  for (int i = 0; i < kMaxBase; ++i) {
    r[i] = 0;
    yb[i] = 0;
    if (i < L) {
      const uint64_t qi = K->mod[i].q;
      const uint64_t tx = csub(shoup(xin[(uint64_t)i * n], K->t_m[i], K->t_mp[i], qi), qi);
      r[i] = addmod(tx, K->h_m[i], qi);
    }
  }
  base_conv(&K->q_to_b, r, rb, false);
  for (int b = 0; b < Lb; ++b) {
    const uint64_t bq = K->mod[L + b].q;
    const uint64_t tx = csub(shoup(xin[(uint64_t)(L + b) * n], K->t_m[L + b], K->t_mp[L + b], bq), bq);
    const uint64_t num = submod(addmod(tx, K->h_m[L + b], bq), rb[b], bq);
    yb[b] = csub(shoup(num, K->qinv_b[b], K->qinv_bp[b], bq), bq);
  }
  base_conv(&K->b_to_q, yb, yq, true);
  const int slot = c == 0 ? 0 : (c == 1 ? 3 : 1);
  WALLY_GLOBAL uint64_t* o = gmem(a.c3) + (qq * 4 + slot) * L * n + x;
  for (int j = 0; j < L; ++j) o[(uint64_t)j * n] = yq[j];
  if (c == 0) {
    WALLY_GLOBAL uint64_t* z = gmem(a.c3) + (qq * 4 + 2) * L * n + x;
    for (int j = 0; j < L; ++j) z[(uint64_t)j * n] = 0;
  }
}

// ---------------------------------------------------------------------------
// diagnostics: register-resident butterfly rate.  Every thread keeps 16 words
// in registers and runs `iters` radix-16 passes of the transforms' own
// butterfly (ct_bfly forward, gs_bfly inverse) with four fixed twiddles, one
// per stage: 32 butterflies per pass and no memory traffic inside the loop.
// Forward words are never reduced, so they wrap mod 2^64 (the instruction
// sequence does not depend on the values).  The final words are stored so
// the loop is not removed and its arithmetic can be checked.
// grid (blocks); block 256
template <int INV>
__global__ __launch_bounds__(256) void k_bfly_rate(uint64_t* __restrict__ out, ulonglong2 w0, ulonglong2 w1,
                                                   ulonglong2 w2, ulonglong2 w3, uint64_t q, int iters) {
  const uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t q4 = 4 * q;
  uint64_t x[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) x[e] = (gid * 16 + e) * 0x9E3779B97F4A7C15ull % q;
  const ulonglong2 W[4] = {w0, w1, w2, w3};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int half = 8 >> st;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        if (e & half) continue;
        if (INV) gs_bfly(x[e], x[e + half], W[st], q, q4);
        else ct_bfly(x[e], x[e + half], W[st], q, q4);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) out[gid * 16 + e] = x[e];
}

// ---------------------------------------------------------------------------
// response compression (paper §7.1, "Reducing the response size")

// One workgroup per ciphertext part: the L limbs are transformed to
// coefficient form one after another (each thread keeps its 16 coefficients
// of every limb in registers, as r_0 and y_i = r_i (Q'/q_i)^-1 mod q_i), each
// coefficient is switched to q_0 with exact rounding and its low bits dropped,
// and the part's values are packed through LDS into coalesced 32-bit words of
// the little-endian bit stream.  Input rows are read once; nothing goes back
// to memory but the packed bytes.
template <int LOGN, int L>
__global__ __launch_bounds__((NttShape<LOGN, 3>::T)) void k_resp_compress(const uint64_t* __restrict__ in,
                                                                          uint8_t* __restrict__ out, CompressArgs a,
                                                                          DevModuli M) {
  using S = NttShape<LOGN, 3>;  // 8 words per thread: the L limbs' coefficients stay in registers
  using FM = FirstMap<LOGN, 3>;
  constexpr int YL = L > 1 ? L - 1 : 1;
  __shared__ uint64_t lds[S::LDS_WORDS];
  const int tid = threadIdx.x;
  const uint64_t chunk = blockIdx.x >> 1;
  const int part = (int)(blockIdx.x & 1);
  WALLY_GLOBAL const uint64_t* src = gmem(in) + (chunk * 2 + part) * (uint64_t)L * S::N;
  uint64_t r0[S::E], y[YL][S::E];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const uint64_t q = M.q[i];
    uint64_t x[S::E];
#pragma unroll
    for (int e = 0; e < S::E; ++e) x[e] = __builtin_nontemporal_load(&src[(uint64_t)i * S::N + FM::idx(tid, e)]);
    ntt_inv_nat<LOGN, 3>(x, lds, M.inv[i], q, tid);
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      const uint64_t v = csub(shoup(x[e], M.ninv[i], M.ninvp[i], q), q);  // coefficient mod q_i
      if (i == 0) r0[e] = v;
      else y[(i + YL - 1) % YL][e] = csub(shoup(v, a.minv[i], a.minvp[i], q), q);
    }
  }
  const uint64_t q0 = M.q[0];
  const ModConst mc0 = M.mc[0];
  const uint32_t l = a.drop[part], w = a.width[part];
  const uint64_t half = l ? (1ull << (l - 1)) : 0, mask = (w >= 64) ? ~0ull : ((1ull << w) - 1);
#pragma unroll
  for (int e = 0; e < S::E; ++e) {
    // c' = round(c / Q') mod q_0 = (r_0 - [sum_i y_i Q'/q_i - k Q']_{q0}) Q'^-1 with
    // k = round(sum_i y_i Q'/q_i / Q'), found exactly on the multi-word sum
    uint64_t acc[kMaxWords + 1];
#pragma unroll
    for (int wd = 0; wd <= kMaxWords; ++wd) acc[wd] = 0;
    u128w rq{0, 0};
#pragma unroll
    for (int i = 1; i < L; ++i) {
      const uint64_t yi = y[i - 1][e];
      uint64_t carry = 0;
#pragma unroll
      for (int wd = 0; wd < kMaxWords; ++wd) {
        const uint64_t mw = a.m[i][wd];
        const uint64_t lo = yi * mw, hi = __umul64hi(yi, mw);
        uint64_t sm = acc[wd] + lo;
        uint64_t cy = sm < lo;
        sm += carry;
        cy += sm < carry;
        acc[wd] = sm;
        carry = hi + cy;
      }
      acc[kMaxWords] += carry;
      mac128(rq, yi, a.mq0[i]);
    }
    uint32_t kc = 0;
    bool done = false;
#pragma unroll
    for (int it = 0; it < L; ++it) {  // the sum is below (L - 1) Q'
      bool gt = false, lt = false;
#pragma unroll
      for (int wd = kMaxWords; wd >= 0; --wd) {
        const uint64_t qw = wd < kMaxWords ? a.qp[wd] : 0;
        const bool und = !gt && !lt;
        gt = gt || (und && acc[wd] > qw);
        lt = lt || (und && acc[wd] < qw);
      }
      done = done || lt;
      uint64_t br = 0;
#pragma unroll
      for (int wd = 0; wd <= kMaxWords; ++wd) {
        const uint64_t qw = done ? 0 : (wd < kMaxWords ? a.qp[wd] : 0);
        const uint64_t d = acc[wd] - qw;
        const uint64_t b1 = acc[wd] < qw;
        const uint64_t d2 = d - br;
        br = b1 | (d < br);
        acc[wd] = d2;
      }
      kc += done ? 0 : 1;
    }
    {  // round up when 2 (remainder) > Q' (Q' is odd: no ties)
      bool gt = false, lt = false;
#pragma unroll
      for (int wd = kMaxWords; wd >= 0; --wd) {
        const uint64_t two = (acc[wd] << 1) | (wd ? acc[wd - 1] >> 63 : 0);
        const uint64_t qw = wd < kMaxWords ? a.qp[wd] : 0;
        const bool und = !gt && !lt;
        gt = gt || (und && two > qw);
        lt = lt || (und && two < qw);
      }
      kc += gt;
    }
    const uint64_t rmod = reduce128(rq, q0, mc0.r64, mc0.r64p, mc0.onep);
    const uint64_t kq = csub(shoup((uint64_t)kc, a.qpq0, a.qpq0p, q0), q0);  // k [Q']_{q0}
    const uint64_t rc = submod(rmod, kq, q0);
    const uint64_t d = submod(r0[e], rc, q0);
    const uint64_t cp = csub(shoup(d, a.qpinv, a.qpinvp, q0), q0);  // c' in [0, q0)
    lds[FM::idx(tid, e)] = ((cp + half) >> l) & mask;  // the last exchange ended with a barrier
  }
  __syncthreads();
  const uint64_t nwords = (uint64_t)S::N * w / 32;
  WALLY_GLOBAL uint32_t* o = (WALLY_GLOBAL uint32_t*)(gmem(out) + chunk * (a.part_bytes[0] + a.part_bytes[1]) +
                                                      (part ? a.part_bytes[0] : 0));
  for (uint64_t word = tid; word < nwords; word += S::T) {
    const uint64_t b = word * 32;
    uint64_t k = b / w;
    const uint32_t off = (uint32_t)(b - k * w);
    uint64_t v = lds[k] >> off;
    uint32_t have = w - off;
    for (++k; have < 32 && k < (uint64_t)S::N; ++k) {
      v |= lds[k] << have;
      have += w;
    }
    o[word] = (uint32_t)v;
  }
}

// ---------------------------------------------------------------------------
// launchers

// KERNEL<LOGN, LOGE> with T = n / 2^LOGE threads
#define WALLY_DISPATCH_LOGN(KERNEL, LOGE, GRID, ...)                                                            \
  switch (a.log_n) {                                                                                          \
    case 12: hipLaunchKernelGGL((KERNEL<12, LOGE>), GRID, dim3(NttShape<12, LOGE>::T), 0, st, __VA_ARGS__); break; \
    case 13: hipLaunchKernelGGL((KERNEL<13, LOGE>), GRID, dim3(NttShape<13, LOGE>::T), 0, st, __VA_ARGS__); break; \
    default: return hipErrorInvalidValue;                                                                     \
  }

// the key-switching kernels at the radix of KsArgs::loge (8 or 16 words per thread)
#define WALLY_DISPATCH_KS(KERNEL, GRID, ...)                 \
  if (a.loge == 3) {                                        \
    WALLY_DISPATCH_LOGN(KERNEL, 3, GRID, __VA_ARGS__);      \
  } else {                                                  \
    WALLY_DISPATCH_LOGN(KERNEL, 4, GRID, __VA_ARGS__);      \
  }

hipError_t launch_ks_digits(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  WALLY_DISPATCH_KS(k_ks_digits, dim3(n_items, a.L), items, a, M);
  return hipGetLastError();
}

hipError_t launch_ks_extend(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  WALLY_DISPATCH_KS(k_ks_extend, dim3(xcd_blocks(n_items * a.L, a.L)), items, a, n_items, M);
  return hipGetLastError();
}

hipError_t launch_ks_inner(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, bool all_rows,
                           hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  const int m0 = all_rows ? 0 : a.L;
  const dim3 grid((1u << a.log_n) / 512, a.L + 1 - m0, n_items);
  switch (a.L) {
    case 1: hipLaunchKernelGGL(k_ks_inner<1>, grid, dim3(256), 0, st, items, a, m0, M); break;
    case 2: hipLaunchKernelGGL(k_ks_inner<2>, grid, dim3(256), 0, st, items, a, m0, M); break;
    case 3: hipLaunchKernelGGL(k_ks_inner<3>, grid, dim3(256), 0, st, items, a, m0, M); break;
    case 4: hipLaunchKernelGGL(k_ks_inner<4>, grid, dim3(256), 0, st, items, a, m0, M); break;
    case 5: hipLaunchKernelGGL(k_ks_inner<5>, grid, dim3(256), 0, st, items, a, m0, M); break;
    case 6: hipLaunchKernelGGL(k_ks_inner<6>, grid, dim3(256), 0, st, items, a, m0, M); break;
    case 7: hipLaunchKernelGGL(k_ks_inner<7>, grid, dim3(256), 0, st, items, a, m0, M); break;
    case 8: hipLaunchKernelGGL(k_ks_inner<8>, grid, dim3(256), 0, st, items, a, m0, M); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ks_pinv(int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  WALLY_DISPATCH_KS(k_ks_pinv, dim3(n_items, 2), a, M);
  return hipGetLastError();
}

hipError_t launch_ks_moddown(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, bool fused,
                             hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (fused) {
    WALLY_DISPATCH_KS(k_ks_moddown, dim3(xcd_blocks(n_items, 2 * a.L)), items, a, n_items, M);
  } else {
    WALLY_DISPATCH_KS(k_ks_moddown_u, dim3(xcd_blocks(n_items * 2, a.L)), items, a, n_items, M);
  }
  return hipGetLastError();
}

hipError_t launch_mac_tiles(const KsItem* items, const MacTile* tiles, int n_tiles, const KsArgs& a, int h,
                            const DevModuli& M, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  const dim3 grid((1u << a.log_n) / 64, a.L, n_tiles);
  switch (a.g) {
    case 2: hipLaunchKernelGGL((k_mac_tiles<2, 2>), grid, dim3(256), 0, st, items, tiles, a, h, M); break;
    case 4: hipLaunchKernelGGL((k_mac_tiles<4, 2>), grid, dim3(256), 0, st, items, tiles, a, h, M); break;
    case 8: hipLaunchKernelGGL((k_mac_tiles<8, 2>), grid, dim3(256), 0, st, items, tiles, a, h, M); break;
    case 16: hipLaunchKernelGGL((k_mac_tiles<16, 2>), grid, dim3(256), 0, st, items, tiles, a, h, M); break;
    case 32: hipLaunchKernelGGL((k_mac_tiles<32, 1>), grid, dim3(256), 0, st, items, tiles, a, h, M); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pir_encode(const uint32_t* coeffs, uint64_t* out, int n_pt, int log_n, int L, const DevModuli& M,
                             hipStream_t st) {
  if (n_pt <= 0) return hipSuccess;
  switch (log_n) {
    case 12: hipLaunchKernelGGL(k_pir_encode<12>, dim3(n_pt, L), dim3(NttShape<12, 4>::T), 0, st, coeffs, out, L, M); break;
    case 13: hipLaunchKernelGGL(k_pir_encode<13>, dim3(n_pt, L), dim3(NttShape<13, 4>::T), 0, st, coeffs, out, L, M); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pir_split(const PirSplitArgs& a, int items, const DevModuli& M, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pir_split, dim3((1u << a.log_n) / 256, 2 * a.L, items), dim3(256), 0, st, a, M);
  return hipGetLastError();
}

hipError_t launch_pir_dot(const PirDotArgs& a, const DevModuli& M, hipStream_t st) {
  if (a.nq == 0 || a.d2 == 0) return hipSuccess;
  const uint32_t pairs = ((a.d2 + 1) / 2) * ((a.nq + 1) / 2);
  const dim3 grid((1u << a.log_n) / 512, a.L, pairs);
  if (a.E3) hipLaunchKernelGGL(k_pir_dot<3>, grid, dim3(256), 0, st, a, M);
  else hipLaunchKernelGGL(k_pir_dot<2>, grid, dim3(256), 0, st, a, M);
  return hipGetLastError();
}

hipError_t launch_pir_lin_split(const KsItem* items, int n_items, const PirSplitArgs& a, uint32_t gal,
                                const DevModuli& M, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  switch (a.log_n) {
    case 12: hipLaunchKernelGGL(k_pir_lin_split<12>, dim3(2 * a.L, n_items), dim3(256), 0, st, items, a, gal, M); break;
    case 13: hipLaunchKernelGGL(k_pir_lin_split<13>, dim3(2 * a.L, n_items), dim3(256), 0, st, items, a, gal, M); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_copy_ct(const CopyItem* items, int n_items, uint64_t words, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_ct, dim3(n_items), dim3(256), 0, st, items, words);
  return hipGetLastError();
}

hipError_t launch_encode(const EncodeJob* jobs, int n_jobs, const EncodeArgs& a, const DevModuli& M, hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  switch (a.log_n) {
    case 12:
      hipLaunchKernelGGL(k_encode<12>, dim3(n_jobs, a.d_pad), dim3(NttShape<12, 4>::T), 0, st, jobs, a, M);
      break;
    case 13:
      hipLaunchKernelGGL(k_encode<13>, dim3(n_jobs, a.d_pad), dim3(NttShape<13, 4>::T), 0, st, jobs, a, M);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ntt_rows(uint64_t* data, int rows, int log_n, int mi, int inverse, const DevModuli& M,
                           hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  switch (log_n) {
    case 12: hipLaunchKernelGGL(k_ntt_rows<12>, dim3(rows), dim3(NttShape<12, 4>::T), 0, st, data, mi, inverse, M); break;
    case 13: hipLaunchKernelGGL(k_ntt_rows<13>, dim3(rows), dim3(NttShape<13, 4>::T), 0, st, data, mi, inverse, M); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pir2_coef(const Pir2Args& a, const DevModuli& M, hipStream_t st) {
  const uint32_t rows = a.nq * a.kc * 4 * (uint32_t)a.L;
  if (rows == 0) return hipSuccess;
  switch (a.log_n) {
    case 12: hipLaunchKernelGGL(k_pir2_coef<12>, dim3(rows), dim3(NttShape<12, 4>::T), 0, st, a, M); break;
    case 13: hipLaunchKernelGGL(k_pir2_coef<13>, dim3(rows), dim3(NttShape<13, 4>::T), 0, st, a, M); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pir2_extend(const Pir2Args& a, hipStream_t st) {
  const uint32_t polys = a.nq * a.kc * 4;
  if (polys == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pir2_extend, dim3((1u << a.log_n) / 256, polys), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pir2_tensor(const Pir2Args& a, hipStream_t st) {
  if (a.nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pir2_tensor, dim3((1u << a.log_n) / 256, a.L + a.Lb, a.nq), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pir2_scale(const Pir2Args& a, hipStream_t st) {
  if (a.nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pir2_scale, dim3((1u << a.log_n) / 256, 3, a.nq), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_rows_ntt(uint64_t* data, int rows, int log_n, const Pir2Consts* K, int m0, int period, int inverse,
                           hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  switch (log_n) {
    case 12:
      hipLaunchKernelGGL(k_rows_ntt<12>, dim3(rows), dim3(NttShape<12, 4>::T), 0, st, data, K, m0, period, inverse);
      break;
    case 13:
      hipLaunchKernelGGL(k_rows_ntt<13>, dim3(rows), dim3(NttShape<13, 4>::T), 0, st, data, K, m0, period, inverse);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bfly_rate(uint64_t* out, int blocks, int inverse, const ulonglong2* w, uint64_t q, int iters,
                            hipStream_t st) {
  if (blocks <= 0) return hipSuccess;
  if (inverse)
    hipLaunchKernelGGL(k_bfly_rate<1>, dim3(blocks), dim3(256), 0, st, out, w[0], w[1], w[2], w[3], q, iters);
  else
    hipLaunchKernelGGL(k_bfly_rate<0>, dim3(blocks), dim3(256), 0, st, out, w[0], w[1], w[2], w[3], q, iters);
  return hipGetLastError();
}

hipError_t launch_resp_compress(const uint64_t* in, uint8_t* out, int chunks, const CompressArgs& a,
                                const DevModuli& M, hipStream_t st) {
  if (chunks <= 0) return hipSuccess;
  const dim3 grid((uint32_t)chunks * 2);
#define WALLY_COMPRESS_L(LOGN)                                                                                \
  switch (a.L) {                                                                                              \
    case 1: hipLaunchKernelGGL((k_resp_compress<LOGN, 1>), grid, dim3(NttShape<LOGN, 3>::T), 0, st, in, out, a, M); break; \
    case 2: hipLaunchKernelGGL((k_resp_compress<LOGN, 2>), grid, dim3(NttShape<LOGN, 3>::T), 0, st, in, out, a, M); break; \
    case 3: hipLaunchKernelGGL((k_resp_compress<LOGN, 3>), grid, dim3(NttShape<LOGN, 3>::T), 0, st, in, out, a, M); break; \
    case 4: hipLaunchKernelGGL((k_resp_compress<LOGN, 4>), grid, dim3(NttShape<LOGN, 3>::T), 0, st, in, out, a, M); break; \
    case 5: hipLaunchKernelGGL((k_resp_compress<LOGN, 5>), grid, dim3(NttShape<LOGN, 3>::T), 0, st, in, out, a, M); break; \
    case 6: hipLaunchKernelGGL((k_resp_compress<LOGN, 6>), grid, dim3(NttShape<LOGN, 3>::T), 0, st, in, out, a, M); break; \
    case 7: hipLaunchKernelGGL((k_resp_compress<LOGN, 7>), grid, dim3(NttShape<LOGN, 3>::T), 0, st, in, out, a, M); break; \
    case 8: hipLaunchKernelGGL((k_resp_compress<LOGN, 8>), grid, dim3(NttShape<LOGN, 3>::T), 0, st, in, out, a, M); break; \
    default: return hipErrorInvalidValue;                                                                     \
  }
  switch (a.log_n) {
    case 12: WALLY_COMPRESS_L(12) break;
    case 13: WALLY_COMPRESS_L(13) break;
    default: return hipErrorInvalidValue;
  }
#undef WALLY_COMPRESS_L
  return hipGetLastError();
}


}  // namespace wally

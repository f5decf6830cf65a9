// Shared declarations between the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "items.h"

namespace wally {

constexpr int kMaxLimbs = 8;
constexpr int kMaxMod = kMaxLimbs + 2;  // q_0..q_{L-1}, P, t

struct ModConst {
  uint64_t q, q2;
  uint64_t r64, r64p;  // 2^64 mod q, Shoup factor
  uint64_t onep;       // floor(2^64 / q)
};

// Everything a kernel needs about the moduli, passed by value.
// Index m: 0..L-1 ciphertext primes, L the special prime P, L+1 the plaintext modulus t.
struct DevModuli {
  uint64_t q[kMaxMod];
  ModConst mc[kMaxMod];
  uint64_t ninv[kMaxMod], ninvp[kMaxMod];  // n^-1 mod q and Shoup factor
  uint64_t pinv[kMaxMod], pinvp[kMaxMod];  // P^-1 mod q_j (j < L) and Shoup factor
  uint64_t c27[kMaxMod], c27p[kMaxMod];    // 2^27 mod q and Shoup factor
  const ulonglong2* fwd[kMaxMod];          // (psi^brv(k), Shoup) for k < n
  const ulonglong2* inv[kMaxMod];          // (psi^-brv(k), Shoup)
};

struct KsArgs {
  int log_n, L;
  int loge;  // 2^loge words per thread in the transforms: 3 (radix-8 passes, n/8 threads) or 4 (radix 16, the default)
  uint32_t gal;
  int in_sel, out_sel;
  uint64_t in_off, out_off;
  int giant;   // giant-step index i to fuse acc_i, or -1
  int add_in;  // 1: add the (unpermuted) input to the output (fold step R + Rot(R))
  int key_fold;     // 1: key = item.key_fold + key_off (a fold step), else item.key
  uint64_t key_off;
  int g;
  uint64_t* X;  // scratch [items][L][n]
  uint64_t* U;  // scratch [items][2][L+1][n]: key inner products (m = L: the P part; the others only
                // when moddown reads them)
  uint64_t* Y;  // scratch [items][2][n]
  uint64_t* D;  // scratch [items][L+1][L][n]: extended digits
};


struct EncodeJob {
  const void* emb;      // first entry of the chunk, row-major [.][d], int8 or int16 (EncodeArgs::wide)
  uint64_t n_entries;   // entries of the cluster in this chunk (<= n / fold)
  uint64_t* out;        // [d_pad / fold][L][n]
  uint32_t fold, g;     // fold factor and baby steps of the chunk's cluster (1 and the context's g unless folded)
};

struct EncodeArgs {
  int log_n, L;
  uint32_t d, d_pad;
  uint32_t wide;            // entries are int16 (else int8)
  const uint32_t* slot_of;  // NTT index -> slot
};

// the key-switching kernels, in launch order
// Response compression (paper §7.1, "Reducing the response size").  With
// Q' = q_1 ... q_{L-1} (the limbs switched away), a coefficient c in [0, Q)
// with residues r_i becomes c' = round(c / Q') mod q_0
//   = (r_0 - (sum_i y_i [Q'/q_i]_{q0} - k [Q']_{q0})) [Q'^-1]_{q0}   (mod q_0),
// y_i = [r_i (Q'/q_i)^-1]_{q_i}, k = round(sum_i y_i / q_i), k found exactly
// from the multi-word remainder of sum_i y_i (Q'/q_i) by Q'.
constexpr int kMaxWords = 6;  // 64-bit words of Q' (up to 7 limbs of 54 bits)
struct CompressArgs {
  int log_n, L, words;                 // words of Q' (>= 1)
  uint32_t drop[2], width[2];          // dropped low bits and serialized width per part
  uint64_t part_bytes[2];              // n * width / 8
  uint64_t qp[kMaxWords];              // Q'
  uint64_t m[kMaxMod][kMaxWords];      // Q'/q_i, i = 1 .. L-1
  uint64_t minv[kMaxMod], minvp[kMaxMod];  // (Q'/q_i)^-1 mod q_i and Shoup factor
  uint64_t mq0[kMaxMod], mq0p[kMaxMod];    // Q'/q_i mod q_0 and Shoup factor
  uint64_t qpq0, qpq0p;                // Q' mod q_0 and Shoup factor
  uint64_t qpinv, qpinvp;              // Q'^-1 mod q_0 and Shoup factor
};

// Index PIR (paper §4.2, MulPIR): query expansion and the first dimension.
// Expansion level a over `items` = queries x 2^a ciphertexts (query q, entry
// b < 2^a): x = cur[q][b], y = Subs(x, g_a) (in ybuf[q][b]);
//   next[q][b] = x + y,  next[q][b + 2^a] = (x - y) * X^(-2^a)
// with w = NTT(X^(-2^a)) per limb as (value, Shoup factor) pairs [L][n].
struct PirSplitArgs {
  const uint64_t* cur;
  const uint64_t* ybuf;
  uint64_t* next;
  const ulonglong2* w;
  uint32_t stride;  // ciphertexts per query in cur / next (2^c)
  uint32_t ystride; // ciphertexts per query in ybuf (2^(c-1))
  uint32_t half;    // 2^a
  int log_n, L;
  // Linearised last level (paper §4.2, "Linearizing parts of query
  // expansion"): when e3 is set, the pairs b whose outputs b and b + half both
  // lie outside [col_lo, col_hi) are k_pir_lin_split's (no key switch; their
  // outputs get a third part u2, decrypted against s(X^g), in e3
  // [queries][stride][L][n]); the split kernel skips them and gives the
  // other pairs u2 = 0.
  uint64_t* e3;
  uint32_t col_lo, col_hi;
};
// First dimension: out[q][k] = sum_{r < d1} E[q][r] * PT[k][r], k < d2.
// With E3 (the third parts of a linearised expansion) the sums have three
// parts, written per column as [U0][U2][0][U1] (4 L n words): (U0, U2) is
// the input of the key switch that finishes the column and (0, U1) what it
// adds.
struct PirDotArgs {
  const uint64_t* E;     // expanded ciphertexts [queries][stride][2][L][n]
  const uint64_t* pt;    // plaintexts [d2][d1][L][n]
  uint64_t* const* out;  // per query: [d2][2][L][n], or [d2][4][L][n] with E3
  uint32_t stride, d1, d2, nq;
  int log_n, L;
  const uint64_t* E3;    // null, or [queries][stride][L][n]
};
// Index PIR, second dimension (paper §4.2 "Overview of MulPIR", step 3; the
// products computed in a larger basis and scaled once, §7.1 "Reducing the
// computation of BFV operations").  The extended basis is the L ciphertext
// primes followed by Lb auxiliary primes whose product B exceeds
// t d2 n Q + 2, so that both the tensor sums (below d2 n Q^2 / 2 in
// magnitude) and their scaled values (below t d2 n Q / 2 + 1) are exact.
constexpr int kMaxAux = 12;
constexpr int kMaxBase = kMaxLimbs + kMaxAux;
constexpr int kMaxConvWords = 12;  // 64-bit words of the multi-word sums of a conversion

// One modulus of the extended basis (index < L: q_index; then the auxiliary primes).
struct RowMod {
  uint64_t q, ninv, ninvp, onep, r64, r64p;
  const ulonglong2* fwd;  // (psi^brv(k), Shoup) for k < n
  const ulonglong2* inv;  // (psi^-brv(k), Shoup)
};

// Exact conversion of residues r_i modulo the ns source primes s_i (product S)
// to residues modulo the nt target primes: with y_i = r_i (S/s_i)^-1 mod s_i,
// the integer v = sum_i y_i (S/s_i) - alpha S lies in [0, S) for
// alpha = floor(sum_i y_i (S/s_i) / S), found exactly by multi-word compares
// (one more S is taken off for the centred lift when v > floor(S/2)); its
// residue mod t_j is sum_i y_i [S/s_i]_{t_j} - alpha [S]_{t_j}.
struct BaseConv {
  uint32_t ns, nt;
  uint64_t s[kMaxBase], inv[kMaxBase], invp[kMaxBase];  // source primes, (S/s_i)^-1 mod s_i, Shoup
  uint64_t hat[kMaxBase][kMaxConvWords];                // S / s_i, little-endian words (zero padded)
  uint64_t S[kMaxConvWords], half[kMaxConvWords];       // S and floor(S / 2)
  uint64_t t[kMaxBase];                                 // target primes
  uint64_t hat_t[kMaxBase][kMaxBase], hat_tp[kMaxBase][kMaxBase];  // [i][j]: (S/s_i) mod t_j, Shoup
  uint64_t S_t[kMaxBase], S_tp[kMaxBase];               // S mod t_j, Shoup
};

struct Pir2Consts {
  uint32_t L, Lb;
  RowMod mod[kMaxBase];
  BaseConv q_to_b, b_to_q;
  uint64_t t;
  uint64_t t_m[kMaxBase], t_mp[kMaxBase];  // t mod each modulus of the extended basis, Shoup
  uint64_t h_m[kMaxBase];                  // floor(Q / 2) mod each modulus
  uint64_t qinv_b[kMaxAux], qinv_bp[kMaxAux];  // Q^-1 mod each auxiliary prime, Shoup
};

struct Pir2Args {
  const Pir2Consts* K;   // device copy
  const uint64_t* col;   // first-dimension columns [nq][d2][2][L][n]
  const uint64_t* E;     // expanded ciphertexts [nq][stride][2][L][n]; the second indicator at d1 + k
  uint64_t* cf;          // coefficient form [nq][kc][2 (column, indicator)][2][L][n]
  uint64_t* ext;         // auxiliary residues, then their NTT [nq][kc][2][2][Lb][n]
  uint64_t* x3;          // tensor sums [nq][3][L + Lb][n]
  uint64_t* c3;          // scaled product [nq][4][L][n]: c0, c2, zero, c1 (NTT form once transformed)
  uint32_t stride, d1, d2, k0, kc, nq;  // columns [k0, k0 + kc) in this pass
  int log_n, L, Lb, accumulate;         // accumulate: add to the tensor sums of earlier passes
};
hipError_t launch_pir2_coef(const Pir2Args& a, const DevModuli& M, hipStream_t st);
hipError_t launch_pir2_extend(const Pir2Args& a, hipStream_t st);
hipError_t launch_pir2_tensor(const Pir2Args& a, hipStream_t st);
hipError_t launch_pir2_scale(const Pir2Args& a, hipStream_t st);
// in-place NTT of `rows` rows of n words, row r modulo K->mod[m0 + r % period]
hipError_t launch_rows_ntt(uint64_t* data, int rows, int log_n, const Pir2Consts* K, int m0, int period, int inverse,
                           hipStream_t st);

hipError_t launch_pir_encode(const uint32_t* coeffs, uint64_t* out, int n_pt, int log_n, int L, const DevModuli& M,
                             hipStream_t st);
hipError_t launch_pir_split(const PirSplitArgs& a, int items, const DevModuli& M, hipStream_t st);
// the linearised pairs of a last expansion level: items[b] = {buf0: x, buf1: output b, fin: its third part}
hipError_t launch_pir_lin_split(const KsItem* items, int n_items, const PirSplitArgs& a, uint32_t gal,
                                const DevModuli& M, hipStream_t st);
hipError_t launch_pir_dot(const PirDotArgs& a, const DevModuli& M, hipStream_t st);

hipError_t launch_ks_digits(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st);
hipError_t launch_ks_extend(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st);
// the inner products of every row (all_rows, for k_ks_moddown_u) or of the P rows
hipError_t launch_ks_inner(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, bool all_rows,
                           hipStream_t st);
hipError_t launch_ks_pinv(int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st);
// fused: forms the inner products of the q_j rows itself; else reads them from U
hipError_t launch_ks_moddown(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, bool fused,
                             hipStream_t st);
// acc_i = sum_{j<g} PT[g i + j] * ct'_j for every giant index i of every item
hipError_t launch_mac_tiles(const KsItem* items, const MacTile* tiles, int n_tiles, const KsArgs& a, int h,
                            const DevModuli& M, hipStream_t st);
// responses [chunks][2][L][n] (NTT form mod Q) -> serialized [chunks][part_bytes[0] + part_bytes[1]]
// (out 4-byte aligned)
hipError_t launch_resp_compress(const uint64_t* in, uint8_t* out, int chunks, const CompressArgs& a,
                                const DevModuli& M, hipStream_t st);
// register-resident butterfly loop (diagnostic): out [blocks * 256][16]
hipError_t launch_bfly_rate(uint64_t* out, int blocks, int inverse, const ulonglong2* w, uint64_t q, int iters,
                            hipStream_t st);
hipError_t launch_copy_ct(const CopyItem* items, int n_items, uint64_t words, hipStream_t st);
hipError_t launch_encode(const EncodeJob* jobs, int n_jobs, const EncodeArgs& a, const DevModuli& M, hipStream_t st);
hipError_t launch_ntt_rows(uint64_t* data, int rows, int log_n, int mi, int inverse, const DevModuli& M,
                           hipStream_t st);

}  // namespace wally

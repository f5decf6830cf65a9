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
  uint32_t gal;
  int in_sel, out_sel;
  uint64_t in_off, out_off;
  int giant;   // giant-step index i to fuse acc_i, or -1
  int add_in;  // 1: add the (unpermuted) input to the output (fold step R + Rot(R))
  int key_fold;     // 1: key = item.key_fold + key_off (a fold step), else item.key
  uint64_t key_off;
  int g;
  uint64_t* X;  // scratch [items][L][n]
  uint64_t* U;  // scratch [items][2][L+1][n]: key inner products (m = L: the P part)
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
  uint64_t qpq0;                       // Q' mod q_0
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
};
// First dimension: out[q][k] = sum_{r < d1} E[q][r] * PT[k][r], k < d2.
struct PirDotArgs {
  const uint64_t* E;     // expanded ciphertexts [queries][stride][2][L][n]
  const uint64_t* pt;    // plaintexts [d2][d1][L][n]
  uint64_t* const* out;  // per query: [d2][2][L][n]
  uint32_t stride, d1, d2, nq;
  int log_n, L;
};
hipError_t launch_pir_encode(const uint32_t* coeffs, uint64_t* out, int n_pt, int log_n, int L, const DevModuli& M,
                             hipStream_t st);
hipError_t launch_pir_split(const PirSplitArgs& a, int items, const DevModuli& M, hipStream_t st);
hipError_t launch_pir_dot(const PirDotArgs& a, const DevModuli& M, hipStream_t st);

hipError_t launch_ks_digits(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st);
hipError_t launch_ks_extend(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st);
hipError_t launch_ks_inner(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st);
hipError_t launch_ks_pinv(int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st);
hipError_t launch_ks_moddown(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st);
// acc_i = sum_{j<g} PT[g i + j] * ct'_j for every giant index i of every item
hipError_t launch_mac_tiles(const KsItem* items, const MacTile* tiles, int n_tiles, const KsArgs& a, int h,
                            const DevModuli& M, hipStream_t st);
// rows [chunks][2][L][n], NTT form -> coefficient form in [0, q_i) (in to out)
hipError_t launch_resp_intt(const uint64_t* in, uint64_t* out, int chunks, int log_n, int L, const DevModuli& M,
                            hipStream_t st);
// coefficient rows [chunks][2][L][n] -> serialized responses [chunks][part_bytes[0] + part_bytes[1]]
hipError_t launch_resp_pack(const uint64_t* coef, uint8_t* out, int chunks, const CompressArgs& a, const DevModuli& M,
                            hipStream_t st);
// register-resident butterfly loop (diagnostic): out [blocks * 256][16]
hipError_t launch_bfly_rate(uint64_t* out, int blocks, int inverse, const ulonglong2* w, uint64_t q, int iters,
                            hipStream_t st);
hipError_t launch_copy_ct(const CopyItem* items, int n_items, uint64_t words, hipStream_t st);
hipError_t launch_encode(const EncodeJob* jobs, int n_jobs, const EncodeArgs& a, const DevModuli& M, hipStream_t st);
hipError_t launch_ntt_rows(uint64_t* data, int rows, int log_n, int mi, int inverse, const DevModuli& M,
                           hipStream_t st);

}  // namespace wally

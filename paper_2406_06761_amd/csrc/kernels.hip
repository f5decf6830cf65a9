// HIP kernels of the encrypted scoring path (gfx950).
//
// Ciphertexts are [2][L][n] words in NTT form (entry i of limb l holds the
// polynomial at psi_l^(2 brv(i)+1) mod q_l); Galois keys are [L digits][2][L+1
// moduli][n] with the special prime P last; plaintexts of a cluster chunk are
// [d_pad][L][n].  One workgroup transforms one polynomial (see ntt.h).
//
// Key switching for CtRotate (paper §2.1) follows the hybrid RNS method of
// paper §7.1 with one digit per ciphertext limb and one special prime P:
//   ks_digits : x_i = INTT_{q_i}(sigma(c1)_i)                    (L per item)
//   ks_modup  : u_t[m] = sum_i NTT_m(x_i mod m) * key[i][t][m]     (L+1 per item)
//               for m = P also y_t = INTT_P(u_t[P])
//   ks_moddown: out_t[j] = (u_t[j] - NTT_j([y_t]_centred mod q_j)) * P^-1
//               (+ sigma(c0)_j for t = 0) (+ the giant-step sum)    (L per item)
// The giant-step sum acc_i = sum_j PT[g i + j] * ct'_j (Server Computation
// algorithm, paper §5) is fused into ks_moddown, so one Horner step
// R <- acc_i + Rot(R, g) is three launches.
#include "kernels.h"
#include "ntt.h"

namespace wally {

__device__ __forceinline__ const uint64_t* sel_in(const KsItem& it, int sel, uint64_t off) {
  return sel == 0 ? it.buf0 + off : (sel == 1 ? it.buf1 + off : it.fin + off);
}
__device__ __forceinline__ uint64_t* sel_out(const KsItem& it, int sel, uint64_t off) {
  return sel == 0 ? it.buf0 + off : (sel == 1 ? it.buf1 + off : it.fin + off);
}

// ---------------------------------------------------------------------------
// key switching, step 1: digits
// grid (items, L); block T
template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_ks_digits(const KsItem* __restrict__ items, KsArgs a,
                                                                 DevModuli M) {
  using S = NttShape<LOGN>;
  __shared__ uint64_t lds[S::LDS_WORDS];
  const int tid = threadIdx.x;
  const int b = blockIdx.x, i = blockIdx.y;
  const KsItem it = items[b];
  const uint64_t* c1 = sel_in(it, a.in_sel, a.in_off) + ((uint64_t)a.L + i) * S::N;
  const uint64_t q = M.q[i];
  uint64_t x[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) x[e] = c1[galois_src<LOGN>(LastMap<LOGN>::idx(tid, e), a.gal)];
  ntt_inv<LOGN>(x, lds, M.inv[i], q, tid);
  uint64_t* X = a.X + ((uint64_t)b * a.L + i) * S::N;
#pragma unroll
  for (int e = 0; e < 16; ++e) X[FirstMap<LOGN>::idx(tid, e)] = csub(shoup(x[e], M.ninv[i], M.ninvp[i], q), q);
}

// ---------------------------------------------------------------------------
// key switching, step 2: extension to every modulus and key inner product
// grid (items, L+1); block T
template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_ks_modup(const KsItem* __restrict__ items, KsArgs a,
                                                                DevModuli M) {
  using S = NttShape<LOGN>;
  __shared__ uint64_t lds[S::LDS_WORDS];
  const int tid = threadIdx.x;
  const int b = blockIdx.x, m = blockIdx.y;
  const int L = a.L, MM = a.L + 1;
  const KsItem it = items[b];
  const uint64_t* c1 = sel_in(it, a.in_sel, a.in_off) + (uint64_t)L * S::N;
  const uint64_t q = M.q[m], q2 = 2 * q;
  // extended digits NTT_m(x_i mod m), i != m; each thread later reads back
  // only the words it wrote, so no barrier is needed between the phases
  uint64_t* D = a.D + ((uint64_t)b * MM + m) * L * S::N;
  for (int i = 0; i < L; ++i) {
    if (i == m) continue;
    const uint64_t* X = a.X + ((uint64_t)b * L + i) * S::N;
    uint64_t d[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) d[e] = X[FirstMap<LOGN>::idx(tid, e)];  // < q_i < 2 q_m
    ntt_fwd<LOGN>(d, lds, M.fwd[m], q, tid);
#pragma unroll
    for (int e = 0; e < 16; ++e) D[(uint64_t)i * S::N + LastMap<LOGN>::idx(tid, e)] = reduce4(d[e], q, q2);
  }
  // key inner product, 128-bit lazy accumulation per element
  const ModConst mc = M.mc[m];
  uint64_t u0[16], u1[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const uint32_t p = LastMap<LOGN>::idx(tid, e);
    u128w acc0{0, 0}, acc1{0, 0};
    for (int i = 0; i < L; ++i) {
      const uint64_t d = (i == m) ? c1[(uint64_t)i * S::N + galois_src<LOGN>(p, a.gal)] : D[(uint64_t)i * S::N + p];
      mac128(acc0, d, it.key[(((uint64_t)i * 2 + 0) * MM + m) * S::N + p]);
      mac128(acc1, d, it.key[(((uint64_t)i * 2 + 1) * MM + m) * S::N + p]);
    }
    u0[e] = reduce128(acc0, q, mc.r64, mc.r64p, mc.onep);
    u1[e] = reduce128(acc1, q, mc.r64, mc.r64p, mc.onep);
  }
  if (m < L) {
    uint64_t* U0 = a.U + (((uint64_t)b * 2 + 0) * L + m) * S::N;
    uint64_t* U1 = a.U + (((uint64_t)b * 2 + 1) * L + m) * S::N;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t p = LastMap<LOGN>::idx(tid, e);
      U0[p] = u0[e];
      U1[p] = u1[e];
    }
  } else {
    // the P part back to coefficients, kept in [0, P); centred by the consumer
    ntt_inv<LOGN>(u0, lds, M.inv[m], q, tid);
    ntt_inv<LOGN>(u1, lds, M.inv[m], q, tid);
    uint64_t* Y0 = a.Y + ((uint64_t)b * 2 + 0) * S::N;
    uint64_t* Y1 = a.Y + ((uint64_t)b * 2 + 1) * S::N;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t p = FirstMap<LOGN>::idx(tid, e);
      Y0[p] = csub(shoup(u0[e], M.ninv[m], M.ninvp[m], q), q);
      Y1[p] = csub(shoup(u1[e], M.ninv[m], M.ninvp[m], q), q);
    }
  }
}

// ---------------------------------------------------------------------------
// key switching, step 3: division by P, sigma(c0), optional giant-step sum
// grid (items, L); block T
template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_ks_moddown(const KsItem* __restrict__ items, KsArgs a,
                                                                  DevModuli M) {
  using S = NttShape<LOGN>;
  __shared__ uint64_t lds[S::LDS_WORDS];
  const int tid = threadIdx.x;
  const int b = blockIdx.x, j = blockIdx.y;
  const int L = a.L;
  const KsItem it = items[b];
  const uint64_t* c0 = sel_in(it, a.in_sel, a.in_off) + (uint64_t)j * S::N;
  const uint64_t q = M.q[j], q2 = 2 * q;
  const uint64_t P = M.q[L];
  const uint64_t halfP = (P - 1) / 2;
  uint64_t res[2][16];
  for (int t = 0; t < 2; ++t) {
    const uint64_t* Y = a.Y + ((uint64_t)b * 2 + t) * S::N;
    uint64_t z[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint64_t y = Y[FirstMap<LOGN>::idx(tid, e)];
      z[e] = y > halfP ? y + (q - P) : y;  // centred lift, then mod q_j (P < q_j)
    }
    ntt_fwd<LOGN>(z, lds, M.fwd[j], q, tid);
    const uint64_t* U = a.U + (((uint64_t)b * 2 + t) * L + j) * S::N;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t p = LastMap<LOGN>::idx(tid, e);
      const uint64_t v = submod(U[p], reduce4(z[e], q, q2), q);
      uint64_t r = csub(shoup(v, M.pinv[j], M.pinvp[j], q), q);
      if (t == 0) r = addmod(r, c0[galois_src<LOGN>(p, a.gal)], q);
      res[t][e] = r;
    }
  }
  if (a.giant >= 0) {
    // acc_i = sum_{jj < g} PT[g i + jj] * ct'_jj, for both polynomials
    const ModConst mc = M.mc[j];
    const uint64_t ctw = 2ull * L * S::N;
    const uint64_t* pt = it.pt + ((uint64_t)a.g * a.giant * L + j) * S::N;
    const uint64_t* cp = it.ctp + (uint64_t)j * S::N;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t p = LastMap<LOGN>::idx(tid, e);
      u128w s0{0, 0}, s1{0, 0};
      for (int jj = 0; jj < a.g; ++jj) {
        const uint64_t w = pt[(uint64_t)jj * L * S::N + p];
        mac128(s0, w, cp[jj * ctw + p]);
        mac128(s1, w, cp[jj * ctw + (uint64_t)L * S::N + p]);
      }
      res[0][e] = addmod(res[0][e], reduce128(s0, q, mc.r64, mc.r64p, mc.onep), q);
      res[1][e] = addmod(res[1][e], reduce128(s1, q, mc.r64, mc.r64p, mc.onep), q);
    }
  }
  uint64_t* out = sel_out(it, a.out_sel, a.out_off) + (uint64_t)j * S::N;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const uint32_t p = LastMap<LOGN>::idx(tid, e);
    out[p] = res[0][e];
    out[(uint64_t)L * S::N + p] = res[1][e];
  }
}

// ---------------------------------------------------------------------------
// first giant-step accumulator R = acc_{h-1} (no rotation), elementwise
// grid (items, L); block 256
__global__ __launch_bounds__(256) void k_mac_init(const KsItem* __restrict__ items, KsArgs a, DevModuli M) {
  const int b = blockIdx.x, j = blockIdx.y;
  const int L = a.L;
  const uint64_t n = 1ull << a.log_n;
  const KsItem it = items[b];
  const ModConst mc = M.mc[j];
  const uint64_t q = mc.q;
  const uint64_t ctw = 2ull * L * n;
  const uint64_t* pt = it.pt + ((uint64_t)a.g * a.giant * L + j) * n;
  const uint64_t* cp = it.ctp + (uint64_t)j * n;
  uint64_t* out = sel_out(it, a.out_sel, a.out_off) + (uint64_t)j * n;
  for (uint64_t p = threadIdx.x; p < n; p += blockDim.x) {
    u128w s0{0, 0}, s1{0, 0};
    for (int jj = 0; jj < a.g; ++jj) {
      const uint64_t w = pt[(uint64_t)jj * L * n + p];
      mac128(s0, w, cp[jj * ctw + p]);
      mac128(s1, w, cp[jj * ctw + (uint64_t)L * n + p]);
    }
    out[p] = reduce128(s0, q, mc.r64, mc.r64p, mc.onep);
    out[(uint64_t)L * n + p] = reduce128(s1, q, mc.r64, mc.r64p, mc.onep);
  }
}

// copy each item's source ciphertext into slot 0 of its rotated-copies buffer
// grid (items); block 256
__global__ __launch_bounds__(256) void k_copy_ct(const CopyItem* __restrict__ items, uint64_t words) {
  const CopyItem it = items[blockIdx.x];
  const ulonglong2* src = reinterpret_cast<const ulonglong2*>(it.src);
  ulonglong2* dst = reinterpret_cast<ulonglong2*>(it.dst);
  for (uint64_t k = threadIdx.x; k < words / 2; k += blockDim.x) dst[k] = src[k];
}

// ---------------------------------------------------------------------------
// cluster encoding (Server Initialization algorithm, paper §5; diagonal
// packing, paper §4.1).  One workgroup makes plaintext m of one chunk:
//   slot s of the chunk belongs to entry base + s; diagonal m holds coordinate
//   ((s mod d_pad) + m) mod d_pad of that entry (0 past the cluster or past d);
//   plaintext g*i + j is that diagonal rotated right by g*i within each row;
//   slots -> polynomial mod t (inverse NTT mod t after placing slot s at the
//   NTT index holding it); centred lift; NTT in every ciphertext limb.
// grid (jobs, d_pad); block T
template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_encode(const EncodeJob* __restrict__ jobs, EncodeArgs a,
                                                              DevModuli M) {
  using S = NttShape<LOGN>;
  __shared__ uint64_t lds[S::LDS_WORDS];
  const int tid = threadIdx.x;
  const EncodeJob jb = jobs[blockIdx.x];
  const uint32_t m = blockIdx.y;
  const uint32_t half = S::N / 2;
  const uint32_t dp = a.d_pad, d = a.d;
  const uint32_t rot = (a.g * (m / a.g)) % half;
  const int it = a.L + 1;  // index of t in the modulus tables
  const uint64_t t = M.q[it];
  uint64_t x[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const uint32_t pos = LastMap<LOGN>::idx(tid, e);
    const uint32_t s = a.slot_of[pos];  // slot whose value sits at NTT index pos
    const uint32_t row = s / half, c = s % half;
    const uint32_t s2 = row * half + (c + half - rot) % half;  // pre-rotation (right by g*i)
    const uint64_t entry = s2;
    const uint32_t coord = ((s2 % dp) + m) % dp;
    int v = 0;
    if (entry < jb.n_entries && coord < d) v = jb.emb[entry * d + coord];
    x[e] = v < 0 ? (uint64_t)((int64_t)t + v) : (uint64_t)v;
  }
  ntt_inv<LOGN>(x, lds, M.inv[it], t, tid);
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
    ntt_fwd<LOGN>(x, lds, M.fwd[l], q, tid);
    uint64_t* out = jb.out + ((uint64_t)m * a.L + l) * S::N;
#pragma unroll
    for (int e = 0; e < 16; ++e) out[LastMap<LOGN>::idx(tid, e)] = reduce4(x[e], q, 2 * q);
  }
}

// ---------------------------------------------------------------------------
// diagnostics: in-place NTT / INTT of rows (canonical order) mod modulus `mi`
template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_ntt_rows(uint64_t* data, int mi, int inverse, DevModuli M) {
  using S = NttShape<LOGN>;
  __shared__ uint64_t lds[S::LDS_WORDS];
  const int tid = threadIdx.x;
  uint64_t* row = data + (uint64_t)blockIdx.x * S::N;
  const uint64_t q = M.q[mi];
  uint64_t x[16];
  if (!inverse) {
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = row[FirstMap<LOGN>::idx(tid, e)];
    ntt_fwd<LOGN>(x, lds, M.fwd[mi], q, tid);
#pragma unroll
    for (int e = 0; e < 16; ++e) row[LastMap<LOGN>::idx(tid, e)] = reduce4(x[e], q, 2 * q);
  } else {
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = row[LastMap<LOGN>::idx(tid, e)];
    ntt_inv<LOGN>(x, lds, M.inv[mi], q, tid);
#pragma unroll
    for (int e = 0; e < 16; ++e) row[FirstMap<LOGN>::idx(tid, e)] = csub(shoup(x[e], M.ninv[mi], M.ninvp[mi], q), q);
  }
}

// ---------------------------------------------------------------------------
// launchers

#define WALLY_DISPATCH_LOGN(KERNEL, GRID, ...)                                                     \
  switch (a.log_n) {                                                                               \
    case 12: hipLaunchKernelGGL(KERNEL<12>, GRID, dim3(NttShape<12>::T), 0, st, __VA_ARGS__); break; \
    case 13: hipLaunchKernelGGL(KERNEL<13>, GRID, dim3(NttShape<13>::T), 0, st, __VA_ARGS__); break; \
    default: return hipErrorInvalidValue;                                                          \
  }

hipError_t launch_ks_digits(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  WALLY_DISPATCH_LOGN(k_ks_digits, dim3(n_items, a.L), items, a, M);
  return hipGetLastError();
}

hipError_t launch_ks_modup(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  WALLY_DISPATCH_LOGN(k_ks_modup, dim3(n_items, a.L + 1), items, a, M);
  return hipGetLastError();
}

hipError_t launch_ks_moddown(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  WALLY_DISPATCH_LOGN(k_ks_moddown, dim3(n_items, a.L), items, a, M);
  return hipGetLastError();
}

hipError_t launch_mac_init(const KsItem* items, int n_items, const KsArgs& a, const DevModuli& M, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mac_init, dim3(n_items, a.L), dim3(256), 0, st, items, a, M);
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
      hipLaunchKernelGGL(k_encode<12>, dim3(n_jobs, a.d_pad), dim3(NttShape<12>::T), 0, st, jobs, a, M);
      break;
    case 13:
      hipLaunchKernelGGL(k_encode<13>, dim3(n_jobs, a.d_pad), dim3(NttShape<13>::T), 0, st, jobs, a, M);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ntt_rows(uint64_t* data, int rows, int log_n, int mi, int inverse, const DevModuli& M,
                           hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  switch (log_n) {
    case 12: hipLaunchKernelGGL(k_ntt_rows<12>, dim3(rows), dim3(NttShape<12>::T), 0, st, data, mi, inverse, M); break;
    case 13: hipLaunchKernelGGL(k_ntt_rows<13>, dim3(rows), dim3(NttShape<13>::T), 0, st, data, mi, inverse, M); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace wally

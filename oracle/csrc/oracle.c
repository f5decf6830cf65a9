/*
 * oracle.c -- plain CPU reference for BFV encrypted nearest-neighbour scoring.
 *
 * TEST INFRASTRUCTURE.  This file is the oracle the GPU library is checked
 * against.  It shares no code, header, table or constant with the GPU
 * library and is never linked into it.  It is written to be read against the
 * paper, not to be fast: every modular product is (a*b) mod q on unsigned
 * 128-bit integers, every polynomial product goes through the NTT defined
 * below, and there is no blocking, fusion or lazy reduction.
 *
 * Conventions (the paper leaves them open; each is a reading of it):
 *  - NTT form ("canonical"): entry i of the transform of a(X) mod q is
 *    a(psi^(2*brv(i)+1)) mod q, psi the smallest primitive 2n-th root of
 *    unity mod q.  Arrays are [poly][limb][coefficient]; Galois keys are
 *    [digit][poly][limb][coefficient] with the special prime P last.
 *  - Ciphertext (c0, c1) with c0 + c1*s = Delta*m + e (mod Q), the paper's
 *    decryption identity (paper 2.1, "Somewhat Homomorphic Encryption").
 *  - Slots: slot s = rho*n/2 + c holds m(psi_t^e), e = 3^c mod 2n for rho = 0
 *    and e = -3^c mod 2n for rho = 1, so X -> X^3 rotates both rows left by
 *    one slot (paper 2.1, "CtRotate").
 *  - Key switching: hybrid RNS variant (paper 7.1) with one digit per
 *    ciphertext limb and a single special prime P; digits are the limb
 *    residues in [0, q_i); the P-part is removed with a centred lift.
 *
 * Build: gcc -O2 -shared -fPIC oracle.c -o liboracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define OR_MAX_LIMBS 8

/* Parameter block filled in by the Python side (oracle/params.py). */
typedef struct {
  int32_t log_n;
  int32_t L;          /* ciphertext limbs                           */
  int32_t d;          /* embedding dimension                        */
  int32_t d_pad;      /* padded dimension (power of two)            */
  int32_t g, h;       /* baby / giant step counts, g*h = d_pad      */
  uint64_t q[OR_MAX_LIMBS + 1];   /* q_0..q_{L-1}, then P at index L  */
  uint64_t psi[OR_MAX_LIMBS + 1]; /* smallest primitive 2n-th roots   */
  uint64_t t, psi_t;              /* plaintext modulus and its root   */
  uint64_t delta_mod[OR_MAX_LIMBS]; /* floor(Q/t) mod q_i             */
  uint64_t gal_baby, gal_giant;     /* Galois elements 3, 3^g mod 2n  */
} or_params;

/* ------------------------------------------------------------------ */
/* scalar modular arithmetic                                           */
/* ------------------------------------------------------------------ */

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)(((u128)a * b) % q);
}
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
  uint64_t s = a + b; /* a, b < q < 2^63: no wrap */
  return s >= q ? s - q : s;
}
static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) {
  return a >= b ? a - b : a + (q - b);
}
static uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = mulmod(r, a, q);
    a = mulmod(a, a, q);
    e >>= 1;
  }
  return r;
}
static uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a, q - 2, q); } /* q prime */

/* signed integer -> residue in [0, q) */
static uint64_t smod(int64_t v, uint64_t q) {
  if (v >= 0) return (uint64_t)v % q;
  uint64_t r = (uint64_t)(-(v + 1)) % q; /* avoids overflow at INT64_MIN */
  return q - 1 - r;
}

static uint32_t brv(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

/* ------------------------------------------------------------------ */
/* negacyclic NTT (paper 7.1: polynomial products go through the NTT)  */
/* ------------------------------------------------------------------ */

/* tw[k] = psi^brv(k) */
static void root_table(uint64_t* tw, int log_n, uint64_t q, uint64_t psi) {
  const uint32_t n = 1u << log_n;
  uint64_t p = 1;
  for (uint32_t k = 0; k < n; ++k) {
    tw[brv(k, log_n)] = p;
    p = mulmod(p, psi, q);
  }
}

/* In place: a <- canonical NTT of a (natural-order input, entry i of the
 * output is a(psi^(2 brv(i) + 1))).  Radix-2 Cooley-Tukey. */
void or_ntt(uint64_t* a, int log_n, uint64_t q, uint64_t psi) {
  const uint32_t n = 1u << log_n;
  uint64_t* tw = (uint64_t*)malloc(sizeof(uint64_t) * n);
  root_table(tw, log_n, q, psi);
  for (uint32_t m = 1, t = n / 2; m < n; m *= 2, t /= 2) {
    for (uint32_t i = 0; i < m; ++i) {
      const uint64_t w = tw[m + i];
      for (uint32_t j = 2 * i * t; j < 2 * i * t + t; ++j) {
        const uint64_t u = a[j], v = mulmod(a[j + t], w, q);
        a[j] = addmod(u, v, q);
        a[j + t] = submod(u, v, q);
      }
    }
  }
  free(tw);
}

/* In place inverse of or_ntt: each forward stage undone in reverse order
 * with the inverse twiddle, then a final scaling by n^-1. */
void or_intt(uint64_t* a, int log_n, uint64_t q, uint64_t psi) {
  const uint32_t n = 1u << log_n;
  uint64_t* tw = (uint64_t*)malloc(sizeof(uint64_t) * n);
  root_table(tw, log_n, q, invmod(psi, q));
  for (uint32_t m = n / 2, t = 1; m >= 1; m /= 2, t *= 2) {
    for (uint32_t i = 0; i < m; ++i) {
      const uint64_t w = tw[m + i]; /* = psi^-brv(m+i) */
      for (uint32_t j = 2 * i * t; j < 2 * i * t + t; ++j) {
        const uint64_t u = a[j], v = a[j + t];
        a[j] = addmod(u, v, q);
        a[j + t] = mulmod(submod(u, v, q), w, q);
      }
    }
  }
  const uint64_t ninv = invmod(n % q, q);
  for (uint32_t k = 0; k < n; ++k) a[k] = mulmod(a[k], ninv, q);
  free(tw);
}

/* Galois automorphism on coefficients: a(X) -> a(X^k) mod (X^n + 1, q). */
void or_automorphism(const uint64_t* a, uint64_t* out, int log_n, uint64_t q, uint64_t k) {
  const uint64_t n = 1ull << log_n;
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t e = (i * k) % (2 * n);
    if (e < n) out[e] = a[i];
    else out[e - n] = a[i] ? q - a[i] : 0;
  }
}

/* ------------------------------------------------------------------ */
/* slot encoding mod t (paper 2.1, "Vectorized SHE")                   */
/* ------------------------------------------------------------------ */

/* idx[s] = NTT index holding the value of slot s */
static void slot_table(uint32_t* idx, int log_n) {
  const uint32_t n = 1u << log_n, half = n / 2;
  const uint64_t two_n = 2ull * n;
  uint64_t e = 1; /* 3^c mod 2n */
  for (uint32_t c = 0; c < half; ++c) {
    idx[c] = brv((uint32_t)((e - 1) / 2), log_n);
    idx[half + c] = brv((uint32_t)((two_n - e - 1) / 2), log_n);
    e = (e * 3) % two_n;
  }
}

/* slots (values mod t) -> plaintext polynomial coefficients in [0, t) */
void or_encode_slots(const or_params* p, const uint64_t* slots, uint64_t* poly) {
  const uint32_t n = 1u << p->log_n;
  uint32_t* idx = (uint32_t*)malloc(sizeof(uint32_t) * n);
  slot_table(idx, p->log_n);
  for (uint32_t s = 0; s < n; ++s) poly[idx[s]] = slots[s] % p->t;
  or_intt(poly, p->log_n, p->t, p->psi_t);
  free(idx);
}

/* plaintext polynomial (coefficients in [0, t)) -> slots */
void or_decode_slots(const or_params* p, const uint64_t* poly, uint64_t* slots) {
  const uint32_t n = 1u << p->log_n;
  uint32_t* idx = (uint32_t*)malloc(sizeof(uint32_t) * n);
  uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * n);
  slot_table(idx, p->log_n);
  memcpy(tmp, poly, sizeof(uint64_t) * n);
  or_ntt(tmp, p->log_n, p->t, p->psi_t);
  for (uint32_t s = 0; s < n; ++s) slots[s] = tmp[idx[s]];
  free(tmp);
  free(idx);
}

/* plaintext polynomial mod t -> NTT form in every ciphertext limb, with the
 * coefficients lifted to the centred range (-t/2, t/2] first.
 * out: [L][n] */
void or_lift_plain(const or_params* p, const uint64_t* poly, uint64_t* out) {
  const uint32_t n = 1u << p->log_n;
  for (int l = 0; l < p->L; ++l) {
    uint64_t* o = out + (size_t)l * n;
    for (uint32_t k = 0; k < n; ++k) {
      const int64_t c = poly[k] > (p->t - 1) / 2 ? (int64_t)poly[k] - (int64_t)p->t : (int64_t)poly[k];
      o[k] = smod(c, p->q[l]);
    }
    or_ntt(o, p->log_n, p->q[l], p->psi[l]);
  }
}

/* ------------------------------------------------------------------ */
/* client side: encryption and Galois keys                             */
/* ------------------------------------------------------------------ */

/* ct = (c0, c1), c1 = a, c0 = -a*s + e + Delta*m, all in NTT form.
 * s, e: signed coefficients; m: coefficients in [0, t); a: [L][n] uniform
 * residues already in NTT form; ct: [2][L][n]. */
void or_encrypt(const or_params* p, const int64_t* s, const uint64_t* m, const uint64_t* a,
                const int64_t* e, uint64_t* ct) {
  const uint32_t n = 1u << p->log_n;
  const int L = p->L;
  uint64_t* sn = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* v = (uint64_t*)malloc(sizeof(uint64_t) * n);
  for (int l = 0; l < L; ++l) {
    const uint64_t q = p->q[l];
    for (uint32_t k = 0; k < n; ++k) sn[k] = smod(s[k], q);
    or_ntt(sn, p->log_n, q, p->psi[l]);
    for (uint32_t k = 0; k < n; ++k) v[k] = addmod(smod(e[k], q), mulmod(p->delta_mod[l], m[k] % q, q), q);
    or_ntt(v, p->log_n, q, p->psi[l]);
    uint64_t* c0 = ct + (size_t)l * n;
    uint64_t* c1 = ct + (size_t)(L + l) * n;
    const uint64_t* al = a + (size_t)l * n;
    for (uint32_t k = 0; k < n; ++k) {
      c0[k] = submod(v[k], mulmod(al[k], sn[k], q), q);
      c1[k] = al[k];
    }
  }
  free(sn);
  free(v);
}

/* Galois key for X -> X^gal, switching sigma(s) back to s.
 * For digit i and modulus m (m = L is P):
 *   key[i][1][m] = a_i[m]
 *   key[i][0][m] = -a_i[m]*s + e_i + [m == i] * (P mod q_i) * sigma(s)
 * a: [L][L+1][n] uniform in NTT form; e: [L][n] signed coefficients;
 * key: [L][2][L+1][n]. */
void or_galois_key(const or_params* p, const int64_t* s, uint64_t gal, const uint64_t* a,
                   const int64_t* e, uint64_t* key) {
  const uint32_t n = 1u << p->log_n;
  const int L = p->L, M = L + 1;
  const uint64_t P = p->q[L];
  uint64_t* sn = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* ss = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* en = (uint64_t*)malloc(sizeof(uint64_t) * n);
  for (int i = 0; i < L; ++i) {
    for (int m = 0; m < M; ++m) {
      const uint64_t q = p->q[m];
      for (uint32_t k = 0; k < n; ++k) sn[k] = smod(s[k], q);
      or_automorphism(sn, ss, p->log_n, q, gal);
      or_ntt(sn, p->log_n, q, p->psi[m]);
      or_ntt(ss, p->log_n, q, p->psi[m]);
      for (uint32_t k = 0; k < n; ++k) en[k] = smod(e[(size_t)i * n + k], q);
      or_ntt(en, p->log_n, q, p->psi[m]);
      const uint64_t* am = a + ((size_t)i * M + m) * n;
      uint64_t* b = key + (((size_t)i * 2 + 0) * M + m) * n;
      uint64_t* ka = key + (((size_t)i * 2 + 1) * M + m) * n;
      const uint64_t gadget = (m == i) ? P % q : 0;
      for (uint32_t k = 0; k < n; ++k) {
        uint64_t v = submod(en[k], mulmod(am[k], sn[k], q), q);
        v = addmod(v, mulmod(gadget, ss[k], q), q);
        b[k] = v;
        ka[k] = am[k];
      }
    }
  }
  free(sn);
  free(ss);
  free(en);
}

/* Key-switching key from a target polynomial w (signed coefficients) back to
 * s, in the layout of the Galois keys: for digit i and modulus m (m = L is P)
 *   key[i][1][m] = a_i[m]
 *   key[i][0][m] = -a_i[m]*s + e_i + [m == i] * (P mod q_i) * w.
 * With w = s^2 (the negacyclic square of s) this is the relinearization key
 * that CtCtMult needs (paper 2.1, "Evaluation keys"; hybrid RNS key
 * switching, paper 7.1).  a: [L][L+1][n] uniform in NTT form; e: [L][n]
 * signed; key: [L][2][L+1][n]. */
void or_switch_key(const or_params* p, const int64_t* s, const int64_t* w, const uint64_t* a, const int64_t* e,
                   uint64_t* key) {
  const uint32_t n = 1u << p->log_n;
  const int L = p->L, M = L + 1;
  const uint64_t P = p->q[L];
  uint64_t* sn = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* wn = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* en = (uint64_t*)malloc(sizeof(uint64_t) * n);
  for (int i = 0; i < L; ++i) {
    for (int m = 0; m < M; ++m) {
      const uint64_t q = p->q[m];
      for (uint32_t k = 0; k < n; ++k) {
        sn[k] = smod(s[k], q);
        wn[k] = smod(w[k], q);
        en[k] = smod(e[(size_t)i * n + k], q);
      }
      or_ntt(sn, p->log_n, q, p->psi[m]);
      or_ntt(wn, p->log_n, q, p->psi[m]);
      or_ntt(en, p->log_n, q, p->psi[m]);
      const uint64_t* am = a + ((size_t)i * M + m) * n;
      uint64_t* b = key + (((size_t)i * 2 + 0) * M + m) * n;
      uint64_t* ka = key + (((size_t)i * 2 + 1) * M + m) * n;
      const uint64_t gadget = (m == i) ? P % q : 0;
      for (uint32_t k = 0; k < n; ++k) {
        uint64_t v = submod(en[k], mulmod(am[k], sn[k], q), q);
        v = addmod(v, mulmod(gadget, wn[k], q), q);
        b[k] = v;
        ka[k] = am[k];
      }
    }
  }
  free(sn);
  free(wn);
  free(en);
}

/* Coefficient form of c0 + c1*s in each limb (the decryption phase; the
 * CRT and the scaling by t/Q are done with Python integers). out: [L][n] */
void or_phase(const or_params* p, const int64_t* s, const uint64_t* ct, uint64_t* out) {
  const uint32_t n = 1u << p->log_n;
  const int L = p->L;
  uint64_t* sn = (uint64_t*)malloc(sizeof(uint64_t) * n);
  for (int l = 0; l < L; ++l) {
    const uint64_t q = p->q[l];
    for (uint32_t k = 0; k < n; ++k) sn[k] = smod(s[k], q);
    or_ntt(sn, p->log_n, q, p->psi[l]);
    const uint64_t* c0 = ct + (size_t)l * n;
    const uint64_t* c1 = ct + (size_t)(L + l) * n;
    uint64_t* o = out + (size_t)l * n;
    for (uint32_t k = 0; k < n; ++k) o[k] = addmod(c0[k], mulmod(c1[k], sn[k], q), q);
    or_intt(o, p->log_n, q, p->psi[l]);
  }
  free(sn);
}

/* ------------------------------------------------------------------ */
/* server side                                                         */
/* ------------------------------------------------------------------ */

/* CtRotate (paper 2.1) by the Galois element gal with key switching
 * (paper 7.1, hybrid RNS key switching):
 *   1. c0, c1 to coefficient form, apply X -> X^gal;
 *   2. digits x_i = limb i of sigma(c1), integers in [0, q_i);
 *   3. for every modulus m of Q*P: u_t[m] = sum_i NTT_m(x_i mod m) * key[i][t][m];
 *   4. mod-down: y_t = centred lift of u_t mod P, then
 *      u_t'[j] = (u_t[j] - y_t) * P^-1 mod q_j;
 *   5. output (sigma(c0) + u_0', u_1') in NTT form.
 * ct_in, ct_out: [2][L][n] NTT form; key: [L][2][L+1][n]. */
void or_rotate(const or_params* p, const uint64_t* ct_in, const uint64_t* key, uint64_t gal,
               uint64_t* ct_out) {
  const uint32_t n = 1u << p->log_n;
  const int L = p->L, M = L + 1;
  const uint64_t P = p->q[L];
  const size_t N = n;
  uint64_t* cs = (uint64_t*)malloc(sizeof(uint64_t) * 2 * L * N); /* sigma(c) coefficients */
  uint64_t* u = (uint64_t*)calloc(2 * (size_t)M * N, sizeof(uint64_t));
  uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * N);
  uint64_t* D = (uint64_t*)malloc(sizeof(uint64_t) * N);
  int64_t* y = (int64_t*)malloc(sizeof(int64_t) * N);

  /* step 1 */
  for (int c = 0; c < 2; ++c)
    for (int l = 0; l < L; ++l) {
      memcpy(tmp, ct_in + ((size_t)c * L + l) * N, sizeof(uint64_t) * N);
      or_intt(tmp, p->log_n, p->q[l], p->psi[l]);
      or_automorphism(tmp, cs + ((size_t)c * L + l) * N, p->log_n, p->q[l], gal);
    }
  /* steps 2-3 */
  for (int m = 0; m < M; ++m) {
    const uint64_t qm = p->q[m];
    for (int i = 0; i < L; ++i) {
      const uint64_t* x = cs + ((size_t)L + i) * N; /* digit i = limb i of sigma(c1) */
      for (uint32_t k = 0; k < n; ++k) D[k] = x[k] % qm;
      or_ntt(D, p->log_n, qm, p->psi[m]);
      for (int t = 0; t < 2; ++t) {
        const uint64_t* kk = key + (((size_t)i * 2 + t) * M + m) * N;
        uint64_t* ut = u + ((size_t)t * M + m) * N;
        for (uint32_t k = 0; k < n; ++k) ut[k] = addmod(ut[k], mulmod(D[k], kk[k], qm), qm);
      }
    }
  }
  /* step 4 */
  for (int t = 0; t < 2; ++t) {
    memcpy(tmp, u + ((size_t)t * M + L) * N, sizeof(uint64_t) * N);
    or_intt(tmp, p->log_n, P, p->psi[L]);
    for (uint32_t k = 0; k < n; ++k) y[k] = tmp[k] > (P - 1) / 2 ? (int64_t)tmp[k] - (int64_t)P : (int64_t)tmp[k];
    for (int j = 0; j < L; ++j) {
      const uint64_t qj = p->q[j];
      const uint64_t pinv = invmod(P % qj, qj);
      uint64_t* ut = u + ((size_t)t * M + j) * N;
      or_intt(ut, p->log_n, qj, p->psi[j]);
      for (uint32_t k = 0; k < n; ++k) ut[k] = mulmod(submod(ut[k], smod(y[k], qj), qj), pinv, qj);
    }
  }
  /* step 5 */
  for (int j = 0; j < L; ++j) {
    const uint64_t qj = p->q[j];
    uint64_t* o0 = ct_out + (size_t)j * N;
    uint64_t* o1 = ct_out + ((size_t)L + j) * N;
    const uint64_t* s0 = cs + (size_t)j * N;
    const uint64_t* u0 = u + (size_t)j * N;
    const uint64_t* u1 = u + ((size_t)M + j) * N;
    for (uint32_t k = 0; k < n; ++k) {
      o0[k] = addmod(s0[k], u0[k], qj);
      o1[k] = u1[k];
    }
    or_ntt(o0, p->log_n, qj, p->psi[j]);
    or_ntt(o1, p->log_n, qj, p->psi[j]);
  }
  free(cs);
  free(u);
  free(tmp);
  free(D);
  free(y);
}

/* PtCtMult (paper 2.1): both polynomials times one plaintext in NTT form.
 * pt: [L][n]; ct, out: [2][L][n]. */
void or_ptct_mul(const or_params* p, const uint64_t* pt, const uint64_t* ct, uint64_t* out) {
  const size_t n = (size_t)1 << p->log_n;
  for (int c = 0; c < 2; ++c)
    for (int l = 0; l < p->L; ++l)
      for (size_t k = 0; k < n; ++k)
        out[((size_t)c * p->L + l) * n + k] = mulmod(pt[(size_t)l * n + k], ct[((size_t)c * p->L + l) * n + k], p->q[l]);
}

/* Number of plaintext chunks of a cluster: ceil(N_c / n), at least one. */
uint64_t or_cluster_chunks(const or_params* p, uint64_t n_entries) {
  const uint64_t n = 1ull << p->log_n;
  return n_entries == 0 ? 1 : (n_entries + n - 1) / n;
}

/* Server initialisation for one cluster (paper 5, "Server Initialization
 * Algorithm", and 4.1 "Database and query packing").
 * Slot s of chunk k belongs to entry k*n + s of the cluster.  Diagonal m
 * holds, in slot s, coordinate ((s mod d_pad) + m) mod d_pad of that entry
 * (zero past the cluster end or past d).  Plaintext g*i + j is diagonal
 * g*i + j rotated right by g*i within each row (the baby-step giant-step
 * pre-rotation), slot-encoded mod t, lifted and put in NTT form per limb.
 * emb: int8 [n_entries][d] row-major; out: [chunks][d_pad][L][n]. */
static int64_t entry_value(const void* emb, int elem_bytes, uint64_t i) {
  return elem_bytes == 1 ? (int64_t)((const int8_t*)emb)[i] : (int64_t)((const int16_t*)emb)[i];
}

static void encode_cluster_any(const or_params* p, const void* emb, int elem_bytes, uint64_t n_entries, uint64_t* out);

void or_encode_cluster(const or_params* p, const int8_t* emb, uint64_t n_entries, uint64_t* out) {
  encode_cluster_any(p, emb, 1, n_entries, out);
}

/* The same with int16 entries (higher-precision embeddings for the plaintext
 * CRT variant, paper 7.3). */
void or_encode_cluster16(const or_params* p, const int16_t* emb, uint64_t n_entries, uint64_t* out) {
  encode_cluster_any(p, emb, 2, n_entries, out);
}

static void encode_cluster_any(const or_params* p, const void* emb, int elem_bytes, uint64_t n_entries, uint64_t* out) {
  const uint32_t n = 1u << p->log_n, half = n / 2;
  const uint32_t dp = (uint32_t)p->d_pad, d = (uint32_t)p->d;
  const uint64_t chunks = or_cluster_chunks(p, n_entries);
  uint64_t* diag = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* rot = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* poly = (uint64_t*)malloc(sizeof(uint64_t) * n);
  for (uint64_t k = 0; k < chunks; ++k) {
    for (int i = 0; i < p->h; ++i) {
      for (int j = 0; j < p->g; ++j) {
        const uint32_t m = (uint32_t)(p->g * i + j);
        for (uint32_t s = 0; s < n; ++s) {
          const uint64_t entry = k * n + s;
          const uint32_t coord = ((s % dp) + m) % dp;
          int64_t v = 0;
          if (entry < n_entries && coord < d) v = entry_value(emb, elem_bytes, entry * d + coord);
          diag[s] = smod(v, p->t);
        }
        const uint32_t r = (uint32_t)(p->g * i) % half;
        for (uint32_t s = 0; s < n; ++s) {
          const uint32_t row = s / half, c = s % half;
          rot[s] = diag[row * half + (c + half - r) % half];
        }
        or_encode_slots(p, rot, poly);
        or_lift_plain(p, poly, out + ((k * dp + m) * (size_t)p->L) * n);
      }
    }
  }
  free(diag);
  free(rot);
  free(poly);
}

/* Server computation for one query against one cluster (paper 5, "Server
 * Computation Algorithm", with the giant steps evaluated as the text of that
 * section describes them and only the two rotation keys of 7.1):
 *   baby steps:  ct'_0 = ct, ct'_j = Rot(ct'_{j-1}, 1) for j < g;
 *   per chunk k: acc_i = sum_j PT[k][g*i + j] * ct'_j;
 *                R = acc_{h-1}; for i = h-2 .. 0: R = acc_i + Rot(R, g);
 *   so R = sum_i Rot(acc_i, g*i) and slot s of R_k is the score of entry
 *   k*n + s.
 * ct: [2][L][n]; key_baby/key_giant: [L][2][L+1][n]; pt: [chunks][d_pad][L][n];
 * out: [chunks][2][L][n]. */
void or_score(const or_params* p, const uint64_t* ct, const uint64_t* key_baby, const uint64_t* key_giant,
              const uint64_t* pt, uint64_t chunks, uint64_t* out) {
  const size_t n = (size_t)1 << p->log_n;
  const int L = p->L, g = p->g, h = p->h;
  const size_t ctw = 2 * (size_t)L * n;
  uint64_t* cp = (uint64_t*)malloc(sizeof(uint64_t) * ctw * g);
  uint64_t* R = (uint64_t*)malloc(sizeof(uint64_t) * ctw);
  uint64_t* prod = (uint64_t*)malloc(sizeof(uint64_t) * ctw);
  memcpy(cp, ct, sizeof(uint64_t) * ctw);
  for (int j = 1; j < g; ++j) or_rotate(p, cp + (size_t)(j - 1) * ctw, key_baby, p->gal_baby, cp + (size_t)j * ctw);
  for (uint64_t k = 0; k < chunks; ++k) {
    const uint64_t* ptk = pt + k * (size_t)p->d_pad * L * n;
    for (int i = h - 1; i >= 0; --i) {
      if (i == h - 1) {
        memset(R, 0, sizeof(uint64_t) * ctw);
      } else {
        memcpy(prod, R, sizeof(uint64_t) * ctw);
        or_rotate(p, prod, key_giant, p->gal_giant, R);
      }
      for (int j = 0; j < g; ++j) {
        or_ptct_mul(p, ptk + (size_t)(g * i + j) * L * n, cp + (size_t)j * ctw, prod);
        for (int c = 0; c < 2; ++c)
          for (int l = 0; l < L; ++l)
            for (size_t x = 0; x < n; ++x) {
              const size_t o = ((size_t)c * L + l) * n + x;
              R[o] = addmod(R[o], prod[o], p->q[l]);
            }
      }
    }
    memcpy(out + k * ctw, R, sizeof(uint64_t) * ctw);
  }
  free(cp);
  free(R);
  free(prod);
}

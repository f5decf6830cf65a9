/*
 * wally.h -- C ABI of the MI355X library for server-side encrypted
 * nearest-neighbour scoring (BFV, Halevi-Shoup diagonals, baby-step
 * giant-step rotations).
 *
 * The problem (paper §5, "Server computation"; Server Computation algorithm):
 * the server holds an index of clusters encoded as plaintexts (Server
 * Initialization algorithm, §5) and receives queries (ct, evk, cluster id); for
 * each it returns ceil(N_c / n) ciphertexts whose slot s of chunk k decrypts to
 * the inner product of the query with entry k*n + s of the cluster, mod t.
 * Queries are independent (paper §8: no inter-query synchronisation) and are
 * scored in batches or served as they arrive.
 *
 * Conventions (fixed; the oracle used for testing follows the same ones):
 *   n = 2^log_n; moduli q_0 > ... > q_{L-1} are the largest primes below
 *   2^limb_bits with q = 1 mod 2n; P is the next one (key switching);
 *   t is the smallest prime above 2^t_bits with t = 1 mod 2n.
 *   NTT form: entry i of limb l holds the polynomial at psi_l^(2 brv(i)+1),
 *   psi_l the smallest primitive 2n-th root of unity mod q_l.
 *   Ciphertext:  uint64 [2][L][n], NTT form, words in [0, q_l).
 *   Galois key:  uint64 [L][2][L+1][n] (digit, polynomial b/a, modulus with P
 *                last), NTT form; key_baby is for X -> X^3 (rotate left by 1),
 *                key_giant for X -> X^(3^g mod 2n) (rotate left by g).
 *   Response:    uint64 [chunks][2][L][n] per query, NTT form.
 *   d_pad = next power of two >= dim; g = 2^ceil(log2(d_pad)/2), h = d_pad/g.
 *
 * Errors: every call returns a status code; no exception or abort crosses the
 * ABI.  wally_last_error() gives a message for the last failing call on a
 * context.  Pointers documented as "device" are HIP device pointers the
 * caller owns (e.g. PyTorch tensors) and must keep alive until the work on
 * the given stream has completed.
 */
#ifndef WALLY_H
#define WALLY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WALLY_OK 0
#define WALLY_EINVAL (-1)   /* bad argument: nothing was enqueued            */
#define WALLY_ENOMEM (-2)   /* over the HBM budget or allocation failed      */
#define WALLY_EAGAIN (-3)   /* serving: admission refused now, retry later   */
#define WALLY_EPENDING (-4) /* serving: ticket not finished                  */
#define WALLY_EDEVICE (-5)  /* HIP runtime error (sticky for the context)    */
#define WALLY_ESTATE (-6)   /* call not valid in the current state           */

#define WALLY_LAYOUT_PER_CLUSTER 0 /* each cluster owns ceil(N_c/n) chunks (paper §4.1) */
/* Not in the paper; for indexes whose per-cluster layout exceeds HBM: a
 * cluster of more than n entries owns ceil(N_c/n) chunks (listed first, in
 * cluster order); the others share chunks, packed first-fit decreasing (size
 * descending, ties by index, first shared chunk with room, at its fill
 * level).  A query is scored against its cluster's chunks; its scores start
 * at the cluster's slot base (wally_cluster_info) and the other slots of a
 * shared chunk score other clusters' entries. */
#define WALLY_LAYOUT_COPACK 1
/* Not in the paper; a refinement of the diagonal packing (§4.1) for clusters
 * that fill a small part of a chunk.  Cluster c gets a fold factor B_c, the
 * largest power of two <= fold_max with B_c N_c <= n and d_pad / B_c >= 4
 * (B_c = 1 for clusters of more than n/2 entries, which are laid out exactly
 * as in WALLY_LAYOUT_PER_CLUSTER).  With D = d_pad / B_c, an entry owns B_c
 * slots that each accumulate D of its coordinates: a chunk holds n / B_c
 * entries, entry e (index inside its chunk) is scored in flat slot
 * (e / D) d_pad + e mod D, and the chunk has D plaintexts instead of d_pad.
 * Scoring runs the baby-step giant-step split on the D diagonals
 * (g' = 2^ceil(log2(D)/2), h' = D / g'), then log2 B_c rotate-and-add steps
 * R = R + Rot(R, r) for r = d_pad/2, d_pad/4, ..., D, which sum the partial
 * products.  The query ciphertext is the usual one; the client sends the
 * giant-step key for g' and the fold keys (wally_cluster_fold). */
#define WALLY_LAYOUT_FOLDED 2

#define WALLY_PATH_BATCHED 0 /* queries of all clusters share launches        */
#define WALLY_PATH_PLAIN 1   /* one launch sequence per cluster (baseline)     */
#define WALLY_PATH_GRAPH 2   /* the batched launches captured in hipGraphs      */

typedef struct wally_ctx wally_ctx;

typedef struct {
  uint32_t log_n;      /* 12 or 13                                          */
  uint32_t num_limbs;  /* L, 1..8                                           */
  uint32_t limb_bits;  /* 30..54 bits per ciphertext prime                  */
  uint32_t t_bits;     /* plaintext modulus just above 2^t_bits (< limb_bits)*/
  uint32_t dim;        /* embedding dimension d                             */
  uint32_t layout;     /* WALLY_LAYOUT_PER_CLUSTER, _COPACK or _FOLDED       */
  int32_t device;      /* HIP device ordinal                                */
  uint32_t max_batch;  /* queries resident per wave (0 = 512, at most 32768;
                          max_batch x chunks of the largest cluster at most
                          32768, else scoring returns WALLY_EINVAL)          */
  uint32_t wave_sets;  /* waves in flight on separate streams (0 = 2, at
                          most 8)                                          */
  uint32_t fold_max;   /* WALLY_LAYOUT_FOLDED: largest fold factor, a power
                          of two (0 = 16); must be 0 for the other layouts  */
  uint64_t hbm_budget; /* bytes the context may allocate (0 = 90% of free)  */
} wally_params_desc;

typedef struct {
  uint32_t n, L, d, d_pad, g, h;
  uint64_t q[8];      /* ciphertext primes (first L used)                    */
  uint64_t P;         /* special prime                                      */
  uint64_t t;         /* plaintext modulus                                  */
  uint64_t psi[9];    /* roots for q_0..q_{L-1}, then P                      */
  uint64_t psi_t;
  uint64_t gal_baby, gal_giant;
  uint64_t ct_words;  /* words per ciphertext = 2 L n                       */
  uint64_t key_words; /* words per Galois key = L * 2 * (L+1) * n           */
  uint64_t pt_chunk_words; /* words per encoded chunk = d_pad L n           */
  uint64_t bytes_allocated; /* device bytes held by the context             */
  uint32_t drop_bits[2];         /* low bits dropped from c0, c1 (compression) */
  uint32_t compressed_widths[2]; /* bits per serialized coefficient of c0, c1  */
  uint64_t compressed_chunk_bytes; /* bytes of one compressed response ciphertext */
  uint64_t hbm_budget;           /* device bytes the context may use            */
  uint64_t serve_request_bytes;  /* serving admission charge of a one-chunk
                                    request: ciphertext + two keys + response */
  uint64_t serve_inflight_limit; /* one-chunk requests admitted at once: (budget
                                    - allocated - workspaces not yet allocated)
                                    / serve_request_bytes                    */
} wally_params_info;

/* One query: every pointer is a device pointer, 16-byte aligned (the
 * kernels move rows in 16-byte accesses; a misaligned pointer is refused with
 * EINVAL).  `out` receives chunks(cluster) consecutive ciphertexts.  In WALLY_LAYOUT_FOLDED, key_giant
 * is the key for the cluster's own giant step (wally_cluster_fold) and
 * key_fold holds its log2(fold) fold keys, in the order of gal_fold (NULL
 * allowed when the fold factor is 1); the other layouts ignore key_fold. */
typedef struct {
  uint32_t cluster;
  uint32_t reserved;
  const uint64_t* ct;        /* [2][L][n]                                   */
  const uint64_t* key_baby;  /* [L][2][L+1][n]                              */
  const uint64_t* key_giant; /* [L][2][L+1][n]                              */
  uint64_t* out;             /* [chunks][2][L][n]                           */
  const uint64_t* key_fold;  /* [log2 fold][L][2][L+1][n]                   */
} wally_query;

/* Set up one parameter set on one device.
 *
 * Defined by: the ring R_Q = Z_Q[X]/(X^n + 1) with n slots mod t in two rows
 * of n/2 (paper §2.1, "Somewhat Homomorphic Encryption" and "Vectorized
 * SHE"); the RNS form of BFV with hybrid key switching, which needs the
 * ciphertext primes and one special prime P (§7.1, "Residue Number System
 * (RNS) variant of BFV"); the parameter choices of §7.3 ("SHE parameters":
 * ring degree, limbs of a few tens of bits, plaintext modulus just above a
 * power of two); the baby-step giant-step split of the d_pad diagonals of
 * §4.1 (g * h = d_pad).  The concrete rules are the conventions at the top of
 * this file.
 *
 * desc: host, read only.  log_n 12 or 13; num_limbs 1..8; limb_bits 30..54;
 * t_bits >= 2 with t_bits + 2 <= limb_bits; dim >= 2 with d_pad <= n/2 and
 * d_pad <= 1024 (so g is 2, 4, 8, 16 or 32); max_batch <= 32768; fold_max a
 * power of two <= 256, and 0 outside WALLY_LAYOUT_FOLDED.
 * out: host; on success *out is a new context that owns every device
 * allocation it makes (all counted against hbm_budget) until wally_destroy.
 * Errors: EINVAL for any value outside the ranges above (nothing is
 * allocated, *out = NULL), ENOMEM, EDEVICE. */
int wally_params_init(const wally_params_desc* desc, wally_ctx** out);

/* Parameter values and byte sizes: what the client side needs to build
 * ciphertexts and keys for this context (§2.1; §7.1 and §7.3 for the moduli),
 * plus the serving admission figures of wally_serve_submit.
 * ctx: read only; out: host, filled completely.  EINVAL for NULL. */
int wally_params_query(const wally_ctx* ctx, wally_params_info* out);

/* Server Initialization (paper §5; diagonal packing §4.1): encode K clusters
 * of int8 embeddings into NTT-form plaintexts resident on the device.
 * emb: host, row-major [n_entries][dim]; offsets: host, K+1 entries, cluster
 * c = rows [offsets[c], offsets[c+1]), non-decreasing, offsets[K] = n_entries,
 * every cluster non-empty.  The inputs are copied; the caller keeps them.
 * Replaces any previous index.  Synchronous.  EINVAL, ENOMEM, EDEVICE. */
int wally_encode_clusters(wally_ctx* ctx, const int8_t* emb, uint64_t n_entries, const uint64_t* offsets,
                          uint32_t k);

/* The same with int16 entries: the higher-precision embeddings of the
 * plaintext-CRT variant (paper §7.3), where a context per plaintext modulus
 * (t_bits 16 and 17) scores the query encrypted under each, with the same
 * rotation keys, and the client recombines the two results by the CRT.
 * Entries must be small enough that the dot products stay below t/2 of the
 * combined modulus for the result to be the integer dot product. */
int wally_encode_clusters_i16(wally_ctx* ctx, const int16_t* emb, uint64_t n_entries, const uint64_t* offsets,
                              uint32_t k);

/* Response compression (paper §7.1, "Reducing the response size"): each of
 * `chunks` response ciphertexts in `in` (device, [chunks][2][L][n], NTT form
 * mod Q, as written by wally_score_batch) is switched from Q to the first
 * limb q_0 with rounding, c' = round(c q_0 / Q) per coefficient of each part
 * (exact, in coefficient form), then drop_bits[p] low bits are dropped with
 * rounding, v = floor((c' + 2^(l-1)) / 2^l) mod 2^w with w =
 * compressed_widths[p], and the n values of each part are packed little-endian
 * (value k in stream bits [k w, (k+1) w), stream bit b = bit b%8 of byte b/8).
 * `out` (device) receives [chunks][compressed_chunk_bytes]: part 0, then part
 * 1.  A client recovers c' ~ v 2^l mod q_0 and decrypts at modulus q_0.  Work
 * is enqueued on hip_stream and uses no workspace (calls on different streams
 * are independent).  in: 8-byte aligned; out: 4-byte aligned (the packed
 * stream is written in 32-bit words).  EINVAL for null or misaligned
 * pointers. */
int wally_compress_responses(wally_ctx* ctx, const uint64_t* in, uint64_t chunks, uint8_t* out, void* hip_stream);

/* Where cluster c sits in the encoded index, so that a client can map
 * response slots to entries.  Defined by the packing of §4.1 ("Reducing
 * Communication in Nearest Neighbor Search": entry k n + s of a cluster in
 * slot s of its chunk k) and the Server Initialization algorithm of §5 (one
 * plaintext set per chunk of a cluster).
 * Outputs (host, any may be NULL): the number of chunks of cluster c, the
 * slot of its first entry in its first chunk (0 in the per-cluster and folded
 * layouts) and the device address of its plaintexts [chunks][D][L][n] (D =
 * d_pad except in the folded layout; read only, owned by the context, valid
 * until the next encode or wally_destroy).  Entry e of the cluster is scored
 * in slot (slot_base + e) mod n of chunk (slot_base + e) / n of the response
 * (folded layout: see WALLY_LAYOUT_FOLDED).  EINVAL for c >= K or NULL ctx. */
int wally_cluster_info(const wally_ctx* ctx, uint32_t c, uint32_t* n_chunks, uint32_t* slot_base,
                       const uint64_t** plaintexts);

/* Fold factor of cluster c and what the client needs for its query: the
 * baby-step and giant-step counts g', h' (g' h' = d_pad / fold), the Galois
 * element X -> X^(3^g' mod 2n) of its giant-step key and the log2(fold)
 * elements X -> X^(3^r mod 2n), r = d_pad/2, d_pad/4, ..., d_pad/fold, of its
 * fold keys (gal_fold must have room for 8).  In the other layouts fold = 1
 * and g', h' are the context's g, h.  Any output pointer may be NULL.  EINVAL
 * for c >= K. */
int wally_cluster_fold(const wally_ctx* ctx, uint32_t c, uint32_t* fold, uint32_t* g, uint32_t* h,
                       uint64_t* gal_giant, uint64_t* gal_fold);

/* Index PIR for metadata fetch (paper §4.2, "Overview of MulPIR" and
 * "Reducing evaluation key size"): the query expansion and the first
 * dimension of MulPIR.  The database is d1 x d2 coefficient-encoded
 * plaintexts (a plaintext is n coefficients in [0, t), lifted centred to each
 * limb).  A query for row i is Enc(2^-c X^i) with c = ceil(log2 d1), in NTT
 * form like any ciphertext.  The server expands it: starting from [ct], at
 * level a = 0 .. c-1 each ciphertext x at position b gives x + y at b and
 * (x - y) X^(-2^a) at b + 2^a, with y = Subs(x, g_a), g_a = n/2^a + 1 (the
 * automorphism X -> X^(g_a) followed by key switching); entry r then
 * encrypts [r == i].  Column k of the answer is sum_{r < d1} e_r PT[k][r], an
 * encryption of PT[k][i].  Key reduction: the client sends keys for levels
 * a0 .. c-1 only; a level a < a0 applies Subs(., g_a0) 2^(a0 - a) times
 * (g_a0^(2^(a0-a)) = g_a mod 2n holds for a0 <= floor((log2 n - 1)/2)).
 * wally_pir_answer returns the d2 columns; wally_pir_answer2 (below) adds the
 * second dimension and returns one ciphertext. */
typedef struct {
  const uint64_t* ct;   /* [2][L][n] query                                     */
  const uint64_t* keys; /* [c - a0][L][2][L+1][n] Galois keys of g_a0 .. g_(c-1) */
  uint64_t* out;        /* [d2][2][L][n] answer                                */
} wally_pir_query;

/* Encode a PIR database: coeffs host, [d2][d1][n] uint32 values below t
 * (column k, row r); d1 <= 2048, d2 <= 2048.  first_key_level: a0, or
 * UINT32_MAX for the paper's choice min(c - 1, floor((log2 n - 1)/2)).
 * Replaces the previous PIR database.  Synchronous.  EINVAL, ENOMEM, EDEVICE. */
int wally_pir_encode(wally_ctx* ctx, const uint32_t* coeffs, uint32_t d1, uint32_t d2, uint32_t first_key_level);

/* Expansion depth c, first key level a0 and the Galois elements of the keys a
 * query carries (gal_keys[k] = g_(a0+k), room for c - a0 <= 11 entries).  Any
 * output pointer may be NULL.  EINVAL without a PIR database. */
int wally_pir_info(const wally_ctx* ctx, uint32_t* levels, uint32_t* first_key_level, uint64_t* gal_keys);

/* Both dimensions of MulPIR (paper §4.2, "Overview of MulPIR": one query
 * ciphertext expanded into the two indicator vectors, the first dimension,
 * then d2 ciphertext products and their sum).  The query for entry (row i,
 * column j) is Enc(2^-c (X^i + X^(d1 + j))) with c = ceil(log2(d1 + d2))
 * (wally_pir_info2); its expansion gives the row indicator in entries 0 ..
 * d1-1 and the column indicator in entries d1 .. d1+d2-1.  Column k of the
 * first dimension times indicator entry d1 + k, summed over k, encrypts
 * PT[j][i].  Each BFV product of (a0, a1) and (b0, b1) is taken on the
 * centred integer lifts of the coefficients as (a0 b0, a0 b1 + a1 b0,
 * a1 b1); the d2 products are summed as integers in an extended basis of the
 * L ciphertext primes and auxiliary primes (the NTT-friendly primes of the
 * same size after P, as many as make their product exceed t d2 n Q + 2),
 * scaled once, c = round(t X / Q) mod Q (§7.1: the scaling is skipped between
 * the products), and the three-part result (c0, c1, c2) is relinearized once,
 * (c0, c1) + KeySwitch_{s^2 -> s}(c2), with the query's relinearization key.
 * The answer is bit-exact with that definition. */
typedef struct {
  const uint64_t* ct;        /* [2][L][n] query                                     */
  const uint64_t* keys;      /* [c - a0][L][2][L+1][n] Galois keys of g_a0 .. g_(c-1) (wally_pir_info2) */
  const uint64_t* relin_key; /* [L][2][L+1][n]: digit i, modulus m: (-a s + e + [m == i] (P mod q_i) s^2, a) */
  uint64_t* out;             /* [2][L][n] answer: an encryption of PT[j][i]          */
} wally_pir_query2;

/* Expansion depth c = ceil(log2(d1 + d2)), first key level a0 (the paper's
 * choice min(c - 1, floor((log2 n - 1)/2)) unless wally_pir_encode was given
 * one) and Galois elements of the keys of a two-index query (room for 11),
 * and the number of auxiliary primes.  Any output may be NULL.  EINVAL
 * without a PIR database or when d1 + d2 > 2048. */
int wally_pir_info2(const wally_ctx* ctx, uint32_t* levels, uint32_t* first_key_level, uint64_t* gal_keys,
                    uint32_t* aux_primes);

/* Answer nq two-index queries (device pointers) on hip_stream: expansion,
 * first and second dimension, up to 64 queries at a time (fewer when their
 * buffers would exceed 8 GiB).  Same ordering and ownership rules as
 * wally_pir_answer, whose workspace it shares.  EINVAL (null or misaligned
 * pointers, d1 + d2 > 2048), ESTATE. */
int wally_pir_answer2(wally_ctx* ctx, const wally_pir_query2* q, uint64_t nq, void* hip_stream);

/* Linearised last expansion level (paper §4.2, "Linearizing parts of query
 * expansion") for the answers of both kinds enqueued after this call; off
 * (0) by default.  Key switching is linear, so the key switches of the last
 * level move past the first dimension's sums: at level c - 1 each pair whose
 * two outputs are row entries (or unused) takes the automorphism
 * z = x(X^g), g = g_(c-1), without key switching and gives the three-part
 * ciphertexts (x0 + z0, x1, z1) at b and ((x0 - z0) X^(-2^a), x1 X^(-2^a),
 * -z1 X^(-2^a)) at b + 2^a, which decrypt as u0 + u1 s + u2 s(X^g); pairs
 * that give a column entry of a two-index query are substituted as before.
 * Every first-dimension column (U0, U1, U2) then becomes (U0, U1) +
 * KeySwitch_{s(X^g) -> s}(U2) with the query's Galois key of g_(c-1): one key
 * switch per column instead of one per linearised pair (2^(c-1) of them for
 * a one-index query).  Queries, keys and the client's decryption are
 * unchanged; the answer words differ from those of the plain expansion (the
 * key-switch rounding happens at another point) and decrypt to the same
 * entries.  EINVAL for a null or destroyed ctx. */
int wally_pir_set_linear(wally_ctx* ctx, int on);

/* Answer nq PIR queries (device pointers) on hip_stream: expansion and first
 * dimension, up to 64 queries at a time (fewer for deep expansions, so that a
 * wave's expansion buffers stay within 8 GiB).  Returns once enqueued; caller buffers must
 * stay alive until the stream completes.  The workspace is shared: a call's
 * work runs after the previous call's, whatever stream that was on, and
 * wally_pir_encode waits for answers in flight.  EINVAL, ESTATE. */
int wally_pir_answer(wally_ctx* ctx, const wally_pir_query* q, uint64_t nq, void* hip_stream);

/* Score nq queries (Server Computation algorithm, paper §5): for each, g-1
 * baby-step rotations, then per chunk the giant-step sums of plaintext
 * products combined by h-1 giant rotations.  q: host array of descriptors
 * with device pointers.  `path`: WALLY_PATH_BATCHED (waves of queries of all
 * clusters), WALLY_PATH_PLAIN (one launch sequence per cluster) or
 * WALLY_PATH_GRAPH (the batched launches of the whole batch captured once, in
 * segments of at most 48 waves of max_batch queries with a graph each, and
 * replayed, segment after segment on hip_stream, while the same query array
 * and configuration are passed again; any batch size); all
 * give identical words.  Work is enqueued on hip_stream (a
 * hipStream_t; NULL = default stream) and the call returns once it is
 * enqueued; output is independent of batch composition.  Validation errors
 * are reported before anything is enqueued (EINVAL); ESTATE while serving. */
int wally_score_batch(wally_ctx* ctx, const wally_query* q, uint64_t nq, int path, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the batched
 * path of wally_score_batch with every workspace row and descriptor table in
 * one static device array of WALLY_STATIC_SCRATCH_BYTES, which each GPU the
 * library runs on holds from the first context on it until the process ends.
 * The call allocates nothing (no device memory, no host memory; the pinned
 * descriptor staging and events it uses are made by wally_params_init).
 * Queries run in waves of as many as the array holds, one after another on
 * hip_stream (at n = 8192, L = 4, d_pad = 256 a query needs about 19 MiB, so
 * waves hold 13); the words equal wally_score_batch's.  The caller passes the
 * queries and their output buffers as for wally_score_batch.
 * The array keeps the last call's contents and is shared by every context on
 * the GPU: a call of one context is ordered after that context's previous
 * static call (whatever its stream), but calls of different contexts on one
 * GPU that overlap in time race.  Returns once enqueued.  EINVAL for invalid
 * queries, or when one query's workspace does not fit in the array at these
 * parameters (nothing is enqueued); ESTATE before an encode or while serving. */
#define WALLY_STATIC_SCRATCH_BYTES (256ull << 20)
int wally_score_batch_static(wally_ctx* ctx, const wally_query* q, uint64_t nq, void* hip_stream);

/* One configuration timed by wally_tune. */
typedef struct {
  uint32_t max_batch;  /* queries per wave                                  */
  uint32_t wave_sets;  /* waves in flight (one stream each)                 */
  uint32_t tile_items; /* queries sharing one plaintext chunk per sum tile  */
  uint32_t ntt_radix;  /* key-switch transforms: passes of radix 8 (n/8 threads
                          per transform) or 16 (n/16 threads)              */
  double ms;           /* time of one batched call                          */
} wally_tune_entry;

/* Schedule autotuner: times wally_score_batch (batched path) on the caller's
 * queries for every combination of the candidate wave sizes, wave-stream
 * counts, plaintext-tile sizes and NTT radices of the key-switch transforms
 * (8 or 16) (0-terminated lists; NULL or empty keeps the current value),
 * keeps the fastest for this context and writes every timing to
 * out[0..*n_out).  The words do not depend on the choice.  Synchronous; the
 * outputs of the queries are written (several times).  EINVAL for a radix
 * other than 8 or 16 or an invalid query. */
int wally_tune(wally_ctx* ctx, const wally_query* q, uint64_t nq, const uint32_t* batches, const uint32_t* sets,
               const uint32_t* tiles, const uint32_t* radices, wally_tune_entry* out, uint32_t max_out,
               uint32_t* n_out);

/* Serving (continuous batching).  The protocol runs in epochs and the server
 * must finish every query of an epoch before it ends (§3.1, "Epochs");
 * queries need no synchronisation with each other (§8), so requests that
 * arrive while others are on the GPU join the next wave that a workspace set
 * frees, and their work overlaps on the device.  Each request is scored as in
 * wally_score_batch (§5, Server Computation algorithm) and its words do not
 * depend on the other requests in its wave.
 *
 * start: begin a session on hip_stream (work enqueued before the call is
 * ordered before the session's waves); allocates the workspace sets if they
 * are not there.  ESTATE if already serving or nothing is encoded.
 * submit: non-blocking.  `q` (host, copied) is validated as in
 * wally_score_batch; its device buffers are borrowed until the ticket is
 * returned by poll.  Admission by HBM: a request holds device memory for its
 * ciphertext, its keys and its response chunks while it is in the library
 * (serve_request_bytes in wally_params_info for a one-chunk request); it is
 * admitted only while bytes allocated by the context (index, tables,
 * workspaces) + bytes of the admitted, unfinished requests + its own bytes <=
 * hbm_budget.  EAGAIN when that does not hold now (retry after poll), ENOMEM
 * when the request alone can never fit.  *ticket (host) receives its ticket.
 * poll: non-blocking; writes up to `max` finished tickets to done (host) and
 * their count to *n_done.
 * stop: waits for all admitted requests and ends the session.
 * All four: one thread at a time per context (calls are serialised by a
 * lock); ESTATE outside a session (start inside one); EDEVICE after a device
 * fault. */
int wally_serve_start(wally_ctx* ctx, void* hip_stream);
int wally_serve_submit(wally_ctx* ctx, const wally_query* q, uint64_t* ticket);
int wally_serve_poll(wally_ctx* ctx, uint64_t* done, uint32_t max, uint32_t* n_done);
int wally_serve_stop(wally_ctx* ctx);

const char* wally_strerror(int code);
const char* wally_last_error(const wally_ctx* ctx);
void wally_destroy(wally_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* WALLY_H */

/* Runs every entry point of the C oracle (oracle/csrc/oracle.c, included as
 * one translation unit) on one parameter set under AddressSanitizer and
 * UndefinedBehaviorSanitizer, with deterministic inputs, and writes the
 * outputs that the CPU test compares with the oracle library built without
 * sanitizers.
 *
 * argv[1]: the parameter block (or_params, as oracle/bfv.py fills it);
 * argv[2]: output file.  Exits 1 when a transform round trip fails. */
#include <stdio.h>

#include "../../oracle/csrc/oracle.c"

static uint64_t lcg_state = 0x243F6A8885A308D3ull;
static uint64_t next64(void) {
  lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
  return lcg_state ^ (lcg_state >> 29);
}

static void uniform(uint64_t* a, size_t count, uint64_t q) {
  for (size_t k = 0; k < count; ++k) a[k] = next64() % q;
}

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  or_params p;
  FILE* f = fopen(argv[1], "rb");
  if (!f || fread(&p, sizeof p, 1, f) != 1) return 2;
  fclose(f);
  const size_t n = (size_t)1 << p.log_n;
  const int L = p.L, M = L + 1;
  FILE* out = fopen(argv[2], "wb");
  if (!out) return 2;
  /* transforms: round trip on every modulus */
  uint64_t* a = malloc(n * sizeof *a);
  uint64_t* b = malloc(n * sizeof *b);
  for (int m = 0; m <= M; ++m) {
    const uint64_t q = m < M ? p.q[m] : p.t, psi = m < M ? p.psi[m] : p.psi_t;
    uniform(a, n, q);
    memcpy(b, a, n * sizeof *a);
    or_ntt(b, p.log_n, q, psi);
    or_intt(b, p.log_n, q, psi);
    if (memcmp(a, b, n * sizeof *a)) return 1;
    or_automorphism(a, b, p.log_n, q, p.gal_giant);
    fwrite(b, sizeof *b, n, out);
  }
  /* slots, plaintext lift */
  uint64_t* slots = malloc(n * sizeof *slots);
  uint64_t* poly = malloc(n * sizeof *poly);
  uniform(slots, n, p.t);
  or_encode_slots(&p, slots, poly);
  or_decode_slots(&p, poly, a);
  if (memcmp(a, slots, n * sizeof *a)) return 1;
  uint64_t* pt = malloc((size_t)L * n * sizeof *pt);
  or_lift_plain(&p, poly, pt);
  fwrite(pt, sizeof *pt, (size_t)L * n, out);
  /* client side: encryption, Galois and switching keys, phase */
  int64_t* s = malloc(n * sizeof *s);
  int64_t* e = malloc((size_t)L * n * sizeof *e);
  for (size_t k = 0; k < n; ++k) s[k] = (int64_t)(next64() % 3) - 1;
  for (size_t k = 0; k < (size_t)L * n; ++k) e[k] = (int64_t)(next64() % 43) - 21;
  uint64_t* ua = malloc((size_t)L * M * n * sizeof *ua);
  for (int l = 0; l < L; ++l)
    for (int m = 0; m < M; ++m) uniform(ua + ((size_t)l * M + m) * n, n, p.q[m]);
  uint64_t* ct = malloc(2 * (size_t)L * n * sizeof *ct);
  or_encrypt(&p, s, poly, ua, e, ct);
  fwrite(ct, sizeof *ct, 2 * (size_t)L * n, out);
  const size_t keyw = (size_t)L * 2 * M * n;
  uint64_t* kb = malloc(keyw * sizeof *kb);
  uint64_t* kg = malloc(keyw * sizeof *kg);
  or_galois_key(&p, s, p.gal_baby, ua, e, kb);
  or_galois_key(&p, s, p.gal_giant, ua, e, kg);
  or_switch_key(&p, s, s, ua, e, kg + 0);  /* a switching key to a given target (here s itself) */
  fwrite(kg, sizeof *kg, keyw, out);
  or_galois_key(&p, s, p.gal_giant, ua, e, kg);
  uint64_t* ph = malloc((size_t)L * n * sizeof *ph);
  or_phase(&p, s, ct, ph);
  fwrite(ph, sizeof *ph, (size_t)L * n, out);
  /* server side: rotation, product, encoding, scoring */
  uint64_t* ct2 = malloc(2 * (size_t)L * n * sizeof *ct2);
  or_rotate(&p, ct, kb, p.gal_baby, ct2);
  fwrite(ct2, sizeof *ct2, 2 * (size_t)L * n, out);
  or_ptct_mul(&p, pt, ct, ct2);
  fwrite(ct2, sizeof *ct2, 2 * (size_t)L * n, out);
  const uint64_t entries = n + 37; /* two chunks, the second ragged */
  int8_t* emb = malloc(entries * (size_t)p.d);
  for (size_t k = 0; k < entries * (size_t)p.d; ++k) emb[k] = (int8_t)((int)(next64() % 255) - 127);
  const uint64_t chunks = or_cluster_chunks(&p, entries);
  uint64_t* enc = malloc(chunks * (size_t)p.d_pad * L * n * sizeof *enc);
  or_encode_cluster(&p, emb, entries, enc);
  int16_t* emb16 = malloc(entries * (size_t)p.d * sizeof *emb16);
  for (size_t k = 0; k < entries * (size_t)p.d; ++k) emb16[k] = (int16_t)emb[k];
  uint64_t* enc16 = malloc(chunks * (size_t)p.d_pad * L * n * sizeof *enc16);
  or_encode_cluster16(&p, emb16, entries, enc16);
  if (memcmp(enc, enc16, chunks * (size_t)p.d_pad * L * n * sizeof *enc)) return 1;
  uint64_t* resp = malloc(chunks * 2 * (size_t)L * n * sizeof *resp);
  or_score(&p, ct, kb, kg, enc, chunks, resp);
  fwrite(resp, sizeof *resp, chunks * 2 * (size_t)L * n, out);
  fclose(out);
  free(a), free(b), free(slots), free(poly), free(pt), free(s), free(e), free(ua), free(ct), free(kb), free(kg);
  free(ph), free(ct2), free(emb), free(enc), free(emb16), free(enc16), free(resp);
  return 0;
}

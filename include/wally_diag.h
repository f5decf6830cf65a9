/*
 * wally_diag.h -- component entry points of the MI355X library, for checking
 * single steps of the scoring path against a reference.  Same conventions,
 * ownership and error rules as wally.h.
 */
#ifndef WALLY_DIAG_H
#define WALLY_DIAG_H

#include <stdint.h>

#include "wally.h"

#ifdef __cplusplus
extern "C" {
#endif

/* In-place negacyclic NTT (inverse = 0: coefficients -> NTT form, canonical
 * order; inverse = 1: back, including the n^-1 factor) of `rows` consecutive
 * rows of n words.  mi selects the modulus: 0..L-1 = q_i, L = P, L+1 = t.
 * Input words must be below the modulus.  data: device.  Enqueued on
 * hip_stream. */
int wally_diag_ntt(wally_ctx* ctx, uint32_t mi, uint64_t* data, uint64_t rows, int inverse, void* hip_stream);

/* CtRotate with key switching (paper §2.1; hybrid RNS key switching §7.1) of
 * `count` ciphertexts.  in: [count][2][L][n]; keys: [count][L][2][L+1][n];
 * out: [count][2][L][n] (must not overlap in); which = 0 rotates left by 1
 * (X -> X^3, keys for that element), 1 rotates left by g (X -> X^(3^g)).
 * All device.  Enqueued on hip_stream. */
int wally_diag_rotate(wally_ctx* ctx, const uint64_t* in, const uint64_t* keys, uint64_t* out, uint64_t count,
                      int which, void* hip_stream);

/* Per-launch timing.  When enabled, every kernel launch of the scoring path
 * is bracketed by HIP events recorded on the stream it is launched on;
 * wally_diag_kernel_stats waits for the recorded launches, sums the elapsed
 * times per kernel (index = WALLY_KERNEL_*) into out[0..n), and clears the
 * records. */
#define WALLY_KERNEL_DIGITS 0   /* key switch: INTT of the digits            */
#define WALLY_KERNEL_EXTEND 1   /* key switch: NTT of the extended digits    */
#define WALLY_KERNEL_INNER 2    /* key switch: key inner product, P rows     */
#define WALLY_KERNEL_PINV 3     /* key switch: INTT of the P part            */
#define WALLY_KERNEL_MODDOWN 4  /* key switch: division by P (+ acc_i), with
                                   the inner products of the q_j rows       */
#define WALLY_KERNEL_MAC 5      /* giant-step sums (plaintext products)      */
#define WALLY_KERNEL_COPY 6     /* query copy into the baby-step buffer      */
/* the stored form of the key switch (launches of fewer than 256 items, and
 * every launch of the PIR path): the inner products of every row in one
 * kernel, and the division by P reading them */
#define WALLY_KERNEL_INNER_ALL 7   /* key switch: key inner product, all rows */
#define WALLY_KERNEL_MODDOWN_U 8   /* key switch: division by P, stored u     */
#define WALLY_KERNEL_COUNT 9

/* Register-resident butterfly rate: the peak of the transforms' arithmetic.
 * One launch of `blocks` workgroups of 256 threads; each thread keeps 16
 * words mod q_0 in registers (word e of thread t starts at
 * ((t * 16 + e) * 0x9E3779B97F4A7C15 mod 2^64) mod q_0) and runs `iters`
 * radix-16 passes: stage s = 0..3 pairs words e and e + 8 / 2^s with twiddle
 * W_s = psi_0^(s+1) mod q_0 and its Shoup factor floor(W_s 2^64 / q_0), as a
 * forward lazy Cooley-Tukey butterfly (inverse = 0; words wrap mod 2^64, no
 * reduction) or an inverse Gentleman-Sande butterfly (inverse = 1), the
 * butterflies of the negacyclic NTT (paper §7.1, Harvey butterflies with lazy
 * reduction).  That is 32 butterflies per pass and thread, blocks * 256 * 32 *
 * iters in all.  out (device, [blocks * 256][16] words) receives the final
 * words; *ms (host) the launch's duration from events on hip_stream (the call
 * waits for it).  EINVAL for blocks or iters of 0 or a NULL pointer. */
int wally_diag_bfly_rate(wally_ctx* ctx, int inverse, uint32_t blocks, uint32_t iters, uint64_t* out, double* ms,
                         void* hip_stream);

typedef struct {
  uint64_t launches;
  uint64_t items;   /* work items over all launches (items x grid.y blocks) */
  double total_ms;
} wally_kernel_stat;

int wally_diag_kernel_timing(wally_ctx* ctx, int enable);
int wally_diag_kernel_stats(wally_ctx* ctx, wally_kernel_stat* out, uint32_t n);

#ifdef __cplusplus
}
#endif
#endif /* WALLY_DIAG_H */

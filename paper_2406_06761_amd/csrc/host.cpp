// Host side of the MI355X scoring library: parameter derivation, NTT tables,
// the resident plaintext index, the wave scheduler (batched and per-cluster
// paths) and the serving loop.  The C ABI is declared in include/wally.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "kernels.h"
#include "plan.h"
#include "wally.h"
#include "wally_diag.h"

using namespace wally;
typedef unsigned __int128 u128;

namespace {

// ---------------------------------------------------------------------------
// number theory for the parameter rules (host, exact)

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  for (; e; e >>= 1) {
    if (e & 1) r = mulmod(r, a, m);
    a = mulmod(a, a, m);
  }
  return r;
}

// Deterministic Miller-Rabin for 64-bit n (the first twelve primes as bases).
bool is_prime(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t p : bases)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) d >>= 1, ++s;
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod(x, x, n);
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}

uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

// Smallest primitive two_n-th root of unity mod prime q.
uint64_t min_root(uint64_t q, uint64_t two_n) {
  const uint64_t cof = (q - 1) / two_n;
  uint64_t w = 0;
  for (uint64_t x = 2;; ++x) {
    w = powmod(x, cof, q);
    if (powmod(w, two_n / 2, q) == q - 1) break;
  }
  const uint64_t w2 = mulmod(w, w, q);
  uint64_t best = w, cur = w;
  for (uint64_t k = 1; k < two_n / 2; ++k) {
    cur = mulmod(cur, w2, q);
    best = std::min(best, cur);
  }
  return best;
}

uint64_t shoup_of(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

// responses compressed per launch
constexpr uint64_t kCompressBatch = 1u << 20;

// little-endian multi-word integers for the compression constants
void mw_mul_small(std::vector<uint64_t>& x, uint64_t m) {
  u128 carry = 0;
  for (uint64_t& w : x) {
    const u128 v = (u128)w * m + carry;
    w = (uint64_t)v;
    carry = v >> 64;
  }
  if (carry) x.push_back((uint64_t)carry);
}
uint64_t mw_mod_small(const std::vector<uint64_t>& x, uint64_t q) {
  u128 r = 0;
  for (size_t k = x.size(); k-- > 0;) r = ((r << 64) | x[k]) % q;
  return (uint64_t)r;
}

// Constants of response compression (paper §7.1, "Reducing the response
// size"): switch from Q to q_0, then drop l0 / l1 low bits of the two parts,
// l0 = floor(log2(q_0/t)) - 2 and l1 = floor(log2(q_0/t) - 2 - log2(z sqrt(2n/9)))
// with z = 8 (the bounds of the cited calculation), neither below 0.
bool compress_constants(const uint64_t* mods, int L, int log_n, uint64_t t, CompressArgs& a) {
  a = CompressArgs{};
  a.log_n = log_n;
  a.L = L;
  const uint64_t q0 = mods[0];
  std::vector<uint64_t> qp{1};
  for (int i = 1; i < L; ++i) mw_mul_small(qp, mods[i]);
  if (qp.size() > (size_t)kMaxWords) return false;
  a.words = (int)qp.size();
  for (int w = 0; w < a.words; ++w) a.qp[w] = qp[w];
  for (int i = 1; i < L; ++i) {
    std::vector<uint64_t> m{1};
    for (int j = 1; j < L; ++j)
      if (j != i) mw_mul_small(m, mods[j]);
    for (size_t w = 0; w < m.size() && w < (size_t)kMaxWords; ++w) a.m[i][w] = m[w];
    const uint64_t qi = mods[i];
    a.minv[i] = powmod(mw_mod_small(m, qi), qi - 2, qi);
    a.minvp[i] = shoup_of(a.minv[i], qi);
    a.mq0[i] = mw_mod_small(m, q0);
    a.mq0p[i] = shoup_of(a.mq0[i], q0);
  }
  a.qpq0 = mw_mod_small(qp, q0);
  a.qpq0p = shoup_of(a.qpq0, q0);
  a.qpinv = powmod(a.qpq0, q0 - 2, q0);
  a.qpinvp = shoup_of(a.qpinv, q0);
  const double n = (double)(1u << log_n);
  const double lg = std::log2((double)q0 / (double)t);
  const long l0 = (long)std::floor(lg) - 2;
  const long l1 = (long)std::floor(lg - 2 - std::log2(8.0 * std::sqrt(2.0 * n / 9.0)));
  uint32_t bits = 0;
  while (bits < 64 && (q0 >> bits)) ++bits;
  a.drop[0] = (uint32_t)std::max(0L, l0);
  a.drop[1] = (uint32_t)std::max(0L, l1);
  for (int p = 0; p < 2; ++p) {
    a.width[p] = bits - a.drop[p];
    a.part_bytes[p] = (uint64_t)(1u << log_n) * a.width[p] / 8;
  }
  return true;
}

struct WaveWork {
  // one workspace set: buffers for one wave of queries in flight
  uint64_t* ctp = nullptr;  // [B][g][2][L][n]
  uint64_t* X = nullptr;    // [B][L][n]
  uint64_t* U = nullptr;    // [B][2][L+1][n]
  uint64_t* Y = nullptr;    // [B][2][n]
  uint64_t* D = nullptr;    // [B][L+1][L][n]
  uint64_t* R0 = nullptr;   // [B][2][L][n]
  uint64_t* R1 = nullptr;
  uint64_t* ACC = nullptr;  // [B][h][2][L][n] giant-step sums
  // descriptors: copy items, baby items, giant items
  CopyItem* copy_dev = nullptr;
  KsItem* baby_dev = nullptr;
  KsItem* giant_dev = nullptr;
  CopyItem* copy_host = nullptr;
  KsItem* baby_host = nullptr;
  KsItem* giant_host = nullptr;
  MacTile* tile_dev = nullptr;
  MacTile* tile_host = nullptr;
  size_t giant_cap = 0;
  hipStream_t stream = nullptr;
  hipEvent_t staged = nullptr;  // host descriptors copied
  hipEvent_t done = nullptr;    // wave finished
  bool busy = false;
  std::vector<uint64_t> tickets;  // serving: tickets of the wave in flight
  uint64_t held_bytes = 0;        // serving: admission bytes of those requests
};

struct ServeReq {
  wally_query q;
  uint64_t ticket;
  uint64_t bytes;  // admission charge (request_bytes)
};

struct TimerRec {
  int kernel;
  uint64_t items;
  hipEvent_t a, b;
};

}  // namespace

struct wally_ctx {
  int device = 0;
  int log_n = 0, n = 0, L = 0, d = 0, d_pad = 0, g = 0, h = 0;
  uint64_t mods[kMaxMod] = {};
  uint64_t psi[kMaxMod] = {};
  uint32_t gal_baby = 3, gal_giant = 0;
  DevModuli M{};
  uint64_t budget = 0, allocated = 0;
  std::vector<std::pair<void*, size_t>> allocs;
  void* tables = nullptr;
  uint32_t* slot_of = nullptr;
  // index
  uint32_t K = 0;
  uint32_t layout = WALLY_LAYOUT_PER_CLUSTER;
  std::vector<uint32_t> chunks;      // chunks scored per cluster
  std::vector<uint64_t> chunk_base;  // first chunk of each cluster
  std::vector<uint32_t> slot_base;   // slot of each cluster's first entry in its first chunk
  std::vector<uint32_t> fold;        // fold factor of each cluster (1 unless folded)
  std::vector<uint64_t> chunk_pt;    // word offset of each chunk's plaintexts in pt
  uint32_t fold_max = 1;
  uint64_t gal_fold[8] = {};         // X -> X^(3^r mod 2n), r = d_pad/2, d_pad/4, ...
  uint32_t max_chunks = 0;
  uint64_t n_chunks_total = 0;
  uint64_t* pt = nullptr;
  // index PIR database (paper §4.2): plaintexts [d2][d1][L][n], expansion
  // depth c, lowest key level a0, X^-(2^a) tables [c][L][n]
  uint64_t* pir_pt = nullptr;
  uint32_t pir_d1 = 0, pir_d2 = 0, pir_c = 0, pir_a0 = 0, pir_wq = 0;
  ulonglong2* pir_w = nullptr;
  // PIR workspace: expansion lists [wave][2^c], substitution results
  // [wave][2^(c-1)] (two, for repeated substitutions), key-switch scratch,
  // descriptors (allocated on the first answer after an encode)
  uint64_t* pir_lev[2] = {};
  uint64_t* pir_y[2] = {};
  uint64_t *pir_X = nullptr, *pir_U = nullptr, *pir_Y = nullptr, *pir_D = nullptr;
  KsItem* pir_items_dev = nullptr;
  KsItem* pir_items_host = nullptr;
  CopyItem* pir_copy_dev = nullptr;
  CopyItem* pir_copy_host = nullptr;
  uint64_t** pir_out_dev = nullptr;
  uint64_t** pir_out_host = nullptr;
  hipEvent_t pir_staged = nullptr;
  hipEvent_t pir_done = nullptr;  // after the last answer's work; the next call (any stream) and frees wait for it
  uint64_t pir_work_S = 0;        // expansion size the workspace was made for
  bool pir_work_two = false;      // ... and whether it has the second dimension's buffers
  bool pir_work_lin = false;      // ... and the linearised level's buffers
  bool pir_linear = false;        // linearised last expansion level (wally_pir_set_linear)
  // second dimension: depth and first key level of two-index queries (0
  // levels: not available), the auxiliary primes, constants of the extended
  // basis (device) and the auxiliary transform tables; buffers of one wave
  uint32_t pir_c2 = 0, pir_a02 = 0, pir_Lb = 0, pir2_kc = 0;
  Pir2Consts* pir2_K = nullptr;
  ulonglong2* pir2_tables = nullptr;
  uint64_t *pir2_col = nullptr, *pir2_cf = nullptr, *pir2_ext = nullptr, *pir2_x3 = nullptr, *pir2_c3 = nullptr;
  uint64_t *pir_e3 = nullptr, *pir_cols3 = nullptr;  // third parts of the last level; three-part columns
  // response compression constants
  CompressArgs comp{};
  // wally_score_batch_static: the device's static scratch, pinned host
  // staging for the descriptors of two waves, and their events
  unsigned char* static_scratch = nullptr;
  unsigned char* static_host[2] = {};
  hipEvent_t static_staged[2] = {};
  hipEvent_t static_done = nullptr;  // after each static call; the next one waits for it
  bool static_pending = false;
  // waves
  int B = 0;
  int n_sets = 2;
  uint32_t tile_items = 8;  // giant items per plaintext-sharing tile of the sum kernel
  int ks_loge = 4;          // key-switch transforms: 2^ks_loge words per thread (radix-8 or radix-16 passes)
  // graph path: the captured segments of a whole batch, replayed while the
  // batch (the query array) and the configuration stay the same
  hipStream_t cap_stream = nullptr;
  std::vector<hipGraphExec_t> graph_execs;
  uint64_t graph_key = 0;
  void* graph_desc = nullptr;  // device descriptors of the captured batch
  bool capturing = false;
  hipEvent_t graph_done = nullptr;  // recorded after each graph launch; later eager work waits for it
  bool graph_pending = false;
  std::vector<WaveWork> sets;
  hipEvent_t fork = nullptr;
  std::string err;
  bool dead = false;
  std::mutex mu;
  // serving
  bool serving = false;
  hipStream_t serve_stream = nullptr;
  std::deque<ServeReq> pending;
  std::deque<uint64_t> finished;
  uint64_t next_ticket = 1;
  uint64_t serve_bytes = 0;  // admission bytes of the admitted, unfinished requests
  // optional per-launch timing (events on the launch stream)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<TimerRec> timers;

  uint64_t ctw() const { return 2ull * L * n; }
  uint64_t keyw() const { return (uint64_t)L * 2 * (L + 1) * n; }
  uint64_t ptw() const { return (uint64_t)d_pad * L * n; }
};

namespace {

int set_err(wally_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  if (code == WALLY_EDEVICE && c) c->dead = true;
  return code;
}

#define HIP_OK(c, call)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return set_err((c), WALLY_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));  \
  } while (0)

int dalloc(wally_ctx* c, size_t bytes, void** p) {
  if (c->allocated + bytes > c->budget)
    return set_err(c, WALLY_ENOMEM, "device allocation of %zu bytes exceeds the budget (%llu of %llu in use)", bytes,
                   (unsigned long long)c->allocated, (unsigned long long)c->budget);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_err(c, WALLY_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  c->allocated += bytes;
  c->allocs.push_back({*p, bytes});
  return WALLY_OK;
}

void dfree(wally_ctx* c, void* p) {
  if (!p) return;
  for (size_t i = 0; i < c->allocs.size(); ++i)
    if (c->allocs[i].first == p) {
      c->allocated -= c->allocs[i].second;
      c->allocs.erase(c->allocs.begin() + i);
      break;
    }
  (void)hipFree(p);
}

int check_live(wally_ctx* c) {
  if (!c) return WALLY_EINVAL;
  if (c->dead) return WALLY_EDEVICE;
  HIP_OK(c, hipSetDevice(c->device));
  return WALLY_OK;
}

hipEvent_t pool_event(wally_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch through `fn`, bracketed by timing events on `st` when timing is on.
template <class F>
hipError_t timed(wally_ctx* c, hipStream_t st, int kernel, uint64_t items, F fn) {
  if (!c->timing || c->capturing) return fn();
  hipEvent_t a = pool_event(c), b = pool_event(c);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st);
  if (e == hipSuccess) e = fn();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  c->timers.push_back(TimerRec{kernel, items, a, b});
  return e;
}

// Launches of at least this many items form the inner products of the q_j
// rows inside the division by P (less HBM traffic; each workgroup then does
// more work, at two workgroups per CU); smaller launches keep them in the
// inner-product kernel, whose many small workgroups fill the chip sooner.
// The saving shows where another stream's kernels compete for HBM (the
// scoring waves); alone on one stream the two forms take the same time for
// 512 items and the stored form is faster for the PIR path's launches, so
// callers there pass may_fuse = false.
constexpr int kKsFuseItems = 256;

hipError_t keyswitch(wally_ctx* c, const KsItem* items, int n, const KsArgs& a, hipStream_t st,
                     bool may_fuse = true) {
  const bool fused = may_fuse && n >= kKsFuseItems;
  hipError_t e = timed(c, st, WALLY_KERNEL_DIGITS, n, [&] { return launch_ks_digits(items, n, a, c->M, st); });
  if (e == hipSuccess) e = timed(c, st, WALLY_KERNEL_EXTEND, n, [&] { return launch_ks_extend(items, n, a, c->M, st); });
  if (e == hipSuccess)
    e = timed(c, st, fused ? WALLY_KERNEL_INNER : WALLY_KERNEL_INNER_ALL, n,
              [&] { return launch_ks_inner(items, n, a, c->M, !fused, st); });
  if (e == hipSuccess) e = timed(c, st, WALLY_KERNEL_PINV, n, [&] { return launch_ks_pinv(n, a, c->M, st); });
  if (e == hipSuccess)
    e = timed(c, st, fused ? WALLY_KERNEL_MODDOWN : WALLY_KERNEL_MODDOWN_U, n,
              [&] { return launch_ks_moddown(items, n, a, c->M, fused, st); });
  return e;
}

// Scratch of wally_score_batch_static, for callers that cannot allocate:
// every workspace row and descriptor table of its waves.  Each GPU holds its
// own copy for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress gives on that device (static_scratch_of).
static __device__ __align__(256) unsigned char scratch[WALLY_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on device dev (current), looked up once per device.
hipError_t static_scratch_of(int dev, unsigned char** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = (unsigned char*)p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// Descriptor capacity of one static wave (pinned host staging and device
// table alike): copy and baby items per query, giant items and tiles.
constexpr uint64_t kStaticQueries = 1024, kStaticItems = 4096;
constexpr uint64_t kStaticCopyAt = 0, kStaticBabyAt = kStaticCopyAt + kStaticQueries * sizeof(CopyItem),
                   kStaticGiantAt = kStaticBabyAt + kStaticQueries * sizeof(KsItem),
                   kStaticTileAt = kStaticGiantAt + kStaticItems * sizeof(KsItem),
                   kStaticDescBytes = (kStaticTileAt + kStaticItems * sizeof(MacTile) + 255) / 256 * 256;
static_assert(kStaticDescBytes < WALLY_STATIC_SCRATCH_BYTES / 8, "descriptor tables take a small part of the scratch");

constexpr int kMaxWaveQueries = 1 << 15;
constexpr size_t kMaxWaveItems = (size_t)1 << 15;

void drop_graph(wally_ctx* c) {
  // a replay still in flight reads the descriptors and workspaces freed here
  if (c->graph_pending) (void)hipEventSynchronize(c->graph_done);
  c->graph_pending = false;
  for (hipGraphExec_t ex : c->graph_execs) (void)hipGraphExecDestroy(ex);
  c->graph_execs.clear();
  c->graph_key = 0;
  dfree(c, c->graph_desc);
  c->graph_desc = nullptr;
}

void free_sets(wally_ctx* c) {
  drop_graph(c);
  for (auto& s : c->sets) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    dfree(c, s.ctp);
    dfree(c, s.X);
    dfree(c, s.U);
    dfree(c, s.Y);
    dfree(c, s.D);
    dfree(c, s.R0);
    dfree(c, s.R1);
    dfree(c, s.ACC);
    dfree(c, s.tile_dev);
    if (s.tile_host) (void)hipHostFree(s.tile_host);
    dfree(c, s.copy_dev);
    dfree(c, s.baby_dev);
    dfree(c, s.giant_dev);
    if (s.copy_host) (void)hipHostFree(s.copy_host);
    if (s.baby_host) (void)hipHostFree(s.baby_host);
    if (s.giant_host) (void)hipHostFree(s.giant_host);
    if (s.staged) (void)hipEventDestroy(s.staged);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
  }
  c->sets.clear();
}

// Workspace sets for waves of up to B queries (allocated on first use and
// whenever the index changes the largest chunk count).
int ensure_sets(wally_ctx* c) {
  // wave size: the item grids of the key-switch kernels stay below 2^32 threads
  if (c->B < 1 || c->B > kMaxWaveQueries) return set_err(c, WALLY_EINVAL, "max_batch must be in 1..%d", kMaxWaveQueries);
  const size_t giant_cap = (size_t)c->B * std::max<uint32_t>(1, c->max_chunks);
  if (giant_cap > kMaxWaveItems)
    return set_err(c, WALLY_EINVAL, "max_batch x chunks of the largest cluster exceeds %zu items per wave", kMaxWaveItems);
  if (!c->sets.empty() && c->sets[0].giant_cap >= giant_cap) return WALLY_OK;
  free_sets(c);
  c->sets.resize(c->n_sets);
  const size_t B = c->B;
  const size_t w8 = sizeof(uint64_t);
  for (auto& s : c->sets) {
    int rc;
    if ((rc = dalloc(c, B * c->g * c->ctw() * w8, (void**)&s.ctp))) return rc;
    if ((rc = dalloc(c, B * c->L * c->n * w8, (void**)&s.X))) return rc;
    if ((rc = dalloc(c, B * 2 * (c->L + 1) * c->n * w8, (void**)&s.U))) return rc;
    if ((rc = dalloc(c, B * 2 * c->n * w8, (void**)&s.Y))) return rc;
    if ((rc = dalloc(c, B * (c->L + 1) * c->L * c->n * w8, (void**)&s.D))) return rc;
    if ((rc = dalloc(c, B * c->ctw() * w8, (void**)&s.R0))) return rc;
    if ((rc = dalloc(c, B * c->ctw() * w8, (void**)&s.R1))) return rc;
    if ((rc = dalloc(c, B * c->h * c->ctw() * w8, (void**)&s.ACC))) return rc;
    if ((rc = dalloc(c, giant_cap * sizeof(MacTile), (void**)&s.tile_dev))) return rc;
    HIP_OK(c, hipHostMalloc((void**)&s.tile_host, giant_cap * sizeof(MacTile), hipHostMallocDefault));
    if ((rc = dalloc(c, B * sizeof(CopyItem), (void**)&s.copy_dev))) return rc;
    if ((rc = dalloc(c, B * sizeof(KsItem), (void**)&s.baby_dev))) return rc;
    if ((rc = dalloc(c, giant_cap * sizeof(KsItem), (void**)&s.giant_dev))) return rc;
    HIP_OK(c, hipHostMalloc((void**)&s.copy_host, B * sizeof(CopyItem), hipHostMallocDefault));
    HIP_OK(c, hipHostMalloc((void**)&s.baby_host, B * sizeof(KsItem), hipHostMallocDefault));
    HIP_OK(c, hipHostMalloc((void**)&s.giant_host, giant_cap * sizeof(KsItem), hipHostMallocDefault));
    HIP_OK(c, hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
    HIP_OK(c, hipEventCreateWithFlags(&s.staged, hipEventDisableTiming));
    HIP_OK(c, hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
    s.giant_cap = giant_cap;
  }
  return WALLY_OK;
}

// Device bytes ensure_sets allocates for one workspace set (the descriptor
// tables included), at the current wave size and largest chunk count.
uint64_t set_bytes(const wally_ctx* c) {
  const uint64_t B = c->B, w8 = 8, giant_cap = B * std::max<uint32_t>(1, c->max_chunks);
  const uint64_t n = c->n, L = c->L, ctw = c->ctw();
  return w8 * B * (c->g * ctw + L * n + 2 * (L + 1) * n + 2 * n + (L + 1) * L * n + 2 * ctw + c->h * ctw) +
         giant_cap * (sizeof(MacTile) + sizeof(KsItem)) + B * (sizeof(CopyItem) + sizeof(KsItem));
}

// Serving admission charge of one request: the device memory it holds while
// it is in the library (its ciphertext, its keys and its response chunks).
uint64_t request_bytes(const wally_ctx* c, const wally_query& q) {
  const uint64_t fold_keys = c->K ? (uint64_t)__builtin_ctz(c->fold[q.cluster]) : 0;
  const uint64_t chunks = c->K ? c->chunks[q.cluster] : 1;
  return 8 * (c->ctw() + (2 + fold_keys) * c->keyw() + chunks * c->ctw());
}

KsArgs base_args(const wally_ctx* c, const WaveWork& s) {
  KsArgs a{};
  a.log_n = c->log_n;
  a.L = c->L;
  a.loge = c->ks_loge;
  a.g = c->g;
  a.giant = -1;
  a.X = s.X;
  a.U = s.U;
  a.Y = s.Y;
  a.D = s.D;
  return a;
}

// Enqueue the kernels of a planned wave on stream st, reading the
// descriptors from device memory.
int launch_wave(wally_ctx* c, WaveWork& s, const WavePlan& p, const CopyItem* copy, const KsItem* baby,
                const KsItem* giant, const MacTile* tiles, hipStream_t st) {
  const uint64_t ctw = c->ctw();
  const int w = p.w;
  const FoldCls& fc = p.cls;
  // baby steps: ct'_0 = ct, ct'_j = Rot(ct'_{j-1}, 1)
  HIP_OK(c, timed(c, st, WALLY_KERNEL_COPY, w, [&] { return launch_copy_ct(copy, w, ctw, st); }));
  for (int j = 1; j < (int)fc.g; ++j) {
    KsArgs a = base_args(c, s);
    a.gal = c->gal_baby;
    a.in_sel = 0;
    a.in_off = (uint64_t)(j - 1) * ctw;
    a.out_sel = 0;
    a.out_off = (uint64_t)j * ctw;
    HIP_OK(c, keyswitch(c, baby, w, a, st));
  }
  // giant steps per (query, chunk): acc_i for all i, then
  // R = acc_{h-1}; R = acc_i + Rot(R, g) for i = h-2 .. 0;
  // folded layout: then R = R + Rot(R, r) for r = d_pad/2, ..., d_pad/B
  const int n_fold = __builtin_ctz(fc.B);
  for (size_t sw = 0; sw < p.sub_tiles.size(); ++sw) {
    const size_t g0 = sw * (size_t)c->B;
    const int cnt = (int)std::min<size_t>(c->B, p.ng - g0);
    const KsItem* items = giant + g0;
    const MacTile* tl = tiles + p.sub_tiles[sw].first;
    const int ntile = (int)(p.sub_tiles[sw].second - p.sub_tiles[sw].first);
    KsArgs a = base_args(c, s);
    a.g = (int)fc.g;
    HIP_OK(c, timed(c, st, WALLY_KERNEL_MAC, cnt, [&] { return launch_mac_tiles(items, tl, ntile, a, fc.h, c->M, st); }));
    int cur = 3;  // acc
    uint64_t cur_off = (uint64_t)(fc.h - 1) * ctw;
    int next = 0;
    for (int i = (int)fc.h - 2; i >= 0; --i) {
      KsArgs b = base_args(c, s);
      b.gal = fc.gal_giant;
      b.in_sel = cur;
      b.in_off = cur_off;
      b.out_sel = i == 0 && n_fold == 0 ? 2 : next;
      b.giant = i;
      HIP_OK(c, keyswitch(c, items, cnt, b, st));
      cur = next;
      cur_off = 0;
      next = 1 - next;
    }
    for (int f = 0; f < n_fold; ++f) {
      KsArgs b = base_args(c, s);
      b.gal = (uint32_t)c->gal_fold[f];
      b.in_sel = cur;
      b.in_off = cur_off;
      b.out_sel = f == n_fold - 1 ? 2 : next;
      b.add_in = 1;
      b.key_fold = 1;
      b.key_off = (uint64_t)f * c->keyw();
      HIP_OK(c, keyswitch(c, items, cnt, b, st));
      cur = next;
      cur_off = 0;
      next = 1 - next;
    }
  }
  return WALLY_OK;
}

WaveBufs wave_bufs(const WaveWork& s) { return WaveBufs{s.ctp, s.R0, s.R1, s.ACC}; }

// Eager path: plan into the set's pinned buffers, copy, launch on its stream.
int enqueue_wave(wally_ctx* c, WaveWork& s, const wally_query* const* qs, int w) {
  // host descriptors may be rewritten only after the previous copy landed
  HIP_OK(c, hipEventSynchronize(s.staged));
  WavePlan p;
  plan_wave(c, wave_bufs(s), qs, w, s.copy_host, s.baby_host, s.giant_host, s.tile_host, p);
  HIP_OK(c, hipMemcpyAsync(s.copy_dev, s.copy_host, w * sizeof(CopyItem), hipMemcpyHostToDevice, s.stream));
  HIP_OK(c, hipMemcpyAsync(s.baby_dev, s.baby_host, w * sizeof(KsItem), hipMemcpyHostToDevice, s.stream));
  HIP_OK(c, hipMemcpyAsync(s.giant_dev, s.giant_host, p.ng * sizeof(KsItem), hipMemcpyHostToDevice, s.stream));
  HIP_OK(c, hipMemcpyAsync(s.tile_dev, s.tile_host, p.nt * sizeof(MacTile), hipMemcpyHostToDevice, s.stream));
  HIP_OK(c, hipEventRecord(s.staged, s.stream));
  int rc = launch_wave(c, s, p, s.copy_dev, s.baby_dev, s.giant_dev, s.tile_dev, s.stream);
  if (rc) return rc;
  HIP_OK(c, hipEventRecord(s.done, s.stream));
  return WALLY_OK;
}

int validate_query(wally_ctx* c, const wally_query& q, uint64_t idx) {
  if (q.cluster >= c->K) return set_err(c, WALLY_EINVAL, "query %llu: cluster %u out of range (K = %u)",
                                        (unsigned long long)idx, q.cluster, c->K);
  if (!q.ct || !q.key_baby || !q.key_giant || !q.out)
    return set_err(c, WALLY_EINVAL, "query %llu: null pointer", (unsigned long long)idx);
  if (c->fold[q.cluster] > 1 && !q.key_fold)
    return set_err(c, WALLY_EINVAL, "query %llu: cluster %u is folded (fold %u) and needs its fold keys",
                   (unsigned long long)idx, q.cluster, c->fold[q.cluster]);
  // every row is moved in 16-byte accesses: ciphertext, keys and output alike
  if (((uintptr_t)q.ct | (uintptr_t)q.out | (uintptr_t)q.key_baby | (uintptr_t)q.key_giant | (uintptr_t)q.key_fold) & 15)
    return set_err(c, WALLY_EINVAL, "query %llu: ct, keys and out must be 16-byte aligned", (unsigned long long)idx);
  return WALLY_OK;
}

}  // namespace

// ===========================================================================
// C ABI

extern "C" {

const char* wally_strerror(int code) {
  switch (code) {
    case WALLY_OK: return "ok";
    case WALLY_EINVAL: return "invalid argument";
    case WALLY_ENOMEM: return "out of device memory budget";
    case WALLY_EAGAIN: return "admission refused, retry later";
    case WALLY_EPENDING: return "pending";
    case WALLY_EDEVICE: return "device error";
    case WALLY_ESTATE: return "invalid state";
    default: return "unknown error";
  }
}

const char* wally_last_error(const wally_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int wally_params_init(const wally_params_desc* desc, wally_ctx** out) {
  if (!desc || !out) return WALLY_EINVAL;
  *out = nullptr;
  if (desc->log_n != 12 && desc->log_n != 13) return WALLY_EINVAL;
  if (desc->num_limbs < 1 || desc->num_limbs > kMaxLimbs) return WALLY_EINVAL;
  if (desc->max_batch > (uint32_t)kMaxWaveQueries) return WALLY_EINVAL;
  if (desc->limb_bits < 30 || desc->limb_bits > 54) return WALLY_EINVAL;  // 27-bit halves in the sums
  if (desc->t_bits < 2 || desc->t_bits + 2 > desc->limb_bits) return WALLY_EINVAL;
  // d_pad in 2..1024: the baby-step count g = 2^ceil(log2(d_pad)/2) is then
  // 2..32, the counts the giant-step sum kernel is instantiated for
  if (desc->dim < 2 || desc->dim > 1024) return WALLY_EINVAL;
  if (desc->layout != WALLY_LAYOUT_PER_CLUSTER && desc->layout != WALLY_LAYOUT_COPACK &&
      desc->layout != WALLY_LAYOUT_FOLDED)
    return WALLY_EINVAL;
  // fold_max: a power of two (at most 256, the fold keys gal_fold has room for) in the folded layout
  if (desc->layout != WALLY_LAYOUT_FOLDED && desc->fold_max != 0) return WALLY_EINVAL;
  if (desc->fold_max & (desc->fold_max - 1) || desc->fold_max > 256) return WALLY_EINVAL;
  wally_ctx* c = new (std::nothrow) wally_ctx();
  if (!c) return WALLY_ENOMEM;
  c->layout = desc->layout;
  c->fold_max = desc->layout == WALLY_LAYOUT_FOLDED ? (desc->fold_max ? desc->fold_max : 16) : 1;
  c->device = desc->device;
  c->log_n = desc->log_n;
  c->n = 1 << c->log_n;
  c->L = desc->num_limbs;
  c->d = desc->dim;
  int dp = 1;
  while (dp < c->d) dp *= 2;
  if ((c->n / 2) % dp) {
    delete c;
    return WALLY_EINVAL;
  }
  c->d_pad = dp;
  int lg = 0;
  while ((1 << lg) < dp) ++lg;
  c->g = 1 << ((lg + 1) / 2);
  c->h = dp / c->g;
  const uint64_t two_n = 2ull * c->n;
  c->gal_baby = 3;
  c->gal_giant = (uint32_t)powmod(3, c->g, two_n);
  for (int f = 0, r = dp / 2; f < 8 && r >= 1; ++f, r /= 2) c->gal_fold[f] = powmod(3, r, two_n);
  // moduli: L + 1 largest NTT-friendly primes below 2^limb_bits, then t
  {
    uint64_t top = (desc->limb_bits == 64) ? ~0ull : (1ull << desc->limb_bits) - 1;
    uint64_t cand = (top - 1) / two_n * two_n + 1;
    int found = 0;
    while (found < c->L + 1 && cand > two_n) {
      if (is_prime(cand)) c->mods[found++] = cand;
      cand -= two_n;
    }
    uint64_t t = ((1ull << desc->t_bits) / two_n) * two_n + 1;  // first t = 1 mod 2n above 2^t_bits
    if (t <= (1ull << desc->t_bits)) t += two_n;
    while (!is_prime(t)) t += two_n;
    c->mods[c->L + 1] = t;
  }
  const int nm = c->L + 2;
  for (int m = 0; m < nm; ++m) c->psi[m] = min_root(c->mods[m], two_n);

  if (hipSetDevice(c->device) != hipSuccess) {
    delete c;
    return WALLY_EINVAL;
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    delete c;
    return WALLY_EDEVICE;
  }
  c->budget = desc->hbm_budget ? desc->hbm_budget : (uint64_t)(free_b * 0.9);
  // default schedule: waves of 512 queries, two in flight.  Waves of 128 on
  // six streams can be 1-2% faster for whole batches, but in serving at low
  // rates six waves in flight slow each other down (p50 twice that of two).
  c->B = desc->max_batch ? (int)desc->max_batch : 512;
  c->n_sets = desc->wave_sets ? (int)desc->wave_sets : 2;
  if (c->n_sets > 8) c->n_sets = 8;

  // tables: per modulus n forward + n inverse (w, Shoup) pairs, then slot_of
  const size_t tw_words = (size_t)nm * 2 * c->n * 2;
  std::vector<uint64_t> host(tw_words);
  for (int m = 0; m < nm; ++m) {
    const uint64_t q = c->mods[m], ps = c->psi[m], psi_inv = powmod(ps, q - 2, q);
    uint64_t* f = host.data() + (size_t)m * 4 * c->n;
    uint64_t* iv = f + 2 * (size_t)c->n;
    uint64_t p1 = 1, p2 = 1;
    for (int k = 0; k < c->n; ++k) {
      const uint32_t r = bitrev(k, c->log_n);
      f[2 * r] = p1;
      f[2 * r + 1] = shoup_of(p1, q);
      iv[2 * r] = p2;
      iv[2 * r + 1] = shoup_of(p2, q);
      p1 = mulmod(p1, ps, q);
      p2 = mulmod(p2, psi_inv, q);
    }
    DevModuli& M = c->M;
    M.q[m] = q;
    M.mc[m].q = q;
    M.mc[m].q2 = 2 * q;
    M.mc[m].r64 = (uint64_t)(((u128)1 << 64) % q);
    M.mc[m].r64p = shoup_of(M.mc[m].r64, q);
    M.mc[m].onep = (uint64_t)((((u128)1) << 64) / q);
    M.ninv[m] = powmod(c->n % q, q - 2, q);
    M.ninvp[m] = shoup_of(M.ninv[m], q);
    M.c27[m] = (1ull << 27) % q;
    M.c27p[m] = shoup_of(M.c27[m], q);
  }
  const uint64_t P = c->mods[c->L];
  for (int j = 0; j < c->L; ++j) {
    const uint64_t q = c->mods[j];
    c->M.pinv[j] = powmod(P % q, q - 2, q);
    c->M.pinvp[j] = shoup_of(c->M.pinv[j], q);
  }
  if (!compress_constants(c->mods, c->L, c->log_n, c->mods[c->L + 1], c->comp)) {
    wally_destroy(c);
    return WALLY_EINVAL;
  }
  std::vector<uint32_t> slot_of(c->n);
  {
    const uint32_t half = c->n / 2;
    uint64_t e = 1;
    for (uint32_t col = 0; col < half; ++col) {
      slot_of[bitrev((uint32_t)((e - 1) / 2), c->log_n)] = col;
      slot_of[bitrev((uint32_t)((two_n - e - 1) / 2), c->log_n)] = half + col;
      e = e * 3 % two_n;
    }
  }
  int rc = dalloc(c, tw_words * 8, &c->tables);
  if (!rc) rc = dalloc(c, c->n * sizeof(uint32_t), (void**)&c->slot_of);
  if (rc) {
    wally_destroy(c);
    return rc;
  }
  if (hipMemcpy(c->tables, host.data(), tw_words * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->slot_of, slot_of.data(), c->n * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess) {
    wally_destroy(c);
    return WALLY_EDEVICE;
  }
  // the static scratch of this device, and what its entry point needs on the host
  if (static_scratch_of(c->device, &c->static_scratch) != hipSuccess ||
      hipEventCreateWithFlags(&c->static_done, hipEventDisableTiming) != hipSuccess) {
    wally_destroy(c);
    return WALLY_EDEVICE;
  }
  for (int k = 0; k < 2; ++k)
    if (hipHostMalloc((void**)&c->static_host[k], kStaticDescBytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->static_staged[k], hipEventDisableTiming) != hipSuccess) {
      wally_destroy(c);
      return WALLY_EDEVICE;
    }
  for (int m = 0; m < nm; ++m) {
    const ulonglong2* base = reinterpret_cast<const ulonglong2*>((uint64_t*)c->tables + (size_t)m * 4 * c->n);
    c->M.fwd[m] = base;
    c->M.inv[m] = base + c->n;
  }
  *out = c;
  return WALLY_OK;
}

int wally_params_query(const wally_ctx* c, wally_params_info* o) {
  if (!c || !o) return WALLY_EINVAL;
  memset(o, 0, sizeof *o);
  o->n = c->n;
  o->L = c->L;
  o->d = c->d;
  o->d_pad = c->d_pad;
  o->g = c->g;
  o->h = c->h;
  for (int j = 0; j < c->L; ++j) o->q[j] = c->mods[j];
  o->P = c->mods[c->L];
  o->t = c->mods[c->L + 1];
  for (int j = 0; j <= c->L; ++j) o->psi[j] = c->psi[j];
  o->psi_t = c->psi[c->L + 1];
  o->gal_baby = c->gal_baby;
  o->gal_giant = c->gal_giant;
  o->ct_words = c->ctw();
  o->key_words = c->keyw();
  o->pt_chunk_words = c->ptw();
  o->bytes_allocated = c->allocated;
  o->drop_bits[0] = c->comp.drop[0];
  o->drop_bits[1] = c->comp.drop[1];
  o->compressed_widths[0] = c->comp.width[0];
  o->compressed_widths[1] = c->comp.width[1];
  o->compressed_chunk_bytes = c->comp.part_bytes[0] + c->comp.part_bytes[1];
  o->hbm_budget = c->budget;
  o->serve_request_bytes = 8 * (2 * c->ctw() + 2 * c->keyw());
  // workspaces count as allocated once a session (or a scoring call) made them
  const uint64_t ws = c->sets.empty() ? (uint64_t)c->n_sets * set_bytes(c) : 0;
  const uint64_t used = c->allocated + ws;
  o->serve_inflight_limit = used < c->budget ? (c->budget - used) / o->serve_request_bytes : 0;
  return WALLY_OK;
}

}  // extern "C"

namespace {
int encode_clusters(wally_ctx* c, const void* emb, int elem, uint64_t n_entries, const uint64_t* offsets, uint32_t k);
}  // namespace

extern "C" {

int wally_encode_clusters(wally_ctx* c, const int8_t* emb, uint64_t n_entries, const uint64_t* offsets, uint32_t k) {
  return encode_clusters(c, emb, 1, n_entries, offsets, k);
}

int wally_encode_clusters_i16(wally_ctx* c, const int16_t* emb, uint64_t n_entries, const uint64_t* offsets,
                              uint32_t k) {
  return encode_clusters(c, emb, 2, n_entries, offsets, k);
}

}  // extern "C"

namespace {

int encode_clusters(wally_ctx* c, const void* emb, int elem, uint64_t n_entries, const uint64_t* offsets, uint32_t k) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->serving) return set_err(c, WALLY_ESTATE, "cannot re-encode while serving");
  if (!emb || !offsets || k == 0 || n_entries == 0) return set_err(c, WALLY_EINVAL, "empty or null index input");
  if (offsets[0] != 0 || offsets[k] != n_entries) return set_err(c, WALLY_EINVAL, "offsets must span [0, n_entries)");
  for (uint32_t i = 0; i < k; ++i)
    if (offsets[i + 1] <= offsets[i]) return set_err(c, WALLY_EINVAL, "cluster %u is empty or offsets decrease", i);
  ChunkLayout lay;
  plan_layout(c->layout, offsets, k, c->n, c->d_pad, c->fold_max, lay);
  const uint64_t total = lay.segs.size();
  // plaintexts per chunk: d_pad / fold of the chunk's cluster
  std::vector<uint32_t> chunk_fold(total, 1);
  for (uint32_t cl = 0; cl < k; ++cl)
    for (uint32_t j = 0; j < lay.chunks[cl]; ++j) chunk_fold[lay.first[cl] + j] = lay.fold[cl];
  std::vector<uint64_t> chunk_pt(total);
  uint64_t pt_words = 0;
  for (uint64_t ch = 0; ch < total; ++ch) {
    chunk_pt[ch] = pt_words;
    pt_words += c->ptw() / chunk_fold[ch];
  }
  // drop the previous index and workspaces, then allocate the new one
  free_sets(c);
  dfree(c, c->pt);
  c->pt = nullptr;
  c->K = 0;
  if ((rc = dalloc(c, pt_words * 8, (void**)&c->pt))) return rc;
  // rows in chunk order: a chunk's entries are consecutive rows from slot 0
  // (a copy only where clusters share chunks)
  const uint64_t row_bytes = (uint64_t)c->d * elem;
  std::vector<uint8_t> packed;
  const uint8_t* src = (const uint8_t*)emb;
  if (c->layout == WALLY_LAYOUT_COPACK) {
    packed.resize(n_entries * row_bytes);
    uint64_t r = 0;
    for (const auto& segs : lay.segs)
      for (const auto& sg : segs) {
        std::memcpy(packed.data() + r * row_bytes, src + (offsets[sg.cluster] + sg.offset) * row_bytes,
                    sg.count * row_bytes);
        r += sg.count;
      }
    src = packed.data();
  }
  uint8_t* demb = nullptr;
  EncodeJob* djobs = nullptr;
  if ((rc = dalloc(c, n_entries * row_bytes, (void**)&demb))) return rc;
  if ((rc = dalloc(c, total * sizeof(EncodeJob), (void**)&djobs))) {
    dfree(c, demb);
    return rc;
  }
  std::vector<EncodeJob> jobs(total);
  uint64_t row = 0;
  for (uint64_t ch = 0; ch < total; ++ch) {
    uint64_t cnt = 0;
    for (const auto& sg : lay.segs[ch]) cnt += sg.count;
    jobs[ch] = EncodeJob{demb + row * row_bytes, cnt, c->pt + chunk_pt[ch], chunk_fold[ch], fold_cls(c, chunk_fold[ch]).g};
    row += cnt;
  }
  hipError_t e = hipMemcpy(demb, src, n_entries * row_bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(djobs, jobs.data(), total * sizeof(EncodeJob), hipMemcpyHostToDevice);
  EncodeArgs a{c->log_n, c->L, (uint32_t)c->d, (uint32_t)c->d_pad, elem == 2 ? 1u : 0u, c->slot_of};
  const uint64_t step = 4096;
  for (uint64_t j0 = 0; e == hipSuccess && j0 < total; j0 += step)
    e = launch_encode(djobs + j0, (int)std::min(step, total - j0), a, c->M, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  dfree(c, demb);
  dfree(c, djobs);
  if (e != hipSuccess) return set_err(c, WALLY_EDEVICE, "encode failed: %s", hipGetErrorString(e));
  c->K = k;
  c->chunks = std::move(lay.chunks);
  c->chunk_base = std::move(lay.first);
  c->slot_base = std::move(lay.base);
  c->fold = std::move(lay.fold);
  c->chunk_pt = std::move(chunk_pt);
  c->max_chunks = *std::max_element(c->chunks.begin(), c->chunks.end());
  c->n_chunks_total = total;
  return WALLY_OK;
}

}  // namespace

extern "C" {

int wally_compress_responses(wally_ctx* c, const uint64_t* in, uint64_t chunks, uint8_t* out, void* hip_stream) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (chunks == 0) return WALLY_OK;
  if (!in || !out) return set_err(c, WALLY_EINVAL, "null response or output pointer");
  if ((uintptr_t)in & 7) return set_err(c, WALLY_EINVAL, "responses must be 8-byte aligned");
  if ((uintptr_t)out & 3) return set_err(c, WALLY_EINVAL, "the output must be 4-byte aligned");
  hipStream_t st = (hipStream_t)hip_stream;
  const uint64_t cbytes = c->comp.part_bytes[0] + c->comp.part_bytes[1];
  // two workgroups per response; launches of at most 2^30 workgroups
  for (uint64_t b0 = 0; b0 < chunks; b0 += kCompressBatch) {
    const int nb = (int)std::min(kCompressBatch, chunks - b0);
    HIP_OK(c, launch_resp_compress(in + b0 * c->ctw(), out + b0 * cbytes, nb, c->comp, c->M, st));
  }
  return WALLY_OK;
}

int wally_cluster_info(const wally_ctx* c, uint32_t cl, uint32_t* n_chunks, uint32_t* slot_base,
                       const uint64_t** plaintexts) {
  if (!c || cl >= c->K) return WALLY_EINVAL;
  if (n_chunks) *n_chunks = c->chunks[cl];
  if (slot_base) *slot_base = c->slot_base[cl];
  if (plaintexts) *plaintexts = c->pt + c->chunk_pt[c->chunk_base[cl]];
  return WALLY_OK;
}

int wally_cluster_fold(const wally_ctx* c, uint32_t cl, uint32_t* fold, uint32_t* g, uint32_t* h, uint64_t* gal_giant,
                       uint64_t* gal_fold) {
  if (!c || cl >= c->K) return WALLY_EINVAL;
  const FoldCls fc = fold_cls(c, c->fold[cl]);
  if (fold) *fold = fc.B;
  if (g) *g = fc.g;
  if (h) *h = fc.h;
  if (gal_giant) *gal_giant = fc.gal_giant;
  if (gal_fold)
    for (uint32_t f = 0; (1u << f) < fc.B; ++f) gal_fold[f] = c->gal_fold[f];
  return WALLY_OK;
}

}  // extern "C"

namespace {

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* p = (const unsigned char*)data;
  for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}

// Graph path: the batch's waves cut into segments of at most kGraphSegWaves
// waves; each segment (fork, its waves on the set streams, join) is captured
// into a graph of its own that reads its descriptors from its part of one
// device block, and a replay launches the segments in order on the caller's
// stream.  A capture of about 1,000 waves in one graph (some 150k kernel
// nodes, two chains of 75k) ended the process inside the capture; segments
// keep every graph within the size of the graphs that run.
constexpr size_t kGraphSegWaves = 48;

int capture_segment(wally_ctx* c, const SegmentPlan& sp, const unsigned char* dbase, size_t w0,
                    hipGraphExec_t* exec) {
  const CopyItem* copy_d = (const CopyItem*)(dbase + sp.copy_at);
  const KsItem* baby_d = (const KsItem*)(dbase + sp.baby_at);
  const KsItem* giant_d = (const KsItem*)(dbase + sp.giant_at);
  const MacTile* tile_d = (const MacTile*)(dbase + sp.tile_at);
  HIP_OK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  int rc = WALLY_OK;
  hipError_t e = hipEventRecord(c->fork, c->cap_stream);
  for (size_t k = 0; e == hipSuccess && k < c->sets.size(); ++k) e = hipStreamWaitEvent(c->sets[k].stream, c->fork, 0);
  for (size_t k = 0; e == hipSuccess && !rc && k < sp.plans.size(); ++k) {
    WaveWork& s = c->sets[(w0 + k) % c->sets.size()];
    rc = launch_wave(c, s, sp.plans[k], copy_d + sp.qoff[k], baby_d + sp.qoff[k], giant_d + sp.goff[k],
                     tile_d + sp.toff[k], s.stream);
  }
  for (size_t k = 0; e == hipSuccess && !rc && k < c->sets.size(); ++k) {
    e = hipEventRecord(c->sets[k].done, c->sets[k].stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->cap_stream, c->sets[k].done, 0);
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
  c->capturing = false;
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess || e2 != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return set_err(c, WALLY_EDEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return set_err(c, WALLY_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
  return WALLY_OK;
}

int build_graph(wally_ctx* c, const std::vector<const wally_query*>& ord,
                const std::vector<std::pair<uint64_t, uint64_t>>& waves) {
  drop_graph(c);
  const auto segs = graph_segments(waves.size(), kGraphSegWaves);
  auto bufs = [c](size_t wv) { return wave_bufs(c->sets[wv % c->sets.size()]); };
  std::vector<SegmentPlan> plans(segs.size());
  std::vector<std::vector<unsigned char>> blocks(segs.size());
  std::vector<size_t> at(segs.size());
  size_t total = 0;
  for (size_t k = 0; k < segs.size(); ++k) {
    plan_segment(c, ord, waves, segs[k].first, segs[k].second, bufs, blocks[k], plans[k]);
    at[k] = total;
    total += (plans[k].bytes + 255) / 256 * 256;
  }
  int rc = dalloc(c, std::max<size_t>(total, 256), &c->graph_desc);
  if (rc) return rc;
  unsigned char* dbase = (unsigned char*)c->graph_desc;
  for (size_t k = 0; k < segs.size(); ++k)
    HIP_OK(c, hipMemcpy(dbase + at[k], blocks[k].data(), plans[k].bytes, hipMemcpyHostToDevice));
  if (!c->cap_stream) HIP_OK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIP_OK(c, hipStreamSynchronize(c->cap_stream));
  for (auto& s : c->sets) HIP_OK(c, hipStreamSynchronize(s.stream));
  for (size_t k = 0; k < segs.size(); ++k) {
    hipGraphExec_t ex = nullptr;
    if ((rc = capture_segment(c, plans[k], dbase + at[k], segs[k].first, &ex))) return rc;
    c->graph_execs.push_back(ex);
  }
  return WALLY_OK;
}

int score_locked(wally_ctx* c, const wally_query* q, uint64_t nq, int path, hipStream_t user) {
  int rc;
  for (uint64_t i = 0; i < nq; ++i)
    if ((rc = validate_query(c, q[i], i))) return rc;
  if ((rc = ensure_sets(c))) return rc;
  if (path == WALLY_PATH_GRAPH) {
    uint64_t key = fnv1a(q, nq * sizeof(wally_query));
    key = fnv1a(&c->B, sizeof c->B, key);
    key = fnv1a(&c->tile_items, sizeof c->tile_items, key);
    key ^= (uint64_t)c->sets.size() << 56;
    if (c->graph_execs.empty() || c->graph_key != key) {
      std::vector<const wally_query*> ord;
      std::vector<std::pair<uint64_t, uint64_t>> waves;
      make_waves(c, q, nq, WALLY_PATH_BATCHED, ord, waves);
      if ((rc = build_graph(c, ord, waves))) {
        drop_graph(c);
        return rc;
      }
      c->graph_key = key;
    }
    // earlier eager work on the set streams shares the workspaces
    for (auto& s : c->sets) HIP_OK(c, hipStreamWaitEvent(user, s.done, 0));
    for (hipGraphExec_t ex : c->graph_execs) HIP_OK(c, hipGraphLaunch(ex, user));
    // later eager work may come on another stream: it waits for this event
    if (!c->graph_done) HIP_OK(c, hipEventCreateWithFlags(&c->graph_done, hipEventDisableTiming));
    HIP_OK(c, hipEventRecord(c->graph_done, user));
    c->graph_pending = true;
    return WALLY_OK;
  }
  std::vector<const wally_query*> ord;
  std::vector<std::pair<uint64_t, uint64_t>> waves;
  make_waves(c, q, nq, path, ord, waves);
  // fork: every set stream waits for the caller's stream (and a graph replay
  // still using the workspaces, whatever stream it was launched on)
  HIP_OK(c, hipEventRecord(c->fork, user));
  for (auto& s : c->sets) {
    HIP_OK(c, hipStreamWaitEvent(s.stream, c->fork, 0));
    if (c->graph_pending) HIP_OK(c, hipStreamWaitEvent(s.stream, c->graph_done, 0));
  }
  c->graph_pending = false;
  for (size_t wv = 0; wv < waves.size(); ++wv) {
    WaveWork& s = c->sets[wv % c->sets.size()];
    if ((rc = enqueue_wave(c, s, ord.data() + waves[wv].first, (int)(waves[wv].second - waves[wv].first)))) return rc;
  }
  // join
  for (auto& s : c->sets) {
    HIP_OK(c, hipEventRecord(s.done, s.stream));
    HIP_OK(c, hipStreamWaitEvent(user, s.done, 0));
  }
  return WALLY_OK;
}

}  // namespace

extern "C" {

int wally_score_batch(wally_ctx* c, const wally_query* q, uint64_t nq, int path, void* hip_stream) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->K == 0) return set_err(c, WALLY_ESTATE, "no clusters encoded");
  if (c->serving) return set_err(c, WALLY_ESTATE, "a serving session owns the workspaces");
  if (path != WALLY_PATH_BATCHED && path != WALLY_PATH_PLAIN && path != WALLY_PATH_GRAPH)
    return set_err(c, WALLY_EINVAL, "unknown path %d", path);
  if (nq == 0) return WALLY_OK;
  if (!q) return set_err(c, WALLY_EINVAL, "null query array");
  return score_locked(c, q, nq, path, (hipStream_t)hip_stream);
}

}  // extern "C"

namespace {

// Waves of queries scored in the static scratch: descriptor tables first,
// then one wave's workspace rows for `bs` queries.  c->B is bs while this runs.
int score_static_waves(wally_ctx* c, const wally_query* q, uint64_t nq, uint64_t bs, hipStream_t st) {
  const uint64_t n = c->n, L = c->L, ctw = c->ctw(), w8 = 8;
  unsigned char* at = c->static_scratch + kStaticDescBytes;
  auto carve = [&at](uint64_t bytes) {
    unsigned char* p = at;
    at += (bytes + 255) / 256 * 256;
    return (uint64_t*)p;
  };
  WaveWork ws;
  ws.ctp = carve(w8 * bs * c->g * ctw);
  ws.X = carve(w8 * bs * L * n);
  ws.U = carve(w8 * bs * 2 * (L + 1) * n);
  ws.Y = carve(w8 * bs * 2 * n);
  ws.D = carve(w8 * bs * (L + 1) * L * n);
  ws.R0 = carve(w8 * bs * ctw);
  ws.R1 = carve(w8 * bs * ctw);
  ws.ACC = carve(w8 * bs * c->h * ctw);
  if (at > c->static_scratch + WALLY_STATIC_SCRATCH_BYTES)
    return set_err(c, WALLY_EINVAL, "static scratch overrun (%llu queries per wave)", (unsigned long long)bs);
  unsigned char* dd = c->static_scratch;
  const CopyItem* copy_d = (const CopyItem*)(dd + kStaticCopyAt);
  const KsItem* baby_d = (const KsItem*)(dd + kStaticBabyAt);
  const KsItem* giant_d = (const KsItem*)(dd + kStaticGiantAt);
  const MacTile* tile_d = (const MacTile*)(dd + kStaticTileAt);
  // the previous static call of this context (whatever its stream) is done with the scratch
  if (c->static_pending) HIP_OK(c, hipStreamWaitEvent(st, c->static_done, 0));
  std::vector<const wally_query*> ord;
  std::vector<std::pair<uint64_t, uint64_t>> waves;
  make_waves(c, q, nq, WALLY_PATH_BATCHED, ord, waves);
  for (size_t wv = 0; wv < waves.size(); ++wv) {
    const int w = (int)(waves[wv].second - waves[wv].first);
    const int hb = (int)(wv & 1);
    unsigned char* hh = c->static_host[hb];
    // this staging half was last read by the copy of wave wv - 2
    HIP_OK(c, hipEventSynchronize(c->static_staged[hb]));
    WavePlan p;
    const wally_query* const* qs = ord.data() + waves[wv].first;
    if (wave_giant_items(c, qs, w) > kStaticItems)
      return set_err(c, WALLY_EINVAL, "static wave of %d queries has more than %llu giant items", w,
                     (unsigned long long)kStaticItems);
    plan_wave(c, wave_bufs(ws), qs, w, (CopyItem*)(hh + kStaticCopyAt), (KsItem*)(hh + kStaticBabyAt),
              (KsItem*)(hh + kStaticGiantAt), (MacTile*)(hh + kStaticTileAt), p);
    // same stream: these copies land after the previous wave's kernels read the tables
    HIP_OK(c, hipMemcpyAsync(dd + kStaticCopyAt, hh + kStaticCopyAt, w * sizeof(CopyItem), hipMemcpyHostToDevice, st));
    HIP_OK(c, hipMemcpyAsync(dd + kStaticBabyAt, hh + kStaticBabyAt, w * sizeof(KsItem), hipMemcpyHostToDevice, st));
    HIP_OK(c, hipMemcpyAsync(dd + kStaticGiantAt, hh + kStaticGiantAt, p.ng * sizeof(KsItem), hipMemcpyHostToDevice,
                             st));
    HIP_OK(c, hipMemcpyAsync(dd + kStaticTileAt, hh + kStaticTileAt, p.nt * sizeof(MacTile), hipMemcpyHostToDevice,
                             st));
    HIP_OK(c, hipEventRecord(c->static_staged[hb], st));
    int rc = launch_wave(c, ws, p, copy_d, baby_d, giant_d, tile_d, st);
    if (rc) return rc;
  }
  HIP_OK(c, hipEventRecord(c->static_done, st));
  c->static_pending = true;
  return WALLY_OK;
}

}  // namespace

extern "C" {

int wally_score_batch_static(wally_ctx* c, const wally_query* q, uint64_t nq, void* hip_stream) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->K == 0) return set_err(c, WALLY_ESTATE, "no clusters encoded");
  if (c->serving) return set_err(c, WALLY_ESTATE, "a serving session owns the device queues");
  if (nq == 0) return WALLY_OK;
  if (!q) return set_err(c, WALLY_EINVAL, "null query array");
  if (!c->static_scratch) return set_err(c, WALLY_ESTATE, "no static scratch on device %d", c->device);
  for (uint64_t i = 0; i < nq; ++i)
    if ((rc = validate_query(c, q[i], i))) return rc;
  // queries per wave: as many workspaces as the scratch holds beside the tables
  const uint64_t n = c->n, L = c->L, ctw = c->ctw(), w8 = 8, align = 8 * 256;
  const uint64_t per_query =
      w8 * (c->g * ctw + L * n + 2 * (L + 1) * n + 2 * n + (L + 1) * L * n + 2 * ctw + c->h * ctw);
  const uint64_t room = WALLY_STATIC_SCRATCH_BYTES - kStaticDescBytes - align;
  const uint64_t max_chunks = std::max<uint32_t>(1, c->max_chunks);
  const uint64_t bs = std::min({room / per_query, kStaticQueries, kStaticItems / max_chunks});
  if (bs == 0)
    return set_err(c, WALLY_EINVAL,
                   "the static scratch (%llu bytes) cannot hold one query: its workspace needs %llu bytes and its "
                   "%llu chunks %llu giant items (at most %llu)",
                   (unsigned long long)WALLY_STATIC_SCRATCH_BYTES, (unsigned long long)per_query,
                   (unsigned long long)max_chunks, (unsigned long long)max_chunks, (unsigned long long)kStaticItems);
  const int saved_b = c->B;
  const bool saved_timing = c->timing;
  c->B = (int)bs;
  c->timing = false;
  rc = score_static_waves(c, q, nq, bs, (hipStream_t)hip_stream);
  c->B = saved_b;
  c->timing = saved_timing;
  return rc;
}

int wally_tune(wally_ctx* c, const wally_query* q, uint64_t nq, const uint32_t* batches, const uint32_t* sets,
               const uint32_t* tiles, const uint32_t* radices, wally_tune_entry* out, uint32_t max_out,
               uint32_t* n_out) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->K == 0) return set_err(c, WALLY_ESTATE, "no clusters encoded");
  if (c->serving) return set_err(c, WALLY_ESTATE, "cannot tune while serving");
  if (!q || nq == 0) return set_err(c, WALLY_EINVAL, "empty query array");
  if (n_out) *n_out = 0;
  const uint32_t cur_b[2] = {(uint32_t)c->B, 0}, cur_s[2] = {(uint32_t)c->n_sets, 0}, cur_t[2] = {c->tile_items, 0},
                 cur_r[2] = {1u << c->ks_loge, 0};
  if (!batches || !batches[0]) batches = cur_b;
  if (!sets || !sets[0]) sets = cur_s;
  if (!tiles || !tiles[0]) tiles = cur_t;
  if (!radices || !radices[0]) radices = cur_r;
  for (const uint32_t* pr = radices; *pr; ++pr)
    if (*pr != 8 && *pr != 16) return set_err(c, WALLY_EINVAL, "NTT radix %u: 8 or 16", *pr);
  for (uint64_t i = 0; i < nq; ++i)
    if ((rc = validate_query(c, q[i], i))) return rc;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_OK(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  HIP_OK(c, hipEventCreate(&e0));
  HIP_OK(c, hipEventCreate(&e1));
  const bool timing = c->timing;
  c->timing = false;
  double best = 1e300;
  uint32_t bb = c->B, bs = c->n_sets, bt = c->tile_items, br = 1u << c->ks_loge, k = 0;
  for (const uint32_t* pb = batches; *pb && !rc; ++pb)
    for (const uint32_t* ps = sets; *ps && !rc; ++ps)
      for (const uint32_t* pt = tiles; *pt && !rc; ++pt)
        for (const uint32_t* pr = radices; *pr && !rc; ++pr) {
          free_sets(c);
          c->B = (int)*pb;
          c->n_sets = (int)std::min<uint32_t>(*ps, 8);
          c->tile_items = *pt;
          c->ks_loge = *pr == 8 ? 3 : 4;
          // warm-up (allocates the workspaces), then one timed batch
          if ((rc = score_locked(c, q, nq, WALLY_PATH_BATCHED, st))) break;
          hipError_t e = hipEventRecord(e0, st);
          if (e == hipSuccess) rc = score_locked(c, q, nq, WALLY_PATH_BATCHED, st);
          if (!rc && e == hipSuccess) e = hipEventRecord(e1, st);
          if (!rc && e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (!rc && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e != hipSuccess) rc = set_err(c, WALLY_EDEVICE, "tuning run failed: %s", hipGetErrorString(e));
          if (rc) break;
          if (out && k < max_out) out[k] = wally_tune_entry{*pb, (uint32_t)c->n_sets, *pt, *pr, (double)ms};
          ++k;
          if (ms < best) best = ms, bb = *pb, bs = (uint32_t)c->n_sets, bt = *pt, br = *pr;
        }
  if (n_out) *n_out = std::min(k, max_out);
  free_sets(c);
  c->B = (int)bb;
  c->n_sets = (int)bs;
  c->tile_items = bt;
  c->ks_loge = br == 8 ? 3 : 4;
  c->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  return rc;
}

}  // extern "C"

extern "C" {

// ---------------------------------------------------------------------------
// serving: continuous batching over the workspace sets.  A wave is launched
// whenever a set is idle and requests are pending; poll() retires finished
// waves and launches the next ones.

namespace {
static int serve_pump(wally_ctx* c) {
  int rc;
  for (auto& s : c->sets) {
    if (s.busy) {
      hipError_t e = hipEventQuery(s.done);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return set_err(c, WALLY_EDEVICE, "serving wave failed: %s", hipGetErrorString(e));
      for (uint64_t t : s.tickets) c->finished.push_back(t);
      s.tickets.clear();
      c->serve_bytes -= s.held_bytes;  // the requests' buffers are the caller's again
      s.held_bytes = 0;
      s.busy = false;
    }
    if (!s.busy && !c->pending.empty()) {
      std::vector<const wally_query*> qs;
      std::vector<ServeReq> taken;
      // the oldest request's fold class, then the later requests of that class in order
      const uint32_t cls = c->fold[c->pending.front().q.cluster];
      for (auto it = c->pending.begin(); it != c->pending.end() && (int)taken.size() < c->B;) {
        if (c->fold[it->q.cluster] == cls) {
          taken.push_back(*it);
          it = c->pending.erase(it);
        } else {
          ++it;
        }
      }
      for (auto& r : taken) qs.push_back(&r.q);
      if ((rc = enqueue_wave(c, s, qs.data(), (int)qs.size()))) return rc;
      // descriptors are copied by the enqueue; the request copies may go
      s.held_bytes = 0;
      for (auto& r : taken) s.tickets.push_back(r.ticket), s.held_bytes += r.bytes;
      s.busy = true;
    }
  }
  return WALLY_OK;
}
}  // namespace

int wally_serve_start(wally_ctx* c, void* hip_stream) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->serving) return set_err(c, WALLY_ESTATE, "already serving");
  if (c->K == 0) return set_err(c, WALLY_ESTATE, "no clusters encoded");
  if ((rc = ensure_sets(c))) return rc;
  c->serve_stream = (hipStream_t)hip_stream;
  HIP_OK(c, hipEventRecord(c->fork, c->serve_stream));
  for (auto& s : c->sets) {
    HIP_OK(c, hipStreamWaitEvent(s.stream, c->fork, 0));
    if (c->graph_pending) HIP_OK(c, hipStreamWaitEvent(s.stream, c->graph_done, 0));
  }
  c->graph_pending = false;
  c->pending.clear();
  c->finished.clear();
  c->serve_bytes = 0;
  for (auto& s : c->sets) s.held_bytes = 0;
  c->serving = true;
  return WALLY_OK;
}

int wally_serve_submit(wally_ctx* c, const wally_query* q, uint64_t* ticket) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->serving) return set_err(c, WALLY_ESTATE, "not serving");
  if (!q || !ticket) return set_err(c, WALLY_EINVAL, "null argument");
  if ((rc = validate_query(c, *q, 0))) return rc;
  // admission by HBM: index, tables and workspaces (allocated) + the requests
  // already admitted + this one must stay within the budget
  const uint64_t rb = request_bytes(c, *q);
  if (c->allocated + rb > c->budget)
    return set_err(c, WALLY_ENOMEM, "request of %llu bytes can never be admitted: %llu of the %llu-byte budget are allocated",
                   (unsigned long long)rb, (unsigned long long)c->allocated, (unsigned long long)c->budget);
  if (c->allocated + c->serve_bytes + rb > c->budget) {
    if ((rc = serve_pump(c))) return rc;  // retire finished waves first
    if (c->allocated + c->serve_bytes + rb > c->budget) return WALLY_EAGAIN;
  }
  *ticket = c->next_ticket++;
  c->serve_bytes += rb;
  c->pending.push_back(ServeReq{*q, *ticket, rb});
  return serve_pump(c);
}

int wally_serve_poll(wally_ctx* c, uint64_t* done, uint32_t max, uint32_t* n_done) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->serving) return set_err(c, WALLY_ESTATE, "not serving");
  if (!n_done || (max && !done)) return set_err(c, WALLY_EINVAL, "null argument");
  if ((rc = serve_pump(c))) return rc;
  uint32_t k = 0;
  while (k < max && !c->finished.empty()) {
    done[k++] = c->finished.front();
    c->finished.pop_front();
  }
  *n_done = k;
  return WALLY_OK;
}

int wally_serve_stop(wally_ctx* c) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->serving) return set_err(c, WALLY_ESTATE, "not serving");
  while (!c->pending.empty() || std::any_of(c->sets.begin(), c->sets.end(), [](const WaveWork& s) { return s.busy; })) {
    if ((rc = serve_pump(c))) return rc;
    for (auto& s : c->sets)
      if (s.busy) HIP_OK(c, hipEventSynchronize(s.done));
  }
  for (auto& s : c->sets) {
    HIP_OK(c, hipEventRecord(s.done, s.stream));
    HIP_OK(c, hipStreamWaitEvent(c->serve_stream, s.done, 0));
  }
  c->serving = false;
  return WALLY_OK;
}

void wally_destroy(wally_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  free_sets(c);
  if (c->pir_items_host) (void)hipHostFree(c->pir_items_host);
  if (c->pir_copy_host) (void)hipHostFree(c->pir_copy_host);
  if (c->pir_out_host) (void)hipHostFree(c->pir_out_host);
  if (c->pir_staged) (void)hipEventDestroy(c->pir_staged);
  if (c->pir_done) (void)hipEventDestroy(c->pir_done);
  while (!c->allocs.empty()) dfree(c, c->allocs.back().first);
  if (c->fork) (void)hipEventDestroy(c->fork);
  if (c->graph_done) (void)hipEventDestroy(c->graph_done);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (int k = 0; k < 2; ++k) {
    if (c->static_host[k]) (void)hipHostFree(c->static_host[k]);
    if (c->static_staged[k]) (void)hipEventDestroy(c->static_staged[k]);
  }
  if (c->static_done) (void)hipEventDestroy(c->static_done);
  for (auto& t : c->timers) c->ev_pool.push_back(t.a), c->ev_pool.push_back(t.b);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Index PIR for metadata fetch (paper §4.2, MulPIR): oblivious expansion of
// the query ciphertext by substitutions, with the paper's key reduction, the
// first dimension (plaintext products summed over the expanded rows) and the
// second dimension (ciphertext products with the second indicator, summed in
// an extended basis, scaled once and relinearized).

namespace {
constexpr uint32_t kPirWaveMax = 64;    // queries expanded together, at most
constexpr uint64_t kPirWaveBytes = 8ull << 30;  // expansion and product buffers of one wave, at most
constexpr int kPirKsItems = 1024;       // key-switch items per launch (scratch size)
constexpr uint32_t kPirMaxLevels = 11;  // 2^c <= 2048 expanded entries
constexpr uint32_t kPir2Cols = 16;      // columns of the second dimension per pass

// One query of either kind: rk is the relinearization key of a two-index query.
struct PirQ {
  const uint64_t* ct;
  const uint64_t* keys;
  const uint64_t* rk;
  uint64_t* out;
};

// Expansion depth, first key level, whether the second dimension runs and
// whether the last level is linearised.
struct PirMode {
  uint32_t c, a0;
  bool two, lin;
};

void pir_free_work(wally_ctx* c) {
  if (c->pir_done) (void)hipEventSynchronize(c->pir_done);  // answers in flight read the workspace
  if (c->pir_staged) (void)hipEventSynchronize(c->pir_staged);
  for (int k = 0; k < 2; ++k) {
    dfree(c, c->pir_lev[k]);
    dfree(c, c->pir_y[k]);
    c->pir_lev[k] = c->pir_y[k] = nullptr;
  }
  for (uint64_t** p : {&c->pir_X, &c->pir_U, &c->pir_Y, &c->pir_D, &c->pir2_col, &c->pir2_cf, &c->pir2_ext,
                       &c->pir2_x3, &c->pir2_c3, &c->pir_e3, &c->pir_cols3}) {
    dfree(c, *p);
    *p = nullptr;
  }
  dfree(c, c->pir_items_dev);
  dfree(c, c->pir_copy_dev);
  dfree(c, c->pir_out_dev);
  c->pir_items_dev = nullptr;
  c->pir_copy_dev = nullptr;
  c->pir_out_dev = nullptr;
  if (c->pir_items_host) (void)hipHostFree(c->pir_items_host);
  if (c->pir_copy_host) (void)hipHostFree(c->pir_copy_host);
  if (c->pir_out_host) (void)hipHostFree(c->pir_out_host);
  c->pir_items_host = nullptr;
  c->pir_copy_host = nullptr;
  c->pir_out_host = nullptr;
  c->pir_work_S = 0;
  c->pir_work_two = false;
  c->pir_work_lin = false;
}

// Device bytes per query of a wave: the two expansion lists and the two
// substitution buffers (3 S ciphertexts), for the second dimension the
// columns, one pass's coefficient and auxiliary rows, the tensor sums and the
// scaled product, and for a linearised last level the third parts (S rows of
// L n) and the three-part columns (4 L n words each).
uint64_t pir_query_bytes(const wally_ctx* c, uint64_t S, bool two, bool lin, uint32_t kc) {
  const uint64_t ctw = c->ctw(), n = c->n, L = c->L, Lb = c->pir_Lb;
  uint64_t w = 3 * S * ctw;
  if (two) w += (uint64_t)c->pir_d2 * ctw + kc * 2 * ctw + kc * 4 * Lb * n + 3 * (L + Lb) * n + 4 * L * n;
  if (lin) w += S * L * n + (uint64_t)c->pir_d2 * 4 * L * n;
  return 8 * w;
}

int pir_alloc_work(wally_ctx* c, uint64_t S, bool two, bool lin) {
  const size_t w8 = 8, ctw = c->ctw(), n = c->n, L = c->L, Lb = c->pir_Lb;
  const uint32_t kc = two ? std::min(c->pir_d2, kPir2Cols) : 0;
  c->pir_wq = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>(kPirWaveMax, kPirWaveBytes / pir_query_bytes(c, S, two, lin, kc)));
  const size_t W = c->pir_wq;
  // per query: substitutions (S - 1), one relinearization, and with a
  // linearised last level one key switch per column and up to S / 2
  // automorphism items
  const size_t items = W * (S + (lin ? S / 2 + c->pir_d2 : 0));
  int rc;
  for (int k = 0; k < 2; ++k) {
    if ((rc = dalloc(c, W * S * ctw * w8, (void**)&c->pir_lev[k]))) return rc;
    if ((rc = dalloc(c, W * (S / 2) * ctw * w8, (void**)&c->pir_y[k]))) return rc;
  }
  if ((rc = dalloc(c, kPirKsItems * L * n * w8, (void**)&c->pir_X))) return rc;
  if ((rc = dalloc(c, kPirKsItems * 2 * (L + 1) * n * w8, (void**)&c->pir_U))) return rc;
  if ((rc = dalloc(c, kPirKsItems * 2 * n * w8, (void**)&c->pir_Y))) return rc;
  if ((rc = dalloc(c, kPirKsItems * (L + 1) * L * n * w8, (void**)&c->pir_D))) return rc;
  if (two) {
    if ((rc = dalloc(c, W * c->pir_d2 * ctw * w8, (void**)&c->pir2_col))) return rc;
    if ((rc = dalloc(c, W * kc * 2 * ctw * w8, (void**)&c->pir2_cf))) return rc;
    if ((rc = dalloc(c, W * kc * 4 * Lb * n * w8, (void**)&c->pir2_ext))) return rc;
    if ((rc = dalloc(c, W * 3 * (L + Lb) * n * w8, (void**)&c->pir2_x3))) return rc;
    if ((rc = dalloc(c, W * 4 * L * n * w8, (void**)&c->pir2_c3))) return rc;
    c->pir2_kc = kc;
  }
  if (lin) {
    if ((rc = dalloc(c, W * S * L * n * w8, (void**)&c->pir_e3))) return rc;
    if ((rc = dalloc(c, W * c->pir_d2 * 4 * L * n * w8, (void**)&c->pir_cols3))) return rc;
  }
  if ((rc = dalloc(c, items * sizeof(KsItem), (void**)&c->pir_items_dev))) return rc;
  if ((rc = dalloc(c, W * sizeof(CopyItem), (void**)&c->pir_copy_dev))) return rc;
  if ((rc = dalloc(c, W * sizeof(uint64_t*), (void**)&c->pir_out_dev))) return rc;
  HIP_OK(c, hipHostMalloc((void**)&c->pir_items_host, items * sizeof(KsItem), hipHostMallocDefault));
  HIP_OK(c, hipHostMalloc((void**)&c->pir_copy_host, W * sizeof(CopyItem), hipHostMallocDefault));
  HIP_OK(c, hipHostMalloc((void**)&c->pir_out_host, W * sizeof(uint64_t*), hipHostMallocDefault));
  if (!c->pir_staged) HIP_OK(c, hipEventCreateWithFlags(&c->pir_staged, hipEventDisableTiming));
  c->pir_work_S = S;
  c->pir_work_two = two;
  c->pir_work_lin = lin;
  return WALLY_OK;
}

// The PIR workspace for a mode, all or nothing: a workspace made for another
// expansion size or without the second dimension's buffers is replaced (after
// the answers in flight), and a failed allocation frees what was taken.
int pir_ensure_work(wally_ctx* c, const PirMode& md) {
  const uint64_t S = 1ull << md.c;
  if (c->pir_lev[0] && c->pir_work_S == S && (c->pir_work_two || !md.two) && (c->pir_work_lin || !md.lin))
    return WALLY_OK;
  pir_free_work(c);
  const int rc = pir_alloc_work(c, S, md.two, md.lin);
  if (rc) pir_free_work(c);
  return rc;
}

// Whether pair b of the last level of a linearised expansion is linearised:
// neither of its outputs b, b + S/2 is a column entry of a two-index query.
bool pir_pair_linear(const wally_ctx* c, const PirMode& md, uint64_t b) {
  if (!md.two) return true;
  const uint64_t half = 1ull << (md.c - 1), lo = c->pir_d1, hi = (uint64_t)c->pir_d1 + c->pir_d2;
  return !((b >= lo && b < hi) || (b + half >= lo && b + half < hi));
}

// Expansion of up to pir_wq queries on stream st, then the first dimension
// (into the callers' outputs, or the column buffer for two-index queries),
// then, for two-index queries, the second dimension into the outputs.  With
// a linearised last level the pairs it covers take the automorphism alone
// (k_pir_lin_split), the first dimension sums three parts, and one key switch per
// column (identity automorphism, the key of the last level) finishes them.
int pir_wave(wally_ctx* c, const PirMode& md, const PirQ* q, uint32_t w, hipStream_t st) {
  const uint64_t ctw = c->ctw(), S = 1ull << md.c, keyw = c->keyw();
  HIP_OK(c, hipEventSynchronize(c->pir_staged));  // host descriptors of the last wave were copied
  // descriptors: copies, substitution items of every level, relinearization
  // items, column items, automorphism items, outputs
  size_t base = 0;
  std::vector<size_t> lev_base(md.c), lev_count(md.c);
  for (uint32_t a = 0; a < md.c; ++a) {
    lev_base[a] = base;
    const uint64_t half = 1ull << a;
    const uint32_t ka = std::max(a, md.a0);
    const bool last_lin = md.lin && a + 1 == md.c;
    uint64_t* cur = c->pir_lev[a & 1];
    for (uint32_t i = 0; i < w; ++i)
      for (uint64_t b = 0; b < half; ++b) {
        if (last_lin && pir_pair_linear(c, md, b)) continue;
        KsItem it{};
        it.key = q[i].keys + (uint64_t)(ka - md.a0) * keyw;
        it.buf0 = cur + (i * S + b) * ctw;
        it.buf1 = c->pir_y[0] + (i * (S / 2) + b) * ctw;
        it.fin = c->pir_y[1] + (i * (S / 2) + b) * ctw;
        c->pir_items_host[base++] = it;
      }
    lev_count[a] = base - lev_base[a];
  }
  const size_t relin_base = base;
  const uint64_t p3w = 4ull * c->L * c->n;  // words of one scaled product (c0, c2, 0, c1)
  if (md.two)
    for (uint32_t i = 0; i < w; ++i) {
      // key switch of (c0, c2) with the identity automorphism, + (0, c1): (c0, c1) + KS(c2)
      KsItem it{};
      it.key = q[i].rk;
      it.buf0 = c->pir2_c3 + i * p3w;
      it.acc = c->pir2_c3 + i * p3w + p3w / 2;
      it.fin = q[i].out;
      c->pir_items_host[base++] = it;
    }
  // linearised last level: the column key switches, then the automorphism items
  const uint64_t c3w = 4ull * c->L * c->n;  // words of one three-part column [U0][U2][0][U1]
  const size_t col_base = base;
  if (md.lin)
    for (uint32_t i = 0; i < w; ++i)
      for (uint32_t k = 0; k < c->pir_d2; ++k) {
        KsItem it{};
        it.key = q[i].keys + (uint64_t)(md.c - 1 - md.a0) * keyw;
        it.buf0 = c->pir_cols3 + ((uint64_t)i * c->pir_d2 + k) * c3w;
        it.acc = it.buf0 + c3w / 2;
        it.fin = (md.two ? c->pir2_col + (uint64_t)i * c->pir_d2 * ctw : q[i].out) + (uint64_t)k * ctw;
        c->pir_items_host[base++] = it;
      }
  const size_t sig_base = base;
  if (md.lin) {
    uint64_t* cur = c->pir_lev[(md.c - 1) & 1];
    uint64_t* nxt = c->pir_lev[md.c & 1];
    const uint64_t half = S / 2;
    for (uint32_t i = 0; i < w; ++i)
      for (uint64_t b = 0; b < half; ++b)
        if (pir_pair_linear(c, md, b)) {
          KsItem it{};
          it.buf0 = cur + (i * S + b) * ctw;
          it.buf1 = nxt + (i * S + b) * ctw;
          it.fin = c->pir_e3 + (i * S + b) * c->L * c->n;
          c->pir_items_host[base++] = it;
        }
  }
  for (uint32_t i = 0; i < w; ++i) {
    c->pir_copy_host[i] = CopyItem{q[i].ct, c->pir_lev[0] + i * S * ctw};
    c->pir_out_host[i] = md.lin   ? c->pir_cols3 + (uint64_t)i * c->pir_d2 * c3w
                         : md.two ? c->pir2_col + (uint64_t)i * c->pir_d2 * ctw
                                  : q[i].out;
  }
  HIP_OK(c, hipMemcpyAsync(c->pir_items_dev, c->pir_items_host, base * sizeof(KsItem), hipMemcpyHostToDevice, st));
  HIP_OK(c, hipMemcpyAsync(c->pir_copy_dev, c->pir_copy_host, w * sizeof(CopyItem), hipMemcpyHostToDevice, st));
  HIP_OK(c, hipMemcpyAsync(c->pir_out_dev, c->pir_out_host, w * sizeof(uint64_t*), hipMemcpyHostToDevice, st));
  HIP_OK(c, hipEventRecord(c->pir_staged, st));
  HIP_OK(c, timed(c, st, WALLY_KERNEL_COPY, w, [&] { return launch_copy_ct(c->pir_copy_dev, (int)w, ctw, st); }));
  auto ks_args = [c](uint32_t gal, int in_sel, int out_sel) {
    KsArgs k{};
    k.log_n = c->log_n;
    k.L = c->L;
    k.loge = c->ks_loge;
    k.gal = gal;
    k.in_sel = in_sel;
    k.out_sel = out_sel;
    k.giant = -1;
    k.g = c->g;
    k.X = c->pir_X;
    k.U = c->pir_U;
    k.Y = c->pir_Y;
    k.D = c->pir_D;
    return k;
  };
  for (uint32_t a = 0; a < md.c; ++a) {
    const uint64_t half = 1ull << a;
    const uint32_t ka = std::max(a, md.a0);
    const uint32_t reps = 1u << (ka - a);  // Subs(., g_ka) applied 2^(ka - a) times is Subs(., g_a)
    const int n_items = (int)(w * half);
    const int n_ks = (int)lev_count[a];
    const bool last_lin = md.lin && a + 1 == md.c;  // then ka = a and reps = 1 (a0 <= c - 1)
    int last_out = 1;
    for (uint32_t r = 0; r < reps; ++r) {
      // x, then alternately y0, y1
      const KsArgs ka_args = ks_args(c->n / (1u << ka) + 1, r == 0 ? 0 : (r % 2 == 1 ? 1 : 2), r % 2 == 0 ? 1 : 2);
      for (int i0 = 0; i0 < n_ks; i0 += kPirKsItems)
        HIP_OK(c, keyswitch(c, c->pir_items_dev + lev_base[a] + i0, std::min(kPirKsItems, n_ks - i0), ka_args, st,
                            false));
      last_out = ka_args.out_sel;
    }
    PirSplitArgs sa{};
    sa.cur = c->pir_lev[a & 1];
    sa.ybuf = c->pir_y[last_out == 1 ? 0 : 1];
    sa.next = c->pir_lev[(a + 1) & 1];
    sa.w = c->pir_w + (uint64_t)a * c->L * c->n;
    sa.stride = (uint32_t)S;
    sa.ystride = (uint32_t)(S / 2);
    sa.half = (uint32_t)half;
    sa.log_n = c->log_n;
    sa.L = c->L;
    if (last_lin) {
      sa.e3 = c->pir_e3;
      sa.col_lo = md.two ? c->pir_d1 : 0;
      sa.col_hi = md.two ? c->pir_d1 + c->pir_d2 : 0;
      HIP_OK(c, launch_pir_lin_split(c->pir_items_dev + sig_base, (int)(base - sig_base), sa, c->n / (1u << a) + 1,
                                     c->M, st));
    }
    if (!last_lin || n_ks > 0) HIP_OK(c, launch_pir_split(sa, n_items, c->M, st));
  }
  const uint64_t* E = c->pir_lev[md.c & 1];
  PirDotArgs da{};
  da.E = E;
  da.pt = c->pir_pt;
  da.out = c->pir_out_dev;
  da.stride = (uint32_t)S;
  da.d1 = c->pir_d1;
  da.d2 = c->pir_d2;
  da.nq = w;
  da.log_n = c->log_n;
  da.L = c->L;
  da.E3 = md.lin ? c->pir_e3 : nullptr;
  HIP_OK(c, timed(c, st, WALLY_KERNEL_MAC, w, [&] { return launch_pir_dot(da, c->M, st); }));
  if (md.lin) {  // (U0, U1) + KeySwitch(U2): identity automorphism on (U0, U2), + (0, U1)
    KsArgs fa = ks_args(1, 0, 2);
    fa.giant = 0;
    const int n_cols = (int)(sig_base - col_base);
    for (int i0 = 0; i0 < n_cols; i0 += kPirKsItems)
      HIP_OK(c, keyswitch(c, c->pir_items_dev + col_base + i0, std::min(kPirKsItems, n_cols - i0), fa, st, false));
  }
  if (!md.two) return WALLY_OK;
  // second dimension, columns in passes of pir2_kc
  Pir2Args pa{};
  pa.K = c->pir2_K;
  pa.col = c->pir2_col;
  pa.E = E;
  pa.cf = c->pir2_cf;
  pa.ext = c->pir2_ext;
  pa.x3 = c->pir2_x3;
  pa.c3 = c->pir2_c3;
  pa.stride = (uint32_t)S;
  pa.d1 = c->pir_d1;
  pa.d2 = c->pir_d2;
  pa.nq = w;
  pa.log_n = c->log_n;
  pa.L = c->L;
  pa.Lb = (int)c->pir_Lb;
  for (uint32_t k0 = 0; k0 < c->pir_d2; k0 += c->pir2_kc) {
    pa.k0 = k0;
    pa.kc = std::min(c->pir2_kc, c->pir_d2 - k0);
    pa.accumulate = k0 > 0;
    HIP_OK(c, launch_pir2_coef(pa, c->M, st));
    HIP_OK(c, launch_pir2_extend(pa, st));
    HIP_OK(c, launch_rows_ntt(c->pir2_ext, (int)(w * pa.kc * 4 * c->pir_Lb), c->log_n, c->pir2_K, c->L,
                              (int)c->pir_Lb, 0, st));
    HIP_OK(c, launch_pir2_tensor(pa, st));
  }
  const int MB = c->L + (int)c->pir_Lb;
  HIP_OK(c, launch_rows_ntt(c->pir2_x3, (int)(w * 3 * MB), c->log_n, c->pir2_K, 0, MB, 1, st));
  HIP_OK(c, launch_pir2_scale(pa, st));
  HIP_OK(c, launch_rows_ntt(c->pir2_c3, (int)(w * 4 * c->L), c->log_n, c->pir2_K, 0, c->L, 0, st));
  KsArgs rl = ks_args(1, 0, 2);
  rl.giant = 0;  // + acc = (0, c1)
  HIP_OK(c, keyswitch(c, c->pir_items_dev + relin_base, (int)w, rl, st, false));
  return WALLY_OK;
}

// little-endian multi-word integers (host)
std::vector<uint64_t> mw_prod(const uint64_t* p, int count, int skip = -1) {
  std::vector<uint64_t> x{1};
  for (int i = 0; i < count; ++i)
    if (i != skip) mw_mul_small(x, p[i]);
  return x;
}
int mw_cmp(const std::vector<uint64_t>& a, const std::vector<uint64_t>& b) {
  for (size_t k = std::max(a.size(), b.size()); k-- > 0;) {
    const uint64_t x = k < a.size() ? a[k] : 0, y = k < b.size() ? b[k] : 0;
    if (x != y) return x < y ? -1 : 1;
  }
  return 0;
}
void mw_add_small(std::vector<uint64_t>& x, uint64_t v) {
  for (uint64_t& w : x) {
    const uint64_t s = w + v;
    v = s < w;
    w = s;
    if (!v) return;
  }
  if (v) x.push_back(v);
}

// Constants of the exact conversion from the primes src[0..ns) to tgt[0..nt).
bool make_conv(const uint64_t* src, int ns, const uint64_t* tgt, int nt, BaseConv& C) {
  C = BaseConv{};
  C.ns = (uint32_t)ns;
  C.nt = (uint32_t)nt;
  const std::vector<uint64_t> S = mw_prod(src, ns);
  // the multi-word sums stay below ns S
  std::vector<uint64_t> bound = S;
  mw_mul_small(bound, (uint64_t)ns);
  if (bound.size() > (size_t)kMaxConvWords) return false;
  for (size_t w = 0; w < S.size(); ++w) C.S[w] = S[w];
  for (size_t w = 0; w < S.size(); ++w) C.half[w] = (S[w] >> 1) | (w + 1 < S.size() ? S[w + 1] << 63 : 0);
  for (int i = 0; i < ns; ++i) {
    const uint64_t si = src[i];
    C.s[i] = si;
    const std::vector<uint64_t> hat = mw_prod(src, ns, i);
    for (size_t w = 0; w < hat.size(); ++w) C.hat[i][w] = hat[w];
    C.inv[i] = powmod(mw_mod_small(hat, si), si - 2, si);
    C.invp[i] = shoup_of(C.inv[i], si);
    for (int j = 0; j < nt; ++j) {
      C.hat_t[i][j] = mw_mod_small(hat, tgt[j]);
      C.hat_tp[i][j] = shoup_of(C.hat_t[i][j], tgt[j]);
    }
  }
  for (int j = 0; j < nt; ++j) {
    C.t[j] = tgt[j];
    C.S_t[j] = mw_mod_small(S, tgt[j]);
    C.S_tp[j] = shoup_of(C.S_t[j], tgt[j]);
  }
  return true;
}

// The extended basis of the second dimension for a table with d2 columns:
// auxiliary primes (the NTT-friendly primes of the ciphertext primes' size
// that come after P, descending) until their product B exceeds t d2 n Q + 2,
// their transform tables, and every conversion and scaling constant.
int pir2_setup(wally_ctx* c, uint32_t d2) {
  dfree(c, c->pir2_K);
  dfree(c, c->pir2_tables);
  c->pir2_K = nullptr;
  c->pir2_tables = nullptr;
  c->pir_Lb = 0;
  const uint64_t two_n = 2ull * c->n, t = c->mods[c->L + 1];
  std::vector<uint64_t> need = mw_prod(c->mods, c->L);  // Q
  mw_mul_small(need, t);
  mw_mul_small(need, d2);
  mw_mul_small(need, (uint64_t)c->n);
  mw_add_small(need, 2);
  std::vector<uint64_t> aux, B{1};
  for (uint64_t cand = c->mods[c->L] - two_n; mw_cmp(B, need) <= 0; cand -= two_n) {
    if (cand <= two_n || aux.size() >= (size_t)kMaxAux)
      return set_err(c, WALLY_EINVAL, "no auxiliary basis of at most %d primes for %u columns", kMaxAux, d2);
    if (!is_prime(cand) || cand == t) continue;
    aux.push_back(cand);
    mw_mul_small(B, cand);
  }
  const int L = c->L, Lb = (int)aux.size(), n = c->n;
  Pir2Consts K{};
  K.L = (uint32_t)L;
  K.Lb = (uint32_t)Lb;
  // transform tables of the auxiliary primes, [Lb][fwd n | inv n]
  std::vector<ulonglong2> tab((size_t)Lb * 2 * n);
  for (int b = 0; b < Lb; ++b) {
    const uint64_t q = aux[b], ps = min_root(q, two_n), pinv = powmod(ps, q - 2, q);
    uint64_t p1 = 1, p2 = 1;
    for (int k = 0; k < n; ++k) {
      const uint32_t r = bitrev(k, c->log_n);
      tab[(size_t)b * 2 * n + r] = make_ulonglong2(p1, shoup_of(p1, q));
      tab[(size_t)b * 2 * n + n + r] = make_ulonglong2(p2, shoup_of(p2, q));
      p1 = mulmod(p1, ps, q);
      p2 = mulmod(p2, pinv, q);
    }
  }
  int rc = dalloc(c, tab.size() * sizeof(ulonglong2), (void**)&c->pir2_tables);
  if (rc) return rc;
  HIP_OK(c, hipMemcpy(c->pir2_tables, tab.data(), tab.size() * sizeof(ulonglong2), hipMemcpyHostToDevice));
  std::vector<uint64_t> base(c->mods, c->mods + L);
  base.insert(base.end(), aux.begin(), aux.end());
  for (int m = 0; m < L + Lb; ++m) {
    RowMod& r = K.mod[m];
    const uint64_t q = base[m];
    r.q = q;
    r.ninv = powmod(c->n % q, q - 2, q);
    r.ninvp = shoup_of(r.ninv, q);
    r.onep = (uint64_t)((((u128)1) << 64) / q);
    r.r64 = (uint64_t)(((u128)1 << 64) % q);
    r.r64p = shoup_of(r.r64, q);
    if (m < L) {
      r.fwd = c->M.fwd[m];
      r.inv = c->M.inv[m];
    } else {
      r.fwd = c->pir2_tables + (size_t)(m - L) * 2 * n;
      r.inv = r.fwd + n;
    }
    K.t_m[m] = t % q;
    K.t_mp[m] = shoup_of(K.t_m[m], q);
  }
  const std::vector<uint64_t> Q = mw_prod(c->mods, L);
  std::vector<uint64_t> hq(Q.size());
  for (size_t w = 0; w < Q.size(); ++w) hq[w] = (Q[w] >> 1) | (w + 1 < Q.size() ? Q[w + 1] << 63 : 0);
  for (int m = 0; m < L + Lb; ++m) K.h_m[m] = mw_mod_small(hq, base[m]);
  for (int b = 0; b < Lb; ++b) {
    K.qinv_b[b] = powmod(mw_mod_small(Q, aux[b]), aux[b] - 2, aux[b]);
    K.qinv_bp[b] = shoup_of(K.qinv_b[b], aux[b]);
  }
  K.t = t;
  if (!make_conv(c->mods, L, aux.data(), Lb, K.q_to_b) || !make_conv(aux.data(), Lb, c->mods, L, K.b_to_q))
    return set_err(c, WALLY_EINVAL, "extended basis beyond the conversion word limit");
  if ((rc = dalloc(c, sizeof(Pir2Consts), (void**)&c->pir2_K))) return rc;
  HIP_OK(c, hipMemcpy(c->pir2_K, &K, sizeof(Pir2Consts), hipMemcpyHostToDevice));
  c->pir_Lb = (uint32_t)Lb;
  return WALLY_OK;
}

// Validation of a batch and the workspace, then the waves (one or two dimensions).
int pir_answer_any(wally_ctx* c, const PirMode& md, const std::vector<PirQ>& qs, hipStream_t st) {
  int rc;
  if ((rc = pir_ensure_work(c, md))) return rc;
  // the workspace is shared: this call's work follows the last call's, whatever stream that was on
  if (c->pir_done) HIP_OK(c, hipStreamWaitEvent(st, c->pir_done, 0));
  else HIP_OK(c, hipEventCreateWithFlags(&c->pir_done, hipEventDisableTiming));
  for (uint64_t i0 = 0; i0 < qs.size(); i0 += c->pir_wq)
    if ((rc = pir_wave(c, md, qs.data() + i0, (uint32_t)std::min<uint64_t>(c->pir_wq, qs.size() - i0), st))) return rc;
  HIP_OK(c, hipEventRecord(c->pir_done, st));
  return WALLY_OK;
}
}  // namespace

extern "C" {

int wally_pir_encode(wally_ctx* c, const uint32_t* coeffs, uint32_t d1, uint32_t d2, uint32_t first_key_level) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->serving) return set_err(c, WALLY_ESTATE, "cannot encode while serving");
  if (!coeffs || d1 == 0 || d2 == 0) return set_err(c, WALLY_EINVAL, "empty or null PIR database");
  uint32_t levels = 1;
  while ((1u << levels) < d1) ++levels;
  if (levels > kPirMaxLevels || d2 > 2048)
    return set_err(c, WALLY_EINVAL, "PIR database %u x %u beyond the supported 2048 x 2048", d1, d2);
  const uint32_t top = (uint32_t)(c->log_n - 1) / 2;  // g_a^2 = g_(a-1) mod 2n up to this level
  const uint32_t a0 = first_key_level == UINT32_MAX ? std::min(levels - 1, top) : first_key_level;
  if (a0 > std::min(levels - 1, top))
    return set_err(c, WALLY_EINVAL, "first key level %u above %u (levels %u, squaring holds up to %u)", a0,
                   std::min(levels - 1, top), levels, top);
  // two-index queries expand to d1 + d2 entries (none when that is beyond 2^11)
  uint32_t levels2 = 1;
  while ((1u << levels2) < d1 + d2) ++levels2;
  if (levels2 > kPirMaxLevels) levels2 = 0;
  const uint64_t n_pt = (uint64_t)d1 * d2, t = c->mods[c->L + 1];
  for (uint64_t i = 0; i < n_pt * c->n; ++i)
    if (coeffs[i] >= t) return set_err(c, WALLY_EINVAL, "PIR coefficient %llu is not below t", (unsigned long long)i);
  pir_free_work(c);  // waits for answers still reading the database
  dfree(c, c->pir_pt);
  dfree(c, c->pir_w);
  c->pir_pt = nullptr;
  c->pir_w = nullptr;
  c->pir_d1 = c->pir_d2 = 0;
  if ((rc = dalloc(c, n_pt * c->ptw() / c->d_pad * 8, (void**)&c->pir_pt))) return rc;
  // X^-(2^a) at NTT entry i of limb l: psi_l^(-(2 brv(i) + 1) 2^a), for the deeper of the two expansions
  const uint32_t lev_max = std::max(levels, levels2);
  const uint64_t two_n = 2ull * c->n;
  std::vector<ulonglong2> w((size_t)lev_max * c->L * c->n);
  for (uint32_t a = 0; a < lev_max; ++a)
    for (int l = 0; l < c->L; ++l) {
      const uint64_t q = c->mods[l];
      for (int i = 0; i < c->n; ++i) {
        const uint64_t e = ((2ull * bitrev(i, c->log_n) + 1) << a) % two_n;
        const uint64_t v = powmod(c->psi[l], (two_n - e) % two_n, q);
        w[((size_t)a * c->L + l) * c->n + i] = make_ulonglong2(v, shoup_of(v, q));
      }
    }
  if ((rc = dalloc(c, w.size() * sizeof(ulonglong2), (void**)&c->pir_w))) return rc;
  uint32_t* dco = nullptr;
  const uint64_t chunk = 1024;  // plaintexts per upload
  if ((rc = dalloc(c, chunk * c->n * sizeof(uint32_t), (void**)&dco))) return rc;
  hipError_t e = hipMemcpy(c->pir_w, w.data(), w.size() * sizeof(ulonglong2), hipMemcpyHostToDevice);
  for (uint64_t p0 = 0; e == hipSuccess && p0 < n_pt; p0 += chunk) {
    const uint64_t cnt = std::min(chunk, n_pt - p0);
    e = hipMemcpy(dco, coeffs + p0 * c->n, cnt * c->n * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = launch_pir_encode(dco, c->pir_pt + p0 * c->L * c->n, (int)cnt, c->log_n, c->L, c->M, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  dfree(c, dco);
  if (e != hipSuccess) return set_err(c, WALLY_EDEVICE, "PIR encode failed: %s", hipGetErrorString(e));
  c->pir_c2 = 0;
  if (levels2 && (rc = pir2_setup(c, d2))) return rc;
  c->pir_d1 = d1;
  c->pir_d2 = d2;
  c->pir_c = levels;
  c->pir_a0 = a0;
  c->pir_c2 = levels2;
  c->pir_a02 = first_key_level == UINT32_MAX ? std::min(levels2 - 1, top) : a0;
  return WALLY_OK;
}

int wally_pir_info(const wally_ctx* c, uint32_t* levels, uint32_t* first_key_level, uint64_t* gal_keys) {
  if (!c || !c->pir_d1) return WALLY_EINVAL;
  if (levels) *levels = c->pir_c;
  if (first_key_level) *first_key_level = c->pir_a0;
  if (gal_keys)
    for (uint32_t a = c->pir_a0; a < c->pir_c; ++a) gal_keys[a - c->pir_a0] = c->n / (1u << a) + 1;
  return WALLY_OK;
}

int wally_pir_info2(const wally_ctx* c, uint32_t* levels, uint32_t* first_key_level, uint64_t* gal_keys,
                    uint32_t* aux_primes) {
  if (!c || !c->pir_d1 || !c->pir_c2) return WALLY_EINVAL;
  if (levels) *levels = c->pir_c2;
  if (first_key_level) *first_key_level = c->pir_a02;
  if (gal_keys)
    for (uint32_t a = c->pir_a02; a < c->pir_c2; ++a) gal_keys[a - c->pir_a02] = c->n / (1u << a) + 1;
  if (aux_primes) *aux_primes = c->pir_Lb;
  return WALLY_OK;
}

}  // extern "C"

namespace {
int pir_check(wally_ctx* c, const void* q, uint64_t nq) {
  if (c->serving) return set_err(c, WALLY_ESTATE, "a serving session owns the device queues");
  if (!c->pir_d1) return set_err(c, WALLY_ESTATE, "no PIR database encoded");
  if (nq && !q) return set_err(c, WALLY_EINVAL, "null query array");
  return WALLY_OK;
}
}  // namespace

extern "C" {

int wally_pir_answer(wally_ctx* c, const wally_pir_query* q, uint64_t nq, void* hip_stream) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if ((rc = pir_check(c, q, nq))) return rc;
  std::vector<PirQ> qs(nq);
  for (uint64_t i = 0; i < nq; ++i) {
    if (!q[i].ct || !q[i].keys || !q[i].out)
      return set_err(c, WALLY_EINVAL, "PIR query %llu: null pointer", (unsigned long long)i);
    if (((uintptr_t)q[i].ct | (uintptr_t)q[i].out | (uintptr_t)q[i].keys) & 15)
      return set_err(c, WALLY_EINVAL, "PIR query %llu: ct, keys and out must be 16-byte aligned", (unsigned long long)i);
    qs[i] = PirQ{q[i].ct, q[i].keys, nullptr, q[i].out};
  }
  if (nq == 0) return WALLY_OK;
  return pir_answer_any(c, PirMode{c->pir_c, c->pir_a0, false, c->pir_linear}, qs, (hipStream_t)hip_stream);
}

int wally_pir_answer2(wally_ctx* c, const wally_pir_query2* q, uint64_t nq, void* hip_stream) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if ((rc = pir_check(c, q, nq))) return rc;
  if (!c->pir_c2)
    return set_err(c, WALLY_EINVAL, "two-index queries need d1 + d2 <= %u (database %u x %u)", 1u << kPirMaxLevels,
                   c->pir_d1, c->pir_d2);
  std::vector<PirQ> qs(nq);
  for (uint64_t i = 0; i < nq; ++i) {
    if (!q[i].ct || !q[i].keys || !q[i].relin_key || !q[i].out)
      return set_err(c, WALLY_EINVAL, "PIR query %llu: null pointer", (unsigned long long)i);
    if (((uintptr_t)q[i].ct | (uintptr_t)q[i].out | (uintptr_t)q[i].keys | (uintptr_t)q[i].relin_key) & 15)
      return set_err(c, WALLY_EINVAL, "PIR query %llu: ct, keys, relin_key and out must be 16-byte aligned",
                     (unsigned long long)i);
    qs[i] = PirQ{q[i].ct, q[i].keys, q[i].relin_key, q[i].out};
  }
  if (nq == 0) return WALLY_OK;
  return pir_answer_any(c, PirMode{c->pir_c2, c->pir_a02, true, c->pir_linear}, qs, (hipStream_t)hip_stream);
}

int wally_pir_set_linear(wally_ctx* c, int on) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  c->pir_linear = on != 0;
  return WALLY_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// diagnostics

extern "C" {

int wally_diag_ntt(wally_ctx* c, uint32_t mi, uint64_t* data, uint64_t rows, int inverse, void* hip_stream) {
  int rc = check_live(c);
  if (rc) return rc;
  if (mi > (uint32_t)c->L + 1 || !data) return set_err(c, WALLY_EINVAL, "bad modulus index or null data");
  for (uint64_t r0 = 0; r0 < rows; r0 += 65535)
    HIP_OK(c, launch_ntt_rows(data + r0 * c->n, (int)std::min<uint64_t>(65535, rows - r0), c->log_n, (int)mi,
                              inverse ? 1 : 0, c->M, (hipStream_t)hip_stream));
  return WALLY_OK;
}

int wally_diag_rotate(wally_ctx* c, const uint64_t* in, const uint64_t* keys, uint64_t* out, uint64_t count,
                      int which, void* hip_stream) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (!in || !keys || !out) return set_err(c, WALLY_EINVAL, "null pointer");
  if (which != 0 && which != 1) return set_err(c, WALLY_EINVAL, "which must be 0 or 1");
  if ((rc = ensure_sets(c))) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  WaveWork& s = c->sets[0];
  const uint64_t ctw = c->ctw();
  for (uint64_t i0 = 0; i0 < count; i0 += c->B) {
    const int w = (int)std::min<uint64_t>(c->B, count - i0);
    HIP_OK(c, hipStreamSynchronize(st));
    HIP_OK(c, hipStreamSynchronize(s.stream));
    for (int k = 0; k < w; ++k)
      s.baby_host[k] = KsItem{keys + (i0 + k) * c->keyw(), const_cast<uint64_t*>(in) + (i0 + k) * ctw,
                              out + (i0 + k) * ctw, nullptr, nullptr, nullptr, nullptr, nullptr};
    HIP_OK(c, hipMemcpyAsync(s.baby_dev, s.baby_host, w * sizeof(KsItem), hipMemcpyHostToDevice, st));
    KsArgs a = base_args(c, s);
    a.gal = which ? c->gal_giant : c->gal_baby;
    a.in_sel = 0;
    a.out_sel = 1;
    HIP_OK(c, keyswitch(c, s.baby_dev, w, a, st));
  }
  return WALLY_OK;
}

int wally_diag_bfly_rate(wally_ctx* c, int inverse, uint32_t blocks, uint32_t iters, uint64_t* out, double* ms,
                         void* hip_stream) {
  int rc = check_live(c);
  if (rc) return rc;
  if (!out || !ms || blocks == 0 || iters == 0 || blocks > (1u << 20) || iters > (1u << 24))
    return set_err(c, WALLY_EINVAL, "bad butterfly-rate arguments");
  const uint64_t q = c->mods[0];
  ulonglong2 w[4];
  for (int s = 0; s < 4; ++s) {
    const uint64_t v = powmod(c->psi[0], s + 1, q);
    w[s] = make_ulonglong2(v, shoup_of(v, q));
  }
  hipStream_t st = (hipStream_t)hip_stream;
  hipEvent_t a = nullptr, b = nullptr;
  HIP_OK(c, hipEventCreate(&a));
  hipError_t e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipEventRecord(a, st);
  if (e == hipSuccess) e = launch_bfly_rate(out, (int)blocks, inverse ? 1 : 0, w, q, (int)iters, st);
  if (e == hipSuccess) e = hipEventRecord(b, st);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float f = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
  (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) return set_err(c, WALLY_EDEVICE, "butterfly-rate launch failed: %s", hipGetErrorString(e));
  *ms = f;
  return WALLY_OK;
}

int wally_diag_kernel_timing(wally_ctx* c, int enable) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  c->timing = enable != 0;
  return WALLY_OK;
}

int wally_diag_kernel_stats(wally_ctx* c, wally_kernel_stat* out, uint32_t n) {
  int rc = check_live(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  if (!out && n) return set_err(c, WALLY_EINVAL, "null output");
  for (uint32_t k = 0; k < n; ++k) out[k] = wally_kernel_stat{0, 0, 0.0};
  for (auto& t : c->timers) {
    HIP_OK(c, hipEventSynchronize(t.b));
    float ms = 0.f;
    HIP_OK(c, hipEventElapsedTime(&ms, t.a, t.b));
    if (t.kernel >= 0 && (uint32_t)t.kernel < n) {
      out[t.kernel].launches += 1;
      out[t.kernel].items += t.items;
      out[t.kernel].total_ms += ms;
    }
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->timers.clear();
  return WALLY_OK;
}

}  // extern "C"

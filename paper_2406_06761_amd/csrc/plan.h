// Host-side planning of the scoring path, free of the HIP runtime so that it
// can be built and checked on its own: where each cluster's entries go (the
// chunk layout of the index), how a batch is cut into waves, the descriptors
// of one wave (query copies, baby-step items, giant items per (query, chunk)
// sorted by plaintext chunk, tiles of giant items sharing a chunk), the
// descriptor block of a captured batch, and the cut of a batch into captured
// segments.
//
// The templates take any context type with the index fields of the library's
// context: n, d_pad, g, h, B, tile_items, ctw(), pt, and the per-cluster
// vectors chunks, chunk_base and fold, and chunk_pt per chunk.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "items.h"
#include "wally.h"

namespace wally {

inline uint64_t plan_powmod(uint64_t a, uint64_t e, uint64_t m) {
  unsigned __int128 r = 1 % m, x = a % m;
  for (; e; e >>= 1) {
    if (e & 1) r = r * x % m;
    x = x * x % m;
  }
  return (uint64_t)r;
}

// Where each cluster's entries go.  Per cluster (paper §4.1 packing, Server
// Initialization of §5): cluster c owns ceil(N_c / n) chunks, filled from slot
// 0.  Co-packed: clusters of more than n entries keep chunks of their own (in
// cluster order, first); the others go first-fit decreasing (size descending,
// ties by index) into shared chunks at the chunk's fill level, so a query
// needs one chunk and reads its scores from slot_base on.
struct ChunkSeg {
  uint32_t cluster;
  uint64_t offset, count;  // entries [offset, offset + count) of the cluster
};
struct ChunkLayout {
  std::vector<std::vector<ChunkSeg>> segs;  // per chunk, in slot order
  std::vector<uint64_t> first;
  std::vector<uint32_t> chunks, base, fold;
};

// Fold factor of a cluster in the folded layout (not in the paper): the
// largest power of two B <= fold_max with B N_c <= n and d_pad / B >= 4.
inline uint32_t fold_factor(uint64_t size, uint32_t n, uint32_t d_pad, uint32_t fold_max) {
  uint32_t B = 1;
  while (2 * B <= fold_max && 2 * B * size <= n && d_pad / (2 * B) >= 4) B *= 2;
  return B;
}

// Baby/giant split of the d_pad / B diagonals of a fold class.
struct FoldCls {
  uint32_t B, g, h, gal_giant;
};
template <class Ctx>
FoldCls fold_cls(const Ctx* c, uint32_t B) {
  const uint32_t D = c->d_pad / B;
  int lg = 0;
  while ((1u << lg) < D) ++lg;
  const uint32_t g = 1u << ((lg + 1) / 2);
  return FoldCls{B, g, D / g, (uint32_t)plan_powmod(3, g, 2ull * c->n)};
}

inline void plan_layout(uint32_t layout, const uint64_t* offsets, uint32_t k, uint32_t n, uint32_t d_pad,
                        uint32_t fold_max, ChunkLayout& out) {
  out.segs.clear();
  out.first.assign(k, 0);
  out.chunks.assign(k, 0);
  out.base.assign(k, 0);
  out.fold.assign(k, 1);
  // chunks of cap = n / B entries each
  auto own_chunks = [&](uint32_t c, uint32_t cap) {
    const uint64_t sz = offsets[c + 1] - offsets[c];
    out.first[c] = out.segs.size();
    out.chunks[c] = (uint32_t)((sz + cap - 1) / cap);
    for (uint64_t off = 0; off < sz; off += cap)
      out.segs.push_back({ChunkSeg{c, off, std::min<uint64_t>(cap, sz - off)}});
  };
  if (layout == WALLY_LAYOUT_PER_CLUSTER) {
    for (uint32_t c = 0; c < k; ++c) own_chunks(c, n);
    return;
  }
  if (layout == WALLY_LAYOUT_FOLDED) {
    for (uint32_t c = 0; c < k; ++c) {
      out.fold[c] = fold_factor(offsets[c + 1] - offsets[c], n, d_pad, fold_max);
      own_chunks(c, n / out.fold[c]);
    }
    return;
  }
  std::vector<uint32_t> small;
  for (uint32_t c = 0; c < k; ++c) {
    if (offsets[c + 1] - offsets[c] > n)
      own_chunks(c, n);
    else
      small.push_back(c);
  }
  std::stable_sort(small.begin(), small.end(), [&](uint32_t a, uint32_t b) {
    return offsets[a + 1] - offsets[a] > offsets[b + 1] - offsets[b];
  });
  const size_t shared0 = out.segs.size();
  std::vector<uint32_t> fill;  // used slots of each shared chunk
  for (uint32_t c : small) {
    const uint32_t sz = (uint32_t)(offsets[c + 1] - offsets[c]);
    size_t b = 0;
    while (b < fill.size() && fill[b] + sz > n) ++b;
    if (b == fill.size()) {
      fill.push_back(0);
      out.segs.emplace_back();
    }
    out.first[c] = shared0 + b;
    out.chunks[c] = 1;
    out.base[c] = fill[b];
    out.segs[shared0 + b].push_back(ChunkSeg{c, 0, sz});
    fill[b] += sz;
  }
}

// Queries ordered by chunk (so a wave touches few plaintext chunks) and cut
// into waves: up to B queries of one fold class, of one cluster only on the
// plain path.  ord receives the query order, waves the [first, end) ranges.
template <class Ctx>
void make_waves(const Ctx* c, const wally_query* q, uint64_t nq, int path, std::vector<const wally_query*>& ord,
                std::vector<std::pair<uint64_t, uint64_t>>& waves) {
  ord.resize(nq);
  for (uint64_t i = 0; i < nq; ++i) ord[i] = &q[i];
  // by fold class (a wave runs one baby/giant split), then first chunk, then
  // cluster: clusters that share a chunk land in the same waves and tiles
  const std::vector<uint64_t>& fc = c->chunk_base;
  const std::vector<uint32_t>& fo = c->fold;
  std::stable_sort(ord.begin(), ord.end(), [&fc, &fo](const wally_query* a, const wally_query* b) {
    if (fo[a->cluster] != fo[b->cluster]) return fo[a->cluster] < fo[b->cluster];
    return fc[a->cluster] != fc[b->cluster] ? fc[a->cluster] < fc[b->cluster] : a->cluster < b->cluster;
  });
  waves.clear();
  for (uint64_t i = 0; i < nq;) {
    uint64_t j = i;
    while (j < nq && j - i < (uint64_t)c->B && fo[ord[j]->cluster] == fo[ord[i]->cluster] &&
           (path != WALLY_PATH_PLAIN || ord[j]->cluster == ord[i]->cluster))
      ++j;
    waves.push_back({i, j});
    i = j;
  }
}

// Workspace rows of one wave: rotated query copies [B][g][2][L][n], the two
// Horner buffers and the giant-step sums per giant slot of a sub-wave.
struct WaveBufs {
  uint64_t* ctp;
  uint64_t* R0;
  uint64_t* R1;
  uint64_t* ACC;
};

// Descriptors of one wave: copy and baby items per query, giant items per
// (query, chunk) ordered by plaintext chunk, tiles of giant items sharing a
// chunk, split in sub-waves of at most B giant items.
struct WavePlan {
  int w = 0;
  FoldCls cls{1, 0, 0, 0};  // fold class shared by the wave's clusters
  size_t ng = 0, nt = 0;
  std::vector<std::pair<size_t, size_t>> sub_tiles;  // per sub-wave: [first tile, end tile)
};

// Giant items of a wave: the sum of its queries' chunk counts.
template <class Ctx>
size_t wave_giant_items(const Ctx* c, const wally_query* const* qs, int w) {
  size_t ng = 0;
  for (int k = 0; k < w; ++k) ng += c->chunks[qs[k]->cluster];
  return ng;
}

// Writes copy[0..w), baby[0..w), giant[0..ng) and tiles[0..nt) (nt <= ng) for
// queries qs[0..w), all of one fold class.
template <class Ctx>
void plan_wave(const Ctx* c, const WaveBufs& s, const wally_query* const* qs, int w, CopyItem* copy, KsItem* baby,
               KsItem* giant, MacTile* tiles, WavePlan& p) {
  const uint64_t ctw = c->ctw();
  p.cls = fold_cls(c, c->fold[qs[0]->cluster]);
  const FoldCls& fc = p.cls;
  std::vector<std::pair<uint64_t, uint32_t>> order;  // (global chunk index, item)
  std::vector<std::pair<int, uint32_t>> gq;           // (query slot, chunk)
  for (int k = 0; k < w; ++k) {
    const wally_query& q = *qs[k];
    uint64_t* ctp = s.ctp + (uint64_t)k * c->g * ctw;
    copy[k] = CopyItem{q.ct, ctp};
    baby[k] = KsItem{q.key_baby, ctp, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    for (uint32_t ch = 0; ch < c->chunks[q.cluster]; ++ch) {
      order.push_back({c->chunk_base[q.cluster] + ch, (uint32_t)gq.size()});
      gq.push_back({k, ch});
    }
  }
  std::stable_sort(order.begin(), order.end(),
                   [](const std::pair<uint64_t, uint32_t>& a, const std::pair<uint64_t, uint32_t>& b) {
                     return a.first < b.first;
                   });
  p.w = w;
  p.ng = order.size();
  p.nt = 0;
  p.sub_tiles.clear();
  for (size_t g0 = 0; g0 < p.ng; g0 += c->B) {
    const size_t g1 = std::min(p.ng, g0 + (size_t)c->B);
    const size_t t0 = p.nt;
    for (size_t k = g0; k < g1; ++k) {
      const auto& gi = gq[order[k].second];
      const wally_query& q = *qs[gi.first];
      const size_t slot = k - g0;
      KsItem it{};
      it.key = q.key_giant;
      it.key_fold = q.key_fold;
      it.fin = q.out + (uint64_t)gi.second * ctw;
      it.pt = c->pt + c->chunk_pt[order[k].first];
      it.ctp = s.ctp + (uint64_t)gi.first * c->g * ctw;
      it.buf0 = s.R0 + slot * ctw;
      it.buf1 = s.R1 + slot * ctw;
      it.acc = fc.h == 1 && fc.B == 1 ? it.fin : s.ACC + slot * c->h * ctw;
      giant[k] = it;
      const bool start = k == g0 || order[k].first != order[k - 1].first || tiles[p.nt - 1].count >= c->tile_items;
      if (start) tiles[p.nt++] = MacTile{(uint32_t)(k - g0), 0};
      tiles[p.nt - 1].count++;
    }
    p.sub_tiles.push_back({t0, p.nt});
  }
}

// Descriptors of waves [w0, w1) of a batch in one block, as a captured
// segment reads them: copy items of all its queries, then baby items, then
// giant items, then tiles.  Per wave, the offsets (in elements) of its part of
// each array.
struct SegmentPlan {
  size_t nq = 0, ng = 0, bytes = 0;
  size_t copy_at = 0, baby_at = 0, giant_at = 0, tile_at = 0;  // byte offsets in the block
  std::vector<WavePlan> plans;
  std::vector<size_t> qoff, goff, toff;
};

// Plans waves [w0, w1) into `block` (resized to the segment's bytes); wave wv
// uses the workspace rows bufs_of(wv).
template <class Ctx, class BufsOf>
void plan_segment(const Ctx* c, const std::vector<const wally_query*>& ord,
                  const std::vector<std::pair<uint64_t, uint64_t>>& waves, size_t w0, size_t w1, BufsOf bufs_of,
                  std::vector<unsigned char>& block, SegmentPlan& sp) {
  sp = SegmentPlan{};
  for (size_t wv = w0; wv < w1; ++wv) {
    sp.nq += waves[wv].second - waves[wv].first;
    sp.ng += wave_giant_items(c, ord.data() + waves[wv].first, (int)(waves[wv].second - waves[wv].first));
  }
  sp.copy_at = 0;
  sp.baby_at = sp.copy_at + sp.nq * sizeof(CopyItem);
  sp.giant_at = sp.baby_at + sp.nq * sizeof(KsItem);
  sp.tile_at = sp.giant_at + sp.ng * sizeof(KsItem);
  sp.bytes = sp.tile_at + sp.ng * sizeof(MacTile);
  block.assign(sp.bytes, 0);
  CopyItem* copy_h = (CopyItem*)(block.data() + sp.copy_at);
  KsItem* baby_h = (KsItem*)(block.data() + sp.baby_at);
  KsItem* giant_h = (KsItem*)(block.data() + sp.giant_at);
  MacTile* tile_h = (MacTile*)(block.data() + sp.tile_at);
  const size_t nw = w1 - w0;
  sp.plans.resize(nw);
  sp.qoff.resize(nw);
  sp.goff.resize(nw);
  sp.toff.resize(nw);
  size_t qo = 0, go = 0, to = 0;
  for (size_t k = 0; k < nw; ++k) {
    const size_t wv = w0 + k;
    const int w = (int)(waves[wv].second - waves[wv].first);
    sp.qoff[k] = qo;
    sp.goff[k] = go;
    sp.toff[k] = to;
    plan_wave(c, bufs_of(wv), ord.data() + waves[wv].first, w, copy_h + qo, baby_h + qo, giant_h + go, tile_h + to,
              sp.plans[k]);
    qo += w;
    go += sp.plans[k].ng;
    to += sp.plans[k].nt;
  }
}

// A batch of nw waves cut into the fewest captured segments of at most
// max_waves waves each, of near-equal size: [first, end) wave ranges.
inline std::vector<std::pair<size_t, size_t>> graph_segments(size_t nw, size_t max_waves) {
  std::vector<std::pair<size_t, size_t>> segs;
  if (nw == 0 || max_waves == 0) return segs;
  const size_t k = (nw + max_waves - 1) / max_waves;
  for (size_t i = 0; i < k; ++i) segs.push_back({nw * i / k, nw * (i + 1) / k});
  return segs;
}

}  // namespace wally

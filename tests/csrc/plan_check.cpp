// Checks the host-side planning of the scoring path (chunk layout, waves,
// wave descriptors, captured-segment descriptor blocks) at a given index and
// batch shape.  Built with AddressSanitizer and UndefinedBehaviorSanitizer by
// the CPU tests: every descriptor array is a heap block of exactly the size
// the library allocates for it, so a write past it stops the run; every
// descriptor is also checked against the workspace, index and caller ranges
// it must point into.
//
// Input (binary, little-endian): u32 log_n, L, d_pad, B, tile_items, layout,
// fold_max, sets, seg_waves, K; u64 offsets[K+1]; u64 nq; u32 targets[nq].
// Prints one line of counts; exits 1 with a message on the first violation.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <iterator>

#include <set>
#include <vector>

#include "plan.h"

using namespace wally;

namespace {

struct Ctx {
  int n = 0, d_pad = 0, g = 0, h = 0, B = 0, L = 0;
  uint32_t tile_items = 0;
  std::vector<uint32_t> chunks, fold;
  std::vector<uint64_t> chunk_base, chunk_pt;
  uint64_t* pt = nullptr;
  uint64_t ctw() const { return 2ull * L * n; }
};

[[noreturn]] void fail(const char* what, unsigned long long a, unsigned long long b) {
  fprintf(stderr, "plan_check: %s (%llu, %llu)\n", what, a, b);
  exit(1);
}

#define REQUIRE(cond, what, a, b) \
  do {                            \
    if (!(cond)) fail(what, (unsigned long long)(a), (unsigned long long)(b)); \
  } while (0)

// Addresses that stand for device buffers: never dereferenced, only compared.
uintptr_t fake_base(uint64_t region) { return (uintptr_t)0x100000000000ull + (uintptr_t)region * 0x40000000000ull; }

bool in_range(const void* p, uintptr_t base, uint64_t words) {
  const uintptr_t a = (uintptr_t)p;
  return a >= base && a < base + words * 8 && (a - base) % 8 == 0;
}

struct Sets {
  std::vector<WaveBufs> bufs;
  std::vector<uintptr_t> ctp, r0, r1, acc;
};

// The descriptors of one planned wave, checked against the query array,
// the index and the wave's workspace rows.
void check_wave(const Ctx& c, const Sets& S, size_t set, const wally_query* q0, uint64_t nq,
                const wally_query* const* qs, int w, const CopyItem* copy, const KsItem* baby, const KsItem* giant,
                const MacTile* tiles, const WavePlan& p, uint64_t pt_words) {
  const uint64_t ctw = c.ctw();
  REQUIRE(p.w == w && w >= 1 && w <= c.B, "wave size", p.w, w);
  size_t ng = 0;
  for (int k = 0; k < w; ++k) {
    REQUIRE(qs[k] >= q0 && qs[k] < q0 + nq, "query pointer outside the array", k, w);
    REQUIRE(c.fold[qs[k]->cluster] == p.cls.B, "mixed fold classes in a wave", k, p.cls.B);
    ng += c.chunks[qs[k]->cluster];
    REQUIRE(copy[k].src == qs[k]->ct, "copy source", k, 0);
    REQUIRE((uintptr_t)copy[k].dst == S.ctp[set] + (uintptr_t)k * c.g * ctw * 8, "copy destination", k, set);
    REQUIRE(baby[k].key == qs[k]->key_baby && baby[k].buf0 == copy[k].dst, "baby item", k, 0);
  }
  REQUIRE(p.ng == ng, "giant item count", p.ng, ng);
  REQUIRE(p.nt <= p.ng, "more tiles than items", p.nt, p.ng);
  REQUIRE(p.sub_tiles.size() == (ng + c.B - 1) / c.B, "sub-wave count", p.sub_tiles.size(), ng);
  // every (query, chunk) exactly once
  std::set<std::pair<const wally_query*, uint64_t>> seen;
  std::vector<std::pair<uintptr_t, const wally_query*>> outs;
  for (int j = 0; j < w; ++j) outs.push_back({(uintptr_t)qs[j]->out, qs[j]});
  std::sort(outs.begin(), outs.end());
  for (size_t k = 0; k < ng; ++k) {
    const KsItem& it = giant[k];
    const size_t slot = k % c.B;
    REQUIRE(it.buf0 && (uintptr_t)it.buf0 == S.r0[set] + slot * ctw * 8, "R0 row", k, slot);
    REQUIRE((uintptr_t)it.buf1 == S.r1[set] + slot * ctw * 8, "R1 row", k, slot);
    REQUIRE(in_range(it.ctp, S.ctp[set], (uint64_t)c.B * c.g * ctw), "rotated copies outside the workspace", k, 0);
    REQUIRE(((uintptr_t)it.ctp - S.ctp[set]) % (c.g * ctw * 8) == 0, "rotated copies misaligned", k, 0);
    if (p.cls.h == 1 && p.cls.B == 1)
      REQUIRE(it.acc == it.fin, "h = 1 sums go to the output", k, 0);
    else
      REQUIRE((uintptr_t)it.acc == S.acc[set] + slot * c.h * ctw * 8, "sum rows", k, slot);
    REQUIRE(in_range(it.pt, (uintptr_t)c.pt, pt_words), "plaintexts outside the index", k, 0);
    // which query and chunk: fin = out + ch ctw of one of the wave's queries
    const wally_query* owner = nullptr;
    uint64_t ch = 0;
    auto hit = std::upper_bound(outs.begin(), outs.end(), (uintptr_t)it.fin,
                                [](uintptr_t a, const std::pair<uintptr_t, const wally_query*>& b) { return a < b.first; });
    if (hit != outs.begin()) {
      const wally_query* cand = std::prev(hit)->second;
      const uintptr_t o = (uintptr_t)cand->out;
      if ((uintptr_t)it.fin < o + (uintptr_t)c.chunks[cand->cluster] * ctw * 8 && it.key == cand->key_giant) {
        owner = cand;
        ch = ((uintptr_t)it.fin - o) / (ctw * 8);
        REQUIRE(((uintptr_t)it.fin - o) % (ctw * 8) == 0, "output row misaligned", k, 0);
      }
    }
    REQUIRE(owner, "giant item of no query", k, 0);
    REQUIRE(it.pt == c.pt + c.chunk_pt[c.chunk_base[owner->cluster] + ch], "plaintexts of the wrong chunk", k, ch);
    REQUIRE(seen.insert({owner, ch}).second, "giant item twice", k, ch);
    REQUIRE(it.key_fold == owner->key_fold, "fold keys", k, 0);
  }
  REQUIRE(seen.size() == ng, "missing giant items", seen.size(), ng);
  // tiles: per sub-wave, consecutive, covering it, one chunk each, at most tile_items
  size_t t_expect = 0;
  for (size_t sw = 0; sw < p.sub_tiles.size(); ++sw) {
    const size_t g0 = sw * c.B, cnt = std::min<size_t>(c.B, ng - g0);
    REQUIRE(p.sub_tiles[sw].first == t_expect, "tile ranges not consecutive", sw, t_expect);
    size_t at = 0;
    for (size_t t = p.sub_tiles[sw].first; t < p.sub_tiles[sw].second; ++t) {
      REQUIRE(tiles[t].first == at, "tile start", t, at);
      REQUIRE(tiles[t].count >= 1 && tiles[t].count <= c.tile_items, "tile size", t, tiles[t].count);
      for (uint32_t k = 1; k < tiles[t].count; ++k)
        REQUIRE(giant[g0 + at + k].pt == giant[g0 + at].pt, "tile over two chunks", t, k);
      at += tiles[t].count;
    }
    REQUIRE(at == cnt, "tiles do not cover the sub-wave", at, cnt);
    t_expect = p.sub_tiles[sw].second;
  }
  REQUIRE(t_expect == p.nt, "tile count", t_expect, p.nt);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: plan_check INPUT\n");
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  uint32_t hdr[10];
  if (fread(hdr, 4, 10, f) != 10) return 2;
  const uint32_t log_n = hdr[0], L = hdr[1], d_pad = hdr[2], B = hdr[3], tile = hdr[4], layout = hdr[5],
                 fold_max = hdr[6], n_sets = hdr[7], seg_waves = hdr[8], K = hdr[9];
  std::vector<uint64_t> offsets(K + 1);
  if (fread(offsets.data(), 8, K + 1, f) != K + 1) return 2;
  uint64_t nq = 0;
  if (fread(&nq, 8, 1, f) != 1) return 2;
  std::vector<uint32_t> targets(nq);
  if (nq && fread(targets.data(), 4, nq, f) != nq) return 2;
  fclose(f);

  Ctx c;
  c.n = 1 << log_n;
  c.L = (int)L;
  c.d_pad = (int)d_pad;
  int lg = 0;
  while ((1 << lg) < c.d_pad) ++lg;
  c.g = 1 << ((lg + 1) / 2);
  c.h = c.d_pad / c.g;
  c.B = (int)B;
  c.tile_items = tile;
  // the chunk layout and the plaintext offsets, as the encode computes them
  ChunkLayout lay;
  plan_layout(layout, offsets.data(), K, c.n, d_pad, fold_max, lay);
  c.chunks = lay.chunks;
  c.chunk_base = lay.first;
  c.fold = lay.fold;
  std::vector<uint32_t> chunk_fold(lay.segs.size(), 1);
  for (uint32_t cl = 0; cl < K; ++cl) {
    REQUIRE(lay.chunks[cl] >= 1, "cluster without chunks", cl, 0);
    for (uint32_t j = 0; j < lay.chunks[cl]; ++j) chunk_fold[lay.first[cl] + j] = lay.fold[cl];
  }
  uint64_t pt_words = 0;
  c.chunk_pt.resize(lay.segs.size());
  for (size_t ch = 0; ch < lay.segs.size(); ++ch) {
    c.chunk_pt[ch] = pt_words;
    pt_words += (uint64_t)d_pad * L * c.n / chunk_fold[ch];
  }
  c.pt = (uint64_t*)fake_base(1);
  // every entry placed exactly once, within its chunk's capacity
  std::vector<uint64_t> placed(K, 0);
  for (size_t ch = 0; ch < lay.segs.size(); ++ch) {
    uint64_t used = 0;
    for (const auto& sg : lay.segs[ch]) {
      REQUIRE(sg.offset + sg.count <= offsets[sg.cluster + 1] - offsets[sg.cluster], "segment past its cluster", ch,
              sg.cluster);
      used += sg.count;
      placed[sg.cluster] += sg.count;
    }
    REQUIRE(used <= (uint64_t)c.n / chunk_fold[ch], "chunk over capacity", ch, used);
  }
  for (uint32_t cl = 0; cl < K; ++cl)
    REQUIRE(placed[cl] == offsets[cl + 1] - offsets[cl], "entries placed", cl, placed[cl]);
  uint32_t max_chunks = 0;
  for (uint32_t v : c.chunks) max_chunks = std::max(max_chunks, v);

  // queries with stand-in device addresses: one region per buffer kind
  const uint64_t ctw = c.ctw(), keyw = (uint64_t)L * 2 * (L + 1) * c.n;
  std::vector<wally_query> q(nq);
  uint64_t out_words = 0;
  for (uint64_t i = 0; i < nq; ++i) {
    REQUIRE(targets[i] < K, "target out of range", i, targets[i]);
    q[i].cluster = targets[i];
    q[i].ct = (const uint64_t*)(fake_base(2) + i * ctw * 8);
    q[i].key_baby = (const uint64_t*)(fake_base(3) + i * keyw * 8);
    q[i].key_giant = (const uint64_t*)(fake_base(4) + i * keyw * 8);
    q[i].key_fold = c.fold[targets[i]] > 1 ? (const uint64_t*)(fake_base(5) + i * 8 * keyw * 8) : nullptr;
    q[i].out = (uint64_t*)(fake_base(6) + out_words * 8);
    out_words += (uint64_t)c.chunks[targets[i]] * ctw;
  }
  // workspace sets
  Sets S;
  for (uint32_t k = 0; k < n_sets; ++k) {
    S.ctp.push_back(fake_base(8 + 4 * k));
    S.r0.push_back(fake_base(9 + 4 * k));
    S.r1.push_back(fake_base(10 + 4 * k));
    S.acc.push_back(fake_base(11 + 4 * k));
    S.bufs.push_back(WaveBufs{(uint64_t*)S.ctp.back(), (uint64_t*)S.r0.back(), (uint64_t*)S.r1.back(),
                              (uint64_t*)S.acc.back()});
  }

  unsigned long long total_items = 0, max_wave_items = 0;
  size_t n_waves[2] = {0, 0};
  for (int path : {WALLY_PATH_BATCHED, WALLY_PATH_PLAIN}) {
    std::vector<const wally_query*> ord;
    std::vector<std::pair<uint64_t, uint64_t>> waves;
    make_waves(&c, q.data(), nq, path, ord, waves);
    n_waves[path == WALLY_PATH_PLAIN] = waves.size();
    // waves cover the batch in order, each query once
    std::vector<char> hit(nq, 0);
    uint64_t expect = 0;
    for (const auto& wv : waves) {
      REQUIRE(wv.first == expect && wv.second > wv.first && wv.second - wv.first <= B, "wave range", wv.first,
              wv.second);
      expect = wv.second;
      for (uint64_t i = wv.first; i < wv.second; ++i) {
        const uint64_t idx = ord[i] - q.data();
        REQUIRE(!hit[idx], "query in two waves", idx, 0);
        hit[idx] = 1;
        if (path == WALLY_PATH_PLAIN) REQUIRE(ord[i]->cluster == ord[wv.first]->cluster, "plain wave mixes clusters", i, 0);
      }
    }
    REQUIRE(expect == nq, "waves do not cover the batch", expect, nq);
    // eager path: descriptor arrays of exactly the sizes ensure_sets allocates
    const size_t giant_cap = (size_t)B * std::max<uint32_t>(1, max_chunks);
    for (size_t wv = 0; wv < waves.size(); ++wv) {
      const int w = (int)(waves[wv].second - waves[wv].first);
      std::vector<CopyItem> copy(B);
      std::vector<KsItem> baby(B), giant(giant_cap);
      std::vector<MacTile> tiles(giant_cap);
      const size_t set = wv % n_sets;
      WavePlan p;
      const wally_query* const* qs = ord.data() + waves[wv].first;
      REQUIRE(wave_giant_items(&c, qs, w) <= giant_cap, "wave has more giant items than the set holds", wv, giant_cap);
      plan_wave(&c, S.bufs[set], qs, w, copy.data(), baby.data(), giant.data(), tiles.data(), p);
      check_wave(c, S, set, q.data(), nq, qs, w, copy.data(), baby.data(), giant.data(), tiles.data(), p, pt_words);
      if (path == WALLY_PATH_BATCHED) {
        total_items += p.ng;
        max_wave_items = std::max<unsigned long long>(max_wave_items, p.ng);
      }
    }
    if (path != WALLY_PATH_BATCHED) continue;
    // graph path: segments, each planned into one exactly sized block
    const auto segs = graph_segments(waves.size(), seg_waves);
    size_t next = 0;
    for (const auto& sg : segs) {
      REQUIRE(sg.first == next && sg.second > sg.first && sg.second - sg.first <= seg_waves, "segment range", sg.first,
              sg.second);
      next = sg.second;
      std::vector<unsigned char> block;
      SegmentPlan sp;
      plan_segment(&c, ord, waves, sg.first, sg.second, [&](size_t wv) { return S.bufs[wv % n_sets]; }, block, sp);
      REQUIRE(block.size() == sp.bytes, "segment block size", block.size(), sp.bytes);
      REQUIRE(sp.tile_at + sp.ng * sizeof(MacTile) == sp.bytes && sp.giant_at + sp.ng * sizeof(KsItem) == sp.tile_at,
              "segment block layout", sp.giant_at, sp.tile_at);
      // copy the block's arrays out into exactly sized heap blocks before reading them
      for (size_t k = 0; k < sp.plans.size(); ++k) {
        const size_t wv = sg.first + k;
        const int w = (int)(waves[wv].second - waves[wv].first);
        REQUIRE(sp.qoff[k] + w <= sp.nq && sp.goff[k] + sp.plans[k].ng <= sp.ng && sp.toff[k] + sp.plans[k].nt <= sp.ng,
                "wave part outside its segment", wv, k);
        std::vector<CopyItem> copy(w);
        std::vector<KsItem> baby(w), giant(sp.plans[k].ng);
        std::vector<MacTile> tiles(sp.plans[k].nt);
        memcpy(copy.data(), block.data() + sp.copy_at + sp.qoff[k] * sizeof(CopyItem), w * sizeof(CopyItem));
        memcpy(baby.data(), block.data() + sp.baby_at + sp.qoff[k] * sizeof(KsItem), w * sizeof(KsItem));
        memcpy(giant.data(), block.data() + sp.giant_at + sp.goff[k] * sizeof(KsItem), giant.size() * sizeof(KsItem));
        memcpy(tiles.data(), block.data() + sp.tile_at + sp.toff[k] * sizeof(MacTile), tiles.size() * sizeof(MacTile));
        check_wave(c, S, wv % n_sets, q.data(), nq, ord.data() + waves[wv].first, w, copy.data(), baby.data(),
                   giant.data(), tiles.data(), sp.plans[k], pt_words);
      }
    }
    REQUIRE(next == waves.size(), "segments do not cover the waves", next, waves.size());
    printf("chunks %zu max_chunks %u waves %zu segments %zu giant_items %llu max_wave_items %llu\n",
           lay.segs.size(), max_chunks, waves.size(), segs.size(), total_items, max_wave_items);
  }
  printf("ok waves %zu plain_waves %zu\n", n_waves[0], n_waves[1]);
  return 0;
}

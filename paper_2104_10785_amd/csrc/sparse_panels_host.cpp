// Column-panel layout of a CSR matrix: shape rule, size bound and the host
// builder (layout and work items described in sparse_panels.h).
#include "sparse_panels.h"

#include <algorithm>

namespace gkb {

namespace {

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

int64_t npanels(int64_t C) { return (C + PN_W - 1) / PN_W; }

// Upper bounds of the item counts (each closed stream block ends because the
// next segment would pass PN_BLK entries (then it holds more than
// PN_BLK - PN_BIG), because it has PN_ROWS rows, because a segment of more
// than PN_BIG entries follows, or at the end of a panel; such a segment of L
// entries gives at most 1 + L / PN_CHUNK chunks).
struct Bounds {
  int64_t sblk, witem, segs, jobs, lrow;
};
Bounds bounds(int64_t R, int64_t C, int64_t nnz) {
  const int64_t np = npanels(C);
  Bounds b;
  const int64_t nbig = nnz / (PN_BIG + 1);
  b.sblk = nnz / (PN_BLK - PN_BIG) + np * R / PN_ROWS + nbig + np + 1;
  b.lrow = nnz / (PN_SHORT + 1) + 1;
  b.witem = nbig + nnz / PN_CHUNK + 1;
  b.segs = nbig + 1;
  b.jobs = b.sblk + b.witem;   // every job holds at least one item
  return b;
}

}  // namespace

bool panels_suit(int64_t R, int64_t C, int64_t nnz) {
  if (R < 1 || C < 1 || nnz < 0 || R >= ((int64_t)1 << 31) - 1 || nnz >= ((int64_t)1 << 31) - 1) return false;
  const int64_t np = npanels(C);
  return np == 1 || np * R <= 4 * std::max<int64_t>(nnz, 1);
}

size_t panel_bytes_bound(int64_t R, int64_t C, int64_t nnz) {
  if (!panels_suit(R, C, nnz)) return 0;
  const int64_t np = npanels(C);
  const Bounds b = bounds(R, C, nnz);
  // pidx and pval hold one padding entry past the end
  size_t s = a256((size_t)(nnz + 1) * 2) + a256((size_t)(nnz + 1) * 4) + a256((size_t)np * (R + 1) * 4) +
             a256((size_t)(np + 1) * 8);
  s += a256((size_t)b.jobs * 16) + a256((size_t)b.sblk * 16) + a256((size_t)b.witem * 16) + a256((size_t)b.segs * 16);
  s += a256((size_t)b.witem * 4);                        // chunk-sum slots
  s += a256((size_t)(b.lrow + 1) * 4);                   // long rows of the stream blocks
  if (np > 1) s += a256((size_t)np * R * 4);             // per-panel row sums
  return s + 256;
}

void build_panels(int64_t R, int64_t C, int64_t nnz, const int64_t* ptr, const int32_t* idx, const float* val,
                  int target_jobs, PanelLayout& L) {
  const int np = (int)npanels(C);
  const int64_t R1 = R + 1;
  L.R = R;
  L.C = C;
  L.nnz = nnz;
  L.np = np;
  // segment lengths, then offsets within each panel
  L.poff.assign((size_t)np * R1, 0);
  for (int64_t r = 0; r < R; ++r)
    for (int64_t j = ptr[r]; j < ptr[r + 1]; ++j) ++L.poff[(size_t)(idx[j] / PN_W) * R1 + r + 1];
  L.pbase.assign((size_t)np + 1, 0);
  for (int b = 0; b < np; ++b) {
    int32_t* po = L.poff.data() + (size_t)b * R1;
    for (int64_t r = 1; r <= R; ++r) po[r] += po[r - 1];
    L.pbase[b + 1] = L.pbase[b] + po[R];
  }
  // entries, panel by panel, each row's entries in their CSR order
  L.pidx.assign((size_t)nnz + 1, 0);   // one padding entry: an empty block's clamped read
  L.pval.assign((size_t)nnz + 1, 0.f);
  std::vector<int32_t> cur(L.poff);
  for (int64_t r = 0; r < R; ++r)
    for (int64_t j = ptr[r]; j < ptr[r + 1]; ++j) {
      const int b = idx[j] / PN_W;
      const int64_t pos = L.pbase[b] + cur[(size_t)b * R1 + r]++;
      L.pidx[pos] = (uint16_t)(idx[j] - b * PN_W);
      L.pval[pos] = val[j];
    }
  // items, panel by panel
  L.jobs.clear();
  L.sblk.clear();
  L.witem.clear();
  L.segs.clear();
  L.lrow.clear();
  L.nslot = 0;
  std::vector<size_t> s_first(np + 1), w_first(np + 1);
  for (int b = 0; b < np; ++b) {
    const int32_t* po = L.poff.data() + (size_t)b * R1;
    s_first[b] = L.sblk.size();
    w_first[b] = L.witem.size();
    int32_t r0 = 0, nr = 0, e0 = 0, ecnt = 0;
    std::vector<int32_t> longs;
    auto flush = [&]() {
      if (nr > 0) {
        L.sblk.push_back({r0, pn_pack(nr, ecnt, (int32_t)longs.size()), e0, (int32_t)L.lrow.size()});
        L.lrow.insert(L.lrow.end(), longs.begin(), longs.end());
      }
      nr = 0;
      longs.clear();
    };
    for (int64_t r = 0; r < R; ++r) {
      const int32_t s = po[r], len = po[r + 1] - po[r];
      if (len <= PN_BIG) {
        if (nr == PN_ROWS || ecnt + len > PN_BLK) flush();
        if (nr == 0) {
          r0 = (int32_t)r;
          e0 = s;
          ecnt = 0;
        }
        if (len > PN_SHORT) longs.push_back(nr);
        ++nr;
        ecnt += len;
      } else {
        flush();
        const int32_t nch = (len + PN_CHUNK - 1) / PN_CHUNK;
        L.segs.push_back({b, (int32_t)r, (int32_t)L.nslot, nch});
        for (int32_t c = 0; c < nch; ++c)
          L.witem.push_back({(int32_t)r, s + c * PN_CHUNK, std::min(PN_CHUNK, len - c * PN_CHUNK),
                             (int32_t)L.nslot++});
      }
    }
    flush();
  }
  s_first[np] = L.sblk.size();
  w_first[np] = L.witem.size();
  L.lrow.push_back(0);   // padding: an empty block's clamped read
  // jobs: each panel's stream blocks and wave items cut into parts of about
  // equal cost (entries + 2 per row, entries + 64 per wave item), the number
  // of parts in proportion to the cost, so that all jobs together number
  // about target_jobs (one workgroup per compute unit: a single round)
  auto scost = [](const PnDesc& d) { return (int64_t)((d.b >> 10) & 8191) + 2 * (int64_t)(d.b & 1023); };
  auto wcost = [](const PnDesc& d) { return (int64_t)d.c + 64; };
  std::vector<int64_t> cs(np, 0), cw(np, 0), ks(np, 0), kw(np, 0);
  int64_t total_s = 0, total_w = 0;
  for (int b = 0; b < np; ++b) {
    for (size_t i = s_first[b]; i < s_first[b + 1]; ++i) cs[b] += scost(L.sblk[i]);
    for (size_t i = w_first[b]; i < w_first[b + 1]; ++i) cw[b] += wcost(L.witem[i]);
    total_s += cs[b];
    total_w += cw[b];
  }
  // wave items first (one job per panel that has any, more in proportion to
  // their share of the cost), the rest of the target to the stream blocks
  const int64_t target = std::max(target_jobs, 1);
  auto parts = [](int64_t cost, int64_t share_of, int64_t of, size_t items) -> int64_t {
    if (items == 0) return 0;
    const int64_t k = of > 0 ? (int64_t)((__int128)cost * share_of / of) : 1;
    return std::max<int64_t>(1, std::min<int64_t>({k, cost / PN_JOB_MIN + 1, (int64_t)items}));
  };
  int64_t used = 0;
  for (int b = 0; b < np; ++b) {
    kw[b] = parts(cw[b], target * total_w / std::max<int64_t>(total_s + total_w, 1), total_w,
                  w_first[b + 1] - w_first[b]);
    used += kw[b];
  }
  const int64_t rest = std::max<int64_t>(target - used, 1);
  for (int b = 0; b < np; ++b) ks[b] = parts(cs[b], rest, total_s, s_first[b + 1] - s_first[b]);
  auto cut = [&](int b, int kind, size_t first, size_t last, int64_t cost, int64_t k,
                 int64_t (*c)(const PnDesc&), const std::vector<PnDesc>& items) {
    // part j closes once the cumulative cost reaches (j + 1) cost / k, or at
    // PN_JOB_ITEMS items
    int64_t acc = 0, j = 0;
    size_t j0 = first;
    for (size_t i = first; i < last; ++i) {
      acc += c(items[i]);
      const bool full = (__int128)acc * k >= (__int128)(j + 1) * cost;
      if (full || i + 1 - j0 == (size_t)PN_JOB_ITEMS || i + 1 == last) {
        L.jobs.push_back({b, kind, (int32_t)j0, (int32_t)(i + 1 - j0)});
        j0 = i + 1;
        while ((__int128)acc * k >= (__int128)(j + 1) * cost && j < k) ++j;
      }
    }
  };
  for (int b = 0; b < np; ++b) {
    cut(b, 0, s_first[b], s_first[b + 1], cs[b], ks[b], scost, L.sblk);
    cut(b, 1, w_first[b], w_first[b + 1], cw[b], kw[b], wcost, L.witem);
  }
}

}  // namespace gkb

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
  int64_t sblk, witem, segs, jobs;
};
Bounds bounds(int64_t R, int64_t C, int64_t nnz) {
  const int64_t np = npanels(C);
  Bounds b;
  const int64_t nbig = nnz / (PN_BIG + 1);
  b.sblk = nnz / (PN_BLK - PN_BIG) + np * R / PN_ROWS + nbig + np + 1;
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
  size_t s = a256((size_t)nnz * 2) + a256((size_t)nnz * 4) + a256((size_t)np * (R + 1) * 4) + a256((size_t)(np + 1) * 8);
  s += a256((size_t)b.jobs * 16) + a256((size_t)b.sblk * 16) + a256((size_t)b.witem * 16) + a256((size_t)b.segs * 16);
  s += a256((size_t)b.witem * 4);                        // chunk-sum slots
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
  L.pidx.resize((size_t)nnz);
  L.pval.resize((size_t)nnz);
  std::vector<int32_t> cur(L.poff);
  for (int64_t r = 0; r < R; ++r)
    for (int64_t j = ptr[r]; j < ptr[r + 1]; ++j) {
      const int b = idx[j] / PN_W;
      const int64_t pos = L.pbase[b] + cur[(size_t)b * R1 + r]++;
      L.pidx[pos] = (uint16_t)(idx[j] - b * PN_W);
      L.pval[pos] = val[j];
    }
  // items and jobs
  const int64_t total = nnz + 2 * (int64_t)np * R;
  const int64_t E = std::max<int64_t>(PN_JOB_MIN, total / std::max(target_jobs, 1));
  L.jobs.clear();
  L.sblk.clear();
  L.witem.clear();
  L.segs.clear();
  L.nslot = 0;
  auto cut = [&](int b, int kind, size_t first, const std::vector<PnDesc>& items) {
    int64_t acc = 0;
    size_t j0 = first;
    for (size_t i = first; i < items.size(); ++i) {
      acc += kind == 0 ? (int64_t)items[i].d + 2 * items[i].b : (int64_t)items[i].c + 64;
      if (acc >= E || i + 1 == items.size()) {
        L.jobs.push_back({b, kind, (int32_t)j0, (int32_t)(i + 1 - j0)});
        j0 = i + 1;
        acc = 0;
      }
    }
  };
  for (int b = 0; b < np; ++b) {
    const int32_t* po = L.poff.data() + (size_t)b * R1;
    const size_t s0 = L.sblk.size(), w0 = L.witem.size();
    int32_t r0 = 0, nr = 0, e0 = 0, ecnt = 0;
    auto flush = [&]() {
      if (nr > 0) L.sblk.push_back({r0, nr, e0, ecnt});
      nr = 0;
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
    cut(b, 0, s0, L.sblk);
    cut(b, 1, w0, L.witem);
  }
}

}  // namespace gkb

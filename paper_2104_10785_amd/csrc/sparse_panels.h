// Column-panel layout of a CSR matrix (internal), host side.
//
// The product y = M x of a CSR matrix M (rows R, columns C) gathers one entry
// of x per stored entry of M.  When x is larger than a few hundred kilobytes
// these gathers miss every cache close to the compute units and their request
// rate, not the bytes of M, bounds the product.  The panel layout cuts the
// columns into panels of PN_W columns (PN_W floats of x fit in the LDS of one
// compute unit) and stores M panel by panel: panel b is the CSR matrix of the
// columns [b PN_W, (b + 1) PN_W) of every row, its column indices relative to
// the panel (16 bits) and its values, each row's entries in their order in M.
// A workgroup loads one panel of x into LDS and then streams a run of that
// panel's entries, so every gather is an LDS read.
//
// The work of one panel is cut into items:
//  * stream blocks: runs of consecutive rows whose segments in the panel hold
//    at most PN_BIG entries, at most PN_BLK entries and PN_ROWS rows per block.
//    The block's products go to LDS; a row of at most PN_SHORT entries is
//    added by one thread in entry order, a longer one (listed with the block)
//    by a wave (lane l adds entries l, l + 64, ... in order, the 64 lane sums
//    meet in a fixed butterfly);
//  * wave items: a segment of more than PN_BIG entries, in chunks of at most
//    PN_CHUNK entries (one wave per chunk, summed like a long row), each chunk
//    with a chunk-sum slot; the slots are added in chunk order afterwards.
// Items are grouped into jobs (one workgroup each) of one panel and one kind.
// Every row's sum in a panel, and the sum over panels in panel order, has a
// fixed order, so the products are bitwise reproducible.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace gkb {

constexpr int PN_W = 28672;      // columns per panel (112 KB of float32 x)
constexpr int PN_T = 1024;       // threads of a panel workgroup
constexpr int PN_SHORT = 32;     // rows of a stream block up to this length are added by one thread
constexpr int PN_BLK = 4096;     // entries of a stream block (4 per thread)
constexpr int PN_BIG = 2048;     // longer segments are cut into wave items
constexpr int PN_ROWS = 1023;    // rows of a stream block (thread t adds row t)
constexpr int PN_CHUNK = 4096;   // entries of a wave item
constexpr int PN_JOB_MIN = 8192; // smallest job cost worth a panel load
constexpr int PN_JOB_ITEMS = 256; // items of a job at most (its descriptors sit in LDS)

// 16-byte descriptor (read on the device as one int4)
struct PnDesc {
  int32_t a, b, c, d;
};

// job: {panel, kind (0 stream blocks, 1 wave items), first item, item count}
// stream block: {first row, rows | entries << 10 | long rows << 23, first entry
//                (relative to the panel), first long row in lrow}
// wave item: {row, first entry (relative to the panel), entries, chunk-sum slot}
// chunked segment: {panel, row, first slot, slots}
struct PanelLayout {
  int64_t R = 0, C = 0, nnz = 0;
  int np = 0;                      // panels
  std::vector<int64_t> pbase;      // np + 1: first entry of each panel
  std::vector<int32_t> poff;       // np x (R + 1): row offsets within each panel
  std::vector<uint16_t> pidx;      // nnz column indices relative to the panel (+ one padding entry)
  std::vector<float> pval;         // nnz values (+ one padding entry)
  std::vector<PnDesc> jobs, sblk, witem, segs;
  std::vector<int32_t> lrow;       // per stream block, its rows of more than PN_SHORT entries
                                   // (row within the block), + one padding entry
  int64_t nslot = 0;
};

// Fields of a stream block's second descriptor word.
inline int32_t pn_pack(int32_t rows, int32_t entries, int32_t longs) { return rows | entries << 10 | longs << 23; }
static_assert(PN_ROWS < (1 << 10) && PN_BLK < (1 << 13) && PN_BLK / (PN_SHORT + 1) < (1 << 8),
              "stream block fields do not fit their bits");

// Whether the panel layout is used for a matrix of this shape: one panel, or
// at most 4 row segments (including empty ones) per stored entry, panels of
// fewer than 2^31 entries and rows below 2^31.
bool panels_suit(int64_t R, int64_t C, int64_t nnz);

// Upper bound of the device bytes of the layout (every array 256-byte
// aligned), from the shape alone; 0 if panels_suit is false.
size_t panel_bytes_bound(int64_t R, int64_t C, int64_t nnz);

// Build the layout from host copies of the CSR arrays (ptr validated by the
// caller: non-decreasing from 0 to nnz; idx in [0, C)).  target_jobs: about
// how many jobs to cut the work into (the compute units: one workgroup each).
void build_panels(int64_t R, int64_t C, int64_t nnz, const int64_t* ptr, const int32_t* idx, const float* val,
                  int target_jobs, PanelLayout& L);

}  // namespace gkb

// Tile binning (paper App. B, Steps 0-1): each (tile, sphere) pair goes into
// its tile's list, so every 8x8 tile gets the spheres whose rectangle touches
// it, and the lists are cut into raster work items.
//
// The paper sorts all spheres by earliest possible depth and then filters
// them per image region. The blend of Eq. 1 is a sum and does not need depth
// order, so here the pairs are placed by a counting sort on the tile number:
//   K2 k_bin_count   bin block g (a run of S spheres) counts its pairs per tile
//                    in LDS and writes row g of the count matrix [G, T]; it
//                    also writes the first emission position of each of its
//                    projection blocks (the sphere-major pair numbering)
//   K3 k_bin_scan    per tile, the exclusive prefix of the counts over g
//                    (in place); the block that finishes last scans the tile
//                    totals into tile ranges and emits the work items
//   K4 k_bin_scatter block g places its pairs: rank inside its (g, tile) cell
//                    from wave ballots and per-wave counts packed into one
//                    64-bit LDS word per tile, so the order is deterministic
// The matrix is sliced by tiles (kBinSlice tiles per block of K2 / K4) so
// its LDS fits whatever the number of tiles.
#include "device_common.h"
#include "pulsar_internal.h"

namespace pulsar {

// The tiles of a sphere's tile rectangle in row-major order have increasing
// tile numbers, so those inside a slice [t0, t1) form one run of that
// enumeration, [e0, e0 + nin). The same enumeration index is the pair's
// place after the sphere's first emission position.
struct RectRun {
  uint32_t e0, nin, w;  // first index in the slice, tiles in the slice, rectangle width
};

__device__ __forceinline__ uint32_t tiles_below(const ushort4& tr, uint32_t tile0,
                                                uint32_t tiles_x, uint32_t t) {
  // tiles of the rectangle with number < t
  const uint32_t w = uint32_t(tr.z) - tr.x + 1u;
  uint32_t below = 0;
  for (uint32_t ty = tr.y; ty <= tr.w; ++ty) {
    const uint32_t first = tile0 + ty * tiles_x + tr.x;
    if (t <= first) break;  // later rows start even higher
    below += min(w, t - first);
  }
  return below;
}

__device__ __forceinline__ RectRun rect_run(const ushort4& tr, uint32_t tile0, uint32_t tiles_x,
                                            uint32_t t0, uint32_t t1) {
  RectRun r;
  r.w = uint32_t(tr.z) - tr.x + 1u;
  const uint32_t last = tile0 + uint32_t(tr.w) * tiles_x + tr.z;
  const uint32_t first = tile0 + uint32_t(tr.y) * tiles_x + tr.x;
  if (last < t0 || first >= t1) {
    r.e0 = 0;
    r.nin = 0;
    return r;
  }
  r.e0 = tiles_below(tr, tile0, tiles_x, t0);
  r.nin = tiles_below(tr, tile0, tiles_x, t1) - r.e0;
  return r;
}

__device__ __forceinline__ uint32_t rect_tile(const ushort4& tr, uint32_t tile0, uint32_t tiles_x,
                                              uint32_t w, uint32_t e) {
  const uint32_t dy = e / w;
  return tile0 + (uint32_t(tr.y) + dy) * tiles_x + tr.x + (e - dy * w);
}

// A work unit of K2 / K4: bin block g of scene b (spheres [i0, i1)) and tile
// slice h ([t0, t1) in the global tile numbering); its counts live in the
// matrix row starting at `row` (indexed by the tile's number in the scene).
struct BinUnit {
  int b;
  int i0, i1;
  uint32_t t0, t1, tile0, tiles_x;
  size_t row;
};

__device__ __forceinline__ BinUnit bin_unit(const SceneDev* __restrict__ scenes,
                                            const uint32_t* __restrict__ unit_start, int B,
                                            uint32_t u) {
  BinUnit r;
  r.b = find_scene(unit_start, B, u);
  const SceneDev& sc = scenes[r.b];
  const uint32_t local = u - sc.unit_off;
  const uint32_t g = local / sc.slices, h = local - g * sc.slices;
  r.i0 = int(sc.sph_off + g * sc.bin_S);
  r.i1 = int(min(sc.sph_off + sc.n, uint32_t(r.i0) + sc.bin_S));
  const uint32_t Tb = uint32_t(sc.cam.tiles_x) * uint32_t(sc.cam.tiles_y);
  r.tile0 = sc.tile_off;
  r.tiles_x = uint32_t(sc.cam.tiles_x);
  r.t0 = sc.tile_off + h * uint32_t(kBinSlice);
  r.t1 = min(sc.tile_off + Tb, r.t0 + uint32_t(kBinSlice));
  r.row = size_t(sc.row_off) + size_t(g) * Tb;
  return r;
}

// K2 block size (no ordering inside it matters), the loads a thread issues at
// once, and the flat pairs of a K4 round whose owner is mapped in LDS
constexpr int kCountThreads = 1024;
constexpr int kBinUnroll = 4;
constexpr int kFlatMap = 1024;
static_assert(kBinThreads <= 256, "owners are stored as bytes");

// ---------------------------------------------------------------- K2
__global__ __launch_bounds__(kCountThreads) void k_bin_count(
    const uint32_t* __restrict__ counts, const ushort4* __restrict__ trect,
    const SceneDev* __restrict__ scenes, const uint32_t* __restrict__ unit_start, int B,
    uint32_t* __restrict__ bmat) {
  __shared__ uint32_t s_cnt[kBinSlice];
  const int tid = threadIdx.x;
  const BinUnit U = bin_unit(scenes, unit_start, B, blockIdx.x);
  for (int k = tid; k < kBinSlice; k += kCountThreads) s_cnt[k] = 0u;
  __syncthreads();
  // kBinUnroll spheres per thread at a time, every load issued before any is used
  for (int base = U.i0; base < U.i1; base += kCountThreads * kBinUnroll) {
    uint32_t c[kBinUnroll];
    ushort4 tr[kBinUnroll];
#pragma unroll
    for (int k = 0; k < kBinUnroll; ++k) {
      const int i = min(base + k * kCountThreads + tid, U.i1 - 1);
      c[k] = counts[i];
      tr[k] = trect[i];
    }
#pragma unroll
    for (int k = 0; k < kBinUnroll; ++k) {
      if (base + k * kCountThreads + tid >= U.i1 || c[k] == 0u) continue;
      const RectRun rr = rect_run(tr[k], U.tile0, U.tiles_x, U.t0, U.t1);
      for (uint32_t e = rr.e0; e < rr.e0 + rr.nin; ++e)
        atomicAdd(&s_cnt[rect_tile(tr[k], U.tile0, U.tiles_x, rr.w, e) - U.t0], 1u);
    }
  }
  __syncthreads();
  uint32_t* row = bmat + U.row - U.tile0;
  for (uint32_t t = U.t0 + uint32_t(tid); t < U.t1; t += kCountThreads) row[t] = s_cnt[t - U.t0];
}

// ---------------------------------------------------------------- K3
// Work items: a tile's list of L pairs is cut into L / chunk full chunks and
// one shorter chunk for the rest. Full chunks of all tiles come first in the
// work list (the costlier items start first), then the short ones. A tile
// with several chunks needs one partial blend state per chunk (slots
// soff .. soff + n - 1), merged afterwards, and is listed for the merge.
struct TileChunks {
  uint32_t nf, np, ns, nm;  // full chunks, short chunks (0/1), partial-state slots, merges (0/1)
};

__device__ __forceinline__ TileChunks chunks_of(uint32_t L, uint32_t chunk) {
  TileChunks c;
  c.nf = L / chunk;
  c.np = (L % chunk) != 0u ? 1u : 0u;
  const uint32_t n = c.nf + c.np;
  c.ns = n >= 2 ? n : 0u;
  c.nm = n >= 2 ? 1u : 0u;
  return c;
}

// Exclusive block-wide scan of one value per thread (kScanThreads threads);
// returns the prefix and leaves the total in *total. Uses s_w[kScanWaves].
template <typename V>
__device__ __forceinline__ V block_excl_scan(V v, V* s_w, V* total) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  V incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const V o = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += o;
  }
  __syncthreads();  // earlier users of s_w are done
  if (lane == kWave - 1) s_w[wid] = incl;
  __syncthreads();
  V before = 0, tot = 0;
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    const V x = s_w[w];
    if (w < wid) before += x;
    tot += x;
  }
  *total = tot;
  return before + incl - v;
}

// Sums of one 64-tile group of K3a: pairs, then the work-item counts.
struct TileGroupSums {
  unsigned long long pairs;
  uint32_t nf, np, ns, nm;
};

// K3a: block k handles tiles 64 k .. 64 k + 63, one per lane. The tile's
// scene has G_b bin blocks; wave w adds rows w Gq .. w Gq + Gq - 1 of the
// tile's column (Gq = ceil(G_b / 16) <= kBinRowsPerWave), all loads issued at
// once, and the per-wave sums give each wave's first offset. Each cell of the
// column becomes its offset inside the tile (in place; cells with no pair are
// never read again); the tile's total and the group's sums are written for
// K3b.
__global__ __launch_bounds__(kScanThreads) void k_bin_scan(
    uint32_t T, SceneTable tab, uint32_t chunk, uint32_t* __restrict__ bmat,
    uint32_t* __restrict__ tcount, TileGroupSums* __restrict__ gsum) {
  constexpr int NW = kScanThreads / kWave;
  __shared__ uint32_t s_part[NW][kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const uint32_t t = blockIdx.x * uint32_t(kWave) + uint32_t(lane);
  const bool in = t < T;
  const SceneDev& sc = tab.scenes[find_scene(tab.tile_start, tab.B, in ? t : T - 1u)];
  const int G = int(sc.bin_G);
  const uint32_t Tb = uint32_t(sc.cam.tiles_x) * uint32_t(sc.cam.tiles_y);
  const size_t col = size_t(sc.row_off) + size_t(in ? t - sc.tile_off : 0u);
  const int Gq = (G + NW - 1) / NW;
  const int g0 = w * Gq;
  uint32_t v[kBinRowsPerWave];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kBinRowsPerWave; ++j) {
    const int g = g0 + j;
    v[j] = (in && j < Gq && g < G) ? bmat[col + size_t(g) * Tb] : 0u;
    sum += v[j];
  }
  s_part[w][lane] = sum;
  __syncthreads();
  uint32_t run = 0, tot = 0;
  for (int k = 0; k < NW; ++k) {
    const uint32_t x = s_part[k][lane];
    if (k < w) run += x;
    tot += x;
  }
#pragma unroll
  for (int j = 0; j < kBinRowsPerWave; ++j) {
    if (v[j] != 0u) bmat[col + size_t(g0 + j) * Tb] = run;
    run += v[j];
  }
  if (w == 0) {
    if (in) tcount[t] = tot;
    const TileChunks c = chunks_of(tot, chunk);
    const unsigned long long pairs = wave_sum_u64(tot);
    const uint32_t nf = wave_sum_u32(c.nf), np = wave_sum_u32(c.np), ns = wave_sum_u32(c.ns),
                   nm = wave_sum_u32(c.nm);
    if (lane == 0) gsum[blockIdx.x] = TileGroupSums{pairs, nf, np, ns, nm};
  }
}

// K3b: block j < ntb plans tiles 1024 j .. 1024 j + 1023, one per thread:
// the group sums of K3a give the totals (which decide a capacity overflow)
// and everything before the block; a block scan does the rest. It writes
// every tile's range in the sorted pair list and its work items; block 0
// also writes the totals. Blocks ntb .. ntb + nbo - 1 write the first
// emission position of 1024 projection blocks each (an exclusive scan of
// their pair counts). Work items of a tile of L pairs: L / chunk full chunks
// and one shorter chunk for the rest; full chunks of all tiles come first in
// the work list (the costlier items start first), then the short ones; a
// tile with several chunks gets one partial blend state per chunk and is
// listed for the merge. After a capacity overflow (outputs invalid) no work
// item is written.
constexpr int kPlanThreads = 1024;

__global__ __launch_bounds__(kPlanThreads) void k_bin_plan(
    uint32_t T, uint32_t ntb, const uint32_t* __restrict__ tcount,
    const TileGroupSums* __restrict__ gsum, long long cap, uint32_t chunk, long long pcap,
    int nblk_proj, const unsigned long long* __restrict__ partials,
    unsigned long long* __restrict__ boff, Status* __restrict__ status,
    uint32_t* __restrict__ ranges, uint4* __restrict__ tinfo, uint4* __restrict__ desc,
    uint32_t* __restrict__ mlist) {
  constexpr int NW = kPlanThreads / kWave;
  __shared__ unsigned long long s_w64[NW], s_red64[2][NW];
  __shared__ uint32_t s_w32[NW], s_red32[8][NW];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  if (blockIdx.x >= ntb) {
    // projection blocks a0 .. a0 + 1023: the sum of all earlier ones, then a scan
    const int a0 = int(blockIdx.x - ntb) * kPlanThreads;
    unsigned long long pre = 0;
    for (int k = tid; k < a0; k += kPlanThreads) pre += partials[k];
    const int pb = a0 + tid;
    const unsigned long long v = pb < nblk_proj ? partials[pb] : 0ull;
    pre = wave_sum_u64(pre);
    if (lane == 0) s_red64[0][wv] = pre;
    __syncthreads();
    unsigned long long before = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) before += s_red64[0][w];
    unsigned long long tot;
    before += block_excl_scan<unsigned long long>(v, s_w64, &tot);
    if (pb < nblk_proj) boff[pb] = before;
    return;
  }
  // group sums: all of them (totals) and those before this block (prefix)
  const uint32_t ng = (T + kWave - 1) / kWave, gfirst = blockIdx.x * uint32_t(NW);
  const uint32_t t = blockIdx.x * uint32_t(kPlanThreads) + uint32_t(tid);
  const uint32_t L = t < T ? tcount[t] : 0u;
  unsigned long long ap = 0, bp = 0;
  uint32_t a[4] = {0u, 0u, 0u, 0u}, bb[4] = {0u, 0u, 0u, 0u};
  for (uint32_t k = uint32_t(tid); k < ng; k += kPlanThreads) {
    const TileGroupSums g = gsum[k];
    const uint32_t x[4] = {g.nf, g.np, g.ns, g.nm};
    ap += g.pairs;
    if (k < gfirst) bp += g.pairs;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] += x[q];
      if (k < gfirst) bb[q] += x[q];
    }
  }
  ap = wave_sum_u64(ap);
  bp = wave_sum_u64(bp);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    a[q] = wave_sum_u32(a[q]);
    bb[q] = wave_sum_u32(bb[q]);
  }
  if (lane == 0) {
    s_red64[0][wv] = ap;
    s_red64[1][wv] = bp;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      s_red32[q][wv] = a[q];
      s_red32[4 + q][wv] = bb[q];
    }
  }
  __syncthreads();
  unsigned long long total = 0, pbefore = 0;
  uint32_t tot4[4] = {0u, 0u, 0u, 0u}, pre4[4] = {0u, 0u, 0u, 0u};
  for (int w = 0; w < NW; ++w) {
    total += s_red64[0][w];
    pbefore += s_red64[1][w];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      tot4[q] += s_red32[q][w];
      pre4[q] += s_red32[4 + q][w];
    }
  }
  const bool over = total > (unsigned long long)cap;
  const bool ok = !over && (long long)tot4[2] <= pcap;
  const unsigned long long used = over ? 0ull : total;
  // this tile's offsets: everything before the block plus the block scan
  const TileChunks c = chunks_of(L, chunk);
  unsigned long long xt;
  uint32_t x32;
  const unsigned long long p =
      pbefore + block_excl_scan<unsigned long long>((unsigned long long)L, s_w64, &xt);
  uint32_t f = pre4[0] + block_excl_scan<uint32_t>(c.nf, s_w32, &x32);
  uint32_t q = tot4[0] + pre4[1] + block_excl_scan<uint32_t>(c.np, s_w32, &x32);
  const uint32_t sl = pre4[2] + block_excl_scan<uint32_t>(c.ns, s_w32, &x32);
  const uint32_t m = pre4[3] + block_excl_scan<uint32_t>(c.nm, s_w32, &x32);
  if (t < T) {
    const uint32_t beg = uint32_t(min(p, used));
    ranges[t] = beg;
    const uint32_t nch = ok ? c.nf + c.np : 0u;
    tinfo[t] = make_uint4(sl, nch, 0u, 0u);
    if (ok && c.nm) mlist[m] = t;
    for (uint32_t ci = 0; ci < nch; ++ci) {
      const uint32_t b = beg + ci * chunk;
      const uint32_t e = min(beg + L, b + chunk);
      const uint32_t slot = nch >= 2 ? sl + ci : kNoSlot;
      const uint32_t at = ci < c.nf ? f++ : q++;
      desc[at] = make_uint4(t | (ci == 0 ? kFirstChunk : 0u), b, e, slot);
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    ranges[T] = uint32_t(used);
    status->pairs = total;
    status->used = uint32_t(used);
    status->code = ok ? 0u : uint32_t(-PULSAR_ERR_CAPACITY);
    status->nfull = ok ? tot4[0] : 0u;
    status->nchunks = ok ? tot4[0] + tot4[1] : 0u;
    status->npartials = ok ? tot4[2] : 0u;
    status->nmerge = ok ? tot4[3] : 0u;
  }
}

// ---------------------------------------------------------------- K4
// Block (g, slice) walks its spheres in rounds of kBinThreads, one sphere per
// thread. The round's pairs in the slice are numbered in (sphere, tile)
// order by a block scan of their counts and placed kBinThreads at a time,
// one per thread (the owner sphere of flat pair p found by binary search).
// The rank of a pair inside its (g, tile) cell is: the pairs of earlier
// steps (a running position per tile), those of earlier waves in this step
// (7-bit per-wave counts packed next to that position in one 64-bit LDS
// word) and those of earlier lanes in this wave (ballot match on the tile).
// Every tile's list therefore holds its spheres in the order of the sphere
// index, whatever the scheduling.
__global__ __launch_bounds__(kBinThreads) void k_bin_scatter(
    const uint32_t* __restrict__ counts, const ushort4* __restrict__ trect,
    const SceneDev* __restrict__ scenes, const uint32_t* __restrict__ unit_start, int B,
    const uint32_t* __restrict__ bmat, const uint32_t* __restrict__ ranges,
    const Status* __restrict__ status, long long cap, uint32_t* __restrict__ vals) {
  constexpr int NW = kBinThreads / kWave;
  static_assert(NW * 7 <= 32, "per-wave counts must fit the low word");
  // per tile of the slice: (next position in the sorted list) << 32 | the
  // per-wave counts of the current step, 7 bits per wave
  __shared__ unsigned long long s_st[kBinSlice];
  // the round's spheres: first flat pair, rectangle, first tile in the slice;
  // the owner of each of the round's first kFlatMap flat pairs
  __shared__ uint32_t s_start[kBinThreads + 1];
  __shared__ ushort4 s_tr[kBinThreads];
  __shared__ uint32_t s_e0[kBinThreads];
  __shared__ uint32_t s_wsum[NW];
  __shared__ uint8_t s_owner[kFlatMap];
  if (status->code != 0u) return;  // capacity exceeded: no work items either
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const BinUnit U = bin_unit(scenes, unit_start, B, blockIdx.x);
  const uint32_t* row = bmat + U.row - U.tile0;
  // the slice's running positions, every load of a batch issued at once
  for (uint32_t t0 = U.t0; t0 < U.t1; t0 += kBinThreads * kBinUnroll) {
    uint32_t rg[kBinUnroll], rw[kBinUnroll];
#pragma unroll
    for (int k = 0; k < kBinUnroll; ++k) {
      const uint32_t t = min(t0 + uint32_t(k * kBinThreads + tid), U.t1 - 1u);
      rg[k] = ranges[t];
      rw[k] = row[t];
    }
#pragma unroll
    for (int k = 0; k < kBinUnroll; ++k) {
      const uint32_t t = t0 + uint32_t(k * kBinThreads + tid);
      if (t < U.t1) s_st[t - U.t0] = (unsigned long long)(rg[k] + rw[k]) << 32;
    }
  }
  const uint64_t lt = lanemask_lt(lane);
  // the first round's sphere, then each round requests the next one's
  int inext = min(U.i0 + tid, U.i1 - 1);
  uint32_t cnext = counts[inext];
  ushort4 trnext = trect[inext];
  for (int r0 = U.i0; r0 < U.i1; r0 += kBinThreads) {
    const int i = r0 + tid;
    const uint32_t c = cnext;
    const ushort4 tr = trnext;
    if (r0 + kBinThreads < U.i1) {
      inext = min(i + kBinThreads, U.i1 - 1);
      cnext = counts[inext];
      trnext = trect[inext];
    }
    RectRun rr;
    rr.e0 = rr.nin = 0;
    rr.w = 1;
    if (i < U.i1 && c != 0u) rr = rect_run(tr, U.tile0, U.tiles_x, U.t0, U.t1);
    // flat numbering of the round's pairs in the slice
    const uint32_t incl = wave_incl_scan_u32(rr.nin, lane);
    __syncthreads();  // the previous round's readers of s_start / s_tr are done
    if (lane == kWave - 1) s_wsum[wv] = incl;
    s_tr[tid] = tr;
    s_e0[tid] = rr.e0;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      before += w < wv ? s_wsum[w] : 0u;
      total += s_wsum[w];
    }
    const uint32_t first = before + incl - rr.nin;
    s_start[tid] = first;
    for (uint32_t k = 0; k < rr.nin && first + k < uint32_t(kFlatMap); ++k)
      s_owner[first + k] = uint8_t(tid);
    __syncthreads();
    for (uint32_t p0 = 0; p0 < total; p0 += kBinThreads) {
      const uint32_t p = p0 + uint32_t(tid);
      const bool act = p < total;
      uint32_t key = 0, sph = 0;
      if (act) {
        // owner: from the map, or past it the last thread whose first flat
        // pair is <= p (it has pairs)
        int lo = 0;
        if (p < uint32_t(kFlatMap)) {
          lo = s_owner[p];
        } else {
          int hi = kBinThreads - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= p)
              lo = mid;
            else
              hi = mid - 1;
          }
        }
        const ushort4 otr = s_tr[lo];
        const uint32_t w = uint32_t(otr.z) - otr.x + 1u;
        key = rect_tile(otr, U.tile0, U.tiles_x, w, s_e0[lo] + (p - s_start[lo])) - U.t0;
        sph = uint32_t(r0 + lo);
      }
      uint64_t peers = __ballot(act);
#pragma unroll
      for (int b = 0; b < kBinSliceBits; ++b) {
        const uint64_t m = __ballot((key >> b) & 1u);
        peers &= ((key >> b) & 1u) ? m : ~m;
      }
      const uint32_t rank = uint32_t(__popcll(peers & lt));
      const bool leader = act && rank == 0u;
      if (leader)
        atomicAdd(&s_st[key], (unsigned long long)__popcll(peers) << (7 * wv));
      __syncthreads();
      unsigned long long upd = 0ull;
      if (act) {
        const unsigned long long st = s_st[key];
        const uint32_t fields = uint32_t(st);
        uint32_t below = 0, cnt = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const uint32_t f = (fields >> (7 * w)) & 127u;
          below += w < wv ? f : 0u;
          cnt += f;
        }
        const unsigned long long dest = (st >> 32) + below + rank;
        if ((long long)dest < cap) vals[dest] = sph;
        // the leader of the lowest wave holding this tile moves the step's
        // count into the running position and clears the per-wave counts
        if (leader && (fields & ((1u << (7 * wv)) - 1u)) == 0u)
          upd = ((unsigned long long)cnt << 32) - (unsigned long long)fields;
      }
      __syncthreads();  // every read of this step's counts is done
      if (upd != 0ull) atomicAdd(&s_st[key], upd);
    }
  }
}

void launch_binning(const Plan& q, char* ws, hipStream_t stream) {
  Status* status = ws_ptr<Status>(ws, q.off_status);
  const SceneTable tab = scene_table(q, ws);
  uint32_t* bmat = ws_ptr<uint32_t>(ws, q.off_bmat);
  const uint32_t T = uint32_t(q.T);
  const uint32_t* counts = ws_ptr<uint32_t>(ws, q.off_counts);
  const ushort4* trect = ws_ptr<ushort4>(ws, q.off_trect);
  uint32_t* tcount = ws_ptr<uint32_t>(ws, q.off_tcount);
  auto* gsum = ws_ptr<TileGroupSums>(ws, q.off_gsum);
  // with no spheres there are no units; the scans still plan the (empty) tiles
  if (q.bin_units > 0)
    hipLaunchKernelGGL(k_bin_count, dim3(unsigned(q.bin_units)), dim3(kCountThreads), 0, stream,
                       counts, trect, tab.scenes, tab.unit_start, q.B, bmat);
  hipLaunchKernelGGL(k_bin_scan, dim3(unsigned((q.T + kWave - 1) / kWave)), dim3(kScanThreads),
                     0, stream, T, tab, uint32_t(q.chunk), bmat, tcount, gsum);
  const uint32_t ntb = uint32_t((q.T + kPlanThreads - 1) / kPlanThreads);
  const uint32_t nbo = uint32_t((q.nblk_proj + kPlanThreads - 1) / kPlanThreads);
  hipLaunchKernelGGL(k_bin_plan, dim3(ntb + nbo), dim3(kPlanThreads), 0, stream, T, ntb, tcount,
                     gsum, (long long)q.cap, uint32_t(q.chunk), (long long)q.pcap, q.nblk_proj,
                     ws_ptr<unsigned long long>(ws, q.off_partials),
                     ws_ptr<unsigned long long>(ws, q.off_boff), status,
                     ws_ptr<uint32_t>(ws, q.off_ranges), ws_ptr<uint4>(ws, q.off_tinfo),
                     ws_ptr<uint4>(ws, q.off_desc), ws_ptr<uint32_t>(ws, q.off_mlist));
  if (q.bin_units > 0)
    hipLaunchKernelGGL(k_bin_scatter, dim3(unsigned(q.bin_units)), dim3(kBinThreads), 0, stream,
                       counts, trect, tab.scenes, tab.unit_start, q.B, bmat,
                       ws_ptr<uint32_t>(ws, q.off_ranges), status, (long long)q.cap,
                       ws_ptr<uint32_t>(ws, q.off_vals));
}

}  // namespace pulsar

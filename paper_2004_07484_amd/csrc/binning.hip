// Tile binning (paper App. B, Steps 0-1): each (tile, sphere) pair goes into
// its tile's list, so every 8x8 tile gets the spheres whose rectangle touches
// it, and the lists are cut into raster work items.
//
// The paper sorts all spheres by earliest possible depth and then filters
// them per image region. The blend of Eq. 1 is a sum and does not need depth
// order, so here the pairs are sorted by tile number only, with a stable LSD
// radix sort that keeps every tile's spheres in index order:
//   k_emit          per block of spheres: their pairs in sphere-major order (a
//                   sphere's first pair sits at the sum of the tile counts of
//                   the spheres before it), the first digit's counts, and the
//                   first pair of each projection block
//   k_sort_hist     the counts of a later digit over blocks of the previous
//                   pass's output
//   k_sort_scatter  one stable pass: each block first derives its digits'
//                   offsets from the digit-major block x digit count matrix
//                   (a few hundred KB at most, read from L2 by every block,
//                   which saves a scan launch), then ranks its pairs among
//                   equal digits with wave ballots and per-wave LDS counts
//   k_ranges        each tile's [first, end) from the boundaries of the
//                   sorted keys; it also publishes the pair count and the
//                   capacity status
//   k_plan          each tile's work items; the list, the partial-state
//                   slots and the merge list are allocated per wave with
//                   atomics, a tile's slots contiguous, so what is computed
//                   does not depend on the allocation order
#include "device_common.h"
#include "pulsar_internal.h"

namespace pulsar {

constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kMaxDigits = 1 << kMaxDigitBits;
static_assert(kEmitRound / kProjectBlock == kEmitThreads / kWave,
              "one wave of an emission round covers one projection block");
static_assert(kEmitThreads == kSortThreads, "the scans below assume one block size");
static_assert(kMaxSortBlocks <= 4 * kWave, "a wave reads a count-matrix row in one load");

// Rows of the count matrix (one per digit, one entry per block) are padded
// to a multiple of 4 entries, so a wave reads a row with one 16-byte load per
// lane.
__host__ __device__ __forceinline__ uint32_t mat_stride(uint32_t nb) { return (nb + 3u) & ~3u; }

// Exclusive block-wide scan of one value per thread (kSortThreads threads);
// returns the prefix and leaves the total in *total. Uses s_w[kSortWaves].
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
#pragma unroll
  for (int w = 0; w < kSortWaves; ++w) {
    const V x = s_w[w];
    if (w < wid) before += x;
    tot += x;
  }
  *total = tot;
  return before + incl - v;
}

// ---------------------------------------------------------------- emission
struct EmitArgs {
  int n;
  const uint32_t* counts;
  const ushort4* trect;
  const unsigned long long* partials;  // pairs per projection block
  SceneTable tab;
  int rounds, nblk, nblk_proj;
  uint32_t T;
  long long cap;
  int digit_bits;  // first digit's width (0: a single tile, nothing to sort)
  uint32_t* keys;
  uint32_t* vals;
  unsigned long long* boff;   // [nblk_proj] first pair of each projection block
  unsigned long long* ebase;  // [nblk + 1] first pair of each emission block
  uint32_t* mat;              // [2^digit_bits][nblk] first digit's counts
  uint2* trange;              // [T] cleared here for k_ranges
  Status* status;             // big_spheres set here
};

// Block b covers spheres b S .. b S + S - 1 (S = rounds kEmitRound) in rounds
// of kEmitRound; thread k of a round owns 4 consecutive spheres, so wave w
// covers exactly projection block (first of the round) + w and the
// projection's in-block prefixes (record word 3.w) are this kernel's wave
// prefixes. The pairs of a sphere are written in row-major order over its
// tile rectangle, which is the order pair_position() numbers them in.
__global__ __launch_bounds__(kEmitThreads) void k_emit(EmitArgs A) {
  __shared__ uint32_t s_hist[kMaxDigits];
  __shared__ unsigned long long s_w64[kSortWaves];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int b = blockIdx.x;
  const int ndig = A.digit_bits > 0 ? 1 << A.digit_bits : 0;
  const uint32_t dmask = uint32_t(ndig) - 1u;
  for (int d = tid; d < ndig; d += kEmitThreads) s_hist[d] = 0u;
  // every tile starts with an empty range
  for (uint32_t t = uint32_t(b) * kEmitThreads + uint32_t(tid); t < A.T;
       t += uint32_t(A.nblk) * kEmitThreads)
    A.trange[t] = make_uint2(0u, 0u);
  // a single scene's tile numbering is the same for every sphere
  const bool one_scene = A.tab.B == 1;
  const uint32_t tile0_1 = one_scene ? A.tab.scenes[0].tile_off : 0u;
  const uint32_t tiles_x_1 = one_scene ? uint32_t(A.tab.scenes[0].cam.tiles_x) : 0u;
  const int pb_per_round = kEmitRound / kProjectBlock;
  const int pb0 = b * A.rounds * pb_per_round;
  const unsigned long long cap = (unsigned long long)A.cap;
  unsigned long long base = 0;
  for (int r = 0; r < A.rounds; ++r) {
    const int i0 = (b * A.rounds + r) * kEmitRound + 4 * tid;
    // the round's loads go out first: counts and rectangles of this
    // thread's 4 spheres (counts and trect are 16-byte aligned and padded,
    // so the vector loads stay inside them)
    uint32_t c[4] = {0u, 0u, 0u, 0u};
    uint4 t01 = make_uint4(0u, 0u, 0u, 0u), t23 = t01;
    if (i0 < A.n) {
      const uint4 c4 = *reinterpret_cast<const uint4*>(A.counts + i0);
      const uint4* tp = reinterpret_cast<const uint4*>(A.trect + i0);
      t01 = tp[0];
      t23 = tp[1];
      c[0] = c4.x;
      c[1] = i0 + 1 < A.n ? c4.y : 0u;
      c[2] = i0 + 2 < A.n ? c4.z : 0u;
      c[3] = i0 + 3 < A.n ? c4.w : 0u;
    }
    if (max(max(c[0], c[1]), max(c[2], c[3])) > kBigTiles) atomicOr(&A.status->big_spheres, 1u);
    if (r == 0) {
      // the pairs of every projection block before this emission block
      unsigned long long pre = 0;
      for (int k = tid; k < pb0 && k < A.nblk_proj; k += kEmitThreads) pre += A.partials[k];
      pre = wave_sum_u64(pre);
      if (lane == 0) s_w64[wv] = pre;
      __syncthreads();
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) base += s_w64[w];
      if (tid == 0) A.ebase[b] = base;
    }
    const unsigned long long tsum =
        (unsigned long long)c[0] + c[1] + (unsigned long long)c[2] + c[3];
    const unsigned long long incl = wave_incl_scan_u64(tsum, lane);
    __syncthreads();  // earlier readers of s_w64 are done
    if (lane == kWave - 1) s_w64[wv] = incl;
    __syncthreads();
    unsigned long long before = 0, rtot = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      const unsigned long long x = s_w64[w];
      if (w < wv) before += x;
      rtot += x;
    }
    const int pb = pb0 + r * pb_per_round + wv;
    if (lane == 0 && pb < A.nblk_proj) A.boff[pb] = base + before;
    unsigned long long pos = base + before + incl - tsum;
    const uint32_t tw[8] = {t01.x, t01.y, t01.z, t01.w, t23.x, t23.y, t23.z, t23.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (c[k] == 0u) continue;
      const uint32_t i = uint32_t(i0 + k);
      // ushort4 (x0, y0, x1, y1) as two words
      const uint32_t x0 = tw[2 * k] & 0xffffu, y0 = tw[2 * k] >> 16;
      const uint32_t x1 = tw[2 * k + 1] & 0xffffu, y1 = tw[2 * k + 1] >> 16;
      uint32_t tile0 = tile0_1, tiles_x = tiles_x_1;
      if (!one_scene) {
        const SceneDev& sc = A.tab.scenes[find_scene(A.tab.sph_start, A.tab.B, i)];
        tile0 = sc.tile_off;
        tiles_x = uint32_t(sc.cam.tiles_x);
      }
      for (uint32_t ty = y0; ty <= y1; ++ty) {
        for (uint32_t tx = x0; tx <= x1; ++tx) {
          const uint32_t t = tile0 + ty * tiles_x + tx;
          if (pos < cap) {
            A.keys[pos] = t;
            A.vals[pos] = i;
          }
          if (ndig) atomicAdd(&s_hist[t & dmask], 1u);
          ++pos;
        }
      }
    }
    base += rtot;
  }
  if (b == A.nblk - 1 && tid == 0) A.ebase[A.nblk] = base;  // the pair total
  __syncthreads();
  for (int d = tid; d < ndig; d += kEmitThreads)
    A.mat[size_t(d) * mat_stride(uint32_t(A.nblk)) + b] = s_hist[d];
}

// ---------------------------------------------------------------- radix sort
struct SortArgs {
  const uint32_t* keys_in;
  const uint32_t* vals_in;
  uint32_t* keys_out;
  uint32_t* vals_out;
  uint32_t* mat;
  const unsigned long long* ebase;  // [nblk_emit + 1] first pair of each emission block
  int nblk_emit;
  int first;        // the first pass: its blocks are the emission blocks
  int shift, bits;  // the digit
  long long cap;
};

// Pairs stored by the emission: all of them, or none past the capacity (the
// call then reports PULSAR_ERR_CAPACITY and sorts nothing).
__device__ __forceinline__ uint32_t stored_pairs(const unsigned long long* ebase, int nblk_emit,
                                                 long long cap) {
  const unsigned long long total = ebase[nblk_emit];
  return total > (unsigned long long)cap ? 0u : uint32_t(total);
}

// Later passes cut the pairs into at most kMaxSortBlocks blocks of a multiple
// of 1024 pairs, at least kSortMinBlock.
__device__ __forceinline__ uint32_t sort_block_size(uint32_t used) {
  const uint32_t per = (used + kMaxSortBlocks - 1u) / kMaxSortBlocks;
  const uint32_t s = (per + 1023u) & ~1023u;
  return s > uint32_t(kSortMinBlock) ? s : uint32_t(kSortMinBlock);
}

// The pairs [beg, end) of sorting block b; false past the last block.
__device__ __forceinline__ bool sort_range(const SortArgs& A, uint32_t used, uint32_t* nb,
                                           uint32_t* beg, uint32_t* end) {
  const uint32_t b = blockIdx.x;
  if (A.first) {
    *nb = uint32_t(A.nblk_emit);
    if (b >= *nb) return false;
    *beg = uint32_t(min(A.ebase[b], (unsigned long long)used));
    *end = uint32_t(min(A.ebase[b + 1], (unsigned long long)used));
    return true;
  }
  const uint32_t S = sort_block_size(used);
  *nb = (used + S - 1u) / S;
  if (b >= *nb) return false;
  *beg = b * S;
  *end = min(*beg + S, used);
  return true;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_hist(SortArgs A) {
  __shared__ uint32_t s_hist[kMaxDigits];
  const uint32_t used = stored_pairs(A.ebase, A.nblk_emit, A.cap);
  uint32_t nb, beg, end;
  if (!sort_range(A, used, &nb, &beg, &end)) return;
  const int tid = threadIdx.x;
  const uint32_t ndig = 1u << A.bits, dmask = ndig - 1u;
  for (uint32_t d = tid; d < ndig; d += kSortThreads) s_hist[d] = 0u;
  __syncthreads();
  for (uint32_t j = beg + uint32_t(tid); j < end; j += kSortThreads)
    atomicAdd(&s_hist[(A.keys_in[j] >> A.shift) & dmask], 1u);
  __syncthreads();
  for (uint32_t d = tid; d < ndig; d += kSortThreads)
    A.mat[size_t(d) * mat_stride(nb) + blockIdx.x] = s_hist[d];
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(SortArgs A) {
  __shared__ uint32_t s_off[kMaxDigits];              // next position of each digit
  __shared__ uint32_t s_below[kMaxDigits];            // the digit's pairs in earlier blocks
  __shared__ uint32_t s_cnt[kSortWaves][kMaxDigits];  // this round's counts per wave
  __shared__ uint32_t s_w[kSortWaves];
  const uint32_t used = stored_pairs(A.ebase, A.nblk_emit, A.cap);
  uint32_t nb, beg, end;
  if (!sort_range(A, used, &nb, &beg, &end)) return;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const uint32_t ndig = 1u << A.bits, dmask = ndig - 1u;
  // the first round's pair is requested before the offsets are worked out;
  // each round then prefetches the next one's
  uint32_t key_next = 0u, val_next = 0u;
  if (beg + uint32_t(tid) < end) {
    key_next = A.keys_in[beg + uint32_t(tid)];
    val_next = A.vals_in[beg + uint32_t(tid)];
  }
  for (uint32_t d = tid; d < ndig; d += kSortThreads) {
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) s_cnt[w][d] = 0u;
  }
  {
    // wave w adds rows w, w + 16, ...: each lane one 16-byte piece of the
    // row, then a wave sum of the digit's total and of its part in blocks
    // before this one
    const uint32_t stride = mat_stride(nb);
    const uint32_t e0 = 4u * uint32_t(lane);
    constexpr int kRowsPerWave = kMaxDigits / kSortWaves;
    uint4 v[kRowsPerWave];
    // every row load is in flight before the first is used
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
      const uint32_t d = uint32_t(wv + k * kSortWaves);
      v[k] = make_uint4(0u, 0u, 0u, 0u);
      if (d < ndig && e0 < nb)
        v[k] = *reinterpret_cast<const uint4*>(A.mat + size_t(d) * stride + e0);
    }
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
      const uint32_t d = uint32_t(wv + k * kSortWaves);
      if (d >= ndig) break;  // wave-uniform
      const uint32_t x[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
      uint32_t tot = 0, below = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t bb = e0 + uint32_t(j);
        const uint32_t xv = bb < nb ? x[j] : 0u;
        tot += xv;
        below += bb < blockIdx.x ? xv : 0u;
      }
      tot = wave_sum_u32(tot);
      below = wave_sum_u32(below);
      if (lane == 0) {
        s_off[d] = tot;
        s_below[d] = below;
      }
    }
  }
  __syncthreads();
  {
    // digit d starts after all smaller digits and after its pairs in earlier blocks
    const uint32_t d = uint32_t(tid);
    const uint32_t v = d < ndig ? s_off[d] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<uint32_t>(v, s_w, &tot);
    __syncthreads();
    if (d < ndig) s_off[d] = ex + s_below[d];
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt(lane);
  for (uint32_t r0 = beg; r0 < end; r0 += kSortThreads) {
    const uint32_t j = r0 + uint32_t(tid);
    const bool valid = j < end;
    const uint32_t key = key_next, val = val_next;
    if (j + kSortThreads < end) {
      key_next = A.keys_in[j + kSortThreads];
      val_next = A.vals_in[j + kSortThreads];
    }
    const uint32_t d = (key >> A.shift) & dmask;
    // the lanes of this wave with the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kMaxDigitBits; ++bit) {
      if (bit >= A.bits) break;
      const uint64_t m = __ballot((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? m : ~m;
    }
    const uint32_t below = uint32_t(__popcll(peers & lt));
    if (valid && below == 0u) s_cnt[wv][d] = uint32_t(__popcll(peers));
    __syncthreads();
    if (valid) {
      uint32_t rank = s_off[d] + below;
      for (int w = 0; w < wv; ++w) rank += s_cnt[w][d];
      if (rank < used) {  // always, as the counts and the pairs are the same
        A.keys_out[rank] = key;
        A.vals_out[rank] = val;
      }
    }
    __syncthreads();  // every rank of this round is taken
    for (uint32_t dd = tid; dd < ndig; dd += kSortThreads) {
      uint32_t add = 0;
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) {
        add += s_cnt[w][dd];
        s_cnt[w][dd] = 0u;
      }
      s_off[dd] += add;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- tiles
// A tile's pairs are the run of its number in the sorted keys: its first pair
// is where the key changes to it, its end where the key changes from it.
// Tiles with no pair keep the empty range k_emit wrote. Block 0 also writes
// the call's pair count and capacity status and clears the work-item
// counters for k_plan.
__global__ __launch_bounds__(1024) void k_ranges(uint32_t T, const uint32_t* __restrict__ keys,
                                                 const unsigned long long* __restrict__ ebase,
                                                 int nblk_emit, long long cap, uint32_t hits_k,
                                                 Status* __restrict__ status,
                                                 uint2* __restrict__ trange) {
  const unsigned long long total = ebase[nblk_emit];
  const uint32_t used = stored_pairs(ebase, nblk_emit, cap);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    status->hits_k = hits_k;  // the raster pass that follows stores them
    status->pairs = total;
    status->used = used;
    status->code = total > (unsigned long long)cap ? uint32_t(-PULSAR_ERR_CAPACITY)
                   : status->bad_cam != 0u            ? uint32_t(-PULSAR_ERR_INVALID_ARGUMENT)
                                                      : 0u;
    status->nfull = 0u;
    status->nshort = 0u;
    status->npartials = 0u;
    status->nmerge = 0u;
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < used; i += gridDim.x * blockDim.x) {
    const uint32_t k = keys[i];
    if (k >= T) continue;  // never: keys are tile numbers
    if (i == 0u || keys[i - 1u] != k) trange[k].x = i;
    if (i + 1u == used || keys[i + 1u] != k) trange[k].y = i + 1u;
  }
}

// Work items: a tile's list of L pairs is cut into L / chunk full chunks and
// one shorter chunk for the rest. A tile with several chunks needs one partial
// blend state per chunk, merged afterwards, and is listed for the merge.
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

// Allocates (a, b) units per lane from the adjacent counters ctr[0], ctr[1]
// for the whole wave with one 64-bit atomic (neither count reaches 2^32);
// returns the lane's first unit of each.
__device__ __forceinline__ uint2 wave_alloc2(uint32_t* ctr, uint32_t a, uint32_t b, int lane) {
  const uint32_t ia = wave_incl_scan_u32(a, lane), ib = wave_incl_scan_u32(b, lane);
  const uint32_t ta = __builtin_amdgcn_readlane(ia, kWave - 1);
  const uint32_t tb = __builtin_amdgcn_readlane(ib, kWave - 1);
  unsigned long long base = 0;
  if (lane == 0 && (ta | tb) != 0u)
    base = atomicAdd(reinterpret_cast<unsigned long long*>(ctr),
                     (unsigned long long)ta | ((unsigned long long)tb << 32));
  const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(base), 0);
  const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(base >> 32), 0);
  return make_uint2(lo + ia - a, hi + ib - b);
}

constexpr int kPlanThreads = 256;

// One tile per thread: its work items (full chunks from the front of the
// list, the short one from the back), its contiguous partial-state slots and
// its merge entry. The bounds cannot be exceeded when the pairs fit the
// capacity (at most cap / chunk + T items, 2 cap / chunk + 1 slots, T merge
// tiles); they are checked anyway, and a violation is reported as a
// capacity overflow, after which no work item is taken.
__global__ __launch_bounds__(kPlanThreads) void k_plan(uint32_t T, const uint2* __restrict__ trange,
                                                        uint32_t chunk, long long pcap,
                                                        uint32_t max_items, Status* status,
                                                        uint4* __restrict__ tinfo,
                                                        uint4* __restrict__ desc,
                                                        uint4* __restrict__ mlist) {
  const uint32_t t = blockIdx.x * kPlanThreads + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const bool ok = status->code == 0u;
  const uint2 tr = (t < T && ok) ? trange[t] : make_uint2(0u, 0u);
  const TileChunks c = chunks_of(tr.y - tr.x, chunk);
  const uint2 fs = wave_alloc2(&status->nfull, c.nf, c.np, lane);
  const uint2 pm = wave_alloc2(&status->npartials, c.ns, c.nm, lane);
  const uint32_t f0 = fs.x, s0 = fs.y, sl = pm.x, m = pm.y;
  if (t >= T) return;
  const uint32_t nch = c.nf + c.np;
  const bool fits = (long long)sl + c.ns <= pcap && f0 + c.nf <= max_items &&
                    s0 + c.np <= max_items && m + c.nm <= T;
  if (!fits) atomicMax(&status->code, uint32_t(-PULSAR_ERR_CAPACITY));
  tinfo[t] = make_uint4(sl, fits ? nch : 0u, 0u, 0u);
  if (!fits) return;
  if (c.nm) mlist[m] = make_uint4(t, sl, nch, 0u);
  for (uint32_t ci = 0; ci < nch; ++ci) {
    const uint32_t b = tr.x + ci * chunk;
    const uint32_t e = min(tr.y, b + chunk);
    const uint32_t slot = nch >= 2 ? sl + ci : kNoSlot;
    const uint32_t at = ci < c.nf ? f0 + ci : max_items - 1u - s0;
    desc[at] = make_uint4(t | (ci == 0 ? kFirstChunk : 0u), b, e, slot);
  }
}

// ---------------------------------------------------------------- early termination
// With early termination every tile's list is put in ascending order of
// (earliest possible hit distance, sphere index): the order of the paper's
// depth sort (App. B, Step 0), which the tile lists keep per tile. One block
// per tile sorts 64-bit keys (distance bits above the index; distances are
// positive, so their bits order like the floats) with a bitonic network whose
// every compare-exchange puts the smaller key first: each merge of two
// sorted runs of k/2 starts by comparing element i with its mirror
// i ^ (k - 1), then halves. Positions past the list's end act as +infinity
// keys; with every exchange ascending they never swap, so those compares are
// skipped and a list of any length sorts in place. In LDS for up to
// kTileSortLds keys, else on the list in global memory (each compare gathers
// the two distances), which only extreme scenes need.
constexpr int kTileSortThreads = 256;
constexpr int kTileSortLds = 4096;

__device__ __forceinline__ uint64_t depth_key(const float* __restrict__ tmin, uint32_t sph) {
  return (uint64_t(__float_as_uint(tmin[sph])) << 32) | uint64_t(sph);
}

// One step of the network over L keys: partner of i is i ^ (k - 1) in the
// first step of a merge (flip), i ^ j after it.
template <typename Get, typename Put>
__device__ __forceinline__ void bitonic_step(uint32_t L, uint32_t mask, bool flip, Get get,
                                             Put put) {
  for (uint32_t i = threadIdx.x; i < L; i += kTileSortThreads) {
    const uint32_t ij = i ^ mask;
    if (ij > i && ij < L) {
      const uint64_t a = get(i), b = get(ij);
      if (a > b) {
        put(i, b);
        put(ij, a);
      }
    }
  }
  (void)flip;
}

__global__ __launch_bounds__(kTileSortThreads) void k_tile_sort(
    uint32_t T, const uint2* __restrict__ trange, const float* __restrict__ tmin,
    const Status* __restrict__ status, uint32_t* __restrict__ vals) {
  __shared__ uint64_t s_key[kTileSortLds];
  if (status->code != 0u) return;
  const uint32_t t = blockIdx.x;
  if (t >= T) return;
  const uint2 tr = trange[t];
  const uint32_t L = tr.y - tr.x;
  if (L < 2u) return;
  uint32_t m = 2;
  while (m < L) m <<= 1;
  uint32_t* v = vals + tr.x;
  if (L <= uint32_t(kTileSortLds)) {
    for (uint32_t i = threadIdx.x; i < L; i += kTileSortThreads) s_key[i] = depth_key(tmin, v[i]);
    __syncthreads();
    auto get = [&](uint32_t i) { return s_key[i]; };
    auto put = [&](uint32_t i, uint64_t x) { s_key[i] = x; };
    for (uint32_t k = 2; k <= m; k <<= 1) {
      bitonic_step(L, k - 1u, true, get, put);
      __syncthreads();
      for (uint32_t j = k >> 2; j > 0; j >>= 1) {
        bitonic_step(L, j, false, get, put);
        __syncthreads();
      }
    }
    for (uint32_t i = threadIdx.x; i < L; i += kTileSortThreads) v[i] = uint32_t(s_key[i]);
    return;
  }
  auto get = [&](uint32_t i) { return depth_key(tmin, v[i]); };
  auto put = [&](uint32_t i, uint64_t x) { v[i] = uint32_t(x); };
  for (uint32_t k = 2; k <= m; k <<= 1) {
    bitonic_step(L, k - 1u, true, get, put);
    __threadfence_block();
    __syncthreads();
    for (uint32_t j = k >> 2; j > 0; j >>= 1) {
      bitonic_step(L, j, false, get, put);
      __threadfence_block();
      __syncthreads();
    }
  }
}

void launch_binning(const Plan& q, char* ws, hipStream_t stream) {
  Status* status = ws_ptr<Status>(ws, q.off_status);
  // pass p reads buffer p % 2 and writes the other; the last pass ends in
  // off_keys / off_vals, so the pairs are emitted where that parity starts
  const bool odd = (q.sort_passes & 1) != 0;
  uint32_t* keys[2] = {ws_ptr<uint32_t>(ws, odd ? q.off_keys2 : q.off_keys),
                       ws_ptr<uint32_t>(ws, odd ? q.off_keys : q.off_keys2)};
  uint32_t* vals[2] = {ws_ptr<uint32_t>(ws, odd ? q.off_vals2 : q.off_vals),
                       ws_ptr<uint32_t>(ws, odd ? q.off_vals : q.off_vals2)};
  EmitArgs E;
  E.n = int(q.n);
  E.counts = ws_ptr<uint32_t>(ws, q.off_counts);
  E.trect = ws_ptr<ushort4>(ws, q.off_trect);
  E.partials = ws_ptr<unsigned long long>(ws, q.off_partials);
  E.tab = scene_table(q, ws);
  E.rounds = q.emit_rounds;
  E.nblk = q.nblk_emit;
  E.nblk_proj = q.nblk_proj;
  E.T = uint32_t(q.T);
  E.cap = q.cap;
  E.digit_bits = q.sort_digit;
  E.keys = keys[0];
  E.vals = vals[0];
  E.boff = ws_ptr<unsigned long long>(ws, q.off_boff);
  E.ebase = ws_ptr<unsigned long long>(ws, q.off_ebase);
  E.mat = ws_ptr<uint32_t>(ws, q.off_mat);
  E.trange = ws_ptr<uint2>(ws, q.off_trange);
  E.status = status;
  hipLaunchKernelGGL(k_emit, dim3(unsigned(q.nblk_emit)), dim3(kEmitThreads), 0, stream, E);
  for (int p = 0; p < q.sort_passes; ++p) {
    SortArgs S;
    S.keys_in = keys[p & 1];
    S.vals_in = vals[p & 1];
    S.keys_out = keys[(p + 1) & 1];
    S.vals_out = vals[(p + 1) & 1];
    S.mat = E.mat;
    S.ebase = E.ebase;
    S.nblk_emit = q.nblk_emit;
    S.first = p == 0 ? 1 : 0;
    S.shift = p * q.sort_digit;
    S.bits = q.sort_digit;
    S.cap = q.cap;
    const unsigned grid = p == 0 ? unsigned(q.nblk_emit) : unsigned(kMaxSortBlocks);
    if (p > 0)
      hipLaunchKernelGGL(k_sort_hist, dim3(grid), dim3(kSortThreads), 0, stream, S);
    hipLaunchKernelGGL(k_sort_scatter, dim3(grid), dim3(kSortThreads), 0, stream, S);
  }
  const long long rg = (q.cap + 4095) / 4096;
  hipLaunchKernelGGL(k_ranges, dim3(unsigned(rg < 256 ? rg : 256)), dim3(1024), 0, stream,
                     uint32_t(q.T), ws_ptr<uint32_t>(ws, q.off_keys), E.ebase, q.nblk_emit,
                     (long long)q.cap, q.store_hits ? uint32_t(q.K) : 0u, status, E.trange);
  hipLaunchKernelGGL(k_plan, dim3(unsigned((q.T + kPlanThreads - 1) / kPlanThreads)),
                     dim3(kPlanThreads), 0, stream, uint32_t(q.T), E.trange, uint32_t(q.chunk),
                     (long long)q.pcap, uint32_t(q.max_chunks), status,
                     ws_ptr<uint4>(ws, q.off_tinfo), ws_ptr<uint4>(ws, q.off_desc),
                     ws_ptr<uint4>(ws, q.off_mlist));
  if (q.estop)
    hipLaunchKernelGGL(k_tile_sort, dim3(unsigned(q.T)), dim3(kTileSortThreads), 0, stream,
                       uint32_t(q.T), E.trange, ws_ptr<float>(ws, q.off_tmin), status,
                       ws_ptr<uint32_t>(ws, q.off_vals));
}

}  // namespace pulsar

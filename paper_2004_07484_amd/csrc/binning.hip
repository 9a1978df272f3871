// Tile binning: K3 emission of (tile, depth) keys (each block first sums the
// projection's per-block tile counts before it), K4 LSD radix sort, K5
// per-tile ranges and the work-item plan.
//
// The paper sorts all spheres by their earliest possible hit depth and then
// filters them per image region (App. B, Step 0 and Step 1). Here the same
// order is reached in one structure: every (tile, sphere) pair gets the key
// tile << depth_bits | quantised depth, and a stable radix sort leaves each
// tile's spheres contiguous and in near-to-far order.
#include "device_common.h"
#include "pulsar_internal.h"

namespace pulsar {

// ---------------------------------------------------------------- K3 emit
// Block b re-scans the tile counts of its spheres and writes one
// (key, sphere id) pair per touched tile, dropping pairs beyond capacity. It
// also records its first emission position (boff, read by the raster
// kernels to place pairs), and the last block writes the pair total and the
// capacity status.
__global__ __launch_bounds__(kProjectBlock) void k_emit(
    int n, const uint32_t* __restrict__ counts, const ushort4* __restrict__ trect,
    const uint32_t* __restrict__ qdepth, const unsigned long long* __restrict__ partials,
    unsigned long long* __restrict__ boff, Status* __restrict__ status,
    SceneTable tab, int depth_bits, long long cap, uint32_t* __restrict__ keys,
    uint32_t* __restrict__ vals, uint32_t* __restrict__ sfirst) {
  __shared__ unsigned long long s_wave[kProjectBlock / kWave], s_pre[kProjectBlock / kWave];
  const int i = blockIdx.x * kProjectBlock + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const uint32_t c = i < n ? counts[i] : 0u;
  // this block's first emission position: the sum of the projection block
  // sums before it (a few KB, read from cache by every block, so no
  // separate scan launch is needed)
  unsigned long long pre = 0;
  {
    // eight independent loads in flight per round
    int k = threadIdx.x;
    for (; k + 7 * kProjectBlock < int(blockIdx.x); k += 8 * kProjectBlock) {
      unsigned long long v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partials[k + u * kProjectBlock];
#pragma unroll
      for (int u = 0; u < 8; ++u) pre += v[u];
    }
    for (; k < int(blockIdx.x); k += kProjectBlock) pre += partials[k];
  }
  pre = wave_sum_u64(pre);
  const unsigned long long incl = wave_incl_scan_u64(c, lane);
  if (lane == kWave - 1) s_wave[wid] = incl;
  if (lane == 0) s_pre[wid] = pre;
  __syncthreads();
  unsigned long long before = 0, btot = 0;
#pragma unroll
  for (int w = 0; w < kProjectBlock / kWave; ++w) {
    before += s_pre[w];
    btot += s_wave[w];
  }
  if (threadIdx.x == 0) {
    boff[blockIdx.x] = before;
    if (blockIdx.x == gridDim.x - 1) {
      // the last block knows the total number of pairs
      const unsigned long long total = before + btot;
      status->pairs = total;
      status->used = uint32_t(total < (unsigned long long)cap ? total : (unsigned long long)cap);
      status->code = total > (unsigned long long)cap ? uint32_t(-PULSAR_ERR_CAPACITY) : 0u;
    }
  }
  for (int w = 0; w < wid; ++w) before += s_wave[w];
  if (c == 0) return;
  unsigned long long at = before + incl - c;
  // the sphere's pairs occupy emission positions sfirst .. sfirst + count - 1,
  // in row-major order over its tile rectangle
  sfirst[i] = uint32_t(at < (unsigned long long)cap ? at : (unsigned long long)cap);
  const ushort4 tr = trect[i];
  const uint32_t q = depth_bits > 0 ? qdepth[i] : 0u;  // no depth in the key: not read
  // tiles are numbered scene by scene, row-major inside each scene
  const SceneDev& sc = tab.scenes[find_scene(tab.sph_start, tab.B, uint32_t(i))];
  const uint32_t tiles_x = uint32_t(sc.cam.tiles_x), tile0 = sc.tile_off;
  for (int ty = tr.y; ty <= tr.w; ++ty) {
    for (int tx = tr.x; tx <= tr.z; ++tx, ++at) {
      if (at >= (unsigned long long)cap) return;
      const uint32_t tile = tile0 + uint32_t(ty) * tiles_x + uint32_t(tx);
      keys[at] = (tile << depth_bits) | q;
      vals[at] = uint32_t(i);
    }
  }
}

// ---------------------------------------------------------------- K4 sort
// LSD radix sort, 8-bit digits, three kernels per pass:
//   hist:    per-block digit counts, digit-major [digit][block]; blocks are
//            taken in XCD-contiguous runs (xcd_block) so the counts of
//            neighbouring blocks, which share cache lines, meet in one L2
//   scan:    one block per digit, exclusive scan over blocks + digit total
//   scatter: stable rank inside the block, then write to the global slot
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(
    const uint32_t* __restrict__ keys, const Status* __restrict__ status, int shift,
    int nblk_cap, uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[kSortRadix];
  const int tid = threadIdx.x;
  const uint32_t used = status->used;
  const uint32_t nb = (used + kSortBlock - 1) / kSortBlock;
  if (blockIdx.x >= nb) return;  // past the stored pairs (uniform)
  const uint32_t lb = xcd_block(blockIdx.x, nb);
  s_h[tid] = 0;
  __syncthreads();
  const size_t base = size_t(lb) * kSortBlock;
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const size_t idx = base + size_t(r) * kSortThreads + tid;
    if (idx < used) atomicAdd(&s_h[(keys[idx] >> shift) & (kSortRadix - 1)], 1u);
  }
  __syncthreads();
  hist[size_t(tid) * nblk_cap + lb] = s_h[tid];
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scan(uint32_t* __restrict__ hist,
                                                            const Status* __restrict__ status,
                                                            int nblk_cap,
                                                            uint32_t* __restrict__ dtot) {
  __shared__ uint32_t s_wave[kSortThreads / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const uint32_t used = status->used;
  const int nblk = int((used + kSortBlock - 1) / kSortBlock);
  uint32_t* row = hist + size_t(blockIdx.x) * nblk_cap;
  uint32_t carry = 0;
  for (int base = 0; base < nblk; base += kSortThreads) {
    const int i = base + tid;
    const uint32_t v = i < nblk ? row[i] : 0u;
    const uint32_t incl = wave_incl_scan_u32(v, lane);
    if (lane == kWave - 1) s_wave[wid] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < kSortThreads / kWave; ++w) {
      const uint32_t x = s_wave[w];
      if (w < wid) before += x;
      total += x;
    }
    if (i < nblk) row[i] = carry + before + incl - v;
    carry += total;
    __syncthreads();
  }
  if (tid == 0) dtot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    const Status* __restrict__ status, int shift, int nblk_cap,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ dtot,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t s_base[kSortRadix];                      // next free slot per digit
  __shared__ uint32_t s_cnt[kSortThreads / kWave][kSortRadix];  // per-wave digit counts
  __shared__ uint32_t s_wave[kSortThreads / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const uint32_t used = status->used;
  const uint32_t nb = (used + kSortBlock - 1) / kSortBlock;
  if (blockIdx.x >= nb) return;  // whole block is past the end (uniform)
  // the same logical block as in k_sort_hist
  const uint32_t lb = xcd_block(blockIdx.x, nb);
  const size_t base = size_t(lb) * kSortBlock;
  // exclusive scan of the digit totals gives each digit's global start
  {
    const uint32_t v = dtot[tid];
    const uint32_t incl = wave_incl_scan_u32(v, lane);
    if (lane == kWave - 1) s_wave[wid] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wid; ++w) before += s_wave[w];
    s_base[tid] = before + incl - v + hist[size_t(tid) * nblk_cap + lb];
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; ++w) s_cnt[w][tid] = 0;
  }
  __syncthreads();
  for (int r = 0; r < kSortRounds; ++r) {
    const size_t idx = base + size_t(r) * kSortThreads + tid;
    const bool valid = idx < used;
    const uint32_t key = valid ? keys_in[idx] : 0u;
    const uint32_t val = valid ? vals_in[idx] : 0u;
    const uint32_t d = (key >> shift) & (kSortRadix - 1);
    // lanes of this wave holding the same digit (valid lanes only)
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t m = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    const uint32_t below = uint32_t(__popcll(peers & lanemask_lt(lane)));
    if (valid && below == 0) s_cnt[wid][d] = uint32_t(__popcll(peers));
    __syncthreads();
    if (valid) {
      uint32_t rank = s_base[d] + below;
      for (int w = 0; w < wid; ++w) rank += s_cnt[w][d];
      keys_out[rank] = key;
      vals_out[rank] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; ++w) {
      add += s_cnt[w][tid];
      s_cnt[w][tid] = 0;
    }
    s_base[tid] += add;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- work items
// Each non-empty tile's list is cut into chunks of at most `chunk` records:
// L / chunk full chunks and one shorter chunk for the rest. Full chunks of
// all tiles come first in the work list (the costlier items start first),
// then the short ones. A tile with several chunks needs one partial blend
// state per chunk (slots soff .. soff + n - 1), merged afterwards; such tiles
// are also listed for the merge kernel. Empty tiles get no work item at all.
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

// K5: ranges[t] = first sorted position whose tile is >= t (binary search
// over the sorted keys), ranges[T] = number of stored pairs; and per block of
// 256 tiles the sums of full chunks, short chunks, partial-state slots and
// merge tiles.
__device__ __forceinline__ uint32_t first_of_tile(const uint32_t* __restrict__ keys,
                                                  uint32_t used, int depth_bits, uint32_t t) {
  uint32_t lo = 0, hi = used;
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if ((keys[mid] >> depth_bits) < t)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_tile_plan(const uint32_t* __restrict__ keys,
                                                   const Status* __restrict__ status, int T,
                                                   int depth_bits, uint32_t chunk,
                                                   uint32_t* __restrict__ ranges,
                                                   uint4* __restrict__ cpart) {
  __shared__ uint32_t s_lo[257];
  __shared__ uint32_t s_f[256 / kWave], s_p[256 / kWave], s_s[256 / kWave], s_m[256 / kWave];
  const uint32_t used = status->used;
  const int t0 = blockIdx.x * 256;
  const int t = t0 + threadIdx.x;
  const uint32_t lo = t < T ? first_of_tile(keys, used, depth_bits, uint32_t(t)) : used;
  s_lo[threadIdx.x] = lo;
  if (threadIdx.x == 0)
    s_lo[256] = t0 + 256 < T ? first_of_tile(keys, used, depth_bits, uint32_t(t0 + 256)) : used;
  if (t < T) ranges[t] = lo;
  if (t == T - 1) ranges[T] = used;
  __syncthreads();
  const TileChunks c = t < T ? chunks_of(s_lo[threadIdx.x + 1] - lo, chunk)
                             : TileChunks{0u, 0u, 0u, 0u};
  const uint32_t f = wave_sum_u32(c.nf), pp = wave_sum_u32(c.np), ss = wave_sum_u32(c.ns),
                 mm = wave_sum_u32(c.nm);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_f[threadIdx.x / kWave] = f;
    s_p[threadIdx.x / kWave] = pp;
    s_s[threadIdx.x / kWave] = ss;
    s_m[threadIdx.x / kWave] = mm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0, b = 0, d = 0, e = 0;
    for (int w = 0; w < 256 / kWave; ++w) {
      a += s_f[w];
      b += s_p[w];
      d += s_s[w];
      e += s_m[w];
    }
    cpart[blockIdx.x] = make_uint4(a, b, d, e);
  }
}

__global__ __launch_bounds__(256) void k_chunk_emit(const uint32_t* __restrict__ ranges, int T,
                                                    uint32_t chunk,
                                                    const uint4* __restrict__ cpart, int nblk,
                                                    long long pcap, Status* __restrict__ status,
                                                    uint4* __restrict__ tinfo,
                                                    uint4* __restrict__ desc,
                                                    uint32_t* __restrict__ mlist) {
  __shared__ uint32_t s_f[256 / kWave], s_p[256 / kWave], s_s[256 / kWave], s_m[256 / kWave];
  __shared__ uint4 s_before, s_total;
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  // this block's offsets and the grand totals: sums over the few block sums
  // (one block per 256 tiles), so no separate scan launch is needed
  {
    uint32_t bf = 0, bp = 0, bs = 0, bm = 0, tf = 0, tp = 0, ts = 0, tm = 0;
    for (int k = threadIdx.x; k < nblk; k += 256) {
      const uint4 v = cpart[k];
      if (k < int(blockIdx.x)) {
        bf += v.x;
        bp += v.y;
        bs += v.z;
        bm += v.w;
      }
      tf += v.x;
      tp += v.y;
      ts += v.z;
      tm += v.w;
    }
    bf = wave_sum_u32(bf);
    bp = wave_sum_u32(bp);
    bs = wave_sum_u32(bs);
    bm = wave_sum_u32(bm);
    tf = wave_sum_u32(tf);
    tp = wave_sum_u32(tp);
    ts = wave_sum_u32(ts);
    tm = wave_sum_u32(tm);
    __shared__ uint4 s_b[256 / kWave], s_t[256 / kWave];
    if (lane == 0) {
      s_b[wid] = make_uint4(bf, bp, bs, bm);
      s_t[wid] = make_uint4(tf, tp, ts, tm);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint4 b = make_uint4(0u, 0u, 0u, 0u), tt = b;
      for (int w = 0; w < 256 / kWave; ++w) {
        b.x += s_b[w].x;
        b.y += s_b[w].y;
        b.z += s_b[w].z;
        b.w += s_b[w].w;
        tt.x += s_t[w].x;
        tt.y += s_t[w].y;
        tt.z += s_t[w].z;
        tt.w += s_t[w].w;
      }
      s_before = b;
      s_total = tt;
      if (blockIdx.x == 0) {
        status->nfull = tt.x;
        status->nchunks = tt.x + tt.y;
        status->npartials = tt.z;
        status->nmerge = tt.w;
        if ((long long)tt.z > pcap) status->code = uint32_t(-PULSAR_ERR_CAPACITY);
      }
    }
    __syncthreads();
  }
  const TileChunks c = t < T ? chunks_of(ranges[t + 1] - ranges[t], chunk)
                             : TileChunks{0u, 0u, 0u, 0u};
  const uint32_t inf = wave_incl_scan_u32(c.nf, lane), inp = wave_incl_scan_u32(c.np, lane),
                 ins = wave_incl_scan_u32(c.ns, lane), inm = wave_incl_scan_u32(c.nm, lane);
  if (lane == kWave - 1) {
    s_f[wid] = inf;
    s_p[wid] = inp;
    s_s[wid] = ins;
    s_m[wid] = inm;
  }
  __syncthreads();
  const uint4 base = s_before;
  const uint32_t nfull = s_total.x;
  uint32_t bf = base.x, bp = base.y, bs = base.z, bm = base.w;
  for (int w = 0; w < wid; ++w) {
    bf += s_f[w];
    bp += s_p[w];
    bs += s_s[w];
    bm += s_m[w];
  }
  if (t >= T) return;
  if (c.nm) mlist[bm + inm - 1u] = uint32_t(t);
  const uint32_t foff = bf + inf - c.nf, poff = nfull + bp + inp - c.np;
  const uint32_t soff = bs + ins - c.ns;
  const uint32_t n = c.nf + c.np;
  tinfo[t] = make_uint4(soff, n, 0u, 0u);
  const uint32_t rb = ranges[t], re = ranges[t + 1];
  for (uint32_t ci = 0; ci < n; ++ci) {
    const uint32_t beg = rb + ci * chunk;
    const uint32_t end = min(re, beg + chunk);
    const uint32_t slot = n >= 2 ? soff + ci : kNoSlot;
    const uint32_t at = ci < c.nf ? foff + ci : poff;
    desc[at] = make_uint4(uint32_t(t) | (ci == 0 ? kFirstChunk : 0u), beg, end, slot);
  }
}

void launch_binning(const Plan& q, char* ws, hipStream_t stream) {
  Status* status = ws_ptr<Status>(ws, q.off_status);
  auto* partials = ws_ptr<unsigned long long>(ws, q.off_partials);
  uint32_t* kA = ws_ptr<uint32_t>(ws, q.off_keysA);
  uint32_t* vA = ws_ptr<uint32_t>(ws, q.off_valsA);
  uint32_t* kB = ws_ptr<uint32_t>(ws, q.off_keysB);
  uint32_t* vB = ws_ptr<uint32_t>(ws, q.off_valsB);
  uint32_t* hist = ws_ptr<uint32_t>(ws, q.off_hist);
  uint32_t* dtot = ws_ptr<uint32_t>(ws, q.off_dtot);
  // with no spheres one block still runs, to write the (empty) status
  hipLaunchKernelGGL(k_emit, dim3(q.nblk_proj > 0 ? unsigned(q.nblk_proj) : 1u),
                     dim3(kProjectBlock), 0, stream, int(q.n), ws_ptr<uint32_t>(ws, q.off_counts),
                     ws_ptr<ushort4>(ws, q.off_trect), ws_ptr<uint32_t>(ws, q.off_qdepth),
                     partials, ws_ptr<unsigned long long>(ws, q.off_boff), status,
                     scene_table(q, ws), q.depth_bits, (long long)q.cap, kA, vA,
                     ws_ptr<uint32_t>(ws, q.off_sfirst));
  for (int p = 0; p < q.passes; ++p) {
    const int shift = 8 * p;
    const uint32_t* kin = (p % 2 == 0) ? kA : kB;
    const uint32_t* vin = (p % 2 == 0) ? vA : vB;
    uint32_t* kout = (p % 2 == 0) ? kB : kA;
    uint32_t* vout = (p % 2 == 0) ? vB : vA;
    hipLaunchKernelGGL(k_sort_hist, dim3(q.nblk_sort), dim3(kSortThreads), 0, stream, kin,
                       status, shift, q.nblk_sort, hist);
    hipLaunchKernelGGL(k_sort_scan, dim3(kSortRadix), dim3(kSortThreads), 0, stream, hist,
                       status, q.nblk_sort, dtot);
    hipLaunchKernelGGL(k_sort_scatter, dim3(q.nblk_sort), dim3(kSortThreads), 0, stream, kin,
                       vin, status, shift, q.nblk_sort, hist, dtot, kout, vout);
  }
  const uint32_t* ksorted = sorted_in_a(q) ? kA : kB;
  const int T = int(q.T);
  uint32_t* ranges = ws_ptr<uint32_t>(ws, q.off_ranges);
  uint4* cpart = ws_ptr<uint4>(ws, q.off_cpart);
  const uint32_t chunk = uint32_t(q.chunk);
  hipLaunchKernelGGL(k_tile_plan, dim3(q.nblk_tiles), dim3(256), 0, stream, ksorted, status, T,
                     q.depth_bits, chunk, ranges, cpart);
  hipLaunchKernelGGL(k_chunk_emit, dim3(q.nblk_tiles), dim3(256), 0, stream, ranges, T, chunk,
                     cpart, q.nblk_tiles, (long long)q.pcap, status,
                     ws_ptr<uint4>(ws, q.off_tinfo), ws_ptr<uint4>(ws, q.off_desc),
                     ws_ptr<uint32_t>(ws, q.off_mlist));
}

}  // namespace pulsar

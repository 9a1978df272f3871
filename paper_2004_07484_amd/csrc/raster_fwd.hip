// K6: forward raster (paper App. B, Steps 1-2; Eq. 1).
//
// Work item = a chunk of at most `chunk` depth-sorted records of one non-empty
// 8x8 tile (long tile lists are split, so no wave walks thousands of spheres
// alone); a persistent grid of one-wave blocks takes work items round-robin,
// full chunks first. A batch of 64 sorted pairs names its spheres; their
// records and payload rows are read in place. Per batch of 64 records:
//   A. sphere-parallel: the (record, pixel of its rectangle inside the tile)
//      pairs are flattened over the lanes by a prefix sum over rectangle
//      sizes; each pair runs the cheap FP32 test and a candidate sets bit l
//      of the pixel's hit mask in LDS;
//   B. pixel-parallel: lane p walks the set bits of its mask in ascending
//      order (the tile list is sorted near to far), decides each hit exactly
//      (hit_geometry.h) and blends it.
// Lane p owns pixel p, so no two lanes write the same pixel. Blending keeps a
// running maximum m of the base-2 exponents and rescales when it grows, so
// exp never overflows down to gamma = 1e-5; every hit enters the sum. When
// a backward pass follows, lane p also keeps its K nearest hits, ordered by
// (t, sphere index). The K-th one becomes the pixel's gradient threshold.
// A tile with one chunk writes its pixels directly; otherwise every chunk
// leaves a partial state (m, D, numerator, K-list) and k_fwd_merge combines
// them in chunk order, so the result is deterministic. After its work items
// the same grid fills the tiles that no sphere touches.
#include <cmath>

#include "hit_geometry.h"

namespace pulsar {

// A hit's place in the K-nearest order: (t, sphere index) as one 64-bit key.
// Hit distances are positive, so their float bits order like unsigned
// integers, and the index breaks ties.
__device__ __forceinline__ uint64_t hit_key(float t, uint32_t id) {
  return (uint64_t(__float_as_uint(t)) << 32) | uint64_t(id);
}
constexpr uint64_t kKeyNone = ~uint64_t(0);  // empty slot (no hit)

// K-list in the last K of KM slots, ascending; the leading KM - K slots hold
// key 0 and never move, so the K-th nearest is always slot KM - 1. Insertion
// compares the new key with every slot at once and shifts the larger ones up.
// The test is wave-uniform: lanes whose key does not enter their list run the
// network as a no-op (every comparison is false).
template <int KM>
__device__ __forceinline__ void klist_insert(uint64_t (&kk)[KM], uint64_t key) {
  if (__ballot(key < kk[KM - 1]) == 0ull) return;
  bool lt[KM];
#pragma unroll
  for (int i = 0; i < KM; ++i) lt[i] = key < kk[i];
#pragma unroll
  for (int i = KM - 1; i > 0; --i) kk[i] = lt[i] ? (lt[i - 1] ? kk[i - 1] : key) : kk[i];
  kk[0] = lt[0] ? key : kk[0];
}

// kk := the KM smallest keys of kk and b, ascending (both ascending): the
// elementwise minimum of kk and reversed b is a bitonic sequence holding
// exactly those keys, which a bitonic half-cleaner network then sorts.
// Keys are unique apart from kKeyNone, so the result equals inserting every
// key of b one by one.
template <int KM>
__device__ __forceinline__ void klist_merge(uint64_t (&kk)[KM], const uint64_t (&b)[KM]) {
#pragma unroll
  for (int i = 0; i < KM; ++i) kk[i] = kk[i] < b[KM - 1 - i] ? kk[i] : b[KM - 1 - i];
#pragma unroll
  for (int d = KM / 2; d > 0; d /= 2) {
#pragma unroll
    for (int i = 0; i < KM; ++i) {
      if ((i & d) == 0) {
        const uint64_t lo = kk[i] < kk[i + d] ? kk[i] : kk[i + d];
        const uint64_t hi = kk[i] < kk[i + d] ? kk[i + d] : kk[i];
        kk[i] = lo;
        kk[i + d] = hi;
      }
    }
  }
}

// A K-list of K < KM keys starts with KM - K fixed zeros (below every key).
// For merging, another list's zeros must leave: its keys move to the front
// and kKeyNone fills the end, which keeps it ascending. z = KM - K is the
// same for every lane, so the shifts by its bits branch uniformly.
template <int KM>
__device__ __forceinline__ void klist_drop_zeros(uint64_t (&b)[KM], int z) {
#pragma unroll
  for (int sh = 1; sh < KM; sh <<= 1) {
    if (z & sh) {
#pragma unroll
      for (int i = 0; i < KM; ++i) b[i] = i + sh < KM ? b[i + sh < KM ? i + sh : 0] : kKeyNone;
    }
  }
}

template <int KM>
__device__ __forceinline__ void klist_init(uint64_t (&kk)[KM], int K) {
#pragma unroll
  for (int i = 0; i < KM; ++i) kk[i] = i < KM - K ? uint64_t(0) : kKeyNone;
}

struct FwdKernelArgs {
  SceneTable tab;
  Status* status;
  const uint4* desc;
  uint32_t max_items;  // capacity of the work list (short items fill it from the back)
  const uint4* tinfo;
  const uint4* mlist;  // (tile, first partial slot, work items) of each tile to merge
  const uint32_t* svals;            // sphere index of every sorted pair
  uint32_t last_sph;                 // n - 1: sorted indices are clamped to it
  const float4* rec;                 // sphere records, rec4 float4 per sphere
  int rec4;                          // 8: the payload row follows the geometry
  const float* payload;              // the caller's payload rows [n, C]
  const float* bg;      // [B, C]
  float* image;
  float* aux;
  float4* thr;  // per pixel: K-th nearest hit (t, sphere index), L of the image, 0
  float* pstate;
  long long pcap;
  int C, c0, cn, K, pstride, kfield;  // kfield: first K-list field of a partial state
  int track;                          // keep K-lists (first channel pass, backward state on)
  int topk;                           // blend only hits up to thr (the K nearest)
  int vec4;                           // one channel pass, C % 4 == 0, 16-byte aligned image
  uint32_t T;                         // tiles of all scenes
  int fill_in_tail;                   // empty tiles filled by the work-item kernel
  float eps2;                         // background exponent (base 2)
  // early termination: each sphere's earliest possible hit distance, the
  // per-pixel first skipped hit (t_min, pair position), and log2 of
  // share / (1 - share)
  const float* tmin;
  float2* stop;
  float lrho2;
  uint2* hits;  // PULSAR_STORE_HITS: per pixel the K nearest (t bits, sphere index)
};

template <int CM, int KM>
__device__ __forceinline__ void write_pixel(const FwdKernelArgs& A, const CamDev& cam,
                                            unsigned long long pix_off, int px, int py,
                                            float m2, float D, const float (&N)[CM],
                                            const uint64_t (&kk)[KM],
                                            uint64_t skey = kKeyNone) {
  if (px >= cam.W || py >= cam.H) return;
  const size_t p = size_t(pix_off) + size_t(py) * size_t(cam.W) + size_t(px);
  const float invD = 1.f / D;
#pragma unroll
  for (int c = 0; c < CM; ++c)
    if (c < A.cn) A.image[p * size_t(A.C) + A.c0 + c] = N[c] * invD;
  const float L = (m2 + fast_log2(D)) * 0.69314718055994531f;
  if (A.c0 == 0 && A.aux) A.aux[p] = L;
  // the top-K blend's own L goes beside the thresholds its first pass left,
  // so the record always holds the L of the image
  if (A.c0 == 0 && A.topk && !A.track) reinterpret_cast<float*>(A.thr + p)[2] = L;
  if (A.track) {
    // the K-th nearest hit, or (+inf, none) when the pixel has fewer than K,
    // with L: one 16-byte record per pixel for the backward's gathers
    const uint64_t k = kk[KM - 1];
    A.thr[p] = k == kKeyNone ? make_float4(INFINITY, __uint_as_float(0xffffffffu), L, 0.f)
                             : make_float4(__uint_as_float(uint32_t(k >> 32)),
                                           __uint_as_float(uint32_t(k)), L, 0.f);
    // the stored K nearest hits, nearest first (kKeyNone where fewer)
    if (A.hits) {
      uint2* hp = A.hits + p * size_t(A.K);
#pragma unroll
      for (int i = 0; i < KM; ++i)
        if (i >= KM - A.K)
          hp[i - (KM - A.K)] = make_uint2(uint32_t(kk[i] >> 32), uint32_t(kk[i]));
    }
    // early termination: the first hit the pixel skipped, or none
    if (A.stop)
      A.stop[p] = make_float2(__uint_as_float(uint32_t(skey >> 32)),
                              __uint_as_float(uint32_t(skey)));
  }
}

// Pixels of a tile without any sphere: F = background and L = eps / gamma
// (no gradient threshold: the backward only visits tiles that have work
// items). One wave; the image is written row by row as contiguous runs of
// (pixels in the row) x C floats, so each store instruction covers
// consecutive addresses.
__device__ __forceinline__ void fill_background_tile(const FwdKernelArgs& A, uint32_t tile,
                                                     int lane) {
  const TileScene ts = tile_scene(A.tab, tile);
  const SceneDev& sc = A.tab.scenes[ts.b];
  const int W = sc.cam.W, H = sc.cam.H, C = A.C;
  const int npx = min(kTileW, W - ts.tx0);    // pixels of the tile inside each row
  const int nrows = min(kTileH, H - ts.ty0);
  const float* bg = A.bg + size_t(ts.b) * size_t(C);
  const int run = npx * C;
  if (A.vec4) {
    // whole channel range in this pass and 16-byte aligned rows: float4 units,
    // so each store instruction writes four rows of the tile at once
    const int run4 = run / 4, cq = C / 4;
    const int units = nrows * run4;
    for (int u = lane; u < units; u += kWave) {
      const int r = u / run4, k = u - r * run4;
      const int q = k % cq;
      float4* row = reinterpret_cast<float4*>(
          A.image + (size_t(sc.pix_off) + size_t(ts.ty0 + r) * size_t(W) + size_t(ts.tx0)) *
                        size_t(C));
      row[k] = make_float4(bg[4 * q], bg[4 * q + 1], bg[4 * q + 2], bg[4 * q + 3]);
    }
  } else {
    for (int r = 0; r < nrows; ++r) {
      float* row = A.image + (size_t(sc.pix_off) + size_t(ts.ty0 + r) * size_t(W) +
                              size_t(ts.tx0)) * size_t(C);
      for (int f = lane; f < run; f += kWave) {
        const int ch = f % C;
        if (ch >= A.c0 && ch < A.c0 + A.cn) row[f] = bg[ch];
      }
    }
  }
  const int px = ts.tx0 + lane % kTileW, py = ts.ty0 + lane / kTileW;
  if (A.c0 == 0 && A.aux && px < W && py < H)
    A.aux[size_t(sc.pix_off) + size_t(py) * size_t(W) + size_t(px)] =
        A.eps2 * 0.69314718055994531f;
}

// Empty-tile fill as a launch of its own (when the work-item grid has more
// than a few tiles per block, as in large batches): a block per
// kBgBlockPixels consecutive pixels of one scene (the background-gradient
// blocks), a thread per pixel, so consecutive threads write consecutive
// pixels; a pixel is written when its tile holds no pair.
constexpr int kBgFillThreads = 256;
__global__ __launch_bounds__(kBgFillThreads) void k_fwd_background(FwdKernelArgs A) {
  const uint32_t blk = blockIdx.x;
  const int b = find_scene(A.tab.blk_start, A.tab.B, blk);
  const SceneDev& sc = A.tab.scenes[b];
  const uint32_t W = uint32_t(sc.cam.W);
  const uint32_t npix = W * uint32_t(sc.cam.H);  // at most 65535^2 < 2^32
  const uint32_t p0 = (blk - sc.bgblk_off) * uint32_t(kBgBlockPixels);
  const uint32_t np = min(uint32_t(kBgBlockPixels), npix - p0);
  // the block's first pixel's row and column; each thread then steps along
  // the row (a division by W once per block, not per pixel)
  const uint32_t y0 = p0 / W, x0 = p0 - y0 * W;
  const float inv_w = 1.f / float(W);
  const uint32_t tiles_x = uint32_t(sc.cam.tiles_x);
  const int C = A.C;
  const float* bg = A.bg + size_t(b) * size_t(C);
  for (uint32_t k = threadIdx.x; k < np; k += kBgFillThreads) {
    // row offset of pixel p0 + k: floor((x0 + k) / W), exact after one correction
    const uint32_t xk = x0 + k;
    uint32_t dy = uint32_t(float(xk) * inv_w);
    if (dy * W > xk) --dy;
    if ((dy + 1u) * W <= xk) ++dy;
    const uint32_t x = xk - dy * W, y = y0 + dy;
    const uint32_t tile = sc.tile_off + (y / kTileH) * tiles_x + x / kTileW;
    if (A.tinfo[tile].y != 0u) continue;
    const size_t p = size_t(sc.pix_off) + size_t(p0 + k);
    float* row = A.image + p * size_t(C);
    for (int c = A.c0; c < A.c0 + A.cn; ++c) row[c] = bg[c];
    if (A.c0 == 0 && A.aux) A.aux[p] = A.eps2 * 0.69314718055994531f;
  }
}

// Up to 8 channels and an 8-entry K-list the work-item kernel fits 128 VGPRs
// (4 waves per SIMD, a few registers spilled outside the hit loop); wider
// instances keep the compiler's own register budget.
// The early-termination instances carry the stop state on top and keep the
// compiler's budget (they spilled at 128).
constexpr int fwd_waves_per_simd(int CM, int KM, bool ES = false) {
  return (!ES && CM <= 8 && KM <= 8) ? 4 : 1;
}

// ES: early termination (tiles are single work items, in depth order).
template <int CM, int KM, bool ES>
__global__ __launch_bounds__(kWave, fwd_waves_per_simd(CM, KM, ES)) void k_fwd_chunks(
    FwdKernelArgs A, const SceneDev* __restrict__ scenes, const uint32_t* __restrict__ tile_start,
    const uint4* __restrict__ desc) {
  // the batch's records (part-major: s_rec[q][r] is float4 q of record r)
  // and payloads (channel-major: s_pay[c][r]); both are filled by
  // global-to-LDS loads, one instruction per record part or channel with
  // lane r fetching record r, so no registers hold them on the way
  __shared__ float4 s_rec[4][kWave];
  __shared__ float s_pay[CM][kWave];
  __shared__ uint32_t s_id[kWave];
  __shared__ unsigned long long s_mask[kWave];
  __shared__ float s_iv2[kWave];
  __shared__ uint2 s_ob[kWave];  // per record: first flattened pair, rectangle
  // bit p % 64 of word p / 64 is set when a record's first pair is p (a
  // batch has at most 64 records of at most 64 pixels, so 64 words suffice)
  __shared__ unsigned long long s_start[kWave];
  __shared__ float s_tmin[ES ? kWave : 1];  // early termination: the records' t_min
  const int lane = threadIdx.x;
  s_start[lane] = 0ull;
  // channels past this pass's width are never loaded: keep them zero
#pragma unroll
  for (int c = 0; c < CM; ++c)
    if (c >= A.cn) s_pay[c][lane] = 0.f;
  // the block's first work item is requested with the status: full chunks
  // fill the list from the front, so for the blocks that take them (the
  // costliest items) slot blockIdx.x is the one
  const uint4 dsc0 = desc[min(blockIdx.x, A.max_items - 1u)];
  const uint32_t nchunks = item_count(A.status), nfull = A.status->nfull;
  for (uint32_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const uint4 dsc =
        (chunk == blockIdx.x && chunk < nfull) ? dsc0 : desc[item_slot(chunk, nfull, A.max_items)];
    const uint32_t tile = dsc.x & ~kFirstChunk;
    const bool first = (dsc.x & kFirstChunk) != 0u;
    const uint32_t beg = dsc.y, end = dsc.z, slot = dsc.w;
    const TileScene ts = tile_scene(scenes, tile_start, A.tab.B, tile);
    const SceneDev& sc = scenes[ts.b];
    const CamDev cam = sc.cam;
    const BlendConst bc = sc.bc;
    const int tx0 = ts.tx0, ty0 = ts.ty0;
    const float* bg = A.bg + size_t(ts.b) * size_t(A.C);
    const PixelRay ray = make_ray(cam, tx0 + (lane % kTileW), ty0 + (lane / kTileW));
    // top-K blend: only hits up to the pixel's K-th nearest (t, id) count
    float tk = INFINITY;
    uint32_t ik = 0xffffffffu;
    if (A.topk && ray.px < cam.W && ray.py < cam.H) {
      const float4 th = A.thr[size_t(sc.pix_off) + size_t(ray.py) * size_t(cam.W) +
                              size_t(ray.px)];
      tk = th.x;
      ik = __float_as_uint(th.y);
    }
    __syncthreads();  // the previous chunk's LDS reads are done
    s_iv2[lane] = ray.inv_v2;
    // the background enters only through the tile's first chunk
    float m2 = first ? bc.eps2 : -INFINITY;
    float D = first ? 1.f : 0.f;
    float N[CM];
#pragma unroll
    for (int c = 0; c < CM; ++c) N[c] = (first && c < A.cn) ? bg[A.c0 + c] : 0.f;
    uint64_t kk[KM];
    klist_init(kk, A.K);
    // early termination: whether this pixel has stopped, and at which hit
    bool done = false;
    uint64_t skey = kKeyNone;
    const bool inside = ray.px < cam.W && ray.py < cam.H;

    // the sorted pairs name their spheres, whose records and payload rows are
    // read in place; lanes past the end repeat the last pair, so every load
    // is unconditional. The next batch's sphere indices are requested with
    // this batch's records, so a batch costs one round trip after the first.
    uint32_t sph_next = min(A.svals[min(beg + uint32_t(lane), end - 1u)], A.last_sph);
    for (uint32_t b0 = beg; b0 < end; b0 += kWave) {
      const uint32_t j = b0 + uint32_t(lane);
      const bool valid = j < end;
      const uint32_t sph = sph_next;
      if (b0 + kWave < end)
        sph_next = min(A.svals[min(j + uint32_t(kWave), end - 1u)], A.last_sph);
      __syncthreads();  // previous batch done with s_rec / s_pay / s_mask
      const float4* rp = A.rec + size_t(A.rec4) * size_t(sph);
#pragma unroll
      for (int q = 0; q < 4; ++q) __builtin_amdgcn_global_load_lds(rp + q, &s_rec[q][0], 16, 0, 0);
      // the payload row: in the record's second half when it fits there
      const float* fp = A.rec4 == 8 ? reinterpret_cast<const float*>(rp + 4) + A.c0
                                    : A.payload + size_t(sph) * size_t(A.C) + A.c0;
#pragma unroll
      for (int c = 0; c < CM; ++c)
        if (c < A.cn) __builtin_amdgcn_global_load_lds(fp + c, &s_pay[c][0], 4, 0, 0);
      if (ES) __builtin_amdgcn_global_load_lds(A.tmin + sph, &s_tmin[0], 4, 0, 0);
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);
      __syncthreads();
      const float4 a = s_rec[0][lane], d = s_rec[3][lane];
      // the sphere index breaks ties of equal hit distances
      const uint32_t id = valid ? sph : 0u;
      // the sphere's rectangle inside this tile, in tile coordinates; the
      // (sphere, pixel) pairs are flattened over the wave by a prefix sum
      const uint32_t p0 = __float_as_uint(a.w), p1 = __float_as_uint(d.z);
      const int xa = max(int(p0 & 0xffffu), tx0) - tx0;
      const int xb = min(int(p1 & 0xffffu), tx0 + kTileW - 1) - tx0;
      const int ya = max(int(p0 >> 16), ty0) - ty0;
      const int yb = min(int(p1 >> 16), ty0 + kTileH - 1) - ty0;
      const uint32_t w = valid ? uint32_t(xb - xa + 1) : 1u;
      const uint32_t n = valid ? w * uint32_t(yb - ya + 1) : 0u;
      const uint32_t incl = wave_incl_scan_u32(n, lane);
      const uint32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
      const uint32_t magic = (65536u + w - 1u) / w;  // i / w = (i * magic) >> 16 for i < 64
      s_ob[lane] = make_uint2(incl - n,
                              uint32_t(xa) | (uint32_t(ya) << 3) | (w << 6) | (magic << 10));
      if (n != 0u) atomicOr(&s_start[(incl - n) >> 6], 1ull << ((incl - n) & 63u));
      s_mask[lane] = 0ull;
      s_id[lane] = id;
      __syncthreads();
      // A. every (record, pixel of its rectangle) pair, 64 at a time. Valid
      // records own at least one pair each, so the owner of a pair is the
      // number of records starting at or before it, minus one: a popcount of
      // the start bits, with no search.
      uint32_t before = 0;  // records starting in earlier blocks of 64 pairs
      const uint64_t stopped = ES ? __ballot(done) : 0ull;  // pixels that take no more hits
      for (uint32_t pb = 0; pb < total; pb += kWave) {
        const unsigned long long starts = s_start[pb >> 6];
        const int r = int(before + uint32_t(__popcll(starts & ((2ull << lane) - 1ull)))) - 1;
        before += uint32_t(__popcll(starts));
        const uint32_t pair = pb + uint32_t(lane);
        if (pair >= total) continue;
        const uint2 ob = s_ob[r];
        const uint32_t i = pair - ob.x, box = ob.y;
        const uint32_t bw = (box >> 6) & 15u, yy = (i * (box >> 10)) >> 16;
        const int x = int(box & 7u) + int(i - yy * bw), y = int((box >> 3) & 7u) + int(yy);
        const int pl = y * kTileW + x;
        const float4 ra = s_rec[0][r], rb = s_rec[1][r];
        const uint32_t pk = __float_as_uint(ra.w);
        const float dx = float(tx0 + x - int(pk & 0xffffu)) - ra.x;
        const float dy = float(ty0 + y - int(pk >> 16)) - ra.y;
        const float cr = rb.x * dy - rb.y * dx;
        const float r2 = ra.z * (dx * dx + dy * dy + cr * cr) * s_iv2[pl];
        if (r2 < kRejectR2 && !((stopped >> pl) & 1ull)) atomicOr(&s_mask[pl], 1ull << r);
      }
      s_start[lane] = 0ull;  // for the next batch (this wave's reads above are issued first)
      __syncthreads();
      // B. pixel p over its candidates, in list order. Every lane runs the
      // same body each round (a lane out of candidates, or missing, changes
      // nothing), so the loop has no divergent join to copy its state at;
      // the rare rescale and K-list insertions branch wave-uniformly.
      unsigned long long hits = s_mask[lane];
      // rounds = the most candidates any lane has (a wave-uniform trip count)
      uint32_t rounds = uint32_t(__popcll(hits));
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) rounds = max(rounds, uint32_t(__shfl_xor(int(rounds), off, 64)));
      rounds = __builtin_amdgcn_readfirstlane(rounds);
      for (uint32_t round = 0; round < rounds; ++round) {
        const bool act = hits != 0ull;
        const int k = act ? __builtin_ctzll(hits) : 0;
        hits &= hits - 1ull;
        const SphereRec s = unpack_rec(s_rec[0][k], s_rec[1][k], s_rec[2][k], s_rec[3][k]);
        Hit h;
        bool hit = exact_hit(ray, s, bc.zfar, h) && act &&
                   (h.t < tk || (h.t == tk && s_id[k] <= ik));
        if (ES) {
          // early termination (Sec. 3.2, App. B Step 2): the hits come in
          // depth-sort order; the first whose largest possible weight
          // exp(z(t_min) / gamma) is below share / (1 - share) of the running
          // denominator stops the pixel, and it and every later hit are
          // skipped (base-2 exponents: D holds the sum over 2^m2)
          if (hit && !done) {
            const float bound2 = (bc.zfar - s_tmin[k]) * bc.kz;
            if (bound2 < A.lrho2 + m2 + fast_log2(D)) {
              done = true;
              skey = hit_key(s_tmin[k], s_id[k]);
            }
          }
          hit = hit && !done;
        }
        const float s2 = s.o * (bc.zfar - h.t) * bc.kz;
        const bool grow = hit && s2 > m2;
        if (__ballot(grow) != 0ull) {
          const float sc = grow ? fast_exp2(m2 - s2) : 1.f;
          D *= sc;
#pragma unroll
          for (int ch = 0; ch < CM; ++ch) N[ch] *= sc;
          m2 = grow ? s2 : m2;
        }
        const float wgt = hit ? s.o * h.delta * fast_exp2(s2 - m2) : 0.f;
        D += wgt;
        float fv[CM];
#pragma unroll
        for (int c = 0; c < CM; ++c) fv[c] = s_pay[c][k];
        // a miss adds nothing, even against a non-finite payload
#pragma unroll
        for (int c = 0; c < CM; ++c) N[c] = hit ? fmaf(wgt, fv[c], N[c]) : N[c];
        if (A.track) klist_insert(kk, hit ? hit_key(h.t, s_id[k]) : kKeyNone);
      }
      // early termination: the tile is done once every pixel has stopped
      if (ES && __ballot(inside && !done) == 0ull) break;
    }

    if (slot == kNoSlot) {
      write_pixel(A, cam, sc.pix_off, ray.px, ray.py, m2, D, N, kk, skey);
    } else {
      if ((long long)slot < A.pcap) {
        float* ps = A.pstate + size_t(slot) * size_t(kWave) * size_t(A.pstride);
        ps[0 * kWave + lane] = m2;
        ps[1 * kWave + lane] = D;
#pragma unroll
        for (int ch = 0; ch < CM; ++ch)
          if (ch < A.cn) ps[(2 + ch) * kWave + lane] = N[ch];
        if (A.track) {
#pragma unroll
          for (int i = 0; i < KM; ++i) {
            ps[(A.kfield + i) * kWave + lane] = __uint_as_float(uint32_t(kk[i] >> 32));
            ps[(A.kfield + KM + i) * kWave + lane] = __uint_as_float(uint32_t(kk[i]));
          }
        }
      }
    }
  }
  // then the tiles that no sphere touches, on the same persistent grid (their
  // fill overlaps the uneven end of the work-item loop). This block owns tiles
  // blockIdx.x + i gridDim.x; the wave tests 64 of them at once and fills the
  // empty ones.
  if (!A.fill_in_tail) return;
  for (uint32_t i0 = 0; blockIdx.x + i0 * gridDim.x < A.T; i0 += kWave) {
    const uint32_t t = blockIdx.x + (i0 + uint32_t(lane)) * gridDim.x;
    uint64_t empty = __ballot(t < A.T && A.tinfo[t].y == 0u);
    while (empty != 0ull) {
      const uint32_t k = uint32_t(__builtin_ctzll(empty));
      empty &= empty - 1ull;
      fill_background_tile(A, blockIdx.x + (i0 + k) * gridDim.x, lane);
    }
  }
}

// Tiles with several work items combine their partial states: four waves per
// tile each fold every fourth state (loading the next one while folding the
// current), then wave 0 folds the other three in wave order. The order is
// fixed, so the result is deterministic. A persistent grid walks the list of
// such tiles.
constexpr int kMergeWaves = 4;
constexpr long long kMergeGrid = 2048;

template <int CM, int KM>
__global__ __launch_bounds__(kWave * kMergeWaves) void k_fwd_merge(
    FwdKernelArgs A, const SceneDev* __restrict__ scenes, const uint32_t* __restrict__ tile_start,
    const uint4* __restrict__ tinfo, const uint4* __restrict__ mlist) {
  constexpr int NF = 2 + CM + 2 * KM;  // m, D, numerator[CM], K-list t[KM], id[KM]
  __shared__ float s_state[kMergeWaves - 1][NF][kWave];
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  // the block's first entry is requested with the status (the list holds
  // T entries, so the read stays inside it whatever the count)
  const uint4 first = mlist[min(blockIdx.x, A.T - 1u)];
  const uint32_t nmerge = A.status->code == 0u ? A.status->nmerge : 0u;
  for (uint32_t mi = blockIdx.x; mi < nmerge; mi += gridDim.x) {
    const uint4 me = mi == blockIdx.x ? first : mlist[mi];
    const int tile = int(me.x);
    const uint4 ti = make_uint4(me.y, me.z, 0u, 0u);  // first slot, partial states
    if ((long long)ti.x + ti.y > A.pcap) continue;  // capacity exceeded (reported)
    float m2 = -INFINITY, D = 0.f, N[CM];
    uint64_t kk[KM];
    klist_init(kk, A.K);
#pragma unroll
    for (int c = 0; c < CM; ++c) N[c] = 0.f;
    float cur[NF], nxt[NF];
    auto load_state = [&](float (&dst)[NF], uint32_t slot) {
      const float* ps = A.pstate + size_t(slot) * size_t(kWave) * size_t(A.pstride);
#pragma unroll
      for (int f = 0; f < 2 + CM; ++f) dst[f] = (f < 2 + A.cn) ? ps[f * kWave + lane] : 0.f;
#pragma unroll
      for (int f = 0; f < 2 * KM; ++f)
        dst[2 + CM + f] = A.track ? ps[(A.kfield + f) * kWave + lane] : 0.f;
    };
    auto fold = [&](const float (&st)[NF]) {
      const float mm = fmaxf(m2, st[0]);
      if (mm > -INFINITY) {
        const float sa = fast_exp2(m2 - mm), sb = fast_exp2(st[0] - mm);
        D = D * sa + st[1] * sb;
#pragma unroll
        for (int c = 0; c < CM; ++c) N[c] = N[c] * sa + st[2 + c] * sb;
        m2 = mm;
      }
      if (A.track) {
        uint64_t other[KM];
#pragma unroll
        for (int i = 0; i < KM; ++i)
          other[i] = (uint64_t(__float_as_uint(st[2 + CM + i])) << 32) |
                     uint64_t(__float_as_uint(st[2 + CM + KM + i]));
        // the other list's fixed leading zeros must not enter this one
        klist_drop_zeros(other, KM - A.K);
        klist_merge(kk, other);
      }
    };
    uint32_t ci = uint32_t(wv);
    if (ci < ti.y) load_state(cur, ti.x + ci);
    for (; ci < ti.y; ci += kMergeWaves) {
      if (ci + kMergeWaves < ti.y) load_state(nxt, ti.x + ci + kMergeWaves);
      fold(cur);
#pragma unroll
      for (int f = 0; f < NF; ++f) cur[f] = nxt[f];
    }
    __syncthreads();  // the previous tile's readers are done with s_state
    if (wv > 0) {
      s_state[wv - 1][0][lane] = m2;
      s_state[wv - 1][1][lane] = D;
#pragma unroll
      for (int c = 0; c < CM; ++c) s_state[wv - 1][2 + c][lane] = N[c];
#pragma unroll
      for (int i = 0; i < KM; ++i) {
        s_state[wv - 1][2 + CM + i][lane] = __uint_as_float(uint32_t(kk[i] >> 32));
        s_state[wv - 1][2 + CM + KM + i][lane] = __uint_as_float(uint32_t(kk[i]));
      }
    }
    __syncthreads();
    if (wv == 0) {
      for (int w = 0; w < kMergeWaves - 1; ++w) {
        float st[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) st[f] = s_state[w][f][lane];
        fold(st);
      }
      const TileScene ts = tile_scene(scenes, tile_start, A.tab.B, uint32_t(tile));
      const SceneDev& sc = scenes[ts.b];
      write_pixel(A, sc.cam, sc.pix_off, ts.tx0 + lane % kTileW, ts.ty0 + lane / kTileW, m2, D,
                  N, kk);
    }
  }
}

void launch_project(const Plan& q, const std::vector<SceneDev>& sc, const FwdArgs& a, char* ws,
                    hipStream_t stream);
void launch_binning(const Plan& q, char* ws, hipStream_t stream);

template <int CM, int KM>
static void launch_raster_fwd_cm(const Plan& q, const FwdKernelArgs& A, hipStream_t stream) {
  stage_begin(PULSAR_STAGE_RASTER_FWD, stream);
  if (q.estop)
    hipLaunchKernelGGL((k_fwd_chunks<CM, KM, true>), dim3(unsigned(q.raster_grid)), dim3(kWave),
                       0, stream, A, A.tab.scenes, A.tab.tile_start, A.desc);
  else
    hipLaunchKernelGGL((k_fwd_chunks<CM, KM, false>), dim3(unsigned(q.raster_grid)), dim3(kWave),
                       0, stream, A, A.tab.scenes, A.tab.tile_start, A.desc);
  if (!A.fill_in_tail && A.image)
    hipLaunchKernelGGL(k_fwd_background, dim3(unsigned(q.nbgblk)), dim3(kBgFillThreads), 0,
                       stream, A);
  stage_end(PULSAR_STAGE_RASTER_FWD, stream);
  stage_begin(PULSAR_STAGE_MERGE, stream);
  // merge tiles are a minority of the tiles; a grid of at most kMergeGrid
  // blocks walks them without paying the dispatch of idle blocks
  long long mg = q.T < q.raster_grid ? q.T : q.raster_grid;
  if (mg > kMergeGrid) mg = kMergeGrid;
  hipLaunchKernelGGL((k_fwd_merge<CM, KM>), dim3(unsigned(mg)), dim3(kWave * kMergeWaves), 0,
                     stream, A, A.tab.scenes, A.tab.tile_start, A.tinfo, A.mlist);
  stage_end(PULSAR_STAGE_MERGE, stream);
}

template <int KM>
static void dispatch_cm(const Plan& q, const FwdKernelArgs& A, hipStream_t stream) {
  if (A.cn <= 1)
    launch_raster_fwd_cm<1, KM>(q, A, stream);
  else if (A.cn <= 2)
    launch_raster_fwd_cm<2, KM>(q, A, stream);
  else if (A.cn <= 4)
    launch_raster_fwd_cm<4, KM>(q, A, stream);
  else if (A.cn <= 8)
    launch_raster_fwd_cm<8, KM>(q, A, stream);
  else if (A.cn <= 16)
    launch_raster_fwd_cm<16, KM>(q, A, stream);
  else
    launch_raster_fwd_cm<32, KM>(q, A, stream);
}

static FwdKernelArgs raster_args(const Plan& q, const std::vector<SceneDev>& scenes,
                                 const FwdArgs& a, char* ws) {
  FwdKernelArgs A;
  A.tab = scene_table(q, ws);
  A.status = ws_ptr<Status>(ws, q.off_status);
  A.desc = ws_ptr<uint4>(ws, q.off_desc);
  A.max_items = uint32_t(q.max_chunks);
  A.tinfo = ws_ptr<uint4>(ws, q.off_tinfo);
  A.mlist = ws_ptr<uint4>(ws, q.off_mlist);
  A.svals = ws_ptr<uint32_t>(ws, q.off_vals);
  A.last_sph = q.n > 0 ? uint32_t(q.n - 1) : 0u;
  A.rec = ws_ptr<float4>(ws, q.off_rec);
  A.rec4 = q.rec4;
  A.payload = a.payload;
  A.bg = a.bg;
  A.image = a.image;
  A.aux = a.aux;
  A.thr = ws_ptr<float4>(ws, q.off_thr);
  A.pstate = ws_ptr<float>(ws, q.off_pstate);
  A.pcap = q.pcap;
  A.C = a.C;
  A.K = a.K;
  A.pstride = q.pstride;
  A.kfield = 2 + q.fwd_cm;
  A.eps2 = scenes[0].bc.eps2;  // eps / gamma does not depend on the camera
  A.T = uint32_t(q.T);
  // a few tiles per block fill well in the tail of the work-item kernel; many
  // more (large batches) get a launch of their own with one wave per tile
  A.fill_in_tail = q.T <= 4LL * q.raster_grid ? 1 : 0;
  A.c0 = 0;
  A.cn = 0;
  A.track = 0;
  A.topk = 0;
  A.vec4 = 0;
  A.tmin = q.estop ? ws_ptr<float>(ws, q.off_tmin) : nullptr;
  A.stop = q.estop ? ws_ptr<float2>(ws, q.off_stop) : nullptr;
  A.hits = q.store_hits ? ws_ptr<uint2>(ws, q.off_hits) : nullptr;
  A.lrho2 = q.estop ? float(std::log2(double(a.stop_share) / (1.0 - double(a.stop_share)))) : 0.f;
  return A;
}


static void dispatch_klist(const Plan& q, const FwdKernelArgs& A, hipStream_t stream) {
  if (q.klist_slots <= 4)
    dispatch_cm<4>(q, A, stream);
  else if (q.klist_slots <= 8)
    dispatch_cm<8>(q, A, stream);
  else if (q.klist_slots <= 16)
    dispatch_cm<16>(q, A, stream);
  else
    dispatch_cm<32>(q, A, stream);
}

// Each pixel's K-th nearest hit into thr: one pass with no channel. The
// weights and K-lists are those of the blending pass (the same summation
// order, so the same thresholds), but no payload is read and neither image,
// log-normaliser nor empty tiles are written.
static void launch_thresholds(const Plan& q, const std::vector<SceneDev>& scenes,
                              const FwdArgs& a, char* ws, hipStream_t stream) {
  FwdKernelArgs A = raster_args(q, scenes, a, ws);
  A.image = nullptr;
  A.aux = nullptr;
  A.fill_in_tail = 0;
  A.track = 1;
  dispatch_klist(q, A, stream);
}

static void launch_tile_lists(const Plan& q, const std::vector<SceneDev>& scenes,
                              const FwdArgs& a, char* ws, hipStream_t stream) {
  stage_begin(PULSAR_STAGE_PROJECT, stream);
  launch_project(q, scenes, a, ws, stream);
  stage_end(PULSAR_STAGE_PROJECT, stream);
  stage_begin(PULSAR_STAGE_BINNING, stream);
  launch_binning(q, ws, stream);
  stage_end(PULSAR_STAGE_BINNING, stream);
}

hipError_t launch_forward(const Plan& q, const std::vector<SceneDev>& scenes, const FwdArgs& a,
                          char* ws, hipStream_t stream) {
  launch_tile_lists(q, scenes, a, ws, stream);
  // the top-K blend needs every pixel's K-th nearest hit before blending
  if (a.topk) launch_thresholds(q, scenes, a, ws, stream);
  FwdKernelArgs A = raster_args(q, scenes, a, ws);
  A.topk = a.topk ? 1 : 0;
  for (int c0 = 0; c0 < a.C; c0 += kFwdChannels) {
    A.c0 = c0;
    A.cn = a.C - c0 < kFwdChannels ? a.C - c0 : kFwdChannels;
    A.track = (c0 == 0 && a.track && !a.topk) ? 1 : 0;
    A.vec4 = (a.C <= kFwdChannels && (a.C & 3) == 0 &&
              (reinterpret_cast<uintptr_t>(a.image) & 15u) == 0u)
                 ? 1
                 : 0;
    dispatch_klist(q, A, stream);
  }
  return hipGetLastError();
}

hipError_t launch_rebin(const Plan& q, const std::vector<SceneDev>& scenes, const FwdArgs& a,
                        char* ws, hipStream_t stream) {
  launch_tile_lists(q, scenes, a, ws, stream);
  launch_thresholds(q, scenes, a, ws, stream);
  return hipGetLastError();
}

}  // namespace pulsar

// K6: forward raster (paper App. B, Steps 1-2; Eq. 1).
//
// Work item = a chunk of at most kChunk depth-sorted records of one 8x8 tile
// (long tile lists are split, so no wave walks thousands of spheres alone);
// a persistent grid of one-wave blocks takes chunks round-robin. Per batch of
// 64 records:
//   A. sphere-parallel: lane l tests record l against the pixels of its own
//      rectangle inside the tile (cheap FP32 test) and sets bit l of each
//      candidate pixel's hit mask in LDS;
//   B. pixel-parallel: lane p walks the set bits of its mask in ascending
//      order (the tile list is sorted near to far), decides each hit exactly
//      (hit_geometry.h) and blends it.
// Lane p owns pixel p, so no two lanes write the same pixel. Blending keeps a
// running maximum m of the base-2 exponents and rescales when it grows, so
// exp never overflows down to gamma = 1e-5; every hit enters the sum. When
// a backward pass follows, lane p also keeps its K nearest hits (t, sphere
// index), and the K-th one becomes the pixel's gradient threshold.
// A tile with one chunk writes its pixels directly; otherwise every chunk
// leaves a partial state (m, D, numerator, K-list) and k_fwd_merge combines
// them in chunk order, so the result is deterministic.
#include "hit_geometry.h"

namespace pulsar {

template <int KM>
__device__ __forceinline__ void klist_insert(float (&kt)[KM], uint32_t (&kid)[KM], float t,
                                             uint32_t id) {
  if (!(t < kt[KM - 1] || (t == kt[KM - 1] && id < kid[KM - 1]))) return;
#pragma unroll
  for (int i = 0; i < KM; ++i) {
    const bool lt = t < kt[i] || (t == kt[i] && id < kid[i]);
    const float tt = kt[i];
    const uint32_t ti = kid[i];
    kt[i] = lt ? t : tt;
    kid[i] = lt ? id : ti;
    t = lt ? tt : t;
    id = lt ? ti : id;
  }
}

// K-list of the last K of KM slots, ascending; leading slots hold -inf and
// never move, so the K-th nearest is always slot KM - 1.
template <int KM>
__device__ __forceinline__ void klist_init(float (&kt)[KM], uint32_t (&kid)[KM], int K) {
#pragma unroll
  for (int i = 0; i < KM; ++i) {
    kt[i] = i < KM - K ? -INFINITY : INFINITY;
    kid[i] = 0xffffffffu;
  }
}

struct FwdKernelArgs {
  const Status* status;
  const uint2* desc;
  const uint4* tinfo;
  const uint32_t* ranges;
  const uint32_t* svals;
  const float4* recA;
  const float4* recB;
  const float4* recC;
  const float4* recD;
  const float* payload;
  const float* bg;
  float* image;
  float* aux;
  float2* thr;
  float* pstate;
  long long pcap;
  int C, c0, cn, K, pstride, kfield;  // kfield: first K-list field of a partial state
  int track;                          // keep K-lists (first channel pass with aux)
};

template <int CM, int KM>
__device__ __forceinline__ void write_pixel(const FwdKernelArgs& A, const CamDev& cam,
                                            int px, int py, float m2, float D,
                                            const float (&N)[CM], const float (&kt)[KM],
                                            const uint32_t (&kid)[KM]) {
  if (px >= cam.W || py >= cam.H) return;
  const size_t p = size_t(py) * size_t(cam.W) + size_t(px);
  const float invD = 1.f / D;
#pragma unroll
  for (int c = 0; c < CM; ++c)
    if (c < A.cn) A.image[p * size_t(A.C) + A.c0 + c] = N[c] * invD;
  if (A.c0 == 0 && A.aux) A.aux[p] = (m2 + fast_log2(D)) * 0.69314718055994531f;
  if (A.track) A.thr[p] = make_float2(kt[KM - 1], __uint_as_float(kid[KM - 1]));
}

template <int CM, int KM>
__global__ __launch_bounds__(kWave) void k_fwd_chunks(FwdKernelArgs A, CamDev cam,
                                                      BlendConst bc) {
  __shared__ float s_rec[14][kWave];  // the batch's records, one field per row
  __shared__ uint32_t s_id[kWave];
  __shared__ float s_pay[CM][kWave];
  __shared__ unsigned long long s_mask[kWave];
  __shared__ float s_iv2[kWave];
  const int lane = threadIdx.x;
  const uint32_t nchunks = A.status->nchunks;
  for (uint32_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const uint2 dsc = A.desc[chunk];
    const int tile = int(dsc.x), ci = int(dsc.y);
    const uint4 ti = A.tinfo[tile];
    const uint32_t beg = A.ranges[tile] + uint32_t(ci) * kChunk;
    const uint32_t end = min(A.ranges[tile + 1], beg + kChunk);
    const int tx0 = (tile % cam.tiles_x) * kTileW, ty0 = (tile / cam.tiles_x) * kTileH;
    const PixelRay ray = make_ray(cam, tx0 + (lane % kTileW), ty0 + (lane / kTileW));
    __syncthreads();  // the previous chunk's LDS reads are done
    s_iv2[lane] = ray.inv_v2;
    // the background enters only through the tile's first chunk
    float m2 = ci == 0 ? bc.eps2 : -INFINITY;
    float D = ci == 0 ? 1.f : 0.f;
    float N[CM];
#pragma unroll
    for (int c = 0; c < CM; ++c) N[c] = (ci == 0 && c < A.cn) ? A.bg[A.c0 + c] : 0.f;
    float kt[KM];
    uint32_t kid[KM];
    klist_init(kt, kid, A.K);

    for (uint32_t b0 = beg; b0 < end; b0 += kWave) {
      const uint32_t j = b0 + uint32_t(lane);
      const bool valid = j < end;
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, c = a, d = a;
      uint32_t id = 0;
      if (valid) {
        id = A.svals[j];
        a = A.recA[id];
        b = A.recB[id];
        c = A.recC[id];
        d = A.recD[id];
      }
      __syncthreads();  // previous batch done with s_rec / s_pay / s_mask
      s_mask[lane] = 0ull;
      s_id[lane] = id;
      s_rec[0][lane] = a.x;
      s_rec[1][lane] = a.y;
      s_rec[2][lane] = a.z;
      s_rec[3][lane] = a.w;
      s_rec[4][lane] = b.x;
      s_rec[5][lane] = b.y;
      s_rec[6][lane] = b.z;
      s_rec[7][lane] = b.w;
      s_rec[8][lane] = c.x;
      s_rec[9][lane] = c.y;
      s_rec[10][lane] = c.z;
      s_rec[11][lane] = c.w;
      s_rec[12][lane] = d.x;
      s_rec[13][lane] = d.y;
      const float* fp = A.payload + size_t(id) * size_t(A.C) + A.c0;
#pragma unroll
      for (int ch = 0; ch < CM; ++ch) s_pay[ch][lane] = (valid && ch < A.cn) ? fp[ch] : 0.f;
      __syncthreads();
      // A. record l against the pixels of its rectangle inside this tile
      if (valid) {
        const uint32_t p0 = __float_as_uint(a.w), p1 = __float_as_uint(d.z);
        const int x0 = int(p0 & 0xffffu), y0 = int(p0 >> 16);
        const int xa = max(x0, tx0), xb = min(int(p1 & 0xffffu), tx0 + kTileW - 1);
        const int ya = max(y0, ty0), yb = min(int(p1 >> 16), ty0 + kTileH - 1);
        const unsigned long long bit = 1ull << lane;
        for (int iy = ya; iy <= yb; ++iy) {
          const float dy = float(iy - y0) - a.y;
          for (int ix = xa; ix <= xb; ++ix) {
            const float dx = float(ix - x0) - a.x;
            const float cr = b.x * dy - b.y * dx;
            const int pl = (iy - ty0) * kTileW + (ix - tx0);
            const float r2 = a.z * (dx * dx + dy * dy + cr * cr) * s_iv2[pl];
            if (r2 < kRejectR2) atomicOr(&s_mask[pl], bit);
          }
        }
      }
      __syncthreads();
      // B. pixel p over its candidates, near to far
      unsigned long long hits = s_mask[lane];
      while (__ballot(hits != 0ull) != 0ull) {
        if (hits != 0ull) {
          const int k = __builtin_ctzll(hits);
          hits &= hits - 1ull;
          SphereRec s;
          const uint32_t pk = __float_as_uint(s_rec[3][k]);
          s.x0 = int(pk & 0xffffu);
          s.y0 = int(pk >> 16);
          s.xh = s_rec[0][k];
          s.yh = s_rec[1][k];
          s.kh = s_rec[2][k];
          s.axh = s_rec[4][k];
          s.ayh = s_rec[5][k];
          s.cz = s_rec[6][k];
          s.R = s_rec[7][k];
          s.xl = s_rec[8][k];
          s.yl = s_rec[9][k];
          s.kl = s_rec[10][k];
          s.axl = s_rec[11][k];
          s.ayl = s_rec[12][k];
          s.o = s_rec[13][k];
          Hit h;
          if (exact_hit(ray, s, bc.zfar, h)) {
            const float s2 = s.o * (bc.zfar - h.t) * bc.kz;
            if (s2 > m2) {
              const float sc = fast_exp2(m2 - s2);
              D *= sc;
#pragma unroll
              for (int ch = 0; ch < CM; ++ch) N[ch] *= sc;
              m2 = s2;
            }
            const float wgt = s.o * h.delta * fast_exp2(s2 - m2);
            D += wgt;
#pragma unroll
            for (int ch = 0; ch < CM; ++ch) N[ch] += wgt * s_pay[ch][k];
            if (A.track) klist_insert(kt, kid, h.t, s_id[k]);
          }
        }
      }
    }

    if (ti.y == 1) {
      write_pixel(A, cam, ray.px, ray.py, m2, D, N, kt, kid);
    } else {
      const long long slot = (long long)ti.z + ci;
      if (slot < A.pcap) {
        float* ps = A.pstate + size_t(slot) * size_t(kWave) * size_t(A.pstride);
        ps[0 * kWave + lane] = m2;
        ps[1 * kWave + lane] = D;
#pragma unroll
        for (int ch = 0; ch < CM; ++ch)
          if (ch < A.cn) ps[(2 + ch) * kWave + lane] = N[ch];
        if (A.track) {
#pragma unroll
          for (int i = 0; i < KM; ++i) {
            ps[(A.kfield + i) * kWave + lane] = kt[i];
            ps[(A.kfield + KM + i) * kWave + lane] = __uint_as_float(kid[i]);
          }
        }
      }
    }
  }
}

// Combines the partial states of tiles with several chunks, in chunk order.
template <int CM, int KM>
__global__ __launch_bounds__(kWave) void k_fwd_merge(FwdKernelArgs A, CamDev cam) {
  const int tile = blockIdx.x;
  const int lane = threadIdx.x;
  const uint4 ti = A.tinfo[tile];
  if (ti.y < 2 || (long long)ti.z + ti.y > A.pcap) return;
  const int px = (tile % cam.tiles_x) * kTileW + (lane % kTileW);
  const int py = (tile / cam.tiles_x) * kTileH + (lane / kTileW);
  float m2 = -INFINITY, D = 0.f, N[CM];
  float kt[KM];
  uint32_t kid[KM];
  klist_init(kt, kid, A.K);
#pragma unroll
  for (int c = 0; c < CM; ++c) N[c] = 0.f;
  for (uint32_t ci = 0; ci < ti.y; ++ci) {
    const float* ps = A.pstate + size_t(ti.z + ci) * size_t(kWave) * size_t(A.pstride);
    const float pm = ps[0 * kWave + lane], pD = ps[1 * kWave + lane];
    // the first chunk holds the background, so m2 is finite from there on
    const float mm = ci == 0 ? pm : fmaxf(m2, pm);
    const float sa = ci == 0 ? 0.f : fast_exp2(m2 - mm), sb = fast_exp2(pm - mm);
    D = D * sa + pD * sb;
#pragma unroll
    for (int c = 0; c < CM; ++c)
      if (c < A.cn) N[c] = N[c] * sa + ps[(2 + c) * kWave + lane] * sb;
    m2 = mm;
    if (A.track) {
#pragma unroll
      for (int i = 0; i < KM; ++i) {
        const float t = ps[(A.kfield + i) * kWave + lane];
        if (t < INFINITY && t > -INFINITY)
          klist_insert(kt, kid, t, __float_as_uint(ps[(A.kfield + KM + i) * kWave + lane]));
      }
    }
  }
  write_pixel(A, cam, px, py, m2, D, N, kt, kid);
}

void launch_project(const Plan& q, const CamDev& cam, const FwdArgs& a, char* ws,
                    hipStream_t stream);
void launch_binning(const Plan& q, char* ws, hipStream_t stream);

template <int CM, int KM>
static void launch_raster_fwd_cm(const Plan& q, const CamDev& cam, const BlendConst& bc,
                                 const FwdKernelArgs& A, hipStream_t stream) {
  hipLaunchKernelGGL((k_fwd_chunks<CM, KM>), dim3(kRasterGrid), dim3(kWave), 0, stream, A, cam,
                     bc);
  hipLaunchKernelGGL((k_fwd_merge<CM, KM>), dim3(unsigned(q.T)), dim3(kWave), 0, stream, A, cam);
}

template <int KM>
static void dispatch_cm(const Plan& q, const CamDev& cam, const BlendConst& bc,
                        const FwdKernelArgs& A, hipStream_t stream) {
  if (A.cn <= 1)
    launch_raster_fwd_cm<1, KM>(q, cam, bc, A, stream);
  else if (A.cn <= 2)
    launch_raster_fwd_cm<2, KM>(q, cam, bc, A, stream);
  else if (A.cn <= 4)
    launch_raster_fwd_cm<4, KM>(q, cam, bc, A, stream);
  else if (A.cn <= 8)
    launch_raster_fwd_cm<8, KM>(q, cam, bc, A, stream);
  else if (A.cn <= 16)
    launch_raster_fwd_cm<16, KM>(q, cam, bc, A, stream);
  else
    launch_raster_fwd_cm<32, KM>(q, cam, bc, A, stream);
}

hipError_t launch_forward(const Plan& q, const CamDev& cam, const BlendConst& bc,
                          const FwdArgs& a, char* ws, hipStream_t stream) {
  stage_begin(PULSAR_STAGE_PROJECT, stream);
  launch_project(q, cam, a, ws, stream);
  stage_end(PULSAR_STAGE_PROJECT, stream);
  stage_begin(PULSAR_STAGE_BINNING, stream);
  launch_binning(q, ws, stream);
  stage_end(PULSAR_STAGE_BINNING, stream);
  stage_begin(PULSAR_STAGE_RASTER_FWD, stream);
  FwdKernelArgs A;
  A.status = ws_ptr<Status>(ws, q.off_status);
  A.desc = ws_ptr<uint2>(ws, q.off_desc);
  A.tinfo = ws_ptr<uint4>(ws, q.off_tinfo);
  A.ranges = ws_ptr<uint32_t>(ws, q.off_ranges);
  A.svals = ws_ptr<uint32_t>(ws, sorted_in_a(q) ? q.off_valsA : q.off_valsB);
  A.recA = ws_ptr<float4>(ws, q.off_recA);
  A.recB = ws_ptr<float4>(ws, q.off_recB);
  A.recC = ws_ptr<float4>(ws, q.off_recC);
  A.recD = ws_ptr<float4>(ws, q.off_recD);
  A.payload = a.payload;
  A.bg = a.bg;
  A.image = a.image;
  A.aux = a.aux;
  A.thr = ws_ptr<float2>(ws, q.off_thr);
  A.pstate = ws_ptr<float>(ws, q.off_pstate);
  A.pcap = q.pcap;
  A.C = a.C;
  A.K = a.K;
  A.pstride = q.pstride;
  A.kfield = 2 + q.fwd_cm;
  for (int c0 = 0; c0 < a.C; c0 += kFwdChannels) {
    A.c0 = c0;
    A.cn = a.C - c0 < kFwdChannels ? a.C - c0 : kFwdChannels;
    A.track = (c0 == 0 && a.aux != nullptr) ? 1 : 0;
    if (q.klist_slots <= 4)
      dispatch_cm<4>(q, cam, bc, A, stream);
    else if (q.klist_slots <= 8)
      dispatch_cm<8>(q, cam, bc, A, stream);
    else if (q.klist_slots <= 16)
      dispatch_cm<16>(q, cam, bc, A, stream);
    else
      dispatch_cm<32>(q, cam, bc, A, stream);
  }
  stage_end(PULSAR_STAGE_RASTER_FWD, stream);
  return hipGetLastError();
}

}  // namespace pulsar

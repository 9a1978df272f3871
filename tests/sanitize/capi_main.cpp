// Host sanitizer driver for the C ABI (test infrastructure): libpulsar's
// sources built with AddressSanitizer and UndefinedBehaviorSanitizer on the
// host side, driven through every entry point's host checks (workspace
// planning over small, ragged and maximal sizes, every invalid argument the
// header names, status and stage strings). Without a GPU a valid call ends at
// its first HIP call with PULSAR_ERR_HIP, so no kernel runs; the run checks
// that the host code reads and writes only what it owns and has no undefined
// behaviour (the size arithmetic in particular).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "pulsar.h"

static int g_fail = 0;
#define CHECK(cond, ...)                    \
  do {                                      \
    if (!(cond)) {                          \
      std::fprintf(stderr, "FAIL: " __VA_ARGS__); \
      std::fprintf(stderr, "\n");           \
      g_fail = 1;                           \
    }                                       \
  } while (0)

static pulsar_camera_t camera(int W, int H) {
  pulsar_camera_t c;
  std::memset(&c, 0, sizeof(c));
  c.R[0] = c.R[4] = c.R[8] = 1.0f;
  c.focal = 1.0f;
  c.sensor_width = 2.0f;
  c.znear = 1.0f;
  c.zfar = 10.0f;
  c.width = W;
  c.height = H;
  return c;
}

static pulsar_params_t params(int K = 8, unsigned flags = 0) {
  pulsar_params_t p;
  std::memset(&p, 0, sizeof(p));
  p.gamma = 0.1f;
  p.eps = 1e-5f;
  p.K = K;
  p.flags = flags;
  return p;
}

static void workspace_sizes() {
  const int ns[] = {0, 1, 7, 1000, 1000000, 3000000, std::numeric_limits<int>::max()};
  const int dims[] = {1, 8, 17, 1024, 65535};
  const int Cs[] = {1, 3, 8, 16, 32, 33, 64};
  const int Ks[] = {1, 5, 8, 32};
  const unsigned flagsets[] = {0u, PULSAR_NO_BWD_AUX, PULSAR_REBIN, PULSAR_GRAD_PAPER_NORM,
                               PULSAR_BLEND_TOPK, PULSAR_ORTHO, PULSAR_STORE_HITS,
                               PULSAR_ORTHO | PULSAR_STORE_HITS | PULSAR_GRAD_PAPER_NORM};
  for (int n : ns)
    for (int W : dims)
      for (int H : {1, 9, 1024, 65535})
        for (int C : Cs)
          for (int K : Ks)
            for (unsigned f : flagsets) {
              pulsar_params_t p = params(K, f);
              const size_t s = pulsar_workspace_size(n, W, H, C, &p);
              // small problems always plan; sizes grow with the sphere count
              if (n <= 1000000 && W <= 1024 && H <= 1024)
                CHECK(s > 0, "no plan for n=%d %dx%d C=%d K=%d flags=%#x", n, W, H, C, K, f);
              if (n > 0 && n <= 1000000 && s > 0) {
                const size_t s0 = pulsar_workspace_size(0, W, H, C, &p);
                CHECK(s0 > 0 && s0 <= s, "workspace shrinks with spheres");
              }
            }
  // launch knobs and capacities at their limits
  for (int chunk : {0, 64, 128, 1024})
    for (int rb : {0, 256, 65536})
      for (int mp : {0, 1, 65536, std::numeric_limits<int>::max()})
        for (float stop : {0.0f, 0.01f, 0.5f}) {
          pulsar_params_t p = params();
          p.chunk = chunk;
          p.raster_blocks = rb;
          p.max_pairs = mp;
          p.stop_share = stop;
          (void)pulsar_workspace_size(100000, 512, 512, 3, &p);
          (void)pulsar_workspace_size(std::numeric_limits<int>::max(), 65535, 65535, 64, &p);
        }
  pulsar_params_t p = params();
  p.min_radius_px = PULSAR_MIN_RADIUS_PX_PAPER;
  CHECK(pulsar_workspace_size(1000, 64, 64, 3, &p) > 0, "minimum size preset rejected");
}

static void invalid_params() {
  struct Bad {
    const char* what;
    void (*set)(pulsar_params_t*);
  };
  const Bad bad[] = {
      {"K 0", [](pulsar_params_t* p) { p->K = 0; }},
      {"K 33", [](pulsar_params_t* p) { p->K = 33; }},
      {"gamma 0", [](pulsar_params_t* p) { p->gamma = 0.0f; }},
      {"gamma 2", [](pulsar_params_t* p) { p->gamma = 2.0f; }},
      {"gamma NaN", [](pulsar_params_t* p) { p->gamma = std::nanf(""); }},
      {"eps -1", [](pulsar_params_t* p) { p->eps = -1.0f; }},
      {"eps inf", [](pulsar_params_t* p) { p->eps = INFINITY; }},
      {"min radius -1", [](pulsar_params_t* p) { p->min_radius_px = -1.0f; }},
      {"reserved flag", [](pulsar_params_t* p) { p->flags = 0x80u; }},
      {"top bit", [](pulsar_params_t* p) { p->flags = 0x80000000u; }},
      {"depth bits", [](pulsar_params_t* p) { p->depth_bits = 1; }},
      {"chunk 65", [](pulsar_params_t* p) { p->chunk = 65; }},
      {"chunk 2048", [](pulsar_params_t* p) { p->chunk = 2048; }},
      {"chunk -64", [](pulsar_params_t* p) { p->chunk = -64; }},
      {"raster blocks 100", [](pulsar_params_t* p) { p->raster_blocks = 100; }},
      {"raster blocks 1e6", [](pulsar_params_t* p) { p->raster_blocks = 1000000; }},
      {"max pairs -1", [](pulsar_params_t* p) { p->max_pairs = -1; }},
      {"stop share 1", [](pulsar_params_t* p) { p->stop_share = 1.0f; }},
      {"stop share -0.1", [](pulsar_params_t* p) { p->stop_share = -0.1f; }},
      {"stop share NaN", [](pulsar_params_t* p) { p->stop_share = std::nanf(""); }},
      {"top-K with stop", [](pulsar_params_t* p) {
         p->flags = PULSAR_BLEND_TOPK;
         p->stop_share = 0.01f;
       }},
  };
  for (const Bad& b : bad) {
    pulsar_params_t p = params();
    b.set(&p);
    CHECK(pulsar_workspace_size(1000, 64, 64, 3, &p) == 0, "workspace planned for %s", b.what);
  }
  pulsar_params_t p = params();
  CHECK(pulsar_workspace_size(-1, 64, 64, 3, &p) == 0, "n < 0 planned");
  CHECK(pulsar_workspace_size(10, 0, 64, 3, &p) == 0, "W = 0 planned");
  CHECK(pulsar_workspace_size(10, 64, 65536, 3, &p) == 0, "H = 65536 planned");
  CHECK(pulsar_workspace_size(10, 64, 64, 0, &p) == 0, "C = 0 planned");
  CHECK(pulsar_workspace_size(10, 64, 64, 3, nullptr) == 0, "NULL params planned");
}

static void calls_without_device() {
  const int n = 100, C = 3, W = 40, H = 24;
  std::vector<float> pos(3 * n, 1.0f), rad(n, 0.1f), opa(n, 0.5f), pay(n * C, 0.5f), bg(C, 0.0f);
  std::vector<float> img(W * H * C), aux(W * H), gimg(W * H * C);
  std::vector<float> gp(3 * n), gr(n), go(n), gf(n * C), gb(C), gcam(14);
  pulsar_camera_t cam = camera(W, H);
  pulsar_params_t p = params(5);
  const size_t ws_bytes = pulsar_workspace_size(n, W, H, C, &p);
  CHECK(ws_bytes > 0, "no plan");
  std::vector<unsigned char> ws(ws_bytes);

  // missing arrays and structs are invalid arguments
  CHECK(pulsar_fwd(nullptr, rad.data(), opa.data(), pay.data(), n, C, bg.data(), &cam, &p,
                   img.data(), aux.data(), ws.data(), ws_bytes, nullptr) ==
            PULSAR_ERR_INVALID_ARGUMENT, "fwd without positions");
  CHECK(pulsar_fwd(pos.data(), rad.data(), opa.data(), pay.data(), n, C, bg.data(), nullptr, &p,
                   img.data(), aux.data(), ws.data(), ws_bytes, nullptr) ==
            PULSAR_ERR_INVALID_ARGUMENT, "fwd without camera");
  CHECK(pulsar_fwd(pos.data(), rad.data(), opa.data(), pay.data(), n, C, bg.data(), &cam,
                   nullptr, img.data(), aux.data(), ws.data(), ws_bytes, nullptr) ==
            PULSAR_ERR_INVALID_ARGUMENT, "fwd without params");
  // a workspace one byte short
  CHECK(pulsar_fwd(pos.data(), rad.data(), opa.data(), pay.data(), n, C, bg.data(), &cam, &p,
                   img.data(), aux.data(), ws.data(), ws_bytes - 1, nullptr) ==
            PULSAR_ERR_WORKSPACE, "short workspace accepted");
  // invalid cameras
  pulsar_camera_t bad = cam;
  bad.zfar = bad.znear;
  CHECK(pulsar_fwd(pos.data(), rad.data(), opa.data(), pay.data(), n, C, bg.data(), &bad, &p,
                   img.data(), aux.data(), ws.data(), ws_bytes, nullptr) ==
            PULSAR_ERR_INVALID_ARGUMENT, "zfar = znear accepted");
  bad = cam;
  bad.R[3] = std::nanf("");
  CHECK(pulsar_fwd(pos.data(), rad.data(), opa.data(), pay.data(), n, C, bg.data(), &bad, &p,
                   img.data(), aux.data(), ws.data(), ws_bytes, nullptr) ==
            PULSAR_ERR_INVALID_ARGUMENT, "NaN rotation accepted");
  // a valid request reaches the device and, with none, fails cleanly
  int rc = pulsar_fwd(pos.data(), rad.data(), opa.data(), pay.data(), n, C, bg.data(), &cam, &p,
                      img.data(), aux.data(), ws.data(), ws_bytes, nullptr);
  CHECK(rc == PULSAR_ERR_HIP, "fwd without a device returned %d", rc);
  CHECK(pulsar_last_hip_error() != nullptr, "no HIP error text");
  rc = pulsar_bwd(pos.data(), rad.data(), opa.data(), pay.data(), n, C, bg.data(), &cam, &p,
                  img.data(), aux.data(), gimg.data(), gp.data(), gr.data(), go.data(), gf.data(),
                  gb.data(), ws.data(), ws_bytes, nullptr);
  CHECK(rc == PULSAR_ERR_HIP, "bwd without a device returned %d", rc);
  rc = pulsar_bwd_camera(pos.data(), rad.data(), opa.data(), pay.data(), n, C, bg.data(), &cam,
                         &p, img.data(), aux.data(), gimg.data(), gp.data(), gr.data(), go.data(),
                         gf.data(), gb.data(), nullptr, ws.data(), ws_bytes, nullptr);
  CHECK(rc == PULSAR_ERR_INVALID_ARGUMENT, "camera backward without its output returned %d", rc);
  // a backward after a forward without backward state needs PULSAR_REBIN
  pulsar_params_t noaux = params(5, PULSAR_NO_BWD_AUX);
  rc = pulsar_bwd(pos.data(), rad.data(), opa.data(), pay.data(), n, C, bg.data(), &cam, &noaux,
                  img.data(), aux.data(), gimg.data(), gp.data(), gr.data(), go.data(), gf.data(),
                  gb.data(), ws.data(), ws_bytes, nullptr);
  CHECK(rc == PULSAR_ERR_INVALID_ARGUMENT || rc == PULSAR_ERR_UNSUPPORTED,
        "backward of a forward without state returned %d", rc);

  // the no-allocation forward rejects work beyond its scratch array on the host
  pulsar_camera_t big = camera(4096, 4096);
  rc = pulsar_fwd_noalloc(pos.data(), rad.data(), opa.data(), pay.data(), 2000000, 8, bg.data(),
                          &big, &p, img.data(), aux.data(), nullptr);
  CHECK(rc == PULSAR_ERR_SCRATCH, "oversized no-allocation forward returned %d", rc);
  rc = pulsar_fwd_noalloc(pos.data(), rad.data(), opa.data(), pay.data(), n, C, bg.data(),
                          nullptr, &p, img.data(), aux.data(), nullptr);
  CHECK(rc == PULSAR_ERR_INVALID_ARGUMENT, "no-allocation forward without camera returned %d",
        rc);

  // status block queries
  int64_t pairs = 0;
  CHECK(pulsar_query_status(nullptr, 0, nullptr, &pairs) == PULSAR_ERR_INVALID_ARGUMENT,
        "status of no workspace");
  CHECK(pulsar_query_status(ws.data(), PULSAR_STATUS_BYTES - 1, nullptr, &pairs) != PULSAR_OK,
        "status of a too small workspace");
}

static void batches() {
  pulsar_params_t p = params(5);
  std::vector<pulsar_scene_t> sc(3);
  const int sizes[3][3] = {{10, 16, 16}, {0, 33, 7}, {500, 64, 48}};
  for (int b = 0; b < 3; ++b) {
    sc[b].camera = camera(sizes[b][1], sizes[b][2]);
    sc[b].n = sizes[b][0];
    sc[b].reserved = 0;
  }
  CHECK(pulsar_batch_workspace_size(sc.data(), 3, 3, &p) > 0, "batch not planned");
  CHECK(pulsar_batch_workspace_size(sc.data(), 1, 3, &p) ==
            pulsar_workspace_size(10, 16, 16, 3, &p),
        "a batch of one differs from the single-scene plan");
  CHECK(pulsar_batch_workspace_size(sc.data(), 0, 3, &p) == 0, "empty batch planned");
  CHECK(pulsar_batch_workspace_size(nullptr, 3, 3, &p) == 0, "NULL scenes planned");
  std::vector<pulsar_scene_t> many(PULSAR_MAX_SCENES + 1, sc[0]);
  CHECK(pulsar_batch_workspace_size(many.data(), PULSAR_MAX_SCENES, 3, &p) > 0,
        "largest batch not planned");
  CHECK(pulsar_batch_workspace_size(many.data(), PULSAR_MAX_SCENES + 1, 3, &p) == 0,
        "batch above the scene limit planned");
  sc[1].reserved = 1;
  CHECK(pulsar_batch_workspace_size(sc.data(), 3, 3, &p) == 0, "reserved field accepted");
  sc[1].reserved = 0;
  sc[2].n = -5;
  CHECK(pulsar_batch_workspace_size(sc.data(), 3, 3, &p) == 0, "negative sphere count accepted");
  sc[2].n = 500;
  sc[2].camera.focal = 0.0f;
  CHECK(pulsar_batch_workspace_size(sc.data(), 3, 3, &p) == 0, "focal 0 accepted");
  sc[2].camera.focal = 1.0f;

  const int n = 510, C = 3;
  const size_t P = 16 * 16 + 33 * 7 + 64 * 48;
  std::vector<float> pos(3 * n, 1.0f), rad(n, 0.1f), pay(n * C), bg(3 * C), img(P * C), aux(P);
  const size_t ws_bytes = pulsar_batch_workspace_size(sc.data(), 3, C, &p);
  std::vector<unsigned char> ws(ws_bytes);
  int rc = pulsar_fwd_batched_devcam(sc.data(), 3, nullptr, pos.data(), rad.data(), nullptr,
                                     pay.data(), C, bg.data(), &p, img.data(), aux.data(),
                                     ws.data(), ws_bytes, nullptr);
  CHECK(rc == PULSAR_ERR_INVALID_ARGUMENT, "device-camera batch without cameras returned %d", rc);
  rc = pulsar_fwd_batched(sc.data(), 3, pos.data(), rad.data(), nullptr, pay.data(), C, bg.data(),
                          &p, img.data(), aux.data(), ws.data(), ws_bytes / 2, nullptr);
  CHECK(rc == PULSAR_ERR_WORKSPACE, "short batch workspace returned %d", rc);
  rc = pulsar_fwd_batched(sc.data(), 3, pos.data(), rad.data(), nullptr, pay.data(), C, bg.data(),
                          &p, img.data(), aux.data(), ws.data(), ws_bytes, nullptr);
  CHECK(rc == PULSAR_ERR_HIP, "batch without a device returned %d", rc);
}

static void strings() {
  for (int code = -10; code <= 5; ++code) {
    const char* s = pulsar_status_string(code);
    CHECK(s != nullptr && std::strlen(s) > 0, "no text for status %d", code);
  }
  for (int st = -2; st <= PULSAR_NUM_STAGES + 1; ++st) {
    const char* s = pulsar_stage_name(st);
    CHECK(s != nullptr, "no name for stage %d", st);
  }
  CHECK(pulsar_version() > 0, "version");
  double ms[PULSAR_NUM_STAGES];
  int64_t counts[PULSAR_NUM_STAGES];
  (void)pulsar_timing_enable(1);
  (void)pulsar_timing_read(ms, counts);
  (void)pulsar_timing_enable(0);
}

int main() {
  workspace_sizes();
  invalid_params();
  calls_without_device();
  batches();
  strings();
  if (g_fail) return 1;
  std::printf("C ABI sanitizer run: ok\n");
  return 0;
}

/*
 * Host sanitizer driver for the FP64 oracle (test infrastructure): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer, it runs the oracle's entry
 * points over small scenes in every mode (pinhole, rotated, orthographic,
 * minimum size, no opacity, top-K blend, early stop, row subsets, empty
 * scenes) and its argument checks, so that an out-of-bounds access, a leak or
 * undefined behaviour in the oracle ends the run with an error.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_forward(int n, int C, const double* pos, const double* radius, const double* opacity,
                   const double* payload, const double* bg, const double* cam16, int W, int H,
                   double gamma, double eps, double min_radius_px, int K, double amb_rel,
                   int n_rows, const int* rows, double* F, double* L, int* nhits,
                   double* klist_t, int* klist_id, double* t_next, uint8_t* ambiguous,
                   int n_threads, int blend_topk, double stop_share);
int oracle_backward(int n, int C, const double* pos, const double* radius, const double* opacity,
                    const double* payload, const double* bg, const double* cam16, int W, int H,
                    double gamma, double eps, double min_radius_px, int K, int n_rows,
                    const int* rows, const double* G, const double* F, const double* L,
                    const int* klist_id, double* grad_pos, double* grad_radius,
                    double* grad_opacity, double* grad_payload, double* grad_bg,
                    double* grad_cam, double* grad_cam_abs, double* grad_cam_sphere);
int oracle_pixel_hits(int n, const double* pos, const double* radius, const double* opacity,
                      const double* cam16, int W, int H, double min_radius_px, int i, int j,
                      uint8_t* hit, double* t_out, double* q_out, double* b_out, double* c_out,
                      double* reff_out, double* u_out);

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
/* uniform in [0, 1): splitmix64 */
static double uni(void) {
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int g_fail = 0;
#define CHECK(cond, ...)                    \
  do {                                      \
    if (!(cond)) {                          \
      fprintf(stderr, "FAIL: " __VA_ARGS__); \
      fprintf(stderr, "\n");                \
      g_fail = 1;                           \
    }                                       \
  } while (0)

typedef struct {
  const char* name;
  int n, C, W, H, K;
  int rotate, ortho, no_opacity, topk, rows;
  double min_radius_px, stop_share;
} case_t;

static void camera(double* cam, int rotate, int ortho) {
  memset(cam, 0, 17 * sizeof(double));
  double a = rotate ? 0.2 : 0.0, b = rotate ? -0.15 : 0.0;
  /* R = Rx(a) Ry(b) */
  double ca = cos(a), sa = sin(a), cb = cos(b), sb = sin(b);
  double R[9] = {cb, 0, sb, sa * sb, ca, -sa * cb, -ca * sb, sa, ca * cb};
  memcpy(cam, R, sizeof(R));
  cam[9] = rotate ? 0.05 : 0.0;
  cam[10] = rotate ? -0.03 : 0.0;
  cam[11] = 0.0;
  cam[12] = 1.0;  /* f */
  cam[13] = ortho ? 2.5 : 2.0;  /* s */
  cam[14] = 1.0;  /* near */
  cam[15] = 10.0; /* far */
  cam[16] = ortho ? 1.0 : 0.0;
}

static void run_case(const case_t* c) {
  const int n = c->n, C = c->C, W = c->W, H = c->H, K = c->K;
  const size_t P = (size_t)W * H;
  const size_t n1 = n > 0 ? (size_t)n : 1;
  double* pos = calloc(3 * n1, sizeof(double));
  double* rad = calloc(n1, sizeof(double));
  double* opa = calloc(n1, sizeof(double));
  double* pay = calloc(n1 * C, sizeof(double));
  double* bg = calloc((size_t)C, sizeof(double));
  for (int k = 0; k < n; ++k) {
    pos[3 * k] = 2.0 * uni() - 1.0;
    pos[3 * k + 1] = 2.0 * uni() - 1.0;
    pos[3 * k + 2] = 3.0 + 3.0 * uni();
    rad[k] = 0.02 + 0.25 * uni();
    opa[k] = 0.2 + 0.8 * uni();
    for (int ch = 0; ch < C; ++ch) pay[(size_t)k * C + ch] = uni();
  }
  for (int ch = 0; ch < C; ++ch) bg[ch] = 0.1 * ch;
  double cam[17];
  camera(cam, c->rotate, c->ortho);
  const double* op = c->no_opacity ? NULL : opa;

  int rows[3] = {0, H / 2, H - 1};
  const int nr = c->rows ? 3 : 0;
  const int* rp = c->rows ? rows : NULL;
  double* F = malloc(P * C * sizeof(double));
  double* L = malloc(P * sizeof(double));
  int* nh = malloc(P * sizeof(int));
  double* kt = malloc(P * K * sizeof(double));
  int* kid = malloc(P * K * sizeof(int));
  double* tn = malloc(P * sizeof(double));
  uint8_t* amb = malloc(P);
  for (size_t i = 0; i < P * C; ++i) F[i] = NAN;
  for (size_t i = 0; i < P; ++i) L[i] = NAN;
  for (size_t i = 0; i < P * K; ++i) kid[i] = -1;
  int rc = oracle_forward(n, C, pos, rad, op, pay, bg, cam, W, H, 0.1, 1e-5, c->min_radius_px, K,
                          1e-5, nr, rp, F, L, nh, kt, kid, tn, amb, 2, c->topk, c->stop_share);
  CHECK(rc == 0, "%s: forward rc %d", c->name, rc);
  const int nrows = c->rows ? 3 : H;
  for (int ri = 0; ri < nrows && rc == 0; ++ri) {
    const int i = c->rows ? rows[ri] : ri;
    for (int j = 0; j < W; ++j) {
      const size_t p = (size_t)i * W + j;
      CHECK(isfinite(L[p]), "%s: L not finite at (%d, %d)", c->name, i, j);
      for (int ch = 0; ch < C; ++ch)
        CHECK(isfinite(F[p * C + ch]), "%s: F not finite at (%d, %d)", c->name, i, j);
      for (int q = 0; q < K; ++q)
        CHECK(kid[p * K + q] >= -1 && kid[p * K + q] < n, "%s: bad K-list id", c->name);
    }
  }

  double* G = malloc(P * C * sizeof(double));
  for (size_t i = 0; i < P * C; ++i) G[i] = uni() - 0.5;
  double* gp = malloc(3 * n1 * sizeof(double));
  double* gr = malloc(n1 * sizeof(double));
  double* go = malloc(n1 * sizeof(double));
  double* gf = malloc(n1 * C * sizeof(double));
  double* gb = malloc((size_t)C * sizeof(double));
  double gcam[14], gabs[14];
  double* gsph = malloc(n1 * 14 * sizeof(double));
  if (!c->stop_share && !c->topk) {
    rc = oracle_backward(n, C, pos, rad, op, pay, bg, cam, W, H, 0.1, 1e-5, c->min_radius_px, K,
                         nr, rp, G, F, L, kid, gp, gr, c->no_opacity ? NULL : go, gf, gb, gcam,
                         gabs, gsph);
    CHECK(rc == 0, "%s: backward rc %d", c->name, rc);
    for (size_t k = 0; k < (size_t)n * 3 && rc == 0; ++k)
      CHECK(isfinite(gp[k]), "%s: grad_pos not finite", c->name);
    for (int v = 0; v < 14 && rc == 0; ++v)
      CHECK(isfinite(gcam[v]) && gabs[v] >= 0.0, "%s: camera gradient", c->name);
  }

  uint8_t* hit = malloc(n1);
  double* t = malloc(n1 * sizeof(double));
  double* q = malloc(n1 * sizeof(double));
  double* b = malloc(n1 * sizeof(double));
  double* cc = malloc(3 * n1 * sizeof(double));
  double* reff = malloc(n1 * sizeof(double));
  double u[3];
  rc = oracle_pixel_hits(n, pos, rad, op, cam, W, H, c->min_radius_px, H / 2, W / 2, hit, t, q, b,
                         cc, reff, u);
  CHECK(rc == 0, "%s: pixel_hits rc %d", c->name, rc);
  rc = oracle_pixel_hits(n, pos, rad, op, cam, W, H, c->min_radius_px, H, 0, hit, t, q, b, cc,
                         reff, u);
  CHECK(rc != 0, "%s: pixel_hits accepted a row outside the image", c->name);

  free(pos); free(rad); free(opa); free(pay); free(bg);
  free(F); free(L); free(nh); free(kt); free(kid); free(tn); free(amb);
  free(G); free(gp); free(gr); free(go); free(gf); free(gb); free(gsph);
  free(hit); free(t); free(q); free(b); free(cc); free(reff);
}

static void argument_checks(void) {
  double cam[17];
  camera(cam, 0, 0);
  double pos[3] = {0, 0, 4}, rad[1] = {0.5}, opa[1] = {-0.5}, pay[1] = {1}, bg[1] = {0};
  double F[4], L[4], kt[4], tn[4];
  int nh[4], kid[4];
  uint8_t amb[4];
  CHECK(oracle_forward(1, 1, pos, rad, opa, pay, bg, cam, 2, 2, 0.1, 1e-5, 0, 1, 1e-5, 0, NULL,
                       F, L, nh, kt, kid, tn, amb, 1, 0, 0.0) != 0,
        "negative opacity accepted");
  CHECK(oracle_forward(1, 0, pos, rad, NULL, pay, bg, cam, 2, 2, 0.1, 1e-5, 0, 1, 1e-5, 0, NULL,
                       F, L, nh, kt, kid, tn, amb, 1, 0, 0.0) != 0,
        "C = 0 accepted");
  CHECK(oracle_forward(1, 1, pos, rad, NULL, pay, bg, cam, 2, 2, 0.1, 1e-5, 0, 1, 1e-5, 0, NULL,
                       F, L, nh, kt, kid, tn, amb, 1, 1, 0.01) != 0,
        "top-K blend with early stop accepted");
  CHECK(oracle_forward(1, 1, pos, rad, NULL, pay, bg, cam, 2, 2, 0.1, 1e-5, 0, 1, 1e-5, 0, NULL,
                       F, L, nh, kt, kid, tn, amb, 1, 0, 1.0) != 0,
        "stop share 1 accepted");
}

int main(void) {
  const case_t cases[] = {
      {"pinhole", 60, 3, 24, 20, 4, 0, 0, 0, 0, 0, 0.0, 0.0},
      {"rotated", 60, 3, 24, 20, 4, 1, 0, 0, 0, 0, 0.0, 0.0},
      {"orthographic", 60, 2, 24, 20, 3, 0, 1, 0, 0, 0, 0.0, 0.0},
      {"minimum size", 60, 3, 17, 13, 5, 0, 0, 0, 0, 0, 0.7071067811865476, 0.0},
      {"ortho minimum size", 60, 3, 17, 13, 5, 1, 1, 0, 0, 0, 0.7071067811865476, 0.0},
      {"no opacity", 60, 1, 16, 16, 2, 0, 0, 1, 0, 0, 0.0, 0.0},
      {"top-K blend", 80, 3, 24, 20, 2, 0, 0, 0, 1, 0, 0.0, 0.0},
      {"early stop", 120, 3, 24, 20, 4, 0, 0, 0, 0, 0, 0.0, 0.01},
      {"early stop rows", 120, 3, 24, 20, 4, 1, 0, 0, 0, 1, 0.0, 0.2},
      {"row subset", 60, 5, 24, 20, 32, 0, 0, 0, 0, 1, 0.0, 0.0},
      {"wide payload", 30, 40, 12, 9, 8, 0, 0, 0, 0, 0, 0.0, 0.0},
      {"empty scene", 0, 3, 8, 8, 4, 0, 0, 0, 0, 0, 0.0, 0.0},
      {"one pixel", 5, 1, 1, 1, 1, 0, 0, 0, 0, 0, 0.0, 0.0},
  };
  for (size_t i = 0; i < sizeof(cases) / sizeof(cases[0]); ++i) run_case(&cases[i]);
  argument_checks();
  if (g_fail) return 1;
  printf("oracle sanitizer run: ok\n");
  return 0;
}

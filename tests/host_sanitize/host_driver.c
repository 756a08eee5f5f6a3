/* Host-side driver of the C-ABI for the AddressSanitizer / UndefinedBehaviorSanitizer
 * build of the library's host code (tests/test_host_sanitize.py).  Host-only plans
 * (device -1): descriptor validation for every status code, the integer tables of odd and
 * overhanging geometries, options, the tuning report and its buffer sizes, and the refusal
 * of compute calls.  Prints "ok" and returns 0 when every call returned what it should. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mpbp.h"

static int failures = 0;
#define EXPECT(cond)                                                     \
  do {                                                                   \
    if (!(cond)) {                                                       \
      fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond, mpbp_last_error()); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

static mpbp_peak peak(double gx, double gy, double gz, double ty, double tx, int det, int ry, int rx, int sy,
                      int sx, int oy, int ox) {
  mpbp_peak p;
  memset(&p, 0, sizeof(p));
  p.g[0] = gx; p.g[1] = gy; p.g[2] = gz;
  p.shear[0] = ty; p.shear[1] = tx;
  p.det = det;
  p.scan_n[0] = ry; p.scan_n[1] = rx;
  p.scan_step[0] = sy; p.scan_step[1] = sx;
  p.scan_origin[0] = oy; p.scan_origin[1] = ox;
  return p;
}

static void check_tables(mpbp_plan plan, int nz, int n_peaks) {
  const int64_t F = mpbp_num_frames(plan);
  int32_t* scan = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)F);
  int32_t* shear = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)nz * n_peaks);
  int64_t* y_off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_peaks + 1));
  EXPECT(mpbp_tables(plan, scan, shear, y_off) == MPBP_OK);
  EXPECT(y_off[0] == 0 && y_off[n_peaks] == mpbp_intensity_size(plan));
  EXPECT(mpbp_tables(plan, NULL, NULL, NULL) == MPBP_OK);
  free(scan);
  free(shear);
  free(y_off);
}

int main(void) {
  /* a valid three-peak problem with overhanging windows, odd sizes and both shear signs */
  mpbp_peak pk[3];
  pk[0] = peak(31.4, 0.0, 31.4, 0.3, -0.45, 64, 5, 7, 6, 5, -7, -3);
  pk[1] = peak(-9.0, 12.0, 4.0, -1.2, 0.5, 96, 3, 4, 11, 9, 20, 14);
  pk[2] = peak(0.0, 0.0, 27.0, 0.0, 0.0, 32, 2, 2, 40, 40, 0, 0);
  mpbp_problem pr = {9, 61, 53, 16, 3, pk, 0};
  mpbp_plan plan = NULL;
  EXPECT(mpbp_plan_create(&pr, -1, &plan) == MPBP_OK && plan);
  EXPECT(mpbp_num_frames(plan) == 5 * 7 + 3 * 4 + 2 * 2);
  check_tables(plan, pr.nz, pr.n_peaks);
  int64_t v = 0, len = 0;
  EXPECT(mpbp_set_option(plan, MPBP_OPT_GRAD_BATCH, 16) == MPBP_OK);
  EXPECT(mpbp_get_option(plan, MPBP_OPT_GRAD_BATCH, &v) == MPBP_OK && v == 16);
  EXPECT(mpbp_set_option(plan, MPBP_OPT_RUNS, 2) == MPBP_ERR_INVALID);
  EXPECT(mpbp_set_option(plan, 12345, 0) == MPBP_ERR_INVALID);
  EXPECT(mpbp_tuning(plan, NULL, 0, &len) == MPBP_OK && len > 2);
  char* buf = (char*)malloc((size_t)len);
  EXPECT(mpbp_tuning(plan, buf, len, &len) == MPBP_OK && buf[len - 1] == 0 && buf[0] == '{');
  char small[5];
  EXPECT(mpbp_tuning(plan, small, sizeof(small), &len) == MPBP_ERR_INVALID);
  free(buf);
  EXPECT(mpbp_set_variant(plan, 99, 48, 4, 1) == MPBP_ERR_INVALID);
  float f = 0.f;
  double d = 0.0;
  EXPECT(mpbp_loss_grad(plan, &f, &f, &f, &f, &f, NULL, 0, &d, NULL, &f, &f, &f, NULL) == MPBP_ERR_DEVICE);
  EXPECT(mpbp_loss_grad_static(plan, &f, &f, &f, &f, &f, NULL, 0, &d, NULL, &f, &f, &f, NULL) == MPBP_ERR_DEVICE);
  EXPECT(mpbp_stage_times(plan, NULL, NULL) == MPBP_ERR_DEVICE || mpbp_stage_times(plan, NULL, NULL) == MPBP_OK);
  mpbp_plan_destroy(plan);

  /* every flag combination on a valid geometry */
  for (uint32_t fl = 0; fl < 8; ++fl) {
    mpbp_problem q = pr;
    q.flags = fl;
    plan = NULL;
    EXPECT(mpbp_plan_create(&q, -1, &plan) == MPBP_OK);
    check_tables(plan, q.nz, q.n_peaks);
    mpbp_plan_destroy(plan);
  }

  /* invalid descriptors: every status of plan creation */
  mpbp_problem bad = pr;
  plan = (mpbp_plan)0x1;
  EXPECT(mpbp_plan_create(NULL, -1, &plan) == MPBP_ERR_INVALID && plan == NULL);
  EXPECT(mpbp_plan_create(&pr, -1, NULL) == MPBP_ERR_INVALID);
  bad.flags = 64;
  EXPECT(mpbp_plan_create(&bad, -1, &plan) == MPBP_ERR_INVALID);
  bad = pr; bad.nz = 0;
  EXPECT(mpbp_plan_create(&bad, -1, &plan) == MPBP_ERR_SHAPE);
  bad = pr; bad.n_peaks = 0;
  EXPECT(mpbp_plan_create(&bad, -1, &plan) == MPBP_ERR_SHAPE);
  bad = pr; bad.peaks = NULL;
  EXPECT(mpbp_plan_create(&bad, -1, &plan) == MPBP_ERR_INVALID);
  bad = pr; bad.probe_n = 33;
  EXPECT(mpbp_plan_create(&bad, -1, &plan) == MPBP_ERR_UNSUPPORTED);
  mpbp_peak pb[3];
  memcpy(pb, pk, sizeof(pk));
  pb[1].det = 100;
  bad = pr; bad.peaks = pb;
  EXPECT(mpbp_plan_create(&bad, -1, &plan) == MPBP_ERR_SHAPE);
  memcpy(pb, pk, sizeof(pk));
  pb[0].shear[1] = 9.0;  /* the sheared support leaves the 64 x 64 window */
  EXPECT(mpbp_plan_create(&bad, -1, &plan) == MPBP_ERR_FOOTPRINT);
  memcpy(pb, pk, sizeof(pk));
  pb[2].g[0] = 0.0 / 0.0;
  EXPECT(mpbp_plan_create(&bad, -1, &plan) == MPBP_ERR_INVALID);
  memcpy(pb, pk, sizeof(pk));
  pb[2].scan_step[1] = 0;
  EXPECT(mpbp_plan_create(&bad, -1, &plan) == MPBP_ERR_SHAPE);
  EXPECT(mpbp_plan_create(&pr, -7, &plan) == MPBP_ERR_INVALID);
  EXPECT(mpbp_num_frames(NULL) == -1 && mpbp_intensity_size(NULL) == -1);
  EXPECT(mpbp_tables(NULL, NULL, NULL, NULL) == MPBP_ERR_INVALID);
  mpbp_plan_destroy(NULL);
  EXPECT(strlen(mpbp_last_error()) > 0);
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("ok\n");
  return 0;
}

/* Host-side paths of the C ABI that run without a GPU, for a build of the
 * library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitize_cpu.py): argument validation, context creation over
 * every supported (l_max, k, axes) and the rejected ones (the SH matrices of
 * Sec. 2 / App. B are built on the host at creation), mesh validation and
 * point queries, and the host spherical harmonics of App. A against the
 * addition theorem sum_m Y_lm(d)^2 = (2l+1)/(4 pi).  Prints one line per
 * failure and exits non-zero if any. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "vfp.h"

static int fails = 0;
#define CHECK(cond, ...)               \
  do {                                 \
    if (!(cond)) {                     \
      printf("FAIL: " __VA_ARGS__);    \
      printf("\n");                    \
      ++fails;                         \
    }                                  \
  } while (0)

int main(void) {
  const double pi = 3.14159265358979323846;
  /* harmonics: addition theorem for l <= 11 at scattered directions */
  enum { LM = 11, ND = 17 };
  double th[ND], ph[ND];
  for (int d = 0; d < ND; ++d) {
    th[d] = pi * (d + 0.37) / ND;
    ph[d] = 2.0 * pi * (0.61 * d + 0.13);
  }
  const int n = (LM + 1) * (LM + 1);
  double* Y = (double*)malloc(sizeof(double) * n * ND);
  CHECK(vfp_sh_eval(LM, ND, th, ph, Y) == VFP_OK, "vfp_sh_eval: %s", vfp_last_error());
  for (int d = 0; d < ND; ++d)
    for (int l = 0; l <= LM; ++l) {
      double s = 0.0;
      for (int m = l * l; m < (l + 1) * (l + 1); ++m) s += Y[d * n + m] * Y[d * n + m];
      CHECK(fabs(s - (2 * l + 1) / (4 * pi)) < 1e-12, "addition theorem l=%d d=%d: %.17g", l, d, s);
    }
  CHECK(vfp_sh_eval(LM + 1, ND, th, ph, Y) != VFP_OK, "l_max 12 accepted");
  CHECK(vfp_sh_eval(LM, ND, NULL, ph, Y) != VFP_OK, "null theta accepted");
  free(Y);

  /* contexts over the supported and rejected shapes */
  const int axes_sets[6][3] = {{VFP_AXIS_X, 0, 0}, {VFP_AXIS_X, VFP_AXIS_Y, 0}, {VFP_AXIS_X, VFP_AXIS_Y, VFP_AXIS_Z},
                               {VFP_AXIS_X, VFP_AXIS_LNP, 0}, {VFP_AXIS_X, VFP_AXIS_P, 0}, {VFP_AXIS_LNP, 0, 0}};
  const int naxes[6] = {1, 2, 3, 2, 2, 1};
  int created = 0;
  for (int a = 0; a < 6; ++a)
    for (int lmax = 0; lmax <= 12; ++lmax)
      for (int k = 0; k <= 6; ++k) {
        vfp_ctx* c = NULL;
        const int rc = vfp_create(&c, lmax, k, naxes[a], axes_sets[a], 31u, 1.0, 1.0);
        if (rc == VFP_OK) {
          ++created;
          int64_t nd = -1;
          CHECK(vfp_ndofs(c, &nd) == VFP_ESTATE, "ndofs before the mesh");
          vfp_destroy(c);
        } else {
          CHECK(c == NULL, "a failed create returned a context");
          CHECK(vfp_last_error()[0] != 0, "no message for rc %d", rc);
        }
      }
  CHECK(created > 50, "only %d contexts created", created);

  /* mesh validation and the query of the points (no device needed) */
  {
    vfp_ctx* c = NULL;
    const int ax[1] = {VFP_AXIS_X};
    CHECK(vfp_create(&c, 3, 2, 1, ax, 31u, 1.0, 1.0) == VFP_OK, "create");
    const double bad[4] = {0.0, 1.0, 0.5, 2.0};
    const double good[4] = {0.0, 1.0, 2.5, 3.0};
    const double* nb[1] = {bad};
    const double* ng[1] = {good};
    const int nc[1] = {3}, per[1] = {VFP_BC_PERIODIC}, zin[1] = {VFP_BC_ZERO_INFLOW};
    CHECK(vfp_set_mesh(c, nc, nb, per, per) == VFP_EINVAL, "decreasing nodes accepted");
    CHECK(vfp_set_mesh(c, nc, ng, per, zin) == VFP_EINVAL, "periodic on one end accepted");
    const int rc = vfp_set_mesh(c, nc, ng, zin, zin);
    CHECK(rc == VFP_OK || rc == VFP_EDEVICE, "set_mesh rc %d: %s", rc, vfp_last_error());
    int64_t cnt = 0;
    CHECK(vfp_query_points(c, 0, 0, NULL, &cnt) == VFP_OK && cnt == 9, "point count %lld", (long long)cnt);
    double pts[9];
    CHECK(vfp_query_points(c, 0, 0, pts, &cnt) == VFP_OK, "query points");
    for (int i = 1; i < 9; ++i) CHECK(pts[i] > pts[i - 1], "Gauss points not increasing at %d", i);
    CHECK(vfp_query_points(c, 0, 1, NULL, &cnt) != VFP_OK, "axis 1 of a 1-axis context accepted");
    vfp_destroy(c);
  }
  vfp_destroy(NULL);
  printf("%s: %d failure(s), %d contexts\n", fails ? "FAILED" : "ok", fails, created);
  return fails ? 1 : 0;
}

/*
 * A plain C99 client of the library's C ABI (include/rsc.h), built with gcc -pedantic
 * -Werror and linked against librsc.so.  It uses only the calls that need no device:
 * the FP64 host constructions of both bases, the workspace size of the image plan and
 * the argument errors, and checks what the paper and the mathematics fix for them:
 *   - the disk of an 11x11 patch has 97 pixels (Sec. III-A), of a 15x15 one 177;
 *   - B = S (2T + 1) for the grid of profiles; the annular basis at N = 11 has
 *     T_s = 1, 3, 8, 11, 15 and B = 81;
 *   - the biorthogonal partner inverts the basis on its span: Phi^+ Phi = I (Sec. II-E).
 * Prints one line per check and exits with the number of failed checks.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rsc.h"

static int failures = 0;

static void check(int ok, const char* what) {
  printf("%s %s\n", ok ? "ok  " : "FAIL", what);
  if (!ok) ++failures;
}

/* max |(pinv phi)_{ij} - delta_ij| for phi [NN, B] and pinv [B, NN], both row-major */
static double partner_error(const double* phi, const double* pinv, int NN, int B) {
  double worst = 0.0;
  int i, j, p;
  for (i = 0; i < B; ++i)
    for (j = 0; j < B; ++j) {
      double acc = 0.0;
      for (p = 0; p < NN; ++p) acc += pinv[(size_t)i * NN + p] * phi[(size_t)p * B + j];
      acc -= (i == j) ? 1.0 : 0.0;
      if (fabs(acc) > worst) worst = fabs(acc);
    }
  return worst;
}

static void grid_basis(int N, int S, int T, int n_pix_expected) {
  int n_pix = 0, B = 0, NN = N * N;
  double cond = 0.0;
  double *phi, *pinv;
  char what[128];
  rsc_status st = rsc_basis_host(N, S, T, NULL, 0.0, NULL, NULL, &n_pix, &B, &cond);
  sprintf(what, "grid basis N=%d S=%d T=%d: status, %d disk pixels, B = S(2T+1)", N, S, T, n_pix_expected);
  check(st == RSC_OK && n_pix == n_pix_expected && B == S * (2 * T + 1) && cond >= 1.0, what);
  phi = (double*)malloc(sizeof(double) * (size_t)NN * (size_t)(B > 0 ? B : 1));
  pinv = (double*)malloc(sizeof(double) * (size_t)NN * (size_t)(B > 0 ? B : 1));
  st = rsc_basis_host(N, S, T, NULL, 0.0, phi, pinv, NULL, NULL, NULL);
  sprintf(what, "grid basis N=%d: Phi^+ Phi = I within 1e-10", N);
  check(st == RSC_OK && partner_error(phi, pinv, NN, B) < 1e-10, what);
  free(phi);
  free(pinv);
}

int main(void) {
  int Ts[8] = {0}, B = 0, k;
  size_t bytes = 0;
  rsc_handle* h = NULL;
  const char* msg;
  static const int ts11[5] = {1, 3, 8, 11, 15};
  double *phi, *pinv;
  rsc_status st;

  grid_basis(11, 5, 5, 97);
  grid_basis(15, 7, 7, 177);

  st = rsc_annular_basis_host(11, 0, NULL, NULL, Ts, &B, NULL);
  {
    int same = 1;
    for (k = 0; k < 5; ++k) same = same && Ts[k] == ts11[k];
    check(st == RSC_OK && B == 81 && same, "annular basis N=11: T_s = 1, 3, 8, 11, 15 and B = 81");
  }
  phi = (double*)malloc(sizeof(double) * 121 * 81);
  pinv = (double*)malloc(sizeof(double) * 121 * 81);
  st = rsc_annular_basis_host(11, 0, phi, pinv, NULL, NULL, NULL);
  check(st == RSC_OK && partner_error(phi, pinv, 121, 81) < 1e-10, "annular basis N=11: Phi^+ Phi = I within 1e-10");
  free(phi);
  free(pinv);

  check(rsc_images_workspace_size(10, &bytes) == RSC_OK && bytes == 2 * sizeof(int64_t) * 11,
        "image plan workspace: two int64 prefix sums of n + 1 entries");
  check(rsc_images_workspace_size(-1, &bytes) == RSC_E_INVALID, "image plan workspace: n < 0 is refused");

  /* argument errors are synchronous and leave a message; nothing aborts or prints */
  st = rsc_create(10, 5, 5, NULL, 0.0, RSC_FP32, &h);
  msg = rsc_last_error(NULL);
  check(st == RSC_E_INVALID && h == NULL && msg != NULL && strlen(msg) > 0, "even N is refused with a message");
  check(rsc_create(11, 5, 5, NULL, 0.0, RSC_FP32, NULL) == RSC_E_INVALID, "null out is refused");
  check(rsc_basis_host(12, 5, 5, NULL, 0.0, NULL, NULL, NULL, NULL, NULL) == RSC_E_INVALID,
        "host basis: even N is refused");
  check(rsc_annular_basis_host(4, 0, NULL, NULL, NULL, NULL, NULL) == RSC_E_INVALID,
        "host annular basis: even N is refused");
  check(rsc_destroy(NULL) == RSC_OK, "destroying NULL is a no-op");
  return failures;
}

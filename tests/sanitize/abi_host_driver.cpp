// Drives the host-side paths of the C-ABI (include/islbm.h) for the
// sanitizer build: every call below runs host code only -- argument and mesh
// validation, parameter derivation, interpolation-table and reduction-
// coefficient construction -- and stops at the device check (no GPU is used;
// with one present, create may succeed and the context is destroyed).
// Exit status 0 when every call returned what the header promises.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/islbm.h"

static int failures = 0;

#define EXPECT(cond)                                                    \
  do {                                                                  \
    if (!(cond)) {                                                      \
      std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, \
                   __LINE__, #cond);                                    \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

static std::vector<double> spacing(int kind, int n, double a) {
  std::vector<double> sp(n + 1);
  EXPECT(islbm_mesh_spacing(kind, n, a, sp.data()) == ISLBM_OK);
  const double d = sp[0];
  for (double& h : sp) h /= d;  // lattice units
  return sp;
}

static int create(int lattice, const int n[3], const double* const sp[3], double Ra, double Pr,
                  const islbm_options* o) {
  islbm_ctx* c = reinterpret_cast<islbm_ctx*>(0x1);
  const int rc = islbm_create(&c, lattice, n, sp, Ra, Pr, o);
  if (rc == ISLBM_OK) islbm_destroy(c);
  else EXPECT(c == nullptr && islbm_last_error(nullptr)[0] != '\0');
  return rc;
}

int main() {
  // status texts, including out-of-range codes
  for (int code = 1; code >= -8; --code) EXPECT(islbm_strerror(code) != nullptr);
  islbm_options o;
  islbm_default_options(&o);
  islbm_default_options(nullptr);
  EXPECT(o.T_hot == 0.5 && o.T_cold == -0.5 && o.storage == ISLBM_FP32);

  // buffer sizes
  size_t fb = 0, gb = 0;
  const int n2[3] = {70, 36, 1}, n3[3] = {40, 22, 18}, bad[3] = {2, 5, 5};
  EXPECT(islbm_query_bytes(2, n2, ISLBM_FP32, &fb, &gb) == ISLBM_OK && fb > 0 && gb > 0);
  for (int st = 0; st <= 4; ++st) EXPECT(islbm_query_bytes(3, n3, st, &fb, &gb) == ISLBM_OK);
  EXPECT(islbm_query_bytes(3, n3, 5, &fb, &gb) == ISLBM_EINVAL);
  EXPECT(islbm_query_bytes(4, n3, 0, &fb, &gb) == ISLBM_EINVAL);
  EXPECT(islbm_query_bytes(2, bad, 0, &fb, &gb) == ISLBM_EINVAL);
  EXPECT(islbm_query_bytes(2, nullptr, 0, &fb, &gb) == ISLBM_EINVAL);

  // mesh generators: positive spacings, mirror-symmetric about the centre,
  // summing to x_{N+1} - x_0 ((N+1)/N for the uniform mesh, 1 for the others)
  for (int kind = 0; kind <= 3; ++kind)
    for (int n : {3, 4, 64, 257, 1024}) {
      std::vector<double> sp(n + 1);
      EXPECT(islbm_mesh_spacing(kind, n, 1.5, sp.data()) == ISLBM_OK);
      double sum = 0.0;
      for (int m = 0; m <= n; ++m) {
        sum += sp[m];
        EXPECT(sp[m] > 0.0 && std::fabs(sp[m] - sp[n - m]) <= 1e-9 * sp[m]);  // differences of values near 1
      }
      EXPECT(std::fabs(sum - (kind == 0 ? double(n + 1) / n : 1.0)) < 1e-12);
    }
  std::vector<double> tmp(10);
  EXPECT(islbm_mesh_spacing(5, 9, 1.5, tmp.data()) == ISLBM_EINVAL);
  EXPECT(islbm_mesh_spacing(1, 9, 0.0, tmp.data()) == ISLBM_EINVAL);
  EXPECT(islbm_mesh_spacing(0, 2, 0.0, tmp.data()) == ISLBM_EINVAL);
  EXPECT(islbm_mesh_spacing(0, 9, 0.0, nullptr) == ISLBM_EINVAL);

  // create: argument errors before any device work
  auto sx = spacing(3, 70, 1.5), sy = spacing(3, 36, 1.5), sz = spacing(3, 18, 1.5);
  const double* sp2[3] = {sx.data(), sy.data(), nullptr};
  EXPECT(islbm_create(nullptr, 2, n2, sp2, 1e6, 0.71, nullptr) == ISLBM_EINVAL);
  EXPECT(create(2, nullptr, sp2, 1e6, 0.71, nullptr) == ISLBM_EINVAL);
  EXPECT(create(7, n2, sp2, 1e6, 0.71, nullptr) == ISLBM_EINVAL);
  EXPECT(create(2, n2, sp2, -1.0, 0.71, nullptr) == ISLBM_EINVAL);
  EXPECT(create(2, n2, sp2, 1e6, NAN, nullptr) == ISLBM_EINVAL);
  EXPECT(create(2, bad, sp2, 1e6, 0.71, nullptr) == ISLBM_EINVAL);
  islbm_options ob = o;
  ob.storage = 9;
  EXPECT(create(2, n2, sp2, 1e6, 0.71, &ob) == ISLBM_EINVAL);
  // mesh errors: a spacing below the lattice unit, a non-finite one, unequal ghosts
  auto shrunk = sx;
  shrunk[10] = 0.5;
  const double* sp_bad1[3] = {shrunk.data(), sy.data(), nullptr};
  EXPECT(create(2, n2, sp_bad1, 1e6, 0.71, nullptr) == ISLBM_EMESH);
  auto nanm = sx;
  nanm[5] = NAN;
  const double* sp_bad2[3] = {nanm.data(), sy.data(), nullptr};
  EXPECT(create(2, n2, sp_bad2, 1e6, 0.71, nullptr) == ISLBM_EMESH);
  auto ghost = sx;
  ghost[70] = 1.5;
  const double* sp_bad3[3] = {ghost.data(), sy.data(), nullptr};
  EXPECT(create(2, n2, sp_bad3, 1e6, 0.71, nullptr) == ISLBM_EMESH);
  // stability check: u_f = 0.1 at Ra = 1e3 gives a_T far above 1
  islbm_options fast = o;
  fast.u_f = 0.1;
  EXPECT(create(2, n2, sp2, 1e3, 0.71, &fast) == ISLBM_EPARAM);

  // valid meshes run the whole host set-up (tables, reduction coefficients)
  // and stop at the device check
  for (int st = 0; st <= 4; ++st) {
    islbm_options v = o;
    v.storage = st;
    const int rc2 = create(2, n2, sp2, 1e6, 0.71, &v);
    EXPECT(rc2 == ISLBM_OK || rc2 == ISLBM_EDEVICE);
    const double* sp3[3] = {sx.data(), sy.data(), sz.data()};
    const int n3b[3] = {70, 36, 18};
    const int rc3 = create(3, n3b, sp3, 1e7, 0.71, &v);
    EXPECT(rc3 == ISLBM_OK || rc3 == ISLBM_EDEVICE);
  }
  // smallest mesh (3 nodes per axis) and a uniform mesh (one-hot weights)
  auto s3 = spacing(0, 3, 0.0);
  const double* spm[3] = {s3.data(), s3.data(), s3.data()};
  const int nm[3] = {3, 3, 3};
  const int rcm = create(3, nm, spm, 1e4, 0.71, nullptr);
  EXPECT(rcm == ISLBM_OK || rcm == ISLBM_EDEVICE || rcm == ISLBM_EPARAM);

  // NULL context handling
  islbm_destroy(nullptr);
  EXPECT(islbm_step(nullptr, 1) == ISLBM_EINVAL);
  EXPECT(islbm_nu_re(nullptr, nullptr) == ISLBM_EINVAL);
  EXPECT(islbm_time(nullptr) == -1);
  std::printf("abi host driver: %d failure(s)\n", failures);
  return failures == 0 ? 0 : 1;
}

/* Host-only exercise of libstglbm's C ABI (no device needed): descriptor
 * validation, footprint (and with it the launch-shape, statistics-slot and
 * z-chunk rules over a grid of lattices), unit derivation, status strings and
 * the error paths that return before any HIP call.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code by tests/test_host_sanitizers.py;
 * prints "ok" and exits 0 when every expectation holds. */
#include <stdio.h>
#include <string.h>

#include "stglbm.h"

static int failures = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static stglbm_lattice_desc channel(int nx, int ny, int nz) {
  stglbm_lattice_desc d;
  memset(&d, 0, sizeof d);
  d.nx = nx; d.ny = ny; d.nz = nz;
  d.store = STGLBM_F32;
  d.sponge_cells = 6;
  d.max_modes = 50;
  d.max_rans = 32;
  d.nu_lb = 2.8645e-4;
  d.cs_smag = 0.1;
  d.rho_out = 1.0;
  d.sponge_K = 1000.0;
  d.sponge_p = 3.0;
  return d;
}

int main(void) {
  EXPECT(stglbm_version() > 0);
  for (int code = 0; code >= -6; --code) EXPECT(strlen(stglbm_status_string(code)) > 0);
  EXPECT(strlen(stglbm_status_string(12345)) > 0);

  uint64_t bytes = 0;
  stglbm_lattice_desc d = channel(64, 32, 32);
  EXPECT(stglbm_footprint(&d, &bytes) == STGLBM_OK);
  EXPECT(bytes >= 2ull * 19 * 64 * 32 * 32 * 4);
  for (int q = 15; q <= 27; q += 4) {
    stglbm_lattice_desc v = d;
    v.velocity_set = q == 23 ? 27 : q;
    v.collision = 1;
    uint64_t b = 0;
    EXPECT(stglbm_footprint(&v, &b) == STGLBM_OK);
  }
  /* the launch-shape rules (block shape, statistics slots, unequal z chunks of
   * the 16-bit stores) over a grid of lattices: ragged and narrow rows, few
   * and many rows and z slices, every store and velocity set, both boundary
   * kinds; the footprint always holds the two distribution buffers */
  {
    static const int nxs[] = {2, 48, 64, 100, 448, 512, 520, 1024, 1030};
    static const int nys[] = {2, 3, 7, 64, 128, 256, 300};
    static const int nzs[] = {1, 2, 3, 7, 33, 64, 96, 256, 512, 1000};
    static const int qs[] = {15, 19, 27};
    for (unsigned a = 0; a < sizeof nxs / sizeof nxs[0]; ++a)
      for (unsigned b = 0; b < sizeof nys / sizeof nys[0]; ++b)
        for (unsigned c = 0; c < sizeof nzs / sizeof nzs[0]; ++c)
          for (int store = 0; store <= 2; ++store)
            for (unsigned k = 0; k < 3; ++k)
              for (int per = 0; per <= 1; ++per) {
                stglbm_lattice_desc v = channel(nxs[a], nys[b], nzs[c]);
                v.store = store;
                v.velocity_set = qs[k];
                v.periodic_x = per;
                if (per || nxs[a] < 12) v.sponge_cells = 0;
                uint64_t fb = 0;
                const uint64_t cells = (uint64_t)nxs[a] * nys[b] * nzs[c];
                EXPECT(stglbm_footprint(&v, &fb) == STGLBM_OK);
                EXPECT(fb >= 2ull * qs[k] * cells * (store == STGLBM_F32 ? 4 : 2));
              }
  }
  /* invalid descriptors: each fails on the host with a message */
  stglbm_lattice_desc bad[8];
  for (int i = 0; i < 8; ++i) bad[i] = d;
  bad[0].nx = 1;
  bad[1].nu_lb = -1.0;
  bad[2].store = 7;
  bad[3].velocity_set = 21;
  bad[4].collision = 3;
  bad[5].max_modes = 0;
  bad[6].nx = 65536; bad[6].ny = 65536; bad[6].nz = 1024;     /* 2^42 cells */
  bad[7].rho_out = 0.0;
  for (int i = 0; i < 8; ++i) {
    uint64_t b = 0;
    EXPECT(stglbm_footprint(&bad[i], &b) == STGLBM_E_INVAL);
    EXPECT(strlen(stglbm_last_error(NULL)) > 0);
  }
  EXPECT(stglbm_footprint(NULL, &bytes) == STGLBM_E_INVAL);

  double c_x = 0, c_t = 0, nu = 0;
  EXPECT(stglbm_derive_units(1.0, 128, 0.05, 15.37, 1.0 / 180.0, &c_x, &c_t, &nu) == STGLBM_OK);
  EXPECT(c_x > 0 && c_t > 0 && nu > 0);
  EXPECT(stglbm_derive_units(1.0, 0, 0.05, 15.37, 1.0 / 180.0, &c_x, &c_t, &nu) == STGLBM_E_INVAL);

  /* the paper's worked example: c_x = 1/90 m, c_t = 1.852e-5 s, 1 m/s^2 -> F = 3.086e-8 */
  const double acc[3] = {1.0, 0.0, -2.0};
  double force[3] = {0, 0, 0};
  EXPECT(stglbm_acceleration_to_lattice(1.0 / 90.0, 1.852e-5, acc, force) == STGLBM_OK);
  EXPECT(force[0] > 3.085e-8 && force[0] < 3.087e-8 && force[1] == 0.0 && force[2] == -2.0 * force[0]);
  EXPECT(stglbm_acceleration_to_lattice(0.0, 1.0, acc, force) == STGLBM_E_INVAL);
  EXPECT(stglbm_acceleration_to_lattice(1.0, 1.0, NULL, force) == STGLBM_E_INVAL);
  EXPECT(stglbm_step_noalloc(NULL, 1) == STGLBM_E_INVAL);
  EXPECT(stglbm_set_equilibrium_physical(NULL, NULL, 0, 1.0, 1.0) == STGLBM_E_INVAL);

  /* init without a workspace, and calls on a null handle, fail before touching a device */
  stglbm_t h = (stglbm_t)0x1;
  EXPECT(stglbm_init_lattice(&d, NULL, 0, NULL, &h) == STGLBM_E_INVAL);
  EXPECT(h == NULL);
  EXPECT(stglbm_init_lattice(&d, NULL, 0, NULL, NULL) == STGLBM_E_INVAL);
  EXPECT(stglbm_step(NULL, 1) == STGLBM_E_INVAL);
  EXPECT(stglbm_checkpoint_size(NULL, &bytes) == STGLBM_E_INVAL);
  EXPECT(stglbm_destroy(NULL) == STGLBM_OK);

  if (failures) return 1;
  printf("ok\n");
  return 0;
}

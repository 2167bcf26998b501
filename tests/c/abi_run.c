/* A plain C program that runs the extended LBGK step on the GPU through the
 * elbm ABI alone (no Python, no torch): it allocates the lattice's device
 * buffer with the HIP runtime's C API, initialises a seeded-free field whose
 * values are exact in binary (so any other client can rebuild it bit for
 * bit), steps, and prints the FP64 diagnostics record and the kernel choice.
 * __graft_entry__.build() compiles it next to the library; the GPU test
 * tests/test_gpu_c_client.py compares its output with the Python binding's
 * run of the same problem.
 *
 * Usage: abi_run STORAGE COLLISION   (STORAGE 0 FP32, 1 FP16, 2 BF16;
 *                                     COLLISION 0 LBGK, 1 MRT) */
#define __HIP_PLATFORM_AMD__ 1
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "elbm.h"

#define NX 64
#define NY 32
#define NZ 16

static int check(int32_t s, const char* what) {
  if (s != ELBM_OK) {
    fprintf(stderr, "%s: %s (%s)\n", what, elbm_status_string(s), elbm_last_error());
    return 1;
  }
  return 0;
}

int main(int argc, char** argv) {
  elbm_params p;
  size_t bytes = 0, n = (size_t)NX * NY * NZ, cell;
  void* buf = NULL;
  elbm_handle h = NULL;
  elbm_diag_record d;
  elbm_kernel_info k;
  double *rho, *u;
  int x, y, z, storage, mrt;

  if (argc != 3) {
    fprintf(stderr, "usage: %s STORAGE COLLISION\n", argv[0]);
    return 2;
  }
  storage = atoi(argv[1]);
  mrt = atoi(argv[2]);

  memset(&p, 0, sizeof p);
  p.abi_version = ELBM_ABI_VERSION;
  p.lattice = 27;
  p.n[0] = NX;
  p.n[1] = NY;
  p.n[2] = NZ;
  p.lambda[0] = 2.0;
  p.lambda[1] = 1.0;
  p.lambda[2] = 1.0;
  p.T = 0.5;
  p.omega = 1.7;
  p.bc[1] = ELBM_BC_BOUNCEBACK;
  p.force[0] = 1e-5;
  p.storage = storage;
  p.extended = 1;
  p.collision = mrt ? ELBM_COLLISION_MRT : ELBM_COLLISION_BGK;
  p.omega_bulk = 1.2;
  p.omega_ghost = 1.0;
  p.mode_k[0] = 6.283185307179586 / (NX * 2.0);
  p.mode_dir[2] = 1.0;

  if (check(elbm_query_bytes(&p, &bytes), "elbm_query_bytes")) return 1;
  if (hipMalloc(&buf, bytes) != hipSuccess) {
    fprintf(stderr, "hipMalloc of %lu bytes failed\n", (unsigned long)bytes);
    return 1;
  }
  if (check(elbm_create(&p, buf, bytes, NULL, &h), "elbm_create")) return 1;

  /* rho = 1 + (y mod 4 - 1.5) / 1024, u_x = 0.02, u_z = ((x mod 8) - 3.5) / 400:
   * every value exact in binary */
  rho = (double*)malloc(n * sizeof *rho);
  u = (double*)malloc(3 * n * sizeof *u);
  for (z = 0; z < NZ; ++z)
    for (y = 0; y < NY; ++y)
      for (x = 0; x < NX; ++x) {
        cell = (size_t)x + (size_t)NX * ((size_t)y + (size_t)NY * (size_t)z);
        rho[cell] = 1.0 + ((double)(y % 4) - 1.5) / 1024.0;
        u[cell] = 0.02;
        u[n + cell] = 0.0;
        u[2 * n + cell] = ((double)(x % 8) - 3.5) / 400.0;
      }
  if (check(elbm_init(h, rho, u), "elbm_init")) return 1;
  if (check(elbm_step(h, 50), "elbm_step")) return 1;
  if (check(elbm_diag(h, &d), "elbm_diag")) return 1;
  if (check(elbm_kernel(h, &k), "elbm_kernel")) return 1;

  printf("step %ld\n", (long)d.step);
  printf("mass %.17g\n", d.mass);
  printf("mom %.17g %.17g %.17g\n", d.mom[0], d.mom[1], d.mom[2]);
  printf("ke %.17g\n", d.ke);
  printf("enstrophy %.17g\n", d.enstrophy);
  printf("mode %.17g %.17g\n", d.mode_re, d.mode_im);
  printf("min_rho %.17g\n", d.min_rho);
  printf("nan_count %ld\n", (long)d.nan_count);
  printf("kernel %d %d\n", (int)k.kernel, (int)k.block_threads);

  elbm_destroy(h);
  hipFree(buf);
  free(rho);
  free(u);
  return 0;
}

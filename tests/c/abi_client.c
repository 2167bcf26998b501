/* A plain C client of the elbm ABI: host-only calls (parameter validation,
 * the device footprint, status strings and the thread's last error), so it
 * runs without a GPU. tests/test_c_abi.py builds it as C99 and as C++17 and
 * compares what it prints with the Python binding. */
#include <stdio.h>
#include <string.h>

#include "elbm.h"

static void fill(elbm_params* p, int lattice, long nx, long ny, long nz, int storage) {
  memset(p, 0, sizeof *p);
  p->abi_version = ELBM_ABI_VERSION;
  p->lattice = lattice;
  p->n[0] = nx;
  p->n[1] = ny;
  p->n[2] = nz;
  p->lambda[0] = 2.0;
  p->lambda[1] = 1.0;
  p->lambda[2] = 1.0;
  p->T = 0.5;
  p->omega = 1.8;
  p->storage = storage;
  p->extended = 1;
  p->collision = ELBM_COLLISION_BGK;
}

int main(void) {
  elbm_params p;
  size_t bytes = 0;
  int32_t s;

  fill(&p, 27, 64, 32, 16, ELBM_STORE_F16);
  s = elbm_validate(&p);
  printf("d3q27_f16_validate %d\n", (int)s);
  s = elbm_query_bytes(&p, &bytes);
  printf("d3q27_f16_bytes %d %lu\n", (int)s, (unsigned long)bytes);

  fill(&p, 9, 96, 40, 1, ELBM_STORE_F32);
  p.bc[1] = ELBM_BC_BOUNCEBACK;
  p.force[0] = 1e-5;
  p.collision = ELBM_COLLISION_MRT;
  p.omega_bulk = 1.2;
  p.omega_ghost = 1.0;
  s = elbm_query_bytes(&p, &bytes);
  printf("d2q9_mrt_bytes %d %lu\n", (int)s, (unsigned long)bytes);

  fill(&p, 27, 64, 32, 16, ELBM_STORE_F32);
  p.omega = 2.5;
  s = elbm_validate(&p);
  printf("bad_omega %d %s\n", (int)s, elbm_status_string(s));
  printf("bad_omega_message %s\n", elbm_last_error());

  fill(&p, 27, 64, 32, 16, ELBM_STORE_F32);
  p.abi_version = ELBM_ABI_VERSION + 1u;
  printf("bad_abi %d\n", (int)elbm_validate(&p));

  printf("static_max %d\n", (int)ELBM_STATIC_MAX_LATTICES);
  return 0;
}

// host_sanitize_driver.cpp -- test driver: the host-side argument checking and
// error paths of libdg (workspace query, size limits, null arguments) built
// with AddressSanitizer / UndefinedBehaviorSanitizer on the host side; it
// makes no call that needs a GPU.
#include <cstdio>
#include <cstring>
#include "dg.h"
int main() {
  int fails = 0;
  dg_mesh_desc d;
  std::memset(&d, 0, sizeof d);
  d.nx = d.ny = d.nz = 4; d.degree = 3;
  size_t n = 0;
  if (dg_query_workspace(&d, &n) != DG_OK || n == 0) ++fails;
  d.degree = 9; if (dg_query_workspace(&d, &n) != DG_ERR_UNSUPPORTED) ++fails;
  d.degree = 3; d.nx = 0; if (dg_query_workspace(&d, &n) != DG_ERR_ARG) ++fails;
  d.nx = 162; d.ny = 162; d.nz = 162; d.degree = 7; if (dg_query_workspace(&d, &n) != DG_ERR_ARG) ++fails;
  if (dg_query_workspace(nullptr, &n) != DG_ERR_ARG) ++fails;
  if (std::strlen(dg_last_error(nullptr)) == 0) ++fails;
  dg_ctx* c = nullptr;
  d.nx = d.ny = d.nz = 2; d.degree = 2;
  if (dg_setup(&d, &c, nullptr) != DG_ERR_ARG) ++fails;  // no workspace
  if (dg_apply(nullptr, DG_F64, nullptr, nullptr, nullptr) != DG_ERR_ARG) ++fails;
  if (dg_cg_solve(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) != DG_ERR_ARG) ++fails;
  dg_destroy(nullptr);
  std::printf(fails ? "host driver: %d failures\n" : "host driver: ok\n", fails);
  return fails;
}

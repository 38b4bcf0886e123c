// Host-only driver of the C ABI's argument handling, for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer: fmm_api.cpp is compiled
// for the host only and linked with the stand-in launchers below (no kernel
// is ever reached: every call here is rejected before the device is used, or
// fails at the first HIP call on a machine without a GPU).  Exit status 0
// when every call returned the expected status.
#include <cstdio>
#include <cstring>

#include "../../include/fmm.h"
#include "../../paper_2606_13793_amd/csrc/fmm_internal.h"

namespace fmm {
// stand-ins for the device-side translation units: never called by this driver
template <int P>
hipError_t Impl<P>::upload_constants() { return hipErrorNoDevice; }
template <int P>
hipError_t Impl<P>::tables(fmm_plan*, hipStream_t) { return hipErrorNoDevice; }
template <int P>
hipError_t Impl<P>::solve(fmm_plan*, IoArg, hipStream_t) { return hipErrorNoDevice; }
template <int P>
hipError_t Impl<P>::backward(fmm_plan*, const AdjWs&, const void*, const void*, void*, hipStream_t) {
  return hipErrorNoDevice;
}
template <int P>
hipError_t Impl<P>::adjoint_tables(fmm_plan*, hipStream_t) { return hipErrorNoDevice; }
template <int P>
hipError_t Impl<P>::finish_locals(fmm_plan*, int, hipStream_t) { return hipErrorNoDevice; }
template <int P>
hipError_t Impl<P>::check_finite(fmm_plan*, const void*, int*, hipStream_t) { return hipErrorNoDevice; }
template struct Impl<1>;
template struct Impl<2>;
template struct Impl<3>;
template struct Impl<4>;
template struct Impl<5>;
template struct Impl<6>;
template struct Impl<7>;
template struct Impl<8>;
hipError_t launch_cic(int, long long count, const double*, const double*, double*, hipStream_t) {
  return count == 0 ? hipSuccess : hipErrorNoDevice;  // the library launches nothing for no particles
}
hipError_t launch_fd_force(int, const double*, double*, hipStream_t) { return hipErrorNoDevice; }
hipError_t noalloc_base(int, void**) { return hipErrorNoDevice; }
hipError_t noalloc_zero(double*, long long, hipStream_t) { return hipErrorNoDevice; }
hipError_t noalloc_put_segs(const Seg*, int, Seg*, hipStream_t) { return hipErrorNoDevice; }
}  // namespace fmm

static int bad = 0;
static void expect(int got, int want, const char* what) {
  if (got != want) {
    std::fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, got, want, fmm_last_error());
    bad = 1;
  }
}

int main() {
  fmm_options o;
  expect(fmm_options_default(&o), FMM_OK, "defaults");
  expect(fmm_options_default(nullptr), FMM_ERR_INVALID_ARG, "defaults NULL");
  const int sizes[][3] = {{12, 4, 1}, {4, 4, 1}, {2048, 4, 1}, {16, 0, 1}, {16, 9, 1}, {16, 4, 0}, {16, 4, 2}};
  const int codes[] = {FMM_ERR_INVALID_ARG, FMM_ERR_INVALID_ARG, FMM_ERR_INVALID_ARG, FMM_ERR_INVALID_ARG,
                       FMM_ERR_INVALID_ARG, FMM_ERR_UNSUPPORTED, FMM_ERR_INVALID_ARG};
  for (int i = 0; i < 7; ++i) {
    expect(fmm_plan_create(sizes[i][0], sizes[i][1], sizes[i][2]) ? 0 : fmm_last_status(), codes[i], "sizes");
  }
  struct Case { int field, value, code; } cases[] = {
      {0, 3, FMM_ERR_UNSUPPORTED}, {1, 7, FMM_ERR_INVALID_ARG}, {2, 5, FMM_ERR_INVALID_ARG},
      {3, 4, FMM_ERR_INVALID_ARG}, {4, -1, FMM_ERR_INVALID_ARG}, {5, 12, FMM_ERR_INVALID_ARG}};
  for (const Case& c : cases) {
    fmm_options x;
    fmm_options_default(&x);
    switch (c.field) {
      case 0: x.delta_l = c.value; break;
      case 1: x.nmax = c.value; break;
      case 2: x.precision = c.value; break;
      case 3: x.struct_size = c.value; break;
      case 4: x.coarse_fp64_levels = c.value; break;
      case 5: x.bottom_tile = c.value; break;
    }
    expect(fmm_plan_create_ex(16, 4, 1, &x) ? 0 : fmm_last_status(), c.code, "options");
  }
  fmm_options x;
  fmm_options_default(&x);
  x.delta_l = 2;
  x.bottom_tile = 8;
  expect(fmm_plan_create_ex(32, 4, 1, &x) ? 0 : fmm_last_status(), FMM_ERR_INVALID_ARG, "fmm2 tile");
  // valid arguments: the first HIP call reports the missing device
  expect(fmm_plan_create(16, 4, 1) ? 0 : fmm_last_status(), FMM_ERR_DEVICE, "no device");
  const int ns[3] = {32, 64, 128}, badn[3] = {32, 48, 128};
  expect(fmm_batch_plan_create(0, ns, 4, 1, &o) ? 0 : fmm_last_status(), FMM_ERR_INVALID_ARG, "batch count");
  expect(fmm_batch_plan_create(3, nullptr, 4, 1, &o) ? 0 : fmm_last_status(), FMM_ERR_INVALID_ARG, "batch n");
  expect(fmm_batch_plan_create(3, badn, 4, 1, &o) ? 0 : fmm_last_status(), FMM_ERR_INVALID_ARG, "batch sizes");
  x = o;
  x.check_finite = 1;
  expect(fmm_batch_plan_create(3, ns, 4, 1, &x) ? 0 : fmm_last_status(), FMM_ERR_UNSUPPORTED, "batch check");
  expect(fmm_solve(nullptr, nullptr, nullptr, nullptr, nullptr), FMM_ERR_INVALID_ARG, "solve NULL");
  expect(fmm_solve_backward(nullptr, nullptr, nullptr, nullptr, nullptr), FMM_ERR_INVALID_ARG, "backward NULL");
  expect(fmm_solve_backward_noalloc(nullptr, nullptr, nullptr, nullptr, nullptr), FMM_ERR_INVALID_ARG,
         "noalloc NULL");
  expect(fmm_batch_solve(nullptr, nullptr, nullptr, nullptr, nullptr), FMM_ERR_INVALID_ARG, "batch solve NULL");
  expect(fmm_batch_info(nullptr, nullptr, nullptr, nullptr, nullptr, 0), FMM_ERR_INVALID_ARG, "batch info NULL");
  expect(fmm_plan_info(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr), FMM_ERR_INVALID_ARG, "info NULL");
  expect((int)fmm_plan_workspace_bytes(nullptr), 0, "bytes NULL");
  fmm_plan_destroy(nullptr);
  expect(fmm_profile_enable(nullptr, 1), FMM_ERR_INVALID_ARG, "profile NULL");
  expect(fmm_profile_read(nullptr, nullptr, nullptr, 0), FMM_ERR_INVALID_ARG, "profile read NULL");
  expect(fmm_profile_stage_name(99) == nullptr ? 0 : 1, 0, "stage name");
  int mi[3 * 220];
  expect(fmm_multi_index(9, mi, sizeof(mi) / sizeof(int)), 220, "multi index");
  expect(fmm_multi_index(10, mi, sizeof(mi) / sizeof(int)), FMM_ERR_INVALID_ARG, "multi index P");
  expect(fmm_deposit_cic(12, 1, (double*)8, (double*)8, (double*)8, nullptr), FMM_ERR_INVALID_ARG, "cic n");
  expect(fmm_deposit_cic(16, -1, (double*)8, (double*)8, (double*)8, nullptr), FMM_ERR_INVALID_ARG, "cic count");
  expect(fmm_deposit_cic(16, 0, nullptr, nullptr, nullptr, nullptr), FMM_OK, "cic empty");
  expect(fmm_fd_force(12, (double*)8, (double*)4096, nullptr), FMM_ERR_INVALID_ARG, "fd n");
  expect(fmm_fd_force(16, (double*)8, (double*)808, nullptr), FMM_ERR_INVALID_ARG, "fd overlap");
  expect(fmm_debug_expansions(nullptr, 0, 2, nullptr, 0), FMM_ERR_INVALID_ARG, "debug NULL");
  expect(std::strlen(fmm_last_error()) > 0 ? 0 : 1, 0, "message");
  if (bad) return 1;
  std::printf("host driver: every call returned the expected status\n");
  return 0;
}

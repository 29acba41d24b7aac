// Driver for the sanitizer run of the C-ABI host layer (tests/test_sanitize.py):
// every entry point of include/los.h with NULL handles, NULL arrays and bad
// sizes, and emu_load on truncated, foreign, future-version and corrupted
// files, so that AddressSanitizer and UndefinedBehaviorSanitizer see the
// argument checks and the file parsing.  Runs without a GPU: every call here
// must fail (or be a no-op) before it reaches the device or the handle.
// Exit status 0 when every call returned what it should.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "los.h"

static int failures = 0;

static void expect(bool cond, const char *what) {
  if (!cond) {
    std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, los_last_error());
    ++failures;
  }
}

static void expect_err(int rc, const char *what) {
  expect(rc != LOS_OK && std::strlen(los_last_error()) > 0, what);
}

static void write_file(const std::string &path, const std::vector<unsigned char> &bytes) {
  FILE *f = std::fopen(path.c_str(), "wb");
  if (!f) return;
  std::fwrite(bytes.data(), 1, bytes.size(), f);
  std::fclose(f);
}

int main(int argc, char **argv) {
  const std::string dir = argc > 1 ? argv[1] : ".";
  expect(std::strstr(los_version(), "gfx950") != nullptr, "los_version");
  // a stand-in handle: only calls that reject their arguments before using it get it
  alignas(64) static unsigned char fake[256] = {};
  los_ctx *ctx = reinterpret_cast<los_ctx *>(fake);
  los_emu *emu = reinterpret_cast<los_emu *>(fake);
  const double d[8] = {0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8};
  double out[64];
  void *p = out;

  expect_err(los_ctx_create(nullptr, nullptr), "ctx_create NULL out");
  expect_err(los_bessel_table(nullptr, d, 4, 2, 10, out, nullptr), "bessel_table NULL ctx");
  expect_err(los_project(nullptr, 2, 10, 4, 8, 1.0, d, d, d, d, 1, 0, p, nullptr),
             "project NULL ctx");
  expect_err(los_project_kernels(nullptr, 2, 10, 4, 8, 1.0, d, d, d, d, 1, 0u, 0, p, nullptr),
             "project_kernels NULL ctx");
  expect_err(los_project_tensor(nullptr, 2, 10, 4, 8, 1.0, d, d, d, d, out, nullptr),
             "project_tensor NULL ctx");
  const int32_t pairs[2] = {0, 0};
  expect_err(cl_integrate(nullptr, p, 0, 1, 10, 4, d, d, pairs, 1, out, nullptr),
             "cl_integrate NULL ctx");
  expect_err(cl_integrate_noalloc(nullptr, p, 0, 1, 10, 4, d, d, pairs, 1, out, nullptr),
             "cl_integrate_noalloc NULL ctx");
  expect_err(cl_integrate_noalloc(ctx, p, 0, 0, 10, 4, d, d, pairs, 1, out, nullptr),
             "cl_integrate_noalloc nsrc 0");
  expect_err(cl_integrate_noalloc(ctx, nullptr, 0, 1, 10, 4, d, d, pairs, 1, out, nullptr),
             "cl_integrate_noalloc NULL delta");
  std::vector<int32_t> many(32, 0);
  expect_err(cl_integrate_noalloc(ctx, p, 0, 1, 16000, 20, d, d, many.data(), 16, out, nullptr),
             "cl_integrate_noalloc beyond the scratch");
  const int32_t ls[3] = {2, 5, 9};
  expect_err(los_project_lsample(nullptr, 2, 10, ls, 3, 4, 8, 1.0, d, d, d, d, 1, 0u, out,
                                 nullptr),
             "project_lsample NULL ctx");
  expect_err(los_cl_interp(nullptr, 1, ls, 3, d, 2, 10, out, nullptr), "cl_interp NULL ctx");
  expect_err(los_spline_sources(nullptr, 1, 4, 8, d, d, out, nullptr), "spline NULL ctx");
  expect_err(los_interp_sources(nullptr, 1, 4, 8, d, d, d, 4, d, 0, p, nullptr),
             "interp NULL ctx");

  los_batch *plan = nullptr;
  const int32_t lmax[2] = {100, 200};
  const int64_t koff[3] = {0, 2, 4}, kidx[4] = {0, 1, 0, 2};
  expect_err(los_batch_create(nullptr, 2, 3, lmax, koff, kidx, 3, 8, pairs, 1, 1, &plan),
             "batch_create NULL ctx");
  expect_err(los_batch_create(ctx, 2, 3, lmax, koff, kidx, 3, 8, pairs, 1, 1, nullptr),
             "batch_create NULL out");
  int64_t col[4], ncols = 0;
  int32_t info[10];
  expect_err(los_batch_columns(nullptr, col, &ncols), "batch_columns NULL plan");
  expect_err(los_batch_info(nullptr, info), "batch_info NULL plan");
  expect_err(los_batch_solve(nullptr, 1.0, d, d, d, nullptr, d, d, out, nullptr),
             "batch_solve NULL plan");
  double ms[3];
  int32_t launches[3];
  expect_err(los_batch_solve_timed(nullptr, 1.0, d, d, d, nullptr, d, d, out, ms, launches,
                                   nullptr),
             "batch_solve_timed NULL plan");
  los_batch_destroy(nullptr);

  los_emu *e = nullptr;
  expect_err(emu_create(nullptr, 5, 10, 4, 8, 1, 2, 1, &e), "emu_create NULL ctx");
  int64_t count = 0;
  expect_err(emu_nparams(nullptr, &count), "emu_nparams NULL");
  expect_err(emu_get_params(nullptr, 0, nullptr), "emu_get_params NULL");
  expect_err(emu_set_params(nullptr, 0, nullptr), "emu_set_params NULL");
  expect_err(emu_get_pca(nullptr, out, out, out, out, out, out), "emu_get_pca NULL");
  expect_err(emu_set_pca(nullptr, d, d, d, d, d, d), "emu_set_pca NULL");
  float f32[16];
  expect_err(emu_forward(nullptr, 0, f32, 4, f32, nullptr), "emu_forward NULL");
  expect_err(emu_loss_grad(nullptr, 0, f32, f32, 4, f32, f32, nullptr), "emu_loss_grad NULL");
  expect_err(emu_fit(nullptr, 0, f32, f32, 4, 1, 2, 1e-3, nullptr, nullptr), "emu_fit NULL");
  expect_err(emu_train(nullptr, d, d, d, d, 4, 1, 2, 1e-3, nullptr, nullptr), "emu_train NULL");
  uint8_t flags[16];
  expect_err(emu_infer(nullptr, d, 4, out, f32, flags, 1e-3, nullptr), "emu_infer NULL");
  expect_err(emu_infer_spectra(nullptr, d, 4, out, f32, flags, 1e-3, nullptr),
             "emu_infer_spectra NULL");
  const int64_t rows[2] = {0, 1}, twice[2] = {1, 1}, outside[2] = {0, 9};
  expect_err(emu_merge(nullptr, rows, 2, d, out, 4, nullptr, nullptr, nullptr), "emu_merge NULL");
  expect_err(emu_merge(emu, twice, 2, d, out, 4, nullptr, nullptr, nullptr), "emu_merge twice");
  expect_err(emu_merge(emu, outside, 2, d, out, 4, nullptr, nullptr, nullptr),
             "emu_merge outside");
  expect_err(emu_merge(emu, rows, 3, d, out, 2, nullptr, nullptr, nullptr), "emu_merge nf > n");
  expect(emu_merge(emu, rows, 0, nullptr, nullptr, 4, nullptr, nullptr, nullptr) == LOS_OK,
         "emu_merge nf = 0 is a no-op");
  expect_err(emu_merge_spectrum(emu, 4, rows, 2, d, out, 4, nullptr, nullptr, nullptr),
             "emu_merge_spectrum spectrum 4");
  expect_err(emu_merge_spectrum(emu, 0, twice, 2, d, out, 4, nullptr, nullptr, nullptr),
             "emu_merge_spectrum twice");
  expect_err(emu_merge_spectrum(emu, 0, outside, 2, d, out, 4, nullptr, nullptr, nullptr),
             "emu_merge_spectrum outside");
  expect_err(emu_save(nullptr, (dir + "/none.bin").c_str(), nullptr), "emu_save NULL");
  emu_destroy(nullptr);

  // emulator files that must be refused while parsing (before the context is used)
  expect_err(emu_load(ctx, (dir + "/missing.bin").c_str(), &e), "emu_load missing file");
  expect_err(emu_load(nullptr, (dir + "/missing.bin").c_str(), &e), "emu_load NULL ctx");
  expect_err(emu_load(ctx, nullptr, &e), "emu_load NULL path");
  expect_err(emu_load(ctx, (dir + "/missing.bin").c_str(), nullptr), "emu_load NULL out");
  std::vector<unsigned char> head(64, 0);
  std::memcpy(head.data(), "LOSEMU01", 8);
  write_file(dir + "/short.bin", std::vector<unsigned char>(head.begin(), head.begin() + 40));
  expect_err(emu_load(ctx, (dir + "/short.bin").c_str(), &e), "emu_load short");
  std::vector<unsigned char> foreign(200, 7);
  write_file(dir + "/foreign.bin", foreign);
  expect_err(emu_load(ctx, (dir + "/foreign.bin").c_str(), &e), "emu_load foreign");
  std::vector<unsigned char> corrupt = head;
  corrupt.resize(300, 0);
  write_file(dir + "/corrupt.bin", corrupt);  // right magic, checksum does not match
  expect_err(emu_load(ctx, (dir + "/corrupt.bin").c_str(), &e), "emu_load corrupt");
  expect(e == nullptr, "emu_load leaves *emu NULL on failure");

  if (failures)
    std::fprintf(stderr, "%d failures\n", failures);
  else
    std::printf("sanitized C-ABI host run: every call returned as expected\n");
  return failures ? 1 : 0;
}

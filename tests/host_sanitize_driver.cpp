// Host-only driver for the sanitizer build of the planner and the C ABI's
// argument handling (no GPU needed: every device call reports "no device").
// Built by tests/test_host_sanitizers.py with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of tcfft.cpp and serve.cpp.
// Exits 0 when every check holds; the sanitizers abort on the first error.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../include/tcfft.h"

static int g_fail = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++g_fail;                                                    \
    }                                                              \
  } while (0)

// The description must be one JSON object: balanced braces and brackets.
static bool balanced(const char* s) {
  int b = 0, k = 0;
  for (; *s; ++s) {
    b += *s == '{' ? 1 : *s == '}' ? -1 : 0;
    k += *s == '[' ? 1 : *s == ']' ? -1 : 0;
    if (b < 0 || k < 0) return false;
  }
  return b == 0 && k == 0;
}

int main(int argc, char** argv) {
  const char* tmp = argc > 1 ? argv[1] : "/tmp";
  std::vector<char> buf(1 << 16);
  // every 1D size, both precisions and directions, real and complex, with a
  // truncating buffer too (the description is cut, never overrun)
  for (int lg = 0; lg <= 28; ++lg)
    for (int prec = 0; prec < 3; ++prec)
      for (unsigned flags : {0u, 1u, 8u})
        for (int dir : {-1, 1}) {
          const int64_t dims[1] = {(int64_t)1 << lg};
          int n = tcfft_plan_dry_run(1, dims, 3, dir, prec, flags, buf.data(), buf.size());
          const bool ok = lg >= 4 && lg <= 27 && !(flags & 8u && (prec == 2 || lg < 5));
          CHECK((n > 0) == ok);
          if (n > 0) CHECK(balanced(buf.data()));
          char small[17];
          std::memset(small, 'x', sizeof small);
          int m = tcfft_plan_dry_run(1, dims, 3, dir, prec, flags, small, 16);
          CHECK(m == n);
          CHECK(small[16] == 'x');
          if (m > 0) CHECK(std::strlen(small) == 15);
        }
  // 2D and 3D shapes, in and out of range
  for (int a = 2; a <= 15; ++a)
    for (int b = 2; b <= 15; ++b)
      for (int prec = 0; prec < 2; ++prec) {
        const int64_t d2[2] = {(int64_t)1 << a, (int64_t)1 << b};
        int n = tcfft_plan_dry_run(2, d2, 2, -1, prec, 0, buf.data(), buf.size());
        CHECK((n > 0) == (a >= 4 && a <= 11 && b >= 4 && b <= 14));
        for (int c = 4; c <= 14; c += 5) {
          const int64_t d3[3] = {(int64_t)1 << a, (int64_t)1 << b, (int64_t)1 << c};
          int m = tcfft_plan_dry_run(3, d3, 1, 1, prec, 0, buf.data(), buf.size());
          CHECK((m > 0) == (a >= 4 && a <= 11 && b >= 4 && b <= 11 && a + b + c <= 31));
        }
      }
  // rejected arguments
  const int64_t d1[1] = {4096};
  CHECK(tcfft_plan_dry_run(1, d1, 0, -1, 0, 0, buf.data(), buf.size()) == -TCFFT_ERR_INVALID_ARG);
  CHECK(tcfft_plan_dry_run(1, d1, 1, 0, 0, 0, buf.data(), buf.size()) == -TCFFT_ERR_INVALID_ARG);
  CHECK(tcfft_plan_dry_run(1, d1, 1, -1, 7, 0, buf.data(), buf.size()) == -TCFFT_ERR_INVALID_ARG);
  CHECK(tcfft_plan_dry_run(1, d1, 1, -1, 0, 64, buf.data(), buf.size()) == -TCFFT_ERR_INVALID_ARG);
  CHECK(tcfft_plan_dry_run(4, d1, 1, -1, 0, 0, buf.data(), buf.size()) == -TCFFT_ERR_INVALID_ARG);
  CHECK(tcfft_plan_dry_run(1, nullptr, 1, -1, 0, 0, buf.data(), buf.size()) ==
        -TCFFT_ERR_INVALID_ARG);
  const int64_t big[1] = {(int64_t)1 << 27};
  CHECK(tcfft_plan_dry_run(1, big, 17, -1, 0, 0, buf.data(), buf.size()) == -TCFFT_ERR_UNSUPPORTED);
  // shard plans
  for (int lg = 14; lg <= 28; ++lg)
    for (int g = 1; g <= 64; g *= 2)
      for (int s = -1; s <= g; ++s) {
        int n = tcfft_shard_dry_run((int64_t)1 << lg, 2, -1, 0, g, s, 0, buf.data(), buf.size());
        if (n > 0) CHECK(balanced(buf.data()) && s >= 0 && s < g && g >= 2);
      }
  // autotuner candidates and the wisdom file
  for (int lg = 4; lg <= 27; ++lg) {
    const int64_t dims[1] = {(int64_t)1 << lg};
    int n = tcfft_tune_candidates(1, dims, 1, 0, nullptr, 0);
    CHECK(n > 0);
    std::vector<char> cb((size_t)n + 1);
    CHECK(tcfft_tune_candidates(1, dims, 1, 0, cb.data(), cb.size()) == n);
    CHECK(balanced(cb.data()));
  }
  const std::string wis = std::string(tmp) + "/tcfft_asan_wisdom.txt";
  CHECK(tcfft_tune_cache_save(wis.c_str()) == TCFFT_OK);
  CHECK(tcfft_tune_cache_load(wis.c_str()) == TCFFT_OK);
  FILE* f = std::fopen(wis.c_str(), "w");
  std::fprintf(f, "tcfft-tune 3\nr1_65536x1_b11_p0 256 64 2 256 256 0 0 0 1.0\n"
                  "r1_1024x1_b0_p0 256 64 9 1 2 3 0 0 1.0\n"
                  "%s 1 2 3\n", std::string(300, 'k').c_str());
  std::fclose(f);
  CHECK(tcfft_tune_cache_load(wis.c_str()) == TCFFT_OK);
  CHECK(tcfft_tune_cache_size() == 1);
  f = std::fopen(wis.c_str(), "w");
  std::fprintf(f, "garbage\n");
  std::fclose(f);
  CHECK(tcfft_tune_cache_load(wis.c_str()) == TCFFT_ERR_INVALID_ARG);
  CHECK(tcfft_tune_cache_load("/nonexistent/dir/x") == TCFFT_ERR_INVALID_ARG);
  tcfft_tune_cache_clear();
  std::remove(wis.c_str());
  // device entry points without a device, and null handles
  tcfft_plan p = (tcfft_plan)0x1;
  CHECK(tcfft_plan_create(&p, 1, d1, 1, -1, 0, 0) == TCFFT_ERR_NO_DEVICE);
  CHECK(p == nullptr);
  CHECK(tcfft_plan_create_shard(&p, (int64_t)1 << 20, 1, -1, 0, 4, 1, 0) == TCFFT_ERR_NO_DEVICE);
  CHECK(tcfft_exec(nullptr, nullptr, nullptr, nullptr) == TCFFT_ERR_INVALID_ARG);
  CHECK(tcfft_exec_many(nullptr, nullptr, nullptr, -1, nullptr) == TCFFT_ERR_INVALID_ARG);
  CHECK(tcfft_exec_many(nullptr, nullptr, nullptr, 0, nullptr) == TCFFT_OK);
  CHECK(tcfft_plan_destroy(nullptr) == TCFFT_OK);
  CHECK(tcfft_plan_scale_log2(nullptr) == -1);
  CHECK(tcfft_plan_describe(nullptr, buf.data(), buf.size()) == -1);
  tcfft_server srv = nullptr;
  tcfft_server_config cfg{};
  CHECK(tcfft_server_create(&srv, &cfg) == TCFFT_ERR_INVALID_ARG);
  cfg.nslots = 2;
  cfg.max_batch_jobs = 8;
  cfg.mem_budget_bytes = 1 << 20;
  CHECK(tcfft_server_create(&srv, &cfg) == TCFFT_ERR_NO_DEVICE);
  CHECK(tcfft_server_destroy(nullptr) == TCFFT_OK);
  for (int s = 0; s < 9; ++s) CHECK(tcfft_status_string((tcfft_status)s) != nullptr);
  std::printf("host sanitizer driver: %d failed checks\n", g_fail);
  return g_fail == 0 ? 0 : 1;
}

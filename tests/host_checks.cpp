// Checks of libmihs's host-only code (paper_1912_03514_amd/csrc/host.cpp): the
// momentum rules, the lambda map, the batched schedule on random problem sets
// and the tuning-cache file.  test_host_sanitizers.py builds this file with
// that one under AddressSanitizer and UndefinedBehaviorSanitizer and runs it;
// any finding aborts the run.  Usage: host_checks <scratch directory>.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <random>
#include <string>
#include <vector>

#include "../paper_1912_03514_amd/csrc/internal.hpp"

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                  \
    }                                                              \
  } while (0)

static void momentum_checks() {
  double a = 0, b = 0;
  CHECK(mihs_momentum_cor4(512.0, 2048, &a, &b) == MIHS_OK && b == 0.25 && a == 0.5625);
  CHECK(mihs_momentum_cor4(2048.0, 2048, &a, &b) == MIHS_ERR_INVALID);
  CHECK(mihs_momentum_cor4(NAN, 10, &a, &b) == MIHS_ERR_INVALID);
  CHECK(mihs_momentum_cor4(1.0, 0, &a, &b) == MIHS_ERR_INVALID);
  CHECK(mihs_momentum_cor4(1.0, 4, nullptr, &b) == MIHS_ERR_INVALID);
  for (double eps = 1e-6; eps < 1.0; eps += 0.0625) {
    CHECK(mihs_momentum_thm1(eps, &a, &b) == MIHS_OK);
    CHECK(b > 0.0 && b < 1.0 && a > 0.0 && a <= 1.0);
  }
  CHECK(mihs_momentum_thm1(1.0, &a, &b) == MIHS_ERR_INVALID);
  CHECK(mihs_lambda_from_log(-3.0, &a) == MIHS_OK && a == exp(-3.0));
  CHECK(mihs_lambda_from_log(1e6, &a) == MIHS_ERR_INVALID);
  CHECK(mihs_lambda_from_log(0.0, nullptr) == MIHS_ERR_INVALID);
}

// Every entry has a team inside [0, num_cu), its CG sub-team fits the team, and
// the schedule is a function of its inputs.
static void schedule_checks(std::mt19937_64& rng) {
  std::uniform_int_distribution<int> dprob(1, 400), dlam(1, 40), dd(1, 1024), dcu(1, 304);
  for (int trial = 0; trial < 60; ++trial) {
    const int nprob = dprob(rng), nlam = dlam(rng), num_cu = dcu(rng);
    std::vector<int64_t> n(nprob), d(nprob);
    for (int p = 0; p < nprob; ++p) {
      d[p] = dd(rng);
      n[p] = d[p] + (int64_t)(rng() % 70000);
    }
    const int64_t count = (int64_t)nprob * ((nlam + 15) / 16);
    mihs_batched_tuning_t tn;
    mihs_batched_default_tuning(&tn);
    const int32_t cols[] = {16, 32, 64, 512};
    tn.cg_cols = cols[trial % 4];
    tn.exact = trial % 3 == 0;
    tn.measured = trial % 2;
    std::vector<double> cost(count);
    for (auto& c : cost) c = 1.0 + (double)(rng() % 100000);
    std::vector<int32_t> t0(count), ts(count), tc(count), t0b(count), tsb(count), tcb(count);
    const int rc = mihs_batched_schedule(num_cu, n.data(), d.data(), nprob, nlam, &tn,
                                         tn.measured ? cost.data() : nullptr, t0.data(),
                                         ts.data(), tc.data());
    if (rc == MIHS_ERR_UNSUPPORTED) continue;  // more entries than the workgroups can hold
    CHECK(rc == MIHS_OK);
    const int rc2 = mihs_batched_schedule(num_cu, n.data(), d.data(), nprob, nlam, &tn,
                                          tn.measured ? cost.data() : nullptr, t0b.data(),
                                          tsb.data(), tcb.data());
    CHECK(rc2 == MIHS_OK && t0 == t0b && ts == tsb && tc == tcb);
    for (int64_t i = 0; i < count; ++i) {
      CHECK(ts[i] >= 1 && t0[i] >= 0 && t0[i] + ts[i] <= num_cu);
      CHECK(tc[i] >= 1 && tc[i] <= ts[i]);
    }
  }
  mihs_batched_tuning_t bad;
  mihs_batched_default_tuning(&bad);
  bad.cg_cols = 48;
  int64_t n1 = 100, d1 = 10;
  int32_t o[1];
  CHECK(mihs_batched_schedule(8, &n1, &d1, 1, 1, &bad, nullptr, o, o, o) == MIHS_ERR_INVALID);
  CHECK(mihs_batched_schedule(0, &n1, &d1, 1, 1, &bad, nullptr, o, o, o) == MIHS_ERR_INVALID);
}

static void write_file(const std::string& path, const std::string& text) {
  FILE* f = fopen(path.c_str(), "wb");
  if (!f) {
    ++failures;
    return;
  }
  fwrite(text.data(), 1, text.size(), f);
  fclose(f);
}

static void cache_checks(const std::string& dir, std::mt19937_64& rng) {
  mihs_handle h{};
  h.device = 0;
  h.num_cu = 256;
  strcpy(h.arch, "gfx950");
  for (int k = 0; k < 5; ++k) {
    mihs_tuned_set t;
    t.key = rng();
    mihs_batched_default_tuning(&t.tuning);
    t.tuning.cg_cols = k % 2 ? 512 : 16;
    t.tuning.inner_weight = 6.25 * (k + 1);
    t.tuning.measured = k % 2;
    t.tuning.exact = k == 3;
    for (int j = 0; j < 3 * k; ++j) t.cost.push_back(1.0 + 1e3 * (double)(rng() % 997) / 7.0);
    h.tuned.push_back(t);
  }
  const std::string path = dir + "/tuning.json";
  CHECK(mihs_tuning_cache_save(&h, path.c_str()) == MIHS_OK);
  mihs_handle g{};
  g.num_cu = 256;
  strcpy(g.arch, "gfx950");
  int32_t loaded = -1;
  CHECK(mihs_tuning_cache_load(&g, path.c_str(), &loaded) == MIHS_OK && loaded == 5);
  CHECK(g.tuned.size() == h.tuned.size());
  for (size_t i = 0; i < h.tuned.size() && i < g.tuned.size(); ++i) {
    CHECK(g.tuned[i].key == h.tuned[i].key);
    CHECK(memcmp(&g.tuned[i].tuning.cg_cols, &h.tuned[i].tuning.cg_cols, 8) == 0);
    CHECK(g.tuned[i].tuning.inner_weight == h.tuned[i].tuning.inner_weight);
    CHECK(g.tuned[i].tuning.exact == h.tuned[i].tuning.exact);
    CHECK(g.tuned[i].cost == h.tuned[i].cost);  // %.17g round trip is exact
  }
  // loading twice replaces equal keys instead of adding them
  CHECK(mihs_tuning_cache_load(&g, path.c_str(), &loaded) == MIHS_OK && g.tuned.size() == 5);
  // another device: read, ignored
  mihs_handle other{};
  other.num_cu = 80;
  strcpy(other.arch, "gfx950");
  CHECK(mihs_tuning_cache_load(&other, path.c_str(), &loaded) == MIHS_OK && loaded == 0 &&
        other.tuned.empty());
  // malformed or foreign files are rejected and leave the handle unchanged
  const char* bad[] = {
      "",
      "{",
      "[]",
      "{\"format\": \"something else\", \"version\": 1, \"arch\": \"gfx950\", \"num_cu\": 256, "
      "\"entries\": []}",
      "{\"format\": \"libmihs-batched-tuning\", \"version\": 2, \"arch\": \"gfx950\", "
      "\"num_cu\": 256, \"entries\": []}",
      "{\"format\": \"libmihs-batched-tuning\", \"version\": 1, \"arch\": \"gfx950\", "
      "\"num_cu\": 256, \"entries\": [{\"key\": \"12\", \"cg_cols\": 32}]}",
      "{\"format\": \"libmihs-batched-tuning\", \"version\": 1, \"arch\": \"gfx950\", "
      "\"num_cu\": 256, \"entries\": [{\"key\": \"00000000000000ab\", \"cg_cols\": 48, "
      "\"a_dma\": 1, \"inner_weight\": 100, \"measured\": 0, \"exact\": 0, \"cost\": []}]}",
      "{\"format\": \"libmihs-batched-tuning\", \"version\": 1, \"arch\": \"gfx\\\"950\", "
      "\"num_cu\": 256, \"entries\": []}",
      "{\"format\": \"libmihs-batched-tuning\", \"version\": 1} trailing",
  };
  for (const char* text : bad) {
    write_file(dir + "/bad.json", text);
    const size_t before = g.tuned.size();
    CHECK(mihs_tuning_cache_load(&g, (dir + "/bad.json").c_str(), &loaded) ==
          MIHS_ERR_INVALID);
    CHECK(g.tuned.size() == before);
  }
  // random truncations and byte flips of a valid file never crash the reader
  FILE* f = fopen(path.c_str(), "rb");
  std::string good;
  char buf[4096];
  size_t got;
  while (f && (got = fread(buf, 1, sizeof(buf), f)) > 0) good.append(buf, got);
  if (f) fclose(f);
  for (int k = 0; k < 300; ++k) {
    std::string t = good.substr(0, rng() % (good.size() + 1));
    if (!t.empty() && k % 2) t[rng() % t.size()] = (char)(rng() % 256);
    write_file(dir + "/fuzz.json", t);
    mihs_handle z{};
    z.num_cu = 256;
    strcpy(z.arch, "gfx950");
    const int rc = mihs_tuning_cache_load(&z, (dir + "/fuzz.json").c_str(), &loaded);
    CHECK(rc == MIHS_OK || rc == MIHS_ERR_INVALID);
  }
  CHECK(mihs_tuning_cache_load(&g, (dir + "/missing.json").c_str(), &loaded) == MIHS_ERR_INVALID);
}

int main(int argc, char** argv) {
  if (argc < 2) {
    fprintf(stderr, "usage: host_checks <scratch directory>\n");
    return 2;
  }
  std::mt19937_64 rng(12345);
  momentum_checks();
  schedule_checks(rng);
  cache_checks(argv[1], rng);
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("host checks passed\n");
  return 0;
}

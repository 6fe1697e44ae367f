// Host-only parts of libmihs: the momentum rules, the lambda parametrisation,
// the batched launch's schedule and tuning records, and the tuning-cache file.
// Plain C++ (no device code), so that it also builds with the host compiler
// alone, e.g. under AddressSanitizer / UndefinedBehaviorSanitizer in the CPU
// tests.
#include <errno.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.hpp"

namespace mihs {

bool block_tuning_valid(const mihs_batched_tuning_t& t) {
  return (t.cg_cols == 16 || t.cg_cols == 32 || t.cg_cols == 64 || t.cg_cols == 128 ||
          t.cg_cols == 512) &&
         (t.a_dma == 0 || t.a_dma == 1) && t.inner_weight >= 1.0 && t.inner_weight <= 1e4 &&
         (t.measured == 0 || t.measured == 1) && (t.exact == 0 || t.exact == 1);
}

// Sizing from measured costs c_i (entry i on one workgroup): the smallest
// makespan L (bisection) for which teams of ceil(c_i / L) workgroups for the
// entries above L and first-fit-decreasing bins of capacity L for the rest
// (team members offering what their team entry leaves of L) fit
// in G workgroups.
static bool makespan_schedule(const std::vector<double>& c, int G, double L, Schedule* S) {
  const int64_t count = (int64_t)c.size();
  std::vector<int64_t> order(count);
  for (int64_t i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return c[x] > c[y]; });
  S->team0.assign(count, 0);
  S->tsize.assign(count, 1);
  S->tcg.assign(count, 1);
  S->items.assign(G, std::vector<int>());
  std::vector<double> load(G, 0.0);
  int next = 0;
  for (int64_t i : order) {
    if (c[i] <= L) break;
    const int t = (int)std::ceil(c[i] / L - 1e-9);
    if (next + t > G) return false;
    S->team0[i] = next;
    S->tsize[i] = t;
    for (int u = 0; u < t; ++u) {
      S->items[next + u].push_back((int)i);
      load[next + u] = c[i] / t;
    }
    next += t;
  }
  // the rest first-fit in decreasing cost over every workgroup, the team
  // members' remaining capacity included (a team entry always comes first in
  // its members' lists, so no team waits on a member busy elsewhere)
  for (int64_t i : order) {
    if (c[i] > L) continue;
    int g = 0;
    while (g < G && load[g] + c[i] > L * (1.0 + 1e-9)) ++g;
    if (g == G) return false;
    load[g] += c[i];
    S->team0[i] = g;
    S->items[g].push_back((int)i);
  }
  return true;
}

int make_schedule(const BlockEntryDesc* ents, int64_t count, int G,
                  const mihs_batched_tuning_t& tn, const std::vector<double>* cost,
                  Schedule* S) {
  if (tn.measured && cost && (int64_t)cost->size() == count) {
    double hi = 0.0, sum = 0.0;
    for (double v : *cost) {
      hi = std::max(hi, std::max(v, 1.0));
      sum += std::max(v, 1.0);
    }
    std::vector<double> c(count);
    for (int64_t i = 0; i < count; ++i) c[i] = std::max((*cost)[i], 1.0);
    double lo = std::max(sum / G, 1.0);
    hi = std::max(hi, sum);  // one entry per workgroup in turn always fits when count <= G
    Schedule T;
    if (!makespan_schedule(c, G, hi, &T)) return MIHS_ERR_UNSUPPORTED;
    for (int it = 0; it < 48 && hi > lo * (1.0 + 1e-4); ++it) {
      const double mid = 0.5 * (lo + hi);
      Schedule U;
      if (makespan_schedule(c, G, mid, &U)) {
        hi = mid;
        T = U;
      } else {
        lo = mid;
      }
    }
    *S = T;
    for (int64_t i = 0; i < count; ++i)
      S->tcg[i] = tn.exact ? std::min(S->tsize[i], kBlockRhs) : std::max(
          1, std::min(S->tsize[i], (int)((ents[i].d + tn.cg_cols - 1) / tn.cg_cols)));
    S->stride = 1;
    for (int g = 0; g < G; ++g) S->stride = std::max(S->stride, S->items[g].size() + 1);
    return MIHS_OK;
  }
  // weight: one A pass plus the expected inner solve on H per outer iteration
  // (inner_weight passes over H; lockstep CGs over 16 lambdas down to
  // 1e-6 sigma_1^2 take ~100 steps)
  std::vector<double> wgt(count);
  double total = 0.0;
  for (int64_t i = 0; i < count; ++i) {
    wgt[i] = (double)ents[i].n * ents[i].d + tn.inner_weight * (double)ents[i].d * ents[i].d;
    total += wgt[i];
  }
  std::vector<int64_t> order(count);
  for (int64_t i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t x, int64_t y) { return wgt[x] > wgt[y]; });
  S->team0.assign(count, 0);
  S->tsize.assign(count, 1);
  S->tcg.assign(count, 1);
  S->items.assign(G, std::vector<int>());
  // An entry gets a share of the still-free workgroups proportional to its
  // share of the still-unassigned weight, keeping one workgroup free while
  // other entries remain; entries worth fewer than two go to the bins.
  int next = 0;
  int64_t first_small = count;
  double left = total;
  for (int64_t oi = 0; oi < count; ++oi) {
    const int64_t i = order[oi];
    const int free_wg = G - next;
    const int reserve = (oi + 1 < count) ? 1 : 0;
    int want = (int)std::floor(wgt[i] / left * free_wg + 0.5);
    want = std::min(want, free_wg - reserve);
    if (want < 2) {
      first_small = oi;
      break;
    }
    S->team0[i] = next;
    S->tsize[i] = want;
    for (int t = 0; t < want; ++t) S->items[next + t].push_back((int)i);
    next += want;
    left -= wgt[i];
  }
  std::vector<double> load(G, 0.0);
  for (int64_t oi = first_small; oi < count; ++oi) {
    const int64_t i = order[oi];
    if (next >= G) return MIHS_ERR_UNSUPPORTED;
    int best = next;
    for (int g = next; g < G; ++g)
      if (load[g] < load[best]) best = g;
    S->team0[i] = best;
    S->tsize[i] = 1;
    S->items[best].push_back((int)i);
    load[best] += wgt[i];
  }
  // CG sub-team: about cg_cols columns of H per member, at most the whole team
  // (exact sub-solves: every member up to one per column)
  for (int64_t i = 0; i < count; ++i)
    S->tcg[i] = tn.exact ? std::min(S->tsize[i], kBlockRhs) : std::max(
        1, std::min(S->tsize[i], (int)((ents[i].d + tn.cg_cols - 1) / tn.cg_cols)));
  S->stride = 1;
  for (int g = 0; g < G; ++g) S->stride = std::max(S->stride, S->items[g].size() + 1);
  return MIHS_OK;
}

static uint64_t mix64(uint64_t h, uint64_t v) {
  // FNV-1a over the 8 bytes of v
  for (int b = 0; b < 8; ++b) {
    h ^= (v >> (8 * b)) & 0xFFu;
    h *= 1099511628211ull;
  }
  return h;
}

uint64_t block_signature(const BlockEntryDesc* ents, int64_t count) {
  uint64_t s = 1469598103934665603ull;
  s = mix64(s, (uint64_t)count);
  for (int64_t i = 0; i < count; ++i) {
    s = mix64(s, (uint64_t)ents[i].n);
    s = mix64(s, (uint64_t)ents[i].d);
    s = mix64(s, (uint64_t)ents[i].m);
    s = mix64(s, (uint64_t)ents[i].ncols);
    s = mix64(s, (uint64_t)ents[i].sa_group);
  }
  return s;
}

mihs_batched_tuning_t block_tuning_for(mihs_handle* h, const BlockEntryDesc* ents, int64_t count,
                                       std::vector<double>* cost) {
  mihs_batched_tuning_t tn;
  mihs_batched_default_tuning(&tn);
  if (cost) cost->clear();
  const uint64_t key = block_signature(ents, count);
  std::lock_guard<std::mutex> lock(h->tune_mu);
  for (const auto& t : h->tuned)
    if (t.key == key) {
      if (cost) *cost = t.cost;
      return t.tuning;
    }
  return tn;
}

bool block_tuning_lookup(mihs_handle* h, const BlockEntryDesc* ents, int64_t count,
                         mihs_batched_tuning_t* tuning) {
  const uint64_t key = block_signature(ents, count);
  std::lock_guard<std::mutex> lock(h->tune_mu);
  for (const auto& t : h->tuned)
    if (t.key == key) {
      *tuning = t.tuning;
      return true;
    }
  return false;
}

void block_tuning_store(mihs_handle* h, const BlockEntryDesc* ents, int64_t count,
                        const mihs_batched_tuning_t& tuning, const std::vector<double>& cost) {
  const uint64_t key = block_signature(ents, count);
  std::lock_guard<std::mutex> lock(h->tune_mu);
  for (auto& t : h->tuned)
    if (t.key == key) {
      t.tuning = tuning;
      t.cost = cost;
      return;
    }
  h->tuned.push_back(mihs_tuned_set{key, tuning, cost});
}

int block_team_sizes(const mihs_handle* h, const BlockEntryDesc* ents, int64_t count,
                     const mihs_batched_tuning_t& tuning, const std::vector<double>* cost,
                     std::vector<int>* tsize) {
  Schedule S;
  const int rc = make_schedule(ents, count, h->num_cu, tuning, cost, &S);
  if (rc) return rc;
  *tsize = S.tsize;
  return MIHS_OK;
}

}  // namespace mihs

extern "C" int mihs_batched_schedule(int32_t num_cu, const int64_t* n, const int64_t* d,
                                     int64_t nprob, int64_t nlam,
                                     const mihs_batched_tuning_t* tuning, const double* cost,
                                     int32_t* team0, int32_t* tsize, int32_t* tcg) {
  if (num_cu < 1 || !n || !d || nprob < 1 || nlam < 1 || !tuning || !team0 || !tsize || !tcg)
    return MIHS_ERR_INVALID;
  if (!mihs::block_tuning_valid(*tuning)) return MIHS_ERR_INVALID;
  std::vector<mihs::BlockEntryDesc> ents;
  for (int64_t p = 0; p < nprob; ++p) {
    if (n[p] < 1 || d[p] < 1 || n[p] < d[p]) return MIHS_ERR_INVALID;
    for (int64_t g0 = 0; g0 < nlam; g0 += 16) {
      mihs::BlockEntryDesc e;
      memset(&e, 0, sizeof(e));
      e.n = n[p];
      e.d = d[p];
      e.ncols = (int)((nlam - g0) < 16 ? (nlam - g0) : 16);
      e.sa_group = p;
      ents.push_back(e);
    }
  }
  const int64_t count = (int64_t)ents.size();
  std::vector<double> c;
  if (cost) c.assign(cost, cost + count);
  mihs::Schedule S;
  const int rc = mihs::make_schedule(ents.data(), count, num_cu, *tuning, cost ? &c : nullptr, &S);
  if (rc) return rc;
  for (int64_t i = 0; i < count; ++i) {
    team0[i] = S.team0[i];
    tsize[i] = S.tsize[i];
    tcg[i] = S.tcg[i];
  }
  return MIHS_OK;
}

extern "C" void mihs_batched_default_tuning(mihs_batched_tuning_t* t) {
  if (!t) return;
  t->cg_cols = 32;
  t->a_dma = 1;
  t->inner_weight = 100.0;
  t->measured = 0;
  t->exact = 0;
}

// ---- tuning cache file ----------------------------------------------------
// One JSON document:
//   {"format": "libmihs-batched-tuning", "version": 1, "arch": "gfx950",
//    "num_cu": 256, "entries": [{"key": "<16 hex digits>", "cg_cols": 32,
//    "a_dma": 1, "inner_weight": 100, "measured": 1, "exact": 0,
//    "cost": [..]}, ...]}
// The reader accepts exactly this shape (any whitespace, keys in any order).
namespace {

struct Reader {
  const char* p;
  const char* end;
  bool ok = true;
  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
  }
  bool lit(char c) {
    ws();
    if (p < end && *p == c) {
      ++p;
      return true;
    }
    return false;
  }
  void expect(char c) {
    if (!lit(c)) ok = false;
  }
  std::string str() {
    std::string out;
    ws();
    if (p >= end || *p != '"') {
      ok = false;
      return out;
    }
    ++p;
    while (p < end && *p != '"') {
      if (*p == '\\' || (unsigned char)*p < 0x20) {  // no escapes in this format
        ok = false;
        return out;
      }
      out.push_back(*p++);
    }
    if (p >= end) {
      ok = false;
      return out;
    }
    ++p;
    return out;
  }
  double num() {
    ws();
    char buf[64];
    size_t k = 0;
    while (p < end && k + 1 < sizeof(buf) && (strchr("+-.eE0123456789", *p) != nullptr))
      buf[k++] = *p++;
    buf[k] = 0;
    char* q = nullptr;
    errno = 0;
    const double v = strtod(buf, &q);
    if (k == 0 || q != buf + k || errno != 0 || !std::isfinite(v)) ok = false;
    return v;
  }
};

bool parse_entry(Reader& r, mihs_tuned_set* e) {
  int seen = 0;
  r.expect('{');
  if (!r.ok) return false;
  if (r.lit('}')) return false;
  do {
    const std::string k = r.str();
    r.expect(':');
    if (!r.ok) return false;
    if (k == "key") {
      const std::string v = r.str();
      if (v.size() != 16) return false;
      char* q = nullptr;
      e->key = strtoull(v.c_str(), &q, 16);
      if (q != v.c_str() + 16) return false;
      seen |= 1;
    } else if (k == "cg_cols") {
      e->tuning.cg_cols = (int32_t)r.num();
      seen |= 2;
    } else if (k == "a_dma") {
      e->tuning.a_dma = (int32_t)r.num();
      seen |= 4;
    } else if (k == "inner_weight") {
      e->tuning.inner_weight = r.num();
      seen |= 8;
    } else if (k == "measured") {
      e->tuning.measured = (int32_t)r.num();
      seen |= 16;
    } else if (k == "exact") {
      e->tuning.exact = (int32_t)r.num();
      seen |= 32;
    } else if (k == "cost") {
      r.expect('[');
      e->cost.clear();
      if (!r.lit(']')) {
        do {
          e->cost.push_back(r.num());
        } while (r.ok && r.lit(','));
        r.expect(']');
      }
      seen |= 64;
    } else {
      return false;
    }
  } while (r.ok && r.lit(','));
  r.expect('}');
  return r.ok && seen == 127 && mihs::block_tuning_valid(e->tuning);
}

}  // namespace

extern "C" int mihs_tuning_cache_save(mihs_handle_t handle, const char* path) {
  if (!handle || !path) return MIHS_ERR_INVALID;
  std::vector<mihs_tuned_set> sets;
  {
    std::lock_guard<std::mutex> lock(handle->tune_mu);
    sets = handle->tuned;
  }
  std::string out = "{\"format\": \"libmihs-batched-tuning\", \"version\": 1, \"arch\": \"";
  for (const char* c = handle->arch; *c; ++c)
    if (*c != '"' && *c != '\\' && (unsigned char)*c >= 0x20) out.push_back(*c);
  char buf[256];
  snprintf(buf, sizeof(buf), "\", \"num_cu\": %d, \"entries\": [", handle->num_cu);
  out += buf;
  for (size_t i = 0; i < sets.size(); ++i) {
    const mihs_tuned_set& t = sets[i];
    snprintf(buf, sizeof(buf),
             "%s\n  {\"key\": \"%016llx\", \"cg_cols\": %d, \"a_dma\": %d, \"inner_weight\": "
             "%.17g, \"measured\": %d, \"exact\": %d, \"cost\": [",
             i ? "," : "", (unsigned long long)t.key, t.tuning.cg_cols, t.tuning.a_dma,
             t.tuning.inner_weight, t.tuning.measured, t.tuning.exact);
    out += buf;
    for (size_t j = 0; j < t.cost.size(); ++j) {
      snprintf(buf, sizeof(buf), "%s%.17g", j ? ", " : "", t.cost[j]);
      out += buf;
    }
    out += "]}";
  }
  out += "\n]}\n";
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return MIHS_ERR_INVALID;
  const bool wrote = fwrite(out.data(), 1, out.size(), f) == out.size();
  if (fclose(f) != 0 || !wrote || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return MIHS_ERR_INVALID;
  }
  return MIHS_OK;
}

extern "C" int mihs_tuning_cache_load(mihs_handle_t handle, const char* path, int32_t* loaded) {
  if (!handle || !path) return MIHS_ERR_INVALID;
  if (loaded) *loaded = 0;
  FILE* f = fopen(path, "rb");
  if (!f) return MIHS_ERR_INVALID;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0) {
    text.append(buf, got);
    if (text.size() > ((size_t)64 << 20)) break;  // not a tuning cache
  }
  fclose(f);
  Reader r{text.data(), text.data() + text.size()};
  std::string arch;
  int num_cu = -1;
  bool fmt = false;
  std::vector<mihs_tuned_set> sets;
  r.expect('{');
  if (r.ok && !r.lit('}')) {
    do {
      const std::string k = r.str();
      r.expect(':');
      if (!r.ok) break;
      if (k == "format") {
        fmt = r.str() == "libmihs-batched-tuning";
      } else if (k == "version") {
        if (r.num() != 1.0) r.ok = false;
      } else if (k == "arch") {
        arch = r.str();
      } else if (k == "num_cu") {
        num_cu = (int)r.num();
      } else if (k == "entries") {
        r.expect('[');
        if (r.ok && !r.lit(']')) {
          do {
            mihs_tuned_set e;
            if (!parse_entry(r, &e)) r.ok = false;
            else sets.push_back(e);
          } while (r.ok && r.lit(','));
          r.expect(']');
        }
      } else {
        r.ok = false;
      }
    } while (r.ok && r.lit(','));
    r.expect('}');
  }
  r.ws();
  if (!r.ok || !fmt || r.p != r.end) return MIHS_ERR_INVALID;
  // shapes tuned on another device type or size do not apply here
  if (arch != handle->arch || num_cu != handle->num_cu) return MIHS_OK;
  std::lock_guard<std::mutex> lock(handle->tune_mu);
  for (const mihs_tuned_set& e : sets) {
    bool replaced = false;
    for (auto& t : handle->tuned)
      if (t.key == e.key) {
        t = e;
        replaced = true;
      }
    if (!replaced) handle->tuned.push_back(e);
  }
  if (loaded) *loaded = (int32_t)sets.size();
  return MIHS_OK;
}

extern "C" {

int mihs_set_row_weights(mihs_handle_t handle, const int32_t* weights) {
  if (!handle) return MIHS_ERR_INVALID;
  if (weights)
    for (int k = 0; k < mihs::kXcds; ++k)
      if (weights[k] < 1 || weights[k] > mihs::kRowWeightMax) return MIHS_ERR_INVALID;
  for (int k = 0; k < mihs::kXcds; ++k)
    handle->row_weight[k] = weights ? weights[k] : mihs::kRowWeightMax;
  return MIHS_OK;
}

int mihs_get_row_weights(mihs_handle_t handle, int32_t* weights) {
  if (!handle || !weights) return MIHS_ERR_INVALID;
  for (int k = 0; k < mihs::kXcds; ++k) weights[k] = handle->row_weight[k];
  return MIHS_OK;
}

int mihs_row_split(int64_t n, int32_t G, const int32_t* weights, int64_t* bounds) {
  if (n < 0 || G < 1 || !weights || !bounds) return MIHS_ERR_INVALID;
  for (int k = 0; k < mihs::kXcds; ++k)
    if (weights[k] < 1 || weights[k] > mihs::kRowWeightMax) return MIHS_ERR_INVALID;
  for (int v = 0; v <= G; ++v) bounds[v] = mihs::row_split_bound(n, G, weights, v);
  return MIHS_OK;
}

int mihs_momentum_cor4(double sd, int64_t m, double* alpha, double* beta) {
  if (!alpha || !beta || !isfinite(sd) || m < 1) return MIHS_ERR_INVALID;
  const double b = sd / (double)m;
  if (!(b > 0.0) || !(b < 1.0)) return MIHS_ERR_INVALID;
  *beta = b;
  *alpha = (1.0 - b) * (1.0 - b);
  return MIHS_OK;
}

int mihs_momentum_thm1(double eps, double* alpha, double* beta) {
  if (!alpha || !beta || !(eps > 0.0) || !(eps < 1.0)) return MIHS_ERR_INVALID;
  // The eigenvalues of the preconditioned Hessian lie in [1/(1+eps), 1/(1-eps)];
  // the optimal heavy-ball rate for that interval is
  // (sqrt(1+eps) - sqrt(1-eps)) / (sqrt(1+eps) + sqrt(1-eps)) = eps / (1 + sqrt(1-eps^2)),
  // reached with step 4 (1-eps^2) / (sqrt(1+eps) + sqrt(1-eps))^2.
  const double up = sqrt(1.0 + eps), lo = sqrt(1.0 - eps);
  const double rate = (up - lo) / (up + lo);
  *beta = rate * rate;
  *alpha = 4.0 * (1.0 - eps) * (1.0 + eps) / ((up + lo) * (up + lo));
  return MIHS_OK;
}

int mihs_lambda_from_log(double log_lambda, double* lambda) {
  if (!lambda) return MIHS_ERR_INVALID;
  const double v = exp(log_lambda);
  if (!(v > 0.0) || !isfinite(v)) return MIHS_ERR_INVALID;
  *lambda = v;
  return MIHS_OK;
}

}  // extern "C"

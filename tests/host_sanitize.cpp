// Host-side checks of libtuckvsie built with AddressSanitizer and
// UndefinedBehaviorSanitizer on its host code (device code unchanged), run
// without a GPU: plan packing for many shapes and both precisions, arena and
// workspace sizing for every launch configuration a plan accepts, factor
// export round trips, compression and assembly sizing, argument errors.
// Any out-of-bounds access, leak or undefined operation on these host paths
// aborts the program; a wrong result returns 1.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "tuckvsie.h"

namespace {

int failures = 0;

#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #c, \
                   tv_last_error());                                     \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

struct Factors {
  std::vector<int32_t> ranks;
  std::vector<double> cores, u1, u2, u3;
};

Factors random_factors(const tv_grid& g, int rmax, unsigned seed) {
  std::mt19937 rng(seed);
  std::normal_distribution<double> nd;
  Factors f;
  const int64_t K = (int64_t)g.q * g.m;
  const int dims[3] = {g.n1, g.n2, g.n3};
  for (int64_t t = 0; t < K; ++t)
    for (int d = 0; d < 3; ++d) {
      const int cap = std::min(rmax, dims[d]);
      f.ranks.push_back(1 + (int)(rng() % (unsigned)cap));
    }
  for (int64_t t = 0; t < K; ++t) {
    const int32_t* r = &f.ranks[3 * t];
    for (int64_t i = 0; i < 2LL * r[0] * r[1] * r[2]; ++i) f.cores.push_back(nd(rng));
    for (int64_t i = 0; i < 2LL * g.n1 * r[0]; ++i) f.u1.push_back(nd(rng));
    for (int64_t i = 0; i < 2LL * g.n2 * r[1]; ++i) f.u2.push_back(nd(rng));
    for (int64_t i = 0; i < 2LL * g.n3 * r[2]; ++i) f.u3.push_back(nd(rng));
  }
  return f;
}

void check_plan(const tv_grid& g, int rmax, unsigned seed, tv_precision prec) {
  Factors f = random_factors(g, rmax, seed);
  tv_plan p = nullptr;
  CHECK(tv_plan_from_factors(&g, f.ranks.data(), f.cores.data(), f.u1.data(), f.u2.data(),
                             f.u3.data(), prec, &p) == TV_OK);
  if (!p) return;
  size_t need = 0;
  CHECK(tv_plan_required_bytes(p, &need) == TV_OK && need > 0);
  tv_plan_info_t info;
  CHECK(tv_plan_info(p, &info) == TV_OK);
  CHECK(info.device_bytes == need);
  CHECK(info.flops_matvec > 0 && info.flops_rmatvec > info.flops_matvec);

  // export round trip: the FP64 factors as given
  std::vector<int32_t> r2(f.ranks.size());
  std::vector<double> c2(f.cores.size()), a2(f.u1.size()), b2(f.u2.size()), d2(f.u3.size());
  CHECK(tv_plan_export_factors(p, r2.data(), c2.data(), a2.data(), b2.data(), d2.data()) ==
        TV_OK);
  CHECK(r2 == f.ranks);
  for (size_t i = 0; i < c2.size(); ++i) CHECK(c2[i] == f.cores[i]);
  for (size_t i = 0; i < a2.size(); ++i) CHECK(a2[i] == f.u1[i]);
  for (size_t i = 0; i < b2.size(); ++i) CHECK(b2[i] == f.u2[i]);
  for (size_t i = 0; i < d2.size(); ++i) CHECK(d2[i] == f.u3[i]);

  // every launch configuration the products accept, and the workspace each needs
  for (int op = 0; op < 2; ++op) {
    size_t ws = 0;
    CHECK(tv_workspace_bytes(p, op, 1, &ws) == TV_OK);
    for (int slab : {0, 1, 3, g.n3}) {
      for (int nbw : {1, 2, 4}) {
        for (int splits : {1, 2, 5, 64}) {
          for (int order : {0, 1}) {
            tv_launch_config c = {1, 0, splits, 0, slab, nbw, order};
            const tv_status s = tv_plan_configure(p, op, &c);
            if (s == TV_OK) {
              CHECK(tv_workspace_bytes(p, op, 3, &ws) == TV_OK);
              tv_plan_info_t i2;
              CHECK(tv_plan_info(p, &i2) == TV_OK && i2.kernel[op] == 2);
            } else {
              CHECK(s == TV_ERR_INVALID_ARG || s == TV_ERR_NOT_SUPPORTED);
            }
          }
        }
      }
    }
    for (int t2 : {0, 2, 8, 32}) {
      for (int cap : {2, 3, 8}) {
        tv_launch_config c = {0, t2, 2, cap, 0, 0, 0};
        const tv_status s = tv_plan_configure(p, op, &c);
        CHECK(s == TV_OK || s == TV_ERR_INVALID_ARG || s == TV_ERR_NOT_SUPPORTED);
        CHECK(tv_workspace_bytes(p, op, 1, &ws) == TV_OK);
      }
    }
  }
  // refusals before any device work
  CHECK(tv_plan_bind_arena(p, nullptr, need, nullptr) == TV_ERR_INVALID_ARG);
  CHECK(tv_plan_bind_arena(p, (void*)(uintptr_t)(1 << 20), need - 1, nullptr) ==
        TV_ERR_WORKSPACE);
  CHECK(tv_matvec(p, (void*)16, g.m, 1, (void*)4096, (int64_t)g.q * g.n1 * g.n2 * g.n3,
                  nullptr, 0, nullptr) == TV_ERR_INVALID_ARG);   // not bound
  CHECK(tv_plan_destroy(p) == TV_OK);
}

void check_errors() {
  tv_grid g = {8, 6, 5, 3, 2};
  Factors f = random_factors(g, 4, 7);
  tv_plan p = nullptr;
  std::vector<int32_t> bad = f.ranks;
  bad[0] = 0;
  CHECK(tv_plan_from_factors(&g, bad.data(), f.cores.data(), f.u1.data(), f.u2.data(),
                             f.u3.data(), TV_PREC_FP32, &p) == TV_ERR_RANK);
  bad[0] = TV_MAX_RANK + 1;
  CHECK(tv_plan_from_factors(&g, bad.data(), f.cores.data(), f.u1.data(), f.u2.data(),
                             f.u3.data(), TV_PREC_FP32, &p) == TV_ERR_RANK);
  std::vector<double> nan_core = f.cores;
  nan_core[3] = std::nan("");
  CHECK(tv_plan_from_factors(&g, f.ranks.data(), nan_core.data(), f.u1.data(), f.u2.data(),
                             f.u3.data(), TV_PREC_FP32, &p) == TV_ERR_NUMERIC);
  tv_grid z = g;
  z.n1 = 0;
  CHECK(tv_plan_from_factors(&z, f.ranks.data(), f.cores.data(), f.u1.data(), f.u2.data(),
                             f.u3.data(), TV_PREC_FP32, &p) != TV_OK);
  CHECK(tv_plan_from_factors(&g, f.ranks.data(), f.cores.data(), f.u1.data(), f.u2.data(),
                             f.u3.data(), (tv_precision)7, &p) == TV_ERR_INVALID_ARG);
  CHECK(tv_plan_destroy(nullptr) == TV_OK);
  size_t b = 0;
  CHECK(tv_workspace_bytes(nullptr, 0, 1, &b) == TV_ERR_INVALID_ARG);
  for (int s = 0; s >= -8; --s) CHECK(std::strlen(tv_status_string((tv_status)s)) > 0);
  CHECK(std::strlen(tv_status_string((tv_status)-99)) > 0);

  // compression and assembly sizing
  tv_plan h = nullptr;
  CHECK(tv_compress_begin(&g, 1e-3, 1, 4, TV_PREC_FP32, &h) == TV_OK);
  size_t w2 = 0, w4 = 0;
  CHECK(tv_compress_workspace_bytes(h, 2, &w2) == TV_OK);
  CHECK(tv_compress_workspace_bytes(h, 4, &w4) == TV_OK && w4 > w2);
  CHECK(tv_compress_append(h, (void*)(uintptr_t)(1 << 20), 2, nullptr, w2, nullptr) !=
        TV_OK);
  CHECK(tv_plan_finalize(h, nullptr) != TV_OK);   // no column appended
  CHECK(tv_plan_destroy(h) == TV_OK);
  CHECK(tv_compress_begin(&g, -1.0, 1, 0, TV_PREC_FP32, &h) == TV_ERR_INVALID_ARG);
  tv_grid ga = {10, 8, 12, 3, 40};
  size_t a4 = 0, a2 = 0;
  CHECK(tv_aca_assemble_workspace_bytes(&ga, 4, 1e-3, 1e-3, 1, 0, TV_PREC_FP32, &a4) == TV_OK);
  CHECK(tv_aca_assemble_workspace_bytes(&ga, 4, 1e-3, 1e-3, 1, 2, TV_PREC_FP32, &a2) == TV_OK);
  CHECK(a2 < a4);
}

}  // namespace

int main() {
  const struct { tv_grid g; int rmax; } cases[] = {
      {{20, 13, 7, 2, 5}, 5},   {{64, 32, 24, 3, 9}, 12}, {{96, 40, 33, 3, 6}, 20},
      {{130, 24, 10, 1, 7}, 32}, {{17, 9, 5, 12, 1}, 4},  {{33, 9, 7, 2, 4}, 7},
      {{1, 1, 1, 3, 2}, 1},      {{256, 16, 9, 3, 4}, 10},
  };
  unsigned seed = 1;
  for (const auto& c : cases)
    for (tv_precision prec : {TV_PREC_FP32, TV_PREC_BF16X3}) check_plan(c.g, c.rmax, seed++, prec);
  check_errors();
  std::printf("host sanitizer checks: %d failures\n", failures);
  return failures ? 1 : 0;
}

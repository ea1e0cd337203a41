// Autotuner for the fused single-vector kernels: per plan and direction it
// times every workgroup column tile (t2 x t3), column split count and (for
// the adjoint) row-block cap per wave on the device with HIP events and keeps
// the fastest; results are cached in a small JSON file keyed by device, grid,
// precision and a hash of the ranks.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "tv_internal.h"

namespace tv {

static std::string plan_key(const tv_plan_s* p, int op) {
  hipDeviceProp_t prop;
  int dev = 0;
  std::string arch = "gpu";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the ranks
  for (int32_t r : p->ranks) {
    h ^= (uint32_t)r;
    h *= 1099511628211ull;
  }
  char buf[256];
  snprintf(buf, sizeof buf, "k4|%s|%dx%dx%d|q%d|m%lld|p%d|r%016llx|op%d", arch.c_str(), p->grid.n1,
           p->grid.n2, p->grid.n3, p->grid.q, (long long)p->grid.m, (int)p->precision,
           (unsigned long long)h, op);
  for (char* c = buf; *c; ++c)
    if (*c == '"' || *c == '\\') *c = '_';
  return buf;
}

struct TuneChoice {
  int t2, split, cap;
};

// The cache is a flat JSON object {"key": [t2, split, cap], ...}.
static std::map<std::string, TuneChoice> read_cache(const char* path) {
  std::map<std::string, TuneChoice> out;
  if (!path) return out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t pos = 0;
  for (;;) {
    const size_t q0 = s.find('"', pos);
    if (q0 == std::string::npos) break;
    const size_t q1 = s.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    const size_t b0 = s.find('[', q1), b1 = s.find(']', q1);
    if (b0 == std::string::npos || b1 == std::string::npos) break;
    int t2 = 0, sp = 0, cap = 0;
    if (sscanf(s.c_str() + b0 + 1, "%d , %d , %d", &t2, &sp, &cap) == 3)
      out[s.substr(q0 + 1, q1 - q0 - 1)] = {t2, sp, cap};
    pos = b1 + 1;
  }
  return out;
}

static void write_cache(const char* path, const std::map<std::string, TuneChoice>& m) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m) {
      f << "  \"" << kv.first << "\": [" << kv.second.t2 << ", " << kv.second.split << ", "
        << kv.second.cap << "]" << (++i < m.size() ? ",\n" : "\n");
    }
    f << "}\n";
  }
  std::rename(tmp.c_str(), path);
}

static tv_status apply_config(tv_plan_s* p, int op, int t2, int split, int cap) {
  if (op == 0 && cap != nb_cap(p, 0)) return set_error(TV_ERR_INVALID_ARG, "forward cap");
  if (op == 1 && cap != 2 && cap != 3) return set_error(TV_ERR_INVALID_ARG, "adjoint cap");
  Tiling T;
  tv_status s = make_tiling(p->grid, t2, cap, &T);
  if (s != TV_OK) return s;
  // the packed U1 rows hold nbt_pack blocks: no tiling may read past them
  if (T.nbt > p->nbt_pack) return set_error(TV_ERR_NOT_SUPPORTED, "tiling wider than the pack");
  if (fused_lds_bytes(p, T, op == 1) > 160 * 1024)
    return set_error(TV_ERR_NOT_SUPPORTED, "tile too large for LDS");
  if ((s = set_split(p, op, split)) != TV_OK) return s;
  if (op == 0) {
    p->tiling = T;
  } else {
    p->tiling_a = T;
    p->nbcap_a = cap;
  }
  return TV_OK;
}

}  // namespace tv

using namespace tv;

extern "C" tv_status tv_autotune(tv_plan p, int32_t op, const char* cache_path, void* stream) {
  clear_error();
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  if (!p->finalized) return set_error(TV_ERR_INVALID_ARG, "plan is not finalized");
  if (op < 0 || op > 2) return set_error(TV_ERR_INVALID_ARG, "op must be 0, 1 or 2");
  hipStream_t st = (hipStream_t)stream;
  auto cache = read_cache(cache_path);
  const tv_grid& g = p->grid;
  const int64_t rows = (int64_t)g.q * g.n1 * g.n2 * g.n3;
  bool dirty = false;
  for (int o = 0; o < 2; ++o) {
    if (op != 2 && op != o) continue;
    const std::string key = plan_key(p, o);
    auto it = cache.find(key);
    if (it != cache.end() &&
        apply_config(p, o, it->second.t2, it->second.split, it->second.cap) == TV_OK)
      continue;
    // candidates: (cap, t2) pairs, then column splits
    std::vector<std::pair<int, int>> shapes;
    std::vector<int> splits;
    int prev_nb = -1, prev_wm = -1;
    for (int cap : (o == 0 ? std::vector<int>{nb_cap(p, 0)} : std::vector<int>{2, 3})) {
      Tiling T0;
      tv_status s = make_tiling(g, 0, cap, &T0);
      if (s != TV_OK) return s;
      if (T0.nb == prev_nb && T0.wm == prev_wm) continue;  // same tiling as the last cap
      prev_nb = T0.nb;
      prev_wm = T0.wm;
      for (int t2 = T0.nwg; t2 >= 2; t2 /= 2) shapes.push_back({cap, t2});
    }
    const int smax = o == 0 ? 16 : 64;
    for (int sp = 1; sp <= smax && sp <= g.m; sp *= 2) {
      if (o == 0 && sp > 1 && (double)sp * rows * 8 > 2e9) break;  // forward partials
      splits.push_back(sp);
    }
    // buffers sized for the largest candidate
    size_t wsb = 16;
    for (const auto& sh : shapes) {
      Tiling T;
      if (make_tiling(g, sh.second, sh.first, &T) != TV_OK) continue;
      const size_t b = o == 0 ? (size_t)8 * splits.back() * rows : (size_t)8 * g.q * T.tiles * g.m;
      wsb = std::max(wsb, b);
    }
    void *x = nullptr, *y = nullptr, *ws = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&x, (size_t)8 * g.m);
    if (e == hipSuccess) e = hipMalloc(&y, (size_t)8 * rows);
    if (e == hipSuccess) e = hipMalloc(&ws, wsb);
    if (e == hipSuccess) e = hipMemsetAsync(x, 0, (size_t)8 * g.m, st);
    if (e == hipSuccess) e = hipMemsetAsync(y, 0, (size_t)8 * rows, st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int keep_t2 = o == 0 ? p->tiling.t2 : p->tiling_a.t2;
    const int keep_sp = o == 0 ? p->split_f : p->split_a;
    const int keep_cap = nb_cap(p, o);
    float best = -1.f;
    int best_t2 = keep_t2, best_sp = keep_sp, best_cap = keep_cap;
    for (size_t a = 0; e == hipSuccess && a < shapes.size(); ++a)
      for (size_t b = 0; e == hipSuccess && b < splits.size(); ++b) {
        if (apply_config(p, o, shapes[a].second, splits[b], shapes[a].first) != TV_OK) continue;
        auto run = [&]() {
          return o == 0 ? tv_matvec(p, x, g.m, 1, y, rows, ws, wsb, stream)
                        : tv_rmatvec(p, y, rows, 1, x, g.m, ws, wsb, stream);
        };
        bool ok = true;
        for (int w = 0; w < 2 && ok; ++w) ok = run() == TV_OK;
        if (!ok) continue;
        e = hipEventRecord(e0, st);
        for (int r = 0; r < 5 && ok && e == hipSuccess; ++r) ok = run() == TV_OK;
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (ok && e == hipSuccess && (best < 0.f || ms < best)) {
          best = ms;
          best_t2 = shapes[a].second;
          best_sp = splits[b];
          best_cap = shapes[a].first;
        }
      }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(x);
    hipFree(y);
    hipFree(ws);
    if (e != hipSuccess) {
      apply_config(p, o, keep_t2, keep_sp, keep_cap);
      return hip_error(e, "tv_autotune");
    }
    tv_status s = apply_config(p, o, best_t2, best_sp, best_cap);
    if (s != TV_OK) return s;
    cache[key] = {best_t2, best_sp, best_cap};
    dirty = true;
  }
  if (dirty) write_cache(cache_path, cache);
  clear_error();
  return TV_OK;
}

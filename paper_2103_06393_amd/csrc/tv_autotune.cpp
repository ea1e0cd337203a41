// Autotuner for the single-vector products: per plan and direction it times
// every workgroup column tile (t2 x t3), column split count and (for the
// adjoint) row-block cap per wave of the fused kernels, and for the forward
// the decompress-then-GEMM path over its slab sizes, GEMM tiles and k-step
// splits, on the device with HIP events, and keeps the fastest; results are
// cached in a small JSON file keyed by device, grid, precision and a hash of
// the ranks.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "tv_internal.h"

namespace tv {

static std::string plan_key(const tv_plan_s* p, int op) {
  const std::string arch = device_arch();
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the ranks
  for (int32_t r : p->ranks) {
    h ^= (uint32_t)r;
    h *= 1099511628211ull;
  }
  char buf[256];
  snprintf(buf, sizeof buf, "k9|%s|%dx%dx%d|q%d|m%lld|p%d|r%016llx|op%d", arch.c_str(), p->grid.n1,
           p->grid.n2, p->grid.n3, p->grid.q, (long long)p->grid.m, (int)p->precision,
           (unsigned long long)h, op);
  for (char* c = buf; *c; ++c)
    if (*c == '"' || *c == '\\') *c = '_';
  return buf;
}

// The cache is a flat JSON object {"key": [int, ...], ...}: plan entries
// hold [path, t2, split, cap, slab, nbw, order], batch entries [tsplit,
// workgroups per CU].
std::map<std::string, std::vector<int>> read_tune_cache(const char* path) {
  std::map<std::string, std::vector<int>> out;
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
    std::vector<int> v;
    const char* c = s.c_str() + b0 + 1;
    const char* end = s.c_str() + b1;
    while (c < end) {
      char* nx = nullptr;
      const long x = strtol(c, &nx, 10);
      if (nx == c) {
        ++c;
        continue;
      }
      v.push_back((int)x);
      c = nx;
    }
    out[s.substr(q0 + 1, q1 - q0 - 1)] = v;
    pos = b1 + 1;
  }
  return out;
}

void write_tune_cache(const char* path, const std::map<std::string, std::vector<int>>& m) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m) {
      f << "  \"" << kv.first << "\": [";
      for (size_t j = 0; j < kv.second.size(); ++j) f << (j ? ", " : "") << kv.second[j];
      f << "]" << (++i < m.size() ? ",\n" : "\n");
    }
    f << "}\n";
  }
  std::rename(tmp.c_str(), path);
}

std::string device_arch() {
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    return prop.gcnArchName;
  return "gpu";
}

static std::vector<int> to_vec(const tv_launch_config& c) {
  return {c.path, c.tile_t2, c.splits, c.row_cap, c.slab_i3, c.gemm_nbw, c.gemm_order};
}
static bool from_vec(const std::vector<int>& v, tv_launch_config* c) {
  if (v.size() != 7) return false;
  *c = tv_launch_config{v[0], v[1], v[2], v[3], v[4], v[5], v[6]};
  return true;
}

static tv_status apply_config(tv_plan_s* p, int op, const tv_launch_config& c) {
  if (c.path == 1) {
    if (!dtg_supported(p)) return set_error(TV_ERR_NOT_SUPPORTED, "plan has no GEMM operand");
    if (c.slab_i3 < 0) return set_error(TV_ERR_INVALID_ARG, "slab_i3 must be >= 0");
    const int slab = c.slab_i3 ? std::min(c.slab_i3, p->grid.n3) : p->grid.n3;
    // row_cap: 0 (the default tile) or 8 row blocks per wave, a workgroup over
    // all 512 voxel rows (BF16X3 plans with 2 n1 = 512, gemm_nbw 2)
    if (c.row_cap != 0 && c.row_cap != 8)
      return set_error(TV_ERR_INVALID_ARG, "the GEMM takes row_cap 0 or 8");
    if (c.row_cap == 8 && (p->precision != TV_PREC_BF16X3 || c.gemm_nbw != 2 ||
                           p->dtg_nbtp != 16))
      return set_error(TV_ERR_NOT_SUPPORTED,
                       "row_cap 8 needs a BF16X3 plan with 2 n1 = 512 and gemm_nbw 2");
    if (op == 1) {
      if (c.gemm_nbw != 2 && c.gemm_nbw != 4)
        return set_error(TV_ERR_INVALID_ARG, "the adjoint GEMM takes gemm_nbw 2 or 4");
      if (c.splits < 1 || c.splits > 64)
        return set_error(TV_ERR_INVALID_ARG, "the adjoint GEMM takes splits 1..64");
      if (c.gemm_order != 0 && c.gemm_order != 1)
        return set_error(TV_ERR_INVALID_ARG, "the adjoint GEMM takes gemm_order 0 or 1");
      p->dtg_split_a = c.splits;
      p->dtg_nbw_a = c.gemm_nbw;
      p->dtg_s3_a = slab;
      p->dtg_order_a = c.gemm_order;
      p->dtg_mbw[1] = c.row_cap;
      p->use_dtg[1] = true;
      return TV_OK;
    }
    if (c.gemm_nbw != 2 && c.gemm_nbw != 4)
      return set_error(TV_ERR_INVALID_ARG, "the GEMM takes gemm_nbw 2 or 4");
    if (c.splits < 1 || c.splits > 64) return set_error(TV_ERR_INVALID_ARG, "GEMM splits");
    p->dtg_nbw = c.gemm_nbw;
    p->dtg_split = c.splits;
    p->dtg_s3 = slab;
    p->dtg_mbw[0] = c.row_cap;
    p->use_dtg[0] = true;
    return TV_OK;
  }
  if (c.path != 0) return set_error(TV_ERR_INVALID_ARG, "path must be 0 or 1");
  const int t2 = c.tile_t2, split = c.splits, cap = c.row_cap;
  if (op == 0 && cap != nb_cap(p, 0)) return set_error(TV_ERR_INVALID_ARG, "forward cap");
  if (op == 1 && cap != 2 && cap != 3) return set_error(TV_ERR_INVALID_ARG, "adjoint cap");
  if (split < 1) return set_error(TV_ERR_INVALID_ARG, "splits must be >= 1");
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
  p->use_dtg[op] = false;
  return TV_OK;
}

static tv_launch_config current_config(const tv_plan_s* p, int op) {
  tv_launch_config c{};
  if (p->use_dtg[op]) {
    c.path = 1;
    c.splits = op == 0 ? p->dtg_split : p->dtg_split_a;
    c.slab_i3 = op == 0 ? p->dtg_s3 : p->dtg_s3_a;
    c.gemm_nbw = op == 0 ? p->dtg_nbw : p->dtg_nbw_a;
    c.gemm_order = op == 0 ? 0 : p->dtg_order_a;
    c.row_cap = p->dtg_mbw[op];
    return c;
  }
  c.tile_t2 = op == 0 ? p->tiling.t2 : p->tiling_a.t2;
  c.splits = op == 0 ? p->split_f : p->split_a;
  c.row_cap = nb_cap(p, op);
  return c;
}

}  // namespace tv

using namespace tv;

extern "C" tv_status tv_plan_configure(tv_plan p, int32_t op, const tv_launch_config* cfg) {
  clear_error();
  if (!p || !cfg) return set_error(TV_ERR_INVALID_ARG, "plan and cfg must be non-NULL");
  if (!p->finalized) return set_error(TV_ERR_INVALID_ARG, "plan is not finalized");
  if (op != 0 && op != 1) return set_error(TV_ERR_INVALID_ARG, "op must be 0 or 1");
  const tv_launch_config keep = current_config(p, op);
  tv_status s = apply_config(p, op, *cfg);
  if (s != TV_OK) apply_config(p, op, keep);  // keeps the error message of the refusal
  return s;
}

extern "C" tv_status tv_autotune(tv_plan p, int32_t op, const char* cache_path, void* stream) {
  clear_error();
  if (!p) return set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  if (!p->finalized) return set_error(TV_ERR_INVALID_ARG, "plan is not finalized");
  if (!p->bound) return set_error(TV_ERR_INVALID_ARG, "plan has no device arena (tv_plan_bind_arena)");
  if (op < 0 || op > 2) return set_error(TV_ERR_INVALID_ARG, "op must be 0, 1 or 2");
  hipStream_t st = (hipStream_t)stream;
  auto cache = read_tune_cache(cache_path);
  const tv_grid& g = p->grid;
  const int64_t rows = (int64_t)g.q * g.n1 * g.n2 * g.n3;
  const bool bf = p->precision == TV_PREC_BF16X3;
  bool dirty = false;
  for (int o = 0; o < 2; ++o) {
    if (op != 2 && op != o) continue;
    const std::string key = plan_key(p, o);
    auto it = cache.find(key);
    tv_launch_config cached{};
    if (it != cache.end() && from_vec(it->second, &cached) && apply_config(p, o, cached) == TV_OK)
      continue;
    std::vector<tv_launch_config> cands;
    // fused kernels: (cap, t2) pairs times column splits
    std::vector<int> splits;
    const int smax = o == 0 ? 16 : 64;
    for (int sp = 1; sp <= smax && sp <= g.m; sp *= 2) {
      if (o == 0 && sp > 1 && (double)sp * rows * 8 > 2e9) break;  // forward partials
      splits.push_back(sp);
    }
    int prev_nb = -1, prev_wm = -1;
    for (int cap : (o == 0 ? std::vector<int>{nb_cap(p, 0)} : std::vector<int>{2, 3})) {
      Tiling T0;
      tv_status s = make_tiling(g, 0, cap, &T0);
      if (s != TV_OK) return s;
      if (T0.nb == prev_nb && T0.wm == prev_wm) continue;  // same tiling as the last cap
      prev_nb = T0.nb;
      prev_wm = T0.wm;
      for (int t2 = T0.nwg; t2 >= 2; t2 /= 2)
        for (int sp : splits) {
          tv_launch_config c{};
          c.tile_t2 = t2;
          c.splits = sp;
          c.row_cap = cap;
          cands.push_back(c);
        }
    }
    // decompress-then-GEMM: slabs of B within 16 GiB; forward GEMM tiles and
    // k-step splits while the launch has fewer than 1024 workgroups
    if (dtg_supported(p)) {
      for (int slab = g.n3; slab >= 1; slab = (slab + 1) / 2) {
        std::vector<int> nbws = o == 1 ? std::vector<int>{2} : std::vector<int>{2, 4};
        for (int nbw : nbws) {
          tv_launch_config c{};
          c.path = 1;
          c.slab_i3 = slab;
          c.gemm_nbw = nbw;
          c.splits = 1;
          const tv_launch_config keep = current_config(p, o);
          if (apply_config(p, o, c) != TV_OK) continue;
          const size_t need = dtg_workspace_bytes(p, o);
          apply_config(p, o, keep);
          if (need > ((size_t)16 << 30)) continue;
          if (o == 1) {
            // the column GEMM: both tiles and workgroup orders, every
            // distinct column split count (as launched: at least the
            // accumulation-chain minimum) up to the fewest giving 4096
            // workgroups (small grids can win with fewer workgroups than
            // CUs: shorter partial sums), the partials of Z within 4 GiB
            // where that allows
            const int nslabs = (g.n3 + slab - 1) / slab;
            for (int cnbw : {2, 4}) {
              const int64_t tiles = dtg_colgemm_tiles(p, cnbw);
              std::vector<int> sps;
              int last = 0;
              for (int sp = 1; sp <= 64; sp *= 2) {
                const int keep_split = p->dtg_split_a;
                p->dtg_split_a = sp;
                const int eff = dtg_colgemm_splits(p, std::min(slab, g.n3));
                p->dtg_split_a = keep_split;
                if (eff == last) continue;
                if (!sps.empty() && (double)nslabs * eff * p->dtg_rows * g.n1 * 8 >
                                        4.0 * (1u << 30))
                  break;
                sps.push_back(sp);
                last = eff;
                if (tiles * eff >= 4096) break;
              }
              if (sps.empty()) sps.push_back(1);
              const bool full_m = bf && cnbw == 2 && p->dtg_nbtp == 16;
              for (int sp : sps)
                for (int order : {0, 1})
                  for (int rc : {0, 8}) {
                    if (rc == 8 && !full_m) continue;
                    tv_launch_config cc = c;
                    cc.gemm_nbw = cnbw;
                    cc.splits = sp;
                    cc.gemm_order = order;
                    cc.row_cap = rc;
                    cands.push_back(cc);
                  }
            }
            continue;
          }
          const int64_t tiles = dtg_launch_tiles(p, slab, nbw);
          for (int sp = 1; sp <= 16; sp *= 2) {
            if (sp > 1 && tiles * (sp / 2) >= 1024) break;
            if (sp > 1 && (double)sp * rows * 8 > 2e9) break;
            c.splits = sp;
            c.row_cap = 0;
            cands.push_back(c);
            if (bf && nbw == 2 && p->dtg_nbtp == 16) {
              c.row_cap = 8;
              cands.push_back(c);
              c.row_cap = 0;
            }
          }
        }
        if (slab <= 8 || (int64_t)g.n2 * slab < 4096) break;
      }
    }
    // buffers sized for the largest candidate
    size_t wsb = 16;
    {
      const tv_launch_config keep = current_config(p, o);
      for (const auto& c : cands) {
        if (apply_config(p, o, c) != TV_OK) continue;
        size_t b = 0;
        if (tv_workspace_bytes(p, o, 1, &b) == TV_OK) wsb = std::max(wsb, b);
      }
      apply_config(p, o, keep);
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
    const tv_launch_config keep = current_config(p, o);
    float best = -1.f;
    tv_launch_config best_c = keep;
    for (size_t a = 0; e == hipSuccess && a < cands.size(); ++a) {
      if (apply_config(p, o, cands[a]) != TV_OK) continue;
      auto run = [&]() {
        return o == 0 ? tv_matvec(p, x, g.m, 1, y, rows, ws, wsb, stream)
                      : tv_rmatvec(p, y, rows, 1, x, g.m, ws, wsb, stream);
      };
      // one warm-up call, one timed call; calls under 20 ms are timed again
      // over five repetitions
      bool ok = run() == TV_OK;
      if (!ok) continue;
      float ms = 0.f;
      for (int reps : {1, 5}) {
        e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && ok && e == hipSuccess; ++r) ok = run() == TV_OK;
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)reps;  // per call
        if (!ok || e != hipSuccess || ms > 20.f) break;
      }
      if (ok && e == hipSuccess && (best < 0.f || ms < best)) {
        best = ms;
        best_c = cands[a];
      }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(x);
    hipFree(y);
    hipFree(ws);
    if (e != hipSuccess) {
      apply_config(p, o, keep);
      return hip_error(e, "tv_autotune");
    }
    tv_status s = apply_config(p, o, best_c);
    if (s != TV_OK) return s;
    cache[key] = to_vec(best_c);
    dirty = true;
  }
  if (dirty) write_tune_cache(cache_path, cache);
  clear_error();
  return TV_OK;
}

// Whole-step entry points: the eager launch sequence of one step, its capture
// into a HIP graph, the plan's tunable launch shapes and their autotuner.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "plan.h"

using namespace lhf;

struct lhf_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const lhf_plan_s* plan = nullptr;
  uint64_t tuning_gen = 0;   // the plan's tuning generation at capture
};

namespace {

int32_t hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return LHF_OK;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return LHF_ERR_HIP;
}

int32_t check_args(const lhf_plan_s* p, const lhf_step_args* a) {
  if (!p || !a) { set_error("NULL plan or args"); return LHF_ERR_INVALID; }
  const bool refine = p->prec == LHF_PREC_MIXED && (a->heev_flags & LHF_HEEV_REFINE_FP64);
  if (refine && !(a->H_gen64 && a->S_gen64)) {
    set_error("refinement in a step needs the FP64 generator stacks H_gen64 and S_gen64");
    return LHF_ERR_INVALID;
  }
  if ((a->H_bar64 == nullptr) != (a->S_bar64 == nullptr)) {
    set_error("give both complex128 block stacks or neither");
    return LHF_ERR_INVALID;
  }
  if (!a->H_gen && !(refine && a->H_bar64)) {
    set_error("H_gen may be NULL only in a refined mixed step that fills the complex128 blocks");
    return LHF_ERR_INVALID;
  }
  if ((a->H_bar == nullptr) != (a->S_bar == nullptr) || (!a->H_bar && (a->H_gen || !a->H_bar64))) {
    set_error("H_bar and S_bar may be NULL only together, in a refined mixed step without H_gen");
    return LHF_ERR_INVALID;
  }
  return LHF_OK;
}

// Enqueue the step's stages; `which` selects stages (bit 0 assemble, 1 DFT, 2 eigensolve).
int32_t run_stages(lhf_plan_s* p, const lhf_step_args* a, hipStream_t s, int which) {
  int32_t st = LHF_OK;
  const bool mixed = p->prec == LHF_PREC_MIXED;
  const bool refine = mixed && (a->heev_flags & LHF_HEEV_REFINE_FP64);
  const bool direct = refine && a->H_bar64 && !a->H_gen && !a->H_bar;
  // separable formation of the complex128 blocks from the FP64 Grams (FP64
  // plans, and mixed plans whose FP32 solve reads the complex128 blocks)
  const bool sep = p->sep_ok && p->fourier_sep && (!mixed || direct);
  if ((which & 1) && sep) {
    st = lhf_assemble_blocks(p, nullptr, nullptr, a->grams64, nullptr, nullptr, a->ws, a->ws_bytes, s);
    if (st != LHF_OK) return st;
  } else if (which & 1) {
    st = lhf_assemble_blocks(p, a->H_gen, a->S_gen, a->grams64, mixed ? a->H_gen64 : nullptr,
                             mixed ? a->S_gen64 : nullptr, a->ws, a->ws_bytes, s);
    if (st != LHF_OK) return st;
  }
  if ((which & 2) && sep) {
    st = lhf_fourier_blocks(p, a->grams64, mixed ? a->H_bar64 : a->H_bar, mixed ? a->S_bar64 : a->S_bar, a->ws,
                            a->ws_bytes, s);
    if (st != LHF_OK) return st;
  } else if ((which & 2) && direct) {
    // the FP32 solve reads the complex128 blocks: one FP64 transform
    st = lhf_block_fft(p, LHF_PREC_FP64, a->H_gen64, a->S_gen64, a->H_bar64, a->S_bar64, a->ws, a->ws_bytes, s);
    if (st != LHF_OK) return st;
  } else if ((which & 2) && refine && a->H_bar64 && !a->H_gen) {
    // one FP64 transform writes the complex128 blocks and their complex64 copies
    st = lhf_block_fft_dual(p, a->H_gen64, a->S_gen64, a->H_bar64, a->S_bar64, a->H_bar, a->S_bar, a->ws,
                            a->ws_bytes, s);
    if (st != LHF_OK) return st;
  } else if (which & 2) {
    st = lhf_block_fft(p, p->prec, a->H_gen, a->S_gen, a->H_bar, a->S_bar, a->ws, a->ws_bytes, s);
    if (st != LHF_OK) return st;
    if (refine && a->H_bar64) {
      st = lhf_block_fft(p, LHF_PREC_FP64, a->H_gen64, a->S_gen64, a->H_bar64, a->S_bar64, a->ws, a->ws_bytes, s);
      if (st != LHF_OK) return st;
    }
  }
  if (which & 4) {
    st = lhf_heev_batched(p, a->heev_flags, a->H_bar, a->S_bar, refine ? a->H_bar64 : nullptr,
                          refine ? a->S_bar64 : nullptr, refine ? a->H_gen64 : nullptr,
                          refine ? a->S_gen64 : nullptr, a->w, a->V, a->info, a->ws, a->ws_bytes, s);
  }
  return st;
}

// Rebuild the work tables that depend on the tunables and upload them into
// the plan's existing device arrays (their sizes do not depend on them,
// except the Gram item list, which is reallocated when it changes length).
int32_t apply_tuning(lhf_plan_s* p) {
  for (LatDev& L : p->lat)
    for (int d = 0; d < 3; ++d) set_gram_split(L, d, p->gram_split);
  std::vector<GramItem> items;
  plan_grams(p->lat, items, p->gram_tile);
  std::vector<DftTask> tasks;
  std::vector<DftLaunch> launches;
  std::vector<FusedTask> fused;
  int64_t tmp = 0, fwgs = 0;
  int32_t fbmax = 0, flds = 0;
  plan_block_dft(p->lat, p->dft_target_threads, tasks, launches, tmp, fused, fwgs, fbmax, flds);
  if (tmp != p->dft_tmp_elems) { set_error("internal: DFT intermediate size changed"); return LHF_ERR_INVALID; }
  hipError_t e = hipMemcpy(p->d_lat, p->lat.data(), sizeof(LatDev) * p->lat.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && (int32_t)items.size() != p->n_gram_items) {
    (void)hipFree(p->d_gram_items);
    p->d_gram_items = nullptr;
    e = hipMalloc(reinterpret_cast<void**>(&p->d_gram_items), sizeof(GramItem) * items.size());
  }
  if (e == hipSuccess)
    e = hipMemcpy(p->d_gram_items, items.data(), sizeof(GramItem) * items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_dft_tasks, tasks.data(), sizeof(DftTask) * tasks.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_status(e, "upload of tuned plan tables");
  p->n_gram_items = (int32_t)items.size();
  p->dft_launches = launches;
  return LHF_OK;
}

void get_tuning(const lhf_plan_s* p, lhf_tuning* t) {
  std::memset(t, 0, sizeof(*t));
  t->dft_threads = p->dft_target_threads;
  t->gram_split = p->gram_split;
  t->gram_grid = p->gram_grid;
  t->tol32_scale = p->tol32_scale;
  t->heev_wide = 0;
  for (int c = 0; c < 4; ++c) t->heev_wide |= p->heev_wide[c] ? 1 << c : 0;
  t->fourier_sep = p->fourier_sep && p->sep_ok ? 1 : 0;
  t->gram_tile = p->gram_tile;
  t->heev_fp64 = 0;
  if (p->prec == LHF_PREC_MIXED)
    for (int c = 0; c < 4; ++c) t->heev_fp64 |= p->heev_fp64[c] ? 1 << c : 0;
}

int32_t set_tuning(lhf_plan_s* p, const lhf_tuning* t) {
  if (t->dft_threads < 1024 || t->dft_threads > (1 << 24) || t->gram_split < 1 || t->gram_split > kGramSplitMax ||
      t->gram_grid < 1 || t->gram_grid > (1 << 20) || t->tol32_scale < 1 || t->tol32_scale > (1 << 16) ||
      t->heev_wide < 0 || t->heev_wide > 15 || t->fourier_sep < 0 || t->fourier_sep > 1 ||
      t->heev_fp64 < 0 || t->heev_fp64 > 15 || (t->gram_tile != 64 && t->gram_tile != 32)) {
    set_error("tuning value out of range");
    return LHF_ERR_INVALID;
  }
  const bool tables = t->dft_threads != p->dft_target_threads || t->gram_split != p->gram_split ||
                      t->gram_tile != p->gram_tile;
  // launch shapes, kernels and work tables are baked into captured graphs:
  // any change makes them stale
  lhf_tuning was;
  get_tuning(p, &was);
  if (was.dft_threads != t->dft_threads || was.gram_split != t->gram_split || was.gram_grid != t->gram_grid ||
      was.tol32_scale != t->tol32_scale || was.heev_wide != t->heev_wide ||
      was.fourier_sep != (t->fourier_sep && p->sep_ok ? 1 : 0) ||
      (p->prec == LHF_PREC_MIXED && was.heev_fp64 != t->heev_fp64) || was.gram_tile != t->gram_tile)
    ++p->tuning_gen;
  p->gram_tile = t->gram_tile;
  p->dft_target_threads = t->dft_threads;
  p->gram_split = t->gram_split;
  p->gram_grid = t->gram_grid;
  p->tol32_scale = t->tol32_scale;
  for (int c = 0; c < 4; ++c) p->heev_wide[c] = (t->heev_wide >> c) & 1;
  p->fourier_sep = t->fourier_sep;
  for (int c = 0; c < 4; ++c) p->heev_fp64[c] = p->prec == LHF_PREC_MIXED && ((t->heev_fp64 >> c) & 1);
  return tables ? apply_tuning(p) : LHF_OK;
}

std::string cache_key(const lhf_plan_s* p) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (char& c : arch)
    if (c == '"' || c == '\\') c = '_';
  char buf[64];
  std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)p->signature);
  return std::string(buf) + ":" + arch + ":" + std::to_string(cus);
}

// The cache holds one JSON object, one entry per line:
//   "key": {"dft_threads": 131072, "gram_split": 256, ...},
std::map<std::string, std::string> read_cache(const char* path) {
  std::map<std::string, std::string> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t a = line.find('"');
    if (a == std::string::npos) continue;
    const size_t b = line.find('"', a + 1);
    const size_t o = line.find('{', b == std::string::npos ? a : b);
    const size_t c = line.rfind('}');
    if (b == std::string::npos || o == std::string::npos || c == std::string::npos || c < o) continue;
    out[line.substr(a + 1, b - a - 1)] = line.substr(o, c - o + 1);
  }
  return out;
}

bool field(const std::string& body, const char* name, double& v) {
  const std::string k = std::string("\"") + name + "\":";
  const size_t at = body.find(k);
  if (at == std::string::npos) return false;
  char* end = nullptr;
  const char* start = body.c_str() + at + k.size();
  v = std::strtod(start, &end);
  return end != start;
}

bool parse_entry(const std::string& body, lhf_tuning& t) {
  double a, b, c, d, e = 0.0;
  if (!field(body, "dft_threads", a) || !field(body, "gram_split", b) || !field(body, "gram_grid", c) ||
      !field(body, "tol32_scale", d))
    return false;
  field(body, "step_ms", e);
  double w = -1.0;
  t.heev_wide = field(body, "heev_wide", w) && w >= 0.0 ? (int32_t)w : t.heev_wide;
  w = -1.0;
  t.fourier_sep = field(body, "fourier_sep", w) && w >= 0.0 ? (int32_t)w : t.fourier_sep;
  w = -1.0;
  t.heev_fp64 = field(body, "heev_fp64", w) && w >= 0.0 ? (int32_t)w : t.heev_fp64;
  w = -1.0;
  t.gram_tile = field(body, "gram_tile", w) && w >= 0.0 ? (int32_t)w : t.gram_tile;
  t.dft_threads = (int32_t)a;
  t.gram_split = (int32_t)b;
  t.gram_grid = (int32_t)c;
  t.tol32_scale = (int32_t)d;
  t.step_ms = e;
  return true;
}

void write_cache(const char* path, std::map<std::string, std::string> entries, const std::string& key,
                 const lhf_tuning& t) {
  char buf[256];
  std::snprintf(buf, sizeof(buf),
                "{\"dft_threads\": %d, \"gram_split\": %d, \"gram_grid\": %d, \"tol32_scale\": %d, "
                "\"heev_wide\": %d, \"fourier_sep\": %d, \"heev_fp64\": %d, \"gram_tile\": %d, "
                "\"step_ms\": %.6f}",
                t.dft_threads, t.gram_split, t.gram_grid, t.tol32_scale, t.heev_wide, t.fourier_sep, t.heev_fp64,
                t.gram_tile, t.step_ms);
  entries[key] = buf;
  std::ofstream f(path, std::ios::trunc);
  f << "{\n";
  size_t i = 0;
  for (const auto& kv : entries) f << "\"" << kv.first << "\": " << kv.second << (++i < entries.size() ? ",\n" : "\n");
  f << "}\n";
}

}  // namespace

extern "C" {

int32_t lhf_step(lhf_plan_t p, const lhf_step_args* a, lhf_stream_t stream) {
  int32_t st = check_args(p, a);
  if (st != LHF_OK) return st;
  return run_stages(p, a, static_cast<hipStream_t>(stream), 7);
}

int32_t lhf_graph_create(lhf_plan_t p, const lhf_step_args* a, lhf_graph_t* out) {
  if (!out) { set_error("out is NULL"); return LHF_ERR_INVALID; }
  *out = nullptr;
  int32_t st = check_args(p, a);
  if (st != LHF_OK) return st;
  hipStream_t cs = nullptr;
  if ((st = hip_status(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream")) != LHF_OK) return st;
  hipGraph_t graph = nullptr;
  st = hip_status(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
  if (st == LHF_OK) {
    st = run_stages(p, a, cs, 7);
    const int32_t end = hip_status(hipStreamEndCapture(cs, &graph), "end capture");
    if (st == LHF_OK) st = end;
  }
  (void)hipStreamDestroy(cs);
  if (st != LHF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  auto* g = new (std::nothrow) lhf_graph_s();
  if (!g) { (void)hipGraphDestroy(graph); set_error("out of host memory"); return LHF_ERR_ALLOC; }
  g->graph = graph;
  g->plan = p;
  g->tuning_gen = p->tuning_gen;
  st = hip_status(hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0), "graph instantiation");
  if (st != LHF_OK) { lhf_graph_destroy(g); return st; }
  *out = g;
  return LHF_OK;
}

int32_t lhf_graph_launch(lhf_graph_t g, lhf_stream_t stream) {
  if (!g || !g->exec) { set_error("NULL graph"); return LHF_ERR_INVALID; }
  if (g->plan->tuning_gen != g->tuning_gen) {
    set_error("the plan's tuning changed after this graph was captured: capture it again");
    return LHF_ERR_INVALID;
  }
  return hip_status(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)), "graph launch");
}

int32_t lhf_graph_destroy(lhf_graph_t g) {
  if (!g) return LHF_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return LHF_OK;
}

int32_t lhf_plan_get_tuning(lhf_plan_t p, lhf_tuning* out) {
  if (!p || !out) { set_error("NULL plan or output"); return LHF_ERR_INVALID; }
  get_tuning(p, out);
  return LHF_OK;
}

int32_t lhf_plan_set_tuning(lhf_plan_t p, const lhf_tuning* in) {
  if (!p || !in) { set_error("NULL plan or input"); return LHF_ERR_INVALID; }
  return set_tuning(p, in);
}

int32_t lhf_plan_autotune(lhf_plan_t p, const lhf_step_args* a, lhf_stream_t stream, const char* cache_path,
                          lhf_tuning* out) {
  int32_t st = check_args(p, a);
  if (st != LHF_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = hip_status(hipStreamSynchronize(s), "synchronize")) != LHF_OK) return st;
  const std::string key = cache_key(p);
  std::map<std::string, std::string> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    auto it = cache.find(key);
    lhf_tuning t{};
    get_tuning(p, &t);   // entries without a field keep the plan's value
    if (it != cache.end() && parse_entry(it->second, t)) {
      if ((st = set_tuning(p, &t)) != LHF_OK) return st;
      if (out) { get_tuning(p, out); out->step_ms = t.step_ms; out->from_cache = 1; }
      return LHF_OK;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((st = hip_status(hipEventCreate(&e0), "event")) != LHF_OK) return st;
  if ((st = hip_status(hipEventCreate(&e1), "event")) != LHF_OK) { (void)hipEventDestroy(e0); return st; }
  // mean time of `reps` runs of the selected stages, after two untimed runs
  auto timed = [&](int which, int reps, double& ms) -> int32_t {
    int32_t r = LHF_OK;
    for (int i = 0; i < 2 && r == LHF_OK; ++i) r = run_stages(p, a, s, which);
    if (r == LHF_OK) r = hip_status(hipEventRecord(e0, s), "event record");
    for (int i = 0; i < reps && r == LHF_OK; ++i) r = run_stages(p, a, s, which);
    if (r == LHF_OK) r = hip_status(hipEventRecord(e1, s), "event record");
    if (r == LHF_OK) r = hip_status(hipEventSynchronize(e1), "event synchronize");
    float f = 0.f;
    if (r == LHF_OK) r = hip_status(hipEventElapsedTime(&f, e0, e1), "event time");
    ms = (double)f / reps;
    return r;
  };
  // keep the fastest of whole candidate settings, timed on the selected stages
  auto pick = [&](int which, const lhf_tuning* cand, int ncand) -> int32_t {
    int best = 0;
    double best_ms = 1e300;
    for (int i = 0; i < ncand; ++i) {
      int32_t r = hip_status(hipStreamSynchronize(s), "synchronize");
      if (r == LHF_OK) r = set_tuning(p, &cand[i]);
      double ms = 0.0;
      if (r == LHF_OK) r = timed(which, 20, ms);
      if (r != LHF_OK) return r;
      if (ms < best_ms) { best_ms = ms; best = i; }
    }
    int32_t r = hip_status(hipStreamSynchronize(s), "synchronize");
    return r == LHF_OK ? set_tuning(p, &cand[best]) : r;
  };
  // coordinate search: each knob only moves the time of its own stage
  auto search = [&](int which, int32_t lhf_tuning::*knob, const int32_t* cand, int ncand) -> int32_t {
    lhf_tuning cur{};
    get_tuning(p, &cur);
    std::vector<lhf_tuning> c(ncand, cur);
    for (int i = 0; i < ncand; ++i) c[i].*knob = cand[i];
    return pick(which, c.data(), ncand);
  };
  static const int32_t split_c[] = {16, 32, 64, 128, 256};
  static const int32_t grid_c[] = {1024, 2048, 4096, 8192};
  static const int32_t dft_c[] = {32768, 65536, 131072, 262144, 524288};
  static const int32_t tol_c[] = {1, 16, 256, 4096};
  double step_ms = 0.0;
  st = timed(7, 1, step_ms);   // fills every buffer the later stages read
  static const int32_t tile_c[] = {64, 32};
  if (st == LHF_OK) st = search(1, &lhf_tuning::gram_tile, tile_c, 2);
  if (st == LHF_OK) st = search(1, &lhf_tuning::gram_split, split_c, 5);
  if (st == LHF_OK) st = search(1, &lhf_tuning::gram_grid, grid_c, 4);
  // Fourier blocks: separable formation or generator stacks and block DFT, timed over whole steps (the
  // route also changes where the blocks sit when the eigensolver reads them)
  static const int32_t sep_c[] = {0, 1};
  if (st == LHF_OK && p->sep_ok) st = search(7, &lhf_tuning::fourier_sep, sep_c, 2);
  if (st == LHF_OK) st = search(2, &lhf_tuning::dft_threads, dft_c, 5);
  // eigensolver, one size class at a time: layout, and on mixed plans given
  // the complex128 blocks, FP32 solve + FP64 refinement or the FP64 solve alone
  // (the latter wins where the cost of a rotation, not its arithmetic, sets
  // the time); the two are searched together, since the best layout of one
  // solver need not be that of the other
  const bool alone = p->prec == LHF_PREC_MIXED && (a->heev_flags & LHF_HEEV_REFINE_FP64) && a->H_bar64 &&
                     !(a->heev_flags & LHF_HEEV_FP32_SOLVE);
  for (int c = 0; c < 4 && st == LHF_OK; ++c) {
    if (p->ncanon[c] == 0) continue;
    lhf_tuning cur{};
    get_tuning(p, &cur);
    lhf_tuning cand[4];
    for (int i = 0; i < 4; ++i) {
      cand[i] = cur;
      cand[i].heev_wide = (i & 1) ? cur.heev_wide | (1 << c) : cur.heev_wide & ~(1 << c);
      cand[i].heev_fp64 = (i & 2) ? cur.heev_fp64 | (1 << c) : cur.heev_fp64 & ~(1 << c);
    }
    st = pick(4, cand, alone ? 4 : 2);
  }
  if (st == LHF_OK && p->prec == LHF_PREC_MIXED) st = search(4, &lhf_tuning::tol32_scale, tol_c, 4);
  if (st == LHF_OK) st = timed(7, 10, step_ms);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LHF_OK) return st;
  lhf_tuning t{};
  get_tuning(p, &t);
  t.step_ms = step_ms;
  if (cache_path) write_cache(cache_path, cache, key, t);
  if (out) *out = t;
  return LHF_OK;
}

}  // extern "C"

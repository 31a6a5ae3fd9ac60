// Plan creation: validation of the lattice descriptors, derivation of grids,
// bands, split factors and buffer offsets, upload of the device tables.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

namespace lhf {

namespace {
thread_local std::string g_last_error;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool finite(double x) { return std::isfinite(x); }
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

// FNV-1a over the derived lattice tables and the precision choices: equal
// signatures mean equal work, so tuned launch shapes carry over.
uint64_t plan_signature(const lhf_plan_s* p) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* data, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  };
  mix(&p->prec, sizeof(p->prec));
  mix(&p->gram, sizeof(p->gram));
  mix(p->lat.data(), sizeof(LatDev) * p->lat.size());
  return h;
}

Ws ws_view(const lhf_plan_s* p, void* base) {
  char* b = static_cast<char*>(base);
  Ws w;
  w.fac = reinterpret_cast<double*>(b + p->ws_fac);
  w.grams64 = reinterpret_cast<double*>(b + p->ws_grams64);
  w.grams32 = reinterpret_cast<float*>(b + p->ws_grams32);
  w.part64 = reinterpret_cast<double*>(b + p->ws_part64);
  w.part32 = reinterpret_cast<float*>(b + p->ws_part32);
  w.dft = b + p->ws_dft;
  w.U = reinterpret_cast<float2*>(b + p->ws_U);
  w.info32 = reinterpret_cast<int32_t*>(b + p->ws_info);
  w.gh = p->sep_ok ? reinterpret_cast<double2*>(b + p->ws_gh) : nullptr;
  return w;
}

// Split-K of the Gram contraction of dimension d over 64 x 64 workgroup
// tiles: at least one 32-node chunk of the window per split, about `target`
// workgroups per (lattice, dimension).  The split count is monotone in
// `target`, so a plan sized with kGramSplitMax has room for every smaller
// target.
void set_gram_split(LatDev& L, int d, int target) {
  DimDev& D = L.dim[d];
  const int M = L.T * L.m0, N = D.nshift * L.m0;
  const int64_t tiles = (int64_t)((M + 63) / 64) * ((N + 63) / 64);
  int ks = (int)std::max<int64_t>(1, (target + tiles - 1) / tiles);
  ks = std::min(ks, std::max(1, (D.kwin + 31) / 32));
  const int kchunk = ((D.kwin + ks - 1) / ks + 31) / 32 * 32;
  D.kchunk = kchunk;
  D.ksplit = (D.kwin + kchunk - 1) / kchunk;
}

// Grouped Gram work list: one item per (lattice, dimension, 64x64 tile, split).
void plan_grams(const std::vector<LatDev>& lats, std::vector<GramItem>& items, int tile) {
  items.clear();
  for (int i = 0; i < (int)lats.size(); ++i) {
    const LatDev& L = lats[i];
    for (int d = 0; d < 3; ++d) {
      const DimDev& D = L.dim[d];
      const int M = L.T * L.m0, N = D.nshift * L.m0;
      for (int tm = 0; tm < (M + tile - 1) / tile; ++tm)
        for (int tn = 0; tn < (N + tile - 1) / tile; ++tn)
          for (int ks = 0; ks < D.ksplit; ++ks) items.push_back(GramItem{i, d, tm, tn, ks, 0});
    }
  }
  // longest first (LPT): an item's work is its share of the window (the
  // tiles are equal); workgroups take items grid-stride in this order, so
  // the long ones start first and the short ones fill the tail.  The kernel
  // reads every output location from the item, so the order is free.
  auto cost = [&](const GramItem& it) {
    const DimDev& D = lats[it.li].dim[it.d];
    return std::min(D.kchunk, D.kwin - it.ks * D.kchunk);
  };
  std::stable_sort(items.begin(), items.end(),
                   [&](const GramItem& a, const GramItem& b) { return cost(a) > cost(b); });
}

// Fill one lattice's device descriptor; returns LHF_OK or an error code.
static int32_t derive_lattice(const lhf_lattice& in, int idx, LatDev& L, std::string& err) {
  std::memset(&L, 0, sizeof(L));
  const lhf_cell& c = in.cell;
  auto bad = [&](const std::string& m) {
    err = "lattice " + std::to_string(idx) + ": " + m;
    return LHF_ERR_INVALID;
  };
  if (c.m0 < 1) return bad("m0 must be >= 1");
  if (c.m0 > kMaxM0) { err = "lattice " + std::to_string(idx) + ": m0 > 32 unsupported"; return LHF_ERR_UNSUPPORTED; }
  if (!c.alpha || !c.centre) return bad("alpha and centre are required");
  if (c.M0 < 1 || !c.Z || !c.nuc) return bad("at least one nucleus with Z and position is required");
  if (c.M0 > kMaxNuc) { err = "lattice " + std::to_string(idx) + ": more than 4 nuclei per cell unsupported"; return LHF_ERR_UNSUPPORTED; }
  if (in.R < 1) return bad("R must be >= 1");
  if (in.R > kMaxR || c.M0 * in.R > kMaxTerms - 2) {
    err = "lattice " + std::to_string(idx) + ": R > 64 or M0 R > 96 unsupported";
    return LHF_ERR_UNSUPPORTED;
  }
  if (!(in.a > 0) || !finite(in.a)) return bad("lattice step a must be positive");
  if (!(in.sinc_step > 0) || !finite(in.sinc_step) || !finite(in.sinc_u0)) return bad("bad sinc parameters");
  if (in.bc != LHF_BC_PERIODIC && in.bc != LHF_BC_DIRICHLET) return bad("bc must be periodic or Dirichlet");

  L.m0 = c.m0; L.M0 = c.M0; L.R = in.R; L.T = 2 + c.M0 * in.R;
  double amin = 1e300, jmax = 0.0;
  for (int mu = 0; mu < c.m0; ++mu) {
    double al = c.alpha[mu];
    if (!(al > 0) || !finite(al)) return bad("exponents must be positive and finite");
    int ang = c.ang ? c.ang[mu] : LHF_ANG_S;
    if (ang < 0 || ang > 3) return bad("angular type must be 0..3");
    L.alpha[mu] = al;
    amin = std::min(amin, al);
    for (int d = 0; d < 3; ++d) {
      double x = c.centre[3 * mu + d];
      if (!finite(x)) return bad("centres must be finite");
      L.cen[mu][d] = x;
      jmax = std::max(jmax, std::fabs(x));
      int pw = (ang == d + 1) ? 1 : 0;
      L.lpow[mu][d] = pw;
      double base = std::pow(2.0 * al / M_PI, 0.25);
      L.norm[mu][d] = pw ? base * 2.0 * std::sqrt(al) : base;
    }
  }
  for (int nu = 0; nu < c.M0; ++nu) {
    if (!(c.Z[nu] > 0) || !finite(c.Z[nu])) return bad("charges must be positive");
    L.Z[nu] = c.Z[nu];
    for (int d = 0; d < 3; ++d) {
      if (!finite(c.nuc[3 * nu + d])) return bad("nuclear positions must be finite");
      L.nuc[nu][d] = c.nuc[3 * nu + d];
    }
  }
  for (int q = 0; q < in.R; ++q) {
    double t = std::exp(in.sinc_u0 + q * in.sinc_step);
    L.tq[q] = t;
    L.wq[q] = (2.0 / std::sqrt(M_PI)) * in.sinc_step * t;
  }
  int64_t nblk = 1;
  for (int d = 0; d < 3; ++d) {
    DimDev& D = L.dim[d];
    int Ld = in.L[d], nd = in.n[d];
    if (Ld < 1) return bad("L must be >= 1");
    if (Ld > 32768) {
      err = "lattice " + std::to_string(idx) + ": more than 32768 cells along one dimension unsupported";
      return LHF_ERR_UNSUPPORTED;
    }
    if (nd < 4) return bad("n must be >= 4");
    L.L[d] = Ld;
    nblk *= Ld;
    D.L = Ld; D.n = nd; D.a = in.a;
    bool periodic = in.bc == LHF_BC_PERIODIC && Ld >= 2;
    if (periodic) {
      if (nd % Ld != 0) return bad("on a periodic dimension n must be a multiple of L");
      D.periodic = 1; D.replicate = 1;
      D.nc = nd / Ld; D.npot = D.nc;
      if (D.nc < 2) return bad("need at least two nodes per cell");
      if (D.nc > 256) {
        err = "lattice " + std::to_string(idx) + ": more than 256 nodes per cell unsupported";
        return LHF_ERR_UNSUPPORTED;
      }
      D.h = Ld * in.a / nd;
      D.x0 = 0.0;
      D.X0 = 0.5 * in.a;
      D.y0 = -0.5 * in.a;
      D.period = Ld * in.a;
      D.nimg = (int)std::ceil(std::sqrt(800.0 / amin) / D.period) + 1;
    } else {
      if (Ld >= 2) {
        err = "lattice " + std::to_string(idx) + ": Dirichlet dimensions with L >= 2 are handled by lhf_toeplitz_create";
        return LHF_ERR_UNSUPPORTED;
      }
      if (!(in.pad[d] >= 0) || !finite(in.pad[d])) return bad("pad must be >= 0");
      double W = Ld * in.a + 2.0 * in.pad[d];
      D.h = W / (nd + 1);
      D.x0 = -0.5 * W + D.h;
      D.X0 = -0.5 * Ld * in.a + 0.5 * in.a;
      D.y0 = 0.0;
      D.replicate = 0; D.npot = nd; D.nc = 0; D.nimg = 0;
    }
    // band half-width
    int L0 = in.L0[d];
    if (L0 < 0) {
      double reach = 2.0 * jmax + std::sqrt(101.4 / amin);
      L0 = (int)std::ceil(reach / in.a);
    }
    if (Ld == 1) {
      D.full = 1; D.nshift = 1; D.L0 = 0;
    } else if (2 * L0 + 1 >= Ld) {
      D.full = 1; D.nshift = Ld; D.L0 = (Ld - 1) / 2;
    } else {
      D.full = 0; D.nshift = 2 * L0 + 1; D.L0 = L0;
    }
    // Gram contraction window: every summand contains a cell-0 factor
    // (G_0[nu] in Op_t G_0), which is below 1e-25 of its peak farther than
    // W cells from cell 0, with W a >= sqrt(57.6 / alpha_min) + 2 max|centre|.
    D.kstart = 0;
    D.kwin = nd;
    if (periodic) {
      const int W = (int)std::ceil((std::sqrt(57.6 / amin) + 2.0 * jmax) / in.a);
      if ((int64_t)(2 * W + 1) * D.nc < nd) {
        D.kwin = (2 * W + 1) * D.nc;
        D.kstart = nd - W * D.nc;
      }
    }
    set_gram_split(L, d, kGramSplitMax);
  }
  if (nblk * c.m0 * c.m0 >= ((int64_t)1 << 31)) {
    err = "lattice " + std::to_string(idx) + ": L1 L2 L3 m0^2 >= 2^31 unsupported";
    return LHF_ERR_UNSUPPORTED;
  }
  L.nblk = (int32_t)nblk;
  return LHF_OK;
}

}  // namespace lhf

using namespace lhf;

extern "C" {

const char* lhf_last_error(void) { return g_last_error.c_str(); }

const char* lhf_status_string(int32_t s) {
  switch (s) {
    case LHF_OK: return "ok";
    case LHF_ERR_INVALID: return "invalid argument";
    case LHF_ERR_UNSUPPORTED: return "unsupported";
    case LHF_ERR_WORKSPACE: return "workspace too small";
    case LHF_ERR_HIP: return "HIP runtime error";
    case LHF_ERR_ALLOC: return "allocation failed";
    default: return "unknown status";
  }
}

int32_t lhf_version(void) { return 1; }

int32_t lhf_plan_create(const lhf_lattice* lats, int32_t nlat, int32_t prec, int32_t gram,
                        lhf_plan_t* out) {
  if (!out) { set_error("out is NULL"); return LHF_ERR_INVALID; }
  *out = nullptr;
  if (!lats || nlat < 1) { set_error("need at least one lattice"); return LHF_ERR_INVALID; }
  if (prec != LHF_PREC_FP64 && prec != LHF_PREC_MIXED) { set_error("bad precision"); return LHF_ERR_INVALID; }
  if (gram < LHF_GRAM_FP64 || gram > LHF_GRAM_FP16X3) { set_error("bad gram mode"); return LHF_ERR_INVALID; }
  auto* p = new (std::nothrow) lhf_plan_s();
  if (!p) { set_error("out of host memory"); return LHF_ERR_ALLOC; }
  p->prec = prec; p->gram = gram; p->nlat = nlat;
  p->lat.resize(nlat);
  std::string err;
  int64_t fac = 0, grams = 0, part = 0, tw = 0, gen = 0, w = 0, blk = 0, gh = 0, half = 0;
  for (int i = 0; i < nlat; ++i) {
    int32_t st = derive_lattice(lats[i], i, p->lat[i], err);
    if (st != LHF_OK) { set_error(err); delete p; return st; }
    LatDev& L = p->lat[i];
    for (int d = 0; d < 3; ++d) {
      DimDev& D = L.dim[d];
      D.g_off = fac; fac += (int64_t)D.n * L.m0;
      D.p_off = fac; fac += (int64_t)(L.M0 * L.R) * D.npot;
      D.gram_off = grams; grams += (int64_t)L.T * D.nshift * L.m0 * L.m0;
      D.part_off = part; part += (int64_t)D.ksplit * (L.T * L.m0) * (D.nshift * L.m0);
      D.tw_off = tw; tw += D.L;
      D.gh_off = -1;
      if (d > 0) { D.gh_off = gh; gh += (int64_t)L.T * D.L * L.m0 * L.m0; }
    }
    L.gen_off = gen; gen += (int64_t)L.nblk * L.m0 * L.m0;
    L.half_off = half; half += (int64_t)L.L[0] * L.L[1] * (L.L[2] / 2 + 1) * L.m0 * L.m0;
    L.w_off = w; w += (int64_t)L.nblk * L.m0;
    L.blk_off = blk; blk += L.nblk;
  }
  p->signature = plan_signature(p);
  std::vector<DftTask> dft_tasks;
  int64_t dtmp = 0;
  std::vector<FusedTask> fused;
  plan_block_dft(p->lat, p->dft_target_threads, dft_tasks, p->dft_launches, dtmp, fused, p->fused_wgs,
                 p->fused_bmax, p->fused_lds);
  p->n_fused = (int32_t)fused.size();
  std::vector<FusedTask> sep;
  std::vector<GhItem> gh_items;
  std::vector<FusedTask> sep_chain;
  plan_separable(p->lat, sep, gh_items, p->sep_wgs, p->sep_bmax, p->sep_lds, p->gh_threads, sep_chain,
                 p->sep_chain_wgs, p->sep_ok, p->sep_async);
  p->n_sep = (int32_t)sep.size();
  p->n_sep_chain = (int32_t)sep_chain.size();
  p->n_gh_items = (int32_t)gh_items.size();
  p->gh_elems = gh;
  p->sizes.nlat = nlat;
  p->sizes.nblocks = blk;
  p->sizes.gen_elems = gen;
  p->sizes.half_elems = half;
  p->sizes.w_elems = w;
  p->sizes.grams_elems = grams;
  p->fac_doubles = fac;
  p->part_elems = part;
  p->dft_tmp_elems = dtmp;
  size_t off = 0;
  p->ws_fac = off; off = align256(off + (size_t)fac * 8);
  p->ws_grams64 = off; off = align256(off + (size_t)grams * 8);
  p->ws_part64 = off; off = align256(off + (size_t)part * 8);
  if (prec == LHF_PREC_MIXED) {
    p->ws_grams32 = off; off = align256(off + (size_t)grams * 4);
    p->ws_part32 = off; off = align256(off + (size_t)part * 4);
    p->ws_U = off; off = align256(off + (size_t)gen * 8);
    p->ws_info = off; off = align256(off + (size_t)blk * 4);
  }
  p->ws_dft = off; off = align256(off + (size_t)dtmp * 16);   // complex128 (either precision)
  if (p->sep_ok) { p->ws_gh = off; off = align256(off + (size_t)gh * 16); }
  p->sizes.ws_bytes = off;

  std::vector<GramItem> items;
  plan_grams(p->lat, items, p->gram_tile);
  p->n_gram_items = (int32_t)items.size();

  // grouped factor work
  std::vector<FacItem> fac_items;
  plan_factors(p->lat, fac_items);
  p->n_fac_items = (int32_t)fac_items.size();

  // combine: thread range of each lattice starts at a multiple of 256
  std::vector<int64_t> elem_start(nlat);
  int64_t ct = 0;
  for (int i = 0; i < nlat; ++i) {
    elem_start[i] = ct;
    ct += ((int64_t)p->lat[i].nblk * p->lat[i].m0 * p->lat[i].m0 + 255) / 256 * 256;
  }
  p->combine_threads = ct;

  // canonical blocks per eigensolver size class: j with (-j mod L) >= j in
  // linear order, as (lattice, block)
  std::vector<int2> canon[4];
  for (int i = 0; i < nlat; ++i) {
    const LatDev& L = p->lat[i];
    std::vector<int2>& cl = canon[heev_class(L.m0)];
    for (int b = 0; b < L.nblk; ++b) {
      const int k3 = b % L.L[2], k2 = (b / L.L[2]) % L.L[1], k1 = b / (L.L[2] * L.L[1]);
      const int c1 = k1 ? L.L[0] - k1 : 0, c2 = k2 ? L.L[1] - k2 : 0, c3 = k3 ? L.L[2] - k3 : 0;
      const int cb = (c1 * L.L[1] + c2) * L.L[2] + c3;
      if (cb >= b) cl.push_back(make_int2(i, b));
    }
  }
  for (int c = 0; c < 4; ++c) {
    p->ncanon[c] = (int32_t)canon[c].size();
    // wavefronts of the four-entries-per-thread launch: (M/2)^2 threads per
    // matrix, 64 / that many matrices per wavefront when below 64
    const int m = 4 << c, tpm = (m / 2) * (m / 2);
    const int64_t waves = tpm >= 64 ? (int64_t)p->ncanon[c] * (tpm / 64) : ((int64_t)p->ncanon[c] * tpm + 63) / 64;
    p->heev_wide[c] = p->ncanon[c] > 0 && waves < lhf_plan_s::kWideWaves;
  }

  // twiddle tables exp(-2 pi i m / L)
  std::vector<double2> tw64(tw);
  std::vector<float2> tw32(tw);
  for (int i = 0; i < nlat; ++i) {
    for (int d = 0; d < 3; ++d) {
      const DimDev& D = p->lat[i].dim[d];
      for (int m = 0; m < D.L; ++m) {
        double ang = -2.0 * M_PI * (double)m / (double)D.L;
        tw64[D.tw_off + m] = make_double2(std::cos(ang), std::sin(ang));
        tw32[D.tw_off + m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      }
    }
  }
  bool ok = hipGetDevice(&p->device) == hipSuccess;
  auto upload = [&](auto*& dst, const auto* src, size_t count) {
    if (!ok || count == 0) return;
    const size_t bytes = sizeof(*src) * count;
    ok = hipMalloc(reinterpret_cast<void**>(&dst), bytes) == hipSuccess &&
         hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  upload(p->d_lat, p->lat.data(), (size_t)nlat);
  upload(p->d_tw64, tw64.data(), (size_t)tw);
  upload(p->d_tw32, tw32.data(), (size_t)tw);
  upload(p->d_gram_items, items.data(), items.size());
  upload(p->d_fac_items, fac_items.data(), fac_items.size());
  upload(p->d_elem_start, elem_start.data(), elem_start.size());
  upload(p->d_dft_tasks, dft_tasks.data(), dft_tasks.size());
  upload(p->d_fused, fused.data(), fused.size());
  if (p->sep_ok) {
    upload(p->d_sep, sep.data(), sep.size());
    upload(p->d_sep_chain, sep_chain.data(), sep_chain.size());
    upload(p->d_gh_items, gh_items.data(), gh_items.size());
  }
  for (int c = 0; c < 4; ++c) upload(p->d_canon[c], canon[c].data(), canon[c].size());
  if (!ok) {
    set_error("allocation or upload of the plan tables failed");
    lhf_plan_destroy(p);
    return LHF_ERR_ALLOC;
  }
  *out = p;
  return LHF_OK;
}

int32_t lhf_plan_sizes(lhf_plan_t plan, lhf_sizes* out) {
  if (!plan || !out) { set_error("NULL plan or output"); return LHF_ERR_INVALID; }
  *out = plan->sizes;
  return LHF_OK;
}

int32_t lhf_plan_band(lhf_plan_t plan, int32_t index, int32_t* nshift, int32_t* L0, int32_t* full) {
  if (!plan || !nshift || !L0 || !full || index < 0 || index >= plan->nlat) {
    set_error("lhf_plan_band: bad argument");
    return LHF_ERR_INVALID;
  }
  for (int d = 0; d < 3; ++d) {
    const DimDev& D = plan->lat[index].dim[d];
    nshift[d] = D.nshift;
    L0[d] = D.L0;
    full[d] = D.full;
  }
  return LHF_OK;
}

size_t lhf_workspace_size(lhf_plan_t plan) { return plan ? plan->sizes.ws_bytes : 0; }

int32_t lhf_plan_destroy(lhf_plan_t plan) {
  if (!plan) return LHF_OK;
  void* tables[] = {plan->d_lat, plan->d_tw64, plan->d_tw32, plan->d_gram_items, plan->d_fac_items,
                    plan->d_elem_start, plan->d_dft_tasks, plan->d_fused, plan->d_canon[0], plan->d_canon[1],
                    plan->d_canon[2], plan->d_canon[3], plan->d_sep, plan->d_sep_chain, plan->d_gh_items};
  for (void* t : tables)
    if (t) (void)hipFree(t);
  delete plan;
  return LHF_OK;
}

}  // extern "C"

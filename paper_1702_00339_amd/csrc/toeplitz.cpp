// Dirichlet-chain operators: validation and derivation of the perturbed
// block-Toeplitz model or of the exact box operator, their assembly on the
// device, the matvec entry point and the block LOBPCG driver for the lowest
// eigenpairs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "plan.h"
#include "toeplitz.h"
#include "toeplitz3.h"

using namespace lhf;

struct lhf_toeplitz_s {
  ToepDev host{};
  int device = 0;
  bool exact = false;                   // the exact box operator: block-sparse, no Toeplitz part
  bool three = false;                   // the three-level Toeplitz operator of a box lattice
  Toep3Dev host3{};
  Toep3Dev* d_desc3 = nullptr;
  double* d_grams3 = nullptr;           // three-level: 1D Grams per dimension and shift
  void* d_tw3_64[3] = {nullptr, nullptr, nullptr};
  void* d_tw3_32[3] = {nullptr, nullptr, nullptr};
  int L = 0, m0 = 0, L0 = 0, P = 0, N = 0, nX = 0, ncb = 0, njobs = 0, nrows = 0, nent = 0;
  double sigma = 0.0;
  std::vector<void*> allocs;            // every device allocation, freed by destroy
  ToepDev* d_desc = nullptr;
  Defect* d_defs = nullptr;
  double* d_vrep = nullptr;
  double* d_vbox = nullptr;             // exact operator: finite-lattice potential [M0 R][n]
  int32_t* d_cell_def = nullptr;        // exact operator: defect index per cell or -1
  double* d_trans = nullptr;
  ScalePair* d_pairs = nullptr;
  ToepJob* d_jobs = nullptr;
  double* d_blkH = nullptr;             // [njobs][m0][m0]: generators A_0..A_L0, then cross blocks
  double* d_blkS = nullptr;
  int32_t* d_cross_km = nullptr;
  int32_t* d_row_ptr = nullptr;
  int32_t* d_row_cell = nullptr;
  CrossEntry* d_ent = nullptr;
  double* d_dH = nullptr;
  double* d_dS = nullptr;
  double2* d_cH = nullptr;
  double2* d_cS = nullptr;
  float2* d_cH32 = nullptr;
  float2* d_cS32 = nullptr;
  double2* d_minv64 = nullptr;
  float2* d_minv32 = nullptr;
  double2* d_tw64 = nullptr;
  float2* d_tw32 = nullptr;
};

namespace {

int32_t hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return LHF_OK;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return LHF_ERR_HIP;
}

template <typename T>
bool dalloc(lhf_toeplitz_s* t, T*& ptr, size_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(1, count) * sizeof(T)) != hipSuccess) return false;
  t->allocs.push_back(p);
  ptr = static_cast<T*>(p);
  return true;
}

template <typename T>
bool upload(lhf_toeplitz_s* t, T*& ptr, const T* src, size_t count) {
  return dalloc(t, ptr, count) &&
         (count == 0 || hipMemcpy(ptr, src, count * sizeof(T), hipMemcpyHostToDevice) == hipSuccess);
}

bool finite(double x) { return std::isfinite(x); }

int32_t bad(const std::string& m) {
  set_error("lhf_toeplitz_create: " + m);
  return LHF_ERR_INVALID;
}

int32_t unsupported(const std::string& m) {
  set_error("lhf_toeplitz_create: " + m);
  return LHF_ERR_UNSUPPORTED;
}

// Validate the descriptor and fill the device descriptor (model readings of
// the header: cell-aligned chain nodes, band from the smallest exponent).
int32_t derive(const lhf_box& b, ToepDev& D, std::vector<Defect>& defs) {
  const lhf_lattice& in = b.lat;
  const lhf_cell& c = in.cell;
  std::memset(&D, 0, sizeof(D));
  if (in.bc != LHF_BC_DIRICHLET) return unsupported("the chain operator needs Dirichlet boundaries");
  if (in.L[0] < 1 || in.L[1] != 1 || in.L[2] != 1) return unsupported("an L x 1 x 1 chain is required");
  if (c.m0 < 1) return bad("m0 must be >= 1");
  if (c.m0 > kMaxM0) return unsupported("m0 > 32");
  if (!c.alpha || !c.centre) return bad("alpha and centre are required");
  if (c.M0 < 1 || !c.Z || !c.nuc) return bad("at least one nucleus is required");
  if (c.M0 > kMaxNuc) return unsupported("more than 4 nuclei per cell");
  if (in.R < 1) return bad("R must be >= 1");
  if (in.R > kMaxR || c.M0 * in.R > kMaxTerms - 2) return unsupported("R > 64 or M0 R > 96");
  if (!(in.a > 0) || !finite(in.a)) return bad("lattice step a must be positive");
  if (!(in.sinc_step > 0) || !finite(in.sinc_step) || !finite(in.sinc_u0)) return bad("bad sinc parameters");
  const int L = in.L[0];
  if (in.n[0] % L) return unsupported("n1 must be a multiple of L");
  const int nc = in.n[0] / L;
  if (nc < 2) return bad("need at least two nodes per cell");
  if (nc > 256) return unsupported("more than 256 nodes per cell");
  if (std::fabs(in.pad[0] - 0.5 * in.a / nc) > 1e-12 * in.a) return unsupported("chain nodes must be cell aligned: pad1 = a / (2 nc)");
  for (int d = 1; d < 3; ++d) {
    if (in.n[d] < 4) return bad("n must be >= 4");
    if (!(in.pad[d] >= 0) || !finite(in.pad[d])) return bad("pad must be >= 0");
  }
  if (b.ndef < 0 || (b.ndef > 0 && (!b.def_cells || !b.def_Z || !b.def_scale))) return bad("bad defect arrays");
  D.L = L;
  D.nc = nc;
  D.n = in.n[0];
  D.m0 = c.m0;
  D.M0 = c.M0;
  D.R = in.R;
  D.a = in.a;
  D.h = in.a / nc;
  D.x0 = -0.5 * (L * in.a + 2.0 * in.pad[0]);
  for (int d = 0; d < 2; ++d) {
    const double Wt = in.a + 2.0 * in.pad[1 + d];
    D.nt[d] = in.n[1 + d];
    D.ht[d] = Wt / (in.n[1 + d] + 1);
    D.t0[d] = -0.5 * Wt;
  }
  double amin = 1e300, jmax = 0.0;
  for (int mu = 0; mu < c.m0; ++mu) {
    const double al = c.alpha[mu];
    if (!(al > 0) || !finite(al)) return bad("exponents must be positive");
    const int ang = c.ang ? c.ang[mu] : LHF_ANG_S;
    if (ang < 0 || ang > 3) return bad("angular type must be 0..3");
    D.alpha[mu] = al;
    amin = std::min(amin, al);
    for (int d = 0; d < 3; ++d) {
      const double x = c.centre[3 * mu + d];
      if (!finite(x)) return bad("centres must be finite");
      D.cen[mu][d] = x;
      jmax = std::max(jmax, std::fabs(x));
      D.lpow[mu][d] = ang == d + 1 ? 1 : 0;
    }
  }
  for (int nu = 0; nu < c.M0; ++nu) {
    if (!(c.Z[nu] > 0) || !finite(c.Z[nu])) return bad("charges must be positive");
    D.Z[nu] = c.Z[nu];
    for (int d = 0; d < 3; ++d) {
      if (!finite(c.nuc[3 * nu + d])) return bad("nuclear positions must be finite");
      D.nuc[nu][d] = c.nuc[3 * nu + d];
    }
  }
  for (int q = 0; q < in.R; ++q) {
    D.tq[q] = std::exp(in.sinc_u0 + q * in.sinc_step);
    D.wq[q] = (2.0 / std::sqrt(M_PI)) * in.sinc_step * D.tq[q];
  }
  std::set<int> seen;
  double smin = 1.0;
  for (int i = 0; i < b.ndef; ++i) {
    const int cell = b.def_cells[i];
    if (cell < 0 || cell >= L || !seen.insert(cell).second) return bad("defect cells must be distinct and in [0, L)");
    if (!(b.def_Z[i] > 0) || !finite(b.def_Z[i])) return bad("defect charges must be positive");
    if (!(b.def_scale[i] > 0) || !finite(b.def_scale[i])) return bad("defect scale factors must be positive");
    defs.push_back(Defect{cell, 0, b.def_Z[i], b.def_scale[i]});
    smin = std::min(smin, b.def_scale[i]);
  }
  D.ndef = b.ndef;
  const double am = amin * smin;
  D.L0 = std::min(L - 1, (int)std::ceil((2.0 * jmax + std::sqrt(101.4 / am)) / in.a));
  D.margin = (int)std::ceil((std::sqrt(80.6 / am) + jmax) / in.a) + 1;
  int P = 2;
  while (P < L + D.L0) P *= 2;
  if (P > 4096) return unsupported("circulant embedding longer than 4096 cells");
  D.P = P;
  return LHF_OK;
}

}  // namespace

extern "C" int32_t lhf_toeplitz_destroy(lhf_toeplitz_t t) {
  if (!t) return LHF_OK;
  for (void* p : t->allocs) (void)hipFree(p);
  delete t;
  return LHF_OK;
}

namespace {

// Spectrum of the embedding's per-frequency pencils (C_H(f), C_S(f)) by the
// batched Hermitian solver over the P = P1 P2 P3 frequency blocks (frequency
// f and -f mod P per level are conjugate), the shift sigma below it (half its
// width lower) and the preconditioner blocks (C_H(f) - sigma C_S(f))^-1.
// Synchronous; on error the caller destroys t.
int32_t build_preconditioner(lhf_toeplitz_s* t, int dev, hipStream_t s) {
  const int m0 = t->m0, P = t->P;
  const size_t mm = (size_t)m0 * m0;
  const int P1 = t->three ? t->host3.P[0] : P, P2 = t->three ? t->host3.P[1] : 1, P3 = t->three ? t->host3.P[2] : 1;
  lhf_plan_s fp;
  fp.prec = LHF_PREC_FP64;
  fp.nlat = 1;
  fp.device = dev;
  LatDev ld{};
  ld.m0 = m0;
  ld.L[0] = P1; ld.L[1] = P2; ld.L[2] = P3;
  ld.nblk = P;
  fp.lat.push_back(ld);
  std::vector<int2> canon;
  for (int f = 0; f < P; ++f) {
    const int f1 = f / (P2 * P3), f2 = (f / P3) % P2, f3 = f % P3;
    const int cf = (((P1 - f1) % P1) * P2 + (P2 - f2) % P2) * P3 + (P3 - f3) % P3;
    if (cf >= f) canon.push_back(make_int2(0, f));
  }
  const int cls = heev_class(m0);
  fp.ncanon[cls] = (int32_t)canon.size();
  double* d_w = nullptr;
  double2* d_V = nullptr;
  int32_t* d_info = nullptr;
  hipError_t e = hipSuccess;
  const bool ok = upload(t, fp.d_lat, fp.lat.data(), 1) && upload(t, fp.d_canon[cls], canon.data(), canon.size()) &&
                  dalloc(t, d_w, (size_t)P * m0) && dalloc(t, d_V, (size_t)P * mm) && dalloc(t, d_info, (size_t)P);
  if (ok) e = launch_heev(&fp, LHF_HEEV_VECTORS, t->d_cH, t->d_cS, nullptr, nullptr, nullptr, nullptr, d_w, d_V,
                          d_info, nullptr, nullptr, s);
  fp.d_lat = nullptr;                 // owned by t->allocs
  fp.d_canon[cls] = nullptr;
  if (!ok) { set_error("lhf_toeplitz_create: device allocation failed"); return LHF_ERR_ALLOC; }
  std::vector<double> w((size_t)P * m0);
  std::vector<int32_t> info(P);
  if (e == hipSuccess) e = hipMemcpy(w.data(), d_w, w.size() * sizeof(double), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(info.data(), d_info, info.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_status(e, "lhf_toeplitz_create");
  for (int f = 0; f < P; ++f)
    if (info[f] != 0) {
      set_error("lhf_toeplitz_create: the embedding's overlap block of frequency " + std::to_string(f) +
                " is not positive definite (status " + std::to_string(info[f]) + ")");
      return LHF_ERR_INVALID;
    }
  const double wmin = *std::min_element(w.begin(), w.end()), wmax2 = *std::max_element(w.begin(), w.end());
  t->sigma = wmin - 0.5 * std::max(wmax2 - wmin, 1.0);
  e = toep_launch_minv(d_V, d_w, t->sigma, t->d_minv64, t->d_minv32, P, m0, s);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return hip_status(e, "lhf_toeplitz_create");
}

int32_t create(const lhf_box* box, bool exact, lhf_toeplitz_t* out) {
  if (!out) { set_error("out is NULL"); return LHF_ERR_INVALID; }
  *out = nullptr;
  if (!box) { set_error("box is NULL"); return LHF_ERR_INVALID; }
  ToepDev D;
  std::vector<Defect> defs;
  int32_t st = derive(*box, D, defs);
  if (st != LHF_OK) return st;
  const int L = D.L, m0 = D.m0, L0 = D.L0, nc = D.nc, mm = m0 * m0;
  std::vector<int> defect_of(L, -1);
  for (int i = 0; i < (int)defs.size(); ++i) defect_of[defs[i].cell] = i;
  // X: defect cells and cells within L0 of a wall; every cell for the exact
  // operator, whose blocks are all computed
  std::set<int> X;
  for (int k = 0; k < L; ++k)
    if (exact || k < L0 || k > L - 1 - L0 || defect_of[k] >= 0) X.insert(k);
  // scale pairs and jobs: generators first, then cross blocks (k <= m) ascending
  std::map<std::pair<int, int>, int> pair_id;
  std::vector<ScalePair> pairs;
  auto pid = [&](int dk, int dm) {
    auto key = std::make_pair(dk, dm);
    auto it = pair_id.find(key);
    if (it != pair_id.end()) return it->second;
    const int id = (int)pairs.size();
    pairs.push_back(ScalePair{dk, dm});
    pair_id[key] = id;
    return id;
  };
  std::vector<ToepJob> jobs;
  for (int s = 0; s <= L0; ++s)
    jobs.push_back(ToepJob{0, s, 0, pid(-1, -1), 1 - D.margin * nc, (s + 1 + D.margin) * nc, -1, -1});
  std::set<std::pair<int, int>> cross;
  for (int c : X)
    for (int m = std::max(0, c - L0); m <= std::min(L - 1, c + L0); ++m) cross.insert({std::min(c, m), std::max(c, m)});
  std::vector<int32_t> km;
  for (const auto& kmp : cross) {
    const int k = kmp.first, m = kmp.second;
    const int dk = defect_of[k], dm = defect_of[m];
    jobs.push_back(ToepJob{k, m, exact ? 2 : 1, pid(dk, dm), std::max(1, (k - D.margin) * nc + 1),
                           std::min(D.n, (m + 1 + D.margin) * nc), dk, dm});
    km.push_back(k);
    km.push_back(m);
  }
  int wmax = 0;
  for (const ToepJob& j : jobs) wmax = std::max(wmax, j.ihi - j.ilo + 1);
  const size_t lds_blocks = sizeof(double) * (2 * (size_t)m0 * (wmax + 2) + (size_t)wmax);
  hipDeviceProp_t prop;
  int dev = 0;
  if ((st = hip_status(hipGetDevice(&dev), "device")) != LHF_OK) return st;
  if ((st = hip_status(hipGetDeviceProperties(&prop, dev), "device properties")) != LHF_OK) return st;
  if (lds_blocks > prop.sharedMemPerBlock) return unsupported("chain window of the Grams does not fit in LDS");
  // cross corrections grouped by block row
  std::map<int, std::vector<CrossEntry>> rows;
  int b = 0;
  for (const auto& kmp : cross) {
    const int k = kmp.first, m = kmp.second;
    rows[k].push_back(CrossEntry{m, b, 0, 0});
    if (m != k) rows[m].push_back(CrossEntry{k, b, 1, 0});
    ++b;
  }
  std::vector<int32_t> row_ptr{0}, row_cell;
  std::vector<CrossEntry> ent;
  for (auto& r : rows) {
    std::sort(r.second.begin(), r.second.end(), [](const CrossEntry& x, const CrossEntry& y) { return x.m < y.m; });
    row_cell.push_back(r.first);
    for (const CrossEntry& e : r.second) ent.push_back(e);
    row_ptr.push_back((int32_t)ent.size());
  }
  // twiddles exp(-2 pi i k / P), k < P / 2
  const int P = D.P;
  std::vector<double2> tw64(P / 2);
  std::vector<float2> tw32(P / 2);
  for (int k = 0; k < P / 2; ++k) {
    const double ang = -2.0 * M_PI * k / P;
    tw64[k] = make_double2(std::cos(ang), std::sin(ang));
    tw32[k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }

  auto* t = new (std::nothrow) lhf_toeplitz_s();
  if (!t) { set_error("out of host memory"); return LHF_ERR_ALLOC; }
  t->host = D;
  t->device = dev;
  t->exact = exact;
  t->L = L; t->m0 = m0; t->L0 = L0; t->P = P; t->N = m0 * L; t->nX = (int)X.size();
  t->ncb = (int)cross.size();
  t->njobs = (int)jobs.size();
  t->nrows = (int)row_cell.size();
  t->nent = (int)ent.size();
  const int M0R = D.M0 * D.R, T2 = 2 + M0R;
  bool ok = upload(t, t->d_desc, &D, 1) && upload(t, t->d_defs, defs.data(), defs.size()) &&
            upload(t, t->d_pairs, pairs.data(), pairs.size()) && upload(t, t->d_jobs, jobs.data(), jobs.size()) &&
            upload(t, t->d_cross_km, km.data(), km.size()) && upload(t, t->d_row_ptr, row_ptr.data(), row_ptr.size()) &&
            upload(t, t->d_row_cell, row_cell.data(), row_cell.size()) && upload(t, t->d_ent, ent.data(), ent.size()) &&
            upload(t, t->d_tw64, tw64.data(), tw64.size()) && upload(t, t->d_tw32, tw32.data(), tw32.size()) &&
            dalloc(t, t->d_vrep, (size_t)M0R * nc) && dalloc(t, t->d_trans, (size_t)pairs.size() * 2 * T2 * mm) &&
            dalloc(t, t->d_blkH, (size_t)jobs.size() * mm) && dalloc(t, t->d_blkS, (size_t)jobs.size() * mm) &&
            dalloc(t, t->d_dH, (size_t)ent.size() * mm) && dalloc(t, t->d_dS, (size_t)ent.size() * mm) &&
            dalloc(t, t->d_cH, (size_t)P * mm) && dalloc(t, t->d_cS, (size_t)P * mm) &&
            dalloc(t, t->d_cH32, (size_t)P * mm) && dalloc(t, t->d_cS32, (size_t)P * mm) &&
            dalloc(t, t->d_minv64, (size_t)P * mm) && dalloc(t, t->d_minv32, (size_t)P * mm);
  if (ok && exact)
    ok = upload(t, t->d_cell_def, defect_of.data(), defect_of.size()) && dalloc(t, t->d_vbox, (size_t)M0R * D.n);
  if (!ok) { lhf_toeplitz_destroy(t); set_error("lhf_toeplitz_create: device allocation failed"); return LHF_ERR_ALLOC; }
  hipStream_t s = nullptr;
  hipError_t e = toep_launch_vrep(t->d_desc, t->d_vrep, M0R, nc, s);
  if (e == hipSuccess && exact) e = toep_launch_vbox(t->d_desc, t->d_defs, t->d_cell_def, t->d_vbox, M0R, D.n, s);
  if (e == hipSuccess)
    e = toep_launch_transverse(t->d_desc, t->d_defs, t->d_pairs, (int)pairs.size(), m0, M0R, t->d_trans, s);
  if (e == hipSuccess)
    e = toep_launch_blocks(t->d_desc, t->d_defs, t->d_jobs, t->njobs, m0, wmax, t->d_vrep, t->d_vbox, t->d_trans,
                           t->d_blkH, t->d_blkS, s);
  const double* genH = t->d_blkH;
  const double* genS = t->d_blkS;
  const double* crH = t->d_blkH + (size_t)(L0 + 1) * mm;
  const double* crS = t->d_blkS + (size_t)(L0 + 1) * mm;
  // correction entries D = H_model - T; for the exact operator the blocks themselves
  if (e == hipSuccess)
    e = toep_launch_delta(t->d_desc, t->d_row_ptr, t->d_row_cell, t->nrows, t->d_ent, exact ? nullptr : genH,
                          exact ? nullptr : genS, crH, crS, t->d_dH, t->d_dS, m0, s);
  if (e == hipSuccess) e = toep_launch_chat(t->d_desc, genH, genS, t->d_cH, t->d_cS, m0, P, L0, s);
  if (e == hipSuccess) e = toep_launch_to32(t->d_cH, t->d_cH32, (int64_t)P * mm, s);
  if (e == hipSuccess) e = toep_launch_to32(t->d_cS, t->d_cS32, (int64_t)P * mm, s);
  st = e == hipSuccess ? build_preconditioner(t, dev, s) : hip_status(e, "lhf_toeplitz_create");
  if (st != LHF_OK) {
    lhf_toeplitz_destroy(t);
    return st;
  }
  *out = t;
  return LHF_OK;
}

// The three-level block-Toeplitz operator of a box lattice (readings of
// lhf_toeplitz3_create in the header): validation, grids and bands per
// dimension, the 1D Grams, the embedding's per-frequency blocks and the
// preconditioner.
int32_t create3(const lhf_lattice* lat, lhf_toeplitz_t* out) {
  if (!out) { set_error("out is NULL"); return LHF_ERR_INVALID; }
  *out = nullptr;
  if (!lat) { set_error("lattice is NULL"); return LHF_ERR_INVALID; }
  const lhf_lattice& in = *lat;
  const lhf_cell& c = in.cell;
  auto bad3 = [](const std::string& m) { set_error("lhf_toeplitz3_create: " + m); return LHF_ERR_INVALID; };
  auto uns3 = [](const std::string& m) { set_error("lhf_toeplitz3_create: " + m); return LHF_ERR_UNSUPPORTED; };
  if (in.bc != LHF_BC_DIRICHLET) return uns3("the three-level operator is for a lattice in a box (Dirichlet)");
  if (c.m0 < 1) return bad3("m0 must be >= 1");
  if (c.m0 > kMaxM0) return uns3("m0 > 32");
  if (!c.alpha || !c.centre) return bad3("alpha and centre are required");
  if (c.M0 < 1 || !c.Z || !c.nuc) return bad3("at least one nucleus is required");
  if (c.M0 > kMaxNuc) return uns3("more than 4 nuclei per cell");
  if (in.R < 1) return bad3("R must be >= 1");
  if (in.R > kMaxR || c.M0 * in.R > kMaxTerms - 2) return uns3("R > 64 or M0 R > 96");
  if (!(in.a > 0) || !finite(in.a)) return bad3("lattice step a must be positive");
  if (!(in.sinc_step > 0) || !finite(in.sinc_step) || !finite(in.sinc_u0)) return bad3("bad sinc parameters");
  Toep3Dev D;
  std::memset(&D, 0, sizeof(D));
  D.m0 = c.m0;
  D.M0 = c.M0;
  D.R = in.R;
  D.a = in.a;
  double amin = 1e300, jmax = 0.0;
  for (int mu = 0; mu < c.m0; ++mu) {
    const double al = c.alpha[mu];
    if (!(al > 0) || !finite(al)) return bad3("exponents must be positive");
    const int ang = c.ang ? c.ang[mu] : LHF_ANG_S;
    if (ang < 0 || ang > 3) return bad3("angular type must be 0..3");
    D.alpha[mu] = al;
    amin = std::min(amin, al);
    for (int d = 0; d < 3; ++d) {
      const double x = c.centre[3 * mu + d];
      if (!finite(x)) return bad3("centres must be finite");
      D.cen[mu][d] = x;
      jmax = std::max(jmax, std::fabs(x));
      D.lpow[mu][d] = ang == d + 1 ? 1 : 0;
    }
  }
  for (int nu = 0; nu < c.M0; ++nu) {
    if (!(c.Z[nu] > 0) || !finite(c.Z[nu])) return bad3("charges must be positive");
    D.Z[nu] = c.Z[nu];
    for (int d = 0; d < 3; ++d) {
      if (!finite(c.nuc[3 * nu + d])) return bad3("nuclear positions must be finite");
      D.nuc[nu][d] = c.nuc[3 * nu + d];
    }
  }
  for (int q = 0; q < in.R; ++q) {
    D.tq[q] = std::exp(in.sinc_u0 + q * in.sinc_step);
    D.wq[q] = (2.0 / std::sqrt(M_PI)) * in.sinc_step * D.tq[q];
  }
  const int band = (int)std::ceil((2.0 * jmax + std::sqrt(101.4 / amin)) / in.a);
  const int E = (int)std::ceil((std::sqrt(80.6 / amin) + jmax) / in.a) + 1;
  const int T = 2 + c.M0 * in.R, m0 = c.m0;
  const size_t mm = (size_t)m0 * m0;
  std::vector<Gram3Job> jobs;
  int64_t vpot = 0, grams = 0, gh = 0;
  int64_t Ptot = 1, cells = 1;
  int wmax = 0;
  for (int d = 0; d < 3; ++d) {
    const int L = in.L[d], n = in.n[d];
    if (L < 1) return bad3("L must be >= 1");
    if (n < 4) return bad3("n must be >= 4");
    if (!(in.pad[d] >= 0) || !finite(in.pad[d])) return bad3("pad must be >= 0");
    D.L[d] = L;
    D.n[d] = n;
    if (L >= 2) {
      if (n % L) return uns3("multi-cell dimensions need n a multiple of L");
      const int nc = n / L;
      if (nc < 2) return bad3("need at least two nodes per cell");
      if (nc > 256) return uns3("more than 256 nodes per cell");
      if (std::fabs(in.pad[d] - 0.5 * in.a / nc) > 1e-12 * in.a)
        return uns3("multi-cell dimensions need cell-aligned nodes: pad = a / (2 nc)");
      D.h[d] = in.a / nc;
      D.x0[d] = -0.5 * (L * in.a + 2.0 * in.pad[d]);
      D.L0[d] = std::min(L - 1, band);
      int P = 2;
      while (P < L + D.L0[d]) P *= 2;
      if (P > 4096) return uns3("embedding longer than 4096 cells in one dimension");
      D.P[d] = P;
      D.vpot_len[d] = nc;
      for (int sh = 0; sh <= D.L0[d]; ++sh) {
        const Gram3Job j{d, sh, 1 - E * nc, (sh + 1 + E) * nc};
        jobs.push_back(j);
        wmax = std::max(wmax, j.ihi - j.ilo + 1);
      }
    } else {
      const double W = in.a + 2.0 * in.pad[d];
      D.h[d] = W / (n + 1);
      D.x0[d] = -0.5 * W;
      D.L0[d] = 0;
      D.P[d] = 1;
      D.vpot_len[d] = n;
      jobs.push_back(Gram3Job{d, 0, 1, n});
      wmax = std::max(wmax, n);
    }
    D.vpot_off[d] = vpot; vpot += (int64_t)c.M0 * in.R * D.vpot_len[d];
    D.gram_off[d] = grams; grams += (int64_t)(D.L0[d] + 1) * T * mm;
    D.gh_off[d] = gh; gh += (int64_t)T * D.P[d] * mm;
    Ptot *= D.P[d];
    cells *= L;
  }
  if (Ptot > (1 << 22)) return uns3("embedding with more than 2^22 frequencies");
  hipDeviceProp_t prop;
  int dev = 0;
  int32_t st;
  if ((st = hip_status(hipGetDevice(&dev), "device")) != LHF_OK) return st;
  if ((st = hip_status(hipGetDeviceProperties(&prop, dev), "device properties")) != LHF_OK) return st;
  const size_t lds = sizeof(double) * (2 * (size_t)m0 * (wmax + 2) + (size_t)wmax);
  if (lds > prop.sharedMemPerBlock) return uns3("node window of the Grams does not fit in LDS");
  auto* t = new (std::nothrow) lhf_toeplitz_s();
  if (!t) { set_error("out of host memory"); return LHF_ERR_ALLOC; }
  t->three = true;
  t->host3 = D;
  t->device = dev;
  t->L = (int)cells;
  t->m0 = m0;
  t->L0 = std::max(D.L0[0], std::max(D.L0[1], D.L0[2]));
  t->P = (int)Ptot;
  t->N = (int)(cells * m0);
  std::vector<std::vector<double2>> tw64(3);
  std::vector<std::vector<float2>> tw32(3);
  bool ok = upload(t, t->d_desc3, &D, 1);
  Gram3Job* d_jobs = nullptr;
  double* d_vpot = nullptr;
  double2* d_gh = nullptr;
  ok = ok && upload(t, d_jobs, jobs.data(), jobs.size()) && dalloc(t, d_vpot, (size_t)vpot) &&
       dalloc(t, t->d_grams3, (size_t)grams) && dalloc(t, d_gh, (size_t)gh) &&
       dalloc(t, t->d_cH, (size_t)Ptot * mm) && dalloc(t, t->d_cS, (size_t)Ptot * mm) &&
       dalloc(t, t->d_cH32, (size_t)Ptot * mm) && dalloc(t, t->d_cS32, (size_t)Ptot * mm) &&
       dalloc(t, t->d_minv64, (size_t)Ptot * mm) && dalloc(t, t->d_minv32, (size_t)Ptot * mm);
  for (int d = 0; d < 3 && ok; ++d) {
    const int P = D.P[d], nh = std::max(1, P / 2);
    tw64[d].resize(nh);
    tw32[d].resize(nh);
    for (int k = 0; k < nh; ++k) {
      const double ang = -2.0 * M_PI * k / P;
      tw64[d][k] = make_double2(std::cos(ang), std::sin(ang));
      tw32[d][k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    double2* p64 = nullptr;
    float2* p32 = nullptr;
    ok = upload(t, p64, tw64[d].data(), nh) && upload(t, p32, tw32[d].data(), nh);
    t->d_tw3_64[d] = p64;
    t->d_tw3_32[d] = p32;
  }
  if (!ok) { lhf_toeplitz_destroy(t); set_error("lhf_toeplitz3_create: device allocation failed"); return LHF_ERR_ALLOC; }
  hipStream_t s = nullptr;
  hipError_t e = toep3_launch_assembly(t->d_desc3, D, d_jobs, (int)jobs.size(), wmax, d_vpot, t->d_grams3, d_gh,
                                       t->d_cH, t->d_cS, s);
  if (e == hipSuccess) e = toep_launch_to32(t->d_cH, t->d_cH32, Ptot * (int64_t)mm, s);
  if (e == hipSuccess) e = toep_launch_to32(t->d_cS, t->d_cS32, Ptot * (int64_t)mm, s);
  st = e == hipSuccess ? build_preconditioner(t, dev, s) : hip_status(e, "lhf_toeplitz3_create");
  if (st != LHF_OK) {
    lhf_toeplitz_destroy(t);
    return st;
  }
  *out = t;
  return LHF_OK;
}

}  // namespace

extern "C" {

int32_t lhf_toeplitz_create(const lhf_box* box, lhf_toeplitz_t* out) { return create(box, false, out); }

int32_t lhf_box_exact_create(const lhf_box* box, lhf_toeplitz_t* out) { return create(box, true, out); }

int32_t lhf_toeplitz3_create(const lhf_lattice* lat, lhf_toeplitz_t* out) { return create3(lat, out); }

int32_t lhf_toeplitz3_generators(lhf_toeplitz_t t, double* gH, double* gS) {
  if (!t) { set_error("NULL operator"); return LHF_ERR_INVALID; }
  if (!t->three) { set_error("not a three-level operator (lhf_toeplitz3_create)"); return LHF_ERR_INVALID; }
  if (!gH || !gS) { set_error("gen_H and gen_S are required"); return LHF_ERR_INVALID; }
  hipError_t e = toep3_launch_generators(t->d_desc3, t->host3, t->d_grams3, gH, gS, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return hip_status(e, "lhf_toeplitz3_generators");
}

int32_t lhf_toeplitz_get_info(lhf_toeplitz_t t, lhf_toeplitz_info* out) {
  if (!t || !out) { set_error("NULL operator or output"); return LHF_ERR_INVALID; }
  out->L = t->L;
  out->m0 = t->m0;
  out->L0 = t->L0;
  out->N = t->N;
  out->P = t->P;
  out->ncross = t->nX;
  out->ncross_blocks = t->ncb;
  out->sigma = t->sigma;
  return LHF_OK;
}

int32_t lhf_toeplitz_blocks(lhf_toeplitz_t t, double* gH, double* gS, int32_t* km, double* cH, double* cS) {
  if (!t) { set_error("NULL operator"); return LHF_ERR_INVALID; }
  if (t->three) { set_error("a three-level operator: use lhf_toeplitz3_generators"); return LHF_ERR_UNSUPPORTED; }
  const size_t mm = (size_t)t->m0 * t->m0, ng = (size_t)(t->L0 + 1) * mm, nc = (size_t)t->ncb * mm;
  hipError_t e = hipSuccess;
  if (gH && e == hipSuccess) e = hipMemcpy(gH, t->d_blkH, ng * 8, hipMemcpyDeviceToDevice);
  if (gS && e == hipSuccess) e = hipMemcpy(gS, t->d_blkS, ng * 8, hipMemcpyDeviceToDevice);
  if (km && e == hipSuccess) e = hipMemcpy(km, t->d_cross_km, (size_t)t->ncb * 8, hipMemcpyDeviceToDevice);
  if (cH && e == hipSuccess) e = hipMemcpy(cH, t->d_blkH + ng, nc * 8, hipMemcpyDeviceToDevice);
  if (cS && e == hipSuccess) e = hipMemcpy(cS, t->d_blkS + ng, nc * 8, hipMemcpyDeviceToDevice);
  return hip_status(e, "lhf_toeplitz_blocks");
}

size_t lhf_toeplitz_matvec_workspace(lhf_toeplitz_t t, int32_t ncols) {
  if (!t || ncols < 1) return 0;
  if (t->three) return toep3_apply_ws_bytes(t->host3, ncols, true);
  return 3 * (size_t)t->P * t->m0 * ncols * sizeof(double2);
}

int32_t lhf_toeplitz_matvec(lhf_toeplitz_t t, int32_t prec, int32_t ncols, const double* x, double* yH, double* yS,
                            int32_t ld, void* ws, size_t ws_bytes, lhf_stream_t stream) {
  if (!t) { set_error("NULL operator"); return LHF_ERR_INVALID; }
  if (prec != LHF_PREC_FP64 && prec != LHF_PREC_MIXED) { set_error("bad precision"); return LHF_ERR_INVALID; }
  if (ncols < 1 || ncols > kMaxCols || ld < ncols) { set_error("need 1 <= ncols <= 128 and ld >= ncols"); return LHF_ERR_INVALID; }
  if (!x || !yH) { set_error("x and y_H are required"); return LHF_ERR_INVALID; }
  const size_t need = lhf_toeplitz_matvec_workspace(t, ncols);
  if (!ws || ws_bytes < need) {
    set_error("workspace of " + std::to_string(ws_bytes) + " bytes given, " + std::to_string(need) + " needed");
    return LHF_ERR_WORKSPACE;
  }
  const bool f64 = prec == LHF_PREC_FP64;
  if (t->three) {
    const void* tw3[3] = {f64 ? t->d_tw3_64[0] : t->d_tw3_32[0], f64 ? t->d_tw3_64[1] : t->d_tw3_32[1],
                          f64 ? t->d_tw3_64[2] : t->d_tw3_32[2]};
    const void* o3H = f64 ? (const void*)t->d_cH : (const void*)t->d_cH32;
    const void* o3S = yS ? (f64 ? (const void*)t->d_cS : (const void*)t->d_cS32) : nullptr;
    return hip_status(toep3_launch_apply(t->host3, prec, tw3, ncols, x, ld, o3H, o3S, yH, yS, ws,
                                         static_cast<hipStream_t>(stream)),
                      "lhf_toeplitz_matvec");
  }
  char* w = static_cast<char*>(ws);
  const size_t part = (size_t)t->P * t->m0 * ncols * sizeof(double2);
  const void* opH = f64 ? (const void*)t->d_cH : (const void*)t->d_cH32;
  const void* opS = yS ? (f64 ? (const void*)t->d_cS : (const void*)t->d_cS32) : nullptr;
  hipError_t e = toep_launch_apply(prec, t->L, t->m0, t->P, ncols, x, ld, opH, opS,
                                   f64 ? (const void*)t->d_tw64 : (const void*)t->d_tw32, w, w + part, w + 2 * part,
                                   yH, yS, t->d_row_ptr, t->d_row_cell, t->nrows, t->d_ent, t->d_dH, t->d_dS,
                                   static_cast<hipStream_t>(stream), t->exact);
  return hip_status(e, "lhf_toeplitz_matvec");
}

int32_t lhf_toeplitz_matvec_f32(lhf_toeplitz_t t, int32_t ncols, const float* x, float* yH, float* yS, int32_t ld,
                                void* ws, size_t ws_bytes, lhf_stream_t stream) {
  if (!t) { set_error("NULL operator"); return LHF_ERR_INVALID; }
  if (t->three) { set_error("FP32 input and output: one-level and exact box operators only"); return LHF_ERR_UNSUPPORTED; }
  if (ncols < 1 || ncols > kMaxCols || ld < ncols) { set_error("need 1 <= ncols <= 128 and ld >= ncols"); return LHF_ERR_INVALID; }
  if (!x || !yH) { set_error("x and y_H are required"); return LHF_ERR_INVALID; }
  const size_t need = lhf_toeplitz_matvec_workspace(t, ncols);
  if (!ws || ws_bytes < need) {
    set_error("workspace of " + std::to_string(ws_bytes) + " bytes given, " + std::to_string(need) + " needed");
    return LHF_ERR_WORKSPACE;
  }
  char* w = static_cast<char*>(ws);
  const size_t part = (size_t)t->P * t->m0 * ncols * sizeof(double2);
  hipError_t e = toep_launch_apply32(t->L, t->m0, t->P, ncols, x, ld, t->d_cH32, yS ? t->d_cS32 : nullptr, t->d_tw32,
                                     w, w + part, w + 2 * part, yH, yS, t->d_row_ptr, t->d_row_cell, t->nrows,
                                     t->d_ent, t->d_dH, t->d_dS, static_cast<hipStream_t>(stream), t->exact);
  return hip_status(e, "lhf_toeplitz_matvec_f32");
}

}  // extern "C"

namespace {

constexpr int kGuard = 4;     // block vectors beyond the wanted ones
constexpr int kChunks = 256;   // row chunks of the residual norms (a workgroup each)
constexpr int kGramChunks = 64;   // row chunks of the Gram products
constexpr double kDropPivot = 1e-10;   // Cholesky-QR: squared relative distance below which a column is dropped

struct EigWs {
  double *X, *HX, *SX, *P, *R, *W, *Q, *HQ, *SQ, *Q2, *HQ2, *SQ2;
  double *G, *lam, *T, *GH, *th, *C, *C2, *norms, *part, *rpart;
  char* mv;
  size_t mv_bytes;
};

size_t eigs_layout(const lhf_toeplitz_s* t, int nev, EigWs* w, char* base) {
  const int nb = nev + kGuard, mx = 3 * nb;
  const size_t N = (size_t)t->N;
  size_t off = 0;
  auto take = [&](double*& p, size_t count) {
    p = base ? reinterpret_cast<double*>(base + off) : nullptr;
    off += (count * sizeof(double) + 255) & ~size_t(255);
  };
  EigWs d;
  take(d.X, N * nb); take(d.HX, N * nb); take(d.SX, N * nb); take(d.P, N * nb);
  take(d.R, N * nb); take(d.W, N * nb);
  take(d.Q, N * mx); take(d.HQ, N * mx); take(d.SQ, N * mx);
  take(d.Q2, N * mx); take(d.HQ2, N * mx); take(d.SQ2, N * mx);
  const size_t sq = (size_t)kMaxSmall * kMaxSmall;
  take(d.G, sq); take(d.lam, kMaxSmall);
  take(d.T, sq); take(d.GH, sq); take(d.th, kMaxSmall); take(d.C, sq); take(d.C2, sq); take(d.norms, kMaxSmall);
  take(d.part, (size_t)kGramChunks * sq); take(d.rpart, (size_t)kChunks * kMaxSmall);
  d.mv_bytes = lhf_toeplitz_matvec_workspace(const_cast<lhf_toeplitz_s*>(t), mx);
  d.mv = base ? base + off : nullptr;
  off += d.mv_bytes;
  if (w) *w = d;
  return off;
}

}  // namespace

extern "C" {

size_t lhf_toeplitz_eigs_workspace(lhf_toeplitz_t t, int32_t nev) {
  if (!t || nev < 1 || 3 * (nev + kGuard) > kMaxSmall) return 0;
  return eigs_layout(t, nev, nullptr, nullptr);
}

int32_t lhf_toeplitz_eigs(lhf_toeplitz_t t, int32_t nev, int32_t maxit, double tol, uint64_t seed, double* d_w,
                          double* d_V, int32_t* iters, double* resid, void* ws, size_t ws_bytes, lhf_stream_t stream) {
  if (!t) { set_error("NULL operator"); return LHF_ERR_INVALID; }
  const int nb = nev + kGuard;
  if (nev < 1 || nb > t->N || 3 * nb > kMaxSmall) {
    set_error("need nev >= 1, nev + 4 <= N and 3 (nev + 4) <= 112");
    return LHF_ERR_INVALID;
  }
  if (maxit < 1 || !(tol > 0)) { set_error("maxit >= 1 and tol > 0 required"); return LHF_ERR_INVALID; }
  if (!d_w) { set_error("d_w is required"); return LHF_ERR_INVALID; }
  const size_t need = lhf_toeplitz_eigs_workspace(t, nev);
  if (!ws || ws_bytes < need) {
    set_error("workspace of " + std::to_string(ws_bytes) + " bytes given, " + std::to_string(need) + " needed");
    return LHF_ERR_WORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  EigWs w;
  eigs_layout(t, nev, &w, static_cast<char*>(ws));
  const int N = t->N, mx = 3 * nb, S = kMaxSmall;
  hipError_t e = hipSuccess;
  int32_t st = LHF_OK;
  auto ck = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  auto matvec = [&](int prec, int ncols, const double* x, int ld, double* yH, double* yS) {
    if (e != hipSuccess) return;
    const int32_t r = lhf_toeplitz_matvec(t, prec, ncols, x, yH, yS, ld, w.mv, w.mv_bytes, stream);
    if (r != LHF_OK) e = hipErrorUnknown;
  };
  std::vector<double> hl(S), hn(S), hist;
  int prec = LHF_PREC_MIXED;
  bool haveP = false;
  int it = 0;
  double rmax = 0.0;
  ck(dense_random(N, nb, seed, w.X, nb, s));
  for (it = 0; it <= maxit && e == hipSuccess; ++it) {
    int m = nb;
    if (it == 0) {
      ck(dense_copy_cols(N, nb, w.X, nb, w.Q, mx, s));
    } else {
      // residuals of the current block and the convergence test
      ck(dense_residual(N, nb, w.HX, w.SX, nb, w.th, w.R, nb, w.rpart, kChunks, w.norms, s));
      ck(hipMemcpyAsync(hn.data(), w.norms, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
      ck(hipStreamSynchronize(s));
      if (e != hipSuccess) break;
      rmax = *std::max_element(hn.begin(), hn.begin() + nev);
      if (!std::isfinite(rmax)) { st = LHF_ERR_INVALID; set_error("LOBPCG residuals are not finite"); break; }
      if (prec == LHF_PREC_FP64 && rmax < tol) break;
      if (it == maxit) break;
      // FP64 matvecs once the residual is below 1e-4, or once the FP32 ones
      // stall (no 30% drop over the last five iterations: the complex64
      // transform's error floor, which grows with the operator's norm)
      bool stalled = false;
      if (hist.size() >= 5) {
        const double best = *std::min_element(hist.end() - 5, hist.end());
        stalled = rmax > 0.7 * best;
      }
      hist.push_back(rmax);
      if (prec == LHF_PREC_MIXED && (rmax < 1e-4 || stalled)) prec = LHF_PREC_FP64;
      // W = preconditioned residuals: (H_c - sigma S_c)^-1 per frequency of the embedding
      if (t->three) {
        const void* tw3[3] = {t->d_tw3_32[0], t->d_tw3_32[1], t->d_tw3_32[2]};
        ck(toep3_launch_apply(t->host3, LHF_PREC_MIXED, tw3, nb, w.R, nb, t->d_minv32, nullptr, w.W, nullptr, w.mv,
                              s));
      } else {
        ck(toep_launch_apply(LHF_PREC_MIXED, t->L, t->m0, t->P, nb, w.R, nb, t->d_minv32, nullptr, t->d_tw32, w.mv,
                             w.mv + w.mv_bytes / 3, w.mv + 2 * (w.mv_bytes / 3), w.W, nullptr, nullptr, nullptr, 0,
                             nullptr, nullptr, nullptr, s));
      }
      ck(dense_copy_cols(N, nb, w.X, nb, w.Q, mx, s));
      ck(dense_copy_cols(N, nb, w.W, nb, w.Q + nb, mx, s));
      m = 2 * nb;
      if (haveP) {
        ck(dense_copy_cols(N, nb, w.P, nb, w.Q + 2 * nb, mx, s));
        m = 3 * nb;
      }
    }
    // images of the basis, then its S-orthonormalisation: Cholesky-QR of the
    // scaled Gram matrix in the column order [X W P], dropping columns that
    // are numerically in the span of the ones before them
    matvec(prec, m, w.Q, mx, w.HQ, w.SQ);
    ck(dense_gram(N, m, m, w.Q, mx, w.SQ, mx, w.part, kGramChunks, w.G, S, s));
    ck(dense_cholqr(m, w.G, S, kDropPivot, w.T, S, w.lam, s));
    ck(hipMemcpyAsync(hl.data(), w.lam, sizeof(double), hipMemcpyDeviceToHost, s));
    ck(hipStreamSynchronize(s));
    if (e != hipSuccess) break;
    const int kk = (int)hl[0];
    if (kk < nb) { st = LHF_ERR_INVALID; set_error("LOBPCG basis lost rank"); break; }
    ck(dense_combine3(N, m, kk, w.Q, w.HQ, w.SQ, mx, w.T, S, w.Q2, w.HQ2, w.SQ2, mx, s));
    // Rayleigh-Ritz in FP64
    ck(dense_gram(N, kk, kk, w.Q2, mx, w.HQ2, mx, w.part, kGramChunks, w.GH, S, s));
    ck(dense_syev_low(kk, nb, w.GH, S, w.th, w.C, S, s));   // reads (GH + GH^T) / 2
    ck(dense_combine3(N, kk, nb, w.Q2, w.HQ2, w.SQ2, mx, w.C, S, w.W, w.HX, w.SX, nb, s));   // X_new, HX, SX
    if (it > 0) {
      // P = X_new - X (X^T S X_new)
      ck(dense_gram(N, nb, nb, w.X, nb, w.SX, nb, w.part, kGramChunks, w.C2, S, s));
      ck(dense_combine(N, nb, nb, w.X, nb, w.C2, S, -1.0, w.W, nb, w.P, nb, s));
      // P currently holds X C2 - X_new; its sign does not matter for the span
      haveP = true;
    }
    std::swap(w.X, w.W);
  }
  if (e == hipSuccess && st == LHF_OK) {
    ck(hipMemcpyAsync(d_w, w.th, sizeof(double) * nev, hipMemcpyDeviceToDevice, s));
    if (d_V) ck(dense_copy_cols(N, nev, w.X, nb, d_V, nev, s));
    ck(hipStreamSynchronize(s));
  }
  if (iters) *iters = std::min(it, maxit);
  if (resid) *resid = rmax;
  if (st != LHF_OK) return st;
  return hip_status(e, "lhf_toeplitz_eigs");
}

}  // extern "C"

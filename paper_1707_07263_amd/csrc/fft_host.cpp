// Host runtime of the MI355X FFT: variant registry, planning (pass count,
// N1 x N2 split, variant choice), twiddle tables, and the C ABI of mi355fft.h.
//
// Planning follows Sec. 2.3.2: a transform whose length fits one workgroup's
// LDS is done in one kernel; a longer 1-D transform is split in global memory
// as N = N1*N2 into two kernels (N1-point column transforms with the twiddle
// W_N^{n2*k1} fused into their store, then N2-point column transforms), the
// kernel boundary being the only global synchronisation; a 2-D transform is a
// row kernel followed by a column kernel (rows first, then columns).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mi355fft.h"
#include "levels.hpp"
#include "many.hpp"
#include "mfma.hpp"
#include "xlane.hpp"
#include "twiddle.hpp"
#include "variants.hpp"

using namespace mfft;

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return FFT_ERR_HIP;
}

// ---------------------------------------------------------------------------
// variant registry
// ---------------------------------------------------------------------------
std::vector<Variant>* g_variants = nullptr;
std::once_flag g_variants_once;

void add_one(const Variant& v) { g_variants->push_back(v); }

const std::vector<Variant>& variants() {
  std::call_once(g_variants_once, [] {
    g_variants = new std::vector<Variant>();
    add_variants_c64_row(add_one);
    add_variants_c64_a(add_one);
    add_variants_c64_col(add_one);
    add_variants_c64_col2(add_one);
    add_variants_c64_pipe(add_one);
    add_variants_c64_rowcol(add_one);
    add_variants_c16(add_one);
  });
  return *g_variants;
}

const Variant* find_by_name(const std::string& name) {
  for (const Variant& v : variants())
    if (name == v.name) return &v;
  return nullptr;
}

// Best variant of a role/length/dtype: never more lines per tile than there
// are to transform when some variant allows that (a hard filter: a tile
// wider than the lines would compute and drop whole lines, and plans whose
// tiles must cover their lines exactly refuse it); among those prefer
// P = 16, then the W closest to `want_w` from below, then the thread count
// closest to 256.
const Variant* pick(int role, int L, int dtype, int want_w, int64_t lines) {
  bool some_fit = false;
  for (const Variant& v : variants())
    if (v.role == role && v.L == L && v.dtype == dtype && v.W <= lines) some_fit = true;
  const Variant* best = nullptr;
  double best_score = 1e300;
  for (const Variant& v : variants()) {
    if (v.role != role || v.L != L || v.dtype != dtype) continue;
    if (some_fit && v.W > lines) continue;
    double score = 0;
    score += (v.P == 16 || v.P == v.L) ? 0 : 1000;
    const int w_cap = (int)std::max<int64_t>(1, std::min<int64_t>(want_w, lines));
    score += v.W > w_cap ? 100.0 * v.W / w_cap : 10.0 * std::fabs(std::log2((double)w_cap / v.W));
    score += std::fabs(std::log2(v.threads / 256.0));
    if (score < best_score) {
      best_score = score;
      best = &v;
    }
  }
  return best;
}

int ilog2_64(int64_t v) {
  int r = 0;
  while (((int64_t)1 << r) < v) ++r;
  return r;
}
bool pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }
size_t esize(int dtype) { return dtype == FFT_C64 ? 8 : 4; }

// ---------------------------------------------------------------------------
// schedule (host-only description of the launches)
// ---------------------------------------------------------------------------
enum Sel { SEL_IN = 0, SEL_OUT = 1, SEL_WS = 2 };

struct PassSpec {
  const Variant* v = nullptr;  // nullptr: copy-scale
  PassArgs args{};
  int src = SEL_IN, dst = SEL_OUT;
  int64_t copy_n = 0;          // copy-scale: points
  bool first = false, last = false;
  int64_t tw_N = 0;            // inter-pass twiddle modulus (0: none)
  int64_t tw_rows = 0;         // rows of its step table
  int64_t colr_N = 0;          // fused row pass: its column twiddles W_R^e, e < colr_N (0: none)
  int64_t scale_len = 0;       // transform length this pass accounts for (0: the variant's L)
  std::vector<int32_t> line_map;  // row pass of the three-pass 2-D plan
  // launched once per transform of the batch, pointers advanced by the
  // transform's length (the last pass of the three-pass 1-D plan)
  bool per_transform = false;
};

struct Schedule {
  std::vector<PassSpec> passes;
  int64_t split[2] = {0, 0};
  int64_t points = 0;
  bool inplace_needs_ws = false;
  // every exec needs a workspace of `points` elements (passes read or write
  // SEL_WS); the plan allocates one unless the caller sets its own
  bool always_ws = false;
  // one global-memory kernel per radix-2 level instead of LDS passes
  bool levels = false;
  // 256-point transforms with matrix-core radix-16 stages (experiment)
  bool mfma = false;
  // 256-point transforms whose exchange moves across lanes (experiment):
  // 1 DPP and ds_swizzle, 2 ds_bpermute
  int xlane = 0;
};

struct Overrides {
  int64_t split = 0;
  // per pass, 1: consecutive tiles run on one XCD.  One digit applies to
  // every pass; otherwise one digit per pass, first pass first.
  std::string xcd = "0";
  int col3 = -1;  // 2-D columns in two sub-passes: 1 yes, 0 no, -1 automatic
  int64_t split2 = 0;  // three-pass 1-D: second-pass length
  bool levels = false;  // method=levels: the per-level global-memory method
  bool mfma = false;    // method=mfma: matrix-core radix-16 stages (N = 256)
  int xlane = 0;        // method=xlane (1) | xlane_bperm (2): cross-lane exchange (N = 256)
  int blk = 0;  // 2-D: intermediate in column blocks of blk columns (0: natural order)
  int rowcol = 0;  // 2-D: row pass fused with a radix-rowcol column step (0: off)
  std::string a, b, row, col, single, colt;
};

// pass name of a single-launch 256-point experiment plan
const char* dft256_name(const Schedule& S) {
  return S.xlane == 2 ? "xlane_bperm_dft256" : S.xlane ? "xlane_dft256" : "mfma_dft256";
}

int parse_schedule(const char* s, Overrides* o) {
  if (!s) return FFT_OK;
  std::string str(s);
  size_t pos = 0;
  while (pos < str.size()) {
    size_t end = str.find(';', pos);
    if (end == std::string::npos) end = str.size();
    std::string item = str.substr(pos, end - pos);
    pos = end + 1;
    if (item.empty()) continue;
    size_t eq = item.find('=');
    if (eq == std::string::npos) return FFT_ERR_INVALID_ARGUMENT;
    std::string key = item.substr(0, eq), val = item.substr(eq + 1);
    if (key == "split") {
      char* e = nullptr;
      long long v = strtoll(val.c_str(), &e, 10);
      if (!e || *e || v < 1) return FFT_ERR_INVALID_ARGUMENT;
      o->split = v;
    } else if (key == "split2") {
      char* e = nullptr;
      long long v = strtoll(val.c_str(), &e, 10);
      if (!e || *e || v < 2) return FFT_ERR_INVALID_ARGUMENT;
      o->split2 = v;
    } else if (key == "xcd") {
      if (val.empty() || val.size() > 4 || val.find_first_not_of("01") != std::string::npos)
        return FFT_ERR_INVALID_ARGUMENT;
      o->xcd = val;
    } else if (key == "col3") {
      if (val != "0" && val != "1") return FFT_ERR_INVALID_ARGUMENT;
      o->col3 = val == "1";
    } else if (key == "blk") {
      if (val == "0") o->blk = 0;
      else if (val == "8") o->blk = 8;
      else if (val == "16") o->blk = 16;
      else if (val == "32") o->blk = 32;
      else return FFT_ERR_INVALID_ARGUMENT;
    } else if (key == "rowcol") {
      if (val == "0") o->rowcol = 0;
      else if (val == "2") o->rowcol = 2;
      else if (val == "4") o->rowcol = 4;
      else return FFT_ERR_INVALID_ARGUMENT;
    } else if (key == "method") {
      if (val != "lds" && val != "levels" && val != "mfma" && val != "xlane" && val != "xlane_bperm")
        return FFT_ERR_INVALID_ARGUMENT;
      o->levels = val == "levels";
      o->mfma = val == "mfma";
      o->xlane = val == "xlane" ? 1 : val == "xlane_bperm" ? 2 : 0;
    } else if (key == "colt") o->colt = val;
    else if (key == "a") o->a = val;
    else if (key == "b") o->b = val;
    else if (key == "row") o->row = val;
    else if (key == "col") o->col = val;
    else if (key == "single") o->single = val;
    else return FFT_ERR_INVALID_ARGUMENT;
  }
  return FFT_OK;
}

// Resolve an override name (must match role, L and dtype) or pick a default.
int choose(const std::string& name, int role, int L, int dtype, int want_w, int64_t lines,
           const Variant** out) {
  if (!name.empty()) {
    const Variant* v = find_by_name(name);
    if (!v || v->role != role || v->L != L || v->dtype != dtype) return FFT_ERR_INVALID_ARGUMENT;
    *out = v;
    return FFT_OK;
  }
  *out = pick(role, L, dtype, want_w, lines);
  return *out ? FFT_OK : FFT_ERR_UNSUPPORTED_SIZE;
}

constexpr int kSingleMaxLog2 = 14;  // one-kernel transforms up to 2^14 points
constexpr int kSplitMinLog2 = 6, kSplitMaxLog2 = 12;

// 1-D lengths beyond two passes of 2^12: N = N1*N2*N3 in three passes, the
// four-step identity applied twice.  With n = N2*N3*n1 + N3*n2 + n3 and
// k = k1 + N1*k2 + N1*N2*k3, W_N^{nk} factors as
//   W_N1^{n1 k1} * W_N^{m k1} (m = N3 n2 + n3) * W_N2^{n2 k2} * W_M^{n3 k2} * W_N3^{n3 k3}
// with M = N2*N3, so
//   pass 1: N1-point columns of x viewed as [N1][M], times W_N^{m k1},
//           stored transposed as T1[m*N1 + k1]           (in -> workspace)
//   pass 2: N2-point columns (line n3*N1 + k1, stride N3*N1), times
//           W_M^{n3 k2}, in place                          (workspace)
//   pass 3: N3-point columns (line k1 of block k2, stride N1), stored at
//           X[k1 + N1 k2 + N1 N2 k3]                       (workspace -> out)
int build_three_pass_1d(int64_t N, int64_t batch, int dtype, const Overrides& ov, Schedule* outp) {
  Schedule& S = *outp;
  const int l = ilog2_64(N);
  const int l1 = ov.split ? ilog2_64(ov.split) : 10;
  const int l2 = ov.split2 ? ilog2_64(ov.split2) : 7;
  const int l3 = l - l1 - l2;
  if ((ov.split && !pow2(ov.split)) || (ov.split2 && !pow2(ov.split2))) return FFT_ERR_INVALID_ARGUMENT;
  if (l1 < 1 || l2 < 1 || l3 < 1 || l1 > kSplitMaxLog2 || l2 > 7 || l3 > kSingleMaxLog2)
    return FFT_ERR_INVALID_ARGUMENT;
  const int64_t N1 = (int64_t)1 << l1, N2 = (int64_t)1 << l2, N3 = (int64_t)1 << l3;
  const int64_t M = N2 * N3;
  PassSpec A, C, B;
  int rc = choose(ov.a, ROLE_SPLIT_A, (int)N1, dtype, 16, M, &A.v);
  if (rc) return rc;
  rc = choose(ov.colt, ROLE_COL_TW, (int)N2, dtype, 64, N3 * N1, &C.v);
  if (rc) return rc;
  rc = choose(ov.b.empty() ? ov.col : ov.b, ROLE_COL, (int)N3, dtype, 16, N1, &B.v);
  if (rc) return rc;
  if (M > INT32_MAX || N3 * N1 > INT32_MAX) return FFT_ERR_UNSUPPORTED_SIZE;
  PassArgs& a = A.args;
  a.in_batch = a.out_batch = N;
  a.in_line = 1;
  a.in_elem = M;
  a.out_line = N1;
  a.out_elem = 1;
  a.lines = (int32_t)M;
  a.tiles_per_batch = (int32_t)((M + A.v->W - 1) / A.v->W);
  a.total_tiles = (int64_t)a.tiles_per_batch * batch;
  a.tw_shift = (l + 1) / 2;
  a.tw_mask = (1 << a.tw_shift) - 1;
  A.tw_N = N;
  A.tw_rows = M;
  A.src = SEL_IN;
  A.dst = SEL_WS;
  A.first = true;
  PassArgs& c = C.args;
  c.in_batch = c.out_batch = N;
  c.in_line = c.out_line = 1;
  c.in_elem = c.out_elem = N3 * N1;
  c.lines = (int32_t)(N3 * N1);
  c.tiles_per_batch = (int32_t)(N3 * N1 / C.v->W);
  c.total_tiles = (int64_t)c.tiles_per_batch * batch;
  c.tw_shift = (l2 + l3 + 1) / 2;
  c.tw_mask = (1 << c.tw_shift) - 1;
  c.tw_line_shift = l1;
  C.tw_N = M;
  C.tw_rows = N3;
  C.src = SEL_WS;
  C.dst = SEL_WS;
  PassArgs& b = B.args;
  b.in_batch = N3 * N1;  // block k2
  b.out_batch = N1;
  b.in_line = b.out_line = 1;
  b.in_elem = N1;
  b.out_elem = N1 * N2;
  b.lines = (int32_t)N1;
  b.tiles_per_batch = (int32_t)((N1 + B.v->W - 1) / B.v->W);
  b.total_tiles = (int64_t)b.tiles_per_batch * N2;  // one transform; launched per transform
  B.per_transform = true;
  B.src = SEL_WS;
  B.dst = SEL_OUT;
  B.last = true;
  if (C.v->W > N3 * N1 || a.total_tiles > INT32_MAX || c.total_tiles > INT32_MAX || b.total_tiles > INT32_MAX)
    return FFT_ERR_UNSUPPORTED_SIZE;
  S.split[0] = N1;
  S.split[1] = M;
  S.always_ws = true;
  S.passes.push_back(A);
  S.passes.push_back(C);
  S.passes.push_back(B);
  return FFT_OK;
}

// Columns of length R = Sq*Sq as two in-place column passes (the
// three-exchange decomposition: the image viewed as [Sq][Sq][C]), then the
// row pass, which also undoes the digit transposition the second column pass
// leaves (row k1*Sq + k2 holds frequency k1 + Sq*k2) by swapping each row
// with its transpose.
int build_three_pass_2d(int64_t R, int64_t C, int64_t batch, int dtype, const Overrides& ov,
                      Schedule* outp) {
  Schedule& S = *outp;
  const int lgR = ilog2_64(R);
  if ((lgR & 1) || lgR < 2 || C < 2) return FFT_ERR_INVALID_ARGUMENT;
  const int64_t Sq = (int64_t)1 << (lgR / 2);
  if (Sq * C > INT32_MAX || R * batch > INT32_MAX) return FFT_ERR_UNSUPPORTED_SIZE;
  PassSpec c1, c2, rw;
  int rc = choose(ov.colt, ROLE_COL_TW, (int)Sq, dtype, 64, C, &c1.v);
  if (rc) return rc;
  rc = choose(ov.col, ROLE_COL, (int)Sq, dtype, 64, C, &c2.v);
  if (rc) return rc;
  rc = choose(ov.row, ROLE_ROW, (int)C, dtype, 2, R, &rw.v);
  if (rc) return rc;
  // row tiles of an even number of rows never split a transpose pair (the
  // map lists the pairs first, then the diagonal rows), and whole tiles
  // cover the R rows of an image
  if (c1.v->W > C || c2.v->W > C || (rw.v->W & 1) || R % rw.v->W) return FFT_ERR_INVALID_ARGUMENT;
  // pass 1: line (n2, c) at offset n2*C + c, points n1 at stride Sq*C;
  // times W_R^{n2*k1}, n2 = line >> log2(C)
  PassArgs& a1 = c1.args;
  a1.in_batch = a1.out_batch = R * C;
  a1.in_line = a1.out_line = 1;
  a1.in_elem = a1.out_elem = Sq * C;
  a1.lines = (int32_t)(Sq * C);
  a1.tiles_per_batch = (int32_t)(Sq * C / c1.v->W);
  a1.total_tiles = (int64_t)a1.tiles_per_batch * batch;
  a1.tw_shift = (lgR + 1) / 2;
  a1.tw_mask = (1 << a1.tw_shift) - 1;
  a1.tw_line_shift = ilog2_64(C);
  c1.tw_N = R;
  c1.tw_rows = Sq;
  c1.src = SEL_IN;
  c1.dst = SEL_OUT;
  // pass 2: for each block k1 of Sq rows: line c, points n2 at stride C
  PassArgs& a2 = c2.args;
  a2.in_batch = a2.out_batch = Sq * C;
  a2.in_line = a2.out_line = 1;
  a2.in_elem = a2.out_elem = C;
  a2.lines = (int32_t)C;
  a2.tiles_per_batch = (int32_t)(C / c2.v->W);
  a2.total_tiles = (int64_t)a2.tiles_per_batch * batch * Sq;
  c2.src = SEL_OUT;
  c2.dst = SEL_OUT;
  // pass 3: rows, each tile a set of rows closed under transposition
  PassArgs& a3 = rw.args;
  a3.in_batch = a3.out_batch = R * C;
  a3.in_line = a3.out_line = C;
  a3.in_elem = a3.out_elem = 1;
  a3.lines = (int32_t)R;
  a3.tiles_per_batch = (int32_t)(R / rw.v->W);
  a3.total_tiles = (int64_t)a3.tiles_per_batch * batch;
  a3.tr_shift = lgR / 2;
  std::vector<int32_t>& mp = rw.line_map;
  for (int64_t x = 0; x < Sq; ++x)
    for (int64_t y = x + 1; y < Sq; ++y) {
      mp.push_back((int32_t)(x * Sq + y));
      mp.push_back((int32_t)(y * Sq + x));
    }
  for (int64_t x = 0; x < Sq; ++x) mp.push_back((int32_t)(x * Sq + x));
  rw.src = SEL_OUT;
  rw.dst = SEL_OUT;
  if (c1.args.total_tiles > INT32_MAX || c2.args.total_tiles > INT32_MAX) return FFT_ERR_UNSUPPORTED_SIZE;
  S.passes.push_back(c1);
  S.passes.push_back(c2);
  S.passes.push_back(rw);
  S.passes.front().first = true;
  S.passes.back().last = true;
  return FFT_OK;
}

int build_schedule_inner(const int64_t* n, int64_t batch, int dims, int dtype, const Overrides& ov,
                         Schedule* out) {
  Schedule S;
  if (dims == 1) {
    const int64_t N = n[0];
    if (ov.rowcol) return FFT_ERR_INVALID_ARGUMENT;  // 2-D only
    if (!pow2(N) || ilog2_64(N) > FFT_MAX_LOG2_1D) return FFT_ERR_UNSUPPORTED_SIZE;
    if (batch > ((int64_t)1 << 40) / N) return FFT_ERR_UNSUPPORTED_SIZE;
    S.points = N * batch;
    const int l = ilog2_64(N);
    if (ov.levels && N > 1) {
      S.levels = true;
      *out = S;
      return FFT_OK;
    }
    if (ov.mfma || ov.xlane) {
      if (N != 256 || dtype != FFT_C64) return FFT_ERR_INVALID_ARGUMENT;
      S.mfma = ov.mfma;
      S.xlane = ov.xlane;
      *out = S;
      return FFT_OK;
    }
    if (l > 2 * kSplitMaxLog2 || ov.split2) {
      int rc = build_three_pass_1d(N, batch, dtype, ov, &S);
      if (rc) return rc;
      *out = S;
      return FFT_OK;
    }
    if (N == 1) {
      PassSpec p;
      p.copy_n = batch;
      p.first = p.last = true;
      S.passes.push_back(p);
    } else if (l <= kSingleMaxLog2 && ov.split == 0) {
      PassSpec p;
      int rc = choose(ov.single.empty() ? ov.row : ov.single, ROLE_ROW, (int)N, dtype, 64, batch, &p.v);
      if (rc) return rc;
      PassArgs& a = p.args;
      a.in_batch = a.out_batch = 0;
      a.in_line = a.out_line = N;
      a.in_elem = a.out_elem = 1;
      a.lines = (int32_t)std::min<int64_t>(batch, INT32_MAX);
      if (batch > INT32_MAX) return FFT_ERR_UNSUPPORTED_SIZE;
      a.tiles_per_batch = (int32_t)((batch + p.v->W - 1) / p.v->W);
      a.total_tiles = a.tiles_per_batch;
      p.first = p.last = true;
      S.passes.push_back(p);
    } else {
      int64_t N1 = ov.split ? ov.split : ((int64_t)1 << ((l + 1) / 2));
      if (!pow2(N1) || N1 < 2 || N1 >= N) return FFT_ERR_INVALID_ARGUMENT;
      int64_t N2 = N / N1;
      if (ilog2_64(N1) > kSingleMaxLog2 || ilog2_64(N2) > kSingleMaxLog2) return FFT_ERR_UNSUPPORTED_SIZE;
      S.split[0] = N1;
      S.split[1] = N2;
      PassSpec A, B;
      int rc = choose(ov.a, ROLE_SPLIT_A, (int)N1, dtype, 16, N2, &A.v);
      if (rc) return rc;
      rc = choose(ov.b.empty() ? ov.col : ov.b, ROLE_COL, (int)N2, dtype, 16, N1, &B.v);
      if (rc) return rc;
      // pass A: x viewed as [N1][N2]; line n2 (column), point n1; writes
      // T[n2*N1 + k1] times W_N^{n2*k1}.
      PassArgs& a = A.args;
      a.in_batch = a.out_batch = N;
      a.in_line = 1;
      a.in_elem = N2;
      a.out_line = N1;
      a.out_elem = 1;
      a.lines = (int32_t)N2;
      a.tiles_per_batch = (int32_t)((N2 + A.v->W - 1) / A.v->W);
      a.total_tiles = (int64_t)a.tiles_per_batch * batch;
      a.tw_shift = (l + 1) / 2;
      a.tw_mask = (1 << a.tw_shift) - 1;
      A.tw_N = N;
      A.tw_rows = N2;
      A.first = true;
      // pass B: T viewed as [N2][N1]; line k1 (column), point n2; writes
      // X[k1 + N1*k2] in place of its own columns.
      PassArgs& b = B.args;
      b.in_batch = b.out_batch = N;
      b.in_line = b.out_line = 1;
      b.in_elem = b.out_elem = N1;
      b.lines = (int32_t)N1;
      b.tiles_per_batch = (int32_t)((N1 + B.v->W - 1) / B.v->W);
      b.total_tiles = (int64_t)b.tiles_per_batch * batch;
      B.last = true;
      A.src = SEL_IN;
      A.dst = SEL_OUT;
      B.src = SEL_OUT;
      B.dst = SEL_OUT;
      S.inplace_needs_ws = true;
      S.passes.push_back(A);
      S.passes.push_back(B);
      if (a.total_tiles > INT32_MAX || b.total_tiles > INT32_MAX) return FFT_ERR_UNSUPPORTED_SIZE;
    }
  } else {
    const int64_t R = n[0], C = n[1];
    if (ov.levels || ov.mfma || ov.xlane) return FFT_ERR_INVALID_ARGUMENT;  // 1-D only
    if (!pow2(R) || !pow2(C) || ilog2_64(R) > FFT_MAX_LOG2_2D || ilog2_64(C) > FFT_MAX_LOG2_2D)
      return FFT_ERR_UNSUPPORTED_SIZE;
    if (batch > ((int64_t)1 << 40) / (R * C)) return FFT_ERR_UNSUPPORTED_SIZE;
    S.points = R * C * batch;
    const int lgR = ilog2_64(R);
    if (ov.rowcol) {
      // rows fused with the first radix-r step of the columns (R = r*M),
      // then M-point columns over rows r*n1 + k2 for each k2, in place
      const int r = ov.rowcol;
      if (ov.col3 == 1 || ov.blk || R < 2 * r || C < 2) return FFT_ERR_INVALID_ARGUMENT;
      const int64_t M = R / r;
      PassSpec f, cl;
      if (!ov.row.empty()) {
        f.v = find_by_name(ov.row);
        if (!f.v || f.v->role != ROLE_ROWCOL || f.v->L != C || f.v->dtype != dtype) return FFT_ERR_INVALID_ARGUMENT;
      } else {
        // the first registered fused variant of this row length and radix
        for (const Variant& v : variants())
          if (v.role == ROLE_ROWCOL && v.L == C && v.dtype == dtype && v.W == r) {
            f.v = &v;
            break;
          }
        if (!f.v) return FFT_ERR_UNSUPPORTED_SIZE;
      }
      if (f.v->W != r) return FFT_ERR_INVALID_ARGUMENT;
      int rc;
      rc = choose(ov.col, ROLE_COL, (int)M, dtype, 16, C, &cl.v);
      if (rc) return rc;
      if (M * batch > INT32_MAX) return FFT_ERR_UNSUPPORTED_SIZE;
      PassArgs& a = f.args;
      a.in_batch = a.out_batch = R * C;
      a.in_line = a.out_line = C;
      a.in_elem = a.out_elem = 1;
      a.lines = (int32_t)R;
      a.tiles_per_batch = (int32_t)M;
      a.total_tiles = M * batch;
      a.tw_shift = ilog2_64(M);
      f.colr_N = R;
      f.scale_len = r * C;
      f.src = SEL_IN;
      f.dst = SEL_OUT;
      f.first = true;
      // columns: line c, points k1 at stride r*C; block k2 starts at row k2
      // (one image per launch when batched)
      PassArgs& b = cl.args;
      b.in_line = b.out_line = 1;
      b.in_elem = b.out_elem = r * C;
      b.in_batch = b.out_batch = C;
      b.lines = (int32_t)C;
      b.tiles_per_batch = (int32_t)((C + cl.v->W - 1) / cl.v->W);
      b.total_tiles = (int64_t)b.tiles_per_batch * r;
      cl.per_transform = true;
      cl.src = SEL_OUT;
      cl.dst = SEL_OUT;
      cl.last = true;
      S.inplace_needs_ws = true;
      S.passes.push_back(f);
      S.passes.push_back(cl);
      *out = S;
      return FFT_OK;
    }
    if (ov.blk) {
      // the intermediate in column blocks (row pass -> workspace, column
      // pass -> out): every column tile then reads one contiguous block
      if (ov.col3 == 1 || R < 2 || C < ov.blk || C % ov.blk) return FFT_ERR_INVALID_ARGUMENT;
      PassSpec rw, cl;
      int rc = choose(ov.row, ROLE_ROW, (int)C, dtype, 64, R * batch, &rw.v);
      if (rc) return rc;
      rc = choose(ov.col, ROLE_COL, (int)R, dtype, ov.blk, ov.blk, &cl.v);
      if (rc) return rc;
      const int64_t T = C / rw.v->P;  // lanes per row (C >= P for every row variant with C >= 8)
      if (rw.v->P > C || T % ov.blk || ov.blk % cl.v->W || R * batch > INT32_MAX) return FFT_ERR_INVALID_ARGUMENT;
      PassArgs& a = rw.args;
      a.in_batch = a.out_batch = 0;
      a.in_line = a.out_line = C;
      a.in_elem = a.out_elem = 1;
      a.lines = (int32_t)(R * batch);
      a.tiles_per_batch = (int32_t)((R * batch + rw.v->W - 1) / rw.v->W);
      a.total_tiles = a.tiles_per_batch;
      a.blk_lg = ilog2_64(ov.blk);
      a.blk_rows_lg = lgR;
      rw.src = SEL_IN;
      rw.dst = SEL_WS;
      rw.first = true;
      // column pass, per image: block j (R rows of blk columns, contiguous)
      // is one "batch" of blk lines
      PassArgs& b = cl.args;
      b.in_batch = R * ov.blk;
      b.out_batch = ov.blk;
      b.in_line = b.out_line = 1;
      b.in_elem = ov.blk;
      b.out_elem = C;
      b.lines = ov.blk;
      b.tiles_per_batch = ov.blk / cl.v->W;
      b.total_tiles = (int64_t)b.tiles_per_batch * (C / ov.blk);
      cl.src = SEL_WS;
      cl.dst = SEL_OUT;
      cl.last = true;
      cl.per_transform = true;
      S.always_ws = true;
      S.passes.push_back(rw);
      S.passes.push_back(cl);
      *out = S;
      return FFT_OK;
    }
    const bool three = ov.col3 == 1 ? true
                       : ov.col3 == 0 ? false
                                      : (lgR >= 12 && C >= 16);
    if (three) {
      Schedule S3 = S;
      int rc3 = build_three_pass_2d(R, C, batch, dtype, ov, &S3);
      if (rc3 == FFT_OK) {
        *out = S3;
        return FFT_OK;
      }
      if (ov.col3 == 1) return rc3;  // asked for explicitly: report why not
    }
    if (C > 1) {
      PassSpec p;
      int rc = choose(ov.row, ROLE_ROW, (int)C, dtype, 64, R * batch, &p.v);
      if (rc) return rc;
      PassArgs& a = p.args;
      a.in_batch = a.out_batch = 0;
      a.in_line = a.out_line = C;
      a.in_elem = a.out_elem = 1;
      if (R * batch > INT32_MAX) return FFT_ERR_UNSUPPORTED_SIZE;
      a.lines = (int32_t)(R * batch);
      a.tiles_per_batch = (int32_t)((R * batch + p.v->W - 1) / p.v->W);
      a.total_tiles = a.tiles_per_batch;
      p.src = SEL_IN;
      p.dst = SEL_OUT;
      S.passes.push_back(p);
    }
    if (R > 1) {
      PassSpec p;
      int rc = choose(ov.col, ROLE_COL, (int)R, dtype, 16, C, &p.v);
      if (rc) return rc;
      PassArgs& a = p.args;
      a.in_batch = a.out_batch = R * C;
      a.in_line = a.out_line = 1;
      a.in_elem = a.out_elem = C;
      a.lines = (int32_t)C;
      a.tiles_per_batch = (int32_t)((C + p.v->W - 1) / p.v->W);
      a.total_tiles = (int64_t)a.tiles_per_batch * batch;
      if (a.total_tiles > INT32_MAX) return FFT_ERR_UNSUPPORTED_SIZE;
      p.src = S.passes.empty() ? SEL_IN : SEL_OUT;
      p.dst = SEL_OUT;
      S.passes.push_back(p);
    }
    if (S.passes.empty()) {
      PassSpec p;
      p.copy_n = batch;
      S.passes.push_back(p);
    }
    S.passes.front().first = true;
    S.passes.back().last = true;
  }
  *out = S;
  return FFT_OK;
}

int apply_xcd(const std::string& mask, Schedule* S) {
  if (S->levels || S->mfma || S->xlane) return mask == "0" || mask == "1" ? FFT_OK : FFT_ERR_INVALID_ARGUMENT;
  const size_t n = S->passes.size();
  if (mask.size() != 1 && mask.size() != n) return FFT_ERR_INVALID_ARGUMENT;
  for (size_t i = 0; i < n; ++i)
    S->passes[i].args.xcd_remap = (mask.size() == 1 ? mask[0] : mask[i]) == '1';
  return FFT_OK;
}

int build_schedule(const int64_t* n, int64_t batch, int dims, int dtype, const char* sched,
                   Schedule* out) {
  if (!n || batch < 1 || (dims != 1 && dims != 2)) return FFT_ERR_INVALID_ARGUMENT;
  if (dtype != FFT_C64 && dtype != FFT_C16F && dtype != FFT_C16BF) return FFT_ERR_INVALID_ARGUMENT;
  Overrides ov;
  if (parse_schedule(sched, &ov) != FFT_OK) return FFT_ERR_INVALID_ARGUMENT;
  Schedule S;
  int rc = build_schedule_inner(n, batch, dims, dtype, ov, &S);
  if (rc) return rc;
  rc = apply_xcd(ov.xcd, &S);
  if (rc) return rc;
  *out = S;
  return FFT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// plan object
// ---------------------------------------------------------------------------
struct fft_plan_s {
  int kind = 0;  // 0 = strided passes, 1 = batched uneven (many), 2 = per-level method,
                 // 3 = matrix-core 256-point transforms
  void* lv_buf = nullptr;  // kind 2: ping-pong buffer (also listed in aux)
  int cus = 0;
  int64_t n[2] = {1, 1};
  int dims = 1, dtype = 0, direction = -1;
  int64_t batch = 1;
  double scale = 1.0;
  bool scale_user = false;
  Schedule sched;
  float2* d_tables = nullptr;
  size_t table_bytes = 0;
  std::vector<void*> aux;  // other plan-owned device buffers (row maps)
  bool gpu_twiddles = false;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  int device = 0;
  // profiling: a ring of `prof_slots` exec slots, 2 events per launch each
  bool prof = false;
  int prof_slots = 0, prof_next = 0, prof_pending = 0;
  int prof_every = 1;    // time one exec in `prof_every`
  int64_t prof_seq = 0;  // execs seen since timing was enabled
  bool prof_take = false;
  size_t prof_npass = 0;
  std::vector<hipEvent_t> ev;
  std::vector<double> prof_ms;
  std::vector<int64_t> prof_n;
  // batched uneven sizes
  ManyPlan many;
};

namespace {

// Append (L, P) stage tables and the split's inter-pass tables to `segs`,
// recording offsets in the pass arguments (resolved to pointers later).
struct TableBuild {
  std::vector<TwSeg> segs;
  int64_t total = 0;
  std::map<std::pair<int, int>, int64_t> stage_off;
  int64_t add(int64_t count, int64_t R, int64_t M, int64_t mul) {
    TwSeg s{total, count, R, M, mul};
    segs.push_back(s);
    total += count;
    return s.off;
  }
  // one segment per stage s >= 1 of the (L, P) schedule
  int64_t add_stage_table(int L, int P) {
    auto key = std::make_pair(L, P);
    auto it = stage_off.find(key);
    if (it != stage_off.end()) return it->second;
    const int lp = ilog2(P < L ? P : L);
    const int PP = 1 << lp;
    const int S = (ilog2(L) + lp - 1) / lp;
    const int FIRST = L >> ((S - 1) * lp);
    const int64_t start = total;
    int ns = FIRST;
    for (int s = 1; s < S; ++s) {
      add((int64_t)ns * PP, PP, (int64_t)ns * PP, 1);
      ns *= PP;
    }
    if (total == start) add(1, 0, 1, 0);  // one-stage transform: placeholder entry
    stage_off[key] = start;
    return start;
  }
};

void host_fill(const std::vector<TwSeg>& segs, std::vector<float2>& tab) {
  for (const TwSeg& s : segs)
    for (int64_t i = 0; i < s.count; ++i) {
      double c, sn;
      twiddle_fp64(seg_exponent(s, i), s.M, &c, &sn);
      tab[s.off + i] = make_float2((float)c, (float)-sn);
    }
}

int upload_tables(fft_plan_s* p, TableBuild& tb, bool on_gpu) {
  const size_t bytes = (size_t)std::max<int64_t>(tb.total, 1) * sizeof(float2);
  hipError_t e = hipMalloc((void**)&p->d_tables, bytes);
  if (e != hipSuccess) {
    p->d_tables = nullptr;
    return e == hipErrorOutOfMemory ? FFT_ERR_NO_MEMORY : hip_fail(e);
  }
  p->table_bytes = bytes;
  if (!on_gpu) {
    std::vector<float2> tab((size_t)std::max<int64_t>(tb.total, 1));
    host_fill(tb.segs, tab);
    e = hipMemcpy(p->d_tables, tab.data(), (size_t)tb.total * sizeof(float2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
    return FFT_OK;
  }
  // float64 generation on the GPU: upload the segment list, run the kernel
  TwSeg* d_segs = nullptr;
  e = hipMalloc((void**)&d_segs, tb.segs.size() * sizeof(TwSeg));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? FFT_ERR_NO_MEMORY : hip_fail(e);
  e = hipMemcpy(d_segs, tb.segs.data(), tb.segs.size() * sizeof(TwSeg), hipMemcpyHostToDevice);
  int64_t maxc = 1;
  for (const TwSeg& s : tb.segs) maxc = std::max(maxc, s.count);
  if (e == hipSuccess) e = launch_twiddle_fp64(p->d_tables, d_segs, (int)tb.segs.size(), maxc, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  hipFree(d_segs);
  if (e != hipSuccess) return hip_fail(e);
  p->gpu_twiddles = true;
  return FFT_OK;
}

void set_default_scale(fft_plan_s* p) {
  double total = 1;
  if (p->kind == 0) total = (double)p->n[0] * (double)(p->dims == 2 ? p->n[1] : 1);
  p->scale = p->direction > 0 ? 1.0 / total : 1.0;
}

int check_ptr(const void* ptr, int dtype) {
  return ((uintptr_t)ptr % esize(dtype)) ? FFT_ERR_ALIGNMENT : FFT_OK;
}

constexpr int kGpuTwiddleMinLog2 = 22;
constexpr int64_t kManyWaitDefaultUs = 2000000;  // 2 s per dependency wait

}  // namespace

// ---------------------------------------------------------------------------
// batched uneven sizes: host side of the persistent launch
// ---------------------------------------------------------------------------
namespace mfft {

size_t many_workspace_bytes(const ManyPlan& mp) {
  return (size_t)(kManyWsHeader + mp.count + kManyMaxQueues) * sizeof(int32_t);
}

hipError_t many_reset_workspace(const ManyPlan& mp, void* ws) {
  return hipMemset(ws, 0, many_workspace_bytes(mp));
}

int many_alloc_workspace(const ManyPlan& mp, void** ws, size_t* bytes) {
  const size_t b = many_workspace_bytes(mp);
  hipError_t e = hipMalloc(ws, b);
  if (e != hipSuccess) {
    *ws = nullptr;
    if (e == hipErrorOutOfMemory) return FFT_ERR_NO_MEMORY;
    g_last_hip = (int)e;
    return FFT_ERR_HIP;
  }
  e = hipMemset(*ws, 0, b);
  if (e != hipSuccess) {
    hipFree(*ws);
    *ws = nullptr;
    g_last_hip = (int)e;
    return FFT_ERR_HIP;
  }
  *bytes = b;
  return FFT_OK;
}

hipError_t many_launch(const ManyPlan& mp, const void* in, void* out, void* ws, int32_t* watchdog,
                       float scale, bool use_scale, bool inverse, hipStream_t s) {
  if (!ws) return hipErrorInvalidValue;
  ManyArgs a = mp.args;
  a.in = in;
  a.out = out;
  a.ws = (int32_t*)ws;
  a.watchdog = watchdog ? watchdog : (int32_t*)ws + 2;
  a.scale = scale;
  a.use_scale = use_scale ? 1 : 0;
  a.inverse = inverse ? 1 : 0;
  return mp.var->launch(a, mp.grid, s);
}

void many_free(ManyPlan& mp) {
  if (mp.d_items) hipFree(mp.d_items);
  if (mp.d_itx) hipFree(mp.d_itx);
  if (mp.d_q_off) hipFree(mp.d_q_off);
  mp.d_itx = nullptr;
  mp.d_q_off = nullptr;
  if (mp.d_xf) hipFree(mp.d_xf);
  if (mp.d_order) hipFree(mp.d_order);
  if (mp.d_order_off) hipFree(mp.d_order_off);
  if (mp.d_tw_img) hipFree(mp.d_tw_img);
  mp.d_items = nullptr;
  mp.d_xf = nullptr;
  mp.d_order = nullptr;
  mp.d_order_off = nullptr;
  mp.d_tw_img = nullptr;
  mp.active = false;
}

}  // namespace mfft

namespace {

struct ManyOptions {
  int P = 16, threads = 512, pass2 = 0;  // pass2 0: two passes above the longest one-tile length
  bool given_order = false;
  // 0: shared queue with completion counters; 1: software-pipelined, one
  // workgroup per CU, round-robin items, completion counters; 2 (default):
  // software-pipelined, two launches per exec, no waits
  int pipe = 2;
  // 0: every first-pass tile ahead of every second-pass tile; k > 0: the
  // second-pass tiles of split transform i follow the first-pass tiles of
  // split transform i + k, so its intermediate is still in the last-level
  // cache when it is read back
  int lag = 0;
  // per length 2^L: two passes forced (2) or refused (1), 0 = by `pass2`;
  // and log2 of the first-pass length N1 of a two-pass transform (0 = the
  // default, ceil(L/2) capped at the longest tile)
  int passes_for[FFT_MAX_LOG2_1D + 1] = {};
  // two-launch kernel: stores with the nontemporal hint for every item, or
  // for the last `nt_tail` items of each launch (what is still dirty in the
  // caches when a launch ends is written back before the next one starts)
  int nt_store = 0;
  int nt_tail = 0;
  int lg1_for[FFT_MAX_LOG2_1D + 1] = {};
};

int parse_many_schedule(const char* s, ManyOptions* o) {
  if (!s) return FFT_OK;
  std::string str(s);
  size_t pos = 0;
  while (pos < str.size()) {
    size_t end = str.find(';', pos);
    if (end == std::string::npos) end = str.size();
    std::string item = str.substr(pos, end - pos);
    pos = end + 1;
    if (item.empty()) continue;
    size_t eq = item.find('=');
    if (eq == std::string::npos) return FFT_ERR_INVALID_ARGUMENT;
    std::string key = item.substr(0, eq), val = item.substr(eq + 1);
    if (key == "order") {
      if (val == "given") o->given_order = true;
      else if (val == "bigfirst") o->given_order = false;
      else return FFT_ERR_INVALID_ARGUMENT;
      continue;
    }
    char* e = nullptr;
    long v = strtol(val.c_str(), &e, 10);
    if (!e || *e) return FFT_ERR_INVALID_ARGUMENT;
    // per-length items: 'n1.L=l1' and 'pass.L=1|2'
    const size_t dot = key.find('.');
    if (dot != std::string::npos) {
      const std::string k0 = key.substr(0, dot), k1 = key.substr(dot + 1);
      char* e2 = nullptr;
      const long L = strtol(k1.c_str(), &e2, 10);
      if (k1.empty() || !e2 || *e2 || L < 1 || L > FFT_MAX_LOG2_1D) return FFT_ERR_INVALID_ARGUMENT;
      if (k0 == "n1") {
        if (v < 1 || v >= L) return FFT_ERR_INVALID_ARGUMENT;
        o->lg1_for[L] = (int)v;
      } else if (k0 == "pass") {
        if (v != 1 && v != 2) return FFT_ERR_INVALID_ARGUMENT;
        o->passes_for[L] = (int)v;
      } else {
        return FFT_ERR_INVALID_ARGUMENT;
      }
      continue;
    }
    if (key == "p") o->P = (int)v;
    else if (key == "threads") o->threads = (int)v;
    else if (key == "pass2") {
      if (v < 1) return FFT_ERR_INVALID_ARGUMENT;
      o->pass2 = (int)v;
    } else if (key == "pipe") {
      if (v < 0 || v > 2) return FFT_ERR_INVALID_ARGUMENT;
      o->pipe = (int)v;

    } else if (key == "ntst") {
      if (v != 0 && v != 1) return FFT_ERR_INVALID_ARGUMENT;
      o->nt_store = (int)v;
    } else if (key == "ntail") {
      if (v < 0 || v > (1 << 24)) return FFT_ERR_INVALID_ARGUMENT;
      o->nt_tail = (int)v;
    } else if (key == "lag") {
      if (v < 0 || v > (1 << 24)) return FFT_ERR_INVALID_ARGUMENT;
      o->lag = (int)v;
    }
    else return FFT_ERR_INVALID_ARGUMENT;
  }
  return FFT_OK;
}

// lines of a 2^lg tile in a workgroup of `threads` lanes, P points per lane
int tile_lines(int lg, int P, int threads) {
  if (lg == 0) return threads;
  const int L = 1 << lg;
  const int T = L / std::min(P, L);
  return threads / T;
}

}  // namespace

namespace {

// Event pair array of the next profiling slot, or nullptr when profiling is off.
// Timing events are not recorded into a stream that is being captured into
// a graph (their elapsed times cannot be read back from graph replays).
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

hipEvent_t* prof_slot(fft_plan_s* p, hipStream_t s) {
  p->prof_take = false;
  if (!p->prof || p->prof_slots <= 0 || capturing(s)) return nullptr;
  p->prof_take = p->prof_seq++ % p->prof_every == 0;
  return p->prof_take ? p->ev.data() + (size_t)p->prof_next * 2 * p->prof_npass : nullptr;
}

void prof_commit(fft_plan_s* p, hipStream_t) {
  if (!p->prof_take) return;
  p->prof_take = false;
  p->prof_next = (p->prof_next + 1) % p->prof_slots;
  p->prof_pending = std::min(p->prof_pending + 1, p->prof_slots);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int fft_plan_ex(const int64_t* n, int64_t batch, int dims, int dtype, int direction,
                const char* schedule, fft_plan_t* out) {
  if (!out) return FFT_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (direction != FFT_FORWARD && direction != FFT_INVERSE) return FFT_ERR_INVALID_ARGUMENT;
  Schedule S;
  int rc = build_schedule(n, batch, dims, dtype, schedule, &S);
  if (rc) return rc;
  fft_plan_s* p = new (std::nothrow) fft_plan_s();
  if (!p) return FFT_ERR_NO_MEMORY;
  p->kind = S.levels ? 2 : (S.mfma || S.xlane) ? 3 : 0;
  p->dims = dims;
  p->n[0] = n[0];
  p->n[1] = dims == 2 ? n[1] : 1;
  p->batch = batch;
  p->dtype = dtype;
  p->direction = direction;
  p->sched = S;
  set_default_scale(p);
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e);
  }
  // twiddle tables
  TableBuild tb;
  std::vector<int64_t> stage_off(S.passes.size(), 0);
  std::vector<int64_t> lo_off(S.passes.size(), -1), hi_off(S.passes.size(), -1),
      step_off(S.passes.size(), -1);
  for (size_t i = 0; i < S.passes.size(); ++i) {
    const PassSpec& ps = S.passes[i];
    if (!ps.v) continue;
    if (ps.v->tw_split) {
      // the two factor tables of W_L: W_L^i (i < 2^a), W_L^{i 2^a}
      const int lg = ilog2_64(ps.v->L), la = (lg + 1) / 2;
      stage_off[i] = tb.add((int64_t)1 << la, 0, ps.v->L, 1);
      tb.add((int64_t)1 << (lg - la), 0, ps.v->L, (int64_t)1 << la);
    } else {
      stage_off[i] = tb.add_stage_table(ps.v->L, ps.v->P);
    }
    if (ps.tw_N) {
      // W_M^{row*k} with k = t + q*T: a per-lane base W_M^{row*t} (lo/hi
      // factors) times a per-row step W_M^{row*q*T} (table [rows][P])
      const int64_t M = ps.tw_N;
      const int sh = ps.args.tw_shift;
      const int64_t T = ps.v->L / ps.v->P;
      lo_off[i] = tb.add((int64_t)1 << sh, 0, M, 1);
      hi_off[i] = tb.add(M >> sh, 0, M, (int64_t)1 << sh);
      step_off[i] = tb.add(ps.tw_rows * ps.v->P, ps.v->P, M, T);
    }
    if (ps.colr_N) lo_off[i] = tb.add(ps.colr_N, 0, ps.colr_N, 1);  // W_R^e, e < R
  }
  if (S.levels) tb.add(n[0] / 2, 0, n[0], 1);  // W_N^m, m < N/2
  if (S.mfma || S.xlane) tb.add(256, 0, 256, 1);          // W_256^m, m < 256
  const bool on_gpu = dims == 1 && ilog2_64(n[0]) >= kGpuTwiddleMinLog2;
  rc = upload_tables(p, tb, on_gpu);
  if (rc) {
    fft_destroy(p);
    return rc;
  }
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) {
    fft_destroy(p);
    return hip_fail(e);
  }
  p->cus = cus;
  if (S.always_ws) {
    // plan-owned workspace (the caller may replace it with fft_set_workspace)
    const size_t bytes = (size_t)S.points * esize(dtype);
    e = hipMalloc(&p->ws, bytes);
    if (e != hipSuccess) {
      p->ws = nullptr;
      fft_destroy(p);
      return e == hipErrorOutOfMemory ? FFT_ERR_NO_MEMORY : hip_fail(e);
    }
    p->ws_bytes = bytes;
    p->ws_owned = true;
  }
  if (S.levels) {
    e = hipMalloc(&p->lv_buf, (size_t)S.points * esize(dtype));
    if (e != hipSuccess) {
      p->lv_buf = nullptr;
      fft_destroy(p);
      return e == hipErrorOutOfMemory ? FFT_ERR_NO_MEMORY : hip_fail(e);
    }
    p->aux.push_back(p->lv_buf);
  }
  for (size_t i = 0; i < p->sched.passes.size(); ++i) {
    PassSpec& ps = p->sched.passes[i];
    if (!ps.v) continue;
    if (ps.v->persistent) {
      // persistent variants launch the resident workgroups only
      const int per_cu = std::max(1, ps.v->blocks_per_cu());
      ps.args.grid = (int32_t)std::min<int64_t>(ps.args.total_tiles, (int64_t)per_cu * cus);
    }
    ps.args.tw = p->d_tables + stage_off[i];
    if (ps.tw_N) {
      ps.args.tw_lo = p->d_tables + lo_off[i];
      ps.args.tw_hi = p->d_tables + hi_off[i];
      ps.args.tw_step = p->d_tables + step_off[i];
    }
    if (ps.colr_N) ps.args.tw_lo = p->d_tables + lo_off[i];
    if (!ps.line_map.empty()) {
      const size_t bytes = ps.line_map.size() * sizeof(int32_t);
      int32_t* d = nullptr;
      e = hipMalloc((void**)&d, bytes);
      if (e == hipSuccess) e = hipMemcpy(d, ps.line_map.data(), bytes, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        if (d) hipFree(d);
        fft_destroy(p);
        return e == hipErrorOutOfMemory ? FFT_ERR_NO_MEMORY : hip_fail(e);
      }
      p->aux.push_back(d);
      ps.args.line_map = d;
    }
  }
  *out = p;
  return FFT_OK;
}

int fft_plan(const int64_t* n, int64_t batch, int dims, int dtype, int direction, fft_plan_t* out) {
  return fft_plan_ex(n, batch, dims, dtype, direction, nullptr, out);
}

int fft_set_scale(fft_plan_t p, double scale) {
  if (!p || !std::isfinite(scale)) return FFT_ERR_INVALID_ARGUMENT;
  p->scale = scale;
  p->scale_user = true;
  return FFT_OK;
}

int fft_workspace_size(fft_plan_t p, size_t* bytes) {
  if (!p || !bytes) return FFT_ERR_INVALID_ARGUMENT;
  if (p->kind == 1) *bytes = many_workspace_bytes(p->many);
  else *bytes = (p->sched.inplace_needs_ws || p->sched.always_ws) ? (size_t)p->sched.points * esize(p->dtype) : 0;
  return FFT_OK;
}

int fft_set_workspace(fft_plan_t p, void* ptr, size_t bytes) {
  if (!p) return FFT_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  fft_workspace_size(p, &need);
  if (ptr && bytes < need) return FFT_ERR_INVALID_ARGUMENT;
  if (ptr && ((uintptr_t)ptr % 16)) return FFT_ERR_ALIGNMENT;
  if (p->ws_owned && p->ws) {
    hipFree(p->ws);
  }
  p->ws_owned = false;
  p->ws = ptr;
  p->ws_bytes = ptr ? bytes : 0;
  if (!ptr && p->kind == 0 && p->sched.always_ws) {
    // back to a plan-owned workspace
    hipError_t e = hipMalloc(&p->ws, need);
    if (e != hipSuccess) {
      p->ws = nullptr;
      return e == hipErrorOutOfMemory ? FFT_ERR_NO_MEMORY : hip_fail(e);
    }
    p->ws_bytes = need;
    p->ws_owned = true;
  } else if (!ptr && p->kind == 1) {
    // back to a plan-owned queue workspace
    int rc = many_alloc_workspace(p->many, &p->ws, &p->ws_bytes);
    if (rc) return rc == FFT_ERR_HIP ? hip_fail((hipError_t)g_last_hip) : rc;
    p->ws_owned = true;
  } else if (ptr && p->kind == 1) {
    hipError_t e = many_reset_workspace(p->many, ptr);
    if (e != hipSuccess) return hip_fail(e);
  }
  return FFT_OK;
}

namespace {

// Bytes of workspace one exec of `p` with these buffers reads or writes (0:
// none): the batched plan's queue state, the in-place two-pass intermediate,
// or the three-pass intermediate.
size_t exec_scratch_bytes(const fft_plan_s* p, const void* in, const void* out) {
  if (p->kind == 1) return many_workspace_bytes(p->many);
  if (p->kind != 0) return 0;
  const Schedule& S = p->sched;
  const bool ws = S.always_ws || (in == out && S.passes.size() > 1 && S.inplace_needs_ws);
  return ws ? (size_t)S.points * esize(p->dtype) : 0;
}

__global__ void k_zero_words(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// fft_exec with the plan's workspace replaced by `ws_over` when it is not
// NULL (the caller has checked its size); a batched plan's queue state there
// is cleared by a fill kernel first.
int exec_impl(fft_plan_t p, const void* in, void* out, void* stream, void* ws_over) {
  if (!p || !in || !out) return FFT_ERR_INVALID_ARGUMENT;
  if (check_ptr(in, p->dtype) || check_ptr(out, p->dtype)) return FFT_ERR_ALIGNMENT;
  hipStream_t s = (hipStream_t)stream;
  void* const plan_ws = ws_over ? ws_over : p->ws;
  if (p->kind == 1) {
    const size_t mbytes = (size_t)p->many.points * esize(p->dtype);
    const char* mi = (const char*)in;
    const char* mo = (const char*)out;
    if (in != out && mi < mo + mbytes && mo < mi + mbytes) return FFT_ERR_INPLACE;
    if (p->many.has_split && in == out) return FFT_ERR_INPLACE;
    if (ws_over) {
      const int64_t words = (int64_t)(many_workspace_bytes(p->many) / sizeof(uint32_t));
      hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 1024)), dim3(256),
                         0, s, (uint32_t*)ws_over, words);
      hipError_t e0 = hipGetLastError();
      if (e0 != hipSuccess) return hip_fail(e0);
    }
    hipEvent_t* slot = prof_slot(p, s);
    if (slot) hipEventRecord(slot[0], s);
    // with the static scratch, bounded waits flag the plan's own watchdog word
    // (read by fft_many_watchdog) when the plan has a workspace
    int32_t* wd = (ws_over && p->ws) ? (int32_t*)p->ws + 2 : nullptr;
    hipError_t e = many_launch(p->many, in, out, plan_ws, wd, (float)p->scale, p->scale_user,
                               p->direction > 0, s);
    if (slot) hipEventRecord(slot[1], s);
    if (e != hipSuccess) return hip_fail(e);
    prof_commit(p, s);
    return FFT_OK;
  }
  const Schedule& S = p->sched;
  const size_t bytes = (size_t)S.points * esize(p->dtype);
  const char* ib = (const char*)in;
  const char* ob = (const char*)out;
  const bool overlap = ib < ob + bytes && ob < ib + bytes;
  const bool same = in == out;
  if (overlap && !same) return FFT_ERR_INPLACE;
  if (p->kind == 3) {
    hipEvent_t* slot = prof_slot(p, s);
    if (slot) hipEventRecord(slot[0], s);
    const bool inv = p->direction > 0;
    const float sc = p->scale_user ? (float)p->scale : (inv ? 1.0f / 256.0f : 1.0f);
    hipError_t e =
        p->sched.xlane
            ? launch_dft256_xlane(in, out, p->batch, p->d_tables, sc, inv ? 1 : 0, inv ? 1 : 0, p->sched.xlane - 1, s)
            : launch_dft256_mfma(in, out, p->batch, p->d_tables, sc, inv ? 1 : 0, inv ? 1 : 0, s);
    if (slot) hipEventRecord(slot[1], s);
    if (e != hipSuccess) return hip_fail(e);
    prof_commit(p, s);
    return FFT_OK;
  }
  if (p->kind == 2) {
    LevelsArgs la;
    la.in = in;
    la.out = out;
    la.buf = p->lv_buf;
    la.batch = p->batch;
    la.lgN = ilog2_64(p->n[0]);
    la.dtype = p->dtype;
    la.tw = p->d_tables;
    la.scale = (float)p->scale;
    la.user_scale = p->scale_user;
    la.inverse = p->direction > 0;
    la.cus = p->cus;
    hipEvent_t* slot = prof_slot(p, s);
    if (slot) hipEventRecord(slot[0], s);
    hipError_t e = launch_levels(la, s);
    if (slot) hipEventRecord(slot[1], s);
    if (e != hipSuccess) return hip_fail(e);
    prof_commit(p, s);
    return FFT_OK;
  }
  void* ws = nullptr;
  if (same && S.passes.size() > 1 && S.inplace_needs_ws) {
    if (!plan_ws) return FFT_ERR_INPLACE;
    ws = plan_ws;
  }
  if (S.always_ws && !plan_ws) return FFT_ERR_INPLACE;
  const bool inv = p->direction > 0;
  hipEvent_t* slot = prof_slot(p, s);
  for (size_t i = 0; i < S.passes.size(); ++i) {
    const PassSpec& ps = S.passes[i];
    // out of place: each pass reads `in` (first) or `out` and writes `out`;
    // in place with a workspace: A reads in and writes ws, B reads ws, writes out;
    // plans that always use the workspace name their buffers per pass
    void* src;
    void* dst;
    if (S.always_ws) {
      src = ps.src == SEL_IN ? (void*)in : ps.src == SEL_WS ? plan_ws : out;
      dst = ps.dst == SEL_IN ? (void*)in : ps.dst == SEL_WS ? plan_ws : out;
    } else {
      src = ws ? (i == 0 ? (void*)in : ws) : (ps.src == SEL_IN ? (void*)in : out);
      dst = ws ? (i == 0 ? ws : out) : out;
    }
    // a single kernel launch takes the events itself (its own start and end
    // times); a copy or a per-transform loop is bracketed by markers
    const bool one_launch = ps.v && !(ps.per_transform && p->batch > 1);
    if (slot && !one_launch) hipEventRecord(slot[2 * i], s);
    hipError_t e;
    if (!ps.v) {
      e = launch_scale_copy(p->dtype, src, dst, ps.copy_n, (float)p->scale, s);
    } else {
      PassArgs a = ps.args;
      a.in = src;
      a.out = dst;
      // the default inverse scale 1/N is applied as 1/L per pass (exact
      // powers of two, so the result is unchanged, and 16-bit intermediates
      // stay in range); a scale set by the caller is applied by the last pass
      a.scale = p->scale_user ? (ps.last ? (float)p->scale : 1.0f)
                              : (inv ? 1.0f / (float)(ps.scale_len ? ps.scale_len : ps.v->L) : 1.0f);
      a.conj_in = (inv && ps.first) ? 1 : 0;
      a.conj_out = (inv && ps.last) ? 1 : 0;
      if (ps.per_transform && p->batch > 1) {
        const size_t step = (size_t)(S.points / p->batch) * esize(p->dtype);
        e = hipSuccess;
        for (int64_t b = 0; b < p->batch && e == hipSuccess; ++b) {
          a.in = (const char*)src + b * step;
          a.out = (char*)dst + b * step;
          e = ps.v->launch(a, s, nullptr, nullptr);
        }
      } else {
        e = ps.v->launch(a, s, slot ? slot[2 * i] : nullptr, slot ? slot[2 * i + 1] : nullptr);
      }
    }
    if (slot && !one_launch) hipEventRecord(slot[2 * i + 1], s);
    if (e != hipSuccess) return hip_fail(e);
  }
  prof_commit(p, s);
  return FFT_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free exec: the scratch comes from this library's own device
// array.  Each device holds its own copy of `scratch` (at its own address)
// from the time the library's code is loaded on it until the process ends.
// In host code the name `scratch` is only a host-side stand-in; the device
// address comes from hipGetSymbolAddress, looked up once per device with that
// device current, and only that address is passed to kernels.
// ---------------------------------------------------------------------------
__device__ __align__(256) unsigned char scratch[FFT_STATIC_SCRATCH_BYTES];

constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kScratchMaxDevices] = {};

// Device address of `scratch` on the current device `dev`.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kScratchMaxDevices) return FFT_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (!ptr) return FFT_ERR_INVALID_ARGUMENT;
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return FFT_OK;
}

}  // namespace

int fft_exec(fft_plan_t p, const void* in, void* out, void* stream) {
  return exec_impl(p, in, out, stream, nullptr);
}

int fft_exec_static(fft_plan_t p, const void* in, void* out, void* stream) {
  if (!p || !in || !out) return FFT_ERR_INVALID_ARGUMENT;
  const size_t need = exec_scratch_bytes(p, in, out);
  if (need == 0) return exec_impl(p, in, out, stream, nullptr);
  if (need > (size_t)FFT_STATIC_SCRATCH_BYTES) return FFT_ERR_SCRATCH_LIMIT;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev != p->device) return FFT_ERR_INVALID_ARGUMENT;
  void* ws = nullptr;
  const int rc = scratch_address(dev, &ws);
  if (rc) return rc;
  return exec_impl(p, in, out, stream, ws);
}

int fft_plan_info(fft_plan_t p, fft_plan_info_t* info) {
  if (!p || !info) return FFT_ERR_INVALID_ARGUMENT;
  memset(info, 0, sizeof(*info));
  info->n[0] = p->n[0];
  info->n[1] = p->n[1];
  info->batch = p->batch;
  info->dims = p->dims;
  info->dtype = p->dtype;
  info->direction = p->direction;
  info->gpu_twiddles = p->gpu_twiddles ? 1 : 0;
  const double es = (double)esize(p->dtype);
  if (p->kind == 1) {
    info->passes = 1;
    // the batched kernel: many_2launch (two launches, no waits), many_queue
    // (shared queue, completion counters), many_pipe (round-robin items,
    // completion counters)
    const int pipe = p->many.var ? p->many.var->pipe : 0;
    snprintf(info->pass_variant[0], 32, "%s", pipe == 2 ? "many_2launch" : pipe == 1 ? "many_pipe" : "many_queue");
    info->points = p->many.points;
    info->flops = p->many.flops;
    info->bytes_min = 2.0 * es * (double)p->many.points;
    info->bytes_pass[0] = 2.0 * es * (double)p->many.pass_points;
    return FFT_OK;
  }
  const Schedule& S = p->sched;
  if (p->kind == 3) {
    info->passes = 1;
    snprintf(info->pass_variant[0], 32, "%s", dft256_name(S));
    info->points = S.points;
    info->flops = 5.0 * 256.0 * 8.0 * (double)p->batch;
    info->bytes_min = 2.0 * es * (double)S.points;
    info->bytes_pass[0] = 2.0 * es * (double)S.points;
    return FFT_OK;
  }
  if (p->kind == 2) {
    // the whole sequence of log2 N level launches is reported as one entry
    const double lg = (double)ilog2_64(p->n[0]);
    info->passes = 1;
    snprintf(info->pass_variant[0], 32, "%s", "levels_radix2");
    info->points = S.points;
    info->flops = 5.0 * (double)p->n[0] * lg * (double)p->batch;
    info->bytes_min = 2.0 * es * (double)S.points;
    info->bytes_pass[0] = lg * 2.0 * es * (double)S.points;
    return FFT_OK;
  }
  info->passes = (int)S.passes.size();
  info->split[0] = S.split[0];
  info->split[1] = S.split[1];
  info->points = S.points;
  const double N = (double)p->n[0] * (double)p->n[1];
  info->flops = 5.0 * N * std::log2(std::max(N, 1.0)) * (double)p->batch;
  info->bytes_min = 2.0 * es * (double)S.points;
  for (size_t i = 0; i < S.passes.size() && i < 4; ++i) {
    snprintf(info->pass_variant[i], 32, "%s", S.passes[i].v ? S.passes[i].v->name : "copy_scale");
    info->bytes_pass[i] = 2.0 * es * (double)S.points;
  }
  return FFT_OK;
}

int fft_destroy(fft_plan_t p) {
  if (!p) return FFT_OK;
  for (hipEvent_t e : p->ev) hipEventDestroy(e);
  if (p->d_tables) hipFree(p->d_tables);
  for (void* b : p->aux) hipFree(b);
  if (p->ws_owned && p->ws) hipFree(p->ws);
  many_free(p->many);
  delete p;
  return FFT_OK;
}

const char* fft_error_string(int status) {
  switch (status) {
    case FFT_OK: return "ok";
    case FFT_ERR_INVALID_ARGUMENT: return "invalid argument";
    case FFT_ERR_UNSUPPORTED_SIZE: return "unsupported size (not a power of two, or out of range)";
    case FFT_ERR_ALIGNMENT: return "pointer not aligned to the element size";
    case FFT_ERR_INPLACE: return "in-place or overlapping multi-pass exec needs a workspace";
    case FFT_ERR_HIP: return "HIP runtime error (see fft_last_hip_error)";
    case FFT_ERR_NO_MEMORY: return "out of memory";
    case FFT_ERR_WATCHDOG: return "batched kernel wait limit expired";
    case FFT_ERR_SCRATCH_LIMIT: return "exec needs more scratch than the library's static array holds";
    default: return "unknown status";
  }
}

int fft_last_hip_error(void) { return g_last_hip; }

int fft_variant_count(void) { return (int)variants().size(); }

const char* fft_variant_name(int i) {
  if (i < 0 || i >= (int)variants().size()) return nullptr;
  return variants()[i].name;
}

int fft_variant_describe(int i, int* L, int* P, int* W, int* threads, int* role, int* dtype) {
  if (i < 0 || i >= (int)variants().size()) return FFT_ERR_INVALID_ARGUMENT;
  const Variant& v = variants()[i];
  if (L) *L = v.L;
  if (P) *P = v.P;
  if (W) *W = v.W;
  if (threads) *threads = v.threads;
  if (role) *role = v.role;
  if (dtype) *dtype = v.dtype;
  return FFT_OK;
}

int fft_describe(const int64_t* n, int64_t batch, int dims, int dtype, const char* schedule,
                 int* passes, char names[4][32], int64_t split[2]) {
  Schedule S;
  int rc = build_schedule(n, batch, dims, dtype, schedule, &S);
  if (rc) return rc;
  if (passes) *passes = (S.levels || S.mfma || S.xlane) ? 1 : (int)S.passes.size();
  if (names)
    for (size_t i = 0; i < 4; ++i)
      snprintf(names[i], 32, "%s",
               S.levels ? (i == 0 ? "levels_radix2" : "")
               : (S.mfma || S.xlane) ? (i == 0 ? dft256_name(S) : "")
                        : i < S.passes.size() ? (S.passes[i].v ? S.passes[i].v->name : "copy_scale") : "");
  if (split) {
    split[0] = S.split[0];
    split[1] = S.split[1];
  }
  return FFT_OK;
}

int fft_profile_enable(fft_plan_t p, int slots) {
  if (!p || slots < 0) return FFT_ERR_INVALID_ARGUMENT;
  for (hipEvent_t e : p->ev) hipEventDestroy(e);
  p->ev.clear();
  p->prof = false;
  p->prof_slots = 0;
  p->prof_next = 0;
  p->prof_pending = 0;
  p->prof_seq = 0;
  p->prof_npass = p->kind != 0 ? 1 : p->sched.passes.size();
  p->prof_ms.assign(p->prof_npass, 0.0);
  p->prof_n.assign(p->prof_npass, 0);
  if (!slots) return FFT_OK;
  p->ev.resize((size_t)slots * 2 * p->prof_npass);
  // timing-only events: no system-scope fence (cache writeback and
  // invalidate) when they are recorded, so that timing a pass does not slow
  // the pass after it
  for (auto& e : p->ev) {
    hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    if (r != hipSuccess) return hip_fail(r);
  }
  p->prof_slots = slots;
  p->prof = true;
  return FFT_OK;
}

int fft_profile_collect(fft_plan_t p) {
  if (!p) return FFT_ERR_INVALID_ARGUMENT;
  if (!p->prof) return FFT_OK;
  // oldest pending slot first
  int slot = (p->prof_next - p->prof_pending + p->prof_slots) % p->prof_slots;
  for (int k = 0; k < p->prof_pending; ++k, slot = (slot + 1) % p->prof_slots) {
    hipEvent_t* ev = p->ev.data() + (size_t)slot * 2 * p->prof_npass;
    for (size_t i = 0; i < p->prof_npass; ++i) {
      float ms = 0;
      hipError_t r = hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
      if (r != hipSuccess) return hip_fail(r);
      p->prof_ms[i] += ms;
      p->prof_n[i] += 1;
    }
  }
  p->prof_pending = 0;
  return FFT_OK;
}

int fft_profile_sample(fft_plan_t p, int every) {
  if (!p || every < 1) return FFT_ERR_INVALID_ARGUMENT;
  p->prof_every = every;
  p->prof_seq = 0;
  return FFT_OK;
}

int fft_profile_read(fft_plan_t p, int pass, double* total_ms, int64_t* launches) {
  if (!p || pass < 0 || pass >= (int)p->prof_ms.size()) return FFT_ERR_INVALID_ARGUMENT;
  if (total_ms) *total_ms = p->prof_ms[pass];
  if (launches) *launches = p->prof_n[pass];
  return FFT_OK;
}

}  // extern "C"

namespace {

struct ManyBuild {
  ManyOptions opt;
  const ManyVariant* var = nullptr;
  int max_tile = 0, max_lg = 0;
  std::vector<ManyXform> xf;
  std::vector<ManyItem> items;
  std::vector<int32_t> order;
  int64_t points = 0, pass_points = 0;
  double flops = 0;
  bool has_split = false;
  // two-launch kernel: items (in `items`) in launch order, launch p running
  // items q_off[p] .. q_off[p+1]-1
  std::vector<int32_t> q_off;
};

// The two launches of the two-launch kernel (pipe 2): every first-pass tile,
// then the one-pass tiles, in the first; every second-pass tile in the
// second (the kernel boundary orders each transform's passes).  Within a
// launch, items keep the queue's order (largest transforms first).
// Reorders mb->items in place.
void split_launches(ManyBuild* mb) {
  std::vector<ManyItem> a, one, b;
  for (const ManyItem& it : mb->items)
    (it.kind == MANY_A ? a : it.kind == MANY_B ? b : one).push_back(it);
  mb->items.clear();
  mb->items.insert(mb->items.end(), a.begin(), a.end());
  mb->items.insert(mb->items.end(), one.begin(), one.end());
  mb->q_off = {0, (int32_t)mb->items.size(), 0};
  mb->items.insert(mb->items.end(), b.begin(), b.end());
  mb->q_off[2] = (int32_t)mb->items.size();
}

// Host-only part of a batched plan: per-transform descriptors, the ordered
// work queue and the one-pass groups.  No GPU calls.
int build_many(const int64_t* sizes, int64_t count, int dtype, int direction, const char* schedule,
               ManyBuild* mb) {
  if (!sizes || count < 1 || count > (1 << 24)) return FFT_ERR_INVALID_ARGUMENT;
  if (direction != FFT_FORWARD && direction != FFT_INVERSE) return FFT_ERR_INVALID_ARGUMENT;
  if (dtype != FFT_C64 && dtype != FFT_C16F && dtype != FFT_C16BF) return FFT_ERR_INVALID_ARGUMENT;
  ManyOptions& opt = mb->opt;
  if (parse_many_schedule(schedule, &opt)) return FFT_ERR_INVALID_ARGUMENT;
  for (int i = 0; i < many_variant_count(); ++i) {
    const ManyVariant* v = many_variant(i);
    if (v->dtype == dtype && v->P == opt.P && v->threads == opt.threads && v->pipe == opt.pipe)
      mb->var = v;
  }
  if (!mb->var) return FFT_ERR_INVALID_ARGUMENT;
  const int max_tile = std::min(mb->var->max_lg, ilog2_64((int64_t)opt.threads * opt.P));
  mb->max_tile = max_tile;
  if (opt.pass2 == 0) opt.pass2 = max_tile + 1;
  if (opt.pass2 < 1 || opt.pass2 > max_tile + 1) return FFT_ERR_INVALID_ARGUMENT;

  std::vector<ManyXform>& xf = mb->xf;
  xf.assign((size_t)count, ManyXform{});
  std::vector<int> lgs((size_t)count);
  int64_t off = 0;
  for (int64_t i = 0; i < count; ++i) {
    const int64_t n = sizes[i];
    if (!pow2(n) || ilog2_64(n) > FFT_MAX_LOG2_1D) return FFT_ERR_UNSUPPORTED_SIZE;
    const int lg = ilog2_64(n);
    if (lg > 2 * max_tile) return FFT_ERR_UNSUPPORTED_SIZE;
    lgs[i] = lg;
    mb->max_lg = std::max(mb->max_lg, lg);
    ManyXform& x = xf[i];
    x.off = off;
    x.lg = lg;
    // two passes need two sub-lengths of at least 2 points each
    bool split = (lg >= opt.pass2 || lg > max_tile) && lg >= 2;
    if (opt.passes_for[lg] == 2 || opt.lg1_for[lg]) {
      if (lg < 2) return FFT_ERR_INVALID_ARGUMENT;
      split = true;
    }
    if (opt.passes_for[lg] == 1) {
      if (lg > max_tile) return FFT_ERR_INVALID_ARGUMENT;
      split = false;
    }
    if (split) {
      x.lg1 = opt.lg1_for[lg] ? opt.lg1_for[lg] : (lg + 1) / 2;
      if (!opt.lg1_for[lg] && x.lg1 > max_tile) x.lg1 = max_tile;
      if (x.lg1 > max_tile || lg - x.lg1 > max_tile || x.lg1 < 1 || lg - x.lg1 < 1) return FFT_ERR_INVALID_ARGUMENT;
      const int64_t N2 = (int64_t)1 << (lg - x.lg1);
      const int wa = tile_lines(x.lg1, opt.P, opt.threads);
      x.nA = (int32_t)((N2 + wa - 1) / wa);
      mb->pass_points += 2 * n;
    } else {
      mb->pass_points += n;
    }
    off += n;
    mb->points += n;
    mb->flops += 5.0 * (double)n * (double)lg;
  }
  if (off > ((int64_t)1 << 40)) return FFT_ERR_UNSUPPORTED_SIZE;

  // transform order: biggest first (stable), or as given
  std::vector<int32_t> ids((size_t)count);
  for (int64_t i = 0; i < count; ++i) ids[i] = (int32_t)i;
  if (!opt.given_order)
    std::stable_sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) { return lgs[a] > lgs[b]; });

  // items: first-pass tiles, one-pass tiles, second-pass tiles.  Every
  // first-pass tile of a transform precedes its second-pass tiles, so the
  // tiles a waiting second-pass tile depends on have all been taken by
  // running workgroups, which never wait themselves.
  std::vector<ManyItem>& items = mb->items;
  std::vector<int32_t>& order = mb->order;
  std::vector<int32_t> split_ids;
  for (int32_t id : ids)
    if (xf[id].nA) split_ids.push_back(id);
  auto push_b = [&](int32_t id) {
    const ManyXform& x = xf[id];
    const int lg2 = x.lg - x.lg1;
    const int64_t N1 = (int64_t)1 << x.lg1;
    const int wb = tile_lines(lg2, opt.P, opt.threads);
    const int nb = (int)((N1 + wb - 1) / wb);
    for (int t = 0; t < nb; ++t) items.push_back({MANY_B, lg2, id, t});
  };
  size_t b_next = 0;  // split transforms whose second-pass tiles are queued
  for (size_t i = 0; i < split_ids.size(); ++i) {
    const ManyXform& x = xf[split_ids[i]];
    mb->has_split = true;
    for (int t = 0; t < x.nA; ++t) items.push_back({MANY_A, x.lg1, split_ids[i], t});
    if (opt.lag > 0 && i >= (size_t)opt.lag) push_b(split_ids[b_next++]);
  }
  {
    // one-pass transforms grouped by length, W lines per tile
    std::vector<std::vector<int32_t>> by_lg(max_tile + 1);
    for (int32_t id : ids)
      if (xf[id].nA == 0) by_lg[xf[id].lg].push_back(id);
    std::vector<int> lg_order;
    if (opt.given_order) {
      std::vector<bool> seen(max_tile + 1, false);
      for (int32_t id : ids)
        if (xf[id].nA == 0 && !seen[xf[id].lg]) {
          seen[xf[id].lg] = true;
          lg_order.push_back(xf[id].lg);
        }
    } else {
      for (int lg = max_tile; lg >= 0; --lg) lg_order.push_back(lg);
    }
    for (int lg : lg_order) {
      const auto& v = by_lg[lg];
      const int W = tile_lines(lg, opt.P, opt.threads);
      for (size_t j = 0; j < v.size(); j += W) {
        const int g = (int)std::min<size_t>(W, v.size() - j);
        items.push_back({MANY_SINGLE, lg, (int32_t)order.size(), g});
        for (int k = 0; k < g; ++k) order.push_back(v[j + k]);
      }
    }
  }
  while (b_next < split_ids.size()) push_b(split_ids[b_next++]);
  if (items.size() > (size_t)INT32_MAX / 2) return FFT_ERR_UNSUPPORTED_SIZE;
  if (opt.pipe == 2) split_launches(mb);
  return FFT_OK;
}

}  // namespace

extern "C" {

int fft_describe_many(const int64_t* sizes, int64_t count, int dtype, const char* schedule,
                      int32_t* items, int64_t max_items, int64_t* n_items, int32_t* first_len,
                      int32_t* first_tiles) {
  if (!n_items) return FFT_ERR_INVALID_ARGUMENT;
  ManyBuild mb;
  int rc = build_many(sizes, count, dtype, FFT_FORWARD, schedule, &mb);
  if (rc) return rc;
  *n_items = (int64_t)mb.items.size();
  if (items) {
    if (max_items < (int64_t)mb.items.size()) return FFT_ERR_INVALID_ARGUMENT;
    for (size_t i = 0; i < mb.items.size(); ++i) {
      const ManyItem& it = mb.items[i];
      // one-pass items are reported as (0, lg, first transform, lines)
      const int32_t a = it.kind == MANY_SINGLE ? mb.order[it.a] : it.a;
      items[4 * i] = it.kind;
      items[4 * i + 1] = it.lg;
      items[4 * i + 2] = a;
      items[4 * i + 3] = it.b;
    }
  }
  for (int64_t i = 0; i < count; ++i) {
    if (first_len) first_len[i] = mb.xf[i].nA ? (1 << mb.xf[i].lg1) : 0;
    if (first_tiles) first_tiles[i] = mb.xf[i].nA;
  }
  return FFT_OK;
}

int fft_describe_many_launches(const int64_t* sizes, int64_t count, int dtype, const char* schedule,
                               int32_t* q_off, int64_t max_q, int64_t* n_q) {
  if (!n_q) return FFT_ERR_INVALID_ARGUMENT;
  ManyBuild mb;
  int rc = build_many(sizes, count, dtype, FFT_FORWARD, schedule, &mb);
  if (rc) return rc;
  if (mb.q_off.empty()) {
    *n_q = 1;
    if (q_off) {
      if (max_q < 2) return FFT_ERR_INVALID_ARGUMENT;
      q_off[0] = 0;
      q_off[1] = (int32_t)mb.items.size();
    }
    return FFT_OK;
  }
  *n_q = (int64_t)mb.q_off.size() - 1;
  if (q_off) {
    if (max_q < (int64_t)mb.q_off.size()) return FFT_ERR_INVALID_ARGUMENT;
    for (size_t i = 0; i < mb.q_off.size(); ++i) q_off[i] = mb.q_off[i];
  }
  return FFT_OK;
}

int fft_plan_many_ex(const int64_t* sizes, int64_t count, int dtype, int direction,
                     const char* schedule, fft_plan_t* out) {
  if (!out) return FFT_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  ManyBuild mb;
  int rc0 = build_many(sizes, count, dtype, direction, schedule, &mb);
  if (rc0) return rc0;
  const ManyOptions& opt = mb.opt;
  const ManyVariant* var = mb.var;
  const int max_tile = mb.max_tile;
  const int max_lg = mb.max_lg;
  std::vector<ManyXform>& xf = mb.xf;
  std::vector<ManyItem>& items = mb.items;
  std::vector<int32_t>& order = mb.order;
  const int64_t points = mb.points, pass_points = mb.pass_points;
  const double flops = mb.flops;
  const bool has_split = mb.has_split;
  fft_plan_s* p = new (std::nothrow) fft_plan_s();
  if (!p) return FFT_ERR_NO_MEMORY;
  p->kind = 1;
  p->dims = 1;
  p->n[0] = count;
  p->n[1] = 1;
  p->batch = count;
  p->dtype = dtype;
  p->direction = direction;
  p->scale = direction > 0 ? 0.0 : 1.0;  // per-transform default unless set
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e);
  }
  // twiddle tables: stage tables of every tile length, inter-pass per split length
  TableBuild tb;
  ManyPlan& mp = p->many;
  std::vector<bool> used(max_tile + 1, false);
  for (const ManyItem& it : items)
    if (it.lg >= 1) used[it.lg] = true;
  std::vector<int64_t> soff(kManyMaxLg + 1, 0);
  for (int lg = 1; lg <= max_tile; ++lg)
    if (used[lg]) soff[lg] = tb.add_stage_table(1 << lg, opt.P);
  std::map<int, int64_t> inter;
  for (int64_t i = 0; i < count; ++i) {
    ManyXform& x = xf[i];
    if (x.nA == 0) continue;
    auto it = inter.find(x.lg);
    if (it == inter.end()) {
      const int64_t N = (int64_t)1 << x.lg;
      const int64_t N1 = (int64_t)1 << x.lg1, N2 = N >> x.lg1;
      const int64_t lo = tb.add(N1, 0, N, 1);
      tb.add(N2, 0, N, N1);
      // step rows W_N^{n2*q*T}, T = N1/P: entry n2*P + q
      const int pp = (int)std::min<int64_t>(opt.P, N1);
      tb.add(N2 * pp, pp, N, N1 / pp);
      it = inter.emplace(x.lg, lo).first;
    }
    x.tw_lo = it->second;
    {
      const int64_t N1 = (int64_t)1 << x.lg1, N2 = ((int64_t)1 << x.lg) >> x.lg1;
      x.tw_step = x.tw_lo + N1 + N2;
    }
  }
  int rc = upload_tables(p, tb, max_lg >= kGpuTwiddleMinLog2);
  if (rc) {
    fft_destroy(p);
    return rc;
  }
  auto upload = [&](void** dptr, const void* src, size_t bytes) -> int {
    hipError_t r = hipMalloc(dptr, std::max<size_t>(bytes, 16));
    if (r != hipSuccess) {
      *dptr = nullptr;
      return r == hipErrorOutOfMemory ? FFT_ERR_NO_MEMORY : hip_fail(r);
    }
    if (bytes) {
      r = hipMemcpy(*dptr, src, bytes, hipMemcpyHostToDevice);
      if (r != hipSuccess) return hip_fail(r);
    }
    return FFT_OK;
  };
  rc = upload((void**)&mp.d_items, items.data(), items.size() * sizeof(ManyItem));
  if (!rc && opt.pipe == 2) {
    // one self-contained record per item, grouped by queue
    std::vector<ManyItemX> itx(items.size());
    size_t launch = 0;
    for (size_t i = 0; i < items.size(); ++i) {
      const ManyItem& it = items[i];
      ManyItemX& d = itx[i];
      memset(&d, 0, sizeof(d));
      d.kind = it.kind;
      d.lg = it.lg;
      d.a = it.a;
      d.b = it.b;
      while (launch + 2 < mb.q_off.size() && i >= (size_t)mb.q_off[launch + 1]) ++launch;
      d.nt = opt.nt_store || (int64_t)i >= (int64_t)mb.q_off[launch + 1] - opt.nt_tail;
      if (it.kind != MANY_SINGLE) {
        const ManyXform& x = xf[it.a];
        d.off = x.off;
        d.tw_lo = x.tw_lo;
        d.tw_step = x.tw_step;
        d.lg1 = x.lg1;
        d.lgN = x.lg;
      }
    }
    rc = upload((void**)&mp.d_itx, itx.data(), itx.size() * sizeof(ManyItemX));
    if (!rc) rc = upload((void**)&mp.d_q_off, mb.q_off.data(), mb.q_off.size() * sizeof(int32_t));
  }
  if (!rc) rc = upload((void**)&mp.d_xf, xf.data(), xf.size() * sizeof(ManyXform));
  if (!rc) rc = upload((void**)&mp.d_order, order.data(), order.size() * sizeof(int32_t));
  std::vector<int64_t> order_off(order.size());
  for (size_t i = 0; i < order.size(); ++i) order_off[i] = xf[order[i]].off;
  if (!rc) rc = upload((void**)&mp.d_order_off, order_off.data(), order_off.size() * sizeof(int64_t));
  if (rc) {
    fft_destroy(p);
    return rc;
  }
  mp.active = true;
  mp.var = var;
  mp.d_tw = p->d_tables;
  mp.count = count;
  mp.n_items = (int64_t)items.size();
  mp.points = points;
  mp.pass_points = pass_points;
  mp.flops = flops;
  mp.dtype = dtype;
  mp.has_split = has_split;
  mp.gpu_twiddles = p->gpu_twiddles;
  ManyArgs& a = mp.args;
  memset(&a, 0, sizeof(a));
  a.items = mp.d_items;
  a.xf = mp.d_xf;
  a.order = mp.d_order;
  a.order_off = mp.d_order_off;
  a.tw = mp.d_tw;
  for (int lg = 0; lg <= kManyMaxLg; ++lg) a.stage_off[lg] = soff[lg];
  a.tw_used = 0;
  for (int lg = 1; lg <= max_tile; ++lg)
    if (used[lg]) a.tw_used |= 1 << lg;
  if (var->pipe) {
    // the pipelined kernel's LDS image of the stage twiddles, gathered once
    std::vector<int32_t> map;
    const int len = many_tw_image_map(a.stage_off, a.tw_used, opt.P, var->max_lg, &map);
    int32_t* d_map = nullptr;
    rc = upload((void**)&d_map, map.data(), map.size() * sizeof(int32_t));
    if (!rc) {
      e = hipMalloc((void**)&mp.d_tw_img, std::max<size_t>(map.size(), 1) * sizeof(float2));
      if (e != hipSuccess) {
        mp.d_tw_img = nullptr;
        rc = e == hipErrorOutOfMemory ? FFT_ERR_NO_MEMORY : hip_fail(e);
      }
    }
    if (!rc) {
      e = launch_gather_f2(mp.d_tw_img, p->d_tables, d_map, (int)map.size(), nullptr);
      if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
      if (e != hipSuccess) rc = hip_fail(e);
    }
    if (d_map) hipFree(d_map);
    if (rc) {
      fft_destroy(p);
      return rc;
    }
    a.tw_img = mp.d_tw_img;
    a.tw_img_len = len;
    // each launch of the two-launch kernel copies only the lengths it runs
    a.tw_img_len_ph[0] = a.tw_img_len_ph[1] = len;
    if (opt.pipe == 2) {
      int mx[2] = {0, 0};
      for (size_t i = 0; i < items.size(); ++i) {
        const int ph = (int)i >= mb.q_off[1] ? 1 : 0;
        mx[ph] = std::max(mx[ph], items[i].lg);
      }
      for (int ph = 0; ph < 2; ++ph) a.tw_img_len_ph[ph] = std::max(1, many_tw_image_prefix(opt.P, mx[ph]));
    }
  }
  a.n_items = (int32_t)items.size();
  a.n_xforms = (int32_t)count;
  a.wait_ticks = kManyWaitDefaultUs * 100;
  a.itx = mp.d_itx;
  a.q_off = mp.d_q_off;
  a.phase = 0;
  a.n_phase2 = opt.pipe == 2 ? mb.q_off[2] - mb.q_off[1] : 0;
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) {
    fft_destroy(p);
    return hip_fail(e);
  }
  const int per_cu = std::max(1, var->max_blocks_per_cu());
  mp.grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)per_cu * cus, mp.n_items));
  // the two-launch kernel runs the full resident grid: with claims from the
  // queue head every workgroup is useful until the launch's items run out
  if (opt.pipe == 2) mp.grid = std::max(1, per_cu * cus);
  rc = many_alloc_workspace(mp, &p->ws, &p->ws_bytes);
  if (rc) {
    fft_destroy(p);
    return rc;
  }
  p->ws_owned = true;
  *out = p;
  return FFT_OK;
}

int fft_plan_many(const int64_t* sizes, int64_t count, int dtype, int direction, fft_plan_t* out) {
  return fft_plan_many_ex(sizes, count, dtype, direction, nullptr, out);
}

int fft_many_watchdog(fft_plan_t p, int clear) {
  if (!p || p->kind != 1 || !p->ws) return FFT_ERR_INVALID_ARGUMENT;
  int32_t flag = 0;
  hipError_t e = hipMemcpy(&flag, (int32_t*)p->ws + 2, sizeof(flag), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e);
  if (flag && clear) {
    int32_t z = 0;
    e = hipMemcpy((int32_t*)p->ws + 2, &z, sizeof(z), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
  }
  return flag ? FFT_ERR_WATCHDOG : FFT_OK;
}

int fft_many_set_wait_limit(fft_plan_t p, int64_t microseconds) {
  if (!p || p->kind != 1 || microseconds < 1 || microseconds > ((int64_t)1 << 40))
    return FFT_ERR_INVALID_ARGUMENT;
  p->many.args.wait_ticks = microseconds * 100;
  return FFT_OK;
}

int fft_twiddle_host(int64_t count, int64_t R, int64_t M, int64_t mul, float* out) {
  if (!out || count < 0 || R < 0 || M < 1 || (M & (M - 1))) return FFT_ERR_INVALID_ARGUMENT;
  TwSeg sg{0, count, R, M, mul};
  for (int64_t i = 0; i < count; ++i) {
    double c, sn;
    twiddle_fp64(seg_exponent(sg, i), M, &c, &sn);
    out[2 * i] = (float)c;
    out[2 * i + 1] = (float)-sn;
  }
  return FFT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// host-to-host pipe: copy in, transform and copy out of successive chunks on
// three streams, ordered per staging slot by events
// ---------------------------------------------------------------------------
struct fft_pipe_s {
  fft_plan_t plan = nullptr;
  int slots = 0;
  size_t chunk_bytes = 0;
  std::vector<void*> d_in, d_out;
  hipStream_t s_in = nullptr, s_run = nullptr, s_out = nullptr;
  std::vector<hipEvent_t> ev_in, ev_run, ev_out;
  int64_t issued = 0;  // chunks queued so far, over every exec of this pipe
};

namespace {

void pipe_free(fft_pipe_s* q) {
  if (q->s_out) hipStreamSynchronize(q->s_out);
  if (q->s_run) hipStreamSynchronize(q->s_run);
  if (q->s_in) hipStreamSynchronize(q->s_in);
  for (void* b : q->d_in) if (b) hipFree(b);
  for (void* b : q->d_out) if (b) hipFree(b);
  for (auto* v : {&q->ev_in, &q->ev_run, &q->ev_out})
    for (hipEvent_t e : *v) if (e) hipEventDestroy(e);
  if (q->s_in) hipStreamDestroy(q->s_in);
  if (q->s_run) hipStreamDestroy(q->s_run);
  if (q->s_out) hipStreamDestroy(q->s_out);
  delete q;
}

}  // namespace

extern "C" {

int fft_pipe_create(fft_plan_t plan, int slots, fft_pipe_t* out) {
  if (!out) return FFT_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!plan || slots < 2 || slots > 64) return FFT_ERR_INVALID_ARGUMENT;
  fft_plan_info_t info;
  int rc = fft_plan_info(plan, &info);
  if (rc) return rc;
  fft_pipe_s* q = new (std::nothrow) fft_pipe_s();
  if (!q) return FFT_ERR_NO_MEMORY;
  q->plan = plan;
  q->slots = slots;
  q->chunk_bytes = (size_t)info.points * esize(info.dtype);
  q->d_in.assign(slots, nullptr);
  q->d_out.assign(slots, nullptr);
  q->ev_in.assign(slots, nullptr);
  q->ev_run.assign(slots, nullptr);
  q->ev_out.assign(slots, nullptr);
  hipError_t e = hipSuccess;
  for (int i = 0; i < slots && e == hipSuccess; ++i) {
    e = hipMalloc(&q->d_in[i], std::max<size_t>(q->chunk_bytes, 16));
    if (e == hipSuccess) e = hipMalloc(&q->d_out[i], std::max<size_t>(q->chunk_bytes, 16));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&q->ev_in[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&q->ev_run[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&q->ev_out[i], hipEventDisableTiming);
  }
  // default priority on purpose (no priority streams)
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->s_in, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->s_run, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->s_out, hipStreamNonBlocking);
  if (e != hipSuccess) {
    pipe_free(q);
    return e == hipErrorOutOfMemory ? FFT_ERR_NO_MEMORY : hip_fail(e);
  }
  *out = q;
  return FFT_OK;
}

int fft_pipe_exec(fft_pipe_t q, const void* host_in, void* host_out, int64_t chunks) {
  if (!q || chunks < 0 || (chunks > 0 && (!host_in || !host_out))) return FFT_ERR_INVALID_ARGUMENT;
  const char* hi = (const char*)host_in;
  char* ho = (char*)host_out;
  for (int64_t c = 0; c < chunks; ++c) {
    // slots are used round-robin across execs, so that an exec queued before
    // the previous one finished still waits for the slot it reuses
    const int64_t g = q->issued++;
    const int s = (int)(g % q->slots);
    hipError_t e = hipSuccess;
    // slot s is free once the copy out of the chunk queued `slots` earlier
    // has finished (its transform, which read d_in[s], finished before it)
    if (g >= q->slots) e = hipStreamWaitEvent(q->s_in, q->ev_out[s], 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(q->d_in[s], hi + (size_t)c * q->chunk_bytes, q->chunk_bytes,
                         hipMemcpyHostToDevice, q->s_in);
    if (e == hipSuccess) e = hipEventRecord(q->ev_in[s], q->s_in);
    if (e == hipSuccess) e = hipStreamWaitEvent(q->s_run, q->ev_in[s], 0);
    if (e != hipSuccess) return hip_fail(e);
    int rc = fft_exec(q->plan, q->d_in[s], q->d_out[s], q->s_run);
    if (rc) return rc;
    e = hipEventRecord(q->ev_run[s], q->s_run);
    if (e == hipSuccess) e = hipStreamWaitEvent(q->s_out, q->ev_run[s], 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ho + (size_t)c * q->chunk_bytes, q->d_out[s], q->chunk_bytes,
                         hipMemcpyDeviceToHost, q->s_out);
    if (e == hipSuccess) e = hipEventRecord(q->ev_out[s], q->s_out);
    if (e != hipSuccess) return hip_fail(e);
  }
  return FFT_OK;
}

int fft_pipe_wait(fft_pipe_t q) {
  if (!q) return FFT_ERR_INVALID_ARGUMENT;
  hipError_t e = hipStreamSynchronize(q->s_out);
  if (e == hipSuccess) e = hipStreamSynchronize(q->s_run);
  if (e == hipSuccess) e = hipStreamSynchronize(q->s_in);
  return e == hipSuccess ? FFT_OK : hip_fail(e);
}

int fft_pipe_destroy(fft_pipe_t q) {
  if (!q) return FFT_OK;
  pipe_free(q);
  return FFT_OK;
}

}  // extern "C"

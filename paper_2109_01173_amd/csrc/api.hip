// C-ABI entry points of libmofem: operator and preconditioner handles, the
// batched MO-PCG driver (Sec. 5, eqs. (77)-(78)) and the IMEX Euler step
// (Sec. 6, eqs. (89)-(96); DIB kinetics Sec. 7).
//
// Every step of the solve runs in this library's kernels (k_band.hip,
// k_gemm.hip, k_vec.hip); the host only sequences launches, keeps per-item
// convergence flags and reads a few bytes of residual norms per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"
#include "mofem_internal.h"

using namespace mofem;

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(MOFEM_E_HIP, std::string("HIP error in ") + #expr + ": " +           \
                                   hipGetErrorString(_e));                             \
  } while (0)

namespace {

template <class T>
int dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(MOFEM_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  return MOFEM_OK;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// bump allocator over a caller-provided device workspace
struct Carve {
  char* base;
  size_t used = 0, cap;
  Carve(void* b, size_t c) : base((char*)b), cap(c) {}
  template <class T>
  T* take(size_t count) {
    size_t off = align_up(used, 256);
    used = off + align_up(count * sizeof(T), 256);
    return used <= cap ? (T*)(base + off) : nullptr;
  }
};

// ---- kernel tracing: HIP event pairs around every launch -------------------
struct TraceRec {
  int cls;
  double items;
  hipEvent_t e0, e1;
};
struct TraceState {
  std::mutex mu;
  bool on = false;
  unsigned mask = ~0u;  // classes that record events (mofem_trace_select)
  std::vector<TraceRec> recs;
  std::vector<hipEvent_t> pool;
  double total_ms[MOFEM_TRACE_CLASSES] = {};
  long long launches[MOFEM_TRACE_CLASSES] = {};
  double items[MOFEM_TRACE_CLASSES] = {};
};
TraceState& trace_state() {
  static TraceState t;
  return t;
}
hipEvent_t trace_event(TraceState& t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  // timing-only events: no system-scope fence, so a record does not write back
  // and invalidate the caches between the traced kernels
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) == hipSuccess) return e;
  (void)hipGetLastError();
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
// caller holds the mutex
void trace_resolve(TraceState& t) {
  for (TraceRec& r : t.recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
      t.total_ms[r.cls] += ms;
      t.launches[r.cls] += 1;
      t.items[r.cls] += r.items;
    }
    t.pool.push_back(r.e0);
    t.pool.push_back(r.e1);
  }
  t.recs.clear();
}
// Tracing is suspended on a thread while it captures a HIP graph (event
// records inside a graph would not describe individual replays).
thread_local int g_trace_suspended = 0;
struct TraceCapture {
  TraceCapture() { ++g_trace_suspended; }
  ~TraceCapture() { --g_trace_suspended; }
};
// Correct the item count of a class after the fact (launches whose item
// count was only known later, e.g. under device-side masking).
void trace_add_items(int cls, double delta) {
  if (g_trace_suspended) return;
  TraceState& t = trace_state();
  std::lock_guard<std::mutex> g(t.mu);
  if (t.on && ((t.mask >> cls) & 1u)) t.items[cls] += delta;
}
// RAII: records e0 now and e1 when the scope (one kernel launch) ends
struct TraceScope {
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int cls;
  double items;
  TraceScope(int c, double n, hipStream_t st) : s(st), cls(c), items(n) {
    if (g_trace_suspended) return;
    TraceState& t = trace_state();
    std::lock_guard<std::mutex> g(t.mu);
    if (!t.on || !((t.mask >> c) & 1u)) return;
    e0 = trace_event(t);
    e1 = trace_event(t);
    if (e0 && e1) (void)hipEventRecord(e0, s);
  }
  ~TraceScope() {
    if (!e0 || !e1) return;
    TraceState& t = trace_state();
    std::lock_guard<std::mutex> g(t.mu);
    (void)hipEventRecord(e1, s);
    t.recs.push_back({cls, items, e0, e1});
    if (t.recs.size() > 16384) trace_resolve(t);
  }
};

}  // namespace

extern "C" int mofem_trace_enable(int on) {
  clear_error();
  TraceState& t = trace_state();
  std::lock_guard<std::mutex> g(t.mu);
  if (on) {
    trace_resolve(t);
    for (int c = 0; c < MOFEM_TRACE_CLASSES; ++c) {
      t.total_ms[c] = 0.0;
      t.launches[c] = 0;
      t.items[c] = 0.0;
    }
  }
  t.on = on != 0;
  return MOFEM_OK;
}

extern "C" int mofem_trace_select(unsigned mask) {
  clear_error();
  TraceState& t = trace_state();
  std::lock_guard<std::mutex> g(t.mu);
  t.mask = mask;
  return MOFEM_OK;
}

extern "C" int mofem_trace_read(int cls, double* total_ms, long long* launches, double* items) {
  clear_error();
  if (cls < 0 || cls >= MOFEM_TRACE_CLASSES) return fail(MOFEM_E_ARG, "trace_read: unknown class");
  TraceState& t = trace_state();
  std::lock_guard<std::mutex> g(t.mu);
  trace_resolve(t);
  if (total_ms) *total_ms = t.total_ms[cls];
  if (launches) *launches = t.launches[cls];
  if (items) *items = t.items[cls];
  return MOFEM_OK;
}

// ============================================================================
// operator
// ============================================================================
// One launch of the band kernel over at most band_pass_terms(kb) terms (6 for
// kb <= 2, 4 above); an operator with more (distinct) terms runs several
// passes, the later ones adding to Y.
struct OpPass {
  int nt = 0, scaled_mask = 0, pattern = 0;
  int n_rowblk[2] = {0, 0}, n_tiles[2] = {0, 0};  // default and small row blocks
  double* d_left = nullptr;   // [ns_in][nt][2kb+1]: left bands by input row (transposed)
  double* d_right = nullptr;  // [nt][2kb+1][qt]
};
struct mofem_op_s {
  int kb = 0, qs = 0, qt = 0, ns_in = 0, nt_in = 0;
  int off_s = 0, off_t = 0, ph_s = 0, full_input = 0, full_output = 0;
  int n_terms = 0;              // distinct terms after merging
  int n_pass = 0;
  OpPass pass[2];               // at most 8 terms, at least 4 per pass
  int n_tiles_max = 0;          // most tiles of the last pass (the one that forms <X, Y>) in any variant
  int n_cu = 256;               // compute units of the device (grid-fill rule of op_variant)
  double* d_partial = nullptr;  // dot partials for mofem_op_apply
  int partial_batch = 0;
};

// P_k element structure of the transposed left bands: input row a (node row
// a - delta, element phase (a - delta) mod kb) feeds output rows a - off_s + e - kb
// only for e inside the element(s) of that node
static bool element_structured(const std::vector<double>& leftT, int n_in, int nt, int kb, int delta) {
  const int W = 2 * kb + 1;
  for (int a = 0; a < n_in; ++a) {
    int phase = (a - delta) % kb;
    int dlo = phase == 0 ? 0 : kb - phase, dhi = phase == 0 ? 2 * kb : 2 * kb - phase;
    for (int t = 0; t < nt; ++t)
      for (int d = 0; d < W; ++d)
        if ((d < dlo || d > dhi) && leftT[((size_t)a * nt + t) * W + d] != 0.0) return false;
  }
  return true;
}

namespace {
// one term in the kernel's index space: left coefficients (coefficient folded
// in) [qs][2kb+1] by output row, right coefficients [2kb+1][qt] by output column
struct TermArrays {
  std::vector<double> l, r;
  int scaled;
};
}  // namespace

extern "C" int mofem_op_create(const mofem_op_desc* desc, mofem_op_t* out) {
  clear_error();
  if (!desc || !out) return fail(MOFEM_E_ARG, "op_create: NULL argument");
  *out = nullptr;
  const mofem_op_desc& D = *desc;
  if (D.kb < 1 || D.kb > 4) return fail(MOFEM_E_ARG, "op_create: kb must be 1..4");
  if (D.n_terms < 1 || D.n_terms > MOFEM_MAX_TERMS)
    return fail(MOFEM_E_ARG, "op_create: n_terms must be 1..MOFEM_MAX_TERMS (8)");
  if ((D.trim_s != 0 && D.trim_s != 1) || (D.trim_t != 0 && D.trim_t != 1))
    return fail(MOFEM_E_ARG, "op_create: trim flags must be 0 or 1");
  if (D.n_s - 2 * D.trim_s < 1 || D.n_t - 2 * D.trim_t < 1 || D.n_s < D.kb + 1 || D.n_t < D.kb + 1)
    return fail(MOFEM_E_ARG, "op_create: matrices too small for the band");
  for (int t = 0; t < D.n_terms; ++t)
    if (!D.left[t] || !D.right[t]) return fail(MOFEM_E_ARG, "op_create: NULL band");
  if (D.full_input && D.full_output) return fail(MOFEM_E_ARG, "op_create: full_input and full_output exclude each other");

  const int kb = D.kb, W = 2 * kb + 1;
  const int ns = D.n_s, ntt = D.n_t;
  // output rows/columns: the unknowns, or all nodes for full_output
  const int qs = D.full_output ? ns : ns - 2 * D.trim_s, qt = D.full_output ? ntt : ntt - 2 * D.trim_t;
  const int row0 = D.full_output ? 0 : D.trim_s, col0 = D.full_output ? 0 : D.trim_t;  // node of output 0
  std::vector<TermArrays> terms;
  for (int t = 0; t < D.n_terms; ++t) {
    const double* Lb = D.left[t];
    const double* Rb = D.right[t];
    const double c = D.coef[t];
    TermArrays ta{std::vector<double>((size_t)qs * W, 0.0), std::vector<double>((size_t)W * qt, 0.0),
                  D.scaled[t] ? 1 : 0};
    for (int i = 0; i < qs; ++i) {
      int gi = i + row0;
      for (int d = 0; d < W; ++d) {
        int ga = gi + d - kb;  // node index of the input row
        bool ok = D.full_input ? (ga >= 0 && ga < ns) : (ga >= D.trim_s && ga < ns - D.trim_s);
        if (!ok) continue;
        double v = D.left_transpose[t] ? Lb[(size_t)(2 * kb - d) * ns + ga] : Lb[(size_t)d * ns + gi];
        ta.l[(size_t)i * W + d] = c * v;
      }
    }
    for (int j = 0; j < qt; ++j) {
      int gj = j + col0;
      for (int d = 0; d < W; ++d) {
        int gb = gj + d - kb;  // node index of the input column
        bool ok = D.full_input ? (gb >= 0 && gb < ntt) : (gb >= D.trim_t && gb < ntt - D.trim_t);
        if (!ok) continue;
        // coefficient R[gb][gj] (or R^T[gb][gj] = R[gj][gb])
        double v = D.right_transpose[t] ? Rb[(size_t)d * ntt + gj] : Rb[(size_t)(2 * kb - d) * ntt + gb];
        ta.r[(size_t)d * qt + j] = v;
      }
    }
    for (double v : ta.l)
      if (!std::isfinite(v)) return fail(MOFEM_E_NOTFINITE, "op_create: non-finite band entry");
    for (double v : ta.r)
      if (!std::isfinite(v)) return fail(MOFEM_E_NOTFINITE, "op_create: non-finite band entry");
    // merge with an earlier term of the same scaling that shares a factor:
    // L1 X R + L2 X R = (L1 + L2) X R, and L X R1 + L X R2 = L X (R1 + R2)
    bool merged = false;
    for (TermArrays& u : terms) {
      if (u.scaled != ta.scaled) continue;
      if (u.r == ta.r) {
        for (size_t e = 0; e < u.l.size(); ++e) u.l[e] += ta.l[e];
      } else if (u.l == ta.l) {
        for (size_t e = 0; e < u.r.size(); ++e) u.r[e] += ta.r[e];
      } else {
        continue;
      }
      merged = true;
      break;
    }
    if (!merged) terms.push_back(std::move(ta));
  }
  // passes of at most band_pass_terms(kb) terms
  const int n_terms = (int)terms.size();
  const int per_pass = band_pass_terms(kb);
  const int n_pass = (n_terms + per_pass - 1) / per_pass;
  auto* op = new mofem_op_s();
  op->kb = kb;
  op->qs = qs;
  op->qt = qt;
  op->full_input = D.full_input;
  op->full_output = D.full_output;
  op->n_terms = n_terms;
  op->n_pass = n_pass;
  // input index of output (i, j) is (i + off_s, j + off_t)
  op->ns_in = D.full_input ? ns : ns - 2 * D.trim_s;
  op->nt_in = D.full_input ? ntt : ntt - 2 * D.trim_t;
  op->off_s = D.full_input ? D.trim_s : (D.full_output ? -D.trim_s : 0);
  op->off_t = D.full_input ? D.trim_t : (D.full_output ? -D.trim_t : 0);
  op->ph_s = row0;
  int t0 = 0;
  for (int ps = 0; ps < n_pass; ++ps) {
    // split evenly: 7 terms run as 4 + 3, 8 as 4 + 4 (5 as 3 + 2 when kb >= 3)
    const int take = (n_terms - t0 + (n_pass - ps) - 1) / (n_pass - ps);
    const int nt = take;
    // left bands transposed, by input row a: leftT[a][t][e] is the coefficient
    // of input row a in output row i = a - off_s + e - kb, i.e. L_t[i][2kb - e]
    // of the row layout (zero where i is not an output row)
    const int n_in = op->ns_in;
    std::vector<double> leftT((size_t)n_in * nt * W, 0.0), right((size_t)nt * W * qt, 0.0);
    int mask = 0;
    for (int t = 0; t < take; ++t) {
      const TermArrays& ta = terms[t0 + t];
      if (ta.scaled) mask |= 1 << t;
      for (int ar = 0; ar < n_in; ++ar)
        for (int e = 0; e < W; ++e) {
          const int i = ar - op->off_s + e - kb;
          if (i >= 0 && i < qs) leftT[((size_t)ar * nt + t) * W + e] = ta.l[(size_t)i * W + (2 * kb - e)];
        }
      // right bands in difference form: the centre slot holds the column sum
      // (the kernel forms sum_{d != kb} R[d] (x[d] - x[kb]) + (sum_d R[d]) x[kb])
      for (int j = 0; j < qt; ++j) {
        long double sum = 0.0L;
        for (int d = 0; d < W; ++d) sum += ta.r[(size_t)d * qt + j];
        for (int d = 0; d < W; ++d)
          right[((size_t)t * W + d) * qt + j] = d == kb ? (double)sum : ta.r[(size_t)d * qt + j];
      }
    }
    OpPass& P = op->pass[ps];
    P.nt = nt;
    P.scaled_mask = mask;
    P.pattern = (D.elem_order >= 2 && D.elem_order == kb &&
                 element_structured(leftT, n_in, nt, kb, op->off_s - op->ph_s)) ? 1 : 0;
    // left bands in telescoped form: output row i with coefficients c_k on its
    // input rows (k = 0 .. 2kb, the row layout's d) and first coupled k_lo
    // (0, or kb - phase for an element-interior node when the element
    // structure is used) takes the suffix sums S_k = sum_{k' >= k} c_k' for
    // k >= k_lo and 0 below; slot e of input row a carries S_{2kb - e}
    std::fill(leftT.begin(), leftT.end(), 0.0);
    for (int t = 0; t < take; ++t) {
      const TermArrays& ta = terms[t0 + t];
      for (int i = 0; i < qs; ++i) {
        const int phase = (i + op->ph_s) % kb;
        const int klo = (!P.pattern || phase == 0) ? 0 : kb - phase;
        long double suffix = 0.0L;
        for (int k = 2 * kb; k >= klo; --k) {
          suffix += ta.l[(size_t)i * W + k];
          const int ar = i + op->off_s + k - kb;  // input row of slot e = 2kb - k
          if (ar >= 0 && ar < n_in) leftT[((size_t)ar * nt + t) * W + (2 * kb - k)] = (double)suffix;
        }
      }
    }
    t0 += take;
    const int SW = band_cols_per_block(kb);
    for (int v = 0; v < 2; ++v) {
      const int TI = band_rows_per_block(kb, nt, v);
      P.n_rowblk[v] = (qs + op->ph_s + TI - 1) / TI;
      P.n_tiles[v] = ((qt + SW - 1) / SW) * P.n_rowblk[v];
    }
    int rc = dev_alloc(&P.d_left, leftT.size());
    if (rc == MOFEM_OK) rc = dev_alloc(&P.d_right, right.size());
    if (rc != MOFEM_OK) {
      mofem_op_destroy(op);
      return rc;
    }
    if (hipMemcpy(P.d_left, leftT.data(), leftT.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P.d_right, right.data(), right.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
      mofem_op_destroy(op);
      return fail(MOFEM_E_HIP, "op_create: upload failed");
    }
  }
  op->n_tiles_max = std::max(op->pass[n_pass - 1].n_tiles[0], op->pass[n_pass - 1].n_tiles[1]);
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
      op->n_cu = ncu;
  }
  *out = op;
  return MOFEM_OK;
}

extern "C" int mofem_op_destroy(mofem_op_t op) {
  if (!op) return MOFEM_OK;
  for (OpPass& P : op->pass) {
    if (P.d_left) (void)hipFree(P.d_left);
    if (P.d_right) (void)hipFree(P.d_right);
  }
  if (op->d_partial) (void)hipFree(op->d_partial);
  delete op;
  return MOFEM_OK;
}

extern "C" int mofem_op_shape(mofem_op_t op, int* qs, int* qt, int* in_s, int* in_t) {
  clear_error();
  if (!op) return fail(MOFEM_E_ARG, "op_shape: NULL handle");
  if (qs) *qs = op->qs;
  if (qt) *qt = op->qt;
  if (in_s) *in_s = op->ns_in;
  if (in_t) *in_t = op->nt_in;
  return MOFEM_OK;
}

namespace {
// Row-block variant of a launch over `batch` items: the small row blocks when
// the default grid would give fewer than two blocks per compute unit (two
// items share a lane where they can, so the default grid has tiles x
// ceil(batch / 2) blocks).  Every launch of one operator over one batch size
// takes the same variant, so its tile count (op_tiles) is known beforehand.
int op_variant(mofem_op_t op, int batch) {
  if (!band_has_small(op->kb)) return 0;
  const long long blocks = (long long)op->pass[op->n_pass - 1].n_tiles[0] * ((batch + 1) / 2);
  return blocks < 2LL * op->n_cu ? 1 : 0;
}
// partial sums per item of the fused <X, Y> of a launch over `batch` items
int op_tiles(mofem_op_t op, int batch) { return op->pass[op->n_pass - 1].n_tiles[op_variant(op, batch)]; }

// partial_stride: entries between items of `partial` (0: the launch's own
// tile count; a grouped solve of several operators uses their maximum)
int op_launch(mofem_op_t op, const double* X, long long in_stride, double* Y, long long stride, int batch,
              const double* item_scale, double* partial, const int* active, hipStream_t s,
              int n_items = -1, int partial_stride = 0) {
  TraceScope trace(MOFEM_TRACE_BAND, n_items < 0 ? batch : n_items, s);
  const int v = op_variant(op, batch);
  for (int ps = 0; ps < op->n_pass; ++ps) {
    const OpPass& P = op->pass[ps];
    const bool last = ps == op->n_pass - 1;
    BandArgs a{};
    a.X = X;
    a.in_stride = in_stride;
    a.ld_x = op->nt_in;
    a.Y = Y;
    a.out_stride = stride;
    a.ld_y = op->qt;
    a.qs = op->qs;
    a.qt = op->qt;
    a.ns_in = op->ns_in;
    a.nt_in = op->nt_in;
    a.off_s = op->off_s;
    a.off_t = op->off_t;
    a.ph_s = op->ph_s;
    a.n_rowblk = P.n_rowblk[v];
    a.left = P.d_left;
    a.right = P.d_right;
    a.scaled_mask = P.scaled_mask;
    a.item_scale = item_scale;
    a.dot_partial = last ? partial : nullptr;
    a.n_partial = partial_stride > 0 ? partial_stride : P.n_tiles[v];
    a.active = active;
    a.accumulate = ps > 0;  // later passes add to the earlier passes' Y
    a.batch = batch;
    if (launch_band_apply(a, op->kb, P.nt, batch, P.pattern != 0, v, s) != 0)
      return fail(MOFEM_E_UNSUPPORTED, "op_apply: unsupported band/term combination");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MOFEM_E_HIP, std::string("op_apply launch: ") + hipGetErrorString(e));
  }
  return MOFEM_OK;
}
}  // namespace

extern "C" int mofem_op_apply(mofem_op_t op, const double* X, long long in_stride, double* Y, long long stride,
                              int batch, const double* item_scale, double* dot_xy, void* stream) {
  clear_error();
  if (!op) return fail(MOFEM_E_ARG, "op_apply: NULL handle");
  if (batch < 0) return fail(MOFEM_E_ARG, "op_apply: negative batch");
  if (batch == 0) return MOFEM_OK;
  if (!X || !Y) return fail(MOFEM_E_ARG, "op_apply: NULL argument");
  if (in_stride < (long long)op->ns_in * op->nt_in || stride < (long long)op->qs * op->qt)
    return fail(MOFEM_E_ARG, "op_apply: stride smaller than one item");
  if (dot_xy && (op->full_input || op->full_output))
    return fail(MOFEM_E_ARG, "op_apply: <X, Y> needs a square operator");
  hipStream_t s = (hipStream_t)stream;
  double* partial = nullptr;
  if (dot_xy) {
    if (op->partial_batch < batch) {
      if (op->d_partial) {
        HIP_TRY(hipStreamSynchronize(s));
        (void)hipFree(op->d_partial);
        op->d_partial = nullptr;
      }
      int rc = dev_alloc(&op->d_partial, (size_t)batch * op->n_tiles_max);
      if (rc != MOFEM_OK) return rc;
      op->partial_batch = batch;
    }
    partial = op->d_partial;
  }
  int rc = op_launch(op, X, in_stride, Y, stride, batch, item_scale, partial, nullptr, s);
  if (rc != MOFEM_OK) return rc;
  if (dot_xy && launch_reduce(partial, op_tiles(op, batch), dot_xy, batch, s) != 0)
    return fail(MOFEM_E_HIP, "op_apply: reduce launch failed");
  return MOFEM_OK;
}

// ----------------------------------------------------------------------------
// Allocation-free operator apply: the per-tile partial sums of <X, Y> live in a
// file-scope device array (one copy per GPU, held until the process ends)
// instead of a buffer the handle allocates.  In host code `scratch` names a
// host-side stand-in, never the device copy: its device address is looked up
// once per device with hipGetSymbolAddress and only that address is used.
// ----------------------------------------------------------------------------
namespace {
constexpr size_t kScratchDoubles = MOFEM_NOALLOC_SCRATCH_BYTES / sizeof(double);
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kScratchDoubles];
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

int scratch_address(double** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MOFEM_E_ARG, "op_apply_noalloc: device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MOFEM_E_HIP, std::string("op_apply_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch_dev[dev] = (double*)p;
  }
  *out = g_scratch_dev[dev];
  return MOFEM_OK;
}
}  // namespace

extern "C" int mofem_op_apply_noalloc(mofem_op_t op, const double* X, long long in_stride, double* Y,
                                      long long stride, int batch, const double* item_scale, double* dot_xy,
                                      void* stream) {
  clear_error();
  if (!op) return fail(MOFEM_E_ARG, "op_apply_noalloc: NULL handle");
  if (batch < 0) return fail(MOFEM_E_ARG, "op_apply_noalloc: negative batch");
  if (batch == 0) return MOFEM_OK;
  if (!X || !Y) return fail(MOFEM_E_ARG, "op_apply_noalloc: NULL argument");
  if (in_stride < (long long)op->ns_in * op->nt_in || stride < (long long)op->qs * op->qt)
    return fail(MOFEM_E_ARG, "op_apply_noalloc: stride smaller than one item");
  if (dot_xy && (op->full_input || op->full_output))
    return fail(MOFEM_E_ARG, "op_apply_noalloc: <X, Y> needs a square operator");
  double* partial = nullptr;
  if (dot_xy) {
    const size_t need = (size_t)batch * op_tiles(op, batch);
    if (need > kScratchDoubles)
      return fail(MOFEM_E_ARG, "op_apply_noalloc: batch * tiles = " + std::to_string(need) +
                                   " partial sums exceed the static scratch of " +
                                   std::to_string(kScratchDoubles) + " (MOFEM_NOALLOC_SCRATCH_BYTES)");
    int rc = scratch_address(&partial);
    if (rc != MOFEM_OK) return rc;
  }
  TraceCapture no_trace;  // records no timing events (they would be created on demand)
  hipStream_t s = (hipStream_t)stream;
  // every tile of every item writes its partial sum, so nothing needs clearing
  int rc = op_launch(op, X, in_stride, Y, stride, batch, item_scale, partial, nullptr, s);
  if (rc != MOFEM_OK) return rc;
  if (dot_xy && launch_reduce(partial, op_tiles(op, batch), dot_xy, batch, s) != 0)
    return fail(MOFEM_E_HIP, "op_apply_noalloc: reduce launch failed");
  return MOFEM_OK;
}

// ============================================================================
// preconditioner
// ============================================================================
struct mofem_prec_s {
  int qs = 0, qt = 0, ps = 0, pt = 0;  // sizes and padded sizes
  double alpha = 0, bs = 0, bt = 0, dl = 0;
  int precision = MOFEM_PREC_F64;
  std::vector<double> h_lam, h_mu;
  double* lam = nullptr;
  double* mu = nullptr;
  double *Vs = nullptr, *VsT = nullptr, *Vt = nullptr, *VtT = nullptr;  // FP64 padded
  unsigned short *Vs_h = nullptr, *Vs_l = nullptr, *VsT_h = nullptr, *VsT_l = nullptr;
  unsigned short *Vt_h = nullptr, *Vt_l = nullptr, *VtT_h = nullptr, *VtT_l = nullptr;
  float *Vs_f = nullptr, *VsT_f = nullptr, *Vt_f = nullptr, *VtT_f = nullptr;  // FP32 padded
  // INT8 digit planes and row exponents of the padded bases (MOFEM_PREC_F64_INT8)
  signed char *Vs_i8 = nullptr, *VsT_i8 = nullptr, *Vt_i8 = nullptr, *VtT_i8 = nullptr;
  int *Vs_ex = nullptr, *VsT_ex = nullptr, *Vt_ex = nullptr, *VtT_ex = nullptr;
  std::vector<std::pair<long long, int>> tuned;  // (precision << 32 | batch) -> block tile
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // product preconditioner by banded Cholesky (mofem_prec_setup_banded)
  int banded = 0, kb = 0, n_sets = 0;
  double *Lf_s = nullptr, *Lb_s = nullptr, *Lf_t = nullptr, *Lb_t = nullptr, *scales = nullptr;
  std::vector<double> h_scales;  // host copy of the factor pairs' scales
};

namespace {
unsigned short host_bf16(float x) {
  unsigned u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
float host_bf16_to_f(unsigned short h) {
  unsigned u = ((unsigned)h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// padded copy (rows x cols -> pr x pc, zero padding), optionally transposed
std::vector<double> padded(const std::vector<double>& V, int q, int pr, int pc, bool transpose) {
  std::vector<double> P((size_t)pr * pc, 0.0);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) P[(size_t)i * pc + j] = transpose ? V[(size_t)j * q + i] : V[(size_t)i * q + j];
  return P;
}

int upload_f64(double** d, const std::vector<double>& h) {
  int rc = dev_alloc(d, h.size());
  if (rc) return rc;
  HIP_TRY(hipMemcpy(*d, h.data(), h.size() * 8, hipMemcpyHostToDevice));
  return MOFEM_OK;
}
int upload_f32(float** d, const std::vector<double>& h) {
  std::vector<float> f(h.size());
  for (size_t i = 0; i < h.size(); ++i) f[i] = (float)h[i];
  int rc = dev_alloc(d, f.size());
  if (rc) return rc;
  HIP_TRY(hipMemcpy(*d, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  return MOFEM_OK;
}

int upload_split(unsigned short** hi, unsigned short** lo, const std::vector<double>& h) {
  std::vector<unsigned short> vh(h.size()), vl(h.size());
  for (size_t i = 0; i < h.size(); ++i) {
    float f = (float)h[i];
    unsigned short a = host_bf16(f);
    vh[i] = a;
    vl[i] = host_bf16(f - host_bf16_to_f(a));
  }
  int rc = dev_alloc(hi, vh.size());
  if (rc) return rc;
  rc = dev_alloc(lo, vl.size());
  if (rc) return rc;
  HIP_TRY(hipMemcpy(*hi, vh.data(), vh.size() * 2, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(*lo, vl.data(), vl.size() * 2, hipMemcpyHostToDevice));
  return MOFEM_OK;
}
}  // namespace

extern "C" int mofem_prec_destroy(mofem_prec_t p) {
  if (!p) return MOFEM_OK;
  void* ptrs[] = {p->lam, p->mu, p->Vs, p->VsT, p->Vt, p->VtT, p->Vs_h, p->Vs_l, p->VsT_h,
                  p->VsT_l, p->Vt_h, p->Vt_l, p->VtT_h, p->VtT_l, p->Vs_f, p->VsT_f, p->Vt_f, p->VtT_f,
                  p->Vs_i8, p->VsT_i8, p->Vt_i8, p->VtT_i8, p->Vs_ex, p->VsT_ex, p->Vt_ex, p->VtT_ex,
                  p->ws, p->Lf_s, p->Lb_s, p->Lf_t, p->Lb_t, p->scales};
  for (void* x : ptrs)
    if (x) (void)hipFree(x);
  delete p;
  return MOFEM_OK;
}

namespace {
int prec_upload(mofem_prec_s* p, const std::vector<double>& Vs, const std::vector<double>& Vt);
}

extern "C" int mofem_prec_setup(const mofem_prec_desc* desc, mofem_prec_t* out) {
  clear_error();
  if (!desc || !out) return fail(MOFEM_E_ARG, "prec_setup: NULL argument");
  *out = nullptr;
  const mofem_prec_desc& D = *desc;
  if (D.kb < 1 || D.kb > 4) return fail(MOFEM_E_ARG, "prec_setup: kb must be 1..4");
  if (!D.Ks || !D.Ms || !D.Kt || !D.Mt) return fail(MOFEM_E_ARG, "prec_setup: NULL band");
  if ((D.trim_s != 0 && D.trim_s != 1) || (D.trim_t != 0 && D.trim_t != 1))
    return fail(MOFEM_E_ARG, "prec_setup: trim flags must be 0 or 1");
  if (D.precision < MOFEM_PREC_F64 || D.precision > MOFEM_PREC_BF16_FWD_VS)
    return fail(MOFEM_E_ARG, "prec_setup: unknown precision");
  const int qs = D.n_s - 2 * D.trim_s, qt = D.n_t - 2 * D.trim_t;
  if (qs < 1 || qt < 1) return fail(MOFEM_E_ARG, "prec_setup: empty matrices");
  for (const mofem_band_sum* bs : {&D.Ks_add, &D.Kt_add}) {
    if (bs->n < 0 || bs->n > MOFEM_MAX_BAND_SUM) return fail(MOFEM_E_ARG, "prec_setup: added bands: 0..4 terms");
    for (int i = 0; i < bs->n; ++i)
      if (!bs->band[i]) return fail(MOFEM_E_ARG, "prec_setup: NULL added band");
  }
  // K + sum_i coef_i band_i on the host (the same DIA layout)
  std::vector<double> ks_sum, kt_sum;
  auto with_added = [&](const double* K, const mofem_band_sum& A, int n, std::vector<double>& sum) {
    if (A.n == 0) return K;
    const size_t nb = (size_t)(2 * D.kb + 1) * n;
    sum.assign(K, K + nb);
    for (int t = 0; t < A.n; ++t)
      for (size_t i = 0; i < nb; ++i) sum[i] += A.coef[t] * A.band[t][i];
    return (const double*)sum.data();
  };
  const double* Ks = with_added(D.Ks, D.Ks_add, D.n_s, ks_sum);
  const double* Kt = with_added(D.Kt, D.Kt_add, D.n_t, kt_sum);

  auto* p = new mofem_prec_s();
  p->qs = qs;
  p->qt = qt;
  p->ps = pad_up(qs);
  p->pt = pad_up(qt);
  p->alpha = D.alpha;
  p->bs = D.beta_s;
  p->bt = D.beta_t;
  p->dl = D.delta;
  p->precision = D.precision;
  std::vector<double> Vs((size_t)qs * qs), Vt((size_t)qt * qt);
  p->h_lam.resize(qs);
  p->h_mu.resize(qt);
  // the two one-dimensional decompositions are independent: the t pencil runs
  // on a second host thread (or is copied when it equals the s pencil, as on
  // the square of eq. (28))
  const size_t nbs = (size_t)(2 * D.kb + 1) * D.n_s;
  const bool same = D.n_s == D.n_t && D.trim_s == D.trim_t &&
                    std::memcmp(Ks, Kt, nbs * sizeof(double)) == 0 &&
                    std::memcmp(D.Ms, D.Mt, nbs * sizeof(double)) == 0;
  int rc_t = MOFEM_OK;
  std::string msg_t;
  std::thread worker;
  // the two decompositions share this call's host threads
  const int threads = host_threads(), share = same ? threads : std::max(1, (threads + 1) / 2);
  if (!same) {
    worker = std::thread([&]() {
      set_thread_share(share);
      rc_t = mofem_geneig_host(D.n_t, D.kb, Kt, D.Mt, D.trim_t, p->h_mu.data(), Vt.data());
      if (rc_t != MOFEM_OK) msg_t = mofem_last_error();  // thread-local message of the worker
    });
  }
  const int prev_share = set_thread_share(share);
  int rc = mofem_geneig_host(D.n_s, D.kb, Ks, D.Ms, D.trim_s, p->h_lam.data(), Vs.data());
  set_thread_share(prev_share);
  std::string msg = rc != MOFEM_OK ? std::string(mofem_last_error()) : std::string();
  if (worker.joinable()) worker.join();
  if (same && rc == MOFEM_OK) {
    p->h_mu = p->h_lam;
    Vt = Vs;
  }
  if (rc == MOFEM_OK && rc_t != MOFEM_OK) {
    rc = rc_t;
    msg = msg_t;
  }
  if (rc != MOFEM_OK) {
    mofem_prec_destroy(p);
    return fail(rc, "prec_setup: " + msg);
  }
  rc = prec_upload(p, Vs, Vt);
  if (rc) {
    mofem_prec_destroy(p);
    return rc;
  }
  *out = p;
  return MOFEM_OK;
}

// Spectral preconditioner from given generalised eigenpairs (e.g. the closed
// forms of mofem_eig_p1_closed), no eigen-decomposition.
extern "C" int mofem_prec_setup_eig(int q_s, int q_t, const double* lam, const double* Vs, const double* mu,
                                    const double* Vt, double alpha, double beta_s, double beta_t, double delta,
                                    int precision, mofem_prec_t* out) {
  clear_error();
  if (!out || !lam || !Vs || !mu || !Vt) return fail(MOFEM_E_ARG, "prec_setup_eig: NULL argument");
  *out = nullptr;
  if (q_s < 1 || q_t < 1) return fail(MOFEM_E_ARG, "prec_setup_eig: empty matrices");
  if (precision < MOFEM_PREC_F64 || precision > MOFEM_PREC_BF16_FWD_VS)
    return fail(MOFEM_E_ARG, "prec_setup_eig: unknown precision");
  auto* p = new mofem_prec_s();
  p->qs = q_s;
  p->qt = q_t;
  p->ps = pad_up(q_s);
  p->pt = pad_up(q_t);
  p->alpha = alpha;
  p->bs = beta_s;
  p->bt = beta_t;
  p->dl = delta;
  p->precision = precision;
  p->h_lam.assign(lam, lam + q_s);
  p->h_mu.assign(mu, mu + q_t);
  std::vector<double> vs(Vs, Vs + (size_t)q_s * q_s), vt(Vt, Vt + (size_t)q_t * q_t);
  int rc = prec_upload(p, vs, vt);
  if (rc) {
    mofem_prec_destroy(p);
    return rc;
  }
  *out = p;
  return MOFEM_OK;
}

namespace {
// Upload the eigenvalues (p->h_lam, p->h_mu) and the bases V_s, V_t (row-major,
// column j = eigenvector j) and their transposes, padded, in FP64, split BF16
// and FP32.
int prec_upload(mofem_prec_s* p, const std::vector<double>& Vs, const std::vector<double>& Vt) {
  const int qs = p->qs, qt = p->qt;
  int rc = MOFEM_OK;
  auto Vs_p = padded(Vs, qs, p->ps, p->ps, false), VsT_p = padded(Vs, qs, p->ps, p->ps, true);
  auto Vt_p = padded(Vt, qt, p->pt, p->pt, false), VtT_p = padded(Vt, qt, p->pt, p->pt, true);
  rc = upload_f64(&p->lam, p->h_lam);
  if (!rc) rc = upload_f64(&p->mu, p->h_mu);
  if (!rc) rc = upload_f64(&p->Vs, Vs_p);
  if (!rc) rc = upload_f64(&p->VsT, VsT_p);
  if (!rc) rc = upload_f64(&p->Vt, Vt_p);
  if (!rc) rc = upload_f64(&p->VtT, VtT_p);
  if (!rc) rc = upload_split(&p->Vs_h, &p->Vs_l, Vs_p);
  if (!rc) rc = upload_split(&p->VsT_h, &p->VsT_l, VsT_p);
  if (!rc) rc = upload_split(&p->Vt_h, &p->Vt_l, Vt_p);
  if (!rc) rc = upload_split(&p->VtT_h, &p->VtT_l, VtT_p);
  if (!rc) rc = upload_f32(&p->Vs_f, Vs_p);
  if (!rc) rc = upload_f32(&p->VsT_f, VsT_p);
  if (!rc) rc = upload_f32(&p->Vt_f, Vt_p);
  if (!rc) rc = upload_f32(&p->VtT_f, VtT_p);
  // INT8 digit planes of the padded FP64 bases, cut on the device (bases
  // wider than the INT8 products take stay without them)
  if (!rc && p->ps <= kOzMaxK && p->pt <= kOzMaxK) {
    struct {
      const double* src;
      int n;
      signed char** out;
      int** ex;
    } bases[4] = {{p->Vs, p->ps, &p->Vs_i8, &p->Vs_ex}, {p->VsT, p->ps, &p->VsT_i8, &p->VsT_ex},
                  {p->Vt, p->pt, &p->Vt_i8, &p->Vt_ex}, {p->VtT, p->pt, &p->VtT_i8, &p->VtT_ex}};
    for (auto& B : bases) {
      if (!rc) rc = dev_alloc(B.out, (size_t)kOzSlices * B.n * B.n);
      if (!rc) rc = dev_alloc(B.ex, (size_t)B.n);
      if (!rc && launch_slice_rows(B.src, 0, B.n, B.n, B.n, *B.out, 0, *B.ex, 0, 1, nullptr, nullptr))
        rc = fail(MOFEM_E_HIP, "prec_setup: slice launch failed");
    }
    if (!rc) HIP_TRY(hipStreamSynchronize(nullptr));
  }
  if (!rc && p->precision == MOFEM_PREC_F64_INT8 && !p->Vs_i8)
    rc = fail(MOFEM_E_UNSUPPORTED, "prec_setup: INT8 transforms take padded widths up to 16384");
  return rc;
}
}  // namespace

// Product preconditioner S U T by banded Cholesky: factor S_j = a Ms + c_j bs Ks
// and T_j = a Mt + c_j bt Kt (interior rows and columns) for every scale c_j.
extern "C" int mofem_prec_setup_banded(const mofem_bprec_desc* desc, mofem_prec_t* out) {
  clear_error();
  if (!desc || !out) return fail(MOFEM_E_ARG, "prec_setup_banded: NULL argument");
  *out = nullptr;
  const mofem_bprec_desc& D = *desc;
  if (D.kb < 1 || D.kb > 4) return fail(MOFEM_E_ARG, "prec_setup_banded: kb must be 1..4");
  for (const mofem_band_sum* bs : {&D.Ks, &D.Ms, &D.Kt, &D.Mt}) {
    if (bs->n < 0 || bs->n > MOFEM_MAX_BAND_SUM) return fail(MOFEM_E_ARG, "prec_setup_banded: band sum of 0..4 terms");
    for (int i = 0; i < bs->n; ++i)
      if (!bs->band[i]) return fail(MOFEM_E_ARG, "prec_setup_banded: NULL band");
  }
  if (D.Ks.n < 1 || D.Kt.n < 1 || (D.a != 0.0 && (D.Ms.n < 1 || D.Mt.n < 1)))
    return fail(MOFEM_E_ARG, "prec_setup_banded: Ks and Kt (and Ms, Mt when a != 0) need at least one band");
  if ((D.trim_s != 0 && D.trim_s != 1) || (D.trim_t != 0 && D.trim_t != 1))
    return fail(MOFEM_E_ARG, "prec_setup_banded: trim flags must be 0 or 1");
  if (D.n_scales < 1 || D.n_scales > MOFEM_MAX_SCALES) return fail(MOFEM_E_ARG, "prec_setup_banded: n_scales 1..8");
  const int qs = D.n_s - 2 * D.trim_s, qt = D.n_t - 2 * D.trim_t;
  if (qs < 1 || qt < 1) return fail(MOFEM_E_ARG, "prec_setup_banded: empty matrices");
  const int kb = D.kb, w = 2 * kb + 1, c = kb + 1;
  // entry (DIA offset d, node i) of a band sum (DIA input: band[d * n + i] = K[i][i + d - kb])
  auto entry = [](const mofem_band_sum& B, size_t at) {
    double v = 0.0;
    for (int t = 0; t < B.n; ++t) v += B.coef[t] * B.band[t][at];
    return v;
  };
  // interior band rows of a Ms + sc b Ks
  auto combine = [&](int n, int trim, const mofem_band_sum& K, const mofem_band_sum& M, double b, double sc) {
    const int q = n - 2 * trim;
    std::vector<double> S((size_t)q * w, 0.0);
    for (int i = 0; i < q; ++i)
      for (int d = 0; d < w; ++d) {
        const int j = i + d - kb;
        if (j < 0 || j >= q) continue;
        const size_t at = (size_t)d * n + i + trim;
        S[(size_t)i * w + d] = (D.a != 0.0 ? D.a * entry(M, at) : 0.0) + sc * b * entry(K, at);
      }
    return S;
  };
  std::vector<double> Lf_s((size_t)D.n_scales * qs * c), Lb_s(Lf_s.size());
  std::vector<double> Lf_t((size_t)D.n_scales * qt * c), Lb_t(Lf_t.size());
  std::vector<double> sc(D.scales, D.scales + D.n_scales);
  for (int j = 0; j < D.n_scales; ++j) {
    auto S = combine(D.n_s, D.trim_s, D.Ks, D.Ms, D.bs, sc[j]);
    auto T = combine(D.n_t, D.trim_t, D.Kt, D.Mt, D.bt, sc[j]);
    if (band_cholesky(qs, kb, S.data(), &Lf_s[(size_t)j * qs * c], &Lb_s[(size_t)j * qs * c]) != MOFEM_OK ||
        band_cholesky(qt, kb, T.data(), &Lf_t[(size_t)j * qt * c], &Lb_t[(size_t)j * qt * c]) != MOFEM_OK)
      return fail(MOFEM_E_NUMERIC, "prec_setup_banded: a factor is not positive definite");
  }
  auto* p = new mofem_prec_s();
  p->qs = qs;
  p->qt = qt;
  p->ps = qs;
  p->pt = qt;
  p->precision = MOFEM_PREC_F64;
  p->banded = 1;
  p->kb = kb;
  p->n_sets = D.n_scales;
  int rc = upload_f64(&p->Lf_s, Lf_s);
  if (!rc) rc = upload_f64(&p->Lb_s, Lb_s);
  if (!rc) rc = upload_f64(&p->Lf_t, Lf_t);
  if (!rc) rc = upload_f64(&p->Lb_t, Lb_t);
  if (!rc) rc = upload_f64(&p->scales, sc);
  if (rc) {
    mofem_prec_destroy(p);
    return rc;
  }
  p->h_scales = sc;
  *out = p;
  return MOFEM_OK;
}

extern "C" int mofem_prec_set_coeffs(mofem_prec_t p, double a, double bs, double bt, double d) {
  clear_error();
  if (!p) return fail(MOFEM_E_ARG, "prec_set_coeffs: NULL handle");
  if (p->banded) return fail(MOFEM_E_UNSUPPORTED, "prec_set_coeffs: banded product preconditioner");
  p->alpha = a;
  p->bs = bs;
  p->bt = bt;
  p->dl = d;
  return MOFEM_OK;
}

extern "C" int mofem_prec_set_precision(mofem_prec_t p, int precision) {
  clear_error();
  if (!p) return fail(MOFEM_E_ARG, "prec_set_precision: NULL handle");
  if (precision < MOFEM_PREC_F64 || precision > MOFEM_PREC_BF16_FWD_VS) return fail(MOFEM_E_ARG, "unknown precision");
  if (precision == MOFEM_PREC_F64_INT8 && !p->banded && (p->ps > kOzMaxK || p->pt > kOzMaxK))
    return fail(MOFEM_E_UNSUPPORTED, "prec_set_precision: INT8 transforms take padded widths up to 16384");
  if (p->banded && precision != MOFEM_PREC_F64)
    return fail(MOFEM_E_UNSUPPORTED, "prec_set_precision: the banded product preconditioner is FP64 only");
  p->precision = precision;
  return MOFEM_OK;
}

extern "C" int mofem_prec_eigenvalues(mofem_prec_t p, double* lam, double* mu) {
  clear_error();
  if (!p) return fail(MOFEM_E_ARG, "prec_eigenvalues: NULL handle");
  if (p->banded) return fail(MOFEM_E_UNSUPPORTED, "prec_eigenvalues: banded product preconditioner");
  if (lam) std::memcpy(lam, p->h_lam.data(), sizeof(double) * p->qs);
  if (mu) std::memcpy(mu, p->h_mu.data(), sizeof(double) * p->qt);
  return MOFEM_OK;
}

extern "C" size_t mofem_prec_workspace_size(mofem_prec_t p, int batch) {
  if (!p || batch < 1) return 0;
  // sized for the widest precision (FP64 intermediates), so that a workspace
  // stays valid when mofem_prec_set_precision switches the handle
  size_t items = (size_t)p->ps * p->pt * batch;
  if (p->banded) return 2 * align_up(items * 8, 256) + 2048;  // substitution scratch, S^-1 R
  return 3 * align_up(items * 8, 256) + 2048;
}

namespace {
// Product mode of the four transforms of a split-BF16 family precision.
void split_modes(int precision, int* mode) {
  const int m = precision == MOFEM_PREC_BF16     ? GEMM_BF16
                : precision == MOFEM_PREC_BF16X2 ? GEMM_BF16X2
                                                 : GEMM_BF16X3;
  for (int i = 0; i < 4; ++i) mode[i] = m;
  if (precision == MOFEM_PREC_BF16_FWD || precision == MOFEM_PREC_BF16_FWD_VS)
    mode[0] = mode[1] = GEMM_BF16;  // forward in BF16
  if (precision == MOFEM_PREC_BF16_FWD_VS) mode[2] = GEMM_BF16X2;  // V_s split, S plain
}
int split_trace_class(int gemm_mode) {
  return gemm_mode == GEMM_BF16 ? MOFEM_TRACE_GEMM_BF16
         : gemm_mode == GEMM_BF16X2 ? MOFEM_TRACE_GEMM_BF16X2
                                    : MOFEM_TRACE_GEMM_BF16X3;
}

// The padded first-transform operand inside a preconditioner workspace (the
// first buffer prec_launch carves): FP64, or split BF16 as two halves.
struct PrecInput {
  double* f64 = nullptr;
  float* f32 = nullptr;
  unsigned short* hi = nullptr;
  unsigned short* lo = nullptr;
  long long stride = 0;  // elements between items
};
PrecInput prec_input(mofem_prec_t p, void* ws, size_t ws_bytes, int batch) {
  PrecInput in;
  if (p->banded) return in;  // the solves read R itself
  const size_t items = (size_t)p->ps * p->pt;
  Carve c(ws, ws_bytes);
  if (p->precision == MOFEM_PREC_F64 || p->precision == MOFEM_PREC_F64_INT8) {
    in.f64 = c.take<double>(items * batch);  // INT8: cut into digits from there
  } else if (p->precision == MOFEM_PREC_F32) {
    in.f32 = c.take<float>(items * batch);
  } else {
    in.hi = c.take<unsigned short>(items * batch);
    in.lo = c.take<unsigned short>(items * batch);
    int mode[4];
    split_modes(p->precision, mode);
    if (mode[0] == GEMM_BF16) in.lo = nullptr;  // the first transform reads hi only
  }
  in.stride = (long long)items;
  return in;
}

// Block tile of the transforms for this batch: the tuned choice if
// mofem_prec_tune measured one, else 128 unless the 128-tile grid would not
// give every CU two blocks.
int prec_tile(mofem_prec_t p, int batch) {
  const long long key = ((long long)p->precision << 32) | (unsigned)batch;
  for (auto& kv : p->tuned)
    if (kv.first == key) return kv.second;
  const long long blocks128 = (long long)(p->ps / 128) * (p->pt / 128) * batch;
  return blocks128 < 2 * 256 ? 64 : 128;
}

// Per-item device pointer tables of a grouped solve (instances of one shape,
// each with its own preconditioner): table k of item b at tabs[k * batch + b].
enum PrecTab {
  TB_VS64, TB_VST64, TB_VT64, TB_VTT64, TB_VS32, TB_VST32, TB_VT32, TB_VTT32,
  TB_VSH, TB_VSTH, TB_VTH, TB_VTTH, TB_VSL, TB_VSTL, TB_VTL, TB_VTTL,
  TB_VSI8, TB_VSTI8, TB_VTI8, TB_VTTI8, TB_VSEX, TB_VSTEX, TB_VTEX, TB_VTTEX,
  TB_LAM, TB_MU, TB_COUNT
};
// the tables' entries for one preconditioner
void prec_tab_entries(mofem_prec_t p, const void** e) {
  const void* v[TB_COUNT] = {p->Vs, p->VsT, p->Vt, p->VtT, p->Vs_f, p->VsT_f, p->Vt_f, p->VtT_f,
                             p->Vs_h, p->VsT_h, p->Vt_h, p->VtT_h, p->Vs_l, p->VsT_l, p->Vt_l, p->VtT_l,
                             p->Vs_i8, p->VsT_i8, p->Vt_i8, p->VtT_i8, p->Vs_ex, p->VsT_ex, p->Vt_ex, p->VtT_ex,
                             p->lam, p->mu};
  for (int k = 0; k < TB_COUNT; ++k) e[k] = v[k];
}

// input_ready: the padded operand of R is already in the workspace (written
// by the fused CG update).  z32: if set (FP32 and BF16 transforms only), the
// last transform writes Z in FP32 there (same item stride) instead of Z.
// tabs: per-item bases and eigenvalues of a grouped solve (PrecTab), or null
// (every item uses p's).
int prec_launch(mofem_prec_t p, const double* R, double* Z, long long stride, int batch,
                const double* item_scale, void* ws, size_t ws_bytes, const int* active, hipStream_t s,
                int n_items = -1, int input_ready = 0, float* z32 = nullptr, const void* const* tabs = nullptr) {
  const double items_done = n_items < 0 ? batch : n_items;
  if (tabs && p->banded) return fail(MOFEM_E_UNSUPPORTED, "prec_apply: grouped banded preconditioners");
  const size_t items = (size_t)p->ps * p->pt;
  if (p->banded) {
    // Z = S^-1 R T^-1: two transposing banded solves
    Carve c(ws, ws_bytes);
    double* W = c.take<double>(items * batch);
    double* Yt = c.take<double>(items * batch);
    if (!W || !Yt) return fail(MOFEM_E_ARG, "prec_apply: workspace too small");
    BcholArgs a{};
    a.W = W;
    a.w_stride = (long long)items;
    a.scales = p->scales;
    a.n_sets = p->n_sets;
    a.item_scale = item_scale;
    a.active = active;
    a.X = R; a.x_stride = stride; a.ld_x = p->qt;
    a.Out = Yt; a.o_stride = (long long)items; a.ld_o = p->qs;
    a.n_rows = p->qs; a.n_cols = p->qt; a.Lf = p->Lf_s; a.Lb = p->Lb_s;
    {
      TraceScope trace(MOFEM_TRACE_BCHOL, items_done, s);
      if (launch_bchol(a, p->kb, batch, s)) return fail(MOFEM_E_HIP, "banded solve launch");
    }
    a.X = Yt; a.x_stride = (long long)items; a.ld_x = p->qs;
    a.Out = Z; a.o_stride = stride; a.ld_o = p->qt;
    a.n_rows = p->qt; a.n_cols = p->qs; a.Lf = p->Lf_t; a.Lb = p->Lb_t;
    {
      TraceScope trace(MOFEM_TRACE_BCHOL, items_done, s);
      if (launch_bchol(a, p->kb, batch, s)) return fail(MOFEM_E_HIP, "banded solve launch");
    }
    return MOFEM_OK;
  }
  GemmArgs g{};
  g.lam = p->lam;
  g.mu = p->mu;
  g.alpha = p->alpha;
  g.beta_s = p->bs;
  g.beta_t = p->bt;
  g.delta = p->dl;
  g.item_scale = item_scale;
  g.out_scale = 1.0;
  g.active = active;
  // per-item basis operands (grouped solves): the data operand never has a table
  auto tab = [&](int k) -> const void* const* { return (tabs && k >= 0) ? tabs + (size_t)k * batch : nullptr; };
  g.lam_item = (const double* const*)tab(TB_LAM);
  g.mu_item = (const double* const*)tab(TB_MU);
  auto item_tabs = [&](int ah, int al, int ae, int bh, int bl, int be) {
    g.a_item = tab(ah);
    g.a_item_lo = tab(al);
    g.a_exp_item = (const int* const*)tab(ae);
    g.b_item = tab(bh);
    g.b_item_lo = tab(bl);
    g.b_exp_item = (const int* const*)tab(be);
  };
  const int prec = p->precision == MOFEM_PREC_F64        ? GEMM_F64
                   : p->precision == MOFEM_PREC_F32      ? GEMM_F32
                   : p->precision == MOFEM_PREC_BF16     ? GEMM_BF16
                   : p->precision == MOFEM_PREC_BF16X2   ? GEMM_BF16X2
                   : p->precision == MOFEM_PREC_F64_INT8 ? GEMM_I8
                                                         : GEMM_BF16X3;  // BF16X3 and both forward-BF16 modes: split branch
  const int tcls = prec == GEMM_F64      ? MOFEM_TRACE_GEMM_F64
                   : prec == GEMM_F32    ? MOFEM_TRACE_GEMM_F32
                   : prec == GEMM_BF16   ? MOFEM_TRACE_GEMM_BF16
                   : prec == GEMM_BF16X2 ? MOFEM_TRACE_GEMM_BF16X2
                   : prec == GEMM_I8     ? MOFEM_TRACE_GEMM_I8
                                         : MOFEM_TRACE_GEMM_BF16X3;
  const int tile = prec_tile(p, batch);
  auto gemm = [&](int omode) -> int {
    TraceScope trace(tcls, items_done, s);
    return launch_gemm(g, prec, omode, batch, tile, s);
  };
  Carve c(ws, ws_bytes);
  if (prec == GEMM_F64) {
    double* T0 = c.take<double>(items * batch);  // padded R
    double* T1 = c.take<double>(items * batch);  // T' then W
    double* T2 = c.take<double>(items * batch);  // S'
    if (!T0 || !T1 || !T2) return fail(MOFEM_E_ARG, "prec_apply: workspace too small");
    const long long istr = (long long)items;
    if (!input_ready) {
      TraceScope trace(MOFEM_TRACE_VEC, items_done, s);
      if (launch_pad_operand(R, stride, p->qs, p->qt, T0, nullptr, nullptr, nullptr, istr, 0, batch, active, s))
        return fail(MOFEM_E_HIP, "pad launch");
    }
    // G1: T' = (R V_t)^T
    g.M = p->qs; g.N = p->qt; g.K = p->qt;
    g.a64 = T0; g.a_stride = istr; g.b64 = p->VtT; g.b_stride = 0;
    g.c64 = T1; g.c_stride = istr; g.divide = 0;
    item_tabs(-1, -1, -1, TB_VTT64, -1, -1);
    if (gemm(O_PAD_T)) return fail(MOFEM_E_HIP, "gemm launch");
    // G2: S' = (V_s^T T ./ D)^T
    g.M = p->qs; g.N = p->qt; g.K = p->qs;
    g.a64 = p->VsT; g.a_stride = 0; g.b64 = T1; g.b_stride = istr;
    g.c64 = T2; g.c_stride = istr; g.divide = 1;
    item_tabs(TB_VST64, -1, -1, -1, -1, -1);
    if (gemm(O_PAD_T)) return fail(MOFEM_E_HIP, "gemm launch");
    // G3: W = V_s S
    g.M = p->qs; g.N = p->qt; g.K = p->qs;
    g.a64 = p->Vs; g.a_stride = 0; g.b64 = T2; g.b_stride = istr;
    g.c64 = T1; g.c_stride = istr; g.divide = 0;
    item_tabs(TB_VS64, -1, -1, -1, -1, -1);
    if (gemm(O_PAD_N)) return fail(MOFEM_E_HIP, "gemm launch");
    // G4: Z = W V_t^T
    g.M = p->qs; g.N = p->qt; g.K = p->qt;
    g.a64 = T1; g.a_stride = istr; g.b64 = p->Vt; g.b_stride = 0;
    g.c64 = Z; g.c_stride = stride; g.divide = 0;
    item_tabs(-1, -1, -1, TB_VT64, -1, -1);
    if (gemm(O_F64_RAW)) return fail(MOFEM_E_HIP, "gemm launch");
  } else if (prec == GEMM_I8) {
    // FP64 intermediates (R padded, T', S', W in turn), each cut into digit
    // planes before the product that reads it
    double* T = c.take<double>(items * batch);
    signed char* SL = c.take<signed char>((size_t)kOzSlices * items * batch);
    const int pmax = std::max(p->ps, p->pt);
    int* EX = c.take<int>((size_t)pmax * batch);
    if (!T || !SL || !EX) return fail(MOFEM_E_ARG, "prec_apply: workspace too small");
    if (!p->Vs_i8) return fail(MOFEM_E_UNSUPPORTED, "prec_apply: INT8 transforms take padded widths up to 16384");
    const long long istr = (long long)items, sstr = (long long)kOzSlices * items;
    auto slice = [&](const double* X, long long xs, int ld, int M, int K) -> int {
      TraceScope trace(MOFEM_TRACE_VEC, items_done, s);
      return launch_slice_rows(X, xs, ld, M, K, SL, sstr, EX, pmax, batch, active, s);
    };
    auto gemm8 = [&](int omode) -> int {
      TraceScope trace(tcls, items_done, s);
      return launch_gemm_i8(g, omode, batch, s);
    };
    // R (raw, or padded by the fused CG update) -> digits
    if (input_ready ? slice(T, istr, p->pt, p->qs, p->qt) : slice(R, stride, p->qt, p->qs, p->qt))
      return fail(MOFEM_E_HIP, "slice launch");
    // G1: T' = (R V_t)^T
    g.M = p->qs; g.N = p->qt; g.K = p->qt;
    g.a_i8 = SL; g.a_stride = sstr; g.a_exp = EX; g.a_exp_stride = pmax;
    g.b_i8 = p->VtT_i8; g.b_stride = 0; g.b_exp = p->VtT_ex; g.b_exp_stride = 0;
    g.c64 = T; g.c_stride = istr; g.divide = 0;
    item_tabs(-1, -1, -1, TB_VTTI8, -1, TB_VTTEX);
    if (gemm8(O_PAD_T) || slice(T, istr, p->ps, p->qt, p->qs)) return fail(MOFEM_E_HIP, "gemm launch");
    // G2: S' = (V_s^T T ./ D)^T
    g.M = p->qs; g.N = p->qt; g.K = p->qs;
    g.a_i8 = p->VsT_i8; g.a_stride = 0; g.a_exp = p->VsT_ex; g.a_exp_stride = 0;
    g.b_i8 = SL; g.b_stride = sstr; g.b_exp = EX; g.b_exp_stride = pmax;
    g.c64 = T; g.c_stride = istr; g.divide = 1;
    item_tabs(TB_VSTI8, -1, TB_VSTEX, -1, -1, -1);
    if (gemm8(O_PAD_T) || slice(T, istr, p->ps, p->qt, p->qs)) return fail(MOFEM_E_HIP, "gemm launch");
    // G3: W = V_s S
    g.M = p->qs; g.N = p->qt; g.K = p->qs;
    g.a_i8 = p->Vs_i8; g.a_stride = 0; g.a_exp = p->Vs_ex; g.a_exp_stride = 0;
    g.b_i8 = SL; g.b_stride = sstr; g.b_exp = EX; g.b_exp_stride = pmax;
    g.c64 = T; g.c_stride = istr; g.divide = 0;
    item_tabs(TB_VSI8, -1, TB_VSEX, -1, -1, -1);
    if (gemm8(O_PAD_N) || slice(T, istr, p->pt, p->qs, p->qt)) return fail(MOFEM_E_HIP, "gemm launch");
    // G4: Z = W V_t^T
    g.M = p->qs; g.N = p->qt; g.K = p->qt;
    g.a_i8 = SL; g.a_stride = sstr; g.a_exp = EX; g.a_exp_stride = pmax;
    g.b_i8 = p->Vt_i8; g.b_stride = 0; g.b_exp = p->Vt_ex; g.b_exp_stride = 0;
    g.c64 = Z; g.c_stride = stride; g.divide = 0;
    item_tabs(-1, -1, -1, TB_VTI8, -1, TB_VTEX);
    if (gemm8(O_F64_RAW)) return fail(MOFEM_E_HIP, "gemm launch");
  } else if (prec == GEMM_F32) {
    float* T0 = c.take<float>(items * batch);  // padded R
    float* T1 = c.take<float>(items * batch);  // T' then W
    float* T2 = c.take<float>(items * batch);  // S'
    if (!T0 || !T1 || !T2) return fail(MOFEM_E_ARG, "prec_apply: workspace too small");
    const long long istr = (long long)items;
    if (!input_ready) {
      TraceScope trace(MOFEM_TRACE_VEC, items_done, s);
      if (launch_pad_operand(R, stride, p->qs, p->qt, nullptr, T0, nullptr, nullptr, istr, 0, batch, active, s))
        return fail(MOFEM_E_HIP, "pad launch");
    }
    g.M = p->qs; g.N = p->qt; g.K = p->qt;
    g.a_hi = T0; g.a_stride = istr; g.b_hi = p->VtT_f; g.b_stride = 0;
    g.c_hi = T1; g.c_stride = istr; g.divide = 0;
    item_tabs(-1, -1, -1, TB_VTT32, -1, -1);
    if (gemm(O_PAD_T)) return fail(MOFEM_E_HIP, "gemm launch");
    g.M = p->qs; g.N = p->qt; g.K = p->qs;
    g.a_hi = p->VsT_f; g.a_stride = 0; g.b_hi = T1; g.b_stride = istr;
    g.c_hi = T2; g.c_stride = istr; g.divide = 1;
    item_tabs(TB_VST32, -1, -1, -1, -1, -1);
    if (gemm(O_PAD_T)) return fail(MOFEM_E_HIP, "gemm launch");
    g.M = p->qs; g.N = p->qt; g.K = p->qs;
    g.a_hi = p->Vs_f; g.a_stride = 0; g.b_hi = T2; g.b_stride = istr;
    g.c_hi = T1; g.c_stride = istr; g.divide = 0;
    item_tabs(TB_VS32, -1, -1, -1, -1, -1);
    if (gemm(O_PAD_N)) return fail(MOFEM_E_HIP, "gemm launch");
    g.M = p->qs; g.N = p->qt; g.K = p->qt;
    g.a_hi = T1; g.a_stride = istr; g.b_hi = p->Vt_f; g.b_stride = 0;
    g.c64 = Z; g.c_hi = z32; g.c_stride = stride; g.divide = 0;
    item_tabs(-1, -1, -1, TB_VT32, -1, -1);
    if (gemm(z32 ? O_F32_RAW : O_F64_RAW)) return fail(MOFEM_E_HIP, "gemm launch");
  } else {
    unsigned short* T0h = c.take<unsigned short>(items * batch);
    unsigned short* T0l = c.take<unsigned short>(items * batch);
    unsigned short* T1h = c.take<unsigned short>(items * batch);
    unsigned short* T1l = c.take<unsigned short>(items * batch);
    unsigned short* T2h = c.take<unsigned short>(items * batch);
    unsigned short* T2l = c.take<unsigned short>(items * batch);
    if (!T0h || !T0l || !T1h || !T1l || !T2h || !T2l) return fail(MOFEM_E_ARG, "prec_apply: workspace too small");
    const long long istr = (long long)items;
    // product mode of each transform G1..G4 and whether it reads its operands' lo halves
    int mode[4];
    split_modes(p->precision, mode);
    // A two-product transform splits the data operand (exact-BF16 bases) or,
    // in the first back transform of MOFEM_PREC_BF16_FWD_VS, the eigenbasis.
    const int data_is_a[4] = {1, 0, 0, 1};
    const bool basis_split = p->precision == MOFEM_PREC_BF16_FWD_VS;
    auto split_a = [&](int i) { return basis_split ? !data_is_a[i] : (bool)data_is_a[i]; };
    auto a_lo = [&](int i) { return mode[i] == GEMM_BF16X3 || (mode[i] == GEMM_BF16X2 && split_a(i)); };
    auto b_lo = [&](int i) { return mode[i] == GEMM_BF16X3 || (mode[i] == GEMM_BF16X2 && !split_a(i)); };
    auto run = [&](int i, int omode) -> int {
      g.split_a = split_a(i);
      TraceScope trace(split_trace_class(mode[i]), items_done, s);
      return launch_gemm(g, mode[i], omode, batch, tile, s);
    };
    if (!input_ready) {
      TraceScope trace(MOFEM_TRACE_VEC, items_done, s);
      if (launch_pad_operand(R, stride, p->qs, p->qt, nullptr, nullptr, T0h, a_lo(0) ? T0l : nullptr, istr, 1, batch,
                             active, s))
        return fail(MOFEM_E_HIP, "pad launch");
    }
    // G1: T' = (R V_t)^T
    g.M = p->qs; g.N = p->qt; g.K = p->qt;
    g.a_hi = T0h; g.a_lo = T0l; g.a_stride = istr; g.b_hi = p->VtT_h; g.b_lo = p->VtT_l; g.b_stride = 0;
    g.c_hi = T1h; g.c_lo = b_lo(1) ? T1l : nullptr; g.c_stride = istr; g.divide = 0;
    item_tabs(-1, -1, -1, TB_VTTH, TB_VTTL, -1);
    if (run(0, O_PAD_T)) return fail(MOFEM_E_HIP, "gemm launch");
    // G2: S' = (V_s^T T ./ D)^T
    g.M = p->qs; g.N = p->qt; g.K = p->qs;
    g.a64 = nullptr; g.a_hi = p->VsT_h; g.a_lo = p->VsT_l; g.a_stride = 0;
    g.b_hi = T1h; g.b_lo = T1l; g.b_stride = istr;
    g.c_hi = T2h; g.c_lo = b_lo(2) ? T2l : nullptr; g.c_stride = istr; g.divide = 1;
    item_tabs(TB_VSTH, TB_VSTL, -1, -1, -1, -1);
    if (run(1, O_PAD_T)) return fail(MOFEM_E_HIP, "gemm launch");
    // G3: W = V_s S
    g.M = p->qs; g.N = p->qt; g.K = p->qs;
    g.a_hi = p->Vs_h; g.a_lo = p->Vs_l; g.a_stride = 0;
    g.b_hi = T2h; g.b_lo = T2l; g.b_stride = istr;
    g.c_hi = T1h; g.c_lo = a_lo(3) ? T1l : nullptr; g.c_stride = istr; g.divide = 0;
    item_tabs(TB_VSH, TB_VSL, -1, -1, -1, -1);
    if (run(2, O_PAD_N)) return fail(MOFEM_E_HIP, "gemm launch");
    // G4: Z = W V_t^T
    g.M = p->qs; g.N = p->qt; g.K = p->qt;
    g.a_hi = T1h; g.a_lo = T1l; g.a_stride = istr;
    g.b_hi = p->Vt_h; g.b_lo = p->Vt_l; g.b_stride = 0;
    g.c64 = Z; g.c_hi = z32; g.c_lo = nullptr; g.c_stride = stride; g.divide = 0;
    item_tabs(-1, -1, -1, TB_VTH, TB_VTL, -1);
    if (run(3, z32 ? O_F32_RAW : O_F64_RAW)) return fail(MOFEM_E_HIP, "gemm launch");
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MOFEM_E_HIP, std::string("prec_apply launch: ") + hipGetErrorString(e));
  return MOFEM_OK;
}

int ensure_internal_ws(void** ws, size_t* have, size_t need, hipStream_t s) {
  if (*have >= need) return MOFEM_OK;
  if (*ws) {
    HIP_TRY(hipStreamSynchronize(s));
    (void)hipFree(*ws);
    *ws = nullptr;
    *have = 0;
  }
  char* p = nullptr;
  int rc = dev_alloc(&p, need);
  if (rc) return rc;
  *ws = p;
  *have = need;
  return MOFEM_OK;
}
}  // namespace

extern "C" int mofem_prec_apply(mofem_prec_t p, const double* R, double* Z, long long stride, int batch,
                                const double* item_scale, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  if (!p) return fail(MOFEM_E_ARG, "prec_apply: NULL handle");
  if (batch < 0) return fail(MOFEM_E_ARG, "prec_apply: negative batch");
  if (batch == 0) return MOFEM_OK;
  if (!R || !Z) return fail(MOFEM_E_ARG, "prec_apply: NULL argument");
  if (stride < (long long)p->qs * p->qt) return fail(MOFEM_E_ARG, "prec_apply: stride smaller than one item");
  hipStream_t s = (hipStream_t)stream;
  size_t need = mofem_prec_workspace_size(p, batch);
  if (!workspace) {
    int rc = ensure_internal_ws(&p->ws, &p->ws_bytes, need, s);
    if (rc) return rc;
    workspace = p->ws;
    ws_bytes = p->ws_bytes;
  } else if (ws_bytes < need) {
    return fail(MOFEM_E_ARG, "prec_apply: workspace too small");
  }
  return prec_launch(p, R, Z, stride, batch, item_scale, workspace, ws_bytes, nullptr, s);
}

extern "C" int mofem_prec_set_tile(mofem_prec_t p, int batch, int tile) {
  clear_error();
  if (!p || batch < 1 || (tile != 64 && tile != 128)) return fail(MOFEM_E_ARG, "prec_set_tile: bad argument");
  if (p->banded) return fail(MOFEM_E_UNSUPPORTED, "prec_set_tile: banded product preconditioner");
  const long long key = ((long long)p->precision << 32) | (unsigned)batch;
  auto it = std::find_if(p->tuned.begin(), p->tuned.end(), [&](auto& kv) { return kv.first == key; });
  if (it == p->tuned.end()) p->tuned.push_back({key, tile});
  else it->second = tile;
  return MOFEM_OK;
}

// Autotuner: time one preconditioner application per block tile on the
// handle's shapes and this batch (zero input; the cost does not depend on
// the values) and keep the faster for (precision, batch).
extern "C" int mofem_prec_tune(mofem_prec_t p, int batch, int* tile_out, void* stream) {
  clear_error();
  if (!p || batch < 1) return fail(MOFEM_E_ARG, "prec_tune: bad argument");
  if (p->banded) return fail(MOFEM_E_UNSUPPORTED, "prec_tune: banded product preconditioner");
  hipStream_t s = (hipStream_t)stream;
  const long long n = (long long)p->qs * p->qt;
  double *R = nullptr, *Z = nullptr;
  char* ws = nullptr;
  const size_t wsb = mofem_prec_workspace_size(p, batch);
  int rc = dev_alloc(&R, (size_t)n * batch);
  if (!rc) rc = dev_alloc(&Z, (size_t)n * batch);
  if (!rc) rc = dev_alloc(&ws, wsb);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float best = 1e30f;
  int best_tile = 128;
  const long long key = ((long long)p->precision << 32) | (unsigned)batch;
  if (!rc && launch_fill(R, 0.0, n, n, batch, s)) rc = fail(MOFEM_E_HIP, "prec_tune: launch failed");
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = fail(MOFEM_E_HIP, "prec_tune: events");
  for (int tile : {128, 64}) {
    if (rc) break;
    auto it = std::find_if(p->tuned.begin(), p->tuned.end(), [&](auto& kv) { return kv.first == key; });
    if (it == p->tuned.end()) p->tuned.push_back({key, tile});
    else it->second = tile;
    rc = prec_launch(p, R, Z, n, batch, nullptr, ws, wsb, nullptr, s);  // warm-up
    if (rc) break;
    if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(MOFEM_E_HIP, "prec_tune: event"); break; }
    for (int r = 0; r < 3 && !rc; ++r) rc = prec_launch(p, R, Z, n, batch, nullptr, ws, wsb, nullptr, s);
    float ms = 0.f;
    if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = fail(MOFEM_E_HIP, "prec_tune: timing");
    if (!rc && ms < best) {
      best = ms;
      best_tile = tile;
    }
  }
  if (!rc) {
    auto it = std::find_if(p->tuned.begin(), p->tuned.end(), [&](auto& kv) { return kv.first == key; });
    it->second = best_tile;
    if (tile_out) *tile_out = best_tile;
  }
  (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (R) (void)hipFree(R);
  if (Z) (void)hipFree(Z);
  if (ws) (void)hipFree(ws);
  return rc;
}

// ============================================================================
// MO-PCG
// ============================================================================
namespace {
struct PcgWs {
  double *R, *Z, *Q, *Y;
  double *part_a, *part_b, *part_op;
  double *rz, *rz_new, *qy, *rr, *zy, *alpha, *beta, *rhs2, *tr, *target2;
  int *active, *claim, *restart, *status, *iters, *live;  // device-side control, see k_vec.hip
  void* prec_ws;
  size_t prec_bytes;
};

// np: operator partial sums per item (0: op's tile count)
size_t pcg_bytes(mofem_op_t op, mofem_prec_t prec, int batch, size_t* prec_part, int np = 0) {
  size_t n = (size_t)op->qs * op->qt;
  size_t b = 0;
  b += 4 * align_up(n * batch * 8, 256);
  b += 2 * align_up((size_t)batch * kVecBlocks * 8, 256);
  b += align_up((size_t)batch * (np > 0 ? np : op->n_tiles_max) * 8, 256);
  b += 11 * align_up((size_t)batch * 8, 256);
  b += 6 * align_up((size_t)batch * 4, 256);
  size_t pp = mofem_prec_workspace_size(prec, batch);
  if (prec_part) *prec_part = pp;
  return b + pp + 4096;
}

bool carve_pcg(mofem_op_t op, mofem_prec_t prec, int batch, void* ws, size_t bytes, PcgWs* w, int np = 0) {
  Carve c(ws, bytes);
  size_t n = (size_t)op->qs * op->qt;
  w->R = c.take<double>(n * batch);
  w->Z = c.take<double>(n * batch);
  w->Q = c.take<double>(n * batch);
  w->Y = c.take<double>(n * batch);
  w->part_a = c.take<double>((size_t)batch * kVecBlocks);
  w->part_b = c.take<double>((size_t)batch * kVecBlocks);
  w->part_op = c.take<double>((size_t)batch * (np > 0 ? np : op->n_tiles_max));
  double** scal[] = {&w->rz, &w->rz_new, &w->qy, &w->rr, &w->zy, &w->alpha, &w->beta, &w->rhs2, &w->tr,
                     &w->target2};
  for (double** x : scal) *x = c.take<double>(batch);
  (void)c.take<double>(batch);  // spare
  int** flags[] = {&w->active, &w->claim, &w->restart, &w->status, &w->iters, &w->live};
  for (int** x : flags) *x = c.take<int>(batch);
  w->prec_bytes = mofem_prec_workspace_size(prec, batch);
  w->prec_ws = c.take<char>(w->prec_bytes);
  return w->prec_ws != nullptr;
}

// Pinned host buffer for the few bytes the solve reads back; kept per thread.
struct PinnedHost {
  void* p = nullptr;
  size_t bytes = 0;
  ~PinnedHost() {
    if (p) (void)hipHostFree(p);
  }
  void* get(size_t need) {
    if (need <= bytes) return p;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    if (hipHostMalloc(&p, need) != hipSuccess) return nullptr;
    bytes = need;
    return p;
  }
};
}  // namespace

extern "C" size_t mofem_pcg_workspace_size(mofem_op_t op, mofem_prec_t prec, int batch) {
  if (!op || !prec || batch < 1) return 0;
  return pcg_bytes(op, prec, batch, nullptr);
}

namespace {
// One MO-PCG solve under device-side control: every kernel skips the items
// whose `active` flag is clear, and convergence, breakdown and the
// true-residual confirmation (with a restart on drift) are decided on the
// device (pcg_init / pcg_check / pcg_confirm), so the launches of an
// iteration never depend on the host.
struct PcgRun {
  mofem_op_t op;
  mofem_prec_t prec;
  const double* Rhs;
  double* U;
  long long stride, n;
  int batch;
  const double* item_scale;
  double tol;
  unsigned flags;
  hipStream_t s;
  PcgWs w{};
  PrecInput pin;
  float* z32 = nullptr;  // FP32 Z (in w.Z's memory) for FP32 / BF16 preconditioners
  int n_trace;  // item count recorded with traced launches
  double rec_band = 0, rec_prec = 0;
  // grouped solve: items [b0, b1) use operator `op` (their own bases come
  // through tabs); np operator partial sums per item
  struct OpRange {
    mofem_op_t op;
    int b0, b1;
  };
  std::vector<OpRange> ranges;
  int np = 0;
  const void* const* tabs = nullptr;

  int n_partial() const { return np > 0 ? np : op_tiles(op, batch); }
  // Y = L(X) over every item (one launch per operator of a grouped solve)
  int run_op(const double* X, long long xs, double* Y, long long ys, double* partial, const int* act, int ntr) {
    if (ranges.empty()) return op_launch(op, X, xs, Y, ys, batch, item_scale, partial, act, s, ntr);
    for (size_t k = 0; k < ranges.size(); ++k) {
      const OpRange& R = ranges[k];
      int rc = op_launch(R.op, X + (size_t)R.b0 * xs, xs, Y + (size_t)R.b0 * ys, ys, R.b1 - R.b0,
                         item_scale ? item_scale + R.b0 : nullptr, partial ? partial + (size_t)R.b0 * np : nullptr,
                         act ? act + R.b0 : nullptr, s, k == 0 ? ntr : 0, np);
      if (rc != MOFEM_OK) return rc;
    }
    return MOFEM_OK;
  }

  int launch_fail() { return fail(MOFEM_E_HIP, "pcg_solve: launch failed"); }
#define PCG_LTRY(x)                                       \
  do {                                                    \
    TraceScope _trace(MOFEM_TRACE_VEC, n_trace, s);       \
    if ((x) != 0) return launch_fail();                   \
  } while (0)
#define PCG_TRY(x)                   \
  do {                               \
    int _rc = (x);                   \
    if (_rc != MOFEM_OK) return _rc; \
  } while (0)

  // ||Rhs||^2, R = Rhs - L(U) (or Rhs with a zero guess), targets, Z = P^-1(R), Q = Z
  int begin() {
    PCG_LTRY(launch_dot_partial(Rhs, Rhs, n, stride, batch, w.part_a, nullptr, s));
    PCG_LTRY(launch_reduce(w.part_a, vec_blocks(n), w.rhs2, batch, s));
    if (flags & MOFEM_PCG_ZERO_GUESS) {
      PCG_LTRY(launch_fill(U, 0.0, n, stride, batch, s));
      PCG_LTRY(launch_copy(Rhs, w.R, n, stride, n, batch, s));
      PCG_LTRY(launch_dot_partial(w.R, w.R, n, n, batch, w.part_a, nullptr, s));
    } else {
      PCG_TRY(run_op(U, stride, w.Y, n, nullptr, nullptr, n_trace));
      PCG_LTRY(launch_residual(Rhs, w.Y, w.R, n, n, stride, batch, w.part_a, nullptr, s));
    }
    PCG_LTRY(launch_reduce(w.part_a, vec_blocks(n), w.rr, batch, s));
    PCG_LTRY(launch_pcg_init(w.rhs2, w.rr, w.target2, w.active, w.claim, w.restart, w.status, w.iters, tol * tol,
                             (flags & MOFEM_PCG_TAU_STOP) ? 1 : 0, batch, s));
    PCG_TRY(prec_launch(prec, w.R, w.Z, n, batch, item_scale, w.prec_ws, w.prec_bytes, w.active, s, n_trace, 0,
                        z32, tabs));
    rec_prec += n_trace;
    if (z32) {
      PCG_LTRY(launch_dot_partial(w.R, z32, n, n, batch, w.part_a, w.active, s));
    } else {
      PCG_LTRY(launch_dot_partial(w.R, w.Z, n, n, batch, w.part_a, w.active, s));
    }
    PCG_LTRY(launch_reduce(w.part_a, vec_blocks(n), w.rz, batch, s));
    if (z32) {
      PCG_LTRY(launch_direction(w.Q, z32, nullptr, n, n, batch, w.active, s));
    } else {
      PCG_LTRY(launch_direction(w.Q, w.Z, nullptr, n, n, batch, w.active, s));
    }
    return MOFEM_OK;
  }

  int iteration() {
    // Y = L(Q), <Q, Y>
    PCG_TRY(run_op(w.Q, n, w.Y, n, w.part_op, w.active, n_trace));
    rec_band += n_trace;
    PCG_LTRY(launch_reduce(w.part_op, n_partial(), w.qy, batch, s));
    // alpha = <R, Z> / <Q, Y>; R -= alpha Y; ||R||^2; R's padded transform operand.
    // U += alpha Q is deferred to the direction pass of this iteration (which
    // reads Q anyway), for every item whose step is valid (live)
    PCG_LTRY(launch_cg_update_pad(nullptr, w.R, w.Q, w.Y, w.rz, w.qy, w.alpha, op->qs, op->qt, n, stride, batch,
                                  w.part_a, w.active, pin.hi, pin.lo, pin.f64, pin.f32, pin.stride, s));
    PCG_LTRY(launch_check(w.part_a, vec_blocks(n), w.rr, w.qy, w.target2, w.active, w.claim, w.status, w.iters,
                          w.live, batch, s));
    // items that claim convergence: confirm on the true residual of U + alpha Q,
    // Rhs - L(U) - alpha Y (Y = L(Q)); where it fails, continue from the true
    // residual with a fresh direction
    PCG_TRY(run_op(U, stride, w.Z, n, nullptr, w.claim, 0));
    PCG_LTRY(launch_residual_step(Rhs, w.Z, w.Y, w.alpha, w.Z, n, n, stride, batch, w.part_b, w.claim, s));
    PCG_LTRY(launch_confirm(w.part_b, vec_blocks(n), w.tr, w.target2, w.active, w.claim, w.restart, batch, s));
    PCG_LTRY(launch_copy_masked(w.Z, w.R, n, n, n, batch, w.restart, s));
    if (pin.f64 || pin.f32 || pin.hi)
      PCG_LTRY(launch_pad_operand(w.R, n, op->qs, op->qt, pin.f64, pin.f32, pin.hi, pin.lo, pin.stride,
                                  (pin.hi != nullptr) ? 1 : 0, batch, w.restart, s));
    // Z = P^{-1}(R); <R, Z>, <Z, Y>; beta (zero after a restart); Q = Z + beta Q
    PCG_TRY(prec_launch(prec, w.R, w.Z, n, batch, item_scale, w.prec_ws, w.prec_bytes, w.active, s, n_trace, 1,
                        z32, tabs));
    rec_prec += n_trace;
    if (z32) {
      PCG_LTRY(launch_zdots_partial(w.R, z32, w.Y, n, n, batch, w.part_a, w.part_b, w.active, s));
    } else {
      PCG_LTRY(launch_zdots_partial(w.R, w.Z, w.Y, n, n, batch, w.part_a, w.part_b, w.active, s));
    }
    PCG_LTRY(launch_beta(w.part_a, w.part_b, vec_blocks(n), w.rz_new, w.zy, w.rz, w.alpha, w.beta, w.restart,
                         (flags & MOFEM_PCG_FLEXIBLE) ? 1 : 0, w.active, batch, s));
    // U += alpha Q (live items), Q = Z + beta Q (items still active)
    if (z32) {
      PCG_LTRY(launch_step_direction(w.Q, z32, w.beta, U, w.alpha, n, n, stride, batch, w.live, w.active, s));
    } else {
      PCG_LTRY(launch_step_direction(w.Q, w.Z, w.beta, U, w.alpha, n, n, stride, batch, w.live, w.active, s));
    }
    return MOFEM_OK;
  }

  // final true residuals of every item and the per-item result on the device
  int finish(int* iters_dev, int* status_dev, double* relres_dev) {
    PCG_TRY(run_op(U, stride, w.Z, n, nullptr, nullptr, batch));
    PCG_LTRY(launch_residual(Rhs, w.Z, w.Z, n, n, stride, batch, w.part_b, nullptr, s));
    PCG_LTRY(launch_reduce(w.part_b, vec_blocks(n), w.tr, batch, s));
    PCG_LTRY(launch_pcg_final(w.tr, w.rhs2, w.target2, w.status, w.iters, iters_dev, status_dev, relres_dev, batch,
                              s));
    return MOFEM_OK;
  }
#undef PCG_LTRY
#undef PCG_TRY
};

int pcg_prepare(PcgRun& r, mofem_op_t op, mofem_prec_t prec, const double* Rhs, double* U, long long stride,
                int batch, const double* item_scale, double tol, int maxit, unsigned flags, void* workspace,
                size_t ws_bytes, hipStream_t s) {
  if (!op || !prec) return fail(MOFEM_E_ARG, "pcg_solve: NULL handle");
  if (batch < 0 || maxit < 0 || !(tol >= 0.0)) return fail(MOFEM_E_ARG, "pcg_solve: bad batch/maxit/tol");
  if (batch > 0 && (!Rhs || !U)) return fail(MOFEM_E_ARG, "pcg_solve: NULL argument");
  if (op->full_input || op->full_output)
    return fail(MOFEM_E_ARG, "pcg_solve: operator must map unknowns to unknowns");
  if (op->qs != prec->qs || op->qt != prec->qt)
    return fail(MOFEM_E_ARG, "pcg_solve: operator and preconditioner sizes differ");
  const long long n = (long long)op->qs * op->qt;
  if (stride < n) return fail(MOFEM_E_ARG, "pcg_solve: stride smaller than one item");
  if (batch == 0) return MOFEM_OK;
  if (!workspace || ws_bytes < pcg_bytes(op, prec, batch, nullptr))
    return fail(MOFEM_E_ARG, "pcg_solve: workspace too small");
  r.op = op;
  r.prec = prec;
  r.Rhs = Rhs;
  r.U = U;
  r.stride = stride;
  r.n = n;
  r.batch = batch;
  r.item_scale = item_scale;
  r.tol = tol;
  r.flags = flags;
  r.s = s;
  r.n_trace = batch;
  if (!carve_pcg(op, prec, batch, workspace, ws_bytes, &r.w)) return fail(MOFEM_E_ARG, "pcg_solve: workspace too small");
  r.pin = prec_input(prec, r.w.prec_ws, r.w.prec_bytes, batch);
  // the preconditioned residual of a low-precision preconditioner is kept in
  // FP32 (its own error is far larger); the recurrence stays FP64
  r.z32 = (!prec->banded && prec->precision != MOFEM_PREC_F64 && prec->precision != MOFEM_PREC_F64_INT8)
              ? reinterpret_cast<float*>(r.w.Z)
              : nullptr;
  return MOFEM_OK;
}

int trace_class_of(mofem_prec_t p) {
  if (p->banded) return MOFEM_TRACE_BCHOL;
  return p->precision == MOFEM_PREC_F64        ? MOFEM_TRACE_GEMM_F64
         : p->precision == MOFEM_PREC_F32      ? MOFEM_TRACE_GEMM_F32
         : p->precision == MOFEM_PREC_BF16     ? MOFEM_TRACE_GEMM_BF16
         : p->precision == MOFEM_PREC_BF16X2   ? MOFEM_TRACE_GEMM_BF16X2
         : p->precision == MOFEM_PREC_F64_INT8 ? MOFEM_TRACE_GEMM_I8
                                               : MOFEM_TRACE_GEMM_BF16X3;
}

int status_error(int result) {
  if (result == MOFEM_E_MAXIT) return fail(result, "pcg_solve: tolerance not reached within maxit");
  if (result == MOFEM_E_BREAKDOWN) return fail(result, "pcg_solve: breakdown, <Q, L(Q)> <= 0");
  if (result == MOFEM_E_NOTFINITE) return fail(result, "pcg_solve: non-finite residual");
  return result;
}
}  // namespace

// The host reads the active flags one iteration behind (the next iteration
// is already queued), so the device never waits on the host inside the
// loop; at most one masked iteration runs after the last item converged.
extern "C" int mofem_pcg_solve(mofem_op_t op, mofem_prec_t prec, const double* Rhs, double* U, long long stride,
                               int batch, const double* item_scale, double tol, int maxit, unsigned flags,
                               void* workspace, size_t ws_bytes, int* iters_out, double* relres_out,
                               void* stream) {
  clear_error();
  hipStream_t s = (hipStream_t)stream;
  if (op && prec && batch > 0 && !workspace) {
    static thread_local void* own_ws = nullptr;
    static thread_local size_t own_bytes = 0;
    int rc = ensure_internal_ws(&own_ws, &own_bytes, pcg_bytes(op, prec, batch, nullptr), s);
    if (rc) return rc;
    workspace = own_ws;
    ws_bytes = own_bytes;
  }
  PcgRun r;
  int rc = pcg_prepare(r, op, prec, Rhs, U, stride, batch, item_scale, tol, maxit, flags, workspace, ws_bytes, s);
  if (rc != MOFEM_OK || batch == 0) return rc;
  static thread_local PinnedHost pinned;
  // layout: two slots of active flags, the initial flags, then (aligned) relres, iters, status
  const size_t dbl_off = align_up((size_t)batch * 12, 64);
  char* host = (char*)pinned.get(dbl_off + (size_t)batch * 16);
  if (!host) return fail(MOFEM_E_NOMEM, "pcg_solve: pinned host buffer");
  int* h_flags[2] = {(int*)host, (int*)host + batch};
  int* h_init = (int*)host + 2 * batch;
  double* h_relres = (double*)(host + dbl_off);
  int* h_iters = (int*)(h_relres + batch);
  int* h_status = h_iters + batch;

  rc = r.begin();
  if (rc) return rc;
  // The active set is known on the host one iteration late; launches are traced
  // with the last known count and corrected at the end from the exact counts.
  HIP_TRY(hipMemcpyAsync(h_init, r.w.active, sizeof(int) * batch, hipMemcpyDeviceToHost, s));
  static thread_local hipEvent_t flag_ev[2] = {nullptr, nullptr};
  for (auto& e : flag_ev)
    if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  std::vector<int> cnt;  // active items after iteration j
  int last_it = -1;
  for (int it = 0; it < maxit; ++it) {
    last_it = it;
    rc = r.iteration();
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(h_flags[it & 1], r.w.active, sizeof(int) * batch, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(flag_ev[it & 1], s));
    if (it == 0) continue;
    HIP_TRY(hipEventSynchronize(flag_ev[(it - 1) & 1]));
    int na = 0;
    for (int b = 0; b < batch; ++b) na += h_flags[(it - 1) & 1][b] != 0;
    cnt.push_back(na);
    r.n_trace = na;
    if (na == 0) break;
  }
  // per-item results (iterations, status, relative residual) into scratch arrays
  // of this solve that the iteration no longer needs, then to the host
  rc = r.finish(r.w.claim, r.w.restart, r.w.rr);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(h_relres, r.w.rr, sizeof(double) * batch, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(h_iters, r.w.claim, sizeof(int) * batch, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(h_status, r.w.restart, sizeof(int) * batch, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (last_it >= 0) {
    // exact items: Y = L(Q) of iteration j ran on the items active after j - 1 (the
    // initial set for j = 0), P^-1 of iteration j on those active after j
    int n_last = 0, n_init = 0;
    for (int b = 0; b < batch; ++b) {
      n_last += h_flags[last_it & 1][b] != 0;
      n_init += h_init[b] != 0;
    }
    while ((int)cnt.size() < last_it + 1) cnt.push_back(n_last);
    double ex_band = 0, ex_prec = n_init;
    for (int j = 0; j <= last_it; ++j) {
      ex_band += j == 0 ? n_init : cnt[j - 1];
      ex_prec += cnt[j];
    }
    trace_add_items(MOFEM_TRACE_BAND, ex_band - r.rec_band);
    if (prec->precision == MOFEM_PREC_BF16_FWD || prec->precision == MOFEM_PREC_BF16_FWD_VS) {
      const bool vs = prec->precision == MOFEM_PREC_BF16_FWD_VS;
      trace_add_items(MOFEM_TRACE_GEMM_BF16, 2.0 * (ex_prec - r.rec_prec));
      trace_add_items(MOFEM_TRACE_GEMM_BF16X3, (vs ? 1.0 : 2.0) * (ex_prec - r.rec_prec));
      if (vs) trace_add_items(MOFEM_TRACE_GEMM_BF16X2, ex_prec - r.rec_prec);
    } else {
      trace_add_items(trace_class_of(prec), (prec->banded ? 2.0 : 4.0) * (ex_prec - r.rec_prec));
    }
  }
  int result = MOFEM_OK;
  for (int b = 0; b < batch; ++b) {
    if (relres_out) relres_out[b] = h_relres[b];
    if (iters_out) iters_out[b] = h_iters[b];
    if (h_status[b] != MOFEM_OK && result == MOFEM_OK) result = h_status[b];
  }
  return status_error(result);
}

namespace {
// Per-run results on the host after advance_runs.
struct RunOut {
  std::vector<int> it, st;
  std::vector<double> rr;
};

// Advance prepared and begun runs together: each run's iteration is queued on
// its stream in turn, so the runs overlap on the device, and each run's
// active flags are read one iteration behind, as in mofem_pcg_solve.  Then
// the final true residuals and per-item results of every run.
int advance_runs(const std::vector<PcgRun*>& runs, const std::vector<int>& maxit, std::vector<RunOut>& out) {
  const size_t nr = runs.size();
  out.assign(nr, RunOut());
  std::vector<int> live(nr, 0);
  std::vector<hipEvent_t> ev(2 * nr, nullptr);
  std::vector<int*> hflag(nr, nullptr);   // two slots (alternate iterations) per run
  std::vector<char*> hres(nr, nullptr);   // iters, status, relres
  int rc = MOFEM_OK;
  for (size_t i = 0; i < nr && !rc; ++i) {
    const int B = runs[i]->batch;
    if (B == 0) continue;
    if (hipHostMalloc((void**)&hflag[i], sizeof(int) * 2 * (size_t)B) != hipSuccess ||
        hipHostMalloc((void**)&hres[i], (sizeof(int) * 2 + sizeof(double)) * (size_t)B) != hipSuccess ||
        hipEventCreateWithFlags(&ev[2 * i], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev[2 * i + 1], hipEventDisableTiming) != hipSuccess)
      rc = fail(MOFEM_E_NOMEM, "pcg_solve_many: host buffers");
    live[i] = maxit[i] > 0 ? 1 : 0;
  }
  for (int it = 0; !rc; ++it) {
    int any = 0;
    for (size_t i = 0; i < nr && !rc; ++i) {
      if (!live[i]) continue;
      PcgRun& r = *runs[i];
      int* slot = hflag[i] + (it & 1) * r.batch;
      rc = r.iteration();
      if (!rc && (hipMemcpyAsync(slot, r.w.active, sizeof(int) * r.batch, hipMemcpyDeviceToHost, r.s) != hipSuccess ||
                  hipEventRecord(ev[2 * i + (it & 1)], r.s) != hipSuccess))
        rc = fail(MOFEM_E_HIP, "pcg_solve_many: flags");
      any = 1;
    }
    if (rc || !any) break;
    for (size_t i = 0; i < nr && !rc; ++i) {
      if (!live[i]) continue;
      if (it + 1 >= maxit[i]) {
        live[i] = 0;
        continue;
      }
      if (it == 0) continue;
      if (hipEventSynchronize(ev[2 * i + ((it - 1) & 1)]) != hipSuccess) {
        rc = fail(MOFEM_E_HIP, "pcg_solve_many: event");
        break;
      }
      const int* slot = hflag[i] + ((it - 1) & 1) * runs[i]->batch;
      int na = 0;
      for (int b = 0; b < runs[i]->batch; ++b) na += slot[b] != 0;
      runs[i]->n_trace = na;
      if (na == 0) live[i] = 0;
    }
  }
  // results: device scratch of each run, then to the host
  for (size_t i = 0; i < nr && !rc; ++i) {
    PcgRun& r = *runs[i];
    if (r.batch == 0) continue;
    int* hit = (int*)hres[i];
    int* hst = hit + r.batch;
    double* hrr = (double*)(hst + r.batch);
    rc = r.finish(r.w.claim, r.w.restart, r.w.rr);
    if (!rc && (hipMemcpyAsync(hit, r.w.claim, sizeof(int) * r.batch, hipMemcpyDeviceToHost, r.s) != hipSuccess ||
                hipMemcpyAsync(hst, r.w.restart, sizeof(int) * r.batch, hipMemcpyDeviceToHost, r.s) != hipSuccess ||
                hipMemcpyAsync(hrr, r.w.rr, sizeof(double) * r.batch, hipMemcpyDeviceToHost, r.s) != hipSuccess))
      rc = fail(MOFEM_E_HIP, "pcg_solve_many: results");
  }
  for (size_t i = 0; i < nr && !rc; ++i) {
    PcgRun& r = *runs[i];
    if (r.batch == 0) continue;
    if (hipStreamSynchronize(r.s) != hipSuccess) {
      rc = fail(MOFEM_E_HIP, "pcg_solve_many: synchronise");
      break;
    }
    const int* hit = (const int*)hres[i];
    const int* hst = hit + r.batch;
    const double* hrr = (const double*)(hst + r.batch);
    out[i].it.assign(hit, hit + r.batch);
    out[i].st.assign(hst, hst + r.batch);
    out[i].rr.assign(hrr, hrr + r.batch);
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  for (int* h : hflag)
    if (h) (void)hipHostFree(h);
  for (char* h : hres)
    if (h) (void)hipHostFree(h);
  return rc;
}
}  // namespace

// Several independent batched solves (uneven shapes, each its own operator,
// preconditioner and stream) advanced together (advance_runs).
extern "C" int mofem_pcg_solve_many(int n_groups, const mofem_pcg_group* groups, void* const* streams,
                                    int* status_out) {
  clear_error();
  if (n_groups < 0 || (n_groups > 0 && (!groups || !streams))) return fail(MOFEM_E_ARG, "pcg_solve_many: bad argument");
  std::vector<PcgRun> runs(n_groups);
  std::vector<PcgRun*> rp;
  std::vector<int> maxit;
  for (int gi = 0; gi < n_groups; ++gi) {
    const mofem_pcg_group& G = groups[gi];
    int rc = pcg_prepare(runs[gi], G.op, G.prec, G.rhs, G.u, G.stride, G.batch, G.item_scale, G.tol, G.maxit,
                         G.flags, G.workspace, G.ws_bytes, (hipStream_t)streams[gi]);
    if (rc) return rc;
    if (G.batch == 0) continue;
    rc = runs[gi].begin();
    if (rc) return rc;
    rp.push_back(&runs[gi]);
    maxit.push_back(G.maxit);
  }
  std::vector<RunOut> out;
  int rc = advance_runs(rp, maxit, out);
  if (rc) return rc;
  int result = MOFEM_OK;
  for (int gi = 0, k = 0; gi < n_groups; ++gi) {
    const mofem_pcg_group& G = groups[gi];
    int gst = MOFEM_OK;
    if (G.batch > 0) {
      const RunOut& o = out[k++];
      for (int b = 0; b < G.batch; ++b) {
        if (G.iters_out) G.iters_out[b] = o.it[b];
        if (G.relres_out) G.relres_out[b] = o.rr[b];
        if (o.st[b] != MOFEM_OK && gst == MOFEM_OK) gst = o.st[b];
      }
    }
    if (status_out) status_out[gi] = gst;
    if (gst != MOFEM_OK && result == MOFEM_OK) result = gst;
  }
  return status_error(result);
}

// Grouped solves: the groups of one shape (and the same precision, preconditioner
// coefficients, tolerance, iteration limit and flags) form one class, solved
// as ONE batched solve whose every stage is one launch over all the class's
// items (the operator: one launch per distinct operator); the items reach
// their own preconditioner bases through per-item pointer tables.  Classes
// advance together on the streams of their first groups (advance_runs).
extern "C" int mofem_pcg_solve_grouped(int n_groups, const mofem_pcg_group* groups, void* const* streams,
                                       int* status_out) {
  clear_error();
  if (n_groups < 0 || (n_groups > 0 && (!groups || !streams))) return fail(MOFEM_E_ARG, "pcg_solve_grouped: bad argument");
  for (int gi = 0; gi < n_groups; ++gi) {
    const mofem_pcg_group& G = groups[gi];
    if (!G.op || !G.prec) return fail(MOFEM_E_ARG, "pcg_solve_grouped: NULL handle");
    if (G.batch < 0 || G.maxit < 0 || !(G.tol >= 0.0)) return fail(MOFEM_E_ARG, "pcg_solve_grouped: bad batch/maxit/tol");
    if (G.batch > 0 && (!G.rhs || !G.u)) return fail(MOFEM_E_ARG, "pcg_solve_grouped: NULL argument");
    if (G.op->full_input || G.op->full_output || G.op->qs != G.prec->qs || G.op->qt != G.prec->qt)
      return fail(MOFEM_E_ARG, "pcg_solve_grouped: operator and preconditioner must map unknowns of one shape");
    if (G.stride < (long long)G.op->qs * G.op->qt) return fail(MOFEM_E_ARG, "pcg_solve_grouped: stride smaller than one item");
    if (G.prec->banded) return fail(MOFEM_E_UNSUPPORTED, "pcg_solve_grouped: banded product preconditioners");
  }
  // classes: groups whose items can share every launch
  auto same_class = [&](const mofem_pcg_group& a, const mofem_pcg_group& b) {
    const mofem_prec_s &p = *a.prec, &q = *b.prec;
    return a.op->qs == b.op->qs && a.op->qt == b.op->qt && p.precision == q.precision && p.alpha == q.alpha &&
           p.bs == q.bs && p.bt == q.bt && p.dl == q.dl && a.tol == b.tol && a.maxit == b.maxit &&
           a.flags == b.flags && (a.item_scale != nullptr) == (b.item_scale != nullptr);
  };
  std::vector<int> cls(n_groups, -1);
  std::vector<std::vector<int>> members;
  for (int gi = 0; gi < n_groups; ++gi) {
    if (groups[gi].batch == 0) continue;
    for (size_t c = 0; c < members.size() && cls[gi] < 0; ++c)
      if (same_class(groups[members[c][0]], groups[gi])) {
        cls[gi] = (int)c;
        members[c].push_back(gi);
      }
    if (cls[gi] < 0) {
      cls[gi] = (int)members.size();
      members.push_back({gi});
    }
  }
  const size_t nc = members.size();
  std::vector<PcgRun> runs(nc);
  std::vector<void*> bufs(nc, nullptr);
  std::vector<std::vector<const void*>> htabs(nc);
  std::vector<PcgRun*> rp;
  std::vector<int> maxit;
  int rc = MOFEM_OK;
  for (size_t c = 0; c < nc && !rc; ++c) {
    const mofem_pcg_group& G0 = groups[members[c][0]];
    hipStream_t s = (hipStream_t)streams[members[c][0]];
    // item ranges of one operator (consecutive groups with the same operator
    // merged); each range's launches take the row-block variant of its size
    std::vector<PcgRun::OpRange> ranges;
    int B = 0, np = 0;
    for (int gi : members[c]) {
      const mofem_pcg_group& G = groups[gi];
      if (!ranges.empty() && ranges.back().op == G.op) ranges.back().b1 += G.batch;
      else ranges.push_back({G.op, B, B + G.batch});
      B += G.batch;
    }
    for (const auto& R : ranges) np = std::max(np, op_tiles(R.op, R.b1 - R.b0));
    const long long n = (long long)G0.op->qs * G0.op->qt;
    // class buffer: right-hand sides, solutions, item scales, pointer tables, PCG workspace
    const size_t ws = pcg_bytes(G0.op, G0.prec, B, nullptr, np);
    const size_t bytes = 2 * align_up((size_t)B * n * 8, 256) + align_up((size_t)B * 8, 256) +
                         align_up((size_t)TB_COUNT * B * sizeof(void*), 256) + ws + 1024;
    char* buf = nullptr;
    rc = dev_alloc(&buf, bytes);
    if (rc) break;
    bufs[c] = buf;
    Carve cv(buf, bytes);
    double* Rhs = cv.take<double>((size_t)B * n);
    double* U = cv.take<double>((size_t)B * n);
    double* isc = cv.take<double>((size_t)B);
    const void** dtab = cv.take<const void*>((size_t)TB_COUNT * B);
    void* pws = cv.take<char>(ws);
    std::vector<const void*>& ht = htabs[c];
    ht.assign((size_t)TB_COUNT * B, nullptr);
    int b0 = 0;
    for (int gi : members[c]) {
      const mofem_pcg_group& G = groups[gi];
      const void* e[TB_COUNT];
      prec_tab_entries(G.prec, e);
      for (int b = 0; b < G.batch; ++b)
        for (int k = 0; k < TB_COUNT; ++k) ht[(size_t)k * B + b0 + b] = e[k];
      if (hipMemcpy2DAsync(Rhs + (size_t)b0 * n, n * 8, G.rhs, G.stride * 8, n * 8, G.batch, hipMemcpyDeviceToDevice,
                           s) != hipSuccess ||
          (!(G.flags & MOFEM_PCG_ZERO_GUESS) &&
           hipMemcpy2DAsync(U + (size_t)b0 * n, n * 8, G.u, G.stride * 8, n * 8, G.batch, hipMemcpyDeviceToDevice,
                            s) != hipSuccess) ||
          (G.item_scale && hipMemcpyAsync(isc + b0, G.item_scale, G.batch * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)) {
        rc = fail(MOFEM_E_HIP, "pcg_solve_grouped: gather");
        break;
      }
      b0 += G.batch;
    }
    if (rc) break;
    if (hipMemcpyAsync(dtab, ht.data(), ht.size() * sizeof(void*), hipMemcpyHostToDevice, s) != hipSuccess) {
      rc = fail(MOFEM_E_HIP, "pcg_solve_grouped: tables");
      break;
    }
    PcgRun& r = runs[c];
    rc = pcg_prepare(r, G0.op, G0.prec, Rhs, U, n, B, G0.item_scale ? isc : nullptr, G0.tol, G0.maxit, G0.flags,
                     pws, ws, s);
    if (rc) break;
    // pcg_prepare carved with the first operator's tile count: carve again with np
    if (!carve_pcg(G0.op, G0.prec, B, pws, ws, &r.w, np)) {
      rc = fail(MOFEM_E_ARG, "pcg_solve_grouped: workspace");
      break;
    }
    r.pin = prec_input(G0.prec, r.w.prec_ws, r.w.prec_bytes, B);
    if (r.z32) r.z32 = reinterpret_cast<float*>(r.w.Z);
    r.np = np;
    r.tabs = dtab;
    r.ranges = ranges;
    // operators with fewer tiles than np leave their items' last partial sums unwritten
    if (launch_fill(r.w.part_op, 0.0, (long long)B * np, (long long)B * np, 1, s)) {
      rc = fail(MOFEM_E_HIP, "pcg_solve_grouped: launch failed");
      break;
    }
    rc = r.begin();
    if (rc) break;
    rp.push_back(&r);
    maxit.push_back(G0.maxit);
  }
  std::vector<RunOut> out;
  if (!rc) rc = advance_runs(rp, maxit, out);
  // solutions back to the groups, per-item results to the callers
  int result = MOFEM_OK;
  for (size_t c = 0; c < nc && !rc; ++c) {
    PcgRun& r = runs[c];
    int b0 = 0;
    for (int gi : members[c]) {
      const mofem_pcg_group& G = groups[gi];
      if (hipMemcpy2DAsync(G.u, G.stride * 8, r.U + (size_t)b0 * r.n, r.n * 8, r.n * 8, G.batch,
                           hipMemcpyDeviceToDevice, r.s) != hipSuccess) {
        rc = fail(MOFEM_E_HIP, "pcg_solve_grouped: scatter");
        break;
      }
      int gst = MOFEM_OK;
      for (int b = 0; b < G.batch; ++b) {
        if (G.iters_out) G.iters_out[b] = out[c].it[b0 + b];
        if (G.relres_out) G.relres_out[b] = out[c].rr[b0 + b];
        if (out[c].st[b0 + b] != MOFEM_OK && gst == MOFEM_OK) gst = out[c].st[b0 + b];
      }
      if (status_out) status_out[gi] = gst;
      if (gst != MOFEM_OK && result == MOFEM_OK) result = gst;
      b0 += G.batch;
    }
    if (!rc && hipStreamSynchronize(r.s) != hipSuccess) rc = fail(MOFEM_E_HIP, "pcg_solve_grouped: synchronise");
  }
  if (status_out)
    for (int gi = 0; gi < n_groups; ++gi)
      if (groups[gi].batch == 0) status_out[gi] = MOFEM_OK;
  for (size_t c = 0; c < nc; ++c)
    if (bufs[c]) {
      (void)hipStreamSynchronize(runs[c].s ? runs[c].s : (hipStream_t)streams[members[c][0]]);
      (void)hipFree(bufs[c]);
    }
  if (rc) return rc;
  return status_error(result);
}

extern "C" int mofem_pcg_solve_async(mofem_op_t op, mofem_prec_t prec, const double* Rhs, double* U,
                                     long long stride, int batch, const double* item_scale, double tol, int maxit,
                                     unsigned flags, void* workspace, size_t ws_bytes, int* iters_dev,
                                     int* status_dev, double* relres_dev, void* stream) {
  clear_error();
  if (batch > 0 && (!workspace || !iters_dev || !status_dev || !relres_dev))
    return fail(MOFEM_E_ARG, "pcg_solve_async: NULL workspace or result array");
  PcgRun r;
  hipStream_t s = (hipStream_t)stream;
  int rc = pcg_prepare(r, op, prec, Rhs, U, stride, batch, item_scale, tol, maxit, flags, workspace, ws_bytes, s);
  if (rc != MOFEM_OK || batch == 0) return rc;
  rc = r.begin();
  if (rc) return rc;
  for (int it = 0; it < maxit; ++it) {
    rc = r.iteration();
    if (rc) return rc;
  }
  return r.finish(iters_dev, status_dev, relres_dev);
}

// ============================================================================
// IMEX Euler step
// ============================================================================
extern "C" size_t mofem_imex_workspace_size(const mofem_imex_desc* d, int batch) {
  if (!d || !d->op || !d->prec || !d->mass || batch < 1 || d->n_species < 1 || d->n_species > 2) return 0;
  size_t items = (size_t)d->n_species * batch;
  size_t n = (size_t)d->op->qs * d->op->qt;
  size_t b = align_up(items * n * 8, 256);                 // right-hand sides
  if (d->kinetics == MOFEM_KIN_DIB) b += align_up(items * n * 8, 256);  // transformed states
  b += align_up(items * 8, 256);                           // item scales
  return b + pcg_bytes(d->op, d->prec, (int)items, nullptr) + 4096;
}

namespace {
// a banded product preconditioner must hold a factor pair for every c = d tau
int check_imex_scales(const mofem_imex_desc* d, const char* who) {
  if (!d->prec->banded) return MOFEM_OK;
  const std::vector<double>& sc = d->prec->h_scales;
  for (int sp = 0; sp < d->n_species; ++sp)
    if (std::find(sc.begin(), sc.end(), d->d[sp] * d->tau) == sc.end())
      return fail(MOFEM_E_ARG, std::string(who) + ": the banded preconditioner has no factor pair for the scale "
                                   "d * tau of species " + std::to_string(sp));
  return MOFEM_OK;
}

int imex_check(const mofem_imex_desc* d, const double* state, long long stride, int batch) {
  if (!d || !state || !d->op || !d->prec || !d->mass) return fail(MOFEM_E_ARG, "imex_step: NULL argument");
  if (d->n_species < 1 || d->n_species > 2) return fail(MOFEM_E_ARG, "imex_step: n_species must be 1 or 2");
  if (d->kinetics == MOFEM_KIN_DIB && d->n_species != 2) return fail(MOFEM_E_ARG, "imex_step: DIB needs 2 species");
  if (d->kinetics != MOFEM_KIN_NONE && d->kinetics != MOFEM_KIN_DIB)
    return fail(MOFEM_E_ARG, "imex_step: unknown kinetics");
  if (batch < 0) return fail(MOFEM_E_ARG, "imex_step: negative batch");
  mofem_op_t op = d->op, mass = d->mass;
  if (mass->full_input || mass->full_output || mass->qs != op->qs || mass->qt != op->qt)
    return fail(MOFEM_E_ARG, "imex_step: mass operator must map unknowns to unknowns of the same shape");
  if (stride != (long long)op->qs * op->qt)
    return fail(MOFEM_E_ARG, "imex_step: items must be contiguous (stride = q_s * q_t)");
  return check_imex_scales(d, "imex_step");
}

struct ImexParts {
  double *rhs, *trans, *scale;
  void* pcg_ws;
  size_t pcg_need;
};
int imex_carve(const mofem_imex_desc* d, int batch, void* workspace, size_t ws_bytes, ImexParts* p) {
  const int items = d->n_species * batch;
  const size_t n = (size_t)d->op->qs * d->op->qt;
  Carve c(workspace, ws_bytes);
  p->rhs = c.take<double>((size_t)items * n);
  p->trans = d->kinetics == MOFEM_KIN_DIB ? c.take<double>((size_t)items * n) : nullptr;
  p->scale = c.take<double>(items);
  p->pcg_need = pcg_bytes(d->op, d->prec, items, nullptr);
  p->pcg_ws = c.take<char>(p->pcg_need);
  if (!p->rhs || !p->scale || !p->pcg_ws || (d->kinetics == MOFEM_KIN_DIB && !p->trans))
    return fail(MOFEM_E_ARG, "imex_step: workspace too small");
  return MOFEM_OK;
}

// per-item c = d_species * tau and the right-hand side Mass(U + tau f(U, V)) (eq. (93))
int imex_rhs(const mofem_imex_desc* d, const double* state, int batch, const ImexParts& p, hipStream_t s) {
  const long long n = (long long)d->op->qs * d->op->qt;
  const int items = d->n_species * batch;
  for (int sp = 0; sp < d->n_species; ++sp)
    if (launch_fill(p.scale + (size_t)sp * batch, d->d[sp] * d->tau, batch, batch, 1, s) != 0)
      return fail(MOFEM_E_HIP, "imex_step: launch failed");
  const double* src = state;
  if (d->kinetics == MOFEM_KIN_DIB) {
    if (launch_dib_source(state, state + (size_t)batch * n, p.trans, p.trans + (size_t)batch * n, n, n, batch,
                          d->kin, d->tau, s) != 0)
      return fail(MOFEM_E_HIP, "imex_step: kinetics launch failed");
    src = p.trans;
  }
  return op_launch(d->mass, src, n, p.rhs, n, items, nullptr, nullptr, nullptr, s);
}
}  // namespace

extern "C" int mofem_imex_step(const mofem_imex_desc* d, double* state, long long stride, int batch,
                               void* workspace, size_t ws_bytes, int* iters_out, void* stream) {
  clear_error();
  int rc = imex_check(d, state, stride, batch);
  if (rc != MOFEM_OK || batch == 0) return rc;
  hipStream_t s = (hipStream_t)stream;
  const size_t need = mofem_imex_workspace_size(d, batch);
  static thread_local void* own_ws = nullptr;
  static thread_local size_t own_bytes = 0;
  if (!workspace) {
    rc = ensure_internal_ws(&own_ws, &own_bytes, need, s);
    if (rc) return rc;
    workspace = own_ws;
    ws_bytes = own_bytes;
  } else if (ws_bytes < need) {
    return fail(MOFEM_E_ARG, "imex_step: workspace too small");
  }
  ImexParts p;
  rc = imex_carve(d, batch, workspace, ws_bytes, &p);
  if (rc) return rc;
  rc = imex_rhs(d, state, batch, p, s);
  if (rc) return rc;
  const int items = d->n_species * batch;
  std::vector<double> relres(items);
  // the state is both the guess and the solution; all species in one batched solve
  return mofem_pcg_solve(d->op, d->prec, p.rhs, state, stride, items, p.scale, d->tol, d->maxit,
                         d->flags & ~MOFEM_PCG_ZERO_GUESS, p.pcg_ws, p.pcg_need, iters_out, relres.data(), stream);
}

// ---- the IMEX step as a replayable HIP graph ---------------------------------
struct mofem_imex_graph_s {
  hipGraphExec_t exec = nullptr;
  int items = 0;
  int* d_int = nullptr;        // [4][items]: last iters, last status, max iters, first error
  double* d_relres = nullptr;  // [items]: relative residual of the last step
};

namespace {
// accumulate a step's per-item results over replays: max iterations, first error
__global__ void imex_accum_kernel(const int* __restrict__ iters, const int* __restrict__ status,
                                  int* __restrict__ max_iters, int* __restrict__ first_err, int items) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= items) return;
  if (iters[b] > max_iters[b]) max_iters[b] = iters[b];
  if (first_err[b] == 0 && status[b] != 0) first_err[b] = status[b];
}
__global__ void fill_int_kernel(int* __restrict__ x, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
}  // namespace

extern "C" int mofem_imex_graph_create(const mofem_imex_desc* d, double* state, long long stride, int batch,
                                       void* workspace, size_t ws_bytes, int iters_per_step,
                                       mofem_imex_graph_t* out, void* stream) {
  clear_error();
  if (!out) return fail(MOFEM_E_ARG, "imex_graph_create: NULL output");
  *out = nullptr;
  int rc = imex_check(d, state, stride, batch);
  if (rc != MOFEM_OK) return rc;
  if (batch < 1 || iters_per_step < 1) return fail(MOFEM_E_ARG, "imex_graph_create: batch and iters_per_step >= 1");
  if (!workspace || ws_bytes < mofem_imex_workspace_size(d, batch))
    return fail(MOFEM_E_ARG, "imex_graph_create: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(MOFEM_E_ARG, "imex_graph_create: capture needs a created (non-default) stream");
  ImexParts p;
  rc = imex_carve(d, batch, workspace, ws_bytes, &p);
  if (rc) return rc;
  auto* g = new mofem_imex_graph_s();
  g->items = d->n_species * batch;
  if (dev_alloc(&g->d_int, (size_t)4 * g->items) != MOFEM_OK || dev_alloc(&g->d_relres, (size_t)g->items) != MOFEM_OK) {
    mofem_imex_graph_destroy(g);
    return fail(MOFEM_E_NOMEM, "imex_graph_create: result arrays");
  }
  hipLaunchKernelGGL(fill_int_kernel, dim3((4 * g->items + 255) / 256), dim3(256), 0, s, g->d_int, 0, 4 * g->items);
  HIP_TRY(hipStreamSynchronize(s));
  // capture one step: right-hand side, then exactly iters_per_step masked PCG
  // iterations (no host synchronisation anywhere), then the result accumulation
  TraceCapture no_trace;
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int* it_last = g->d_int;
  int* st_last = g->d_int + g->items;
  rc = imex_rhs(d, state, batch, p, s);
  if (rc == MOFEM_OK)
    rc = mofem_pcg_solve_async(d->op, d->prec, p.rhs, state, stride, g->items, p.scale, d->tol, iters_per_step,
                               d->flags & ~MOFEM_PCG_ZERO_GUESS, p.pcg_ws, p.pcg_need, it_last, st_last, g->d_relres,
                               stream);
  if (rc == MOFEM_OK)
    hipLaunchKernelGGL(imex_accum_kernel, dim3((g->items + 63) / 64), dim3(64), 0, s, it_last, st_last,
                       g->d_int + 2 * g->items, g->d_int + 3 * g->items, g->items);
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (rc != MOFEM_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    mofem_imex_graph_destroy(g);
    return rc != MOFEM_OK ? rc : fail(MOFEM_E_HIP, std::string("imex_graph_create: capture: ") + hipGetErrorString(e));
  }
  e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    mofem_imex_graph_destroy(g);
    return fail(MOFEM_E_HIP, std::string("imex_graph_create: instantiate: ") + hipGetErrorString(e));
  }
  *out = g;
  return MOFEM_OK;
}

extern "C" int mofem_imex_graph_launch(mofem_imex_graph_t g, int nsteps, void* stream) {
  clear_error();
  if (!g || nsteps < 0) return fail(MOFEM_E_ARG, "imex_graph_launch: bad argument");
  for (int i = 0; i < nsteps; ++i) HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return MOFEM_OK;
}

extern "C" int mofem_imex_graph_result(mofem_imex_graph_t g, int* max_iters, int* status, double* relres,
                                       void* stream) {
  clear_error();
  if (!g) return fail(MOFEM_E_ARG, "imex_graph_result: NULL handle");
  hipStream_t s = (hipStream_t)stream;
  std::vector<int> h((size_t)4 * g->items);
  std::vector<double> r(g->items);
  HIP_TRY(hipMemcpyAsync(h.data(), g->d_int, h.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(r.data(), g->d_relres, r.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int result = MOFEM_OK;
  for (int b = 0; b < g->items; ++b) {
    if (max_iters) max_iters[b] = h[(size_t)2 * g->items + b];
    const int st = h[(size_t)3 * g->items + b];
    if (status) status[b] = st;
    if (relres) relres[b] = r[b];
    if (st != MOFEM_OK && result == MOFEM_OK) result = st;
  }
  // start a new accumulation
  hipLaunchKernelGGL(fill_int_kernel, dim3((2 * g->items + 255) / 256), dim3(256), 0, s, g->d_int + 2 * g->items, 0,
                     2 * g->items);
  HIP_TRY(hipGetLastError());
  return result;
}

extern "C" int mofem_imex_graph_destroy(mofem_imex_graph_t g) {
  if (!g) return MOFEM_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->d_int) (void)hipFree(g->d_int);
  if (g->d_relres) (void)hipFree(g->d_relres);
  delete g;
  return MOFEM_OK;
}

// ============================================================================
// Batched Frobenius products and the adjoint IMEX step
// ============================================================================
extern "C" int mofem_dot_accumulate(const double* X, const double* Y, long long n, long long stride, int batch,
                                    double alpha, double beta, double* out, void* stream) {
  clear_error();
  if (batch < 0 || n < 0) return fail(MOFEM_E_ARG, "dot_accumulate: negative size");
  if (batch == 0) return MOFEM_OK;
  if (!X || !Y || !out) return fail(MOFEM_E_ARG, "dot_accumulate: NULL argument");
  if (stride < n) return fail(MOFEM_E_ARG, "dot_accumulate: stride smaller than one item");
  hipStream_t s = (hipStream_t)stream;
  static thread_local void* part = nullptr;
  static thread_local size_t have = 0;
  int rc = ensure_internal_ws(&part, &have, (size_t)batch * kVecBlocks * 8, s);
  if (rc) return rc;
  if (launch_dot_partial(X, Y, n, stride, batch, (double*)part, nullptr, s) ||
      launch_reduce_axpy((const double*)part, vec_blocks(n), out, alpha, beta, batch, s))
    return fail(MOFEM_E_HIP, "dot_accumulate: launch failed");
  return MOFEM_OK;
}

extern "C" size_t mofem_imex_adjoint_workspace_size(const mofem_imex_desc* d, int batch) {
  if (!d || !d->op || !d->prec || !d->mass || batch < 1 || d->n_species < 1 || d->n_species > 2) return 0;
  size_t items = (size_t)d->n_species * batch;
  size_t n = (size_t)d->op->qs * d->op->qt;
  size_t b = 2 * align_up(items * n * 8, 256);               // mu, K(U+) then Mass(mu)
  b += align_up(items * 8, 256);                             // item scales
  b += align_up(items * kVecBlocks * 8, 256);                // dot partials
  return b + pcg_bytes(d->op, d->prec, (int)items, nullptr) + 4096;
}

extern "C" int mofem_imex_adjoint_step(const mofem_imex_desc* d, mofem_op_t stiff, const double* state_n,
                                       const double* state_np1, double* lam, double* grad_d, long long stride,
                                       int batch, void* workspace, size_t ws_bytes, int* iters_out,
                                       void* stream) {
  clear_error();
  if (!d || !d->op || !d->prec || !d->mass || !stiff) return fail(MOFEM_E_ARG, "imex_adjoint_step: NULL argument");
  if (d->n_species < 1 || d->n_species > 2) return fail(MOFEM_E_ARG, "imex_adjoint_step: n_species must be 1 or 2");
  if (d->kinetics == MOFEM_KIN_DIB && d->n_species != 2)
    return fail(MOFEM_E_ARG, "imex_adjoint_step: DIB needs 2 species");
  if (d->kinetics != MOFEM_KIN_NONE && d->kinetics != MOFEM_KIN_DIB)
    return fail(MOFEM_E_ARG, "imex_adjoint_step: unknown kinetics");
  if (batch < 1) return batch == 0 ? MOFEM_OK : fail(MOFEM_E_ARG, "imex_adjoint_step: negative batch");
  if (!state_n || !state_np1 || !lam || !grad_d) return fail(MOFEM_E_ARG, "imex_adjoint_step: NULL argument");
  mofem_op_t op = d->op, mass = d->mass;
  for (mofem_op_t o : {mass, stiff})
    if (o->full_input || o->full_output || o->qs != op->qs || o->qt != op->qt)
      return fail(MOFEM_E_ARG, "imex_adjoint_step: mass and stiffness must map unknowns to unknowns of one shape");
  const long long n = (long long)op->qs * op->qt;
  if (stride != n) return fail(MOFEM_E_ARG, "imex_adjoint_step: items must be contiguous (stride = q_s * q_t)");
  if (int rc0 = check_imex_scales(d, "imex_adjoint_step")) return rc0;
  const int items = d->n_species * batch;
  hipStream_t s = (hipStream_t)stream;
  const size_t need = mofem_imex_adjoint_workspace_size(d, batch);
  static thread_local void* own_ws = nullptr;
  static thread_local size_t own_bytes = 0;
  if (!workspace) {
    int rc = ensure_internal_ws(&own_ws, &own_bytes, need, s);
    if (rc) return rc;
    workspace = own_ws;
    ws_bytes = own_bytes;
  } else if (ws_bytes < need) {
    return fail(MOFEM_E_ARG, "imex_adjoint_step: workspace too small");
  }
  Carve c(workspace, ws_bytes);
  double* mu = c.take<double>((size_t)items * n);
  double* tmp = c.take<double>((size_t)items * n);
  double* scale = c.take<double>(items);
  double* part = c.take<double>((size_t)items * kVecBlocks);
  const size_t pcg_need = pcg_bytes(op, d->prec, items, nullptr);
  void* pcg_ws = c.take<char>(pcg_need);
  if (!mu || !tmp || !scale || !part || !pcg_ws) return fail(MOFEM_E_ARG, "imex_adjoint_step: workspace too small");
  for (int sp = 0; sp < d->n_species; ++sp)
    if (launch_fill(scale + (size_t)sp * batch, d->d[sp] * d->tau, batch, batch, 1, s) != 0)
      return fail(MOFEM_E_HIP, "imex_adjoint_step: launch failed");
  // mu = L_c^{-1}(lam): the operator is symmetric, so the adjoint solve is a forward solve
  int rc = mofem_pcg_solve(op, d->prec, lam, mu, n, items, scale, d->tol, d->maxit,
                           (d->flags & ~MOFEM_PCG_TAU_STOP) | MOFEM_PCG_ZERO_GUESS, pcg_ws, pcg_need, iters_out,
                           nullptr, stream);
  if (rc != MOFEM_OK) return rc;
  // grad_d += -tau <mu, K(U^{n+1})>
  rc = op_launch(stiff, state_np1, n, tmp, n, items, nullptr, nullptr, nullptr, s);
  if (rc) return rc;
  {
    TraceScope trace(MOFEM_TRACE_VEC, items, s);
    if (launch_dot_partial(mu, tmp, n, n, items, part, nullptr, s) ||
        launch_reduce_axpy(part, vec_blocks(n), grad_d, -d->tau, 1.0, items, s))
      return fail(MOFEM_E_HIP, "imex_adjoint_step: launch failed");
  }
  // nu = Mass(mu), then the transpose of the explicit kinetics
  rc = op_launch(mass, mu, n, tmp, n, items, nullptr, nullptr, nullptr, s);
  if (rc) return rc;
  TraceScope trace(MOFEM_TRACE_VEC, items, s);
  int lrc;
  if (d->kinetics == MOFEM_KIN_DIB)
    lrc = launch_dib_adjoint(state_n, state_n + (size_t)batch * n, tmp, tmp + (size_t)batch * n, lam,
                             lam + (size_t)batch * n, n, n, batch, d->kin, d->tau, s);
  else
    lrc = launch_copy(tmp, lam, n, n, n, items, s);
  if (lrc) return fail(MOFEM_E_HIP, "imex_adjoint_step: launch failed");
  return MOFEM_OK;
}

// C ABI of the LRAMM hot path: argument validation, workspace layout and the
// stream-ordered stage sequence of the forward and backward passes.  No
// device memory is allocated here; every buffer is a slice of the caller's
// workspace and no host synchronisation happens inside forward / backward.
//
// Forward (paper Sec. 2.2 range finder + Alg. 1 projection + Sec. 3.2 chain
// of Alg. 2 products, one-sided form):
//   A_r  = quant_rows(A)  [fmt_sketch]      A_c = quant_cols(A) [fmt_proj]
//   B_c  = quant_cols(B)  [fmt_g1]          Om  = quant_cols(Omega) [fmt_sketch]
//   Y    = A_r . Om^T                       Q   = cholqr2(Y)
//   repeat q times:  Z = A_c . quant_cols(Q)^T ; Q_Z = cholqr2(Z)
//                    Y = A_r . quant_cols(Q_Z)^T ; Q = cholqr2(Y)
//   Bt   = quant_cols(Q)[fmt_proj] . A_c^T          (Q^T A, l x k)
//   T^T  = B_c . quant_rows(Bt)[fmt_g1]^T           (n x l)
//   C    = alpha quant_rows(Q)[fmt_g2] . quant_rows(T^T)[fmt_g2]^T + beta C
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <new>
#include <vector>

#include "common.hpp"

struct lramm_plan {
  lramm_desc user;   // as the caller described it
  // the problem the library runs: the caller's A, B, C (side 0) or B^T, A^T,
  // C^T (side 1), with m, n, k and the element types mapped accordingly
  lramm_desc d;
  int at = 0, bt = 0, ct = 0;   // A', B', C' stored transposed
  int chain_mode = lramm::CHAIN_SHARED;   // CHAIN_OFF while a batch issues the plan on one of several streams
  int64_t l, lp;            // sketch width and its 32-padded leading dimension
  // workspace offsets (bytes)
  size_t off_flags;
  size_t off_Ar, off_sAr, off_Ac, off_sAc, off_Bc, off_sBc;
  size_t off_OmT, off_Om, off_sOm;
  size_t off_Y, off_Q, off_Z, off_QZ, off_QZc, off_sQZc;
  size_t off_Qc, off_sQc, off_Qr, off_sQr;
  size_t off_Bt, off_Btq, off_sBt, off_Tt, off_Ttq, off_sTt;
  size_t off_chol, chol_bytes, off_split, split_bytes;
  size_t off_W, off_Bte, off_V;
  bool srht = false;        // structured first sketch (LRAMM_PLAN_SRHT)
  size_t off_srS = 0, off_srD = 0, off_srK = 0;
  bool estimate = false;    // a-posteriori error estimate (LRAMM_PLAN_ESTIMATE)
  int passes = 2;           // Cholesky QR passes per orthonormalisation (1: LRAMM_PLAN_ONE_PASS)
  size_t off_norms = 0;     // ||A'||^2, ||Bt||^2, then the two partial arrays
  // zero-filled at the start of every forward: the status word, then the
  // column-maxima buffers of every column quantisation of the pass
  size_t off_zero, zero_words;
  size_t mx_A, mx_B, mx_Om, mx_Q, mx_QZ, mx_Ar;   // word offsets inside the zero region
  size_t total;
  int64_t pAr, pAc, pBc, pOm, pQZc, pQc, pQr, pBtq, pTtq;
  // A's row codes of the last forward: the workspace copy, or A itself when
  // the bf16 input fed the bf16 sketch directly
  const void* last_Ar = nullptr;
  int64_t last_pAr = 0;
  // whether the last forward's projection / G1 read A / B in place (bf16,
  // K-major) instead of their column codes
  bool last_km_a = false, last_km_b = false;
  // side stream for the work independent of the orthonormalisation chain
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_omega = nullptr, ev_sketch = nullptr;
  // stage timing (measurement only)
  bool timing = false;
  std::vector<hipEvent_t> events;     // pool, reused
  std::vector<int> rec_stage;         // stage of each recorded pair
  std::vector<int> rec_weight;        // kernel launches inside each recorded pair
  size_t next_event = 0;
  double stage_ms[LRAMM_NSTAGES] = {0};
  int64_t stage_n[LRAMM_NSTAGES] = {0};
};

using namespace lramm;

// Scratch of the no-allocation CholeskyQR2 (see lramm_cholqr2_noalloc).
static __device__ __align__(256) uint8_t scratch[LRAMM_NOALLOC_SCRATCH_BYTES];

namespace {

// Events that only order streams of this device: no timing, and a
// device-scope release instead of the default system-scope fence (nothing
// on the host reads what they guard).
constexpr unsigned kOrderEvent = hipEventDisableTiming | hipEventReleaseToDevice;

// Fixed device scratch of lramm_cholqr2_noalloc (callers that cannot
// allocate).  Each GPU holds its own copy of this array for the life of the
// process; host code reaches it only through the address
// hipGetSymbolAddress returns with that GPU current (the array's name in
// host code is a host-side stand-in, not a device address).
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of this GPU's scratch array: looked up once per device
// (with that device current) and kept.
lramm_status scratch_address(void** out) {
  int dev = 0;
  LRAMM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return LRAMM_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LRAMM_E_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LRAMM_OK;
}

bool valid_fmt(int f) { return f == LRAMM_INT8 || f == LRAMM_INT4 || f == LRAMM_FP8 || f == LRAMM_BF16F; }
bool valid_io(int t) { return t == LRAMM_F32 || t == LRAMM_BF16; }

size_t carve(size_t* cur, size_t bytes) {
  size_t o = (size_t)round_up((int64_t)*cur, 256);
  *cur = o + bytes;
  return o;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<uint8_t*>(ws) + off);
}

enum Stage {
  ST_QUANT_A_ROWS, ST_QUANT_A_COLS, ST_QUANT_B, ST_OMEGA, ST_QUANT_OMEGA, ST_SKETCH, ST_CHOLQR2, ST_QUANT_Q_COLS,
  ST_POWER_Z, ST_QUANT_QZ, ST_POWER_Y, ST_PROJ, ST_QUANT_BT, ST_G1, ST_QUANT_Q_ROWS, ST_QUANT_TT, ST_G2
};
const char* kStageNames[LRAMM_NSTAGES] = {
    "quant_A_rows", "quant_A_cols", "quant_B_cols", "omega", "quant_omega", "sketch_gemm", "cholqr2",
    "quant_Q_cols", "power_gemm_Z", "quant_QZ_cols", "power_gemm_Y", "proj_gemm", "quant_Bt_rows", "g1_gemm",
    "quant_Q_rows", "quant_Tt_rows", "g2_gemm", "cholqr2.gram", "cholqr2.chol_panel", "cholqr2.solve",
    "cholqr2.series", "cholqr2.apply"};

// Event pair around one stage when the plan measures (no-op otherwise).
struct StageTimer {
  lramm_plan* p;
  hipStream_t s;
  int stage;
  hipEvent_t stop = nullptr;
  StageTimer(lramm_plan* p_, hipStream_t s_, int st, int weight = 1) : p(p_), s(s_), stage(st) {
    if (!p->timing) return;
    while (p->events.size() < p->next_event + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        p->timing = false;
        return;
      }
      p->events.push_back(e);
    }
    hipEvent_t start = p->events[p->next_event];
    stop = p->events[p->next_event + 1];
    p->next_event += 2;
    p->rec_stage.push_back(stage);
    p->rec_weight.push_back(weight);
    (void)hipEventRecord(start, s);
  }
  ~StageTimer() {
    if (stop) (void)hipEventRecord(stop, s);
  }
};

// Nested timers for launches inside a stage (TimingHook callbacks).
struct HookCtx {
  lramm_plan* p;
  hipStream_t s;
  std::vector<StageTimer*> open;
};
void hook_begin(void* c, int stage) {
  HookCtx* h = static_cast<HookCtx*>(c);
  const int launches = stage >> 16;
  h->open.push_back(new StageTimer(h->p, h->s, stage & 0xffff, launches > 0 ? launches : 1));
}
void hook_end(void* c) {
  HookCtx* h = static_cast<HookCtx*>(c);
  delete h->open.back();
  h->open.pop_back();
}

// Longest K whose products cannot leave the accumulator's range: int32 for
// the integer formats (K * qmax^2 < 2^31); fp8 and bf16 accumulate in FP32,
// where K * 448^2 stays far below FLT_MAX for any supported K.
int64_t qk_bound(int fmt) {
  if (fmt == LRAMM_INT4) return (int64_t)(2147483647LL / 49);
  if (fmt == LRAMM_INT8) return (int64_t)(2147483647LL / 16129);
  return (int64_t)INT32_MAX;
}

}  // namespace

extern "C" {

const char* lramm_status_string(lramm_status s) {
  switch (s) {
    case LRAMM_OK: return "ok";
    case LRAMM_E_INVALID: return "invalid argument";
    case LRAMM_E_SHAPE: return "inconsistent sizes or leading dimensions";
    case LRAMM_E_RANK: return "sketch width l = r + p outside [1, min(m, k)]";
    case LRAMM_E_WORKSPACE: return "workspace missing or too small";
    case LRAMM_E_NONFINITE: return "non-finite value met by a quantiser";
    case LRAMM_E_BREAKDOWN: return "Cholesky breakdown";
    case LRAMM_E_OVERFLOW: return "K too large for the int32 accumulator";
    case LRAMM_E_HIP: return "HIP runtime error";
    case LRAMM_E_UNSUPPORTED: return "unsupported format, type or device";
    case LRAMM_E_STALL: return "a Cholesky wait ran past its bound (result not valid)";
    case LRAMM_E_SCRATCH: return "problem needs more scratch than the no-allocation buffer holds";
    default: return "unknown status";
  }
}

lramm_status lramm_init(void) {
  int dev = 0;
  LRAMM_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  LRAMM_HIP(hipGetDeviceProperties(&prop, dev));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return LRAMM_E_UNSUPPORTED;
  void* sp = nullptr;   // this GPU's no-allocation scratch, looked up once
  return scratch_address(&sp);
}

int64_t lramm_pitch(int64_t K, int32_t fmt) { return pitch_bytes(K, fmt); }

lramm_status lramm_plan_create(const lramm_desc* desc, lramm_plan** out) {
  if (!desc || !out) return LRAMM_E_INVALID;
  if ((desc->trans_a | desc->trans_b) & ~1 || (desc->side & ~1)) return LRAMM_E_INVALID;
  // side 1 sketches the right operand: C^T = B^T A^T with B^T as the left one
  lramm_desc d = *desc;
  if (desc->side) {
    d.m = desc->n;
    d.n = desc->m;
    d.a_type = desc->b_type;
    d.b_type = desc->a_type;
  }
  if (d.m <= 0 || d.n <= 0 || d.k <= 0) return LRAMM_E_SHAPE;
  if (d.m > INT32_MAX || d.n > INT32_MAX || d.k > INT32_MAX) return LRAMM_E_SHAPE;
  if (d.r < 0 || d.p < 0 || d.q < 0 || d.q > 16) return LRAMM_E_INVALID;
  int64_t l = (int64_t)d.r + d.p;
  if (l < 1 || l > d.m || l > d.k) return LRAMM_E_RANK;
  if (!valid_fmt(d.fmt_sketch) || !valid_fmt(d.fmt_proj) || !valid_fmt(d.fmt_g1) || !valid_fmt(d.fmt_g2))
    return LRAMM_E_UNSUPPORTED;
  if (!valid_io(d.a_type) || !valid_io(d.b_type) || !valid_io(d.c_type)) return LRAMM_E_UNSUPPORTED;
  if (d.flags & ~(uint32_t)(LRAMM_PLAN_EXCLUSIVE | LRAMM_PLAN_SRHT | LRAMM_PLAN_ESTIMATE | LRAMM_PLAN_ONE_PASS))
    return LRAMM_E_INVALID;
  if (d.flags & LRAMM_PLAN_SRHT) {
    // the transform runs along rows of A' stored row-major, k' <= 32768
    const int at0 = desc->side ? 1 - desc->trans_b : desc->trans_a;
    if (at0 || d.k < 2 || srht_padded(d.k) > 32768) return LRAMM_E_UNSUPPORTED;
  }
  // int32 accumulator bound of every integer product
  if ((d.fmt_sketch != LRAMM_BF16F && d.k > qk_bound(d.fmt_sketch)) ||
      (d.fmt_proj != LRAMM_BF16F && d.m > qk_bound(d.fmt_proj)) ||
      (d.fmt_g1 != LRAMM_BF16F && d.k > qk_bound(d.fmt_g1)))
    return LRAMM_E_OVERFLOW;
  int64_t lp = round_up(l, 32);
  if (lp > 1024) return LRAMM_E_UNSUPPORTED;    // FP64 TRSM row block must fit LDS

  lramm_plan* p = new (std::nothrow) lramm_plan();
  if (!p) return LRAMM_E_INVALID;
  p->user = *desc;
  p->d = d;
  // storage of the operands the library runs on: A' = B^T is stored
  // transposed when B is stored as is, and so on
  p->at = desc->side ? 1 - desc->trans_b : desc->trans_a;
  p->bt = desc->side ? 1 - desc->trans_a : desc->trans_b;
  p->ct = desc->side;
  p->chain_mode = (d.flags & LRAMM_PLAN_EXCLUSIVE) ? CHAIN_EXCLUSIVE : CHAIN_SHARED;
  p->srht = (d.flags & LRAMM_PLAN_SRHT) != 0;
  p->estimate = (d.flags & LRAMM_PLAN_ESTIMATE) != 0;
  p->passes = (d.flags & LRAMM_PLAN_ONE_PASS) ? 1 : 2;
  p->l = l;
  p->lp = lp;
  const int64_t m = d.m, n = d.n, k = d.k;
  p->pAr = pitch_bytes(k, d.fmt_sketch);
  p->pAc = pitch_bytes(m, d.fmt_proj);
  p->pBc = pitch_bytes(k, d.fmt_g1);
  p->pOm = pitch_bytes(k, d.fmt_sketch);
  p->pQZc = pitch_bytes(k, d.fmt_sketch);
  p->pQc = pitch_bytes(m, d.fmt_proj);
  p->pQr = pitch_bytes(l, d.fmt_g2);
  p->pBtq = pitch_bytes(k, d.fmt_g1);
  p->pTtq = pitch_bytes(l, d.fmt_g2);

  size_t c = 0;
  {
    size_t w = 64;   // status word (first) and padding
    auto seg = [&](size_t words) {
      size_t o = w;
      w += (words + 63) / 64 * 64;
      return o;
    };
    p->mx_A = seg((size_t)k);
    p->mx_B = seg((size_t)n);
    p->mx_Om = seg((size_t)l);
    p->mx_Q = seg((size_t)lp * (d.q + 1));
    p->mx_QZ = seg((size_t)lp * (d.q > 0 ? d.q : 1));
    p->mx_Ar = seg((size_t)m);
    p->zero_words = w;
    p->off_zero = carve(&c, w * 4);
    p->off_flags = p->off_zero;
  }
  p->off_Ar = carve(&c, (size_t)m * p->pAr);
  p->off_sAr = carve(&c, (size_t)m * 4);
  p->off_Ac = carve(&c, (size_t)k * p->pAc);
  p->off_sAc = carve(&c, (size_t)k * 4);
  p->off_Bc = carve(&c, (size_t)n * p->pBc);
  p->off_sBc = carve(&c, (size_t)n * 4);
  p->off_OmT = carve(&c, (size_t)l * k * 4);
  p->off_Om = carve(&c, (size_t)l * p->pOm);
  p->off_sOm = carve(&c, (size_t)l * 4);
  if (p->estimate) p->off_norms = carve(&c, (size_t)(2 + 2 * sumsq_parts_max()) * 8);
  if (p->srht) {
    p->off_srS = carve(&c, (size_t)l * 4);
    p->off_srD = carve(&c, (size_t)(srht_padded(k) + 31) / 32 * 4);
    p->off_srK = carve(&c, (size_t)srht_padded(k) * 4);
  }
  p->off_Y = carve(&c, (size_t)m * lp * 4);
  p->off_Q = carve(&c, (size_t)m * lp * 8);
  if (d.q > 0) {
    p->off_Z = carve(&c, (size_t)k * lp * 4);
    p->off_QZ = carve(&c, (size_t)k * lp * 8);
    p->off_QZc = carve(&c, (size_t)l * p->pQZc);
    p->off_sQZc = carve(&c, (size_t)l * 4);
  }
  p->off_Qc = carve(&c, (size_t)l * p->pQc);
  p->off_sQc = carve(&c, (size_t)l * 4);
  p->off_Qr = carve(&c, (size_t)m * p->pQr);
  p->off_sQr = carve(&c, (size_t)m * 4);
  p->off_Bt = carve(&c, (size_t)l * k * 4);
  p->off_Btq = carve(&c, (size_t)l * p->pBtq);
  p->off_sBt = carve(&c, (size_t)l * 4);
  p->off_Tt = carve(&c, (size_t)n * lp * 4);
  p->off_Ttq = carve(&c, (size_t)n * p->pTtq);
  p->off_sTt = carve(&c, (size_t)n * 4);
  {
    // the orthonormalisations run on m rows (sketches) and k rows (power
    // iterations); the workspace is not monotone in the row count
    const size_t wm = cholqr2_workspace(m, l), wk = cholqr2_workspace(k, l);
    p->chol_bytes = wm > wk ? wm : wk;
  }
  p->off_chol = carve(&c, p->chol_bytes);
  size_t sb = 0, t;
  t = gemm_nt_workspace(m, l, k, d.fmt_sketch); sb = t > sb ? t : sb;
  t = gemm_nt_workspace(k, l, m, d.fmt_proj); sb = t > sb ? t : sb;
  t = gemm_nt_workspace(l, k, m, d.fmt_proj); sb = t > sb ? t : sb;
  t = gemm_nt_workspace(n, l, k, d.fmt_g1); sb = t > sb ? t : sb;
  t = gemm_nt_workspace(l, n, k, d.fmt_g1); sb = t > sb ? t : sb;   // G1 as T = Bt B
  t = gemm_nt_workspace(m, n, l, d.fmt_g2); sb = t > sb ? t : sb;
  t = gemm_nt_workspace(n, m, l, d.fmt_g2); sb = t > sb ? t : sb;   // C' written transposed
  p->split_bytes = sb;
  p->off_split = carve(&c, sb);
  // backward scratch
  p->off_W = carve(&c, (size_t)l * n * 4);
  p->off_Bte = carve(&c, (size_t)l * k * 4);
  p->off_V = carve(&c, (size_t)l * k * 4);
  p->total = c + 256;
  // side stream (default priority) and fork/join events; without them the
  // forward runs everything on the caller's stream
  if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess) p->side = nullptr;
  if (p->side && (hipEventCreateWithFlags(&p->ev_fork, kOrderEvent) != hipSuccess ||
                  hipEventCreateWithFlags(&p->ev_join, kOrderEvent) != hipSuccess ||
                  hipEventCreateWithFlags(&p->ev_omega, kOrderEvent) != hipSuccess ||
                  hipEventCreateWithFlags(&p->ev_sketch, kOrderEvent) != hipSuccess)) {
    (void)hipStreamDestroy(p->side);
    p->side = nullptr;
  }
  *out = p;
  return LRAMM_OK;
}

void lramm_plan_destroy(lramm_plan* plan) {
  if (!plan) return;
  for (hipEvent_t e : plan->events) (void)hipEventDestroy(e);
  if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
  if (plan->ev_join) (void)hipEventDestroy(plan->ev_join);
  if (plan->ev_omega) (void)hipEventDestroy(plan->ev_omega);
  if (plan->ev_sketch) (void)hipEventDestroy(plan->ev_sketch);
  if (plan->side) (void)hipStreamDestroy(plan->side);
  delete plan;
}

lramm_status lramm_plan_set_timing(lramm_plan* plan, int32_t enable) {
  if (!plan) return LRAMM_E_INVALID;
  plan->timing = enable != 0;
  return LRAMM_OK;
}

lramm_status lramm_stage_times(lramm_plan* plan, double* ms, int64_t* counts) {
  if (!plan) return LRAMM_E_INVALID;
  for (size_t i = 0; i < plan->rec_stage.size(); ++i) {
    hipEvent_t a = plan->events[2 * i], b = plan->events[2 * i + 1];
    LRAMM_HIP(hipEventSynchronize(b));
    float t = 0.0f;
    LRAMM_HIP(hipEventElapsedTime(&t, a, b));
    int st = plan->rec_stage[i];
    plan->stage_ms[st] += t;
    plan->stage_n[st] += plan->rec_weight[i];
  }
  plan->rec_stage.clear();
  plan->rec_weight.clear();
  plan->next_event = 0;
  for (int i = 0; i < LRAMM_NSTAGES; ++i) {
    if (ms) ms[i] = plan->stage_ms[i];
    if (counts) counts[i] = plan->stage_n[i];
    plan->stage_ms[i] = 0.0;
    plan->stage_n[i] = 0;
  }
  return LRAMM_OK;
}

const char* lramm_stage_name(int32_t stage) {
  return (stage >= 0 && stage < LRAMM_NSTAGES) ? kStageNames[stage] : "unknown";
}

lramm_status lramm_workspace_bytes(const lramm_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return LRAMM_E_INVALID;
  *bytes = plan->total;
  return LRAMM_OK;
}

}  // extern "C"

namespace {
// The forward; with range_only (B and C unused, may be null) it stops after
// the projection Bt = Q^T A, leaving Q and Bt in the workspace.
lramm_status forward_impl(lramm_plan* P, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                          int64_t ldc, const float* omega, int64_t ldo, void* ws, size_t ws_bytes, void* stream,
                          bool range_only) {
  if (!P || !A || (!range_only && (!B || !C))) return LRAMM_E_INVALID;
  if (!ws || ws_bytes < P->total) return LRAMM_E_WORKSPACE;
  {
    const lramm_desc& u = P->user;
    if (lda < (u.trans_a ? u.m : u.k)) return LRAMM_E_SHAPE;
    if (!range_only && (ldb < (u.trans_b ? u.k : u.n) || ldc < u.n)) return LRAMM_E_SHAPE;
  }
  if (P->user.side) {   // run on A' = B^T, B' = A^T
    std::swap(A, B);
    std::swap(lda, ldb);
  }
  const lramm_desc& d = P->d;
  const int64_t m = d.m, n = d.n, k = d.k, l = P->l, lp = P->lp;
  if (omega && ldo < l) return LRAMM_E_SHAPE;
  if (omega && P->srht) return LRAMM_E_INVALID;   // the structured sketch is drawn from the seed
  hipStream_t s = (hipStream_t)stream;
  uint8_t* base = reinterpret_cast<uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  void* W = base;
  uint32_t* flags = at<uint32_t>(W, P->off_flags);
  uint32_t* zero = at<uint32_t>(W, P->off_zero);
  uint32_t* mxA = zero + P->mx_A;
  uint32_t* mxB = zero + P->mx_B;
  auto mxQ = [&](int c) { return zero + P->mx_Q + (size_t)c * lp; };
  auto mxQZ = [&](int it) { return zero + P->mx_QZ + (size_t)it * lp; };
  void* split = P->split_bytes ? at<void>(W, P->off_split) : nullptr;
  const size_t sb = P->split_bytes;

  uint8_t* Ar = at<uint8_t>(W, P->off_Ar);
  float* sAr = at<float>(W, P->off_sAr);
  uint8_t* Ac = at<uint8_t>(W, P->off_Ac);
  float* sAc = at<float>(W, P->off_sAc);
  uint8_t* Bc = at<uint8_t>(W, P->off_Bc);
  float* sBc = at<float>(W, P->off_sBc);
  uint8_t* Om = at<uint8_t>(W, P->off_Om);
  float* sOm = at<float>(W, P->off_sOm);
  float* Y = at<float>(W, P->off_Y);
  double* Q = at<double>(W, P->off_Q);
  void* cws = at<void>(W, P->off_chol);

  // operand quantisation
  HookCtx hctx{P, s, {}};
  TimingHook hook{&hctx, hook_begin, hook_end};
  const TimingHook* hk = P->timing ? &hook : nullptr;
#define TIMED(stage, expr)                \
  do {                                    \
    StageTimer _t(P, s, stage);           \
    LRAMM_TRY(expr);                      \
  } while (0)
#define TIMED_ON(strm, stage, expr)       \
  do {                                    \
    StageTimer _t(P, strm, stage);        \
    LRAMM_TRY(expr);                      \
  } while (0)
  // The side stream first generates and quantises Omega (arithmetic bound)
  // while the main stream quantises A's rows (bandwidth bound).  A's column
  // codes and B's codes, first needed after the first orthonormalisation,
  // wait for the sketch: started earlier they take CUs and bandwidth from
  // it, while the orthonormalisation's launches leave most CUs idle.
  hipStream_t s2 = P->side ? P->side : s;
  // the status word and the column-maxima accumulators start at zero: one
  // fill on s before any kernel that may set a flag (the side stream forks
  // after it).  Without power iterations nothing precedes the structured
  // sketch on the main stream, so its samples go there directly (no event
  // hop), and their first launch clears the zero region instead of a fill.
  const bool srht_main = P->srht && d.q == 0;
  if (!srht_main) LRAMM_TRY(fill_u32(zero, 0u, (int64_t)P->zero_words, s));
  int32_t* srS = P->srht ? at<int32_t>(W, P->off_srS) : nullptr;
  uint32_t* srD = P->srht ? at<uint32_t>(W, P->off_srD) : nullptr;
  if (srht_main)
    TIMED(ST_OMEGA, launch_srht_samples(d.seed, k, l, srS, srD, at<uint32_t>(W, P->off_srK), s, zero,
                                        (int64_t)P->zero_words));
  // the side stream works before the sketch only for the test matrix (the
  // Gaussian one, or the structured one's samples beside A's row codes)
  const bool side_before = P->side && (P->srht ? !srht_main : omega == nullptr);
  if (side_before) {
    LRAMM_HIP(hipEventRecord(P->ev_fork, s));
    LRAMM_HIP(hipStreamWaitEvent(P->side, P->ev_fork, 0));
  }
  if (P->srht) {
    if (!srht_main) {
      // the sample set and the sign mask, beside A's row codes
      TIMED_ON(s2, ST_OMEGA, launch_srht_samples(d.seed, k, l, srS, srD, at<uint32_t>(W, P->off_srK), s2));
      if (P->side) LRAMM_HIP(hipEventRecord(P->ev_omega, P->side));
    }
  } else if (!omega) {
    if (d.fmt_sketch == LRAMM_BF16F || k <= omega_quant_max_k()) {
      // generated and quantised in one pass
      TIMED_ON(s2, ST_OMEGA, launch_omega_quant(d.seed, k, l, d.fmt_sketch, Om, P->pOm, sOm, s2));
    } else {
      float* OmT = at<float>(W, P->off_OmT);
      TIMED_ON(s2, ST_OMEGA, launch_omega(d.seed, k, l, l, OmT, k, s2));
      TIMED_ON(s2, ST_QUANT_OMEGA,
               launch_quantize(l, k, OmT, k, LRAMM_F32, d.fmt_sketch, 0, Om, P->pOm, sOm, flags, s2));
    }
    if (P->side) LRAMM_HIP(hipEventRecord(P->ev_omega, P->side));
  }
  // bf16 A in a bf16 sketch: the codes are A itself (rows of whole 64-element
  // tiles, 16-byte aligned), no pass over A
  const bool a_direct = d.fmt_sketch == LRAMM_BF16F && d.a_type == LRAMM_BF16 && !P->at && k % 64 == 0 &&
                        (lda * 2) % 16 == 0 && (uintptr_t)A % 16 == 0;
  // bf16 A (B) in a bf16 projection (G1): the products read the operand
  // itself, stored K-major, instead of a transposed copy
  const bool km_a = d.fmt_proj == LRAMM_BF16F && d.a_type == LRAMM_BF16 && !P->at && (lda * 2) % 16 == 0 &&
                    (uintptr_t)A % 16 == 0;
  const bool km_b = !range_only && d.fmt_g1 == LRAMM_BF16F && d.b_type == LRAMM_BF16 && !P->bt &&
                    (ldb * 2) % 16 == 0 && (uintptr_t)B % 16 == 0;
  P->last_km_a = km_a;
  P->last_km_b = km_b;
  // A's row codes (sketch format) and column codes (projection format) in
  // one format: both from two reads of A, before the sketch
  const bool fused_a = !(P->srht && d.q == 0) && !a_direct && !km_a && !P->at && d.fmt_sketch == d.fmt_proj;
  if (P->srht && d.q == 0) {
    Ar = nullptr;   // the structured sketch reads A itself; no sketch-format codes
  } else if (fused_a) {
    TIMED(ST_QUANT_A_ROWS, launch_quantize_both(m, k, A, lda, d.a_type, d.fmt_sketch, Ar, P->pAr, sAr, Ac, P->pAc,
                                                sAc, zero + P->mx_Ar, mxA, flags, s));
  } else if (a_direct) {
    Ar = reinterpret_cast<uint8_t*>(const_cast<void*>(A));
  } else if (!P->at) {
    TIMED(ST_QUANT_A_ROWS, launch_quantize(m, k, A, lda, d.a_type, d.fmt_sketch, 0, Ar, P->pAr, sAr, flags, s));
  } else {   // A' stored k x m: its rows are the stored columns
    TIMED(ST_QUANT_A_ROWS, launch_quantize(k, m, A, lda, d.a_type, d.fmt_sketch, 1, Ar, P->pAr, sAr, flags, s));
  }
  const int64_t pAr = a_direct ? lda * 2 : P->pAr;
  P->last_Ar = Ar;
  P->last_pAr = pAr;
  if (omega) {
    TIMED(ST_QUANT_OMEGA, launch_quantize(k, l, omega, ldo, LRAMM_F32, d.fmt_sketch, 1, Om, P->pOm, sOm, flags, s,
                                          zero + P->mx_Om));
  } else if (P->side && !srht_main) {
    LRAMM_HIP(hipStreamWaitEvent(s, P->ev_omega, 0));   // Omega's codes ready
  }
  // sketch, then the side stream's column codes, then the orthonormalisation
  if (P->srht)
    TIMED(ST_SKETCH, launch_srht(m, k, l, A, lda, d.a_type, srD, srS, Y, lp, s));
  else
    TIMED(ST_SKETCH, launch_gemm_nt(m, l, k, d.fmt_sketch, Ar, pAr, sAr, Om, P->pOm, sOm, 1.0f, 0.0f, Y, lp,
                                    LRAMM_F32, nullptr, 0, split, sb, s));
  // after the sketch it forms A's column codes, B's codes and ||A'||^2 when
  // they are needed; with none of them (bf16 operands read in place) it is
  // left out, and so are the two event hops
  const bool side_after = P->side && (!(fused_a || km_a) || !(range_only || km_b) || P->estimate);
  if (side_after) {
    LRAMM_HIP(hipEventRecord(P->ev_sketch, s));
    LRAMM_HIP(hipStreamWaitEvent(P->side, P->ev_sketch, 0));
  }
  if (fused_a || km_a) {
    // written with the row codes, or read in place
  } else if (!P->at)
    TIMED_ON(s2, ST_QUANT_A_COLS,
             launch_quantize(m, k, A, lda, d.a_type, d.fmt_proj, 1, Ac, P->pAc, sAc, flags, s2, mxA));
  else   // the columns of A' are the stored rows
    TIMED_ON(s2, ST_QUANT_A_COLS, launch_quantize(k, m, A, lda, d.a_type, d.fmt_proj, 0, Ac, P->pAc, sAc, flags, s2));
  if (range_only || km_b) {
  } else if (!P->bt) {
    TIMED_ON(s2, ST_QUANT_B, launch_quantize(k, n, B, ldb, d.b_type, d.fmt_g1, 1, Bc, P->pBc, sBc, flags, s2, mxB));
  } else {
    TIMED_ON(s2, ST_QUANT_B, launch_quantize(n, k, B, ldb, d.b_type, d.fmt_g1, 0, Bc, P->pBc, sBc, flags, s2));
  }
  double* norms = P->estimate ? at<double>(W, P->off_norms) : nullptr;
  if (norms) {
    // ||A'||_F^2 of the stored matrix (any layout), beside the orthonormalisation
    if (!P->at) LRAMM_TRY(launch_sumsq(m, k, A, lda, d.a_type, norms + 2, norms, s2));
    else LRAMM_TRY(launch_sumsq(k, m, A, lda, d.a_type, norms + 2, norms, s2));
  }
  if (side_after) LRAMM_HIP(hipEventRecord(P->ev_join, P->side));
  uint8_t* Qc = at<uint8_t>(W, P->off_Qc);
  float* sQc = at<float>(W, P->off_sQc);
  // bf16 projection and G2: Q's transposed and row codes from one read of Q,
  // or, with one Cholesky QR pass, written by the last solve beside Q itself
  const bool q_both = d.fmt_proj == LRAMM_BF16F && d.fmt_g2 == LRAMM_BF16F;
  bool q_codes = false;
  const QCodesOut q_out = {reinterpret_cast<uint16_t*>(at<uint8_t>(W, P->off_Qr)), P->pQr / 2,
                           at<float>(W, P->off_sQr), reinterpret_cast<uint16_t*>(Qc), P->pQc / 2, sQc, &q_codes};
  const QCodesOut* q_co = (q_both && P->passes == 1) ? &q_out : nullptr;
  TIMED(ST_CHOLQR2, launch_cholqr2(m, l, Y, lp, LRAMM_F32, Q, lp, cws, P->chol_bytes, flags, s, hk, mxQ(0),
                                   P->chain_mode, P->passes, d.q == 0 ? q_co : nullptr));
  if (side_after) LRAMM_HIP(hipStreamWaitEvent(s, P->ev_join, 0));   // join: A_c and B_c ready
  for (int it = 0; it < d.q; ++it) {
    float* Z = at<float>(W, P->off_Z);
    double* QZ = at<double>(W, P->off_QZ);
    uint8_t* QZc = at<uint8_t>(W, P->off_QZc);
    float* sQZc = at<float>(W, P->off_sQZc);
    TIMED(ST_QUANT_Q_COLS,
          launch_quantize(m, l, Q, lp, LRAMM_F64, d.fmt_proj, 1, Qc, P->pQc, sQc, flags, s, mxQ(it), true));
    if (km_a)
      TIMED(ST_POWER_Z, launch_gemm_nt(k, l, m, d.fmt_proj, A, lda * 2, sAc, Qc, P->pQc, sQc, 1.0f, 0.0f, Z, lp,
                                       LRAMM_F32, nullptr, 0, split, sb, s, false, 1));
    else
      TIMED(ST_POWER_Z, launch_gemm_nt(k, l, m, d.fmt_proj, Ac, P->pAc, sAc, Qc, P->pQc, sQc, 1.0f, 0.0f, Z, lp,
                                       LRAMM_F32, nullptr, 0, split, sb, s));
    TIMED(ST_CHOLQR2, launch_cholqr2(k, l, Z, lp, LRAMM_F32, QZ, lp, cws, P->chol_bytes, flags, s, hk, mxQZ(it),
                                     P->chain_mode, P->passes));
    TIMED(ST_QUANT_QZ,
          launch_quantize(k, l, QZ, lp, LRAMM_F64, d.fmt_sketch, 1, QZc, P->pQZc, sQZc, flags, s, mxQZ(it), true));
    TIMED(ST_POWER_Y, launch_gemm_nt(m, l, k, d.fmt_sketch, Ar, pAr, sAr, QZc, P->pQZc, sQZc, 1.0f, 0.0f, Y, lp,
                                     LRAMM_F32, nullptr, 0, split, sb, s));
    TIMED(ST_CHOLQR2,
          launch_cholqr2(m, l, Y, lp, LRAMM_F32, Q, lp, cws, P->chol_bytes, flags, s, hk, mxQ(it + 1),
                         P->chain_mode, P->passes, it + 1 == d.q ? q_co : nullptr));
  }
  // projection Bt = Q^T A  (l x k)
  float* Bt = at<float>(W, P->off_Bt);
  // (no maxima; the G2 codes are formed before they are needed)
  if (q_both) {
    if (!q_codes)
      TIMED(ST_QUANT_Q_COLS, launch_quantize_both(m, l, Q, lp, LRAMM_F64, LRAMM_BF16F, at<uint8_t>(W, P->off_Qr),
                                                  P->pQr, at<float>(W, P->off_sQr), Qc, P->pQc, sQc, nullptr, nullptr,
                                                  flags, s));
  } else
    TIMED(ST_QUANT_Q_COLS,
          launch_quantize(m, l, Q, lp, LRAMM_F64, d.fmt_proj, 1, Qc, P->pQc, sQc, flags, s, mxQ(d.q), true));
  uint8_t* Btq = at<uint8_t>(W, P->off_Btq);
  float* sBt = at<float>(W, P->off_sBt);
  // bf16 G1 and a projection summed over K slices: the slice sum also writes
  // Bt's bf16 row codes (when it does not, the row quantiser below runs)
  bool bt_codes = false;
  const CodesOut bt_out = {reinterpret_cast<uint16_t*>(Btq), P->pBtq / 2, pitch_elems(P->pBtq, LRAMM_BF16F), sBt,
                           &bt_codes, false};
  const CodesOut* bt_co = (!range_only && d.fmt_g1 == LRAMM_BF16F) ? &bt_out : nullptr;
  if (km_a)
    TIMED(ST_PROJ, launch_gemm_nt(l, k, m, d.fmt_proj, Qc, P->pQc, sQc, A, lda * 2, sAc, 1.0f, 0.0f, Bt, k,
                                  LRAMM_F32, nullptr, 0, split, sb, s, false, 2, bt_co));
  else
    TIMED(ST_PROJ, launch_gemm_nt(l, k, m, d.fmt_proj, Qc, P->pQc, sQc, Ac, P->pAc, sAc, 1.0f, 0.0f, Bt, k,
                                  LRAMM_F32, nullptr, 0, split, sb, s, false, 0, bt_co));
  if (norms)   // ||Bt||_F^2 = ||Q^T A'||_F^2 (up to the projection's quantisation)
    LRAMM_TRY(launch_sumsq(l, k, Bt, k, LRAMM_F32, norms + 2 + sumsq_parts_max(), norms + 1, s));
  if (range_only) return LRAMM_OK;
  // G1: T^T = B_c . Bt_q^T  (n x l)
  float* Tt = at<float>(W, P->off_Tt);
  if (!bt_codes)
    TIMED(ST_QUANT_BT, launch_quantize(l, k, Bt, k, LRAMM_F32, d.fmt_g1, 0, Btq, P->pBtq, sBt, flags, s));
  // Tt is T transposed: the row factor of T (that of B~) is this product's
  // column factor, so the epilogue applies it first
  // bf16 G2 and T = Bt_q B summed over K slices: the slice sum also writes
  // T's column codes (when it does not, the column quantiser below runs)
  uint8_t* Ttq = at<uint8_t>(W, P->off_Ttq);
  float* sTt = at<float>(W, P->off_sTt);
  bool tt_codes = false;
  const CodesOut tt_out = {reinterpret_cast<uint16_t*>(Ttq), P->pTtq / 2, pitch_elems(P->pTtq, LRAMM_BF16F), sTt,
                           &tt_codes, true};
  if (km_b)   // T = Bt_q B (l x n, ld n in the same buffer), B read in place as the right operand
    TIMED(ST_G1, launch_gemm_nt(l, n, k, d.fmt_g1, Btq, P->pBtq, sBt, B, ldb * 2, sBc, 1.0f, 0.0f, Tt, n, LRAMM_F32,
                                nullptr, 0, split, sb, s, false, 2, d.fmt_g2 == LRAMM_BF16F ? &tt_out : nullptr));
  else
    TIMED(ST_G1, launch_gemm_nt(n, l, k, d.fmt_g1, Bc, P->pBc, sBc, Btq, P->pBtq, sBt, 1.0f, 0.0f, Tt, lp, LRAMM_F32,
                                nullptr, 0, split, sb, s, true));
  // G2: C = alpha Q_r . Tt_q^T + beta C  (m x n)
  uint8_t* Qr = at<uint8_t>(W, P->off_Qr);
  float* sQr = at<float>(W, P->off_sQr);
  if (!q_both) TIMED(ST_QUANT_Q_ROWS, launch_quantize(m, l, Q, lp, LRAMM_F64, d.fmt_g2, 0, Qr, P->pQr, sQr, flags, s));
  if (km_b) {   // the rows of T^T are the columns of T
    if (!tt_codes)
      TIMED(ST_QUANT_TT, launch_quantize(l, n, Tt, n, LRAMM_F32, d.fmt_g2, 1, Ttq, P->pTtq, sTt, flags, s));
  } else
    TIMED(ST_QUANT_TT, launch_quantize(n, l, Tt, lp, LRAMM_F32, d.fmt_g2, 0, Ttq, P->pTtq, sTt, flags, s));
  if (!P->ct) {
    TIMED(ST_G2, launch_gemm_nt(m, n, l, d.fmt_g2, Qr, P->pQr, sQr, Ttq, P->pTtq, sTt, d.alpha, d.beta, C, ldc,
                                d.c_type, nullptr, 0, split, sb, s));
  } else {
    // C = C'^T written directly: C = T'^T Q'^T, Q's row factor (now the
    // column factor) applied first
    TIMED(ST_G2, launch_gemm_nt(n, m, l, d.fmt_g2, Ttq, P->pTtq, sTt, Qr, P->pQr, sQr, d.alpha, d.beta, C, ldc,
                                d.c_type, nullptr, 0, split, sb, s, true));
  }
#undef TIMED
#undef TIMED_ON
  return LRAMM_OK;
}
}  // namespace

extern "C" {

lramm_status lramm_forward(lramm_plan* P, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                           int64_t ldc, const float* omega, int64_t ldo, void* ws, size_t ws_bytes, void* stream) {
  return forward_impl(P, A, lda, B, ldb, C, ldc, omega, ldo, ws, ws_bytes, stream, false);
}

lramm_status lramm_factors(const lramm_plan* P, const void* ws, const double** Q, int64_t* ldq, const float** Bt,
                           int64_t* ldbt) {
  if (!P || !ws) return LRAMM_E_INVALID;
  const uint8_t* base = reinterpret_cast<const uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  if (Q) *Q = reinterpret_cast<const double*>(base + P->off_Q);
  if (ldq) *ldq = P->lp;
  if (Bt) *Bt = reinterpret_cast<const float*>(base + P->off_Bt);
  if (ldbt) *ldbt = P->d.k;
  return LRAMM_OK;
}

lramm_status lramm_intermediate(const lramm_plan* P, const void* ws, int32_t which, const void** ptr,
                                int64_t* rows, int64_t* cols, int64_t* ld, int32_t* dtype) {
  if (!P || !ws || !ptr || !rows || !cols || !ld || !dtype) return LRAMM_E_INVALID;
  const uint8_t* base = reinterpret_cast<const uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  const lramm_desc& d = P->d;
  switch (which) {
    case LRAMM_VIEW_Y:
      *ptr = base + P->off_Y, *rows = d.m, *cols = P->l, *ld = P->lp, *dtype = LRAMM_F32;
      break;
    case LRAMM_VIEW_Q:
      *ptr = base + P->off_Q, *rows = d.m, *cols = P->l, *ld = P->lp, *dtype = LRAMM_F64;
      break;
    case LRAMM_VIEW_BT:
      *ptr = base + P->off_Bt, *rows = P->l, *cols = d.k, *ld = d.k, *dtype = LRAMM_F32;
      break;
    case LRAMM_VIEW_TT:   // stored as T when G1 read B in place
      if (P->last_km_b) return LRAMM_E_INVALID;
      *ptr = base + P->off_Tt, *rows = d.n, *cols = P->l, *ld = P->lp, *dtype = LRAMM_F32;
      break;
    case LRAMM_VIEW_T:
      if (!P->last_km_b) return LRAMM_E_INVALID;
      *ptr = base + P->off_Tt, *rows = P->l, *cols = d.n, *ld = d.n, *dtype = LRAMM_F32;
      break;
    default: return LRAMM_E_INVALID;
  }
  return LRAMM_OK;
}

lramm_status lramm_codes(const lramm_plan* P, const void* ws, int32_t which, const void** codes, int64_t* rows,
                         int64_t* K, int64_t* pitch, const float** scales, int32_t* fmt) {
  if (!P || !ws || !codes || !rows || !K || !pitch || !scales || !fmt) return LRAMM_E_INVALID;
  const uint8_t* base = reinterpret_cast<const uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  const lramm_desc& d = P->d;
  const int64_t m = d.m, n = d.n, k = d.k, l = P->l;
  auto set = [&](size_t off_codes, size_t off_scales, int64_t r, int64_t kk, int64_t pt, int f) {
    *codes = base + off_codes, *rows = r, *K = kk, *pitch = pt, *fmt = f;
    *scales = reinterpret_cast<const float*>(base + off_scales);
  };
  switch (which) {
    case LRAMM_CODES_A_ROWS:
      if (!P->last_Ar) return LRAMM_E_INVALID;
      set(P->off_Ar, P->off_sAr, m, k, P->last_pAr, d.fmt_sketch);
      *codes = P->last_Ar;
      break;
    case LRAMM_CODES_SKETCH_R:
      if (P->srht && d.q == 0) return LRAMM_E_INVALID;   // the structured sketch takes no codes
      if (d.q > 0) set(P->off_QZc, P->off_sQZc, l, k, P->pQZc, d.fmt_sketch);
      else set(P->off_Om, P->off_sOm, l, k, P->pOm, d.fmt_sketch);
      break;
    case LRAMM_CODES_Q_COLS: set(P->off_Qc, P->off_sQc, l, m, P->pQc, d.fmt_proj); break;
    case LRAMM_CODES_A_COLS:   // not formed when the products read A in place
      if (P->last_km_a) return LRAMM_E_INVALID;
      set(P->off_Ac, P->off_sAc, k, m, P->pAc, d.fmt_proj);
      break;
    case LRAMM_CODES_BT_ROWS: set(P->off_Btq, P->off_sBt, l, k, P->pBtq, d.fmt_g1); break;
    case LRAMM_CODES_B_COLS:
      if (P->last_km_b) return LRAMM_E_INVALID;
      set(P->off_Bc, P->off_sBc, n, k, P->pBc, d.fmt_g1);
      break;
    case LRAMM_CODES_Q_ROWS: set(P->off_Qr, P->off_sQr, m, l, P->pQr, d.fmt_g2); break;
    case LRAMM_CODES_TT_ROWS: set(P->off_Ttq, P->off_sTt, n, l, P->pTtq, d.fmt_g2); break;
    default: return LRAMM_E_INVALID;
  }
  return LRAMM_OK;
}

namespace {
// A logical R x C matrix in memory: t == 0 row-major (element (i, j) at
// p[i*ld + j]), t == 1 stored as its transpose (at p[j*ld + i]).
struct MatV {
  const void* p;
  int64_t ld;
  int t;
  int type;
};

// C[M x N] = L[M x K] R[K x N] on the FP32 MFMA GEMM, C stored row-major
// (ct == 0) or transposed (ct == 1: then C^T = R^T L^T is formed).
lramm_status mm(int64_t M, int64_t N, int64_t K, MatV L, MatV R, void* C, int64_t ldc, int ct, int ctype,
                hipStream_t s) {
  if (!ct) return launch_gemm_f32(M, N, K, L.p, L.ld, L.t, L.type, R.p, R.ld, 1 - R.t, R.type, C, ldc, ctype, s);
  return launch_gemm_f32(N, M, K, R.p, R.ld, 1 - R.t, R.type, L.p, L.ld, L.t, L.type, C, ldc, ctype, s);
}
}  // namespace

lramm_status lramm_backward(lramm_plan* P, const void* dC, int64_t lddc, const void* A, int64_t lda, const void* B,
                            int64_t ldb, void* dA, int64_t ldda, void* dB, int64_t lddb, void* ws, size_t ws_bytes,
                            void* stream) {
  if (!P || !dC) return LRAMM_E_INVALID;
  if (!ws || ws_bytes < P->total) return LRAMM_E_WORKSPACE;
  const lramm_desc& u = P->user;
  if (lddc < u.n) return LRAMM_E_SHAPE;
  const int64_t wa = u.trans_a ? u.m : u.k, wb = u.trans_b ? u.k : u.n;   // stored row lengths of A and B
  if (dA && (!B || ldb < wb || ldda < wa)) return LRAMM_E_SHAPE;
  if (dB && (!A || lda < wa || lddb < wb)) return LRAMM_E_SHAPE;
  // the problem the library ran: A' = side ? B^T : A, B' = side ? A^T : B,
  // dC' = side ? dC^T : dC; the gradient of A' is that of B (transposed) and so on
  const bool sd = u.side != 0;
  const lramm_desc& d = P->d;
  const int64_t m = d.m, n = d.n, k = d.k, l = P->l, lp = P->lp;
  const MatV Ap{sd ? B : A, sd ? ldb : lda, P->at, d.a_type};
  const MatV Bp{sd ? A : B, sd ? lda : ldb, P->bt, d.b_type};
  const MatV dCp{dC, lddc, sd ? 1 : 0, d.c_type};
  void* dAp = sd ? dB : dA;
  void* dBp = sd ? dA : dB;
  const int64_t lddap = sd ? lddb : ldda, lddbp = sd ? ldda : lddb;
  hipStream_t s = (hipStream_t)stream;
  void* W = reinterpret_cast<uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  const double* Q = at<double>(W, P->off_Q);
  float* Wm = at<float>(W, P->off_W);      // l x n
  float* Bte = at<float>(W, P->off_Bte);   // l x k
  float* V = at<float>(W, P->off_V);       // l x k
  const MatV Qv{Q, lp, 0, LRAMM_F64}, QTv{Q, lp, 1, LRAMM_F64};
  // W = Q^T dC'  (l x n)
  LRAMM_TRY(mm(l, n, m, QTv, dCp, Wm, n, 0, LRAMM_F32, s));
  const MatV Wv{Wm, n, 0, LRAMM_F32};
  if (dBp) {
    // Bte = Q^T A' (l x k); dB' = Bte^T W (k x n), stored like B'
    LRAMM_TRY(mm(l, k, m, QTv, Ap, Bte, k, 0, LRAMM_F32, s));
    LRAMM_TRY(mm(k, n, l, MatV{Bte, k, 1, LRAMM_F32}, Wv, dBp, lddbp, P->bt, d.b_type, s));
  }
  if (dAp) {
    // V = W B'^T (l x k); dA' = Q V (m x k), stored like A'
    LRAMM_TRY(mm(l, k, n, Wv, MatV{Bp.p, Bp.ld, 1 - Bp.t, Bp.type}, V, k, 0, LRAMM_F32, s));
    LRAMM_TRY(mm(m, k, l, Qv, MatV{V, k, 0, LRAMM_F32}, dAp, lddap, P->at, d.a_type, s));
  }
  return LRAMM_OK;
}

lramm_status lramm_status_poll(const lramm_plan* P, const void* ws, void* stream, uint32_t* flags) {
  if (!P || !ws) return LRAMM_E_INVALID;
  const uint8_t* base = reinterpret_cast<const uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  uint32_t h = 0;
  hipStream_t s = (hipStream_t)stream;
  LRAMM_HIP(hipMemcpyAsync(&h, base + P->off_flags, sizeof(h), hipMemcpyDeviceToHost, s));
  LRAMM_HIP(hipStreamSynchronize(s));
  if (flags) *flags = h;
  if (h & LRAMM_FLAG_STALL) return LRAMM_E_STALL;
  return (h & LRAMM_FLAG_NONFINITE) ? LRAMM_E_NONFINITE : LRAMM_OK;
}

// ----------------------------------------------------------- uneven batch --
// Independent products, each with its own plan and workspace slice, spread
// over a few streams (longest first, each to the least loaded stream) so that
// small products overlap.  Capturing the sequence as a HIP graph
// (LRAMM_BATCH_GRAPH) is not available: capture attempts crashed inside the
// host runtime (also when capturing on a stream the batch owns, with every
// return code checked), so the flag is rejected.

}  // extern "C"

struct lramm_batch {
  std::vector<lramm_plan*> plans;
  std::vector<size_t> offs;           // workspace offset of each product
  std::vector<int> order;             // issue order (largest first)
  std::vector<int> stream_of;         // stream index of each product
  size_t total = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;       // one per stream
  hipEvent_t fork = nullptr;
};

namespace {

double product_work(const lramm_desc& d) {
  const double l = (double)d.r + d.p;
  return 2.0 * l * ((double)d.m * d.k * (2 + 2 * d.q) + (double)d.k * d.n + (double)d.m * d.n) +
         4.0 * l * l * ((double)d.m * (d.q + 1) + (double)d.k * d.q);
}

void batch_free(lramm_batch* b) {
  for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  delete b;
}

lramm_status batch_issue(lramm_batch* b, const void* const* A, const int64_t* lda, const void* const* B,
                         const int64_t* ldb, void* const* C, const int64_t* ldc, uint8_t* ws, hipStream_t s) {
  LRAMM_HIP(hipEventRecord(b->fork, s));
  for (hipStream_t t : b->streams) LRAMM_HIP(hipStreamWaitEvent(t, b->fork, 0));
  // Products on several streams may run their Cholesky launches at the same
  // time: each then uses the per-panel launches, whose workgroups never wait
  // for one another (one-launch Cholesky grids could keep each other's
  // workgroups off the CUs).
  const bool one_stream = b->streams.size() == 1;
  for (int i : b->order) {
    lramm_plan* P = b->plans[i];
    const int mode = P->chain_mode;
    if (!one_stream) P->chain_mode = CHAIN_OFF;
    const lramm_status st = lramm_forward(P, A[i], lda[i], B[i], ldb[i], C[i], ldc[i], nullptr, 0, ws + b->offs[i],
                                          P->total, b->streams[b->stream_of[i]]);
    P->chain_mode = mode;
    if (st != LRAMM_OK) return st;
  }
  for (size_t t = 0; t < b->streams.size(); ++t) {
    LRAMM_HIP(hipEventRecord(b->done[t], b->streams[t]));
    LRAMM_HIP(hipStreamWaitEvent(s, b->done[t], 0));
  }
  return LRAMM_OK;
}

}  // namespace

extern "C" {

lramm_status lramm_batch_create(int32_t count, lramm_plan* const* plans, int32_t nstreams, uint32_t flags,
                                lramm_batch** out) {
  if (!out || count < 1 || !plans || nstreams < 1 || nstreams > 16) return LRAMM_E_INVALID;
  if (flags & ~LRAMM_BATCH_GRAPH) return LRAMM_E_INVALID;
  if (flags & LRAMM_BATCH_GRAPH) return LRAMM_E_UNSUPPORTED;
  lramm_batch* b = new (std::nothrow) lramm_batch();
  if (!b) return LRAMM_E_INVALID;
  size_t c = 0;
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) {
      delete b;
      return LRAMM_E_INVALID;
    }
    if (plans[i]->timing) plans[i]->timing = false;   // no event timing inside a batch
    b->plans.push_back(plans[i]);
    b->offs.push_back(carve(&c, plans[i]->total));
  }
  b->total = c + 256;
  for (int i = 0; i < count; ++i) b->order.push_back(i);
  std::vector<double> work(count);
  for (int i = 0; i < count; ++i) work[i] = product_work(plans[i]->d);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return work[x] > work[y]; });
  const int ns = nstreams < count ? nstreams : count;
  std::vector<double> load(ns, 0.0);
  b->stream_of.assign(count, 0);
  for (int i : b->order) {
    int t = 0;
    for (int u = 1; u < ns; ++u)
      if (load[u] < load[t]) t = u;
    b->stream_of[i] = t;
    load[t] += work[i];
  }
  bool ok = hipEventCreateWithFlags(&b->fork, kOrderEvent) == hipSuccess;
  for (int t = 0; ok && t < ns; ++t) {
    hipStream_t st;
    hipEvent_t ev;
    ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;   // default priority
    if (ok) b->streams.push_back(st);
    ok = ok && hipEventCreateWithFlags(&ev, kOrderEvent) == hipSuccess;
    if (ok) b->done.push_back(ev);
  }
  if (!ok) {
    batch_free(b);
    return LRAMM_E_HIP;
  }
  *out = b;
  return LRAMM_OK;
}

lramm_status lramm_batch_workspace_bytes(const lramm_batch* b, size_t* bytes) {
  if (!b || !bytes) return LRAMM_E_INVALID;
  *bytes = b->total;
  return LRAMM_OK;
}

void lramm_batch_destroy(lramm_batch* b) {
  if (b) batch_free(b);
}

lramm_status lramm_batched_forward(lramm_batch* b, const void* const* A, const int64_t* lda, const void* const* B,
                                   const int64_t* ldb, void* const* C, const int64_t* ldc, void* ws,
                                   size_t ws_bytes, void* stream) {
  if (!b || !A || !lda || !B || !ldb || !C || !ldc) return LRAMM_E_INVALID;
  if (!ws || ws_bytes < b->total) return LRAMM_E_WORKSPACE;
  const int n = (int)b->plans.size();
  for (int i = 0; i < n; ++i) {
    const lramm_desc& d = b->plans[i]->d;
    if (!A[i] || !B[i] || !C[i]) return LRAMM_E_INVALID;
    const lramm_desc& u = b->plans[i]->user;
    if (lda[i] < (u.trans_a ? u.m : u.k) || ldb[i] < (u.trans_b ? u.k : u.n) || ldc[i] < u.n) return LRAMM_E_SHAPE;
    (void)d;
  }
  hipStream_t s = (hipStream_t)stream;
  uint8_t* base = reinterpret_cast<uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  return batch_issue(b, A, lda, B, ldb, C, ldc, base, s);
}

lramm_status lramm_batch_status_poll(const lramm_batch* b, const void* ws, void* stream, uint32_t* flags) {
  if (!b || !ws) return LRAMM_E_INVALID;
  const uint8_t* base = reinterpret_cast<const uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  uint32_t all = 0;
  for (size_t i = 0; i < b->plans.size(); ++i) {
    uint32_t f = 0;
    lramm_status st = lramm_status_poll(b->plans[i], base + b->offs[i], stream, &f);
    if (st != LRAMM_OK && st != LRAMM_E_NONFINITE) return st;
    all |= f;
  }
  if (flags) *flags = all;
  if (all & LRAMM_FLAG_STALL) return LRAMM_E_STALL;
  return (all & LRAMM_FLAG_NONFINITE) ? LRAMM_E_NONFINITE : LRAMM_OK;
}

// ------------------------------------------------------------ stage APIs --

lramm_status lramm_quantize(int64_t rows, int64_t cols, const void* X, int64_t ldx, int32_t xtype, int32_t fmt,
                            int32_t transpose, void* Xq, int64_t pitch, float* scales, uint32_t* flags,
                            void* stream) {
  if (rows < 0 || cols < 0) return LRAMM_E_SHAPE;
  if ((rows > 0 && cols > 0) && (!X || !Xq || !scales)) return LRAMM_E_INVALID;
  if (!valid_fmt(fmt)) return LRAMM_E_INVALID;
  if (xtype != LRAMM_F32 && xtype != LRAMM_BF16 && xtype != LRAMM_F64) return LRAMM_E_INVALID;
  if (transpose != 0 && transpose != 1) return LRAMM_E_INVALID;
  if (ldx < cols) return LRAMM_E_SHAPE;
  int64_t K = transpose ? rows : cols;
  if (pitch < pitch_bytes(K, fmt) || pitch % 16 != 0) return LRAMM_E_SHAPE;
  if ((uintptr_t)Xq % 16 != 0) return LRAMM_E_INVALID;
  return launch_quantize(rows, cols, X, ldx, xtype, fmt, transpose, Xq, pitch, scales, flags, (hipStream_t)stream);
}

size_t lramm_gemm_nt_workspace(int64_t M, int64_t N, int64_t K, int32_t fmt) {
  return gemm_nt_workspace(M, N, K, fmt);
}

lramm_status lramm_gemm_nt(int64_t M, int64_t N, int64_t K, int32_t fmt, const void* Lq, int64_t ldl,
                           const float* dL, const void* Rq, int64_t ldr, const float* dR, float alpha, float beta,
                           void* C, int64_t ldc, int32_t ctype, int32_t* acc_out, int64_t ld_acc, void* ws,
                           size_t ws_bytes, void* stream) {
  if (M < 0 || N < 0 || K < 0 || M > INT32_MAX || N > INT32_MAX) return LRAMM_E_SHAPE;
  if (!valid_fmt(fmt)) return LRAMM_E_UNSUPPORTED;
  if (ctype != LRAMM_F32 && ctype != LRAMM_BF16) return LRAMM_E_INVALID;
  if (M == 0 || N == 0) return LRAMM_OK;
  if (!Lq || !Rq || !C) return LRAMM_E_INVALID;
  if (fmt != LRAMM_BF16F && (!dL || !dR)) return LRAMM_E_INVALID;
  if (ldl < pitch_bytes(K, fmt) || ldr < pitch_bytes(K, fmt) || ldl % 16 || ldr % 16) return LRAMM_E_SHAPE;
  if ((uintptr_t)Lq % 16 || (uintptr_t)Rq % 16) return LRAMM_E_INVALID;
  if (ldc < N) return LRAMM_E_SHAPE;
  if (acc_out && (fmt == LRAMM_BF16F || fmt == LRAMM_FP8 || ld_acc < N)) return LRAMM_E_INVALID;
  if (fmt != LRAMM_BF16F && K > qk_bound(fmt)) return LRAMM_E_OVERFLOW;
  return launch_gemm_nt(M, N, K, fmt, Lq, ldl, dL, Rq, ldr, dR, alpha, beta, C, ldc, ctype, acc_out, ld_acc, ws,
                        ws_bytes, (hipStream_t)stream);
}

lramm_status lramm_omega(uint64_t seed, int64_t k, int64_t l, float* OmegaT, int64_t ldo, void* stream) {
  if (k < 0 || l < 0) return LRAMM_E_SHAPE;
  if (k == 0 || l == 0) return LRAMM_OK;
  if (!OmegaT) return LRAMM_E_INVALID;
  if (ldo < k) return LRAMM_E_SHAPE;
  return launch_omega(seed, k, l, l, OmegaT, ldo, (hipStream_t)stream);
}

lramm_status lramm_error_estimate(const lramm_plan* P, const void* ws, void* stream, double* out) {
  if (!P || !ws || !out) return LRAMM_E_INVALID;
  if (!P->estimate) return LRAMM_E_INVALID;
  const uint8_t* base = reinterpret_cast<const uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  double h[2] = {0.0, 0.0};
  hipStream_t s = (hipStream_t)stream;
  LRAMM_HIP(hipMemcpyAsync(h, base + P->off_norms, sizeof(h), hipMemcpyDeviceToHost, s));
  LRAMM_HIP(hipStreamSynchronize(s));
  const double a2 = h[0], b2 = h[1];
  const double gap = a2 - b2 > 0.0 ? a2 - b2 : 0.0;
  out[0] = a2 > 0.0 ? sqrt(gap / a2) : 0.0;
  out[1] = a2;
  out[2] = b2;
  return LRAMM_OK;
}

lramm_status lramm_srht_samples(uint64_t seed, int64_t k, int64_t l, int32_t* S, uint32_t* sign_bits,
                                uint32_t* keys, void* stream) {
  if (k < 2 || l < 1) return l < 1 ? LRAMM_E_RANK : LRAMM_E_UNSUPPORTED;
  if (!S || !sign_bits || !keys) return LRAMM_E_INVALID;
  return launch_srht_samples(seed, k, l, S, sign_bits, keys, (hipStream_t)stream);
}

lramm_status lramm_srht_sketch(int64_t m, int64_t k, int64_t l, const void* A, int64_t lda, int32_t a_type,
                               const int32_t* S, const uint32_t* sign_bits, float* Y, int64_t ldy, void* stream) {
  if (m < 0 || k < 2 || l < 1) return m < 0 ? LRAMM_E_SHAPE : (l < 1 ? LRAMM_E_RANK : LRAMM_E_UNSUPPORTED);
  if (lda < k || ldy < l) return LRAMM_E_SHAPE;
  if (m > 0 && (!A || !S || !sign_bits || !Y)) return LRAMM_E_INVALID;
  if (a_type != LRAMM_F32 && a_type != LRAMM_BF16) return LRAMM_E_UNSUPPORTED;
  return launch_srht(m, k, l, A, lda, a_type, sign_bits, S, Y, ldy, (hipStream_t)stream);
}

int64_t lramm_srht_padded(int64_t k) { return k < 1 ? 0 : srht_padded(k); }

size_t lramm_cholqr2_workspace(int64_t rows, int64_t l) { return cholqr2_workspace(rows, l); }

size_t lramm_cholqr2_workspace_min(int64_t rows, int64_t l) { return cholqr2_workspace_min(rows, l); }

int32_t lramm_chol_one_launch(int64_t l, int32_t compute_units, uint32_t plan_flags) {
  if (l < 1 || round_up(l, 32) > 1024 || compute_units < 1) return 0;
  return chain_admits(l, compute_units, (plan_flags & LRAMM_PLAN_EXCLUSIVE) ? CHAIN_EXCLUSIVE : CHAIN_SHARED) ? 1
                                                                                                             : 0;
}

lramm_status lramm_cholqr2(int64_t rows, int64_t l, const void* Y, int64_t ldy, int32_t ytype, double* Q,
                           int64_t ldq, void* ws, size_t ws_bytes, uint32_t* flags, void* stream) {
  if (rows < 0 || l < 0) return LRAMM_E_SHAPE;
  if (rows == 0 || l == 0) return LRAMM_OK;
  if (!Y || !Q) return LRAMM_E_INVALID;
  if (l > rows) return LRAMM_E_RANK;
  if (ldy < l || ldq < round_up(l, 32)) return LRAMM_E_SHAPE;
  if (round_up(l, 32) > 1024) return LRAMM_E_UNSUPPORTED;
  if (ytype != LRAMM_F32 && ytype != LRAMM_F64) return LRAMM_E_UNSUPPORTED;
  if (!ws || ws_bytes < cholqr2_workspace(rows, l)) return LRAMM_E_WORKSPACE;
  return launch_cholqr2(rows, l, Y, ldy, ytype, Q, ldq, ws, ws_bytes, flags, (hipStream_t)stream);
}

lramm_status lramm_r_factor(int64_t rows, int64_t l, const void* Y, int64_t ldy, int32_t ytype, const double* Q,
                            int64_t ldq, double* R, int64_t ldr, void* stream) {
  if (rows < 0 || l < 0) return LRAMM_E_SHAPE;
  if (l == 0) return LRAMM_OK;
  if (!Y || !Q || !R) return LRAMM_E_INVALID;
  if (l > rows) return LRAMM_E_RANK;
  if (ldy < l || ldq < l || ldr < l) return LRAMM_E_SHAPE;
  if (ytype != LRAMM_F32 && ytype != LRAMM_F64) return LRAMM_E_UNSUPPORTED;
  return launch_r_factor(rows, l, Y, ldy, ytype, Q, ldq, R, ldr, (hipStream_t)stream);
}

lramm_status lramm_cholqr2_noalloc(int64_t rows, int64_t l, const void* Y, int64_t ldy, int32_t ytype, double* Q,
                                   int64_t ldq, uint32_t* flags, void* stream) {
  if (rows < 0 || l < 0) return LRAMM_E_SHAPE;
  if (rows == 0 || l == 0) return LRAMM_OK;
  if (!Y || !Q) return LRAMM_E_INVALID;
  if (l > rows) return LRAMM_E_RANK;
  if (ldy < l || ldq < round_up(l, 32)) return LRAMM_E_SHAPE;
  if (round_up(l, 32) > 1024) return LRAMM_E_UNSUPPORTED;
  if (ytype != LRAMM_F32 && ytype != LRAMM_F64) return LRAMM_E_UNSUPPORTED;
  const size_t need = cholqr2_workspace_min(rows, l);   // fewer Gram chunks when the default does not fit
  if (need > (size_t)LRAMM_NOALLOC_SCRATCH_BYTES) return LRAMM_E_SCRATCH;
  void* ws = nullptr;
  LRAMM_TRY(scratch_address(&ws));
  // every scratch word the kernels read is written earlier in the same call
  // (partial Grams, factors, and the gate word and progress counters that
  // the first Gram reduction clears), so the previous call's contents need
  // no clearing
  return launch_cholqr2(rows, l, Y, ldy, ytype, Q, ldq, ws, (size_t)LRAMM_NOALLOC_SCRATCH_BYTES, flags,
                        (hipStream_t)stream);
}

// ------------------------------------------------------------ two-sided --
// Alg. 3: rank-r RSVD of A and of B (each the one-sided range finder and
// projection, then the small SVD of the l x k projection through its Gram
// matrix), Sigma and Gamma absorbed into U~ = Q_A U'_A S_A and
// Z~ = U'_B^T (Q_B^T B) = G_B Z_B^T, and the chain E1 = QM(V^T W, d1),
// E2 = QM(E1 Z~, d2), D = alpha QM(U~ E2, d3) + beta C.

}  // extern "C"

struct lramm_ts_plan {
  lramm_ts_desc d;
  lramm_plan* pa = nullptr;   // RSVD of A: one-sided plan run up to its projection
  lramm_plan* pb = nullptr;   // RSVD of B: B as the left operand (k x n)
  int64_t l = 0, n2 = 0;      // sketch width and its even padding (Jacobi order)
  size_t off_wa = 0, off_wb = 0, off_flags = 0;
  size_t off_GA, off_GB, off_VA, off_VB, off_UpA, off_SA, off_UpSA, off_UpSiA, off_UpB, off_SB, off_UpSB, off_UpSiB;
  size_t off_Ut, off_Vt, off_W, off_Zs, off_E1, off_E2;
  size_t off_Vtq, off_sVt, off_Wq, off_sW, off_E1q, off_sE1, off_Zsq, off_sZs, off_Utq, off_sUt, off_E2q, off_sE2;
  size_t off_split = 0, split_bytes = 0;
  int64_t pVt, pW, pE1, pZs, pUt, pE2;
  size_t total = 0;
};

extern "C" {

lramm_status lramm_ts_plan_create(const lramm_ts_desc* desc, lramm_ts_plan** out) {
  if (!desc || !out) return LRAMM_E_INVALID;
  const lramm_ts_desc& d = *desc;
  if (d.m <= 0 || d.n <= 0 || d.k <= 0 || d.m > INT32_MAX || d.n > INT32_MAX || d.k > INT32_MAX)
    return LRAMM_E_SHAPE;
  if (d.r < 1 || d.p < 0 || d.q < 0 || d.q > 16 || d.flags != 0) return LRAMM_E_INVALID;
  const int64_t l = (int64_t)d.r + d.p;
  if (l > d.m || l > d.k || l > d.n) return LRAMM_E_RANK;
  const int64_t n2 = round_up(l, 2);
  if (n2 > jacobi_max_order()) return LRAMM_E_UNSUPPORTED;
  if (!valid_fmt(d.fmt_e1) || !valid_fmt(d.fmt_e2) || !valid_fmt(d.fmt_e3)) return LRAMM_E_UNSUPPORTED;
  if ((d.fmt_e1 != LRAMM_BF16F && d.k > qk_bound(d.fmt_e1)) ||
      (d.fmt_e2 != LRAMM_BF16F && d.r > qk_bound(d.fmt_e2)) || (d.fmt_e3 != LRAMM_BF16F && d.r > qk_bound(d.fmt_e3)))
    return LRAMM_E_OVERFLOW;
  if (!valid_io(d.c_type)) return LRAMM_E_UNSUPPORTED;
  lramm_desc da{};
  da.m = d.m, da.n = 1, da.k = d.k, da.r = d.r, da.p = d.p, da.q = d.q;
  da.fmt_sketch = d.fmt_sketch, da.fmt_proj = d.fmt_proj, da.fmt_g1 = LRAMM_INT8, da.fmt_g2 = LRAMM_INT8;
  da.a_type = d.a_type, da.b_type = LRAMM_F32, da.c_type = LRAMM_F32, da.seed = d.seed;
  da.alpha = 1.0f, da.beta = 0.0f;
  lramm_desc db = da;
  db.m = d.k, db.k = d.n, db.a_type = d.b_type, db.seed = d.seed + 1;
  lramm_ts_plan* p = new (std::nothrow) lramm_ts_plan();
  if (!p) return LRAMM_E_INVALID;
  p->d = d;
  p->l = l;
  p->n2 = n2;
  lramm_status st = lramm_plan_create(&da, &p->pa);
  if (st == LRAMM_OK) st = lramm_plan_create(&db, &p->pb);
  if (st != LRAMM_OK) {
    lramm_ts_plan_destroy(p);
    return st;
  }
  const int64_t m = d.m, n = d.n, k = d.k, r = d.r;
  size_t c = 0;
  p->off_flags = carve(&c, 256);
  p->off_wa = carve(&c, p->pa->total);
  p->off_wb = carve(&c, p->pb->total);
  const size_t sq = (size_t)n2 * n2 * 8, fr = (size_t)n2 * r * 8;
  p->off_GA = carve(&c, sq), p->off_GB = carve(&c, sq), p->off_VA = carve(&c, sq), p->off_VB = carve(&c, sq);
  p->off_UpA = carve(&c, fr), p->off_UpSA = carve(&c, fr), p->off_UpSiA = carve(&c, fr), p->off_SA = carve(&c, r * 8);
  p->off_UpB = carve(&c, fr), p->off_UpSB = carve(&c, fr), p->off_UpSiB = carve(&c, fr), p->off_SB = carve(&c, r * 8);
  p->off_Ut = carve(&c, (size_t)m * r * 4), p->off_Vt = carve(&c, (size_t)r * k * 4);
  p->off_W = carve(&c, (size_t)k * r * 4), p->off_Zs = carve(&c, (size_t)r * n * 4);
  p->off_E1 = carve(&c, (size_t)r * r * 4), p->off_E2 = carve(&c, (size_t)r * n * 4);
  p->pVt = pitch_bytes(k, d.fmt_e1), p->pW = pitch_bytes(k, d.fmt_e1);
  p->pE1 = pitch_bytes(r, d.fmt_e2), p->pZs = pitch_bytes(r, d.fmt_e2);
  p->pUt = pitch_bytes(r, d.fmt_e3), p->pE2 = pitch_bytes(r, d.fmt_e3);
  p->off_Vtq = carve(&c, (size_t)r * p->pVt), p->off_sVt = carve(&c, r * 4);
  p->off_Wq = carve(&c, (size_t)r * p->pW), p->off_sW = carve(&c, r * 4);
  p->off_E1q = carve(&c, (size_t)r * p->pE1), p->off_sE1 = carve(&c, r * 4);
  p->off_Zsq = carve(&c, (size_t)n * p->pZs), p->off_sZs = carve(&c, n * 4);
  p->off_Utq = carve(&c, (size_t)m * p->pUt), p->off_sUt = carve(&c, m * 4);
  p->off_E2q = carve(&c, (size_t)n * p->pE2), p->off_sE2 = carve(&c, n * 4);
  size_t sb = 0, t;
  t = gemm_nt_workspace(r, r, k, d.fmt_e1); sb = t > sb ? t : sb;
  t = gemm_nt_workspace(r, n, r, d.fmt_e2); sb = t > sb ? t : sb;
  t = gemm_nt_workspace(m, n, r, d.fmt_e3); sb = t > sb ? t : sb;
  p->split_bytes = sb;
  p->off_split = carve(&c, sb);
  p->total = c + 256;
  *out = p;
  return LRAMM_OK;
}

void lramm_ts_plan_destroy(lramm_ts_plan* p) {
  if (!p) return;
  lramm_plan_destroy(p->pa);
  lramm_plan_destroy(p->pb);
  delete p;
}

lramm_status lramm_ts_workspace_bytes(const lramm_ts_plan* p, size_t* bytes) {
  if (!p || !bytes) return LRAMM_E_INVALID;
  *bytes = p->total;
  return LRAMM_OK;
}

lramm_status lramm_ts_forward(lramm_ts_plan* P, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                              int64_t ldc, const float* omega_a, int64_t ldoa, const float* omega_b, int64_t ldob,
                              void* ws, size_t ws_bytes, void* stream) {
  if (!P || !A || !B || !C) return LRAMM_E_INVALID;
  if (!ws || ws_bytes < P->total) return LRAMM_E_WORKSPACE;
  const lramm_ts_desc& d = P->d;
  const int64_t m = d.m, n = d.n, k = d.k, r = d.r, l = P->l, n2 = P->n2;
  if (lda < k || ldb < n || ldc < n) return LRAMM_E_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* W = reinterpret_cast<uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  uint32_t* flags = at<uint32_t>(W, P->off_flags);
  LRAMM_TRY(fill_u32(flags, 0u, 1, s));
  // 1. RSVD range finders and projections: Q_A (m x l), Bt_A = Q_A^T A
  //    (l x k); Q_B (k x l), Bt_B = Q_B^T B (l x n)
  void* wa = W + P->off_wa;
  void* wb = W + P->off_wb;
  LRAMM_TRY(forward_impl(P->pa, A, lda, nullptr, 0, nullptr, 0, omega_a, ldoa, wa, P->pa->total, stream, true));
  LRAMM_TRY(forward_impl(P->pb, B, ldb, nullptr, 0, nullptr, 0, omega_b, ldob, wb, P->pb->total, stream, true));
  const uint8_t* ba = reinterpret_cast<const uint8_t*>(round_up((int64_t)(uintptr_t)wa, 256));
  const uint8_t* bb = reinterpret_cast<const uint8_t*>(round_up((int64_t)(uintptr_t)wb, 256));
  const double* QA = reinterpret_cast<const double*>(ba + P->pa->off_Q);
  const float* BtA = reinterpret_cast<const float*>(ba + P->pa->off_Bt);
  const double* QB = reinterpret_cast<const double*>(bb + P->pb->off_Q);
  const float* BtB = reinterpret_cast<const float*>(bb + P->pb->off_Bt);
  const int64_t lpA = P->pa->lp, lpB = P->pb->lp;
  // 2. small SVDs: Gram of the projections' rows, Jacobi, rank-r factors
  double* GA = at<double>(W, P->off_GA);
  double* GB = at<double>(W, P->off_GB);
  LRAMM_TRY(launch_rowgram((int)l, (int)k, BtA, k, LRAMM_F32, GA, (int)n2, s));
  LRAMM_TRY(launch_rowgram((int)l, (int)n, BtB, n, LRAMM_F32, GB, (int)n2, s));
  double* UpA = at<double>(W, P->off_UpA);
  double* UpSA = at<double>(W, P->off_UpSA);
  double* UpSiA = at<double>(W, P->off_UpSiA);
  double* UpB = at<double>(W, P->off_UpB);
  LRAMM_TRY(launch_jacobi_svd((int)n2, (int)r, GA, at<double>(W, P->off_VA), UpA, at<double>(W, P->off_SA), UpSA,
                              UpSiA, flags, s));
  LRAMM_TRY(launch_jacobi_svd((int)n2, (int)r, GB, at<double>(W, P->off_VB), UpB, at<double>(W, P->off_SB),
                              at<double>(W, P->off_UpSB), at<double>(W, P->off_UpSiB), flags, s));
  // 3. factors in FP64 (rounded once to binary32): U~ = Q_A U'_A S_A (m x r),
  //    V^T = S_A^-1 U'_A^T Bt_A (r x k), W = Q_B U'_B (k x r),
  //    Z~ = U'_B^T Bt_B (r x n); rows of U' past l are zero
  float* Ut = at<float>(W, P->off_Ut);
  float* Vt = at<float>(W, P->off_Vt);
  float* Wf = at<float>(W, P->off_W);
  float* Zs = at<float>(W, P->off_Zs);
  LRAMM_TRY(launch_gemm_f64acc(m, r, l, QA, lpA, 0, LRAMM_F64, UpSA, r, 1, LRAMM_F64, Ut, r, s));
  LRAMM_TRY(launch_gemm_f64acc(r, k, l, UpSiA, r, 1, LRAMM_F64, BtA, k, 1, LRAMM_F32, Vt, k, s));
  LRAMM_TRY(launch_gemm_f64acc(k, r, l, QB, lpB, 0, LRAMM_F64, UpB, r, 1, LRAMM_F64, Wf, r, s));
  LRAMM_TRY(launch_gemm_f64acc(r, n, l, UpB, r, 1, LRAMM_F64, BtB, n, 1, LRAMM_F32, Zs, n, s));
  // 4. the chain of quantised products (Alg. 2 each)
  void* split = P->split_bytes ? at<void>(W, P->off_split) : nullptr;
  const size_t sb = P->split_bytes;
  uint8_t* Vtq = at<uint8_t>(W, P->off_Vtq);
  float* sVt = at<float>(W, P->off_sVt);
  uint8_t* Wq = at<uint8_t>(W, P->off_Wq);
  float* sW = at<float>(W, P->off_sW);
  float* E1 = at<float>(W, P->off_E1);
  LRAMM_TRY(launch_quantize(r, k, Vt, k, LRAMM_F32, d.fmt_e1, 0, Vtq, P->pVt, sVt, flags, s));
  LRAMM_TRY(launch_quantize(k, r, Wf, r, LRAMM_F32, d.fmt_e1, 1, Wq, P->pW, sW, flags, s));
  LRAMM_TRY(launch_gemm_nt(r, r, k, d.fmt_e1, Vtq, P->pVt, sVt, Wq, P->pW, sW, 1.0f, 0.0f, E1, r, LRAMM_F32, nullptr,
                           0, split, sb, s));
  uint8_t* E1q = at<uint8_t>(W, P->off_E1q);
  float* sE1 = at<float>(W, P->off_sE1);
  uint8_t* Zsq = at<uint8_t>(W, P->off_Zsq);
  float* sZs = at<float>(W, P->off_sZs);
  float* E2 = at<float>(W, P->off_E2);
  LRAMM_TRY(launch_quantize(r, r, E1, r, LRAMM_F32, d.fmt_e2, 0, E1q, P->pE1, sE1, flags, s));
  LRAMM_TRY(launch_quantize(r, n, Zs, n, LRAMM_F32, d.fmt_e2, 1, Zsq, P->pZs, sZs, flags, s));
  LRAMM_TRY(launch_gemm_nt(r, n, r, d.fmt_e2, E1q, P->pE1, sE1, Zsq, P->pZs, sZs, 1.0f, 0.0f, E2, n, LRAMM_F32,
                           nullptr, 0, split, sb, s));
  uint8_t* Utq = at<uint8_t>(W, P->off_Utq);
  float* sUt = at<float>(W, P->off_sUt);
  uint8_t* E2q = at<uint8_t>(W, P->off_E2q);
  float* sE2 = at<float>(W, P->off_sE2);
  LRAMM_TRY(launch_quantize(m, r, Ut, r, LRAMM_F32, d.fmt_e3, 0, Utq, P->pUt, sUt, flags, s));
  LRAMM_TRY(launch_quantize(r, n, E2, n, LRAMM_F32, d.fmt_e3, 1, E2q, P->pE2, sE2, flags, s));
  LRAMM_TRY(launch_gemm_nt(m, n, r, d.fmt_e3, Utq, P->pUt, sUt, E2q, P->pE2, sE2, d.alpha, d.beta, C, ldc, d.c_type,
                           nullptr, 0, split, sb, s));
  return LRAMM_OK;
}

lramm_status lramm_ts_intermediate(const lramm_ts_plan* P, const void* ws, int32_t which, const void** ptr,
                                   int64_t* rows, int64_t* cols, int64_t* ld, int32_t* dtype) {
  if (!P || !ws || !ptr || !rows || !cols || !ld || !dtype) return LRAMM_E_INVALID;
  const uint8_t* base = reinterpret_cast<const uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  const lramm_ts_desc& d = P->d;
  const int64_t m = d.m, n = d.n, k = d.k, r = d.r;
  auto set = [&](size_t off, int64_t rr, int64_t cc, int64_t ll, int32_t t) {
    *ptr = base + off, *rows = rr, *cols = cc, *ld = ll, *dtype = t;
  };
  switch (which) {
    case LRAMM_TS_UT: set(P->off_Ut, m, r, r, LRAMM_F32); break;
    case LRAMM_TS_VT: set(P->off_Vt, r, k, k, LRAMM_F32); break;
    case LRAMM_TS_W: set(P->off_W, k, r, r, LRAMM_F32); break;
    case LRAMM_TS_ZS: set(P->off_Zs, r, n, n, LRAMM_F32); break;
    case LRAMM_TS_E1: set(P->off_E1, r, r, r, LRAMM_F32); break;
    case LRAMM_TS_E2: set(P->off_E2, r, n, n, LRAMM_F32); break;
    case LRAMM_TS_SA: set(P->off_SA, r, 1, 1, LRAMM_F64); break;
    case LRAMM_TS_SB: set(P->off_SB, r, 1, 1, LRAMM_F64); break;
    case LRAMM_TS_UPA: set(P->off_UpA, P->l, r, r, LRAMM_F64); break;
    case LRAMM_TS_UPB: set(P->off_UpB, P->l, r, r, LRAMM_F64); break;
    default: return LRAMM_E_INVALID;
  }
  return LRAMM_OK;
}

lramm_status lramm_ts_status_poll(const lramm_ts_plan* P, const void* ws, void* stream, uint32_t* flags) {
  if (!P || !ws) return LRAMM_E_INVALID;
  const uint8_t* base = reinterpret_cast<const uint8_t*>(round_up((int64_t)(uintptr_t)ws, 256));
  uint32_t fa = 0, fb = 0, own = 0;
  lramm_status sa = lramm_status_poll(P->pa, base + P->off_wa, stream, &fa);
  lramm_status sbs = lramm_status_poll(P->pb, base + P->off_wb, stream, &fb);
  if (sa == LRAMM_E_HIP || sbs == LRAMM_E_HIP) return LRAMM_E_HIP;
  hipStream_t s = (hipStream_t)stream;
  LRAMM_HIP(hipMemcpyAsync(&own, base + P->off_flags, sizeof(own), hipMemcpyDeviceToHost, s));
  LRAMM_HIP(hipStreamSynchronize(s));
  const uint32_t all = fa | fb | own;
  if (flags) *flags = all;
  if (all & LRAMM_FLAG_STALL) return LRAMM_E_STALL;
  return (all & LRAMM_FLAG_NONFINITE) ? LRAMM_E_NONFINITE : LRAMM_OK;
}

lramm_status lramm_dense_gemm_nt(int64_t M, int64_t N, int64_t K, int32_t dtype, const void* L, int64_t ldl,
                                 const void* R, int64_t ldr, float* C, int64_t ldc, void* stream) {
  if (M < 0 || N < 0 || K < 0) return LRAMM_E_SHAPE;
  if (M == 0 || N == 0) return LRAMM_OK;
  if (!L || !R || !C) return LRAMM_E_INVALID;
  if (K % 64 || ldl % 64 || ldr % 64 || ldl < K || ldr < K || ldc < N) return LRAMM_E_SHAPE;
  if (dtype != LRAMM_BF16 && dtype != LRAMM_F32) return LRAMM_E_UNSUPPORTED;
  return launch_dense_gemm_nt(M, N, K, dtype, L, ldl, R, ldr, C, ldc, (hipStream_t)stream);
}

}  // extern "C"

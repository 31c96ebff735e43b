// C ABI of libvoxcsf.so: argument checking, dispatch, and the level loop of
// Algorithm 3 (Moroz, arXiv 2406.09857).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "eval.hpp"
#include "grad.hpp"

namespace vx {

static thread_local std::string g_error;

// Set while interval_eval_level_noalloc runs on this host thread: its
// launches record no timing events (creating one is an allocation of the
// runtime).
static thread_local bool g_prof_suppressed = false;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
}

const char* get_error() { return g_error.c_str(); }

static int check_poly(const vx_poly* P, int np, int k) {
  if (!P || np < 1) VX_FAIL(VX_EINVAL, "need at least one polynomial");
  if (np > VX_MAXPOLY) VX_FAIL(VX_EINVAL, "at most %d polynomials per system", VX_MAXPOLY);
  for (int p = 0; p < np; p++) {
    if (P[p].k != k) VX_FAIL(VX_EINVAL, "polynomial %d has k=%d, the box set has k=%d", p, P[p].k, k);
    if (P[p].degree < 0 || P[p].degree > 400) VX_FAIL(VX_EINVAL, "polynomial %d: degree %d outside [0, 400]", p, P[p].degree);
    if (P[p].side < P[p].degree + 1) VX_FAIL(VX_EINVAL, "polynomial %d: side %d < degree+1", p, P[p].side);
    if (!P[p].c_lo) VX_FAIL(VX_EINVAL, "polynomial %d: null coefficients", p);
    int64_t cube = 1;
    for (int i = 0; i < k; i++) cube *= P[p].side;
    if (cube > (int64_t)1 << 31) VX_FAIL(VX_EOVERFLOW, "polynomial %d: coefficient cube too large", p);
  }
  return VX_OK;
}

static int check_csf(const vx_csf* S, bool need_arrays) {
  if (!S) VX_FAIL(VX_EINVAL, "null CSF");
  if (S->k < 1 || S->k > VX_KMAX) VX_FAIL(VX_EINVAL, "k=%d outside [1, %d]", S->k, VX_KMAX);
  if (S->level < 0 || S->level > 29) VX_FAIL(VX_EINVAL, "level %d outside [0, 29]", S->level);
  for (int l = 0; l < S->k; l++) {
    if (S->n[l] < 0) VX_FAIL(VX_EINVAL, "negative node count at depth %d", l + 1);
    if (S->n[l] >= ((int64_t)1 << 31) - 1) VX_FAIL(VX_EOVERFLOW, "depth %d has %lld nodes (int32 limit)", l + 1, (long long)S->n[l]);
    if (l > 0 && S->n[l] < S->n[l - 1]) VX_FAIL(VX_EINVAL, "depth %d has fewer nodes than depth %d", l + 1, l);
    if (need_arrays && S->n[l] > 0 && !S->idx[l]) VX_FAIL(VX_EINVAL, "null labels at depth %d", l + 1);
    if (need_arrays && l + 1 < S->k && S->n[l] > 0 && !S->ptr[l]) VX_FAIL(VX_EINVAL, "null offsets at depth %d", l + 1);
  }
  return VX_OK;
}

static int check_dom(const double* dom, int k) {
  if (!dom) VX_FAIL(VX_EINVAL, "null domain");
  for (int j = 0; j < k; j++) {
    const double a = dom[2 * j], b = dom[2 * j + 1];
    if (!(a < b) || a != a || b != b || a - a != 0.0 || b - b != 0.0)
      VX_FAIL(VX_EINVAL, "axis %d: domain [%g, %g] is not a finite nonempty interval", j, a, b);
  }
  return VX_OK;
}

// The workspace contract: 256-byte aligned (every buffer carved from it is
// aligned to 256 bytes relative to its start, and kernels rely on 16-byte
// alignment of their rows).
static int check_ws(const void* ws) {
  if (ws && (reinterpret_cast<uintptr_t>(ws) & 255))
    VX_FAIL(VX_EINVAL, "workspace %p is not 256-byte aligned", ws);
  return VX_OK;
}

// Node counts of the CSF of the 2^k children of every box of S (the
// bisection of Algorithm 3, child c of box B being 2B + c): depth l + 1 holds
// at most 2^(l+1) n[l] nodes.  Labels and offsets are int32, so a bound that
// reaches 2^31 - 1 is VX_EOVERFLOW; the level loop and filter_subdivide both
// size the next level through this check.
static int next_level_bounds(const vx_csf* S, int64_t* ncap) {
  if (S->level >= 29) VX_FAIL(VX_EOVERFLOW, "level %d cannot be bisected (labels are int32)", S->level);
  for (int l = 0; l < S->k; l++) {
    const int64_t bound = S->n[l] << (l + 1);
    if (bound >= ((int64_t)1 << 31) - 1)
      VX_FAIL(VX_EOVERFLOW, "the next level may hold %lld nodes at depth %d (int32 limit)", (long long)bound, l + 1);
    ncap[l] = bound;
  }
  return VX_OK;
}

static int64_t theorem1_steps(const vx_poly* P, int np, const vx_csf* S) {
  int64_t total = 0;
  for (int p = 0; p < np; p++) {
    const int d = P[p].degree, k = S->k;
    for (int l = 0; l < k; l++) total += (ntup(k - l, d) - ntup(k - l - 1, d)) * S->n[l];
  }
  return total;
}

}  // namespace vx

// ---------------------------------------------------------------------------
// run_subdivision: the level loop.  The workspace is used from both ends:
// S_level sits at one end and the next level's CSF is built at the other, so
// the two swap ends every level without copies; everything else (enclosures,
// keep flags, K, scratch) lives in between.
// ---------------------------------------------------------------------------
namespace vx {

// Largest derivative table set per polynomial of a Taylor test: its k first
// derivatives (order 1), or its k(k+1)/2 second-order polynomials (order 2,
// which also has the k first derivatives: fewer).  Each set is one system of
// at most VX_MAXPOLY polynomials.
static int taylor_tables(int k, int order) { return order == 0 ? 0 : order == 1 ? k : k * (k + 1) / 2; }

static int check_taylor_polys(int np, int k, int order) {
  if (order == 0) return VX_OK;
  if (order >= 3) return VX_OK;  // the general path cuts its term systems into groups of VX_MAXPOLY
  const int per = taylor_tables(k, order);
  if (np * per > VX_MAXPOLY)
    VX_FAIL(VX_EINVAL, "Taylor test of order %d: %d polynomials x %d derivative tables exceeds %d", order, np, per,
            VX_MAXPOLY);
  return VX_OK;
}

// Orders 1..VX_TAYLOR_MAX_ORDER; the multipliers prod_i C(e_i + alpha_i,
// alpha_i) of the coefficient polynomials stay below C(d + m, m), which must
// be exact in double.
static int check_taylor_order(const vx_poly* P, int np, int order) {
  if (order < 1 || order > VX_TAYLOR_MAX_ORDER)
    VX_FAIL(VX_EINVAL, "Taylor order %d is outside 1..%d", order, VX_TAYLOR_MAX_ORDER);
  for (int p = 0; p < np; p++)
    if (binom64(P[p].degree + order, order) >= ((int64_t)1 << 53))
      VX_FAIL(VX_EUNSUPPORTED, "Taylor order %d of degree %d: coefficient multipliers reach 2^53", order,
              P[p].degree);
  return VX_OK;
}

// Algorithm 3 with the inclusion criterion: boxes kept by C0 that C1
// certifies join the output and are not bisected.  cont = keep && !incl
// (the boxes that continue); keep becomes 2 for the certified ones (1:
// continues, 0: excluded); the certified boxes are counted into *count, one
// atomic per wave.
__global__ void k_mark_certified(int64_t n, uint8_t* __restrict__ keep, const uint8_t* __restrict__ incl,
                                 uint8_t* __restrict__ cont, unsigned long long* __restrict__ count) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = 0;
  if (b < n) {
    const bool kp = keep[b] != 0, ce = kp && incl[b] != 0;
    cont[b] = (uint8_t)(kp && !ce);
    if (ce) keep[b] = 2;
    c = ce;
  }
  const uint64_t m = __ballot(c);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(count, (unsigned long long)__popcll(m));
}

// The count into the host-mapped result slot, visible before anything the
// stream does afterwards (the filter's flag).
__global__ void k_put_count(const unsigned long long* __restrict__ count, int64_t* out) {
  if (threadIdx.x == 0) {
    *reinterpret_cast<volatile int64_t*>(out) = (int64_t)*count;
    __threadfence_system();
  }
}

// Spin on the mapped flag instead of a stream wait (lower latency per level).
// The stream is queried now and then so that a failed or idle stream ends the
// wait with an error instead of spinning forever.
static int wait_for_flag(const int64_t* flag, int64_t value, hipStream_t st) {
  const volatile int64_t* f = flag;
  for (uint64_t spin = 0;; spin++) {
    if (*f == value) return VX_OK;
    if ((spin & 1023) == 1023) {
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {  // stream drained: the flag must be visible after a full wait
        VX_HIP(hipStreamSynchronize(st));
        if (*f == value) return VX_OK;
        VX_FAIL(VX_EHIP, "run_subdivision: the stream drained without signalling the level");
      }
      if (e != hipErrorNotReady) VX_FAIL(VX_EHIP, "run_subdivision: %s", hipGetErrorString(e));
    }
  }
}

static size_t csf_bytes(int k, const int64_t* cap) {
  size_t b = 0;
  for (int l = 0; l < k; l++) {
    b += ((size_t)cap[l] * 4 + 255) / 256 * 256;
    if (l + 1 < k) b += ((size_t)(cap[l] + 1) * 4 + 255) / 256 * 256;
  }
  return b;
}

static void csf_place(vx_csf* S, int k, int level, const int64_t* cap, char* base) {
  memset(S, 0, sizeof *S);
  S->k = k;
  S->level = level;
  size_t off = 0;
  for (int l = 0; l < k; l++) {
    S->cap[l] = cap[l];
    S->idx[l] = reinterpret_cast<int32_t*>(base + off);
    off += ((size_t)cap[l] * 4 + 255) / 256 * 256;
    if (l + 1 < k) {
      S->ptr[l] = reinterpret_cast<int32_t*>(base + off);
      off += ((size_t)(cap[l] + 1) * 4 + 255) / 256 * 256;
    }
  }
}

}  // namespace vx

using namespace vx;

extern "C" {

const char* vx_last_error(void) { return get_error(); }

size_t vx_taylor_workspace_bytes(const vx_poly* P, int32_t np, const vx_csf* S, int32_t order) {
  if (check_csf(S, false) || check_poly(P, np, S->k) || order < 1 || order > VX_TAYLOR_MAX_ORDER ||
      check_taylor_order(P, np, order) || check_taylor_polys(np, S->k, order))
    return 0;
  return mv_workspace_bytes(P, np, S, order);
}

size_t vx_workspace_bytes(int32_t which, const vx_poly* P, int32_t np, const vx_csf* S, int64_t n) {
  switch (which) {
    case VX_WS_EVAL:
      if (check_csf(S, false) || check_poly(P, np, S->k)) return 0;
      return eval_workspace_bytes(P, np, S);
    case VX_WS_FILTER:
      if (check_csf(S, false)) return 0;
      return filter_workspace_bytes(S);
    case VX_WS_BUILD:
      if (!S || S->k < 1 || S->k > VX_KMAX || n < 0) return 0;
      return build_workspace_bytes(S->k, n);
    case VX_WS_MEANVALUE:
    case VX_WS_TAYLOR2: {
      const int order = which == VX_WS_TAYLOR2 ? 2 : 1;
      if (check_csf(S, false) || check_poly(P, np, S->k) || np * taylor_tables(S->k, order) > VX_MAXPOLY) return 0;
      return mv_workspace_bytes(P, np, S, order);
    }
    case VX_WS_INCLUSION:
      if (check_csf(S, false) || check_poly(P, np, S->k)) return 0;
      return inclusion_workspace_bytes(P, np, S);
    case VX_WS_ORDER:
      if (check_csf(S, false) || (int64_t)S->k * S->level > 62) return 0;
      return order_workspace_bytes(S);
    case VX_WS_NEWTON:
      if (check_csf(S, false) || check_poly(P, np, S->k) || np > S->k) return 0;
      return newton_workspace_bytes(P, np, S);
    case VX_WS_GRAD:
      if (!P || np < 1 || np > PMAX_GRAD || check_poly(P, np, P[0].k)) return 0;
      if (S && check_csf(S, false)) return 0;
      return grad_workspace_bytes(P, np, S, n);
    default:
      return 0;
  }
}

int interval_eval_level(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, double* lo, double* hi,
                        uint8_t* keep, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_csf(S, true))) return rc;
  if ((rc = check_poly(P, np, S->k))) return rc;
  if ((rc = check_dom(dom, S->k))) return rc;
  if (S->n[S->k - 1] > 0 && (!lo || !hi)) VX_FAIL(VX_EINVAL, "null output arrays");
  if ((rc = check_ws(ws))) return rc;
  return eval_level_impl(P, np, S, dom, lo, hi, keep, ws, ws_bytes, (hipStream_t)stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Scratch of interval_eval_level_noalloc: one array per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: its device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is handed to
// kernels.
// ---------------------------------------------------------------------------
namespace vx {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

static int scratch_address(void** out) {
  int dev = 0;
  VX_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) VX_FAIL(VX_EUNSUPPORTED, "device %d: no scratch slot", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      VX_FAIL(VX_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return VX_OK;
}

// Mapped, coherent host slots through which the level loop's filter publishes
// its counts.  Pinning and mapping host memory costs tens of microseconds per
// call, so a slot returns to a pool when its run ends and serves later runs on
// the same device: one slot per call running at the same time, each held
// until the process ends.
struct CountSlot {
  int64_t* host = nullptr;
  int64_t* dev = nullptr;
  int device = -1;
};
constexpr size_t COUNT_SLOT_BYTES = sizeof(int64_t) * (2 * VX_KMAX + 2);
static std::mutex g_slot_mu;
static std::vector<CountSlot> g_free_slots;

static int take_count_slot(CountSlot* out) {
  int dev = 0;
  VX_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> g(g_slot_mu);
    for (size_t i = 0; i < g_free_slots.size(); i++)
      if (g_free_slots[i].device == dev) {
        *out = g_free_slots[i];
        g_free_slots.erase(g_free_slots.begin() + (long)i);
        return VX_OK;
      }
  }
  CountSlot s;
  s.device = dev;
  VX_HIP(hipHostMalloc((void**)&s.host, COUNT_SLOT_BYTES, hipHostMallocMapped | hipHostMallocCoherent));
  const hipError_t e = hipHostGetDevicePointer((void**)&s.dev, s.host, 0);
  if (e != hipSuccess) {
    (void)hipHostFree(s.host);
    VX_FAIL(VX_EHIP, "hipHostGetDevicePointer: %s", hipGetErrorString(e));
  }
  *out = s;
  return VX_OK;
}

static void give_count_slot(const CountSlot& s) {
  std::lock_guard<std::mutex> g(g_slot_mu);
  g_free_slots.push_back(s);
}

struct ProfSuppress {
  ProfSuppress() { g_prof_suppressed = true; }
  ~ProfSuppress() { g_prof_suppressed = false; }
};

}  // namespace vx

extern "C" {

int interval_eval_level_noalloc(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, double* lo,
                                double* hi, uint8_t* keep, void* stream) {
  int rc;
  if ((rc = check_csf(S, true))) return rc;
  if ((rc = check_poly(P, np, S->k))) return rc;
  if ((rc = check_dom(dom, S->k))) return rc;
  if (S->n[S->k - 1] > 0 && (!lo || !hi)) VX_FAIL(VX_EINVAL, "null output arrays");
  const size_t need = eval_workspace_bytes(P, np, S);
  if (need > NOALLOC_SCRATCH_BYTES)
    VX_FAIL(VX_ECAPACITY, "interval_eval_level_noalloc: this level needs %zu bytes of scratch, the static scratch "
            "holds %zu (use interval_eval_level with a workspace)", need, NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  ProfSuppress quiet;
  return eval_level_impl(P, np, S, dom, lo, hi, keep, ws, NOALLOC_SCRATCH_BYTES, (hipStream_t)stream);
}

int taylor_exclusion(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, int32_t order, double* lo,
                     double* hi, uint8_t* keep, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if (order < 1 || order > VX_TAYLOR_MAX_ORDER)
    VX_FAIL(VX_EINVAL, "Taylor order %d is outside 1..%d", order, VX_TAYLOR_MAX_ORDER);
  if ((rc = check_csf(S, true))) return rc;
  if ((rc = check_poly(P, np, S->k))) return rc;
  if ((rc = check_taylor_order(P, np, order))) return rc;
  if ((rc = check_taylor_polys(np, S->k, order))) return rc;
  if ((rc = check_dom(dom, S->k))) return rc;
  if (S->n[S->k - 1] > 0 && (!lo || !hi)) VX_FAIL(VX_EINVAL, "null output arrays");
  if (!ws) VX_FAIL(VX_EINVAL, "null workspace");
  if ((rc = check_ws(ws))) return rc;
  return mv_impl(P, np, S, dom, lo, hi, keep, ws, ws_bytes, (hipStream_t)stream, order);
}

int mean_value_exclusion(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, double* lo, double* hi,
                         uint8_t* keep, void* ws, size_t ws_bytes, void* stream) {
  return taylor_exclusion(P, np, S, dom, 1, lo, hi, keep, ws, ws_bytes, stream);
}

int taylor_inclusion_test(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, uint8_t* incl, void* ws,
                          size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_csf(S, true))) return rc;
  if ((rc = check_poly(P, np, S->k))) return rc;
  if ((rc = check_taylor_polys(np, S->k, 2))) return rc;
  if ((rc = check_dom(dom, S->k))) return rc;
  if (S->n[S->k - 1] > 0 && !incl) VX_FAIL(VX_EINVAL, "null output flags");
  if (!ws) VX_FAIL(VX_EINVAL, "null workspace");
  if ((rc = check_ws(ws))) return rc;
  return mv_impl(P, np, S, dom, nullptr, nullptr, nullptr, ws, ws_bytes, (hipStream_t)stream, 2, incl);
}

int newton_test(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, uint8_t* incl, double* kout,
                void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_csf(S, true))) return rc;
  if ((rc = check_poly(P, np, S->k))) return rc;
  if (np > S->k)
    VX_FAIL(VX_EINVAL, "the Newton test needs at most as many polynomials as variables (%d polynomials, k = %d)", np,
            S->k);
  if ((rc = check_dom(dom, S->k))) return rc;
  if (S->n[S->k - 1] > 0 && !incl) VX_FAIL(VX_EINVAL, "null output flags");
  if (!ws) VX_FAIL(VX_EINVAL, "null workspace");
  if ((rc = check_ws(ws))) return rc;
  return newton_impl(P, np, S, dom, incl, kout, ws, ws_bytes, (hipStream_t)stream);
}

int inclusion_test(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, uint8_t* incl, void* ws,
                   size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_csf(S, true))) return rc;
  if ((rc = check_poly(P, np, S->k))) return rc;
  if ((rc = check_dom(dom, S->k))) return rc;
  if (S->n[S->k - 1] > 0 && !incl) VX_FAIL(VX_EINVAL, "null output flags");
  if (!ws) VX_FAIL(VX_EINVAL, "null workspace");
  if ((rc = check_ws(ws))) return rc;
  return inclusion_impl(P, np, S, dom, incl, ws, ws_bytes, (hipStream_t)stream);
}

int variable_order_costs(const vx_poly* P, int32_t np, const vx_csf* S, int32_t norders, const int32_t* orders,
                         int64_t* counts, int64_t* steps, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_csf(S, true))) return rc;
  const int k = S->k;
  if (norders < 1 || norders > 24 || !orders) VX_FAIL(VX_EINVAL, "need 1..24 axis orders");
  for (int o = 0; o < norders; o++) {
    int seen = 0;
    for (int l = 0; l < k; l++) {
      const int a = orders[o * k + l];
      if (a < 0 || a >= k || (seen >> a) & 1) VX_FAIL(VX_EINVAL, "order %d is not a permutation of 0..%d", o, k - 1);
      seen |= 1 << a;
    }
  }
  if (steps && (rc = check_poly(P, np, k))) return rc;
  if ((int64_t)k * S->level > 62) VX_FAIL(VX_EUNSUPPORTED, "k * level = %d exceeds the 62-bit key", k * S->level);
  if (!ws) VX_FAIL(VX_EINVAL, "null workspace");
  if ((rc = check_ws(ws))) return rc;
  std::vector<int64_t> c((size_t)norders * k);
  if ((rc = order_counts_impl(S, norders, orders, c.data(), ws, ws_bytes, (hipStream_t)stream))) return rc;
  for (int o = 0; o < norders; o++) {
    vx_csf T = *S;
    for (int l = 0; l < k; l++) T.n[l] = c[(size_t)o * k + l];
    if (counts)
      for (int l = 0; l < k; l++) counts[o * k + l] = T.n[l];
    if (steps) steps[o] = theorem1_steps(P, np, &T);
  }
  return VX_OK;
}

int filter_subdivide(const vx_csf* S, const uint8_t* keep, vx_csf* kept, vx_csf* next, int64_t* d_counts, void* ws,
                     size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_csf(S, true))) return rc;
  const int k = S->k;
  if (S->n[k - 1] > 0 && !keep) VX_FAIL(VX_EINVAL, "null keep flags");
  int64_t bound[VX_KMAX] = {0, 0, 0, 0};
  if (next && (rc = next_level_bounds(S, bound))) return rc;
  for (int l = 0; l < k; l++) {
    if (kept && (kept->k != k || kept->cap[l] < S->n[l] || !kept->idx[l] || (l + 1 < k && !kept->ptr[l])))
      VX_FAIL(VX_ECAPACITY, "kept CSF: depth %d needs capacity %lld", l + 1, (long long)S->n[l]);
    if (next && (next->k != k || next->cap[l] < bound[l] || !next->idx[l] || (l + 1 < k && !next->ptr[l])))
      VX_FAIL(VX_ECAPACITY, "next CSF: depth %d needs capacity %lld", l + 1, (long long)bound[l]);
  }
  if ((rc = check_ws(ws))) return rc;
  if (kept) kept->level = S->level;
  if (next) next->level = S->level + 1;
  return filter_impl(S, keep, kept, next, d_counts, ws, ws_bytes, (hipStream_t)stream);
}

static int check_point_polys(const vx_poly* P, int np) {
  if (!P || np < 1 || np > PMAX_GRAD) VX_FAIL(VX_EINVAL, "point evaluation takes 1..%d polynomials", PMAX_GRAD);
  int rc;
  if ((rc = check_poly(P, np, P[0].k))) return rc;
  for (int p = 0; p < np; p++)
    if (P[p].c_hi && P[p].c_hi != P[p].c_lo)
      VX_FAIL(VX_EINVAL, "point evaluation needs point coefficients (c_hi == NULL)");
  return VX_OK;
}

int eval_grad(const vx_poly* P, int32_t np, const double* x, int64_t n, double* f, double* jac, const double* gbar,
              double* xbar, double* dcoef, const vx_csf* grid, const double* dom, void* ws, size_t ws_bytes,
              void* stream) {
  int rc;
  if ((rc = check_point_polys(P, np))) return rc;
  const int k = P[0].k;
  if (n < 0 || (n > 0 && (f || jac || xbar) && !x && !grid)) VX_FAIL(VX_EINVAL, "bad point list");
  if (xbar && !gbar) VX_FAIL(VX_EINVAL, "xbar needs gbar");
  if (dcoef && !gbar) VX_FAIL(VX_EINVAL, "dcoef needs gbar");
  if (dcoef && !grid) VX_FAIL(VX_EUNSUPPORTED, "coefficient gradients need the points as a CSF grid of centres");
  if (grid) {
    if ((rc = check_csf(grid, true))) return rc;
    if (grid->k != k) VX_FAIL(VX_EINVAL, "grid has k=%d, polynomials k=%d", grid->k, k);
    if (grid->n[k - 1] != n) VX_FAIL(VX_EINVAL, "grid has %lld leaves, n=%lld", (long long)grid->n[k - 1], (long long)n);
    if ((rc = check_dom(dom, k))) return rc;
  }
  if (dcoef)
    for (int p = 0; p < np; p++)
      if (P[p].degree > MAXDEG_ADJ) VX_FAIL(VX_EUNSUPPORTED, "coefficient gradient limited to degree %d", MAXDEG_ADJ);
  if ((rc = check_ws(ws))) return rc;
  return grad_impl(P, np, x, n, f, jac, gbar, xbar, dcoef, grid, dom, ws, ws_bytes, (hipStream_t)stream);
}

int csf_centres(const vx_csf* S, const double* dom, double* x, void* stream) {
  int rc;
  if ((rc = check_csf(S, true))) return rc;
  if ((rc = check_dom(dom, S->k))) return rc;
  if (S->n[S->k - 1] > 0 && !x) VX_FAIL(VX_EINVAL, "null output");
  return centres_impl(S, dom, x, (hipStream_t)stream);
}

int newton_project(const vx_poly* P, int32_t np, double* x, int64_t n, int32_t steps, double* f, void* ws,
                   size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_point_polys(P, np))) return rc;
  if (n < 0 || (n > 0 && !x) || steps < 0 || steps > 100) VX_FAIL(VX_EINVAL, "bad arguments");
  if ((rc = check_ws(ws))) return rc;
  return newton_impl(P, np, x, n, steps, f, ws, ws_bytes, (hipStream_t)stream);
}

int newton_project_grid(const vx_poly* P, int32_t np, double* x, int64_t n, int32_t steps, double* f,
                        const vx_csf* grid, const double* dom, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_point_polys(P, np))) return rc;
  if (n < 0 || (n > 0 && !x) || steps < 0 || steps > 100) VX_FAIL(VX_EINVAL, "bad arguments");
  if (!grid) VX_FAIL(VX_EINVAL, "newton_project_grid: null grid");
  const int k = P[0].k;
  if ((rc = check_csf(grid, true))) return rc;
  if (grid->k != k) VX_FAIL(VX_EINVAL, "grid has k=%d, polynomials k=%d", grid->k, k);
  if (grid->n[k - 1] != n) VX_FAIL(VX_EINVAL, "grid has %lld leaves, n=%lld", (long long)grid->n[k - 1], (long long)n);
  if ((rc = check_dom(dom, k))) return rc;
  if ((rc = check_ws(ws))) return rc;
  return newton_impl(P, np, x, n, steps, f, ws, ws_bytes, (hipStream_t)stream, grid, dom);
}

int vx_copy(void* dst, const void* src, size_t bytes, int32_t kind, void* stream) {
  if (bytes == 0) return VX_OK;
  if (!dst || !src) VX_FAIL(VX_EINVAL, "null pointer");
  hipMemcpyKind mk = kind == 0 ? hipMemcpyDeviceToHost : kind == 1 ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  VX_HIP(hipMemcpyAsync(dst, src, bytes, mk, (hipStream_t)stream));
  VX_HIP(hipStreamSynchronize((hipStream_t)stream));
  return VX_OK;
}


int run_subdivision(const vx_poly* P, int32_t np, const double* dom, int32_t depth, void* ws, size_t ws_bytes,
                    size_t* ws_needed, vx_level_stat* stats, vx_level_cb cb, void* user, void* stream) {
  return run_subdivision_ex(P, np, dom, depth, 0, ws, ws_bytes, ws_needed, stats, cb, user, stream);
}

}  // extern "C"

namespace vx {

// The level loop of Algorithm 3 in the variable order `axes` of the caller's
// polynomials (recorded in the stats; the loop itself is order-blind).
static int run_loop(const vx_poly* P, int32_t np, const double* dom, int32_t depth, int32_t flags, void* ws,
                    size_t ws_bytes, size_t* ws_needed, vx_level_stat* stats, vx_level_cb cb, void* user,
                    void* stream, int32_t axes) {
  if (!P || np < 1) VX_FAIL(VX_EINVAL, "need at least one polynomial");
  const int k = P[0].k;
  int rc;
  if (k < 1 || k > VX_KMAX) VX_FAIL(VX_EINVAL, "k=%d outside [1, %d]", k, VX_KMAX);
  if ((rc = check_poly(P, np, k))) return rc;
  if ((rc = check_dom(dom, k))) return rc;
  if (depth < 0 || depth > 28) VX_FAIL(VX_EINVAL, "depth %d outside [0, 28]", depth);
  if (!ws) VX_FAIL(VX_EINVAL, "null workspace");
  if ((rc = check_ws(ws))) return rc;
  if (flags & ~(VX_RUN_MEAN_VALUE | VX_RUN_TAYLOR2 | VX_RUN_NO_TIMES | VX_RUN_INCLUSION | VX_RUN_INCLUSION_TAYLOR |
                VX_RUN_EARLY_EXIT | VX_RUN_TAYLOR_ORDER(15) | VX_RUN_INCLUSION_FROM(255) | VX_RUN_EARLY_EXIT_FROM(63)))
    VX_FAIL(VX_EINVAL, "unknown flags 0x%x", flags);
  const int incl_mode = (flags & VX_RUN_INCLUSION) ? 1 : (flags & VX_RUN_INCLUSION_TAYLOR) ? 2 : 0;
  const int incl_from = (flags >> 16) & 255;
  if ((flags & VX_RUN_INCLUSION) && (flags & VX_RUN_INCLUSION_TAYLOR))
    VX_FAIL(VX_EINVAL, "VX_RUN_INCLUSION and VX_RUN_INCLUSION_TAYLOR are exclusive");
  // C1 of one polynomial: vertex signs (or their Taylor form); of a system
  // of 2..k polynomials: the Newton test (on the span of the gradients when
  // there are fewer polynomials than variables)
  const bool newton = incl_mode == 1 && np >= 2 && np <= k;
  if (incl_mode && np != 1 && !newton)
    VX_FAIL(VX_EINVAL, "the inclusion criterion needs one polynomial%s (np = %d, k = %d)",
            incl_mode == 1 ? " or a system of at most k" : "", np, k);
  if (incl_mode == 2 && (rc = check_taylor_polys(np, k, 2))) return rc;
  if (!incl_mode && incl_from) VX_FAIL(VX_EINVAL, "VX_RUN_INCLUSION_FROM without an inclusion flag");
  const bool times = stats && !(flags & VX_RUN_NO_TIMES);
  const int order_m = (flags >> 8) & 15;  // VX_RUN_TAYLOR_ORDER(m)
  if (((flags & VX_RUN_MEAN_VALUE) != 0) + ((flags & VX_RUN_TAYLOR2) != 0) + (order_m != 0) > 1)
    VX_FAIL(VX_EINVAL, "VX_RUN_MEAN_VALUE, VX_RUN_TAYLOR2 and VX_RUN_TAYLOR_ORDER are exclusive");
  const int order = order_m ? order_m : (flags & VX_RUN_TAYLOR2) ? 2 : (flags & VX_RUN_MEAN_VALUE) ? 1 : 0;
  const bool mv = order > 0;
  if (mv && (rc = check_taylor_order(P, np, order))) return rc;
  if ((rc = check_taylor_polys(np, k, order))) return rc;
  // Early exit (systems): polynomial p is evaluated only on the boxes that
  // polynomials 0..p-1 kept; the kept sets are those of the plain loop.
  const bool early_on = (flags & VX_RUN_EARLY_EXIT) && np > 1;
  const int early_from = (flags >> 24) & 63;
  if ((flags & VX_RUN_EARLY_EXIT) && (mv || incl_mode))
    VX_FAIL(VX_EINVAL, "VX_RUN_EARLY_EXIT does not combine with the Taylor or inclusion tests");
  if (!(flags & VX_RUN_EARLY_EXIT) && early_from) VX_FAIL(VX_EINVAL, "VX_RUN_EARLY_EXIT_FROM without VX_RUN_EARLY_EXIT");
  hipStream_t st = (hipStream_t)stream;
  // coefficient tables once for the whole run, at the start of the workspace
  // (followed by the mean-value test's derivative tables when requested)
  const size_t qbytes = (prepared_bytes(P, np) + 255) / 256 * 256 + (mv ? mv_run_workspace(P, np, order) : 0);
  if (qbytes > ws_bytes) {
    if (ws_needed) *ws_needed = qbytes + (1 << 20);
    VX_FAIL(VX_ECAPACITY, "workspace too small");
  }
  Prepared Q;
  const size_t qf = (prepared_bytes(P, np) + 255) / 256 * 256;
  if ((rc = prepare_polys(P, np, ws, qf, &Q, st))) return rc;
  void* mvh = nullptr;
  if (mv) {
    mvh = mv_run_begin(P, np, reinterpret_cast<char*>(ws) + qf, qbytes - qf, st, &rc, order);
    if (rc) return rc;
  }
  struct MvGuard {
    void* h;
    ~MvGuard() {
      if (h) mv_run_end(h);
    }
  } mv_guard{mvh};
  char* base = reinterpret_cast<char*>(ws) + qbytes;
  const size_t total = (ws_bytes - qbytes) / 256 * 256;

  // Timing events of two consecutive levels: a level's times are read once
  // the next level is queued, so reading them never idles the GPU.
  hipEvent_t evs[6] = {};
  if (times)
    for (int i = 0; i < 6; i++) VX_HIP(hipEventCreateWithFlags(&evs[i], hipEventDisableSystemFence));  // timing only
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 6; i++)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } guard{evs};
  int pending = -1;  // level whose event times are still to be read
  auto finish_times = [&]() -> int {
    if (pending < 0 || !times) return VX_OK;
    hipEvent_t* e = evs + 3 * (pending & 1);
    VX_HIP(hipEventSynchronize(e[2]));
    float ms = 0;
    VX_HIP(hipEventElapsedTime(&ms, e[0], e[1]));
    stats[pending].eval_ms = ms;
    VX_HIP(hipEventElapsedTime(&ms, e[1], e[2]));
    stats[pending].filter_ms = ms;
    pending = -1;
    return VX_OK;
  };

  // S_0 at the low end.
  int64_t cap[VX_KMAX] = {1, 1, 1, 1};
  vx_csf S;
  size_t s_bytes = csf_bytes(k, cap);
  bool s_low = true;
  if (s_bytes > total) {
    if (ws_needed) *ws_needed = s_bytes + 256;
    VX_FAIL(VX_ECAPACITY, "workspace too small");
  }
  csf_place(&S, k, 0, cap, base);
  if ((rc = init_root_impl(&S, st))) return rc;

  // Per-level counts come back through a mapped pinned host slot written by
  // the filter's last kernel: no copy launch, only the stream wait.
  CountSlot slot;
  if ((rc = take_count_slot(&slot))) return rc;
  struct SlotGuard {
    CountSlot s;
    hipStream_t st;
    bool drained = false;
    ~SlotGuard() {
      // a run that failed may have kernels in flight that still write the slot
      if (!drained) (void)hipStreamSynchronize(st);
      give_count_slot(s);
    }
  } slot_guard{slot, st};
  int64_t* counts = slot.host;
  int64_t* counts_dev = slot.dev;
  counts[2 * VX_KMAX] = 0;      // level-done flag
  counts[2 * VX_KMAX + 1] = 0;  // boxes certified by C1 at the level
  for (int level = 0; level <= depth; level++) {
    S.level = level;
    const int64_t nleaf = S.n[k - 1];
    const bool last = level == depth;
    // next CSF capacity bound
    int64_t ncap[VX_KMAX] = {0, 0, 0, 0};
    if (!last) {
      if ((rc = next_level_bounds(&S, ncap))) return rc;
      for (int l = 0; l < k; l++) ncap[l] = ncap[l] > 0 ? ncap[l] : 1;
    }
    const size_t n_bytes = last ? 0 : csf_bytes(k, ncap);
    // middle region (offsets relative to its start)
    size_t moff = 0;
    auto carve = [&](size_t bytes) {
      const size_t o = moff;
      moff += (bytes + 255) / 256 * 256;
      return o;
    };
    const size_t o_lo = carve(sizeof(double) * (size_t)np * nleaf);
    const size_t o_hi = carve(sizeof(double) * (size_t)np * nleaf);
    const size_t o_keep = carve(nleaf > 0 ? (size_t)nleaf : 1);
    // survival flags of depth k-2, recorded by the leaf when nothing changes
    // keep after it (the plain loop)
    const bool leaf_alive = k >= 2 && !mv && !(incl_mode && level >= incl_from) && !(early_on && level >= early_from);
    const size_t o_alive = leaf_alive ? carve((size_t)(S.n[k - 2] > 0 ? S.n[k - 2] : 1)) : 0;
    const size_t o_cnt = carve(sizeof(int64_t) * 2 * VX_KMAX);
    int64_t kcap[VX_KMAX] = {1, 1, 1, 1};
    for (int l = 0; l < k; l++) kcap[l] = S.n[l] > 0 ? S.n[l] : 1;
    const size_t o_k = carve(csf_bytes(k, kcap));
    const size_t o_mlo = mv ? carve(sizeof(double) * (size_t)np * nleaf) : 0;
    const size_t o_mhi = mv ? carve(sizeof(double) * (size_t)np * nleaf) : 0;
    const bool incl_on = incl_mode && level >= incl_from && nleaf > 0;
    const size_t o_incl = incl_on ? carve((size_t)nleaf) : 0;
    const size_t o_cont = incl_on ? carve((size_t)nleaf) : 0;
    const size_t o_ccnt = incl_on ? carve(sizeof(unsigned long long)) : 0;
    const size_t ews = eval_level_bytes(P, np, &S);
    const size_t fws = filter_workspace_bytes(&S);
    const size_t mws = mv ? mv_level_workspace(P, np, &S, order) : 0;
    const size_t iws = !incl_on ? 0
                       : newton         ? newton_workspace_bytes(P, np, &S)
                       : incl_mode == 1 ? inclusion_workspace_bytes(P, np, &S)
                                        : mv_workspace_bytes(P, np, &S, 2);
    size_t scratch_bytes = ews > fws ? ews : fws;
    scratch_bytes = scratch_bytes > mws ? scratch_bytes : mws;
    scratch_bytes = scratch_bytes > iws ? scratch_bytes : iws;
    // early exit: the survivors of polynomials 0..p-1 as CSFs of their own
    const bool early = early_on && level >= early_from;
    size_t o_sub[VX_MAXPOLY] = {};
    if (early) {
      for (int p = 0; p + 1 < np; p++) o_sub[p] = carve(csf_bytes(k, kcap));
      for (int p = 0; p < np; p++) {
        // node counts of the subsets are only known as bounds here
        const size_t b = eval_level_bytes_bound(P + p, 1, &S);
        scratch_bytes = scratch_bytes > b ? scratch_bytes : b;
      }
    }
    const size_t o_scr = carve(scratch_bytes);
    const size_t mid_bytes = moff;
    const size_t need = s_bytes + n_bytes + mid_bytes;
    if (need > total) {
      if (ws_needed) *ws_needed = need + qbytes + 256;
      VX_FAIL(VX_ECAPACITY, "run_subdivision: level %d needs a %zu-byte workspace (%zu given)", level,
              need + qbytes + 256, ws_bytes);
    }
    // place: S at one end, next at the other, the middle right after S's end.
    char* mid_base;
    char* next_base;
    if (s_low) {
      mid_base = base + s_bytes;
      next_base = base + total - n_bytes;
    } else {
      mid_base = base + n_bytes;
      next_base = base;
    }
    double* lo = reinterpret_cast<double*>(mid_base + o_lo);
    double* hi = reinterpret_cast<double*>(mid_base + o_hi);
    uint8_t* keep = reinterpret_cast<uint8_t*>(mid_base + o_keep);
    uint8_t* alive = leaf_alive ? reinterpret_cast<uint8_t*>(mid_base + o_alive) : nullptr;
    int64_t* d_counts = counts_dev;
    (void)o_cnt;
    vx_csf K;
    csf_place(&K, k, level, kcap, mid_base + o_k);
    char* scratch = mid_base + o_scr;
    vx_csf N;
    if (!last) csf_place(&N, k, level + 1, ncap, next_base);

    hipEvent_t* ev = evs + 3 * (level & 1);
    if (times) VX_HIP(hipEventRecord(ev[0], st));
    // the set the last evaluated polynomial ran on, keep its flags
    vx_csf cur = S;
    int64_t steps = 0;
    if (!early) {
      if ((rc = eval_level_prepared(Q, &S, dom, lo, hi, keep, scratch, scratch_bytes, st, P, 0, nullptr, alive)))
        return rc;
      steps = theorem1_steps(P, np, &S);
    }
    for (int p = 0; early; p++) {
      const Prepared Qp = prepared_subset(Q, &p, 1);
      if ((rc = eval_level_prepared(Qp, &cur, dom, lo + (size_t)p * nleaf, hi + (size_t)p * nleaf, keep, scratch,
                                    scratch_bytes, st, P + p)))
        return rc;
      steps += theorem1_steps(P + p, 1, &cur);
      if (p + 1 == np) break;
      // the survivors of polynomial p; its own counts come back through the
      // mapped slot under a flag value of its own (negative: never a level's)
      vx_csf Kp;
      csf_place(&Kp, k, level, kcap, mid_base + o_sub[p]);
      const int64_t fv = -((int64_t)(level + 1) * VX_MAXPOLY + p + 1);
      if ((rc = filter_impl(&cur, keep, &Kp, nullptr, d_counts, scratch, scratch_bytes, st, counts_dev + 2 * VX_KMAX,
                            fv)))
        return rc;
      if ((rc = wait_for_flag(counts + 2 * VX_KMAX, fv, st))) return rc;
      for (int l = 0; l < k; l++) Kp.n[l] = counts[l];
      // nothing left: the final filter runs on cur with these all-zero flags
      if (Kp.n[k - 1] == 0) break;
      cur = Kp;
    }
    if (mv && nleaf > 0) {
      double* mlo = reinterpret_cast<double*>(mid_base + o_mlo);
      double* mhi = reinterpret_cast<double*>(mid_base + o_mhi);
      if ((rc = mv_run_level(mvh, P, np, &S, dom, mlo, mhi, keep, scratch, scratch_bytes, st))) return rc;
    }
    // C1 on the level's boxes: certified boxes leave, the others continue
    const uint8_t* cont = keep;
    if (incl_on) {
      uint8_t* incl = reinterpret_cast<uint8_t*>(mid_base + o_incl);
      uint8_t* contw = reinterpret_cast<uint8_t*>(mid_base + o_cont);
      unsigned long long* ccnt = reinterpret_cast<unsigned long long*>(mid_base + o_ccnt);
      if (newton) rc = newton_impl(P, np, &S, dom, incl, nullptr, scratch, scratch_bytes, st);
      else if (incl_mode == 1) rc = inclusion_impl(P, np, &S, dom, incl, scratch, scratch_bytes, st);
      else rc = mv_impl(P, np, &S, dom, nullptr, nullptr, nullptr, scratch, scratch_bytes, st, 2, incl);
      if (rc) return rc;
      VX_HIP(hipMemsetAsync(ccnt, 0, sizeof *ccnt, st));
      hipLaunchKernelGGL(k_mark_certified, dim3((unsigned)((nleaf + 255) / 256)), dim3(256), 0, st, nleaf, keep,
                         (const uint8_t*)incl, contw, ccnt);
      VX_CHECK_LAUNCH("k_mark_certified");
      hipLaunchKernelGGL(k_put_count, dim3(1), dim3(64), 0, st, (const unsigned long long*)ccnt,
                         counts_dev + 2 * VX_KMAX + 1);
      VX_CHECK_LAUNCH("k_put_count");
      cont = contw;
    }
    if (times) VX_HIP(hipEventRecord(ev[1], st));
    // the filter publishes its counts (and the flag) as soon as they are known
    if ((rc = filter_impl(&cur, cont, &K, last ? nullptr : &N, d_counts, scratch, scratch_bytes, st,
                          counts_dev + 2 * VX_KMAX, (int64_t)level + 1, alive)))
      return rc;
    if (times) VX_HIP(hipEventRecord(ev[2], st));
    if ((rc = finish_times())) return rc;  // the previous level's times
    if ((rc = wait_for_flag(counts + 2 * VX_KMAX, (int64_t)level + 1, st))) return rc;
    for (int l = 0; l < k; l++) K.n[l] = counts[l];
    if (stats) {
      vx_level_stat& r = stats[level];
      memset(&r, 0, sizeof r);
      r.level = level;
      r.axes = axes;
      for (int l = 0; l < k; l++) {
        r.n[l] = S.n[l];
        r.kept[l] = K.n[l];
      }
      r.steps = steps;
      r.certified = incl_on ? counts[2 * VX_KMAX + 1] : 0;
      pending = level;
    }
    if (cb) {
      // the callback reads this level's buffers: let the filter finish first
      if ((rc = finish_times())) return rc;
      VX_HIP(hipStreamSynchronize(st));
      // early exit: the enclosures and flags cover subsets of S, none is passed
      if (cb(user, level, &S, early ? nullptr : lo, early ? nullptr : hi, early ? nullptr : keep, &K)) break;
    }
    if (last) break;
    // next becomes S (at the other end)
    for (int l = 0; l < k; l++) N.n[l] = counts[k + l];
    S = N;
    for (int l = 0; l < k; l++) S.cap[l] = ncap[l];
    s_bytes = n_bytes;
    s_low = !s_low;
    if (S.n[k - 1] == 0) {
      // nothing left: record empty levels
      for (int lv = level + 1; lv <= depth; lv++) {
        if (stats) {
          memset(&stats[lv], 0, sizeof stats[lv]);
          stats[lv].level = lv;
          stats[lv].axes = axes;
        }
      }
      break;
    }
  }
  if ((rc = finish_times())) return rc;
  // the last filter may still be writing after it published its counts
  VX_HIP(hipStreamSynchronize(st));
  slot_guard.drained = true;
  return VX_OK;
}

// Transposed coefficient cube: new variable l = old variable order[l], i.e.
// out[e'] = in[e] with e[order[l]] = e'[l] (one thread per entry).
__global__ void k_transpose_cube(int k, int side, const double* __restrict__ in, double* __restrict__ out,
                                 int4 order) {
  int64_t total = 1;
  for (int i = 0; i < k; i++) total *= side;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= total) return;
  const int ord[4] = {order.x, order.y, order.z, order.w};
  int e[VX_KMAX] = {0, 0, 0, 0};
  int64_t q = f;
  for (int l = k - 1; l >= 0; l--) {  // e' of this output entry, placed at the old axes
    e[ord[l]] = (int)(q % side);
    q /= side;
  }
  int64_t src = 0;
  for (int i = 0; i < k; i++) src = src * side + e[i];
  out[f] = in[src];
}

static int32_t pack_axes(const int* a, int k) {
  int32_t v = 0;
  for (int l = 0; l < k; l++) v |= a[l] << (4 * l);
  return v;
}

constexpr int AUTO_ORDER_DEFAULT_LEVEL = 6;

struct ProbeState {
  int level;
  int norders;
  const int32_t* orders;
  int64_t* counts;
  void* scratch;
  size_t scratch_bytes;
  hipStream_t st;
  int rc;
  bool done;
};

// At the probe level: node counts of the kept set under every order.
static int probe_cb(void* user, int32_t level, const vx_csf* S, const double*, const double*, const uint8_t*,
                    const vx_csf* K) {
  (void)S;
  ProbeState* ps = reinterpret_cast<ProbeState*>(user);
  if (level != ps->level) return 0;
  ps->rc = order_counts_impl(K, ps->norders, ps->orders, ps->counts, ps->scratch, ps->scratch_bytes, ps->st);
  ps->done = true;
  return 1;
}

// Algorithm 3 in the order of the variables that Theorem 1 finds cheapest on
// the kept set of a probe level (its children's node counts are 2^(l+1)
// times the kept set's, in every order).
static int run_auto_order(const vx_poly* P, int32_t np, const double* dom, int32_t depth, int32_t flags, void* ws,
                          size_t ws_bytes, size_t* ws_needed, vx_level_stat* stats, vx_level_cb cb, void* user,
                          hipStream_t st) {
  if (!P || np < 1) VX_FAIL(VX_EINVAL, "need at least one polynomial");
  const int k = P[0].k;
  int rc;
  if (k < 1 || k > VX_KMAX) VX_FAIL(VX_EINVAL, "k=%d outside [1, %d]", k, VX_KMAX);
  if ((rc = check_poly(P, np, k))) return rc;
  if ((rc = check_dom(dom, k))) return rc;
  if (depth < 0 || depth > 28) VX_FAIL(VX_EINVAL, "depth %d outside [0, 28]", depth);
  if (!ws) VX_FAIL(VX_EINVAL, "null workspace");
  if ((rc = check_ws(ws))) return rc;
  int probe = (flags >> 12) & 15;
  if (probe == 0) probe = AUTO_ORDER_DEFAULT_LEVEL;
  if (probe > depth) probe = depth;
  const int32_t rest = flags & ~(VX_RUN_AUTO_ORDER | VX_RUN_AUTO_ORDER_AT(15));
  // every permutation of the axes, lexicographic (the given order first)
  std::vector<int32_t> orders;
  int perm[VX_KMAX] = {0, 1, 2, 3};
  int norders = 0;
  do {
    for (int l = 0; l < k; l++) orders.push_back(perm[l]);
    norders++;
  } while (std::next_permutation(perm, perm + k));
  // workspace: transposed cubes | (probe run | order scratch at the tail) then the main run
  size_t cubes = 0;
  for (int p = 0; p < np; p++) {
    int64_t c = 1;
    for (int i = 0; i < k; i++) c *= P[p].side;
    cubes += ((size_t)c * 8 + 255) / 256 * 256 * (P[p].c_hi ? 2 : 1);
  }
  vx_csf bound;
  memset(&bound, 0, sizeof bound);
  bound.k = k;
  bound.level = probe;
  for (int l = 0; l < k; l++) {
    const int sh = (l + 1) * probe;
    bound.n[l] = sh >= 26 ? ((int64_t)1 << 26) : ((int64_t)1 << sh);
  }
  const size_t oscratch = (order_workspace_bytes(&bound) + 255) / 256 * 256;
  if (cubes + oscratch + (1 << 20) > ws_bytes) {
    if (ws_needed) *ws_needed = cubes + oscratch + ((size_t)64 << 20);
    VX_FAIL(VX_ECAPACITY, "run_subdivision: workspace too small for the variable-order probe");
  }
  char* base = reinterpret_cast<char*>(ws);
  char* run_ws = base + cubes;
  const size_t run_bytes = (ws_bytes - cubes) / 256 * 256;
  std::vector<int64_t> counts((size_t)norders * k, 0);
  ProbeState ps{probe, norders, orders.data(), counts.data(), run_ws + run_bytes - oscratch, oscratch, st, VX_OK,
                false};
  size_t need = 0;
  rc = run_loop(P, np, dom, probe, VX_RUN_NO_TIMES, run_ws, run_bytes - oscratch, &need, nullptr, probe_cb, &ps, st,
                pack_axes(perm, k));
  if (rc) {
    if (rc == VX_ECAPACITY && ws_needed) *ws_needed = need + cubes + oscratch;
    return rc;
  }
  if (ps.rc) return ps.rc;
  // Theorem 1 on the children of the probe's kept set, order by order
  int best = 0;
  int64_t best_steps = -1;
  if (ps.done) {
    for (int o = 0; o < norders; o++) {
      vx_csf T;
      memset(&T, 0, sizeof T);
      T.k = k;
      for (int l = 0; l < k; l++) T.n[l] = counts[(size_t)o * k + l] << (l + 1);
      const int64_t st1 = theorem1_steps(P, np, &T);
      if (best_steps < 0 || st1 < best_steps) {
        best_steps = st1;
        best = o;
      }
    }
  }
  const int32_t* ord = orders.data() + (size_t)best * k;
  std::vector<vx_poly> Q(P, P + np);
  std::vector<double> domq(2 * k);
  char* at = base;
  int4 o4 = make_int4(0, 0, 0, 0);
  int* o4p = reinterpret_cast<int*>(&o4);
  for (int l = 0; l < k; l++) o4p[l] = ord[l];
  for (int l = 0; l < k; l++) {
    domq[2 * l] = dom[2 * ord[l]];
    domq[2 * l + 1] = dom[2 * ord[l] + 1];
  }
  for (int p = 0; p < np; p++) {
    int64_t c = 1;
    for (int i = 0; i < k; i++) c *= P[p].side;
    const unsigned g = (unsigned)((c + 255) / 256);
    double* lo = reinterpret_cast<double*>(at);
    at += ((size_t)c * 8 + 255) / 256 * 256;
    hipLaunchKernelGGL(k_transpose_cube, dim3(g), dim3(256), 0, st, k, P[p].side, P[p].c_lo, lo, o4);
    VX_CHECK_LAUNCH("k_transpose_cube");
    Q[p].c_lo = lo;
    if (P[p].c_hi) {
      double* hi = reinterpret_cast<double*>(at);
      at += ((size_t)c * 8 + 255) / 256 * 256;
      hipLaunchKernelGGL(k_transpose_cube, dim3(g), dim3(256), 0, st, k, P[p].side, P[p].c_hi, hi, o4);
      VX_CHECK_LAUNCH("k_transpose_cube");
      Q[p].c_hi = hi;
    }
  }
  int ordi[VX_KMAX] = {0, 0, 0, 0};
  for (int l = 0; l < k; l++) ordi[l] = ord[l];
  need = 0;
  rc = run_loop(Q.data(), np, domq.data(), depth, rest, run_ws, run_bytes, &need, stats, cb, user, st,
                pack_axes(ordi, k));
  if (rc == VX_ECAPACITY && ws_needed) *ws_needed = need + cubes;
  return rc;
}

}  // namespace vx

extern "C" {

int run_subdivision_ex(const vx_poly* P, int32_t np, const double* dom, int32_t depth, int32_t flags, void* ws,
                       size_t ws_bytes, size_t* ws_needed, vx_level_stat* stats, vx_level_cb cb, void* user,
                       void* stream) {
  if (flags & VX_RUN_AUTO_ORDER)
    return run_auto_order(P, np, dom, depth, flags, ws, ws_bytes, ws_needed, stats, cb, user, (hipStream_t)stream);
  if (flags & VX_RUN_AUTO_ORDER_AT(15)) VX_FAIL(VX_EINVAL, "VX_RUN_AUTO_ORDER_AT without VX_RUN_AUTO_ORDER");
  const int identity[VX_KMAX] = {0, 1, 2, 3};
  return run_loop(P, np, dom, depth, flags, ws, ws_bytes, ws_needed, stats, cb, user, stream,
                  pack_axes(identity, P && np > 0 && P[0].k >= 1 && P[0].k <= VX_KMAX ? P[0].k : 1));
}

static int check_batch(const vx_poly* P, int32_t nsys, int32_t depth, const int64_t* cap) {
  if (!P || nsys < 1 || nsys > VX_MAXPOLY) VX_FAIL(VX_EINVAL, "batch: 1..%d systems", VX_MAXPOLY);
  if (P[0].k != 3) VX_FAIL(VX_EUNSUPPORTED, "batch: implemented for k = 3 (got k = %d)", P[0].k);
  int rc;
  if ((rc = check_poly(P, nsys, 3))) return rc;
  if (depth < 0 || depth > 28) VX_FAIL(VX_EINVAL, "batch: depth %d outside [0, 28]", depth);
  if (!cap) VX_FAIL(VX_EINVAL, "batch: null capacities");
  if (cap[0] < nsys) VX_FAIL(VX_EINVAL, "batch: cap[0] = %lld < %d systems", (long long)cap[0], nsys);
  for (int l = 0; l <= 3; l++)
    if (cap[l] < 1 || cap[l] >= ((int64_t)1 << 31) - 2)
      VX_FAIL(VX_EINVAL, "batch: cap[%d] = %lld outside [1, 2^31 - 3]", l, (long long)cap[l]);
  return VX_OK;
}

static int check_tune(const vx_batch_tune* t, int n) {
  for (int i = 0; i < n; i++) {
    const int r = t[i].r1;
    if (r != 1 && r != 2 && r != 4 && r != 8) VX_FAIL(VX_EINVAL, "batch tune %d: r1 = %d not in {1, 2, 4, 8}", i, r);
    if (t[i].groups < 1 || t[i].groups > 64) VX_FAIL(VX_EINVAL, "batch tune %d: groups = %d", i, t[i].groups);
    if (t[i].grid < 64 || t[i].grid > 65536) VX_FAIL(VX_EINVAL, "batch tune %d: grid = %d", i, t[i].grid);
  }
  return VX_OK;
}

size_t vx_batch_workspace_bytes(const vx_poly* P, int32_t nsys, int32_t depth, const int64_t* cap) {
  if (check_batch(P, nsys, depth, cap)) return 0;
  return batch_workspace_bytes(P, nsys, depth, cap);
}

int vx_batch_create(const vx_poly* P, int32_t nsys, const double* dom, int32_t depth, const int64_t* cap,
                    const vx_batch_tune* tune, int32_t flags, void* ws, size_t ws_bytes, void* stream,
                    vx_batch** out) {
  int rc;
  if (!out) VX_FAIL(VX_EINVAL, "batch: null handle output");
  *out = nullptr;
  if ((rc = check_batch(P, nsys, depth, cap))) return rc;
  if ((rc = check_dom(dom, 3))) return rc;
  if (tune && (rc = check_tune(tune, depth + 1))) return rc;
  if (flags & ~VX_BATCH_GRAPH) VX_FAIL(VX_EINVAL, "batch: unknown flags 0x%x", flags);
  if (!ws) VX_FAIL(VX_EINVAL, "batch: null workspace");
  if (reinterpret_cast<uintptr_t>(ws) & 255) VX_FAIL(VX_EINVAL, "batch: workspace not 256-byte aligned");
  return batch_create_impl(P, nsys, dom, depth, cap, tune, flags, ws, ws_bytes, (hipStream_t)stream, out);
}

int vx_batch_run(vx_batch* b, void* stream) {
  if (!b) VX_FAIL(VX_EINVAL, "batch: null handle");
  return batch_run_impl(b, (hipStream_t)stream);
}

int vx_batch_result(vx_batch* b, vx_batch_stat* stats, int64_t* need, vx_csf* last, double* lo, double* hi, uint8_t* keep,
                    vx_csf* kept, void* stream) {
  if (!b) VX_FAIL(VX_EINVAL, "batch: null handle");
  return batch_result_impl(b, stats, need, last, lo, hi, keep, kept, (hipStream_t)stream);
}

int vx_batch_autotune(vx_batch* b, const vx_batch_tune* cand, int32_t ncand, int32_t reps, vx_batch_tune* chosen,
                      float* level_ms, void* stream) {
  int rc;
  if (!b) VX_FAIL(VX_EINVAL, "batch: null handle");
  if (!cand || ncand < 1 || ncand > 256 || reps < 1 || reps > 16) VX_FAIL(VX_EINVAL, "batch autotune: bad candidates");
  if ((rc = check_tune(cand, ncand))) return rc;
  return batch_autotune_impl(b, cand, ncand, reps, chosen, level_ms, (hipStream_t)stream);
}

void vx_batch_destroy(vx_batch* b) { batch_destroy_impl(b); }

int csf_build(int32_t k, int32_t level, const int32_t* boxes, int64_t n, vx_csf* out, void* ws, size_t ws_bytes,
              void* stream) {
  if (k < 1 || k > VX_KMAX) VX_FAIL(VX_EINVAL, "k=%d outside [1, %d]", k, VX_KMAX);
  if (level < 0 || level > 29) VX_FAIL(VX_EINVAL, "level %d outside [0, 29]", level);
  if (n < 0 || (n > 0 && !boxes)) VX_FAIL(VX_EINVAL, "bad box list");
  if (!out || out->k != k) VX_FAIL(VX_EINVAL, "output CSF must have k=%d", k);
  if (n >= ((int64_t)1 << 31) - 1) VX_FAIL(VX_EOVERFLOW, "too many boxes");
  for (int l = 0; l < k; l++)
    if (out->cap[l] < n || !out->idx[l] || (l + 1 < k && !out->ptr[l]))
      VX_FAIL(VX_ECAPACITY, "output CSF depth %d needs capacity %lld", l + 1, (long long)n);
  int rc;
  if ((rc = check_ws(ws))) return rc;
  out->level = level;
  return build_impl(k, level, boxes, n, out, nullptr, ws, ws_bytes, (hipStream_t)stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Per-kernel event timing.
// ---------------------------------------------------------------------------
#include <mutex>

#include "profile.hpp"

namespace vx {
namespace {
struct ProfRec {
  const char* name;
  double units;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
// Events are kept and reused across profiling sessions: creating two events
// per timed launch would add host time between launches.
std::vector<hipEvent_t> g_ev_pool;
size_t g_ev_used = 0;
char g_prof_only[32] = "";  // record only regions of this name ("" = all)

hipEvent_t pool_event() {
  if (g_ev_used == g_ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;  // timing only
    g_ev_pool.push_back(e);
  }
  return g_ev_pool[g_ev_used++];
}
}  // namespace

bool profiling() { return g_prof_on && !g_prof_suppressed; }

int prof_start(const char* name, double units, hipStream_t st) {
  if (!g_prof_on || g_prof_suppressed) return -1;
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (g_prof_only[0] && strncmp(g_prof_only, name, sizeof g_prof_only) != 0) return -1;
  ProfRec r{name, units, pool_event(), pool_event()};
  if (!r.a || !r.b || hipEventRecord(r.a, st) != hipSuccess) return -1;
  g_prof.push_back(r);
  return (int)g_prof.size() - 1;
}

void prof_stop(int slot, hipStream_t st) {
  if (slot < 0) return;
  hipEvent_t b;
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (slot >= (int)g_prof.size()) return;
    b = g_prof[slot].b;
  }
  (void)hipEventRecord(b, st);
}

}  // namespace vx

extern "C" {

int vx_profile_select(const char* name) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (name && strlen(name) >= sizeof g_prof_only) VX_FAIL(VX_EINVAL, "profile: kernel name too long");
  snprintf(g_prof_only, sizeof g_prof_only, "%s", name ? name : "");
  return VX_OK;
}

int vx_profile_begin(void) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (auto& r : g_prof) {  // a session that was never ended: wait for its events before reuse
    (void)hipEventSynchronize(r.a);
    (void)hipEventSynchronize(r.b);
  }
  g_prof.clear();
  g_ev_used = 0;
  g_prof_on = true;
  return VX_OK;
}

int vx_profile_end(vx_kernel_stat* out, int32_t max, int32_t* count) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_on = false;
  std::vector<vx_kernel_stat> acc;
  int rc = VX_OK;
  for (auto& r : g_prof) {
    float ms = 0;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      set_error("profile: event timing failed");
      rc = VX_EHIP;
    }
    size_t j = 0;
    while (j < acc.size() && strncmp(acc[j].name, r.name, sizeof acc[j].name) != 0) j++;
    if (j == acc.size()) {
      vx_kernel_stat s;
      memset(&s, 0, sizeof s);
      snprintf(s.name, sizeof s.name, "%s", r.name);
      acc.push_back(s);
    }
    acc[j].launches++;
    acc[j].ms += ms;
    acc[j].units += r.units;
  }
  g_prof.clear();
  g_ev_used = 0;
  if (count) *count = (int32_t)acc.size();
  for (size_t j = 0; j < acc.size() && (int32_t)j < max; j++) out[j] = acc[j];
  return rc;
}

}  // extern "C"

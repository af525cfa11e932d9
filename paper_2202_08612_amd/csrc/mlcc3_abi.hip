// C-ABI of libmlcc3: validation, workspace, and the orchestration of the
// triples path on one stream.  See include/mlcc3.h for the contract.
//
// Data flow of one call (all on the caller's stream):
//   ground prep   Lhat = (1-T)L(1+T); integral blocks ghat = sum_J Lhat Lhat (MFMA GEMMs)
//   W             d-contraction for every ordered occupied triple (MFMA GEMM, K = N_V or 2 N_V)
//                 minus the occupied (N_O-sized) term (MFMA GEMM, accumulating)
//   permute       X~ = contravariant of -(eps - omega)^{-1} P W, written for every ordering
//   back          Y^{aD}_{ij} (K = n_o n_v^2), Y^{ab}_{iL} (K = n_o^2 n_v) GEMMs, small terms
//   out           Delta^{-1}, pair symmetrisation, contravariant -> covariant, block gather
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>
#include <array>

#include "../../include/mlcc3.h"
#include "mlcc3_internal.h"
#include "tile_gemm.h"
#include "dcontract_mixed.h"
#include "triples_kernels.h"

using namespace mlcc3;

// Fixed device scratch of mlcc3_ground_residual_noalloc (one copy per device, held until the
// process ends).  In host code `scratch` only names the symbol: its device address on the current
// device comes from hipGetSymbolAddress, taken once per device (scratch_address); kernels only
// ever receive that address.
constexpr size_t kScratchBytes = (size_t)128 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_last_error;

struct Status {
  int code;
  std::string msg;
};

#define HIPCHK(x)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess) throw Status{MLCC3_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define HIPRT(x)            \
  do {                      \
    if (!g_dry) HIPCHK(x);  \
  } while (0)

// Host-side bounds self-check: every GEMM operand range is checked against the extents of
// the buffers registered for the current call (workspace buffers and the caller's arrays).
struct Extent {
  uintptr_t lo, hi;
  std::string name;
};
thread_local std::vector<Extent> t_ext;

thread_local mlcc3_ws t_ws = nullptr;   // workspace of the running call (timing, split-K scratch)
// test hook MLCC3_TEST_FAIL_ALLOC=<n>: the n-th new workspace allocation of a call fails (ENOMEM)
thread_local long long t_alloc_fail_at = 0, t_alloc_count = 0;
thread_local hipStream_t t_stream = nullptr;
thread_local int t_prec = MLCC3_FP64;   // arithmetic of the d-contractions of the running call
// the contravariant ordered-triple blocks (tau~, R~, L~) of the running call hold float elements
// (the reduced-precision forms of the ground residual and the transforms; never in the densities)
thread_local bool t_xf32 = false;
// occupied slab of the running call: the ordered-triple buffers hold the triples with first
// index t_p0 <= p < t_p0 + t_np at [p - t_p0][q][r]; t_np = 0: all of them (no slab)
thread_local int t_p0 = 0, t_np = 0;
// the unique triples with an index in the slab (device list of t_ntl indices), NULL: all
thread_local const int *t_tl = nullptr;
thread_local int t_ntl = 0;
// core-valence separation of the running call: on/off, active core orbitals as bits, device flags [N_O]
thread_local int t_cvs = 0;
thread_local unsigned long long t_cvs_bits = 0;
thread_local const unsigned char *t_cvs_dev = nullptr;

// MLCC3_LOG=1: one line per compute call on stderr with the device time of its phases, from HIP
// events recorded on the call's stream at the end of each phase (the call then waits for its
// stream before returning)
struct CallLog {
  bool on = false;
  std::string what;
  hipStream_t s = nullptr;
  std::vector<std::pair<std::string, hipEvent_t>> ev;
};
thread_local CallLog t_log;

void log_phase(const char *name) {
  if (!t_log.on || t_log.what.empty() || g_dry) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  if (hipEventRecord(e, t_log.s) != hipSuccess) {
    (void)hipEventDestroy(e);
    return;
  }
  t_log.ev.push_back({name, e});
}

void log_begin(const char *call, hipStream_t s, int no, int nv, int NO, int NV, int nc, int nvec, int prec) {
  if (!t_log.on) return;
  char b[256];
  std::snprintf(b, sizeof b, "%s n_o=%d n_v=%d N_O=%d N_V=%d rank=%d nvec=%d precision=%d", call, no, nv, NO, NV, nc,
                nvec, prec);
  t_log.what = b;
  t_log.s = s;
  log_phase("start");
}

void log_end(int rc) {
  if (!t_log.on || t_log.what.empty()) return;
  std::string line = "mlcc3: " + t_log.what + " status=" + std::to_string(rc);
  if (g_dry) line += " (dry run)";
  if (rc == MLCC3_OK && t_log.ev.size() > 0) {
    log_phase("other");
    if (hipEventSynchronize(t_log.ev.back().second) == hipSuccess) {
      float tot = 0.0f;
      char b[96];
      for (size_t i = 1; i < t_log.ev.size(); i++) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, t_log.ev[i - 1].second, t_log.ev[i].second);
        tot += ms;
        std::snprintf(b, sizeof b, " | %s %.3f", t_log.ev[i].first.c_str(), ms);
        line += b;
      }
      std::snprintf(b, sizeof b, " | total %.3f ms", tot);
      line += b;
    }
  }
  std::fprintf(stderr, "%s\n", line.c_str());
  std::fflush(stderr);
  for (auto &e : t_log.ev) (void)hipEventDestroy(e.second);
  t_log.ev.clear();
  t_log.what.clear();
}

void reg(const void *p, long long count, const char *name) {
  if (!p || count <= 0) return;
  t_ext.push_back({(uintptr_t)p, (uintptr_t)p + (uintptr_t)count * sizeof(double), name});
}

}  // namespace

struct mlcc3_ws_s {
  int device = 0;
  std::map<std::string, std::pair<void *, size_t>> bufs;
  long long total = 0;
  bool prepared = false;
  mlcc3_ground key{};
  unsigned long long fingerprint = 0;  // content fingerprint of the prepared ground-state inputs
  int nu = 0;
  uintptr_t fake_next = (uintptr_t)1 << 44;  // dry-run address space
  // optional per-phase timing (HIP events on the call's stream)
  bool timing = false;
  struct Mark {
    int phase;
    double flops;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  mlcc3_tuning tune{};  // launch-shape choices (0 = default)
  // arena mode (mlcc3_ground_residual_noalloc): buffers are carved from one preallocated range
  // [arena_base, arena_base + arena_cap) and never allocated or freed
  bool arena = false;
  uintptr_t arena_base = 0;
  size_t arena_cap = 0, arena_used = 0;
  bool gle = false;     // "gLE" (left-transform integral block) formed for the prepared ground
  // what the tau~ blocks ("XT", and "Xtau" when xtau) were last formed for (opts.reuse_tau)
  struct TauKey {
    bool valid = false, xtau = false;
    long long tb = 0, te = 0;
    int prec = 0, cvs = 0, xf32 = 0;
    unsigned long long core = 0;
  } tau;
};

namespace {

// launch-shape choices of the running call's workspace (all zero = defaults)
const mlcc3_tuning &tune() {
  static const mlcc3_tuning z{};
  return t_ws ? t_ws->tune : z;
}

double *buf(mlcc3_ws ws, const std::string &name, size_t count, hipStream_t s) {
  auto &b = ws->bufs[name];
  size_t bytes = std::max<size_t>(count * sizeof(double), 256);
  if (b.second >= bytes) {
    reg(b.first, (long long)(b.second / sizeof(double)), "ws");
    return (double *)b.first;
  }
  if (t_alloc_fail_at > 0 && !ws->arena && ++t_alloc_count == t_alloc_fail_at)
    throw Status{MLCC3_ENOMEM, "injected allocation failure (MLCC3_TEST_FAIL_ALLOC) at buffer '" + name + "'"};
  if (ws->arena) {  // a new 256-byte aligned range of the arena (a smaller earlier one is abandoned)
    const size_t off = (ws->arena_used + 255) & ~(size_t)255;
    if (off > ws->arena_cap || bytes > ws->arena_cap - off)
      throw Status{MLCC3_EINVAL, "scratch exhausted at buffer '" + name + "'"};
    b = {(void *)(ws->arena_base + off), bytes};
    ws->arena_used = off + bytes;
    ws->total += bytes;
    reg(b.first, (long long)(bytes / sizeof(double)), "ws");
    return (double *)b.first;
  }
  if (g_dry) {
    b = {(void *)ws->fake_next, bytes};
    ws->fake_next += (bytes + 4095) & ~(uintptr_t)4095;
    ws->total += bytes;
    reg(b.first, (long long)(bytes / sizeof(double)), "ws");
    return (double *)b.first;
  }
  if (b.first) {
    HIPRT(hipStreamSynchronize(s));
    HIPRT(hipFree(b.first));
    ws->total -= b.second;
    b = {nullptr, 0};
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Status{MLCC3_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes for '" + name + "' failed"};
  }
  b = {p, bytes};
  ws->total += bytes;
  reg(p, (long long)(bytes / sizeof(double)), "ws");
  return (double *)p;
}

struct Dims {
  int no, nv, NO, NV, nc;
  long long nv2, nv3, nord;
};

Dims dims_of(const mlcc3_ground *g) {
  Dims d{g->n_o, g->n_v, g->N_O, g->N_V, g->n_chol, 0, 0, 0};
  d.nv2 = (long long)d.nv * d.nv;
  d.nv3 = d.nv2 * d.nv;
  d.nord = (long long)d.no * d.no * d.no;
  return d;
}

void check(bool ok, const char *what) {
  if (!ok) throw Status{MLCC3_EINVAL, what};
}

void validate_ground(const mlcc3_ground *g) {
  check(g != nullptr, "ground is NULL");
  check(g->n_chol >= 1, "n_chol must be >= 1");
  check(g->N_O >= 1 && g->N_V >= 1, "N_O and N_V must be >= 1");
  check(g->n_o >= 0 && g->n_o <= g->N_O, "need 0 <= n_o <= N_O");
  check(g->n_v >= 0 && g->n_v <= g->N_V, "need 0 <= n_v <= N_V");
  const bool act = g->n_o > 0 && g->n_v > 0;  // the t2 blocks are empty otherwise
  check(g->eps_o && g->eps_v && g->L_OO && g->L_OV && g->t1, "NULL pointer in the ground-state inputs");
  check(!act || (g->t2_vVoo && g->t2_vvoO), "NULL t2 block");
  check(g->n_v == 0 || g->L_vV, "L_vV is NULL");
  check((long long)g->n_o * g->n_o * g->n_o * g->n_v * g->n_v * g->n_v < (1LL << 40), "active space too large");
}

void validate_vecs(const mlcc3_ground *g, int nvec, const double *omega, const mlcc3_vec *v, const mlcc3_out *o) {
  check(nvec >= 1, "nvec must be >= 1");
  check(omega && v && o, "NULL omega / vector / output array");
  const bool act = g->n_o > 0 && g->n_v > 0;
  for (int m = 0; m < nvec; m++) {
    check(v[m].x1 && (!act || (v[m].x2_vVoo && v[m].x2_vvoO)), "NULL pointer in an input vector");
    check(o[m].x1 && (!act || (o[m].x2_vVoo && o[m].x2_vvoO)), "NULL pointer in an output vector");
    check(std::isfinite(omega[m]), "omega must be finite");
  }
}

void validate_out(const mlcc3_ground *g, const mlcc3_out *o) {
  const bool act = g->n_o > 0 && g->n_v > 0;
  check(o && o->x1 && (!act || (o->x2_vVoo && o->x2_vvoO)), "NULL output pointer");
}

struct Range {
  long long tb, te;
};

Range range_of(const mlcc3_opts &o, long long nt) {
  long long tb = o.triple_begin, te = o.triple_end;
  if (te < 0 || te > nt) te = nt;
  check(tb >= 0 && tb <= te, "need 0 <= triple_begin <= triple_end");
  return {tb, te};
}

// minimal |eps^{abc}_{ijk} - omega| over active triples with distinct occupied indices
// not all equal (the i=j=k blocks never enter)
void guard_check(const mlcc3_ground *g, const double *omega, int nvec, double guard, hipStream_t s) {
  if (!(guard > 0.0) || g->n_o < 2 || g->n_v < 1 || g_dry) return;
  std::vector<double> eo(g->n_o), ev(g->n_v);
  HIPCHK(hipMemcpyAsync(eo.data(), g->eps_o, sizeof(double) * g->n_o, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(ev.data(), g->eps_v, sizeof(double) * g->n_v, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<double> vs;
  vs.reserve((size_t)g->n_v * g->n_v * g->n_v);
  for (int a = 0; a < g->n_v; a++)
    for (int b = 0; b <= a; b++)
      for (int c = 0; c <= b; c++) vs.push_back(ev[a] + ev[b] + ev[c]);
  std::sort(vs.begin(), vs.end());
  for (int i = 0; i < g->n_o; i++)
    for (int j = 0; j <= i; j++)
      for (int k = 0; k <= j; k++) {
        if (i == j && j == k) continue;
        const double e = eo[i] + eo[j] + eo[k];
        for (int m = 0; m < nvec; m++) {
          const double target = e + omega[m];
          auto it = std::lower_bound(vs.begin(), vs.end(), target);
          double best = 1e300;
          if (it != vs.end()) best = std::min(best, std::fabs(*it - target));
          if (it != vs.begin()) best = std::min(best, std::fabs(*(it - 1) - target));
          if (best < guard)
            throw Status{MLCC3_ESINGULAR, "omega within guard of an orbital-energy denominator"};
        }
      }
}

__global__ void k_nonfinite(const double *x, long long n, int *flag) {
  long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; id < n; id += (long long)gridDim.x * blockDim.x)
    if (!isfinite(x[id])) flag[0] = 1;  // every writer stores the same value
}

void finite_check(mlcc3_ws ws, std::vector<std::pair<const double *, long long>> arrs, hipStream_t s) {
  if (g_dry) return;
  int *flag = (int *)buf(ws, "finite_flag", 1, s);
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), s));
  for (auto &a : arrs)
    if (a.second > 0) hipLaunchKernelGGL(k_nonfinite, dim3(1024), dim3(256), 0, s, a.first, a.second, flag);
  HIPRT(hipGetLastError());
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h) throw Status{MLCC3_ENONFINITE, "NaN or Inf in an input array"};
}

// 64-bit content fingerprint of the ground-state inputs: the sum modulo 2^64 over all elements of
// mix(bits(x) ^ (tag * golden + index)), with mix the SplitMix64 finaliser (Steele, Lea and Flood,
// 2014).  The sum is order-independent, so the parallel reduction is deterministic.
__device__ __forceinline__ unsigned long long fp_mix(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

struct FpArrays {
  const double *x[8];
  long long n[8];
};

// array blockIdx.y (tag blockIdx.y + 1) of the list
__global__ void k_fingerprint(FpArrays a, unsigned long long *out) {
  __shared__ unsigned long long red[256];
  const double *x = a.x[blockIdx.y];
  const long long n = a.n[blockIdx.y];
  const unsigned long long tag = blockIdx.y + 1;
  unsigned long long acc = 0;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n; id += (long long)gridDim.x * blockDim.x)
    acc += fp_mix((unsigned long long)__double_as_longlong(x[id]) ^ (tag * 0x9E3779B97F4A7C15ULL + (unsigned long long)id));
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

// enqueue the fingerprint of every ground-state input array into the workspace word "fingerprint"
// and its copy to *host (valid after the stream has synchronised)
void ground_fingerprint(mlcc3_ws ws, const mlcc3_ground *g, unsigned long long *host, hipStream_t s) {
  *host = 0;
  if (g_dry) return;
  const Dims d = dims_of(g);
  unsigned long long *w = (unsigned long long *)buf(ws, "fingerprint", 1, s);
  HIPCHK(hipMemsetAsync(w, 0, sizeof(unsigned long long), s));
  const std::pair<const double *, long long> arrs[] = {{g->eps_o, d.NO},
                                                       {g->eps_v, d.NV},
                                                       {g->L_OO, (long long)d.nc * d.NO * d.NO},
                                                       {g->L_OV, (long long)d.nc * d.NO * d.NV},
                                                       {g->L_vV, (long long)d.nc * d.nv * d.NV},
                                                       {g->t1, (long long)d.NV * d.NO},
                                                       {g->t2_vVoo, (long long)d.nv * d.NV * d.no * d.no},
                                                       {g->t2_vvoO, (long long)d.nv * d.nv * d.no * d.NO}};
  FpArrays fa;
  for (int i = 0; i < 8; i++) {
    fa.x[i] = arrs[i].first;
    fa.n[i] = arrs[i].second > 0 ? arrs[i].second : 0;
  }
  hipLaunchKernelGGL(k_fingerprint, dim3(512, 8), dim3(256), 0, s, fa, w);   // one launch for all eight
  HIPRT(hipGetLastError());
  HIPCHK(hipMemcpyAsync(host, w, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
}

void ground_finite(mlcc3_ws ws, const mlcc3_ground *g, hipStream_t s) {
  const Dims d = dims_of(g);
  finite_check(ws,
               {{g->eps_o, d.NO},
                {g->eps_v, d.NV},
                {g->L_OO, (long long)d.nc * d.NO * d.NO},
                {g->L_OV, (long long)d.nc * d.NO * d.NV},
                {g->L_vV, (long long)d.nc * d.nv * d.NV},
                {g->t1, (long long)d.NV * d.NO},
                {g->t2_vVoo, (long long)d.nv * d.NV * d.no * d.no},
                {g->t2_vvoO, (long long)d.nv * d.nv * d.no * d.NO}},
               s);
}

void vec_finite(mlcc3_ws ws, const Dims &d, const mlcc3_vec &v, hipStream_t s) {
  finite_check(ws,
               {{v.x1, (long long)d.NV * d.NO},
                {v.x2_vVoo, (long long)d.nv * d.NV * d.no * d.no},
                {v.x2_vvoO, (long long)d.nv * d.nv * d.no * d.NO}},
               s);
}

long long max_off(const Idx2 &f, int X) {
  if (X <= 0) return 0;
  if (f.d <= 0) return (long long)(X - 1) * f.s0;
  const long long q = (X - 1) / f.d, r = (X - 1) % f.d;
  long long best = q * f.s1 + r * f.s0;
  if (q > 0) best = std::max(best, (q - 1) * f.s1 + (long long)(f.d - 1) * f.s0);
  return best;
}

void check_range(const void *p, const Idx2 &row, int R, const Idx2 &col, int Cc, long long batch, int nb,
                 const char *what, long long vstride = 0, int nvec = 1, size_t esz = sizeof(double)) {
  const uintptr_t lo = (uintptr_t)p;
  const uintptr_t hi =
      lo + (uintptr_t)(max_off(row, R) + max_off(col, Cc) + batch * (nb - 1) + vstride * (nvec - 1) + 1) * esz;
  for (const Extent &e : t_ext)
    if (e.lo <= lo && hi <= e.hi) return;
  throw Status{MLCC3_EHIP, std::string("internal bounds check failed for GEMM operand ") + what};
}

void check_bytes(const void *p, size_t bytes, const char *what) {
  const uintptr_t lo = (uintptr_t)p, hi = lo + bytes;
  for (const Extent &e : t_ext)
    if (e.lo <= lo && hi <= e.hi) return;
  throw Status{MLCC3_EHIP, std::string("internal bounds check failed for ") + what};
}

void gemm(const Gemm &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return;
  for (int i = 0; i < g.nseg; i++) {
    const Seg &sg = g.seg[i];
    if (sg.K <= 0) continue;
    if (sg.A.pf) check_range(sg.A.pf, sg.A.row, g.M, sg.A.col, sg.K, sg.A.batch, g.nbatch, "A", 0, 1, sizeof(float));
    else check_range(sg.A.p, sg.A.row, g.M, sg.A.col, sg.K, sg.A.batch, g.nbatch, "A");
    check_range(sg.B.p, sg.B.row, sg.K, sg.B.col, g.N, sg.B.batch, g.nbatch, "B");
  }
  check_range(g.C, g.crow, g.M, g.ccol, g.N, g.cbatch, g.nbatch, "C");
  long long ktot = 0;
  for (int i = 0; i < g.nseg; i++) ktot += g.seg[i].K;
  const long long tiles = gemm_tiles(g);
  Gemm h = g;
  if (tiles < 1024 && ktot >= 2048 && t_ws) {
    // too few workgroups for a long K: split K (about 2048 workgroups, >= 1024 K each) and
    // reduce the partial tiles in a fixed order
    long long ks = std::min<long long>((2048 + tiles - 1) / tiles, ktot / 1024);
    ks = std::max<long long>(1, std::min<long long>(ks, 4096));
    if (ks > 1) {
      h.ksplit = (int)ks;
      h.P = buf(t_ws, "gemm_splitk", (size_t)(ks * g.nbatch * (long long)g.M * g.N), t_stream);
    }
  }
  HIPCHK(gemm_f64(h, s));
}

hipEvent_t pool_event(mlcc3_ws ws) {
  if (!ws->pool.empty()) {
    hipEvent_t e = ws->pool.back();
    ws->pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}

// large-tile GEMM launch with the bounds self-check of its operands; the d-contraction is
// recorded under timing phase 0 when the workspace timer is on
// whole_k: never split K (each output then sums its K terms in the same order whatever N is)
void tgemm(const TileGemm &g, hipStream_t s, bool whole_k = false) {
  if (g.M <= 0 || g.N <= 0) return;
  for (int i = 0; i < g.nseg; i++) {
    const TgSeg &sg = g.seg[i];
    if (sg.K <= 0) continue;
    const void *ap = sg.Af ? (const void *)sg.Af : (const void *)sg.A;
    const size_t ae = sg.Af ? sizeof(float) : sizeof(double);
    if (g.ak) check_range(ap, sg.amap, g.M, plain(1), sg.K, sg.abatch, g.nbatch, "A (tile GEMM)", sg.avec, g.nvec, ae);
    else check_range(ap, sg.amap, sg.K, plain(1), g.M, sg.abatch, g.nbatch, "A (tile GEMM)", sg.avec, g.nvec, ae);
    check_range(sg.B, plain(sg.ldb), sg.K, plain(1), g.N, sg.bbatch, g.nbatch, "B (tile GEMM)", sg.bvec, g.nvec);
  }
  check_range(g.C, g.cmap, g.M, plain(1), g.N, g.cbatch, g.nbatch, "C (tile GEMM)", g.cvec, g.nvec);
  mlcc3_ws ws = t_ws;
  if (!g.dcontract && g.nvec == 1 && !whole_k) {
    // split K when the 128x128 tiles fill the 512 workgroup slots (two per CU) in few, ragged
    // rounds: the part count with the best filled fraction of the last round (>= 256 K each)
    const long long tiles = tile_gemm_blocks(g);
    int kmin = g.seg[0].K;
    for (int i = 1; i < g.nseg; i++) kmin = std::min(kmin, g.seg[i].K);
    int ks = 1;
    double best = 0.0;
    for (int k = 1; k <= 8 && tiles < 2048; k++) {
      if (k > 1 && kmin / k < 256) break;
      const double w = tiles * k / 512.0, eff = w / std::ceil(w);
      if (eff > best + 0.05) {
        best = eff;
        ks = k;
      }
    }
    if (tune().back_ksplit > 0) ks = tune().back_ksplit;
    if (ks > 1 && ws) {
      TileGemm h = g;
      h.ksplit = ks;
      h.C = buf(ws, "tile_splitk", (size_t)ks * g.nbatch * (long long)g.M * g.N, s);
      h.cmap = plain(g.N);
      h.cpart = (long long)g.M * g.N;
      h.cbatch = ks * h.cpart;
      h.alpha = 1.0;
      h.beta = 0.0;
      HIPCHK(tile_gemm_f64(h, s));
      Gemm r;
      r.M = g.M;
      r.N = g.N;
      r.nbatch = g.nbatch;
      r.ksplit = ks;
      r.P = h.C;
      r.C = g.C;
      r.crow = g.cmap;
      r.ccol = plain(1);
      r.cbatch = g.cbatch;
      r.alpha = g.alpha;
      r.beta = g.beta;
      HIPCHK(gemm_reduce_parts(r, s));
      return;
    }
  }
  if (!g.dcontract || !ws || !ws->timing || g_dry) {
    HIPCHK(tile_gemm_f64(g, s));
    return;
  }
  double fl = 0.0;
  for (int i = 0; i < g.nseg; i++) fl += 2.0 * g.M * (double)g.N * g.seg[i].K * g.nbatch * g.nvec;
  mlcc3_ws_s::Mark mk{0, fl, pool_event(ws), pool_event(ws)};
  HIPCHK(hipEventRecord(mk.a, s));
  HIPCHK(tile_gemm_f64(g, s));
  HIPCHK(hipEventRecord(mk.b, s));
  ws->marks.push_back(mk);
}

TgSeg tseg(const double *A, Idx2 amap, long long abatch, const double *B, long long ldb, long long bbatch, int K) {
  TgSeg sg;
  sg.A = A; sg.amap = amap; sg.abatch = abatch;
  sg.B = B; sg.ldb = ldb; sg.bbatch = bbatch;
  sg.K = K;
  return sg;
}

void reg_ground(const mlcc3_ground *g) {
  const long long no = g->n_o, nv = g->n_v, NO = g->N_O, NV = g->N_V, nc = g->n_chol;
  reg(g->eps_o, NO, "eps_o");
  reg(g->eps_v, NV, "eps_v");
  reg(g->L_OO, nc * NO * NO, "L_OO");
  reg(g->L_OV, nc * NO * NV, "L_OV");
  reg(g->L_vV, nc * nv * NV, "L_vV");
  reg(g->t1, NV * NO, "t1");
  reg(g->t2_vVoo, nv * NV * no * no, "t2_vVoo");
  reg(g->t2_vvoO, nv * nv * no * NO, "t2_vvoO");
}

void reg_vec(const mlcc3_ground *g, const double *x1, const double *a, const double *b) {
  const long long no = g->n_o, nv = g->n_v, NO = g->N_O, NV = g->N_V;
  reg(x1, NV * NO, "x1");
  reg(a, nv * NV * no * no, "x2_vVoo");
  reg(b, nv * nv * no * NO, "x2_vvoO");
}

// element count of an ordered-triple buffer of n values in the running call's element type, as
// the double count buf() takes, and the sub-buffer starting e elements in
size_t xcount(long long n) { return t_xf32 ? (size_t)((n + 1) / 2) : (size_t)n; }
double *xsub(double *base, long long e) { return t_xf32 ? (double *)((float *)base + e) : base + e; }
size_t xesz() { return t_xf32 ? sizeof(float) : sizeof(double); }
// element pitch of the vectors of a group in the contravariant buffers: float blocks start on
// 256-byte boundaries (the 16-byte loads of the split-bf16 staging need 16-byte aligned bases)
long long xpitch(long long n) { return t_xf32 ? (n + 63) / 64 * 64 : n; }
// first indices p held by the ordered-triple buffers, and the ordered triples they hold
int snp(const Dims &d) { return t_np > 0 ? t_np : d.no; }
long long sord(const Dims &d) { return (long long)snp(d) * d.no * d.no; }
// the A operand of a segment reads the running call's contravariant blocks (float when t_xf32)
void xa(Seg &sg) {
  if (!t_xf32) return;
  sg.A.pf = (const float *)sg.A.p;
  sg.A.p = nullptr;
}
void xa(TgSeg &sg) {
  if (!t_xf32) return;
  sg.Af = (const float *)sg.A;
  sg.A = nullptr;
}

Seg seg(const double *A, Idx2 arow, Idx2 acol, long long abatch, const double *B, Idx2 brow, Idx2 bcol,
        long long bbatch, int K, double scale = 1.0) {
  Seg sg;
  sg.A.p = A; sg.A.row = arow; sg.A.col = acol; sg.A.batch = abatch;
  sg.B.p = B; sg.B.row = brow; sg.B.col = bcol; sg.B.batch = bbatch;
  sg.K = K;
  sg.scale = scale;
  return sg;
}

// ------------------------------------------------------ Cholesky assemblies
// oovo-kind: C[L][j][k][c] = sum_J A^J_Lj B^J_ck  (A: [nc][NO][NO], B: [nc][nv][NO])
Gemm asm_oovo(const Dims &d, double *C) {
  Gemm g;
  g.M = d.NO * d.no;  // m = L*no + j
  g.N = d.nv * d.no;  // n = c*no + k
  g.crow = plain((long long)d.no * d.nv);
  g.ccol = split(d.no, 1, d.nv);
  g.C = C;
  return g;
}
// A [nc][NO][row pitch pa], B [nc][nv][row pitch pb] (pitch 0: N_O)
Seg asm_oovo_seg(const Dims &d, const double *A, const double *B, long long pa = 0, long long pb = 0) {
  if (pa <= 0) pa = d.NO;
  if (pb <= 0) pb = d.NO;
  return seg(A, split(d.no, pa, 1), plain((long long)d.NO * pa), 0, B, plain((long long)d.nv * pb), split(d.no, pb, 1),
             0, d.nc);
}

// --------------------------------------- one-index transformations of the Cholesky vectors
// C[batch][M][N] = alpha * A B + beta * C for plain row-major operands (A: lda, B: ldb) with
// per-batch strides (0 = shared)
Gemm plain_gemm(int M, int N, int K, int nbatch, const double *A, long long lda, long long abatch, const double *B,
                long long ldb, long long bbatch, double *C, long long ldc, long long cbatch, double alpha,
                double beta) {
  Gemm g;
  g.M = M;
  g.N = N;
  g.nbatch = nbatch;
  g.C = C;
  g.crow = plain(ldc);
  g.ccol = plain(1);
  g.cbatch = cbatch;
  g.alpha = alpha;
  g.beta = beta;
  g.nseg = 1;
  g.seg[0] = seg(A, plain(lda), plain(1), abatch, B, plain(ldb), plain(1), bbatch, K);
  return g;
}

// T1 transform Lhat = (1 - T) L (1 + T) of the Cholesky vectors, T[N_O + A][I] = t^A_I
// (SI, T1-transformed integrals), block by block as MFMA GEMMs batched over the Cholesky index J:
//   Lhat_OO[J][I][K] = L_OO + sum_B L_OV[J][I][B] t[B][K]
//   Lhat_vV[J][a][B] = L_vV - sum_I t[a][I] L_OV[J][I][B]
//   Lhat_Vv[J][D][b] = L_vV[J][b][D] - sum_I t[D][I] L_OV[J][I][b]
//   Lhat_vO[J][c][K] = L_OV[J][K][c] + sum_B L_vV[J][c][B] t[B][K] - sum_I t[c][I] Lhat_OO[J][I][K]
void lhat_blocks(const Dims &d, const mlcc3_ground *g, double *LhOO, double *LhvV, double *LhVv, double *LhvO,
                 hipStream_t s) {
  const int nc = d.nc, NO = d.NO, NV = d.NV, nv = d.nv;
  const double *LOV = g->L_OV, *t1 = g->t1;
  check_bytes(LhOO, sizeof(double) * nc * NO * NO, "Lhat_OO");
  if (!g_dry) HIPRT(hipMemcpyAsync(LhOO, g->L_OO, sizeof(double) * nc * NO * NO, hipMemcpyDeviceToDevice, s));
  gemm(plain_gemm(nc * NO, NO, NV, 1, LOV, NV, 0, t1, NO, 0, LhOO, NO, 0, 1.0, 1.0), s);
  if (nv <= 0) return;
  const long long ov = (long long)NO * NV;
  check_bytes(LhvV, sizeof(double) * nc * nv * NV, "Lhat_vV");
  if (!g_dry) HIPRT(hipMemcpyAsync(LhvV, g->L_vV, sizeof(double) * nc * nv * NV, hipMemcpyDeviceToDevice, s));
  gemm(plain_gemm(nv, NV, NO, nc, t1, NO, 0, LOV, NV, ov, LhvV, NV, (long long)nv * NV, -1.0, 1.0), s);
  check_bytes(LhVv, sizeof(double) * nc * NV * nv, "Lhat_Vv");
  launch_transpose(g->L_vV, LhVv, nc, nv, NV, s);
  gemm(plain_gemm(NV, nv, NO, nc, t1, NO, 0, LOV, NV, ov, LhVv, nv, (long long)NV * nv, -1.0, 1.0), s);
  check_bytes(LhvO, sizeof(double) * nc * nv * NO, "Lhat_vO");
  launch_lhat_vO_init(LOV, nc, NO, NV, nv, LhvO, s);
  gemm(plain_gemm(nc * nv, NO, NV, 1, g->L_vV, NV, 0, t1, NO, 0, LhvO, NO, 0, 1.0, 1.0), s);
  gemm(plain_gemm(nv, NO, NO, nc, t1, NO, 0, LhOO, NO, (long long)NO * NO, LhvO, NO, (long long)nv * NO, -1.0, 1.0), s);
  HIPRT(hipGetLastError());
}

// one-index transformation with a singles vector R, dLhat = Lhat R - R Lhat, as GEMMs:
//   dOO[J][I][K] = sum_A L_OV[J][I][A] R[A][K]
//   dvV[J][a][B] = -sum_I R[a][I] L_OV[J][I][B]
//   dvO[J][c][K] = sum_B Lhat_vV[J][c][B] R[B][K] - sum_I R[c][I] Lhat_OO[J][I][K]
// The two products over the full N_V (dOO and the first term of dvO) are formed for the whole
// group of vectors at once (group_dlhat, rows of pitch nb N_O with vector v at column v N_O);
// the rest per vector (dlhat_rest, on vector v's columns).
void dlhat_rest(const Dims &d, const double *LOV, const double *LhOO, const double *R1, double *dvV, double *dvO,
                long long pitch, hipStream_t s) {
  const int nc = d.nc, NO = d.NO, NV = d.NV, nv = d.nv;
  gemm(plain_gemm(nv, NV, NO, nc, R1, NO, 0, LOV, NV, (long long)NO * NV, dvV, NV, (long long)nv * NV, -1.0, 0.0), s);
  gemm(plain_gemm(nv, NO, NO, nc, R1, NO, 0, LhOO, NO, (long long)NO * NO, dvO, pitch, (long long)nv * pitch, -1.0,
                  1.0),
       s);
}

// X_kc = sum_LD (2 g_kcLD - g_kDLc) x^D_L from bare (ov|ov) = sum_J L_kc L_LD (active k, c):
// s_J = sum_LD L^J_LD x^D_L, y^J_kL = sum_D L^J_kD x^D_L (MFMA GEMM), then
// X_kc = sum_J (2 L^J_kc s_J - sum_L y^J_kL L^J_Lc) summed over J in a fixed order
void fock_like(const Dims &d, const double *LOV, const double *x, double *tmp_x, double *tmp_s, double *tmp_y,
               double *tmp_z, double *out, hipStream_t s) {
  const int nc = d.nc, NO = d.NO, NV = d.NV, no = d.no, nv = d.nv;
  launch_fock_s(LOV, x, nc, NO, NV, tmp_x, tmp_s, s);
  Gemm g;
  g.M = nc * no;
  g.N = NO;
  g.C = tmp_y;
  g.crow = plain(NO);
  g.ccol = plain(1);
  g.nseg = 1;
  g.seg[0] = seg(LOV, split(no, (long long)NO * NV, NV), plain(1), 0, x, plain(NO), plain(1), 0, NV);
  gemm(g, s);
  launch_fock_finish(LOV, tmp_s, tmp_y, nc, NO, NV, no, nv, tmp_z, out, s);
}

// vVvo-kind integral block C[k][D][b][c] = sum_J sum_seg A_seg[J][b][D] B_seg[J][c][k]
// (A: [nc][nv][NV], B: [nc][nv][NO], active k < n_o) through the large-tile GEMM: the active
// columns of B are packed to [nc][nv][n_o], the product (rows (b,D), columns (c,k), K = nc)
// goes to a scratch block, which one pass then permutes into the [k][D][b][c] layout
void vVvo_tiled(mlcc3_ws ws, const Dims &d, int nseg, const double *const *A, const double *const *Bfull, double *C,
                hipStream_t s, const long long *bpitch = nullptr) {
  const int nc = d.nc, nv = d.nv, NV = d.NV, NO = d.NO, no = d.no;
  const long long M = (long long)nv * NV, N = (long long)nv * no;
  if (M <= 0 || N <= 0) return;
  static const char *pn[2] = {"vvvo_b0", "vvvo_b1"};
  double *T = buf(ws, "vvvo_tmp", (size_t)(M * N), s);
  TileGemm g;
  g.M = (int)M;
  g.N = (int)N;
  g.nseg = nseg;
  g.ak = 0;
  g.C = T;
  g.cmap = plain(N);
  for (int i = 0; i < nseg; i++) {
    double *Bp = buf(ws, pn[i], (size_t)nc * nv * no, s);
    check_bytes(Bp, sizeof(double) * nc * nv * no, "packed B (vVvo)");
    const long long ld = bpitch ? bpitch[i] : NO;
    check_bytes(Bfull[i], sizeof(double) * (size_t)(((long long)nc * nv - 1) * ld + no), "B (vVvo)");
    launch_pack_cols(Bfull[i], (long long)nc * nv, (int)ld, no, Bp, s);
    g.seg[i] = tseg(A[i], plain(M), 0, Bp, N, 0, nc);
  }
  tgemm(g, s);
  check_bytes(C, sizeof(double) * M * N, "vVvo block");
  launch_vvvo_permute(T, no, nv, NV, C, s);
  HIPRT(hipGetLastError());
}

// -------------------------------------------------------------- ground prep
bool same_ground(const mlcc3_ground &a, const mlcc3_ground &b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }

void prepare_ground(mlcc3_ws ws, const mlcc3_ground *g, bool reuse, hipStream_t s) {
  if (reuse && ws->prepared && same_ground(ws->key, *g)) {
    // the prepared blocks are reused only if the inputs' contents are those they were made from
    unsigned long long now = 0;
    ground_fingerprint(ws, g, &now, s);
    HIPRT(hipStreamSynchronize(s));
    if (now != ws->fingerprint)
      throw Status{MLCC3_ESTATE, "reuse_ground: the ground-state inputs changed since this workspace prepared its "
                                 "blocks (same pointers, new contents); call with reuse_ground = 0"};
    return;
  }
  ws->prepared = false;
  ws->gle = false;
  ws->tau = mlcc3_ws_s::TauKey{};
  const Dims d = dims_of(g);
  const int no = d.no, nv = d.nv, NO = d.NO, NV = d.NV, nc = d.nc;
  double *LhOO = buf(ws, "LhOO", (size_t)nc * NO * NO, s);
  double *LhvV = buf(ws, "LhvV", (size_t)nc * nv * NV, s);
  double *LhVv = buf(ws, "LhVv", (size_t)nc * NV * nv, s);
  double *LhvO = buf(ws, "LhvO", (size_t)nc * nv * NO, s);
  lhat_blocks(d, g, LhOO, LhvV, LhVv, LhvO, s);
  HIPRT(hipGetLastError());
  const long long LOVs = (long long)NO * NV;
  // G1[k][D][b][c] = ghat_bDck
  double *G1 = buf(ws, "G1", (size_t)no * NV * d.nv2, s);
  {
    const double *A[1] = {LhvV}, *Bv[1] = {LhvO};
    vVvo_tiled(ws, d, 1, A, Bv, G1, s);
  }
  // G2[L][j][k][c] = ghat_Ljck
  double *G2 = buf(ws, "G2", (size_t)NO * no * no * nv, s);
  {
    Gemm gg = asm_oovo(d, G2);
    gg.nseg = 1;
    gg.seg[0] = asm_oovo_seg(d, LhOO, LhvO);
    gemm(gg, s);
  }
  // Gb1[k][b][c][D] = ghat_Dbkc = sum_J Lhat_Db L_kc
  double *Gb1 = buf(ws, "Gb1", (size_t)no * d.nv2 * NV, s);
  {
    Gemm gg;
    gg.M = NV * nv;  // m = D*nv + b
    gg.N = no * nv;  // n = k*nv + c
    gg.crow = split(nv, 1, (long long)nv * NV);
    gg.ccol = split(nv, d.nv2 * NV, NV);
    gg.C = Gb1;
    gg.nseg = 1;
    gg.seg[0] = seg(LhVv, plain(1), plain((long long)NV * nv), 0, g->L_OV, plain(LOVs), split(nv, NV, 1), 0, nc);
    gemm(gg, s);
  }
  // Gb3[j][k][c][L] = ghat_jLkc = sum_J Lhat_jL L_kc
  double *Gb3 = buf(ws, "Gb3", (size_t)no * no * nv * NO, s);
  {
    Gemm gg;
    gg.M = no * NO;  // m = j*NO + L
    gg.N = no * nv;  // n = k*nv + c
    gg.crow = split(NO, (long long)no * nv * NO, 1);
    gg.ccol = plain(NO);
    gg.C = Gb3;
    gg.nseg = 1;
    gg.seg[0] = seg(LhOO, plain(1), plain((long long)NO * NO), 0, g->L_OV, plain(LOVs), split(nv, NV, 1), 0, nc);
    gemm(gg, s);
  }
  // Gb3L[L][j][k][c] (the occupied term of L3 reads G with L outermost); t2xT[i][a][L][b] = t^{ab}_{iL}
  launch_transpose(Gb3, buf(ws, "Gb3L", (size_t)no * no * nv * NO, s), 1, no * no * nv, NO, s);
  launch_occ_xT(g->t2_vvoO, no, nv, NO, buf(ws, "t2xT", (size_t)no * nv * NO * occ_pitch(nv), s), s);
  HIPRT(hipGetLastError());
  // gov[j][k][b][c] = g_jbkc (bare)
  double *gov = buf(ws, "gov", (size_t)no * no * d.nv2, s);
  {
    Gemm gg;
    gg.M = no * nv;  // m = j*nv + b
    gg.N = no * nv;  // n = k*nv + c
    gg.crow = split(nv, (long long)no * d.nv2, nv);
    gg.ccol = split(nv, d.nv2, 1);
    gg.C = gov;
    gg.nseg = 1;
    gg.seg[0] = seg(g->L_OV, split(nv, NV, 1), plain(LOVs), 0, g->L_OV, plain(LOVs), split(nv, NV, 1), 0, nc);
    gemm(gg, s);
  }
  // gLb[k][b][c][L] = g_Lbkc (bare)
  double *gLb = buf(ws, "gLb", (size_t)no * d.nv2 * NO, s);
  {
    Gemm gg;
    gg.M = NO * nv;  // m = L*nv + b
    gg.N = no * nv;  // n = k*nv + c
    gg.crow = split(nv, 1, (long long)nv * NO);
    gg.ccol = split(nv, d.nv2 * NO, NO);
    gg.C = gLb;
    gg.nseg = 1;
    gg.seg[0] = seg(g->L_OV, split(nv, NV, 1), plain(LOVs), 0, g->L_OV, plain(LOVs), split(nv, NV, 1), 0, nc);
    gemm(gg, s);
  }
  // gDo[j][k][c][D] = g_jDkc (bare)
  double *gDo = buf(ws, "gDo", (size_t)no * no * nv * NV, s);
  {
    Gemm gg;
    gg.M = no * NV;  // m = j*NV + D
    gg.N = no * nv;  // n = k*nv + c
    gg.crow = split(NV, (long long)no * nv * NV, 1);
    gg.ccol = plain(NV);
    gg.C = gDo;
    gg.nseg = 1;
    gg.seg[0] = seg(g->L_OV, plain(1), plain(LOVs), 0, g->L_OV, plain(LOVs), split(nv, NV, 1), 0, nc);
    gemm(gg, s);
  }
  // transposed copies so every d- and back-contraction reads unit-stride rows:
  // GL1[k][D][b][c] = ghat_Dbkc (L3 d-term), G1t[k][b][c][D] = ghat_bDck (sigma^{aD}_{ij})
  launch_transpose(Gb1, buf(ws, "GL1", (size_t)no * NV * d.nv2, s), no, (int)d.nv2, NV, s);
  launch_transpose(G1, buf(ws, "G1t", (size_t)no * NV * d.nv2, s), no, NV, (int)d.nv2, s);
  HIPRT(hipGetLastError());
  // F_kc
  double *F = buf(ws, "F", (size_t)no * nv, s);
  fock_like(d, g->L_OV, g->t1, buf(ws, "fock_xT", (size_t)NO * NV, s), buf(ws, "fock_s", nc, s),
            buf(ws, "fock_y", (size_t)nc * no * NO, s),
            buf(ws, "fock_z", (size_t)nc * no * nv, s), F, s);
  // tA[p][q][a][D] = t^{aD}_{pq}
  launch_pack_vVoo(g->t2_vVoo, no, nv, NV, 0, buf(ws, "tA", (size_t)no * no * nv * NV, s), s);
  HIPRT(hipGetLastError());
  // unique triples (including i=j=k, which the permutation kernel zeroes)
  std::vector<UniqueTriple> ut;
  long long canon = 0;
  for (int i = 0; i < no; i++)
    for (int j = 0; j <= i; j++)
      for (int k = 0; k <= j; k++) {
        UniqueTriple u;
        u.i = i; u.j = j; u.k = k;
        const bool alleq = (i == j && j == k);
        u.canon = alleq ? -1 : canon++;
        // the kernels' tile filters locate a triple by its closed-form position
        if (!alleq && canon_index(i, j, k) != u.canon)
          throw Status{MLCC3_EHIP, "internal check failed: canonical triple index"};
        static const int P[6][3] = {{0, 1, 2}, {1, 0, 2}, {2, 1, 0}, {0, 2, 1}, {2, 0, 1}, {1, 2, 0}};
        const int o[3] = {i, j, k};
        int mask = 0;
        for (int sidx = 0; sidx < 6; sidx++) {
          bool dup = false;
          for (int t = 0; t < sidx; t++)
            if (o[P[t][0]] == o[P[sidx][0]] && o[P[t][1]] == o[P[sidx][1]] && o[P[t][2]] == o[P[sidx][2]]) dup = true;
          if (!dup) mask |= 1 << sidx;
        }
        u.mask = mask;
        ut.push_back(u);
      }
  ws->nu = (int)ut.size();
  void *dut = buf(ws, "utriples", ut.size() * sizeof(UniqueTriple) / sizeof(double) + 1, s);
  HIPRT(hipMemcpyAsync(dut, ut.data(), ut.size() * sizeof(UniqueTriple), hipMemcpyHostToDevice, s));
  unsigned long long fp = 0;
  ground_fingerprint(ws, g, &fp, s);
  HIPRT(hipStreamSynchronize(s));  // the host vector goes out of scope; fp is valid
  ws->fingerprint = fp;
  ws->key = *g;
  ws->prepared = true;
}

double *B(mlcc3_ws ws, const char *name) {
  auto it = ws->bufs.find(name);
  if (it == ws->bufs.end()) throw Status{MLCC3_EHIP, std::string("internal: missing buffer ") + name};
  reg(it->second.first, (long long)(it->second.second / sizeof(double)), "ws");
  return (double *)it->second.first;
}

// the occupied-term operands read inside the permutation kernel: x [n_v][n_v][n_o][N_O] and a
// G block of n_o^2 n_v N_O elements (either layout)
void reg_check_occ(const Dims &d, const double *x, const double *G) {
  const long long nx = (long long)d.nv * occ_pitch(d.nv) * d.no * d.NO, ng = (long long)d.no * d.no * d.nv * d.NO;
  check_range(x, plain(1), (int)nx, plain(0), 1, 0, 1, "occupied-term x");
  check_range(G, plain(1), (int)ng, plain(0), 1, 0, 1, "occupied-term G");
}

// ------------------------------------------------------------ W and X~ builders
// GEMM operand given as a strided map: element (row, col) of batch z
struct BMap {
  const double *p;
  Idx2 row, col;
  long long batch;
};

// one product term of the d-contraction: x [(p,q,a)][D] and G [r][D][(b,c)], vector v of a
// group at x + v*xv, G + v*Gv (stride 0: shared by the group)
struct DSeg {
  const double *x = nullptr;
  long long xv = 0;
  const double *G = nullptr;
  long long Gv = 0;
};

// persistent grid of the d-contraction: per_cu workgroups per CU unless the workspace tuning
// says otherwise; 0 = one workgroup per tile
int persist_grid(int per_cu) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (!g_dry && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  const int f = tune().dc_wg_per_cu;
  if (f < 0) return 0;
  return (f > 0 ? f : per_cu) * cus;
}

// the ordered triples a GEMM over rows (p,q,a) and batch r must produce for the call's triple
// range and core-valence separation (off when every triple is needed)
TripleFilter triple_filter(const Dims &d, const Range &r, bool zero) {
  TripleFilter f;
  f.on = (r.tb > 0 || r.te < mlcc3_num_triples(d.no) || t_cvs) ? 1 : 0;
  f.no = d.no;
  f.nv = d.nv;
  f.zero = zero ? 1 : 0;
  f.core = t_cvs ? t_cvs_bits : 0;
  f.tb = r.tb;
  f.te = r.te;
  f.pq0 = t_p0 * d.no;
  return f;
}

// W_v[p][q][r][a][b][c] = sum_seg sum_D x_seg,v[(p,q,a)][D] G_seg,v[r][D][(b,c)] for the nb vectors
// of a group (W_v at W + v*|W|), one persistent launch for the whole group; only the ordered
// triples of the range r (and, under core-valence separation, with a core index) are formed
void w_dterm(const Dims &d, double *W, int nb, const DSeg *seg0, int nseg, const Range &r, hipStream_t s) {
  const long long Wv = sord(d) * d.nv3;
  // rows (p,q,a) of the occupied slab: the x operands start at row t_p0 n_o n_v
  DSeg seg[2];
  for (int i = 0; i < nseg; i++) {
    seg[i] = seg0[i];
    seg[i].x += (long long)t_p0 * d.no * d.nv * d.NV;
  }
  if (t_prec == MLCC3_BF16X3 || t_prec == MLCC3_BF16X6) {
    // split-bf16 products on bf16 planes of the operands (B planes transposed, K-contiguous)
    mlcc3_ws ws = t_ws;
    const int ns = t_prec == MLCC3_BF16X3 ? 2 : 3;
    BfGemm g;
    g.M = snp(d) * d.no * d.nv;
    g.N = (int)d.nv2;
    g.nbatch = d.no;
    g.nvec = nb;
    g.ns = ns;
    g.C = W;
    g.cmap = split(d.nv, (long long)d.no * d.nv3, d.nv2);
    g.cbatch = d.nv3;
    g.cvec = Wv;
    g.nseg = nseg;
    g.persist = persist_grid(2);
    g.tf = triple_filter(d, r, false);
    const int Kp = (d.NV + BF_BK - 1) / BF_BK * BF_BK;
    const int Mp = (g.M + BF_BM - 1) / BF_BM * BF_BM, Np = (g.N + BF_BN - 1) / BF_BN * BF_BN;
    static const char *an[2] = {"bf_A0", "bf_A1"}, *bn[2] = {"bf_B0", "bf_B1"};
    for (int i = 0; i < nseg; i++) {
      const int na_v = seg[i].xv ? nb : 1, nb_v = seg[i].Gv ? nb : 1;
      const long long sa = (long long)Mp * Kp, sb = (long long)d.no * Np * Kp;  // one vector, one plane
      const long long pa = sa * na_v, pb = sb * nb_v;                           // one plane
      uint16_t *A = (uint16_t *)buf(ws, an[i], (size_t)(pa * ns + 3) / 4, s);
      uint16_t *Bm = (uint16_t *)buf(ws, bn[i], (size_t)(pb * ns + 3) / 4, s);
      check_range(seg[i].x, plain(d.NV), g.M, plain(1), d.NV, 0, 1, "A (d-contraction)", seg[i].xv, nb);
      check_range(seg[i].G, plain(d.nv2), d.NV, plain(1), (int)d.nv2, (long long)d.NV * d.nv2, d.no,
                  "B (d-contraction)", seg[i].Gv, nb);
      check_bytes(A, (size_t)(pa * ns) * sizeof(uint16_t), "bf16 A planes (d-contraction)");
      check_bytes(Bm, (size_t)(pb * ns) * sizeof(uint16_t), "bf16 B planes (d-contraction)");
      for (int v = 0; v < na_v; v++)
        HIPCHK(split_bf16(seg[i].x + v * seg[i].xv, 1, g.M, d.NV, A + v * sa, Mp, Kp, pa, ns, 0, s));
      for (int v = 0; v < nb_v; v++)
        HIPCHK(split_bf16(seg[i].G + v * seg[i].Gv, d.no, d.NV, (int)d.nv2, Bm + v * sb, Kp, Np, pb, ns, 1, s));
      g.seg[i].A = A;
      g.seg[i].aplane = pa;
      g.seg[i].avec = seg[i].xv ? sa : 0;
      g.seg[i].B = Bm;
      g.seg[i].bplane = pb;
      g.seg[i].bbatch = (long long)Np * Kp;
      g.seg[i].bvec = seg[i].Gv ? sb : 0;
      g.seg[i].Kp = Kp;
    }
    check_range(W, g.cmap, g.M, plain(1), g.N, g.cbatch, g.nbatch, "C (d-contraction)", g.cvec, nb);
    if (!ws || !ws->timing || g_dry) {
      HIPCHK(dcontract_bf16(g, s));
      return;
    }
    const double fl = 2.0 * g.M * (double)g.N * d.NV * g.nbatch * nseg * nb;
    mlcc3_ws_s::Mark mk{0, fl, pool_event(ws), pool_event(ws)};
    HIPCHK(hipEventRecord(mk.a, s));
    HIPCHK(dcontract_bf16(g, s));
    HIPCHK(hipEventRecord(mk.b, s));
    ws->marks.push_back(mk);
    return;
  }
  if (t_prec == MLCC3_FP32) {
    // FP32 MFMA on rounded, zero-padded copies of the operands; W is written in FP64
    mlcc3_ws ws = t_ws;
    MixGemm g;
    g.M = snp(d) * d.no * d.nv;
    g.N = (int)d.nv2;
    g.nbatch = d.no;
    g.nvec = nb;
    g.C = W;
    g.cmap = split(d.nv, (long long)d.no * d.nv3, d.nv2);
    g.cbatch = d.nv3;
    g.cvec = Wv;
    g.nseg = nseg;
    g.persist = persist_grid(2);
    g.tf = triple_filter(d, r, false);
    const int Kp = (d.NV + 3) / 4 * 4, Np = ((int)d.nv2 + 3) / 4 * 4;
    static const char *an[2] = {"mx_A0", "mx_A1"}, *bn[2] = {"mx_B0", "mx_B1"};
    for (int i = 0; i < nseg; i++) {
      const int na_v = seg[i].xv ? nb : 1, nb_v = seg[i].Gv ? nb : 1;
      const size_t sa = (size_t)g.M * Kp, sb = (size_t)d.no * Kp * Np;
      float *A = (float *)buf(ws, an[i], (sa * na_v + 1) / 2, s);
      float *Bm = (float *)buf(ws, bn[i], (sb * nb_v + 1) / 2, s);
      check_range(seg[i].x, plain(d.NV), g.M, plain(1), d.NV, 0, 1, "A (d-contraction)", seg[i].xv, nb);
      check_range(seg[i].G, plain(d.nv2), d.NV, plain(1), (int)d.nv2, (long long)d.NV * d.nv2, d.no,
                  "B (d-contraction)", seg[i].Gv, nb);
      check_bytes(A, sa * na_v * sizeof(float), "FP32 A (d-contraction)");
      check_bytes(Bm, sb * nb_v * sizeof(float), "FP32 B (d-contraction)");
      for (int v = 0; v < na_v; v++)
        HIPCHK(pad_to_f32(seg[i].x + v * seg[i].xv, 1, g.M, d.NV, A + v * sa, g.M, Kp, s));
      for (int v = 0; v < nb_v; v++)
        HIPCHK(pad_to_f32(seg[i].G + v * seg[i].Gv, d.no, d.NV, (int)d.nv2, Bm + v * sb, Kp, Np, s));
      g.seg[i].A = A;
      g.seg[i].lda = Kp;
      g.seg[i].avec = seg[i].xv ? (long long)sa : 0;
      g.seg[i].B = Bm;
      g.seg[i].ldb = Np;
      g.seg[i].bbatch = (long long)Kp * Np;
      g.seg[i].bvec = seg[i].Gv ? (long long)sb : 0;
      g.seg[i].Kp = Kp;
      g.seg[i].Np = Np;
    }
    check_range(W, g.cmap, g.M, plain(1), g.N, g.cbatch, g.nbatch, "C (d-contraction)", g.cvec, nb);
    if (!ws || !ws->timing || g_dry) {
      HIPCHK(dcontract_f32(g, s));
      return;
    }
    const double fl = 2.0 * g.M * (double)g.N * d.NV * g.nbatch * nseg * nb;
    mlcc3_ws_s::Mark mk{0, fl, pool_event(ws), pool_event(ws)};
    HIPCHK(hipEventRecord(mk.a, s));
    HIPCHK(dcontract_f32(g, s));
    HIPCHK(hipEventRecord(mk.b, s));
    ws->marks.push_back(mk);
    return;
  }
  TileGemm g;
  g.M = snp(d) * d.no * d.nv;
  g.N = (int)d.nv2;
  g.nbatch = d.no;
  g.nvec = nb;
  g.C = W;
  g.cmap = split(d.nv, (long long)d.no * d.nv3, d.nv2);
  g.cbatch = d.nv3;
  g.cvec = Wv;
  g.nseg = nseg;
  g.dcontract = 1;
  g.persist = persist_grid(2);
  g.tf = triple_filter(d, r, false);
  for (int i = 0; i < g.nseg; i++) {
    g.seg[i] = tseg(seg[i].x, plain(d.NV), 0, seg[i].G, d.nv2, (long long)d.NV * d.nv2, d.NV);
    g.seg[i].avec = seg[i].xv;
    g.seg[i].bvec = seg[i].Gv;
  }
  tgemm(g, s);
}

// occupied-term operands: xT[p][a][L][b] (launch_occ_xT of an [a][b][p][L] block) and G stored
// [L][q][r][c] (G2, Uo, Gb3L); vector v of a group at + v*xv, + v*gv (stride 0: shared).  In the
// reduced-precision forms the term is formed from FP32 copies of both operands (workspace
// buffers of the segment, one block per vector or one shared block).
void occ_add(mlcc3_ws ws, OccTerm &ot, const Dims &d, const double *xT, long long xv, const double *G, long long gv,
             int nb, hipStream_t s) {
  const int sg = ot.nseg++;
  ot.NO = d.NO;
  ot.x[sg] = xT;
  ot.G[sg] = G;
  ot.xv[sg] = xv;
  ot.gv[sg] = gv;
  for (int v = 0; v < nb; v++) reg_check_occ(d, xT + v * xv, G + v * gv);
  if (!t_xf32) return;
  static const char *const xname[2] = {"occ_x32_0", "occ_x32_1"}, *const gname[2] = {"occ_g32_0", "occ_g32_1"};
  const long long nx = (long long)d.no * d.nv * d.NO * occ_pitch(d.nv), ng = (long long)d.no * d.no * d.nv * d.NO;
  const int nxb = xv ? nb : 1, ngb = gv ? nb : 1;
  float *xs = (float *)buf(ws, xname[sg], (size_t)((nx * nxb + 1) / 2), s);
  float *gs = (float *)buf(ws, gname[sg], (size_t)((ng * ngb + 1) / 2), s);
  for (int v = 0; v < nxb; v++) launch_to_f32(xT + v * xv, nx, xs + v * nx, s);
  for (int v = 0; v < ngb; v++) launch_to_f32(G + v * gv, ng, gs + v * ng, s);
  ot.xs[sg] = xs;
  ot.Gs[sg] = gs;
  ot.xsv[sg] = xv ? nx : 0;
  ot.gsv[sg] = gv ? ng : 0;
}

// transposed occupied-term copies of nb [a][b][p][L] blocks (block v at x[v]) into workspace
// buffer `name`, stacked with the stride returned in *stride
const double *occ_xT(mlcc3_ws ws, const Dims &d, const double *const *x, int nb, const char *name, long long *stride,
                     hipStream_t s) {
  const long long n = (long long)d.no * d.nv * d.NO * occ_pitch(d.nv);
  double *xT = buf(ws, name, (size_t)(n * nb), s);
  for (int v = 0; v < nb; v++) launch_occ_xT(x[v], d.no, d.nv, d.NO, xT + v * n, s);
  HIPRT(hipGetLastError());
  *stride = n;
  return xT;
}

// symmetrise, divide and convert the W blocks of nb vectors (W_v at W + v*|W|) into X~_v at
// Xt + v*pitch (pitch |W|, padded to 64 elements for float blocks; covariant X into Xc at
// + v*|W|); one launch per pass for the whole group
// passes: 3 both, 1 the symmetrisation only (W -> Xu, added into Xu for a later occupied slab),
// 2 the contravariant pass only (Xu -> Xt for the slab)
void permute(mlcc3_ws ws, const Dims &d, const double *W, double *Xt, const double *eps_o, const double *eps_v,
             const double *omega, int nb, Range r, const LocalTerms &lt, const OccTerm &ot, hipStream_t s,
             double *Xc = nullptr, int passes = 3) {
  check(nb >= 1 && nb <= kMaxVecBatch, "vector group too large");
  // unique-triple blocks Xu[u][a][b][c] with rows of pitch occ_pitch(n_v) (whole 128-byte lines)
  const long long Wv = sord(d) * d.nv3, Xuv = (long long)ws->nu * d.nv2 * occ_pitch(d.nv);
  double *Xu = buf(ws, "Xu", (size_t)(Xuv * nb), s);
  VecBatch vb;
  vb.nvec = nb;
  vb.w = Wv;
  vb.xu = Xuv;
  vb.xt = xpitch(Wv);
  for (int v = 0; v < nb; v++) vb.omega[v] = omega[v];
  vb.cvs = t_cvs;
  vb.core_bits = t_cvs_bits;
  vb.p0 = t_p0;
  vb.np = t_np;
  vb.tl = t_tl;
  vb.ntl = t_ntl;
  const UniqueTriple *ut = (const UniqueTriple *)B(ws, "utriples");
  if (passes & 1) {
    check_bytes(W, sizeof(double) * Wv * nb, "W (permutation)");
    launch_sym_denom(W, Xu, ut, ws->nu, d.no, d.nv, eps_o, eps_v, vb, r.tb, r.te, lt, ot, s);
  }
  if (passes & 2) {
    check_bytes(Xt, xesz() * vb.xt * nb, "X~ (permutation)");
    if (Xc) check_bytes(Xc, sizeof(double) * Wv * nb, "covariant X (permutation)");
    launch_contra(Xu, Xt, Xc, ut, ws->nu, d.no, d.nv, vb, tune().contra_form, s, t_xf32);
  }
  HIPRT(hipGetLastError());
}

// tau~ for all ordered triples into "XT" (and covariant tau into Xc when given).  With reuse,
// the blocks an earlier call on this workspace formed for the same prepared ground state, triple
// range, core-valence setting and precision are kept (returns true) instead of formed again.
bool tau_path(mlcc3_ws ws, const mlcc3_ground *g, const Dims &d, Range r, hipStream_t s, double *Xc = nullptr,
              bool reuse = false) {
  mlcc3_ws_s::TauKey key;
  key.valid = true;
  key.tb = r.tb;
  key.te = r.te;
  key.prec = t_prec;
  key.cvs = t_cvs;
  key.core = t_cvs ? t_cvs_bits : 0;
  key.xf32 = t_xf32;
  const mlcc3_ws_s::TauKey &k = ws->tau;
  if (reuse && !Xc && k.valid && k.tb == key.tb && k.te == key.te && k.prec == key.prec && k.cvs == key.cvs &&
      k.core == key.core && k.xf32 == key.xf32) {
    (void)buf(ws, "XT", xcount(xpitch(d.nord * d.nv3)), s);  // registers the kept buffer for the bounds checks
    return true;
  }
  ws->tau = mlcc3_ws_s::TauKey{};
  double *W = buf(ws, "W", (size_t)(d.nord * d.nv3), s);
  double *XT = buf(ws, "XT", xcount(xpitch(d.nord * d.nv3)), s);
  DSeg sg;
  sg.x = B(ws, "tA");
  sg.G = B(ws, "G1");
  w_dterm(d, W, 1, &sg, 1, r, s);
  OccTerm ot;
  occ_add(ws, ot, d, B(ws, "t2xT"), 0, B(ws, "G2"), 0, 1, s);
  const double zero = 0.0;
  permute(ws, d, W, XT, g->eps_o, g->eps_v, &zero, 1, r, LocalTerms{}, ot, s, Xc);
  ws->tau = key;
  return false;
}


// Y[(i,j,a)][n] = sum_{k,bc} X~[i][j][k][a][b][c] G_k((b,c), n), split over k: the GEMM
// writes one partial product per k into P[k][(i,j,a)][n] and a fixed-order sum reduces them.
// X~ vanishes on the ordered triples outside the range r (and the all-valence ones under
// core-valence separation): the wide GEMM writes zero partial tiles there without computing.
void back_vV(mlcc3_ws ws, const Dims &d, const double *X, const double *G, int N, double *Y0, const Range &r,
             hipStream_t s) {
  // rows (i,j,a) of the occupied slab
  const long long MN = (long long)snp(d) * d.no * d.nv * N;
  double *Y = Y0 + (long long)t_p0 * d.no * d.nv * N;
  double *P = buf(ws, "split_part", (size_t)(MN * d.no), s);
  const Idx2 xrow = split(d.nv, (long long)d.no * d.nv3, d.nv2);
  if (N >= 96 && (t_prec == MLCC3_BF16X3 || t_prec == MLCC3_BF16X6)) {
    // split-bf16 products on the transposed product P^T[k][n][(i,j,a)] = G_k^T X~_k^T: the
    // N_V x n_v^2 integral block (A, split once per call into planes [k][n][(b,c)]) is shared by
    // all column tiles, the triples block (B, FP64, split into planes while it is staged) is read
    // by ceil(N / 128) row tiles; FP32 sums over 64-deep K steps, FP64 across steps
    const int ns = t_prec == MLCC3_BF16X3 ? 2 : 3;
    const int M2 = snp(d) * d.no * d.nv;
    const int Kp = ((int)d.nv2 + BF_BK - 1) / BF_BK * BF_BK, Mp = (N + BF_BM - 1) / BF_BM * BF_BM;
    const long long pa = (long long)d.no * Mp * Kp;  // one plane
    uint16_t *Am = (uint16_t *)buf(ws, "bk_A", (size_t)(pa * ns + 3) / 4, s);
    double *PT = buf(ws, "bk_PT", (size_t)(MN * d.no), s);
    check_range(G, plain(N), (int)d.nv2, plain(1), N, d.nv2 * N, d.no, "G (back-contraction)");
    check_bytes(Am, (size_t)(pa * ns) * sizeof(uint16_t), "bf16 G planes (back-contraction)");
    HIPCHK(split_bf16(G, d.no, (int)d.nv2, N, Am, Kp, Mp, pa, ns, 1, s));
    BfGemm g;
    g.M = N;
    g.N = M2;
    g.nbatch = d.no;
    g.ns = ns;
    g.C = PT;
    g.cmap = plain(M2);
    g.cbatch = MN;
    g.nseg = 1;
    g.tf = triple_filter(d, r, true);
    g.seg[0].A = Am;
    g.seg[0].aplane = pa;
    g.seg[0].abatch = (long long)Mp * Kp;
    if (t_xf32) g.seg[0].B32 = (const float *)X;
    else g.seg[0].B64 = X;
    g.seg[0].bmap = xrow;
    g.seg[0].bbatch = d.nv3;
    g.seg[0].K = (int)d.nv2;
    g.seg[0].Kp = Kp;
    check_range(X, xrow, M2, plain(1), (int)d.nv2, d.nv3, d.no, "X~ (back-contraction)", 0, 1, xesz());
    check_range(PT, plain(M2), N, plain(1), M2, MN, d.no, "C (back-contraction)");
    HIPCHK(dcontract_bf16(g, s));
    // Y[(i,j,a)][n] = sum_k P^T[k][n][(i,j,a)]: fixed-order sum over k, then one transpose
    launch_sum_rows(PT, d.no, MN, P, s);
    launch_transpose(P, Y, 1, N, M2, s);
    HIPRT(hipGetLastError());
    return;
  } else if (N >= 96 && t_prec == MLCC3_FP32 && t_xf32) {
    // FP32 form: FP32 MFMA on the FP32 blocks, read in place, and an FP32 copy of the integral
    // block ([k][(b,c)][n], rows padded to whole 32-deep K slabs); FP32 sums over each slab,
    // FP64 across slabs
    const int Kp = ((int)d.nv2 + 31) / 32 * 32, Np = (N + 3) / 4 * 4;
    float *Gf = (float *)buf(ws, "bk_G32", (size_t)((long long)d.no * Kp * Np + 1) / 2, s);
    check_range(G, plain(N), (int)d.nv2, plain(1), N, d.nv2 * N, d.no, "G (back-contraction)");
    check_bytes(Gf, sizeof(float) * (size_t)d.no * Kp * Np, "FP32 G (back-contraction)");
    HIPCHK(pad_to_f32(G, d.no, (int)d.nv2, N, Gf, Kp, Np, s));
    MixGemm g;
    g.M = snp(d) * d.no * d.nv;
    g.N = N;
    g.nbatch = d.no;
    g.C = P;
    g.cmap = plain(N);
    g.cbatch = MN;
    g.nseg = 1;
    g.tf = triple_filter(d, r, true);
    g.seg[0].A = (const float *)X;
    g.seg[0].amap = xrow;
    g.seg[0].abatch = d.nv3;
    g.seg[0].K = (int)d.nv2;
    g.seg[0].B = Gf;
    g.seg[0].ldb = Np;
    g.seg[0].bbatch = (long long)Kp * Np;
    g.seg[0].Kp = Kp;
    g.seg[0].Np = Np;
    check_range(X, xrow, g.M, plain(1), (int)d.nv2, d.nv3, d.no, "X~ (back-contraction)", 0, 1, xesz());
    check_range(P, plain(N), g.M, plain(1), N, MN, d.no, "C (back-contraction)");
    HIPCHK(dcontract_f32(g, s));
  } else if (N >= 96) {
    TileGemm g;
    g.M = snp(d) * d.no * d.nv;
    g.N = N;
    g.nbatch = d.no;
    g.C = P;
    g.cmap = plain(N);
    g.cbatch = MN;
    g.nseg = 1;
    g.seg[0] = tseg(X, xrow, d.nv3, G, N, d.nv2 * N, (int)d.nv2);
    xa(g.seg[0]);
    g.tf = triple_filter(d, r, true);
    tgemm(g, s);
  } else {
    // narrow N (N_O): the generic GEMM picks 32-wide tiles
    Gemm g;
    g.M = snp(d) * d.no * d.nv;
    g.N = N;
    g.nbatch = d.no;
    g.C = P;
    g.crow = plain(N);
    g.ccol = plain(1);
    g.cbatch = MN;
    g.nseg = 1;
    g.seg[0] = seg(X, xrow, plain(1), d.nv3, G, plain(N), plain(1), d.nv2 * N, (int)d.nv2);
    xa(g.seg[0]);
    gemm(g, s);
  }
  launch_sum_rows(P, d.no, MN, Y, s);
  HIPRT(hipGetLastError());
}

// Bq[r][(b,c)][E] = sum_{(p,q,a)} L~[p][q][r][a][b][c] t^{aE}_{pq} (intermediate of the singles
// terms of the left transform).  FP64: tile GEMM over rows (b,c) and K = (p,q,a) of the occupied
// slab, added into Bq after the first slab.  Split-bf16 forms: L~ is read through its pair
// symmetry, L~[p][q][r][a][b][c] = L~[r][q][p][c][b][a], so that for each r the summed indices
// (q,p,a) run along the ordered buffer with a contiguous; Bq^T[r][E][(b,c)] = sum_{(q,p,a)}
// t^{aE}_{pq} L~[r][q][p][c][b][a] then takes the amplitudes as the pre-split operand (planes
// [E][(q,p,a)]) and L~ as the operand split while staged, K mapped over the (q,p) blocks.  Each
// slab forms its rows r whole; a transpose writes them into Bq.
void form_Bq(mlcc3_ws ws, const Dims &d, const double *XL, double *Bq, hipStream_t s) {
  const int no = d.no, nv = d.nv, NV = d.NV;
  const long long cb = (long long)NV * d.nv2;  // one r of Bq
  if (NV >= 96 && (t_prec == MLCC3_BF16X3 || t_prec == MLCC3_BF16X6)) {
    const int ns = t_prec == MLCC3_BF16X3 ? 2 : 3;
    const int K = no * no * nv, nr = snp(d);
    const int Kp = (K + BF_BK - 1) / BF_BK * BF_BK, Mp = (NV + BF_BM - 1) / BF_BM * BF_BM;
    const long long pa = (long long)Mp * Kp;  // one plane
    const double *tA = B(ws, "tA");
    double *tq = buf(ws, "bq_tq", (size_t)K * NV, s);
    uint16_t *Am = (uint16_t *)buf(ws, "bq_A", (size_t)(pa * ns + 3) / 4, s);
    double *BT = buf(ws, "bq_T", (size_t)(nr * cb), s);
    check_bytes(tA, sizeof(double) * (size_t)K * NV, "t (Bq)");
    launch_swap01(tA, no, (long long)nv * NV, tq, s);  // [q][p][a][E]
    check_bytes(Am, (size_t)(pa * ns) * sizeof(uint16_t), "bf16 t planes (Bq)");
    HIPCHK(split_bf16(tq, 1, K, NV, Am, Kp, Mp, pa, ns, 1, s));
    BfGemm g;
    g.M = NV;
    g.N = (int)d.nv2;
    g.nbatch = nr;
    g.ns = ns;
    g.C = BT;
    g.cmap = plain(d.nv2);
    g.cbatch = cb;
    g.nseg = 1;
    g.seg[0].A = Am;
    g.seg[0].aplane = pa;
    if (t_xf32) g.seg[0].B32 = (const float *)XL;
    else g.seg[0].B64 = XL;
    g.seg[0].bmap = split(nv, nv, d.nv2);             // row (b,c) at b n_v + c n_v^2
    g.seg[0].bbatch = (long long)no * no * d.nv3;     // r: the first index of the ordered buffer
    g.seg[0].K = K;
    g.seg[0].Kp = Kp;
    g.seg[0].kd = nv;                                 // k = (q,p,a) at (q n_o + p) n_v^3 + a
    g.seg[0].ks = d.nv3;
    check_range(XL, g.seg[0].bmap, (int)d.nv2, split(nv, d.nv3, 1), K, g.seg[0].bbatch, nr, "L~ (Bq)", 0, 1,
                xesz());
    check_range(BT, plain(d.nv2), NV, plain(1), (int)d.nv2, cb, nr, "C (Bq)");
    HIPCHK(dcontract_bf16(g, s));
    check_range(Bq + t_p0 * cb, plain(NV), (int)d.nv2, plain(1), NV, cb, nr, "Bq");
    launch_transpose(BT, Bq + t_p0 * cb, nr, NV, (int)d.nv2, s);
    HIPRT(hipGetLastError());
    return;
  }
  TileGemm gg;
  gg.M = (int)d.nv2;
  gg.N = NV;
  gg.nbatch = no;
  gg.ak = 0;
  gg.C = Bq;
  gg.cmap = plain(NV);
  gg.cbatch = cb;
  gg.beta = t_p0 > 0 ? 1.0 : 0.0;
  gg.nseg = 1;
  gg.seg[0] = tseg(XL, split(nv, (long long)no * d.nv3, d.nv2), d.nv3, B(ws, "tA") + (long long)t_p0 * no * nv * NV,
                   NV, 0, snp(d) * no * nv);
  xa(gg.seg[0]);
  tgemm(gg, s, t_np > 0);
}

// Xtau[(i,j,a)][L] = sum tau~ g_Lbkc, kept with the tau~ blocks it was formed from
double *xtau_block(mlcc3_ws ws, const Dims &d, const double *XT, bool tau_kept, const Range &r, hipStream_t s) {
  double *Xtau = buf(ws, "Xtau", (size_t)d.no * d.no * d.nv * d.NO, s);
  if (!(tau_kept && ws->tau.xtau)) {
    back_vV(ws, d, XT, B(ws, "gLb"), d.NO, Xtau, r, s);
    ws->tau.xtau = true;
  }
  return Xtau;
}

// the workspace's tile choice for the N_O-wide back-contractions
void narrow_tile(Gemm &g) {
  const int t = tune().narrow_tile;
  if (t > 0) {
    g.tm = t / 10;
    g.tn = t % 10;
  }
}

// Y[i][(a,b)][L] = alpha * sum_{(j,k,c)} X~[i][j][k][a][b][c] G((j,k,c),L)   (+ second segment)
Gemm back_vO(const Dims &d, const double *X1, BMap G1, const double *X2, BMap G2, double *Y, double alpha) {
  Gemm g;
  g.M = (int)d.nv2;
  g.N = d.NO;
  g.nbatch = snp(d);  // batches i of the occupied slab
  g.C = Y + (long long)t_p0 * d.nv2 * d.NO;
  g.crow = plain(d.NO);
  g.ccol = plain(1);
  g.cbatch = d.nv2 * d.NO;
  g.alpha = alpha;
  g.nseg = X2 ? 2 : 1;
  const int K = d.no * d.no * d.nv;
  const long long xb = (long long)d.no * d.no * d.nv3;
  g.seg[0] = seg(X1, plain(d.nv), split(d.nv, d.nv3, 1), xb, G1.p, G1.row, G1.col, G1.batch, K);
  xa(g.seg[0]);
  if (X2) {
    g.seg[1] = seg(X2, plain(d.nv), split(d.nv, d.nv3, 1), xb, G2.p, G2.row, G2.col, G2.batch, K);
    xa(g.seg[1]);
  }
  narrow_tile(g);
  return g;
}
// G stored [j][k][c][L]
BMap bm_jkcL(const Dims &d, const double *G) { return {G, plain(d.NO), plain(1), 0}; }

// Y[(q,r,c)][M] = sum_{p,(a,b)} X~[p][q][r][a][b][c] x[a][b][p][M], split over p: the partial
// products P[p] of the occupied slab's p go to buffer pname, and (sum) the fixed-order sum over
// all p is written to Y (an occupied-slab caller sums once after the last slab)
void back_qrc(mlcc3_ws ws, const Dims &d, const double *X, const double *x, double *Y, hipStream_t s,
              const char *pname = "split_part", bool sum = true) {
  const long long MN = (long long)d.no * d.no * d.nv * d.NO;
  double *P = buf(ws, pname, (size_t)(MN * d.no), s);
  Gemm g;
  g.M = d.no * d.no * d.nv;
  g.N = d.NO;
  g.nbatch = snp(d);
  g.C = P + t_p0 * MN;
  g.crow = plain(d.NO);
  g.ccol = plain(1);
  g.cbatch = MN;
  g.nseg = 1;
  g.seg[0] = seg(X, split(d.nv, d.nv3, 1), plain(d.nv), (long long)d.no * d.no * d.nv3, x + (long long)t_p0 * d.NO,
                 plain((long long)d.no * d.NO), plain(1), d.NO, (int)d.nv2);
  xa(g.seg[0]);
  narrow_tile(g);
  gemm(g, s);
  if (!sum) return;
  launch_sum_rows(P, d.no, MN, Y, s);
  HIPRT(hipGetLastError());
}

Gemm gemm_plain(int M, int N, double *C, Idx2 crow, Idx2 ccol, double alpha, double beta) {
  Gemm g;
  g.M = M;
  g.N = N;
  g.C = C;
  g.crow = crow;
  g.ccol = ccol;
  g.alpha = alpha;
  g.beta = beta;
  return g;
}

// gLE[k][c][L][E] = sum_J Lh_ck L_LE = ghat_ckLE, the integral block through which the left
// transform's sigma^d_L term contracts Bq: formed once per prepared ground state
double *gle_block(mlcc3_ws ws, const mlcc3_ground *g, const Dims &d, hipStream_t s) {
  const int no = d.no, nv = d.nv, NO = d.NO, NV = d.NV;
  double *gLE = buf(ws, "gLE", (size_t)no * nv * NO * NV, s);
  if (ws->gle) return gLE;
  // rows (k,c) of LhvO[J][c][k]; columns (L,E) of L_OV[J][L][E], unit stride along E
  Gemm gg = gemm_plain(no * nv, NO * NV, gLE, plain((long long)NO * NV), plain(1), 1.0, 0.0);
  gg.nseg = 1;
  gg.seg[0] = seg(B(ws, "LhvO"), split(nv, 1, NO), plain((long long)nv * NO), 0, g->L_OV, plain((long long)NO * NV),
                  plain(1), 0, d.nc);
  gemm(gg, s);
  ws->gle = true;
  return gLE;
}

void zero_out(const Dims &d, const mlcc3_out *o, hipStream_t s) {
  const size_t na = sizeof(double) * d.nv * d.NV * d.no * d.no, nb = sizeof(double) * d.nv * d.nv * d.no * d.NO;
  HIPRT(hipMemsetAsync(o->x1, 0, sizeof(double) * d.NV * d.NO, s));
  if (na) HIPRT(hipMemsetAsync(o->x2_vVoo, 0, na, s));
  if (nb) HIPRT(hipMemsetAsync(o->x2_vvoO, 0, nb, s));
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (g_dry) return;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    HIPCHK(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

template <class F>
int guarded(F &&f) {
  try {
    g_last_error.clear();
    const char *dr = std::getenv("MLCC3_DRYRUN");
    g_dry = dr && dr[0] == '1';
    const char *fa = std::getenv("MLCC3_TEST_FAIL_ALLOC");
    t_alloc_fail_at = fa ? std::atoll(fa) : 0;
    t_alloc_count = 0;
    const char *lg = std::getenv("MLCC3_LOG");
    t_log.on = lg && lg[0] == '1';
    t_log.what.clear();
    t_ext.clear();
    f();
    log_end(MLCC3_OK);
    return MLCC3_OK;
  } catch (const Status &st) {
    g_last_error = st.msg;
    log_end(st.code);
    return st.code;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    log_end(MLCC3_EHIP);
    return MLCC3_EHIP;
  } catch (...) {
    g_last_error = "unknown error";
    log_end(MLCC3_EHIP);
    return MLCC3_EHIP;
  }
}

mlcc3_opts opts_or_default(const mlcc3_opts *o) {
  mlcc3_opts r;
  mlcc3_opts_default(&r);
  if (o) r = *o;
  check(r.precision == MLCC3_FP64 || r.precision == MLCC3_FP32 || r.precision == MLCC3_BF16X3 ||
            r.precision == MLCC3_BF16X6,
        "bad precision");
  t_prec = r.precision;
  t_xf32 = r.precision != MLCC3_FP64;
  t_cvs = 0;
  t_cvs_bits = 0;
  t_cvs_dev = nullptr;
  return r;
}

// ρ/Ω small terms and the output gather shared by the ground residual and the right transform
void finish_right_like(mlcc3_ws ws, const Dims &d, const double *X, const double *T, const double *U,
                       const double *YvV, const double *YvO, int delta, const mlcc3_out *out, hipStream_t s) {
  double *part1 = buf(ws, "part1", (size_t)d.no * d.no * d.nv, s);
  double *Yvv = buf(ws, "Yvv", (size_t)d.no * d.no * d.nv2, s);
  launch_small_right(X, T, B(ws, "gov"), B(ws, "F"), U, d.no, d.nv, part1, Yvv, s, t_xf32);
  launch_singles_out(part1, d.no, d.nv, d.NO, d.NV, out->x1, s);
  DoublesRaw y;
  y.YvV = YvV; y.YvO = YvO; y.Yvv = Yvv;
  y.no = d.no; y.nv = d.nv; y.NO = d.NO; y.NV = d.NV; y.delta = delta;
  launch_doubles_out(y, out->x2_vVoo, out->x2_vvoO, s);
  HIPRT(hipGetLastError());
}


// per-vector sizes of the prepared right-vector blocks (stacked for a group of vectors)
struct RightSizes {
  long long RA, RB, U1, Uo, Ukc, Xi;
};
RightSizes right_sizes(const Dims &d) {
  return {(long long)d.no * d.no * d.nv * d.NV, (long long)d.nv * d.nv * d.no * d.NO, (long long)d.no * d.NV * d.nv2,
          (long long)d.NO * d.no * d.no * d.nv, (long long)d.no * d.nv, (long long)d.no * d.no * d.nv * d.NO};
}

// one-index transformed blocks of right vector `slot` of a group of nb: Rbar packs "RA"
// [p][q][a][D] and "RB" [a][b][p][L], Upsilon_bDck "U1", Upsilon_Ljck "Uo", Upsilon_kc "Ukc",
// Xi_jLkc "Xi"; each buffer holds nb blocks, this vector's at slot * size
void group_dlhat(mlcc3_ws ws, const mlcc3_ground *g, const Dims &d, const mlcc3_vec *R, int nb, hipStream_t s) {
  const int nc = d.nc, NO = d.NO, NV = d.NV, nv = d.nv;
  const long long pitch = (long long)nb * NO;
  double *R1s = buf(ws, "R1s", (size_t)(NV * pitch), s);
  for (int v = 0; v < nb; v++) {
    check_bytes(R[v].x1, sizeof(double) * (size_t)NV * NO, "R1 (group)");
    check_bytes(R1s + v * NO, sizeof(double) * (size_t)((NV - 1) * pitch + NO), "stacked R1");
    if (!g_dry)
      HIPRT(hipMemcpy2DAsync(R1s + v * NO, sizeof(double) * pitch, R[v].x1, sizeof(double) * NO, sizeof(double) * NO,
                             NV, hipMemcpyDeviceToDevice, s));
  }
  double *dOO = buf(ws, "dOO", (size_t)((long long)nc * NO * pitch), s);
  double *dvO = buf(ws, "dvO", (size_t)((long long)nc * nv * pitch), s);
  const double *A[2] = {g->L_OV, B(ws, "LhvV")};
  double *C[2] = {dOO, dvO};
  const int M[2] = {nc * NO, nc * nv};
  for (int i = 0; i < 2; i++) {
    TileGemm tg;
    tg.M = M[i];
    tg.N = (int)pitch;
    tg.nseg = 1;
    tg.ak = 1;
    tg.C = C[i];
    tg.cmap = plain(pitch);
    tg.seg[0] = tseg(A[i], plain(NV), 0, R1s, pitch, 0, NV);
    tgemm(tg, s, true);  // whole K: the same sums for any group size
  }
}

void right_vector_prep(mlcc3_ws ws, const mlcc3_ground *g, const Dims &d, const mlcc3_vec &R, int slot, int nb,
                       hipStream_t s) {
  const int no = d.no, nv = d.nv, NO = d.NO, NV = d.NV, nc = d.nc;
  const RightSizes z = right_sizes(d);
  double *RA = buf(ws, "RA", (size_t)(z.RA * nb), s) + slot * z.RA;
  double *RB = buf(ws, "RB", (size_t)(z.RB * nb), s) + slot * z.RB;
  launch_pack_vVoo(R.x2_vVoo, no, nv, NV, 1, RA, s);
  launch_rbar_vvoO(R.x2_vvoO, no, nv, NO, RB, s);
  // this vector's columns of the group's dOO and dvO (group_dlhat), row pitch nb N_O
  const long long pitch = (long long)nb * NO;
  const double *dOO = B(ws, "dOO") + slot * NO;
  double *dvO = B(ws, "dvO") + slot * NO;
  double *dvV = buf(ws, "dvV", (size_t)nc * nv * NV, s);
  dlhat_rest(d, g->L_OV, B(ws, "LhOO"), R.x1, dvV, dvO, pitch, s);
  HIPRT(hipGetLastError());
  double *U1 = buf(ws, "U1", (size_t)(z.U1 * nb), s) + slot * z.U1;
  {
    const double *A[2] = {dvV, B(ws, "LhvV")}, *Bv[2] = {B(ws, "LhvO"), dvO};
    const long long bp[2] = {NO, pitch};
    vVvo_tiled(ws, d, 2, A, Bv, U1, s, bp);
  }
  double *Uo = buf(ws, "Uo", (size_t)(z.Uo * nb), s) + slot * z.Uo;
  {
    Gemm gg = asm_oovo(d, Uo);
    gg.nseg = 2;
    gg.seg[0] = asm_oovo_seg(d, dOO, B(ws, "LhvO"), pitch, 0);
    gg.seg[1] = asm_oovo_seg(d, B(ws, "LhOO"), dvO, 0, pitch);
    gemm(gg, s);
  }
  double *Ukc = buf(ws, "Ukc", (size_t)(z.Ukc * nb), s) + slot * z.Ukc;
  fock_like(d, g->L_OV, R.x1, B(ws, "fock_xT"), B(ws, "fock_s"), B(ws, "fock_y"), B(ws, "fock_z"), Ukc, s);
  double *Xi = buf(ws, "Xi", (size_t)(z.Xi * nb), s) + slot * z.Xi;
  {
    Gemm gg;
    gg.M = no * no * nv;
    gg.N = NO;
    gg.C = Xi;
    gg.crow = plain(NO);
    gg.ccol = plain(1);
    gg.nseg = 1;
    gg.seg[0] = seg(B(ws, "gDo"), plain(NV), plain(1), 0, R.x1, plain(NO), plain(1), 0, NV);
    gemm(gg, s);
  }
}

// R3 of the nb prepared right vectors of a group (slots 0..nb-1 of the prep buffers):
// contravariant into the vector pitch of Xt (see permute), covariant into Xc (optional)
void build_R3(mlcc3_ws ws, const mlcc3_ground *g, const Dims &d, const mlcc3_vec *R, const double *omega, int nb,
              Range r, double *Xt, double *Xc, hipStream_t s, int passes = 3) {
  const RightSizes z = right_sizes(d);
  double *W = buf(ws, "W", (size_t)(sord(d) * d.nv3 * nb), s);
  DSeg sg[2];
  sg[0].x = B(ws, "RA");
  sg[0].xv = z.RA;
  sg[0].G = B(ws, "G1");
  sg[1].x = B(ws, "tA");
  sg[1].G = B(ws, "U1");
  sg[1].Gv = z.U1;
  w_dterm(d, W, nb, sg, 2, r, s);
  std::vector<const double *> rb(nb);
  for (int v = 0; v < nb; v++) rb[v] = B(ws, "RB") + v * z.RB;
  long long xv = 0;
  const double *RBxT = occ_xT(ws, d, rb.data(), nb, "RBxT", &xv, s);
  OccTerm ot;
  occ_add(ws, ot, d, RBxT, xv, B(ws, "G2"), 0, nb, s);
  occ_add(ws, ot, d, B(ws, "t2xT"), 0, B(ws, "Uo"), z.Uo, nb, s);
  (void)R;
  permute(ws, d, W, Xt, g->eps_o, g->eps_v, omega, nb, r, LocalTerms{}, ot, s, Xc, passes);
}

// L3 (transpose-transformation recipe) of nb left-type vectors into Xt (vector pitch as in permute); packs
// LA/LV (stacked, under the given names) and the singles copy "L1s"
void build_L3(mlcc3_ws ws, const mlcc3_ground *g, const Dims &d, const mlcc3_vec *L, const double *omega, int nb,
              Range r, double *Xt, const char *laname, const char *lvname, hipStream_t s, int passes = 3) {
  const int no = d.no, nv = d.nv, NO = d.NO, NV = d.NV;
  const long long sLA = (long long)no * no * nv * NV, sLV = (long long)no * no * d.nv2, sL1 = (long long)NV * NO;
  double *LA = buf(ws, laname, (size_t)(sLA * nb), s);
  double *LV = buf(ws, lvname, (size_t)(sLV * nb), s);
  double *L1 = buf(ws, "L1s", (size_t)(sL1 * nb), s);
  std::vector<const double *> lb(nb);
  for (int v = 0; v < nb; v++) {
    launch_pack_vVoo(L[v].x2_vVoo, no, nv, NV, 0, LA + v * sLA, s);
    launch_pack_vvoo(L[v].x2_vVoo, no, nv, NV, 0, LV + v * sLV, s);
    if (!g_dry)
      HIPRT(hipMemcpyAsync(L1 + v * sL1, L[v].x1, sizeof(double) * sL1, hipMemcpyDeviceToDevice, s));
    lb[v] = L[v].x2_vvoO;
  }
  double *W = buf(ws, "W", (size_t)(sord(d) * d.nv3 * nb), s);
  DSeg sg;
  sg.x = LA;
  sg.xv = sLA;
  sg.G = B(ws, "GL1");
  w_dterm(d, W, nb, &sg, 1, r, s);
  long long xv = 0;
  const double *LBxT = occ_xT(ws, d, lb.data(), nb, "LBxT", &xv, s);
  OccTerm ot;
  occ_add(ws, ot, d, LBxT, xv, B(ws, "Gb3L"), 0, nb, s);
  LocalTerms lt;
  lt.L1 = L1; lt.gov = B(ws, "gov"); lt.LV = LV; lt.F = B(ws, "F"); lt.NO = NO;
  lt.L1v = sL1;
  lt.LVv = sLV;
  permute(ws, d, W, Xt, g->eps_o, g->eps_v, omega, nb, r, lt, ot, s, nullptr, passes);
}

// core-valence separation of a right or left transform: device copy of the core flags, active
// core bits, and CVS-projected copies of the nvec input vectors (returned in *proj)
void cvs_setup(mlcc3_ws ws, const mlcc3_ground *g, const mlcc3_opts &o, int nvec, const mlcc3_vec *in,
               std::vector<mlcc3_vec> *proj, hipStream_t s) {
  const Dims d = dims_of(g);
  if (!o.cvs_core) return;
  check(d.no <= 64, "core-valence separation needs n_o <= 64");
  unsigned long long bits = 0;
  for (int i = 0; i < d.no; i++)
    if (o.cvs_core[i]) bits |= 1ULL << i;
  unsigned char *flags = (unsigned char *)buf(ws, "cvs_core", (size_t)(d.NO + 7) / 8, s);
  if (!g_dry) {
    HIPRT(hipMemcpyAsync(flags, o.cvs_core, (size_t)d.NO, hipMemcpyHostToDevice, s));
    HIPRT(hipStreamSynchronize(s));  // the host flags may be released when the call returns
  }
  t_cvs = 1;
  t_cvs_bits = bits;
  t_cvs_dev = flags;
  const long long n1 = (long long)d.NV * d.NO, na = (long long)d.nv * d.NV * d.no * d.no,
                  nb = (long long)d.nv * d.nv * d.no * d.NO;
  double *c1 = buf(ws, "cvs_in1", (size_t)(n1 * nvec), s);
  double *ca = buf(ws, "cvs_in2a", (size_t)(na * nvec), s);
  double *cb = buf(ws, "cvs_in2b", (size_t)(nb * nvec), s);
  proj->resize(nvec);
  for (int m = 0; m < nvec; m++) {
    (*proj)[m] = mlcc3_vec{c1 + m * n1, ca + m * na, cb + m * nb};
    launch_cvs_project(in[m].x1, in[m].x2_vVoo, in[m].x2_vvoO, c1 + m * n1, ca + m * na, cb + m * nb, flags, d.no,
                       d.nv, d.NO, d.NV, s);
  }
  HIPRT(hipGetLastError());
}

void cvs_project_out(const Dims &d, const mlcc3_out &o, hipStream_t s) {
  if (!t_cvs) return;
  launch_cvs_project(o.x1, o.x2_vVoo, o.x2_vvoO, o.x1, o.x2_vVoo, o.x2_vvoO, t_cvs_dev, d.no, d.nv, d.NO, d.NV, s);
  HIPRT(hipGetLastError());
}

// vectors per group: several vectors share one launch of the d-contraction and of the
// permutation passes; a group holds two ordered-triple buffers (W, X~) per vector, kept within
// 45% of device memory (environment MLCC3_VEC_BATCH and the workspace tuning cap the group size)
// The W blocks of a vector group and, once the permutation pass has read them, the group's
// contravariant blocks (R~ or L~) share one buffer: the pass reads W into the unique-triple
// blocks before it writes any contravariant element, so one ordered-triple buffer per vector
// (and the shared tau~) is what a transform holds, not two.
double *wx_buffer(mlcc3_ws ws, const Dims &d, int nb, hipStream_t s) {
  const size_t w = (size_t)(d.nord * d.nv3 * nb), x = xcount(xpitch(d.nord * d.nv3) * nb);
  return buf(ws, "W", std::max(w, x), s);
}

int group_size(mlcc3_ws ws, const Dims &d, int nvec) {
  int cap = kMaxVecBatch;
  if (const char *e = std::getenv("MLCC3_VEC_BATCH")) cap = std::max(1, std::min(cap, std::atoi(e)));
  if (tune().vec_group > 0) cap = std::min(cap, tune().vec_group);
  size_t total = (size_t)256 << 30;
  if (!g_dry) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess && tot > 0) total = tot;
  }
  // per vector: the shared W / contravariant buffer and the unique-triple blocks
  const double per = 1.3 * sizeof(double) * (double)(d.nord * d.nv3) + 1.0;
  const int fit = (int)std::max(1.0, std::floor(0.45 * (double)total / per));
  (void)ws;
  return std::max(1, std::min({nvec, cap, fit}));
}

// ------------------------------------------------------ occupied slabs
// For shapes whose ordered-triple buffers do not fit in the device memory, the ground residual
// and the transforms run in occupied slabs: the buffers hold only the ordered triples whose
// first index p lies in the slab ([p - p0][q][r]).  Every ordering of a unique triple
// contributes to its symmetrised block Xu on its own, so Xu is accumulated over one pass of
// slabs (d-contraction and symmetrisation of the slab's W); a second pass of slabs forms the
// slab's contravariant blocks from Xu, and each back-contraction either has p among its output
// rows (the slab's rows) or sums over p (partial products per p, summed once at the end, or a
// GEMM that adds into its output).  A transform holds W, one contravariant slab and Xu.

// first indices per occupied slab: the tuning's cap, else all of them (0: one slab) when W,
// the contravariant blocks and Xu fit in 80% of the device memory, else the widest slab that fits
int slab_width(mlcc3_ws ws, const Dims &d) {
  if (ws->arena) return 0;
  const int cap = tune().occ_slab;
  if (cap > 0) return cap >= d.no ? 0 : cap;
  size_t total = (size_t)256 << 30;
  if (!g_dry) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess && tot > 0) total = tot;
  }
  const double xu = (double)ws->nu * d.nv2 * occ_pitch(d.nv) * sizeof(double);
  const double per_p = 2.0 * sizeof(double) * (double)d.no * d.no * d.nv3;
  const double budget = 0.8 * (double)total - xu - 4.0 * (double)(1 << 30);
  const double fit = std::floor(budget / per_p);
  if (fit >= d.no) return 0;
  check(fit >= 1.0, "the unique-triple blocks leave no room for an occupied slab of one index");
  return (int)fit;
}

// the unique triples each slab of width w visits (those with an index in the slab), as one
// device list "slab_tl" with the slabs' lists back to back; returns the offsets (one per slab
// and the end)
std::vector<int> slab_lists(mlcc3_ws ws, const Dims &d, int w, hipStream_t s) {
  std::vector<int> all, off;
  int u = 0;
  std::vector<std::array<int, 3>> tri;
  for (int i = 0; i < d.no; i++)
    for (int j = 0; j <= i; j++)
      for (int k = 0; k <= j; k++) tri.push_back({i, j, k});  // the order of the prepared triple list
  check((int)tri.size() == ws->nu, "internal: unique triple count");
  for (int p0 = 0; p0 < d.no; p0 += w) {
    off.push_back((int)all.size());
    const int p1 = std::min(d.no, p0 + w);
    for (u = 0; u < ws->nu; u++) {
      const auto &t = tri[u];
      if ((t[0] >= p0 && t[0] < p1) || (t[1] >= p0 && t[1] < p1) || (t[2] >= p0 && t[2] < p1)) all.push_back(u);
    }
  }
  off.push_back((int)all.size());
  int *dl = (int *)buf(ws, "slab_tl", (all.size() * sizeof(int) + sizeof(double) - 1) / sizeof(double) + 1, s);
  if (!g_dry) {
    HIPRT(hipMemcpyAsync(dl, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPRT(hipStreamSynchronize(s));  // the host list goes out of scope
  }
  return off;
}

struct SlabScope {  // sets the occupied slab of the running call, restores "no slab" at exit
  SlabScope(mlcc3_ws ws, const std::vector<int> &off, int w, int p0, int np) {
    t_p0 = p0;
    t_np = np;
    const int sl = p0 / w;
    t_tl = (const int *)B(ws, "slab_tl") + off[sl];
    t_ntl = off[sl + 1] - off[sl];
  }
  ~SlabScope() {
    t_p0 = 0;
    t_np = 0;
    t_tl = nullptr;
    t_ntl = 0;
  }
};

// Xu = 0 before the first slab adds into it
void zero_xu(mlcc3_ws ws, const Dims &d, hipStream_t s) {
  const long long n = (long long)ws->nu * d.nv2 * occ_pitch(d.nv);
  double *Xu = buf(ws, "Xu", (size_t)n, s);
  check_bytes(Xu, sizeof(double) * n, "Xu (zero)");
  launch_zero(Xu, n, s);
  HIPRT(hipGetLastError());
}

// the slab's contravariant blocks from Xu, into "XS"
double *contra_slab(mlcc3_ws ws, const mlcc3_ground *g, const Dims &d, const Range &r, hipStream_t s) {
  double *X = buf(ws, "XS", xcount(xpitch(sord(d) * d.nv3)), s);
  const double zero = 0.0;
  permute(ws, d, nullptr, X, g->eps_o, g->eps_v, &zero, 1, r, LocalTerms{}, OccTerm{}, s, nullptr, 2);
  return X;
}

// Xu of tau3, accumulated over the slabs of width w
void tau_xu_slabs(mlcc3_ws ws, const mlcc3_ground *g, const Dims &d, const Range &r, int w,
                  const std::vector<int> &off, hipStream_t s) {
  zero_xu(ws, d, s);
  for (int p0 = 0; p0 < d.no; p0 += w) {
    SlabScope sc(ws, off, w, p0, std::min(w, d.no - p0));
    double *W = buf(ws, "W", (size_t)(sord(d) * d.nv3), s);
    DSeg sg;
    sg.x = B(ws, "tA");
    sg.G = B(ws, "G1");
    w_dterm(d, W, 1, &sg, 1, r, s);
    OccTerm ot;
    occ_add(ws, ot, d, B(ws, "t2xT"), 0, B(ws, "G2"), 0, 1, s);
    const double zero = 0.0;
    permute(ws, d, W, nullptr, g->eps_o, g->eps_v, &zero, 1, r, LocalTerms{}, ot, s, nullptr, 1);
  }
}

void ground_slabs(mlcc3_ws ws, const mlcc3_ground *g, const Dims &d, const Range &r, int w, const mlcc3_out *out,
                  hipStream_t s) {
  const int no = d.no, nv = d.nv, NO = d.NO, NV = d.NV;
  const std::vector<int> off = slab_lists(ws, d, w, s);
  tau_xu_slabs(ws, g, d, r, w, off, s);
  log_phase("tau3");
  double *YvV = buf(ws, "YvV", (size_t)no * no * nv * NV, s);
  double *YvO = buf(ws, "YvO", (size_t)no * d.nv2 * NO, s);
  double *part1 = buf(ws, "part1", (size_t)no * no * nv, s);
  double *Yvv = buf(ws, "Yvv", (size_t)no * no * d.nv2, s);
  for (int p0 = 0; p0 < no; p0 += w) {
    SlabScope sc(ws, off, w, p0, std::min(w, no - p0));
    double *XT = contra_slab(ws, g, d, r, s);
    back_vV(ws, d, XT, B(ws, "Gb1"), NV, YvV, r, s);
    gemm(back_vO(d, XT, bm_jkcL(d, B(ws, "Gb3")), nullptr, BMap{}, YvO, -1.0), s);
    launch_small_right(XT, nullptr, B(ws, "gov"), B(ws, "F"), nullptr, no, nv, part1, Yvv, s, t_xf32, t_p0, t_np);
  }
  log_phase("back");
  launch_singles_out(part1, no, nv, NO, NV, out->x1, s);
  DoublesRaw y;
  y.YvV = YvV; y.YvO = YvO; y.Yvv = Yvv;
  y.no = no; y.nv = nv; y.NO = NO; y.NV = NV; y.delta = 0;
  launch_doubles_out(y, out->x2_vVoo, out->x2_vvoO, s);
  HIPRT(hipGetLastError());
  log_phase("out");
}

// right transform of one vector (slot 0 of the prepared-vector buffers) in slabs of width w
void right_slabs(mlcc3_ws ws, const mlcc3_ground *g, const Dims &d, const mlcc3_vec &R, double omega, const Range &r,
                 int w, const mlcc3_out &rho, hipStream_t s) {
  const int no = d.no, nv = d.nv, NO = d.NO, NV = d.NV;
  group_dlhat(ws, g, d, &R, 1, s);
  right_vector_prep(ws, g, d, R, 0, 1, s);
  double *Ukc = B(ws, "Ukc"), *Xi = B(ws, "Xi");
  double *YvV = buf(ws, "YvV", (size_t)no * no * nv * NV, s);
  double *YvO = buf(ws, "YvO", (size_t)no * d.nv2 * NO, s);
  double *part1 = buf(ws, "part1", (size_t)no * no * nv, s);
  double *spare = buf(ws, "part1_tau", (size_t)no * no * nv, s);  // the tau~ pass's unused part1
  double *Yvv = buf(ws, "Yvv", (size_t)no * no * d.nv2, s);
  double *Xtau = buf(ws, "Xtau", (size_t)no * no * nv * NO, s);
  // tau~ pass: Xtau = sum tau~ g_Lbkc; YvO = -sum tau~ Xi; Yvv = sum tau~ Upsilon_kc
  const std::vector<int> off = slab_lists(ws, d, w, s);
  tau_xu_slabs(ws, g, d, r, w, off, s);
  log_phase("tau3");
  for (int p0 = 0; p0 < no; p0 += w) {
    SlabScope sc(ws, off, w, p0, std::min(w, no - p0));
    double *XT = contra_slab(ws, g, d, r, s);
    back_vV(ws, d, XT, B(ws, "gLb"), NO, Xtau, r, s);
    gemm(back_vO(d, XT, bm_jkcL(d, Xi), nullptr, BMap{}, YvO, -1.0), s);
    launch_small_right(XT, nullptr, B(ws, "gov"), Ukc, nullptr, no, nv, spare, Yvv, s, t_xf32, t_p0, t_np);
  }
  // R~ pass
  zero_xu(ws, d, s);
  for (int p0 = 0; p0 < no; p0 += w) {
    SlabScope sc(ws, off, w, p0, std::min(w, no - p0));
    build_R3(ws, g, d, &R, &omega, 1, r, nullptr, nullptr, s, 1);
  }
  log_phase("R3");
  for (int p0 = 0; p0 < no; p0 += w) {
    SlabScope sc(ws, off, w, p0, std::min(w, no - p0));
    double *XR = contra_slab(ws, g, d, r, s);
    back_vV(ws, d, XR, B(ws, "Gb1"), NV, YvV, r, s);
    Gemm bo = back_vO(d, XR, bm_jkcL(d, B(ws, "Gb3")), nullptr, BMap{}, YvO, -1.0);
    bo.beta = 1.0;
    gemm(bo, s);
    launch_small_right(XR, nullptr, B(ws, "gov"), B(ws, "F"), nullptr, no, nv, part1, Yvv, s, t_xf32, t_p0, t_np,
                       true);
  }
  log_phase("back");
  {  // Y^{aD}_{ij} -= sum_L Xtau[(i,j,a)][L] R^D_L
    Gemm gg;
    gg.M = no * no * nv;
    gg.N = NV;
    gg.C = YvV;
    gg.crow = plain(NV);
    gg.ccol = plain(1);
    gg.alpha = -1.0;
    gg.beta = 1.0;
    gg.nseg = 1;
    gg.seg[0] = seg(Xtau, plain(NO), plain(1), 0, R.x1, plain(1), plain(NO), 0, NO);
    gemm(gg, s);
  }
  launch_singles_out(part1, no, nv, NO, NV, rho.x1, s);
  DoublesRaw y;
  y.YvV = YvV; y.YvO = YvO; y.Yvv = Yvv;
  y.no = no; y.nv = nv; y.NO = NO; y.NV = NV; y.delta = 1;
  launch_doubles_out(y, rho.x2_vVoo, rho.x2_vvoO, s);
  HIPRT(hipGetLastError());
  log_phase("out");
}

// the triples contractions of the left transform of one vector in slabs of width w: QvV
// ("YvV"), QvO ("YvO"), Bq, Aq, Qtau and Xtau as the one-slab path forms them
void left_slabs(mlcc3_ws ws, const mlcc3_ground *g, const Dims &d, const mlcc3_vec &L, double omega, const Range &r,
                int w, hipStream_t s) {
  const int no = d.no, nv = d.nv, NO = d.NO, NV = d.NV;
  double *Xtau = buf(ws, "Xtau", (size_t)no * no * nv * NO, s);
  double *QvV = buf(ws, "YvV", (size_t)no * no * nv * NV, s);
  double *QvO = buf(ws, "YvO", (size_t)no * d.nv2 * NO, s);
  double *Bq = buf(ws, "Bq", (size_t)no * d.nv2 * NV, s);
  double *Aq = buf(ws, "Aq", (size_t)no * no * nv * NO, s);
  double *Qtau = buf(ws, "Qtau", (size_t)no * no * nv * NO, s);
  // tau~ pass: Xtau, and the partial products of Qtau per p
  const std::vector<int> off = slab_lists(ws, d, w, s);
  tau_xu_slabs(ws, g, d, r, w, off, s);
  log_phase("tau3");
  for (int p0 = 0; p0 < no; p0 += w) {
    SlabScope sc(ws, off, w, p0, std::min(w, no - p0));
    double *XT = contra_slab(ws, g, d, r, s);
    back_vV(ws, d, XT, B(ws, "gLb"), NO, Xtau, r, s);
    back_qrc(ws, d, XT, L.x2_vvoO, Qtau, s, "qrc_tau", false);
  }
  // L~ pass
  zero_xu(ws, d, s);
  for (int p0 = 0; p0 < no; p0 += w) {
    SlabScope sc(ws, off, w, p0, std::min(w, no - p0));
    build_L3(ws, g, d, &L, &omega, 1, r, nullptr, "LA", "LV", s, 1);
  }
  log_phase("L3");
  for (int p0 = 0; p0 < no; p0 += w) {
    SlabScope sc(ws, off, w, p0, std::min(w, no - p0));
    double *XL = contra_slab(ws, g, d, r, s);
    back_vV(ws, d, XL, B(ws, "G1t"), NV, QvV, r, s);
    gemm(back_vO(d, XL, BMap{B(ws, "G2"), plain(1), plain((long long)no * no * nv), 0}, nullptr, BMap{}, QvO, -1.0), s);
    form_Bq(ws, d, XL, Bq, s);
    back_qrc(ws, d, XL, g->t2_vvoO, Aq, s, "qrc_l", false);
  }
  log_phase("back");
  // the fixed-order sums over p of the partial products
  const long long MN = (long long)no * no * nv * NO;
  launch_sum_rows(B(ws, "qrc_l"), no, MN, Aq, s);
  launch_sum_rows(B(ws, "qrc_tau"), no, MN, Qtau, s);
  HIPRT(hipGetLastError());
}

// ------------------------------------------------------ density contractions
// C[k][l] = alpha sum_{(i,j),(abc)} X1[i][j][k][abc] X2[i][j][l][abc] + beta C
void g_kl(const Dims &d, const double *X1, const double *X2, double *C, long long ldc, double alpha, double beta,
          hipStream_t s) {
  if (d.no <= 16 && t_ws) {
    // small occupied output, K = n_o^2 n_v^3: the streaming MFMA Gram kernel
    int nch;
    long long chunk;
    gram_kl_shape(d.no, d.nv3, nch, chunk);
    const long long np = (long long)d.no * d.no * nch * d.no * d.no;
    double *P = buf(t_ws, "gram_part", (size_t)np, s);
    const size_t xb = sizeof(double) * (size_t)(d.nord * d.nv3);
    check_bytes(X1, xb, "X1 (occupied Gram)");
    check_bytes(X2, xb, "X2 (occupied Gram)");
    check_range(C, plain(ldc), d.no, plain(1), d.no, 0, 1, "C (occupied Gram)");
    launch_gram_kl(X1, X2, d.no, d.nv3, P, alpha, beta, C, ldc, s);
    HIPRT(hipGetLastError());
    return;
  }
  Gemm g = gemm_plain(d.no, d.no, C, plain(ldc), plain(1), alpha, beta);
  g.nseg = 1;
  g.seg[0] = seg(X1, plain(d.nv3), split((int)d.nv3, (long long)d.no * d.nv3, 1), 0, X2,
                 split((int)d.nv3, (long long)d.no * d.nv3, 1), plain(d.nv3), 0, (int)(d.no * d.no * d.nv3));
  gemm(g, s);
}
// C[c][d] = alpha sum_{(ijk,ab)} X1[ijk][ab][c] X2[ijk][ab][d] + beta C
void g_cd(const Dims &d, const double *X1, const double *X2, double *C, long long ldc, double alpha, double beta,
          hipStream_t s) {
  if (d.nv > 64 && d.nv <= 160 && t_ws) {
    // the whole n_v x n_v output per workgroup (the generic tiles would be half padding)
    const long long nrows = d.nord * d.nv2;
    const int nw = gram_cd_chunks(nrows);
    double *P = buf(t_ws, "gram_part", (size_t)nw * d.nv * d.nv, s);
    const size_t xb = sizeof(double) * (size_t)(d.nord * d.nv3);
    check_bytes(X1, xb, "X1 (virtual Gram)");
    check_bytes(X2, xb, "X2 (virtual Gram)");
    check_range(C, plain(ldc), d.nv, plain(1), d.nv, 0, 1, "C (virtual Gram)");
    launch_gram_cd(X1, X2, d.nv, nrows, P, alpha, beta, C, ldc, s);
    HIPRT(hipGetLastError());
    return;
  }
  Gemm g = gemm_plain(d.nv, d.nv, C, plain(ldc), plain(1), alpha, beta);
  g.nseg = 1;
  g.seg[0] = seg(X1, plain(1), plain(d.nv), 0, X2, plain(d.nv), plain(1), 0, (int)(d.nord * d.nv2));
  gemm(g, s);
}
// out[(l,d)] = alpha sum_{(ij),(ab)} X[i][j][l][ab][d] Y[i][j][a][b] + beta out; out row map given
void g_ld(const Dims &d, const double *X, const double *Y, double *C, Idx2 crow, double alpha, double beta,
          hipStream_t s) {
  Gemm g = gemm_plain(d.no * d.nv, 1, C, crow, plain(1), alpha, beta);
  g.nseg = 1;
  g.seg[0] = seg(X, split(d.nv, d.nv3, 1), split((int)d.nv2, (long long)d.no * d.nv3, d.nv), 0, Y, plain(1),
                 plain(1), 0, (int)(d.no * d.no * d.nv2));
  gemm(g, s);
}
// run g over its nbatch batches into partial buffers and sum them (fixed order) into g's output
void gemm_sumz(mlcc3_ws ws, const Gemm &g, hipStream_t s) {
  const long long MN = (long long)g.M * g.N;
  double *P = buf(ws, "sumz_part", (size_t)(MN * g.nbatch), s);
  Gemm h = g;
  h.C = P;
  h.crow = plain(g.N);
  h.ccol = plain(1);
  h.cbatch = MN;
  h.alpha = 1.0;
  h.beta = 0.0;
  gemm(h, s);
  Gemm r = g;
  r.ksplit = g.nbatch;
  r.nbatch = 1;
  r.P = P;
  r.cbatch = 0;
  check_range(r.C, r.crow, r.M, r.ccol, r.N, 0, 1, "C");
  HIPRT(gemm_reduce_parts(r, s));
}
// V[(j,k,b)][L] = sum_{i,(a,c)} X[i][j][k][a][b][c] Y[a][c][i][L]   (Y in the [a][b][i][L] block layout)
void v_jkbL(mlcc3_ws ws, const Dims &d, const double *X, const double *Y, double *V, hipStream_t s) {
  Gemm g = gemm_plain(d.no * d.no * d.nv, d.NO, V, plain(d.NO), plain(1), 1.0, 0.0);
  g.nbatch = d.no;
  g.nseg = 1;
  g.seg[0] = seg(X, split(d.nv, d.nv3, d.nv), split(d.nv, d.nv2, 1), (long long)d.no * d.no * d.nv3, Y,
                 plain((long long)d.no * d.NO), plain(1), d.NO, (int)d.nv2);
  gemm_sumz(ws, g, s);
}
// D[L][N_O + D] += alpha sum_{kk} V[kk][L] T[kk][D]  (K = n_o^2 n_v; T [(.,.,.)][N_V])
void d_LD(const Dims &d, const double *V, const double *T, double *Dm, long long N, double alpha, hipStream_t s) {
  Gemm g = gemm_plain(d.NO, d.NV, Dm + d.NO, plain(N), plain(1), alpha, 1.0);
  g.nseg = 1;
  g.seg[0] = seg(V, plain(1), plain(d.NO), 0, T, plain(d.NV), plain(1), 0, d.no * d.no * d.nv);
  gemm(g, s);
}

}  // namespace

// =================================================================== C-ABI
extern "C" {

void mlcc3_opts_default(mlcc3_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = MLCC3_FP64;
  o->triple_begin = 0;
  o->triple_end = -1;
}

int64_t mlcc3_num_triples(int32_t n_o) {
  const long long n = n_o < 0 ? 0 : n_o;
  return n * (n + 1) * (n + 2) / 6 - n;
}

// workspace of a call: the caller's, or (NULL) a temporary one on the current device that is
// destroyed, after the device has finished the call's work, when the call returns
struct CallWs {
  mlcc3_ws ws = nullptr;
  bool own = false;
  explicit CallWs(mlcc3_ws w) {
    if (w) {
      ws = w;
      return;
    }
    int dev = 0;
    if (!g_dry) HIPRT(hipGetDevice(&dev));
    ws = new mlcc3_ws_s();
    ws->device = dev;
    own = true;
  }
  ~CallWs() {
    if (!own) return;
    if (t_ws == ws) t_ws = nullptr;
    (void)mlcc3_ws_destroy(ws);
  }
  CallWs(const CallWs &) = delete;
  CallWs &operator=(const CallWs &) = delete;
};

int mlcc3_ws_create(mlcc3_ws *ws, int device) {
  return guarded([&] {
    check(ws != nullptr, "ws is NULL");
    int n = 1;
    HIPRT(hipGetDeviceCount(&n));
    check(device >= 0 && device < n, "bad device ordinal");
    *ws = new mlcc3_ws_s();
    (*ws)->device = device;
  });
}

int mlcc3_ws_destroy(mlcc3_ws ws) {
  return guarded([&] {
    if (!ws) return;
    if (!g_dry) {
      DeviceGuard dg(ws->device);
      HIPCHK(hipDeviceSynchronize());
      for (auto &kv : ws->bufs)
        if (kv.second.first) (void)hipFree(kv.second.first);
      for (auto &m : ws->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
      }
      for (auto e : ws->pool) (void)hipEventDestroy(e);
    }
    delete ws;
  });
}

int64_t mlcc3_ws_bytes(mlcc3_ws ws) { return ws ? ws->total : 0; }

int mlcc3_ws_timing(mlcc3_ws ws, int32_t enable) {
  return guarded([&] {
    check(ws != nullptr, "ws is NULL");
    ws->timing = enable != 0;
    if (!g_dry)
      for (auto &m : ws->marks) {
        ws->pool.push_back(m.a);
        ws->pool.push_back(m.b);
      }
    ws->marks.clear();
  });
}

int mlcc3_ws_set_tuning(mlcc3_ws ws, const mlcc3_tuning *t) {
  return guarded([&] {
    check(ws != nullptr, "ws is NULL");
    mlcc3_tuning z{};
    if (!t) {
      ws->tune = z;
      return;
    }
    check(t->dc_wg_per_cu == -1 || (t->dc_wg_per_cu >= 0 && t->dc_wg_per_cu <= 8), "dc_wg_per_cu out of range");
    check(t->back_ksplit >= 0 && t->back_ksplit <= 8, "back_ksplit out of range");
    const int tm = t->narrow_tile / 10, tn = t->narrow_tile % 10;
    auto ok = [](int x) { return x == 1 || x == 2 || x == 4; };
    check(t->narrow_tile == 0 || (t->narrow_tile < 100 && ok(tm) && ok(tn)), "narrow_tile must be 10*TM+TN, TM,TN in {1,2,4}");
    check(t->contra_form >= 0 && t->contra_form <= 2, "contra_form out of range");
    check(t->vec_group >= 0, "vec_group < 0");
    check(t->occ_slab >= 0, "occ_slab < 0");
    ws->tune = *t;
  });
}

int mlcc3_ws_get_tuning(mlcc3_ws ws, mlcc3_tuning *t) {
  return guarded([&] {
    check(ws != nullptr && t != nullptr, "NULL argument");
    *t = ws->tune;
  });
}

int mlcc3_ws_phase_stats(mlcc3_ws ws, int32_t phase, int64_t *launches, double *total_ms, double *flops) {
  return guarded([&] {
    check(ws && launches && total_ms && flops, "NULL argument");
    *launches = 0;
    *total_ms = 0.0;
    *flops = 0.0;
    for (auto &m : ws->marks) {
      if (m.phase != phase) continue;
      float ms = 0.f;
      if (!g_dry) {
        HIPCHK(hipEventSynchronize(m.b));
        HIPCHK(hipEventElapsedTime(&ms, m.a, m.b));
      }
      *launches += 1;
      *total_ms += ms;
      *flops += m.flops;
    }
  });
}

int mlcc3_oscillator_strengths(mlcc3_ws ws, int32_t N, int32_t ncomp, const double *A, int32_t nstate,
                               const double *omega, const double *D_m0, const double *D_0m, const double *D_00,
                               const double *s, double *T_m0, double *T_0m, double *f, void *stream) {
  return guarded([&] {
    CallWs call_ws(ws);  // NULL: a temporary workspace for this call
    ws = call_ws.ws;
    check(N >= 1 && ncomp >= 1 && nstate >= 1, "need N, ncomp, nstate >= 1");
    check(A && omega && D_m0 && D_0m && D_00 && s && T_m0 && T_0m && f, "NULL argument");
    for (int m = 0; m < nstate; m++) check(std::isfinite(omega[m]), "omega must be finite");
    t_ws = ws;
    hipStream_t st = (hipStream_t)stream;
    DeviceGuard dg(ws->device);
    double *om = buf(ws, "omega_dev", (size_t)nstate, st);
    if (!g_dry) HIPRT(hipMemcpyAsync(om, omega, sizeof(double) * nstate, hipMemcpyHostToDevice, st));
    launch_strengths(A, N, ncomp, nstate, D_m0, D_0m, D_00, s, om, T_m0, T_0m, f, st);
    HIPRT(hipGetLastError());
    // the host array omega may be released when the call returns
    if (!g_dry) HIPRT(hipStreamSynchronize(st));
  });
}

int mlcc3_vec_map(mlcc3_ws ws, const mlcc3_ground *g, int32_t mode, int32_t nvec, const mlcc3_vec *in,
                  mlcc3_out *out, void *stream) {
  return guarded([&] {
    CallWs call_ws(ws);  // NULL: a temporary workspace for this call
    ws = call_ws.ws;
    check(g != nullptr, "ground is NULL");
    check(g->N_O >= 1 && g->N_V >= 1 && g->n_o >= 0 && g->n_o <= g->N_O && g->n_v >= 0 && g->n_v <= g->N_V,
          "bad dimensions");
    check(mode >= MLCC3_MAP_SYMMETRIZE && mode <= MLCC3_MAP_LEFT_TO_GRAD, "bad mode");
    check(nvec >= 1 && in && out, "need nvec >= 1 and non-NULL vector arrays");
    const bool act = g->n_o > 0 && g->n_v > 0;
    for (int m = 0; m < nvec; m++) {
      check(in[m].x1 && (!act || (in[m].x2_vVoo && in[m].x2_vvoO)), "NULL pointer in an input vector");
      check(out[m].x1 && (!act || (out[m].x2_vVoo && out[m].x2_vvoO)), "NULL pointer in an output vector");
      check(in[m].x2_vVoo != out[m].x2_vVoo && in[m].x2_vvoO != out[m].x2_vvoO, "outputs must not alias inputs");
    }
    hipStream_t s = (hipStream_t)stream;
    DeviceGuard dg(ws->device);
    const long long n1 = (long long)g->N_V * g->N_O;
    for (int m = 0; m < nvec; m++) {
      if (!g_dry && in[m].x1 != out[m].x1)
        HIPRT(hipMemcpyAsync(out[m].x1, in[m].x1, n1 * sizeof(double), hipMemcpyDeviceToDevice, s));
      if (act) {
        launch_vec_map(in[m].x2_vVoo, in[m].x2_vvoO, g->n_o, g->n_v, g->N_O, g->N_V, mode, out[m].x2_vVoo,
                       out[m].x2_vvoO, s);
        HIPRT(hipGetLastError());
      }
    }
  });
}

double mlcc3_flops(const mlcc3_ground *g, int32_t which, int32_t nvec) {
  if (!g) return 0.0;
  const double no = g->n_o, nv = g->n_v, NV = g->N_V;
  const double U = 2.0 * NV * nv * nv * nv * (no * no * no - no);
  if (which == 0) return 2.0 * U;
  return (1.0 + 3.0 * std::max(nvec, 1)) * U;
}

namespace {

// the ground residual on workspace ws (the caller's, a temporary one, or an arena)
void ground_residual_call(mlcc3_ws ws, const mlcc3_ground *g, const mlcc3_opts *opts, mlcc3_out *out, void *stream) {
  t_ws = ws;
  t_stream = (hipStream_t)stream;
  validate_ground(g);
  validate_out(g, out);
  reg_ground(g);
  reg_vec(g, out->x1, out->x2_vVoo, out->x2_vvoO);
  const mlcc3_opts o = opts_or_default(opts);
  check(!o.cvs_core, "core-valence separation applies to the right and left transforms only");
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ws->device);
  const Dims d = dims_of(g);
  log_begin("ground_residual", s, d.no, d.nv, d.NO, d.NV, d.nc, 0, o.precision);
  const Range r = range_of(o, mlcc3_num_triples(d.no));
  if (o.check_finite) ground_finite(ws, g, s);
  if (d.no < 2 || d.nv < 2 || r.tb == r.te) {  // CCSD reduction: triples terms vanish
    zero_out(d, out, s);
    return;
  }
  prepare_ground(ws, g, o.reuse_ground != 0, s);
  log_phase("prep");
  if (const int slab = slab_width(ws, d)) {  // occupied slabs
    ws->tau = mlcc3_ws_s::TauKey{};
    ground_slabs(ws, g, d, r, slab, out, s);
    return;
  }
  tau_path(ws, g, d, r, s, nullptr, o.reuse_tau != 0);
  log_phase("tau3");
  double *XT = B(ws, "XT");
  double *YvV = buf(ws, "YvV", (size_t)d.no * d.no * d.nv * d.NV, s);
  double *YvO = buf(ws, "YvO", (size_t)d.no * d.nv2 * d.NO, s);
  back_vV(ws, d, XT, B(ws, "Gb1"), d.NV, YvV, r, s);
  log_phase("back");
  gemm(back_vO(d, XT, bm_jkcL(d, B(ws, "Gb3")), nullptr, BMap{}, YvO, -1.0), s);
  finish_right_like(ws, d, XT, nullptr, nullptr, YvV, YvO, 0, out, s);
  log_phase("out");
}

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// device address of this device's scratch (the device must be current)
void *scratch_address(int dev) {
  check(dev >= 0 && dev < kMaxDevices, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    check(p != nullptr, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}

}  // namespace

int mlcc3_ground_residual(mlcc3_ws ws, const mlcc3_ground *g, const mlcc3_opts *opts, mlcc3_out *out,
                          void *stream) {
  return guarded([&] {
    CallWs call_ws(ws);  // NULL: a temporary workspace for this call
    ground_residual_call(call_ws.ws, g, opts, out, stream);
  });
}

int64_t mlcc3_noalloc_scratch_bytes(void) { return (int64_t)kScratchBytes; }

int mlcc3_ground_residual_noalloc(const mlcc3_ground *g, const mlcc3_opts *opts, mlcc3_out *out, void *stream) {
  return guarded([&] {
    validate_ground(g);
    validate_out(g, out);
    check(!opts || !opts->reuse_ground, "reuse_ground needs a workspace");
    check(!opts || !opts->reuse_tau, "reuse_tau needs a workspace");
    int dev = 0;
    if (!g_dry) HIPCHK(hipGetDevice(&dev));
    // 1. size: the same orchestration with no device work, carving fake addresses
    size_t need = 0;
    {
      const bool dry = g_dry;
      mlcc3_ws_s probe;
      probe.device = dev;
      probe.arena = true;
      probe.arena_base = (uintptr_t)1 << 44;
      probe.arena_cap = (size_t)1 << 42;
      g_dry = true;
      try {
        ground_residual_call(&probe, g, opts, out, stream);
      } catch (...) {
        g_dry = dry;
        t_ws = nullptr;
        throw;
      }
      g_dry = dry;
      t_ws = nullptr;
      need = probe.arena_used;
    }
    if (need > kScratchBytes)
      throw Status{MLCC3_EINVAL, "problem needs " + std::to_string(need) + " bytes of scratch; the fixed scratch of "
                                     "mlcc3_ground_residual_noalloc holds " + std::to_string(kScratchBytes)};
    // 2. run on the device's fixed scratch
    t_ext.clear();
    mlcc3_ws_s ws;
    ws.device = dev;
    ws.arena = true;
    ws.arena_cap = kScratchBytes;
    if (g_dry) {
      ws.arena_base = (uintptr_t)1 << 44;
    } else {
      DeviceGuard dg(dev);
      ws.arena_base = (uintptr_t)scratch_address(dev);
    }
    try {
      ground_residual_call(&ws, g, opts, out, stream);
    } catch (...) {
      t_ws = nullptr;
      throw;
    }
    t_ws = nullptr;
  });
}

int mlcc3_right_transform(mlcc3_ws ws, const mlcc3_ground *g, int32_t nvec, const double *omega,
                          const mlcc3_vec *R, mlcc3_out *rho, const mlcc3_opts *opts, void *stream) {
  return guarded([&] {
    CallWs call_ws(ws);  // NULL: a temporary workspace for this call
    ws = call_ws.ws;
    t_ws = ws;
    t_stream = (hipStream_t)stream;
    validate_ground(g);
    validate_vecs(g, nvec, omega, R, rho);
    reg_ground(g);
    for (int m = 0; m < nvec; m++) {
      reg_vec(g, R[m].x1, R[m].x2_vVoo, R[m].x2_vvoO);
      reg_vec(g, rho[m].x1, rho[m].x2_vVoo, rho[m].x2_vvoO);
    }
    const mlcc3_opts o = opts_or_default(opts);
    hipStream_t s = (hipStream_t)stream;
    DeviceGuard dg(ws->device);
    const Dims d = dims_of(g);
    log_begin("right_transform", s, d.no, d.nv, d.NO, d.NV, d.nc, nvec, o.precision);
    const Range r = range_of(o, mlcc3_num_triples(d.no));
    if (o.check_finite) {
      ground_finite(ws, g, s);
      for (int m = 0; m < nvec; m++) vec_finite(ws, d, R[m], s);
    }
    guard_check(g, omega, nvec, o.guard, s);
    if (d.no < 2 || d.nv < 2 || r.tb == r.te) {
      for (int m = 0; m < nvec; m++) zero_out(d, &rho[m], s);
      return;
    }
    // core-valence separation: projected copies of the inputs, all-valence triples skipped
    std::vector<mlcc3_vec> Rp;
    const mlcc3_vec *R_in = R;
    cvs_setup(ws, g, o, nvec, R_in, &Rp, s);
    const mlcc3_vec *R = Rp.empty() ? R_in : Rp.data();
    prepare_ground(ws, g, o.reuse_ground != 0, s);
    log_phase("prep");
    const int no = d.no, nv = d.nv, NO = d.NO, NV = d.NV;
    if (const int slab = slab_width(ws, d)) {  // occupied slabs, vector by vector
      ws->tau = mlcc3_ws_s::TauKey{};
      for (int m = 0; m < nvec; m++) {
        right_slabs(ws, g, d, R[m], omega[m], r, slab, rho[m], s);
        cvs_project_out(d, rho[m], s);
      }
      return;
    }
    // tau~ and Xtau[(i,j,a)][L] = sum tau~ g_Lbkc (shared by all vectors)
    const bool tau_kept = tau_path(ws, g, d, r, s, nullptr, o.reuse_tau != 0);
    log_phase("tau3");
    double *XT = B(ws, "XT");
    double *Xtau = xtau_block(ws, d, XT, tau_kept, r, s);
    // vectors in groups: R3 of a whole group in one d-contraction launch and one launch per
    // permutation pass, then the back-contractions vector by vector
    const int ng = group_size(ws, d, nvec);
    const RightSizes z = right_sizes(d);
    for (int m0 = 0; m0 < nvec; m0 += ng) {
      const int nb = std::min(ng, nvec - m0);
      double *XRg = wx_buffer(ws, d, nb, s);  // R~ of the group overwrites its W
      group_dlhat(ws, g, d, R + m0, nb, s);
      for (int v = 0; v < nb; v++) right_vector_prep(ws, g, d, R[m0 + v], v, nb, s);
      build_R3(ws, g, d, R + m0, omega + m0, nb, r, XRg, nullptr, s);
      log_phase("R3");
      for (int v = 0; v < nb; v++) {
        const int m = m0 + v;
        double *XR = xsub(XRg, v * xpitch(d.nord * d.nv3));
        double *Ukc = B(ws, "Ukc") + v * z.Ukc, *Xi = B(ws, "Xi") + v * z.Xi;
        // back-contractions
        double *YvV = buf(ws, "YvV", (size_t)no * no * nv * NV, s);
        double *YvO = buf(ws, "YvO", (size_t)no * d.nv2 * NO, s);
        back_vV(ws, d, XR, B(ws, "Gb1"), NV, YvV, r, s);
        log_phase("back");
        {  // Y^{aD}_{ij} -= sum_L Xtau[(i,j,a)][L] R^D_L
          Gemm gg;
          gg.M = no * no * nv;
          gg.N = NV;
          gg.C = YvV;
          gg.crow = plain(NV);
          gg.ccol = plain(1);
          gg.alpha = -1.0;
          gg.beta = 1.0;
          gg.nseg = 1;
          gg.seg[0] = seg(Xtau, plain(NO), plain(1), 0, R[m].x1, plain(1), plain(NO), 0, NO);
          gemm(gg, s);
        }
        gemm(back_vO(d, XR, bm_jkcL(d, B(ws, "Gb3")), XT, bm_jkcL(d, Xi), YvO, -1.0), s);
        finish_right_like(ws, d, XR, XT, Ukc, YvV, YvO, 1, &rho[m], s);
        log_phase("out");
        cvs_project_out(d, rho[m], s);
      }
    }
  });
}

int mlcc3_left_transform(mlcc3_ws ws, const mlcc3_ground *g, int32_t nvec, const double *omega,
                         const mlcc3_vec *L, mlcc3_out *sigma, const mlcc3_opts *opts, void *stream) {
  return guarded([&] {
    CallWs call_ws(ws);  // NULL: a temporary workspace for this call
    ws = call_ws.ws;
    t_ws = ws;
    t_stream = (hipStream_t)stream;
    validate_ground(g);
    validate_vecs(g, nvec, omega, L, sigma);
    reg_ground(g);
    for (int m = 0; m < nvec; m++) {
      reg_vec(g, L[m].x1, L[m].x2_vVoo, L[m].x2_vvoO);
      reg_vec(g, sigma[m].x1, sigma[m].x2_vVoo, sigma[m].x2_vvoO);
    }
    const mlcc3_opts o = opts_or_default(opts);
    hipStream_t s = (hipStream_t)stream;
    DeviceGuard dg(ws->device);
    const Dims d = dims_of(g);
    log_begin("left_transform", s, d.no, d.nv, d.NO, d.NV, d.nc, nvec, o.precision);
    const Range r = range_of(o, mlcc3_num_triples(d.no));
    if (o.check_finite) {
      ground_finite(ws, g, s);
      for (int m = 0; m < nvec; m++) vec_finite(ws, d, L[m], s);
    }
    guard_check(g, omega, nvec, o.guard, s);
    if (d.no < 2 || d.nv < 2 || r.tb == r.te) {
      for (int m = 0; m < nvec; m++) zero_out(d, &sigma[m], s);
      return;
    }
    // core-valence separation: projected copies of the inputs, all-valence triples skipped
    std::vector<mlcc3_vec> Lp;
    const mlcc3_vec *L_in = L;
    cvs_setup(ws, g, o, nvec, L_in, &Lp, s);
    const mlcc3_vec *L = Lp.empty() ? L_in : Lp.data();
    prepare_ground(ws, g, o.reuse_ground != 0, s);
    log_phase("prep");
    const int no = d.no, nv = d.nv, NO = d.NO, NV = d.NV, nc = d.nc;
    double *LhOO = B(ws, "LhOO"), *LhvV = B(ws, "LhvV"), *LhvO = B(ws, "LhvO");
    const double *gLE = gle_block(ws, g, d, s);
    // the singles of sigma and the output gather, from the triples contractions of vector m:
    // QvV, QvO (doubles), Bq, Aq, Qtau, Xtau
    auto assemble = [&](int m, const double *LA, double *QvV, double *QvO, double *Bq, double *Aq, double *Qtau,
                        const double *Xtau) {
      double *V = buf(ws, "Vkc", (size_t)no * nv, s);  // V_kc = sum tau~ L^{ab}_{ij} = sum_q Qtau[q][k][c][q]
      launch_diag_sum(Qtau, no, nv, NO, V, s);
      HIPRT(hipGetLastError());
      double *s1 = sigma[m].x1;
      HIPRT(hipMemsetAsync(s1, 0, sizeof(double) * NV * NO, s));
      // (i) sigma^D_L += sum_kc V_kc (2 g_kcLD - g_kDLc) = sum_J [2 s_J L_LD - sum_k L_kD u_J[k][L]]
      {
        double *sJ = buf(ws, "vs_J", (size_t)nc, s);
        double *uJ = buf(ws, "vu_J", (size_t)nc * no * NO, s);
        // s_J = sum_kc V_kc L^J_kc  (A: [J][(k,c)] from L_OV)
        Gemm g1 = gemm_plain(nc, 1, sJ, plain(1), plain(1), 1.0, 0.0);
        g1.nseg = 1;
        g1.seg[0] = seg(g->L_OV, plain((long long)NO * NV), split(nv, NV, 1), 0, V, plain(1), plain(1), 0, no * nv);
        gemm(g1, s);
        // u_J[k][L] = sum_c L_OV[J][L][c] V[k][c]   (rows (J,L))
        Gemm g3 = gemm_plain(nc * NO, no, uJ, split(NO, (long long)no * NO, 1), plain(NO), 1.0, 0.0);
        g3.nseg = 1;
        g3.seg[0] = seg(g->L_OV, plain(NV), plain(1), 0, V, plain(1), plain(nv), 0, nv);
        gemm(g3, s);
        // sigma[D][L] += 2 sum_J L_OV[J][L][D] s_J   (rows (L,D))
        Gemm g4 = gemm_plain(NO * NV, 1, s1, split(NV, 1, NO), plain(0), 2.0, 1.0);
        g4.nseg = 1;
        g4.seg[0] = seg(g->L_OV, plain(1), plain((long long)NO * NV), 0, sJ, plain(1), plain(1), 0, nc);
        gemm(g4, s);
        // sigma[D][L] -= sum_{(J,k)} L_OV[J][k][D] u_J[k][L]
        Gemm g5 = gemm_plain(NV, NO, s1, plain(NO), plain(1), -1.0, 1.0);
        g5.nseg = 1;
        g5.seg[0] = seg(g->L_OV, plain(1), split(no, (long long)NO * NV, NV), 0, uJ, plain(NO), plain(1), 0, nc * no);
        gemm(g5, s);
      }
      // (ii) sigma^D_L -= sum L^{aD}_{ij} Xtau[(i,j,a)][L] ; (iii) -= sum g_jDkc Qtau[(j,k,c)][L]
      {
        Gemm gg = gemm_plain(NV, NO, s1, plain(NO), plain(1), -1.0, 1.0);
        gg.nseg = 2;
        gg.seg[0] = seg(LA, plain(1), plain(NV), 0, Xtau, plain(NO), plain(1), 0, no * no * nv);
        gg.seg[1] = seg(B(ws, "gDo"), plain(1), plain(NV), 0, Qtau, plain(NO), plain(1), 0, no * no * nv);
        gemm(gg, s);
      }
      // (iv) sigma^D_l += sum_{J,c} Lh_cD (Hp - H2)[l][J][c] - sum_{J,M} L_MD H3[l][J][M]
      double *Hp = buf(ws, "Hp", (size_t)no * nc * nv, s);
      double *H2 = buf(ws, "H2", (size_t)no * nc * nv, s);
      double *H3 = buf(ws, "H3", (size_t)no * nc * NO, s);
      {
        // Hp[l][J][c] = sum_{(b,E)} Lh_bE Bq[l][b][c][E]
        Gemm gg = gemm_plain(nc, nv, Hp, plain(nv), plain(1), 1.0, 0.0);
        gg.nbatch = no;
        gg.cbatch = (long long)nc * nv;
        gg.nseg = 1;
        gg.seg[0] = seg(LhvV, plain((long long)nv * NV), plain(1), 0, Bq, split(NV, (long long)nv * NV, 1), plain(NV),
                        d.nv2 * NV, nv * NV);
        gemm(gg, s);
        // H2[l][J][c] = sum_{(j,M)} Lh_Mj Aq[j][l][c][M]
        Gemm g2 = gemm_plain(nc, nv, H2, plain(nv), plain(1), 1.0, 0.0);
        g2.nbatch = no;
        g2.cbatch = (long long)nc * nv;
        g2.nseg = 1;
        g2.seg[0] = seg(LhOO, plain((long long)NO * NO), split(NO, 1, NO), 0, Aq,
                        split(NO, (long long)no * nv * NO, 1), plain(NO), (long long)nv * NO, no * NO);
        gemm(g2, s);
        // H3[l][J][M] = sum_{(k,c)} Lh_ck Aq[l][k][c][M]
        Gemm g3 = gemm_plain(nc, NO, H3, plain(NO), plain(1), 1.0, 0.0);
        g3.nbatch = no;
        g3.cbatch = (long long)nc * NO;
        g3.nseg = 1;
        g3.seg[0] = seg(LhvO, plain((long long)nv * NO), split(nv, 1, NO), 0, Aq, plain(NO), plain(1),
                        (long long)no * nv * NO, no * nv);
        gemm(g3, s);
        // sigma[D][l] += sum Lh_cD (Hp - H2)
        Gemm g4 = gemm_plain(NV, no, s1, plain(NO), plain(1), 1.0, 1.0);
        g4.nseg = 2;
        g4.seg[0] = seg(LhvV, plain(1), plain(NV), 0, Hp, plain(1), plain((long long)nc * nv), 0, nc * nv);
        g4.seg[1] = seg(LhvV, plain(1), plain(NV), 0, H2, plain(1), plain((long long)nc * nv), 0, nc * nv, -1.0);
        gemm(g4, s);
        // sigma[D][l] -= sum L_MD H3
        Gemm g5 = gemm_plain(NV, no, s1, plain(NO), plain(1), -1.0, 1.0);
        g5.nseg = 1;
        g5.seg[0] = seg(g->L_OV, plain(1), plain(NV), 0, H3, plain(1), plain((long long)nc * NO), 0, nc * NO);
        gemm(g5, s);
      }
      // (v) sigma^d_L += sum_{J,k} Lh_Lk Z[J][k][d] - sum_{J,E} L_LE sum_{(k,c)} Lh_ck Bq[k][d][c][E];
      //     the second term is taken as sum_{(k,c,E)} Bq[k][d][c][E] ghat_ckLE (gLE, formed once
      //     per ground state) instead of through the rank x n_v N_V intermediate
      {
        double *Am = buf(ws, "Am", (size_t)no * nc * no * nv, s);
        double *Z = buf(ws, "Zl", (size_t)nc * no * nv, s);
        // Am[j][J][(k,d)] = sum_M Lh_Mj Aq[j][k][d][M]
        Gemm g1 = gemm_plain(nc, no * nv, Am, plain((long long)no * nv), plain(1), 1.0, 0.0);
        g1.nbatch = no;
        g1.cbatch = (long long)nc * no * nv;
        g1.nseg = 1;
        g1.seg[0] = seg(LhOO, plain((long long)NO * NO), plain(NO), 1, Aq, plain(1), plain(NO),
                        (long long)no * nv * NO, NO);
        gemm(g1, s);
        launch_left_Z(Am, Hp, nc, no, nv, Z, s);
        HIPRT(hipGetLastError());
        // sigma[d][L] += sum_{(J,k)} Z[J][k][d] Lh_Lk - sum_{(k,c,E)} Bq[k][d][c][E] gLE[k][c][L][E]
        Gemm g3 = gemm_plain(nv, NO, s1, plain(NO), plain(1), 1.0, 1.0);
        g3.nseg = 2;
        g3.seg[0] = seg(Z, plain(1), plain(nv), 0, LhOO, split(no, (long long)NO * NO, 1), plain(NO), 0, nc * no);
        g3.seg[1] = seg(Bq, plain((long long)nv * NV), split(nv * NV, d.nv2 * NV, 1), 0, gLE,
                        split(NV, (long long)NO * NV, 1), plain(NV), 0, no * nv * NV, -1.0);
        gemm(g3, s);
      }
      DoublesRaw y;
      y.YvV = QvV; y.YvO = QvO; y.Yvv = nullptr;
      y.no = no; y.nv = nv; y.NO = NO; y.NV = NV; y.delta = 0;
      launch_doubles_out(y, sigma[m].x2_vVoo, sigma[m].x2_vvoO, s);
      HIPRT(hipGetLastError());
      cvs_project_out(d, sigma[m], s);
    };
    const int slab = slab_width(ws, d);
    if (slab > 0) {  // occupied slabs, vector by vector
      ws->tau = mlcc3_ws_s::TauKey{};
      for (int m = 0; m < nvec; m++) {
        left_slabs(ws, g, d, L[m], omega[m], r, slab, s);
        assemble(m, B(ws, "LA"), B(ws, "YvV"), B(ws, "YvO"), B(ws, "Bq"), B(ws, "Aq"), B(ws, "Qtau"), B(ws, "Xtau"));
      }
      return;
    }
    const bool tau_kept = tau_path(ws, g, d, r, s, nullptr, o.reuse_tau != 0);
    log_phase("tau3");
    double *XT = B(ws, "XT");
    double *Xtau = xtau_block(ws, d, XT, tau_kept, r, s);
    // vectors in groups: L3 of a whole group in one d-contraction launch and one launch per
    // permutation pass, then the back-contractions vector by vector
    const int ng = group_size(ws, d, nvec);
    const long long sLA = (long long)no * no * nv * NV;
    for (int m0 = 0; m0 < nvec; m0 += ng) {
      const int nb = std::min(ng, nvec - m0);
      double *XLg = wx_buffer(ws, d, nb, s);  // L~ of the group overwrites its W
      // L3 (SI transpose transformation, exact-transpose index placement):
      //   sum_D L^{aD}_{ij} g_Dbkc - sum_L L^{ab}_{iL} g_jLkc + local terms
      build_L3(ws, g, d, L + m0, omega + m0, nb, r, XLg, "LA", "LV", s);
      log_phase("L3");
      for (int v = 0; v < nb; v++) {
        const int m = m0 + v;
        const double *L2b = L[m].x2_vvoO;
        double *XL = xsub(XLg, v * xpitch(d.nord * d.nv3));
        double *LA = B(ws, "LA") + v * sLA;
        // doubles: sigma^{aD}_{ij} <- sum L~ g_bDck ; sigma^{ab}_{iL} <- -sum L~ g_Ljck
        double *QvV = buf(ws, "YvV", (size_t)no * no * nv * NV, s);
        double *QvO = buf(ws, "YvO", (size_t)no * d.nv2 * NO, s);
        back_vV(ws, d, XL, B(ws, "G1t"), NV, QvV, r, s);
        log_phase("back");
        gemm(back_vO(d, XL, BMap{B(ws, "G2"), plain(1), plain((long long)no * no * nv), 0}, nullptr, BMap{}, QvO, -1.0),
             s);
        // intermediates of the singles
        double *Bq = buf(ws, "Bq", (size_t)no * d.nv2 * NV, s);
        form_Bq(ws, d, XL, Bq, s);
        // Aq[(q,r,c)][M] = sum L~[p][q][r][a][b][c] t^{ab}_{pM};  Qtau likewise with tau~ and L^{ab}_{pL}
        double *Aq = buf(ws, "Aq", (size_t)no * no * nv * NO, s);
        double *Qtau = buf(ws, "Qtau", (size_t)no * no * nv * NO, s);
        back_qrc(ws, d, XL, g->t2_vvoO, Aq, s);
        back_qrc(ws, d, XT, L2b, Qtau, s);
        assemble(m, LA, QvV, QvO, Bq, Aq, Qtau, Xtau);
      }
    }
  });
}


int mlcc3_triples_densities(mlcc3_ws ws, const mlcc3_ground *g, const double *t2_vVoO, const double *t2_vVOo,
                            int32_t nstate, const double *omega, const mlcc3_vec *L, const mlcc3_vec *R,
                            const mlcc3_vec *lambda, double *D_m0, double *D_0m, double *s_out,
                            const mlcc3_opts *opts, void *stream) {
  return guarded([&] {
    CallWs call_ws(ws);  // NULL: a temporary workspace for this call
    ws = call_ws.ws;
    t_ws = ws;
    t_stream = (hipStream_t)stream;
    validate_ground(g);
    check(nstate >= 1, "nstate must be >= 1");
    check(omega && L && R && lambda && D_m0 && D_0m && s_out, "NULL argument");
    const Dims d = dims_of(g);
    const long long N = (long long)d.NO + d.NV;
    const bool act = d.no > 0 && d.nv > 0;
    check(!act || (t2_vVoO && t2_vVOo), "NULL density t2 block");
    std::vector<mlcc3_out> dummy(nstate);
    for (int m = 0; m < nstate; m++) {
      check(std::isfinite(omega[m]), "omega must be finite");
      check(L[m].x1 && R[m].x1 && (!act || (L[m].x2_vVoo && L[m].x2_vvoO && R[m].x2_vVoo && R[m].x2_vvoO)),
            "NULL pointer in a vector");
    }
    check(lambda->x1 && (!act || (lambda->x2_vVoo && lambda->x2_vvoO)), "NULL pointer in lambda");
    reg_ground(g);
    reg(t2_vVoO, (long long)d.nv * d.NV * d.no * d.NO, "t2_vVoO");
    reg(t2_vVOo, (long long)d.nv * d.NV * d.NO * d.no, "t2_vVOo");
    for (int m = 0; m < nstate; m++) {
      reg_vec(g, L[m].x1, L[m].x2_vVoo, L[m].x2_vvoO);
      reg_vec(g, R[m].x1, R[m].x2_vVoo, R[m].x2_vvoO);
    }
    reg_vec(g, lambda->x1, lambda->x2_vVoo, lambda->x2_vvoO);
    reg(D_m0, nstate * N * N, "D_m0");
    reg(D_0m, nstate * N * N, "D_0m");
    reg(s_out, nstate, "s");
    const mlcc3_opts o = opts_or_default(opts);
    t_xf32 = false;  // the densities read the contravariant blocks in FP64 in every form
    check(!o.cvs_core, "core-valence separation applies to the right and left transforms only");
    hipStream_t s = (hipStream_t)stream;
    DeviceGuard dg(ws->device);
    log_begin("triples_densities", s, d.no, d.nv, d.NO, d.NV, d.nc, nstate, o.precision);
    const Range r = range_of(o, mlcc3_num_triples(d.no));
    if (o.check_finite) {
      ground_finite(ws, g, s);
      for (int m = 0; m < nstate; m++) {
        vec_finite(ws, d, L[m], s);
        vec_finite(ws, d, R[m], s);
      }
      vec_finite(ws, d, *lambda, s);
    }
    guard_check(g, omega, nstate, o.guard, s);
    HIPRT(hipMemsetAsync(D_m0, 0, sizeof(double) * nstate * N * N, s));
    HIPRT(hipMemsetAsync(D_0m, 0, sizeof(double) * nstate * N * N, s));
    HIPRT(hipMemsetAsync(s_out, 0, sizeof(double) * nstate, s));
    if (d.no < 2 || d.nv < 2 || r.tb == r.te) return;  // no triples: the triples terms vanish
    prepare_ground(ws, g, o.reuse_ground != 0, s);
    log_phase("prep");
    const int no = d.no, nv = d.nv, NO = d.NO, NV = d.NV;
    const size_t nbig = (size_t)(d.nord * d.nv3);
    double *XTc = buf(ws, "XTc", nbig, s);
    tau_path(ws, g, d, r, s, XTc);
    log_phase("tau3");
    double *XT = B(ws, "XT");
    double *XLam = buf(ws, "XLam", nbig, s);
    const double zero = 0.0;
    build_L3(ws, g, d, lambda, &zero, 1, r, XLam, "LAlam", "LVlam", s);   // lambda3: L3 recipe at omega = 0
    double *lam2a = buf(ws, "lam2a", (size_t)no * no * d.nv2, s);   // lambda^{ab}_{ij}, [i][j][a][b]
    launch_pack_vvoo(lambda->x2_vVoo, no, nv, NV, 0, lam2a, s);
    double *XL = buf(ws, "XR", nbig, s);
    double *XRt = buf(ws, "W", nbig, s);  // R~ of each state overwrites the W of its R3 (see wx_buffer)
    double *XRc = buf(ws, "XRc", nbig, s);
    double *tA = B(ws, "tA");
    double *V = buf(ws, "dens_V", (size_t)no * no * nv * NO, s);
    double *Xl = buf(ws, "dens_Xl", (size_t)no * no * d.nv2, s);
    double *Yc = buf(ws, "dens_Yc", (size_t)no * nv, s);
    double *Zt = buf(ws, "dens_Zt", (size_t)no * no, s);
    double *Zv = buf(ws, "dens_Zv", (size_t)d.nv2, s);
    double *Rbv = buf(ws, "dens_Rbv", (size_t)no * no * d.nv2, s);
    double *part = buf(ws, "dot_part", 512, s);
    for (int m = 0; m < nstate; m++) {
      double *Dm = D_m0 + (long long)m * N * N, *D0 = D_0m + (long long)m * N * N;
      build_L3(ws, g, d, L + m, omega + m, 1, r, XL, "LA", "LV", s);
      log_phase("L3");
      group_dlhat(ws, g, d, R + m, 1, s);
      right_vector_prep(ws, g, d, R[m], 0, 1, s);
      build_R3(ws, g, d, R + m, omega + m, 1, r, XRt, XRc, s);
      log_phase("R3");
      // ---- D^{m-0} (SI left density) ----
      g_kl(d, XTc, XL, Dm, N, -0.5, 1.0, s);                          // D_kl -= 1/2 L~_{ijl} tau_{ijk}
      g_cd(d, XL, XTc, Dm + NO * N + NO, N, 0.5, 1.0, s);             // D_cd += 1/2 L~^{abc} tau^{abd}
      g_ld(d, XT, B(ws, "LV"), Dm + NO, split(nv, N, 1), 1.0, 1.0, s);  // D_ld += L^{ab}_{ij} tau~^{abd}_{ijl}
      v_jkbL(ws, d, XL, g->t2_vvoO, V, s);                            // V = sum L~ t^{ac}_{iL}
      d_LD(d, V, tA, Dm, N, -1.0, s);                                 // D_LD -= V t^{bD}_{jk}
      // ---- D^{0-m} (SI right density) ----
      {  // X^{bc}_{jk} = sum_{ai} lambda~^{abc}_{ijk} R^a_i
        Gemm gg = gemm_plain(no * no * (int)d.nv2, 1, Xl, plain(1), plain(1), 1.0, 0.0);
        gg.nseg = 1;
        gg.seg[0] = seg(XLam, split((int)d.nv2, d.nv3, 1), split(nv, (long long)no * no * d.nv3, d.nv2), 0, R[m].x1,
                        split(nv, 1, NO), plain(1), 0, no * nv);
        gemm(gg, s);
      }
      {  // D_Kl -= sum t^{bc}_{jK} X^{bc}_{jl}
        Gemm gg = gemm_plain(NO, no, D0, plain(N), plain(1), -1.0, 1.0);
        gg.nseg = 1;
        gg.seg[0] = seg(g->t2_vvoO, plain(1), split((int)d.nv2, NO, (long long)no * NO), 0, Xl,
                        split((int)d.nv2, (long long)no * d.nv2, 1), plain(d.nv2), 0, no * (int)d.nv2);
        gemm(gg, s);
      }
      g_kl(d, XRc, XLam, D0, N, -0.5, 1.0, s);                        // D_kl -= 1/2 lambda~_{ijl} R_{ijk}
      {  // D_ld += sum X^{bc}_{jk} tau^{bcd}_{jkl}
        Gemm gg = gemm_plain(no * nv, 1, D0 + NO, split(nv, N, 1), plain(1), 1.0, 1.0);
        gg.nseg = 1;
        gg.seg[0] = seg(XTc, split(nv, d.nv3, 1), split((int)d.nv2, (long long)no * d.nv3, nv), 0, Xl, plain(1),
                        plain(1), 0, no * no * (int)d.nv2);
        gemm(gg, s);
      }
      {  // D_ld -= sum X^{bc}_{jk} tau^{bcd}_{jlk}   (summed over j batches)
        Gemm gg = gemm_plain(no * nv, 1, D0 + NO, split(nv, N, 1), plain(1), -1.0, 1.0);
        gg.nbatch = no;
        gg.nseg = 1;
        gg.seg[0] = seg(XTc, split(nv, (long long)no * d.nv3, 1), split((int)d.nv2, d.nv3, nv),
                        (long long)no * no * d.nv3, Xl, plain(1), plain(1), (long long)no * d.nv2, no * (int)d.nv2);
        gemm_sumz(ws, gg, s);
      }
      g_ld(d, XRt, lam2a, D0 + NO, split(nv, N, 1), 1.0, 1.0, s);    // D_ld += lambda^{ab}_{ij} R~^{abd}_{ijl}
      launch_pack_vvoo(R[m].x2_vVoo, no, nv, NV, 1, Rbv, s);           // Rbar^{ab}_{ij}
      g_ld(d, XLam, Rbv, Yc, plain(1), 1.0, 0.0, s);                   // Y_kc = sum lambda~^{abc}_{ijk} Rbar^{ab}_{ij}
      {  // D_LD += 1/2 sum Y_kc (2 t^{cD}_{kL} - t^{cD}_{Lk})
        Gemm gg = gemm_plain(NO * NV, 1, D0 + NO, split(NV, N, 1), plain(1), 1.0, 1.0);
        gg.nseg = 2;
        gg.seg[0] = seg(t2_vVoO, split(NV, 1, (long long)no * NO), split(nv, NO, (long long)NV * no * NO), 0, Yc,
                        plain(1), plain(1), 0, no * nv, 1.0);
        gg.seg[1] = seg(t2_vVOo, split(NV, no, (long long)NO * no), split(nv, 1, (long long)NV * NO * no), 0, Yc,
                        plain(1), plain(1), 0, no * nv, -0.5);
        gemm(gg, s);
      }
      v_jkbL(ws, d, XLam, B(ws, "RB"), V, s);                          // V2 = sum lambda~ Rbar^{ac}_{iL}
      d_LD(d, V, tA, D0, N, -1.0, s);                                  // D_LD -= V2 t^{bD}_{jk}
      {  // V3[i][(k,a)][L] = sum_{j,bc} lambda~^{abc}_{ijk} t^{bc}_{jL};  D_LD -= V3 Rbar^{aD}_{ik}
        Gemm gg = gemm_plain(no * nv, NO, V, plain(NO), plain(1), 1.0, 0.0);
        gg.nbatch = no;
        gg.cbatch = (long long)no * nv * NO;
        gg.nseg = 1;
        gg.seg[0] = seg(XLam, split(nv, d.nv3, d.nv2), split((int)d.nv2, (long long)no * d.nv3, 1),
                        (long long)no * no * d.nv3, g->t2_vvoO, split((int)d.nv2, NO, (long long)no * NO), plain(1),
                        0, no * (int)d.nv2);
        gemm(gg, s);
        d_LD(d, V, B(ws, "RA"), D0, N, -1.0, s);
      }
      g_kl(d, XLam, XTc, Zt, no, 1.0, 0.0, s);                         // Z_kl = sum lambda~_{ijk} tau_{ijl}
      {  // D_lD -= 1/2 sum_k Z_kl R^D_k
        Gemm gg = gemm_plain(no, NV, D0 + NO, plain(N), plain(1), -0.5, 1.0);
        gg.nseg = 1;
        gg.seg[0] = seg(Zt, plain(1), plain(no), 0, R[m].x1, plain(1), plain(NO), 0, no);
        gemm(gg, s);
      }
      g_cd(d, XLam, XTc, Zv, nv, 1.0, 0.0, s);                         // Zv_cd = sum lambda~^{abc} tau^{abd}
      {  // D_Ld -= 1/2 sum_c R^c_L Zv_cd
        Gemm gg = gemm_plain(NO, nv, D0 + NO, plain(N), plain(1), -0.5, 1.0);
        gg.nseg = 1;
        gg.seg[0] = seg(R[m].x1, plain(1), plain(NO), 0, Zv, plain(nv), plain(1), 0, nv);
        gemm(gg, s);
      }
      launch_add_vo(D0, NO, (int)N, no, nv, Yc, 0.5, s);             // D_ck += 1/2 Y_kc
      {  // D_cD += sum X^{bc}_{jk} t^{bD}_{jk}
        Gemm gg = gemm_plain(nv, NV, D0 + NO * N + NO, plain(N), plain(1), 1.0, 1.0);
        gg.nseg = 1;
        gg.seg[0] = seg(Xl, plain(1), plain(nv), 0, tA, plain(NV), plain(1), 0, no * no * nv);
        gemm(gg, s);
      }
      g_cd(d, XLam, XRc, D0 + NO * N + NO, N, 0.5, 1.0, s);            // D_cd += 1/2 lambda~^{abc} R^{abd}
      launch_dot(XLam, XRc, (long long)nbig, 1.0 / 6.0, part, s_out + m, s);   // s = 1/6 sum lambda~ R3
      launch_add_diag(D0, NO, (int)N, s_out + m, 2.0, s);              // D_LL += 2 s
      HIPRT(hipGetLastError());
    }
  });
}

const char *mlcc3_status_string(int status) {
  switch (status) {
    case MLCC3_OK: return "ok";
    case MLCC3_EINVAL: return "invalid argument";
    case MLCC3_ESINGULAR: return "omega too close to an orbital-energy denominator";
    case MLCC3_ENOMEM: return "device allocation failed";
    case MLCC3_EHIP: return "HIP runtime error";
    case MLCC3_ENONFINITE: return "non-finite input";
    case MLCC3_ESTATE: return "stale workspace (ground-state inputs changed under reuse_ground)";
    case MLCC3_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

const char *mlcc3_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

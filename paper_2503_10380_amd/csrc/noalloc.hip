// An MTTKRP entry point that allocates nothing: the FP64 matrix-free chain of
// cpppl_mttkrp (the same kernels), with every intermediate in one file-scope
// device array instead of a context's workspace, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).
//
// The operands are the caller's arrays as they are: t[ij][cd] enters the tau
// and H products as a row- or k-contiguous operand, the factors (n x R) enter
// Y as row-contiguous operands, and Y is a batched product over X, so that
// only gamma and rho (transposed, for the Khatri-Rao product and the occupied
// reduction) and B permuted to [p][X][q] (for M) are copied into the array.
#include <algorithm>
#include <mutex>
#include <stdexcept>

#include "../../include/cpppl.h"
#include "gemm.h"
#include "ops.h"

using namespace cpppl;

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
constexpr int MAX_DEVICES = 64;

// Per device, one copy of the array, shared by every call on that device.
static __device__ __align__(256) double scratch[SCRATCH_BYTES / sizeof(double)];

std::mutex g_mutex;
double* g_ptr[MAX_DEVICES] = {};  // device address of `scratch` on each device

// The array's device address on the current device (looked up once per device).
double* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    CPPPL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw std::runtime_error("scratch array has no device address");
    g_ptr[dev] = (double*)p;
  }
  return g_ptr[dev];
}

constexpr size_t AL = 32;  // doubles: 256-byte alignment of every region
size_t up(size_t n) { return (n + AL - 1) / AL * AL; }

struct Layout {
  size_t fg = 0, fr = 0, kt = 0, tau = 0, bp = 0, ya = 0, yb = 0, z = 0, ht = 0, mt = 0, part = 0;
  size_t fixed = 0;   // doubles before the split-K partials
  size_t mn = 0;      // M x N of the split-K product
};

Layout layout(const cpppl_dims& d, int mode) {
  const size_t o = (size_t)d.o, v = (size_t)d.v, X = (size_t)d.nx, R = (size_t)d.rank;
  Layout L;
  size_t off = 0;
  auto take = [&](size_t n) { size_t p = off; off += up(n); return p; };
  if (mode >= 2) {
    L.fg = take(o * R);
    L.fr = take(o * R);
    L.kt = take(R * o * o);
    L.tau = take(R * v * v);
    L.bp = take(X * v * v);
    L.ya = L.yb = take(R * X * v);  // the one Y this mode needs
    L.z = take(R * X * v);
    L.mt = take(R * v);
    L.mn = R * v;
  } else {
    L.fg = take(o * R);  // the other occupied factor, transposed
    L.ya = take(R * X * v);
    L.yb = take(R * X * v);
    L.z = take(R * v * v);  // G
    L.ht = take(R * o * o);
    L.mt = take(R * o);
    L.mn = R * o * o;
  }
  L.fixed = off;
  L.part = off;
  return L;
}

}  // namespace

extern "C" {

CPPPL_API cpppl_status cpppl_mttkrp_noalloc(const cpppl_dims* dims, const double* t, const double* b,
                                            const double* fi, const double* fj, const double* fa,
                                            const double* fb, int mode, double* m_out,
                                            void* hip_stream) {
  if (!dims || !t || !b || !fi || !fj || !fa || !fb || !m_out) return CPPPL_E_ARG;
  if (mode < 0 || mode > 3) return CPPPL_E_ARG;
  const cpppl_dims d = *dims;
  if (d.o <= 0 || d.v <= 0 || d.nx <= 0 || d.rank <= 0 || d.rank > 4096 || d.o > 4096 ||
      d.v > 65536 || d.nx > (1 << 20))
    return CPPPL_E_ARG;
  const Layout L = layout(d, mode);
  const size_t cap = SCRATCH_BYTES / sizeof(double);
  if (L.fixed > cap) return CPPPL_E_NOMEM;  // beyond the array: refused before any work
  try {
    int dev = 0;
    CPPPL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return CPPPL_E_UNSUPPORTED;
    double* S = scratch_ptr(dev);
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t o = d.o, v = d.v, X = d.nx, R = d.rank;
    const int64_t o2 = o * o, v2 = v * v;
    // split-K partials in what is left of the array
    const int64_t room = (int64_t)((cap - L.fixed) / std::max<size_t>(1, L.mn));
    auto splits = [&](int64_t M, int64_t N, int64_t K) {
      int sp = choose_splits(gemm_tiles_f64(M, N), K, 1024, 64, 16);
      return (int)std::max<int64_t>(1, std::min<int64_t>(sp, room));
    };
    // Y[r][X][q] = sum_p F[p][r] B^X_pq: batched over X, F (n x R) row-contiguous
    auto compute_y = [&](const double* F, double* Y) {
      Gemm g;
      g.batch = X; g.M = R; g.N = v; g.K = v;
      g.A = F; g.sam = 1; g.sak = R; g.sab = 0;
      g.B = b; g.sbk = v; g.sbn = 1; g.sbb = v2;
      g.C = Y; g.scm = X * v; g.scb = v; g.ctype = DType::F64;
      gemm_f64(g, s);
    };
    const int64_t n = mode < 2 ? o : v;
    double* MT = S + L.mt;
    if (mode >= 2) {
      // tau[r][cd] = sum_ij gamma_ir rho_jr t[ij][cd]
      transpose_batched(fi, S + L.fg, DType::F64, 1, o, R, s);
      transpose_batched(fj, S + L.fr, DType::F64, 1, o, R, s);
      khatri_rao_t(S + L.fg, S + L.fr, o, R, S + L.kt, DType::F64, s);
      Gemm gt;
      gt.M = R; gt.N = v2; gt.K = o2;
      gt.A = S + L.kt; gt.sam = o2; gt.sak = 1;
      gt.B = t; gt.sbk = v2; gt.sbn = 1;
      gt.C = S + L.tau; gt.scm = v2; gt.ctype = DType::F64;
      gemm_f64(gt, s);
      // Y of the other virtual factor, then Z per r, then M over (X, q)
      compute_y(mode == 2 ? fb : fa, S + L.ya);
      Gemm gz;
      gz.batch = R; gz.M = X; gz.N = v; gz.K = v;
      gz.A = S + L.ya; gz.sam = v; gz.sak = 1; gz.sab = X * v;
      gz.B = S + L.tau; gz.sbb = v2;
      if (mode == 2) { gz.sbn = v; gz.sbk = 1; } else { gz.sbk = v; gz.sbn = 1; }
      gz.C = S + L.z; gz.scm = v; gz.scb = X * v; gz.ctype = DType::F64;
      gemm_f64(gz, s);
      permute_pxq(b, S + L.bp, DType::F64, X, v, s);
      Gemm gm;
      gm.M = R; gm.N = v; gm.K = X * v;
      gm.A = S + L.z; gm.sam = X * v; gm.sak = 1;
      gm.B = S + L.bp; gm.sbn = X * v; gm.sbk = 1;
      gm.C = MT; gm.scm = v; gm.ctype = DType::F64;
      gm.splits = splits(R, v, X * v);
      gm.partial = S + L.part;
      gemm_f64(gm, s);
    } else {
      // G[r][cd] = sum_X Y_alpha[r][X][c] Y_beta[r][X][d], H[r][ij] = sum_cd G[r][cd] t[ij][cd]
      compute_y(fa, S + L.ya);
      compute_y(fb, S + L.yb);
      Gemm gg;
      gg.batch = R; gg.M = v; gg.N = v; gg.K = X;
      gg.A = S + L.ya; gg.sam = 1; gg.sak = v; gg.sab = X * v;
      gg.B = S + L.yb; gg.sbk = v; gg.sbn = 1; gg.sbb = X * v;
      gg.C = S + L.z; gg.scm = v; gg.scb = v2; gg.ctype = DType::F64;
      gemm_f64(gg, s);
      Gemm gh;
      gh.M = R; gh.N = o2; gh.K = v2;
      gh.A = S + L.z; gh.sam = v2; gh.sak = 1;
      gh.B = t; gh.sbn = v2; gh.sbk = 1;
      gh.C = S + L.ht; gh.scm = o2; gh.ctype = DType::F64;
      gh.splits = splits(R, o2, v2);
      gh.partial = S + L.part;
      gemm_f64(gh, s);
      // gamma: sum over j against rho; rho: sum over i against gamma
      transpose_batched(mode == 0 ? fj : fi, S + L.fg, DType::F64, 1, o, R, s);
      occ_reduce(S + L.ht, S + L.fg, MT, o, R, mode == 0 ? 0 : 1, s);
    }
    transpose_batched(MT, m_out, DType::F64, 1, R, n, s);
  } catch (const HipError&) {
    return CPPPL_E_HIP;
  } catch (const std::invalid_argument&) {
    return CPPPL_E_ARG;
  } catch (...) {
    return CPPPL_E_STATE;
  }
  return CPPPL_OK;
}

}  // extern "C"

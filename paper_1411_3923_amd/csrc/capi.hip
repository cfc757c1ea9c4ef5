// C-ABI entry points: handle lifecycle, argument checks and the batched PCG
// driver (Sec. 2.4.2: PCG on the SPD system with the two-level
// preconditioner; the robust formulation's realisations solved together,
// Sec. 4.4).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "big.h"
#include "btri.h"

using namespace tpcg;

namespace {


int fail(tpcg_handle* hh, int code, const std::string& msg) {
  if (hh) reinterpret_cast<Handle*>(hh)->err = msg;
  return code;
}

Handle* H(tpcg_handle* h) { return reinterpret_cast<Handle*>(h); }
const Handle* H(const tpcg_handle* h) { return reinterpret_cast<const Handle*>(h); }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Derive the geometry; returns an error message, or nullptr when the problem
// is usable (no heap allocation either way).
const char* make_geometry(const tpcg_problem& pr, Geometry& g) {
  if (pr.dim != 2 && pr.dim != 3) return "dim must be 2 or 3";
  const int d = pr.dim;
  std::memset(&g, 0, sizeof(g));
  g.dim = d;
  g.nelx = pr.nel[0];
  g.nely = pr.nel[1];
  g.nelz = d == 3 ? pr.nel[2] : 1;
  if (g.nelx < 1 || g.nely < 1 || g.nelz < 1) return "element counts must be positive";
  g.s = pr.sub[0];
  if (g.s < 1) return "sub must be positive";
  if (pr.sub[1] != g.s || (d == 3 && pr.sub[2] != g.s))
    return "subdomains must be square (cubic in 3D): sub[0] == sub[1] (== sub[2])";
  if (g.nelx % g.s || g.nely % g.s || (d == 3 && g.nelz % g.s))
    return "element counts must be multiples of sub";
  if (pr.overlap != 1) return "only overlap = 1 is supported";
  if (!(pr.nu > -1.0 && pr.nu < 0.5)) return "nu must lie in (-1, 0.5)";
  if (!(pr.Emin > 0.0) || !(pr.E0 >= pr.Emin)) return "need 0 < Emin <= E0";
  if (!(pr.penal >= 1.0)) return "penal must be >= 1";
  if (!(pr.lambda_thresh == pr.lambda_thresh)) return "lambda_thresh is NaN";
  if (pr.coarse_dense_max < 0) return "coarse_dense_max must be >= 0";
  g.nnx = g.nelx + 1;
  g.nny = g.nely + 1;
  g.nnz = d == 3 ? g.nelz + 1 : 1;
  g.nnodes = (int64_t)g.nnx * g.nny * g.nnz;
  g.ndof = d * g.nnodes;
  g.nel = (int64_t)g.nelx * g.nely * g.nelz;
  g.gx = g.nelx / g.s;
  g.gy = g.nely / g.s;
  g.gz = d == 3 ? g.nelz / g.s : 1;
  g.nsub = g.gx * g.gy * g.gz;
  g.bn = g.s + 1;
  g.nbox = d == 3 ? g.bn * g.bn * g.bn : g.bn * g.bn;
  g.nloc = d * g.nbox;
  g.nb = d == 3 ? d * g.bn * g.bn : d * g.bn;
  g.nblk = g.bn;
  g.k = pr.ncoarse;
  if (g.k < 1 || g.k > kMaxK) return "ncoarse must lie in 1..16";
  if (g.k > g.nloc) return "ncoarse exceeds the subdomain's DOFs";
  // coarse blocks along the axis with the most subdomains
  const int cnt[3] = {g.gx, g.gy, g.gz};
  g.caxis = 0;
  for (int a = 1; a < d; ++a)
    if (cnt[a] > cnt[g.caxis]) g.caxis = a;
  g.nblkc = cnt[g.caxis];
  g.nbc = g.k * (g.nsub / g.nblkc);
  g.nt = g.nsub * g.k;
  g.dense_max = pr.coarse_dense_max > 0 ? pr.coarse_dense_max : kDenseCoarse;
  g.submap = nullptr;
  g.cband = pr.coarse_band ? 1 : 0;   // set below once the coarse blocks are known
  // packed factor records: B_{b+1} reaches pe diagonals below its main one
  {
    int64_t w = 1;
    for (int a = 1; a < d; ++a) w = w * g.bn + 1;
    w = d * w + d - 1;                       // half-bandwidth of a subdomain matrix
    g.pe = (int)std::min<int64_t>(std::max<int64_t>(w - g.nb + 1, 0), g.nb);
    g.bstride = (g.nb * g.nb + g.nb * g.pe + 3) & ~3;
    int dw = 1;                              // coarse neighbours' distance in block rows
    if (d == 3) dw = 1 + (g.caxis == 0 ? g.gy : g.gx);
    g.pec = std::min(g.nbc, (dw + 1) * g.k);
    g.bstridec = (g.nbc * g.nbc + g.nbc * g.pec + 3) & ~3;
  }
  g.ebn = g.s + 3;
  g.nebox = d == 3 ? g.ebn * g.ebn * g.ebn : g.ebn * g.ebn;
  g.ndpe = d == 3 ? 24 : 8;
  if (g.nt > g.dense_max && !coarse_btri_fits(g)) g.cband = 1;
  return nullptr;
}

// Limits of the factor kernels (checked when the preconditioner is built;
// the matrix-free operator has none): the on-chip block-tridiagonal kernels
// for subdomain blocks up to 96 unknowns, the HBM-resident ones beyond
// (big.h), and the block-tridiagonal coarse factor for coarse spaces above
// dense_max.
std::string precond_limits(const Geometry& g, int big) {
  if (big) {
    const char* why = big_limits(g);
    if (why) return why;
  } else if (stage_bucket(stage_regs_for<double>(g.nb, g.pe)) < 0) {
    return "factor records too long for the staged solve kernels";
  }
  if (!g.cband && (g.nt > g.dense_max || coarse_btri_fits(g))) {
    if (stage_bucket(stage_regs_for<double>(g.nbc, g.pec)) < 0)
      return "coarse factor records too long for the staged solve kernels";
  }
  return "";
}

struct Sizes {
  size_t persistent, setup_peak;
};

Sizes sizes(const tpcg_problem& pr, const Geometry& g, int nsys) {
  const int mixed = pr.precision == TPCG_MIXED;
  const int big = local_is_big(g, pr.big_min_nb);
  int msub = std::min(kMaxSub, g.k + (pr.eig_extra > 0 ? pr.eig_extra : g.k));
  if (msub > g.nloc) msub = g.nloc;
  const size_t frec = big ? (size_t)g.nsub * g.nblk * big_shape(g).rec_dir
                          : (size_t)g.nsub * g.nblk * tile_shape(g.nb).tstride;   // local factors
  const size_t crec = (size_t)g.nblkc * g.bstridec;                // packed coarse factor
  const size_t ts = mixed ? 4 : 8;
  size_t p = 0;
  p += g.ndof + sizeof(double) * g.ndpe * g.ndpe;
  p += sizeof(double) * (size_t)kMaxSys * g.nel;   // filter adjoint factors
  p += (sizeof(double) + ts) * (size_t)g.nsub * g.nloc * g.k;
  p += 2 * sizeof(double) * (size_t)g.nsub * msub;
  p += ts * nsys * (frec + (size_t)g.nel);
  if (!big) p += sizeof(double) * nsys * (size_t)g.nsub * g.nb * (g.nb + 1) / 2;
  if (mixed) p += sizeof(double) * nsys * (size_t)g.nel;
  p += sizeof(int) * (size_t)g.nsub;
  p += (sizeof(unsigned long long) + 4 * sizeof(int)) * (size_t)g.nsub;   // distinct-cell maps
  if (g.nt <= g.dense_max && !g.cband) {
    const size_t T = coarse_tiles(g.nt);
    p += sizeof(double) * nsys * (T * (T + 1) / 2 * kCT * kCT + T * T * kCT);
  }
  if (!g.cband && (g.nt > g.dense_max || coarse_btri_fits(g))) p += sizeof(double) * nsys * crec;
  if (g.cband) p += sizeof(double) * nsys * (coarse_band_elems(g) + (size_t)g.nt);
  p += 5 * sizeof(double) * nsys * g.ndof;
  p += ts * nsys * (size_t)g.nsub * g.nloc;
  p += 2 * sizeof(double) * nsys * (size_t)g.nt;
  if (restrict_splits(g) > 1) p += sizeof(double) * restrict_splits(g) * kMaxSys * (size_t)g.nt;
  p += sizeof(double) * kNumPartSlots * kMaxSys * kMaxParts + 4096;
  return {p, sizeof(double) * build_ws_elems(pr, g, big, msub)};
}

// Fault injection for the tests of the allocation paths: the n-th device
// allocation from now on fails (0: none).
int g_fail_at = 0;
int g_alloc_count = 0;

template <typename T>
int alloc(T*& p, size_t n) {
  void* v = nullptr;
  if (!device_alloc(&v, std::max<size_t>(n, 1) * sizeof(T))) return TPCG_ENOMEM;
  p = reinterpret_cast<T*>(v);
  return TPCG_OK;
}

// A group of device allocations that either all succeed or leave nothing
// behind: the targets are assigned only when every allocation succeeded.
struct AllocGroup {
  std::vector<std::pair<void**, size_t>> want;
  template <typename T>
  void add(T*& dst, size_t elems) {
    want.emplace_back(reinterpret_cast<void**>(&dst), std::max<size_t>(elems, 1) * sizeof(T));
  }
  void add_bytes(void*& dst, size_t bytes) { want.emplace_back(&dst, std::max<size_t>(bytes, 1)); }
  int commit() {
    std::vector<void*> got;
    got.reserve(want.size());
    for (auto& w : want) {
      void* v = nullptr;
      if (!device_alloc(&v, w.second)) {
        for (void* q : got) hipFree(q);
        return TPCG_ENOMEM;
      }
      got.push_back(v);
    }
    for (size_t i = 0; i < want.size(); ++i) *want[i].first = got[i];
    return TPCG_OK;
  }
};

void drop_graphs(Handle* h) {
  for (auto& e : h->gexec)
    if (e) {
      hipGraphExecDestroy(e);
      e = nullptr;
    }
  h->gkey.clear();
}

void release(Handle* h) {
  if (!h) return;
  drop_graphs(h);
  for (auto& ev : h->gprof_ev)
    for (auto& e : ev)
      if (e) hipEventDestroy(e);
  void* ptrs[] = {h->fixed, h->K0,   h->phi,  h->phim,   h->lam, h->kj,     h->eres, h->lfac,
                  h->emod,  h->twist, h->emod64, h->cfac, h->cpk, h->cpart, h->r, h->z,
                  h->p,     h->p2,   h->q,    h->zloc,  h->yc,   h->xc,   h->parts, h->istate,
                  h->dflag, h->build_ws, h->gm_V, h->gm_w, h->gm_i, h->gm_flags, h->gm_out,
                  h->cell_sig, h->submap_d, h->dedup_pairs, h->dedup_flag, h->fscratch,
                  h->cband, h->cband_w, h->ycp};
  for (void* p : ptrs)
    if (p) hipFree(p);
  if (h->hpoll) hipHostFree(h->hpoll);
  if (h->gm_host) hipHostFree(h->gm_host);
  for (auto& e : h->gm_ev)
    if (e) hipEventDestroy(e);
  for (auto& e : h->ev)
    if (e) hipEventDestroy(e);
  if (h->t0) hipEventDestroy(h->t0);
  if (h->t1) hipEventDestroy(h->t1);
  for (auto& e : h->prof_ev)
    if (e) hipEventDestroy(e);
  if (h->fork) hipEventDestroy(h->fork);
  if (h->join) hipEventDestroy(h->join);
  if (h->side) hipStreamDestroy(h->side);
}

int check_hip(Handle* h, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    h->sticky = 1;
    h->err = std::string(where) + ": " + hipGetErrorString(e);
    return TPCG_EHIP;
  }
  return TPCG_OK;
}

// Densities of the entry points that return after enqueueing are checked
// here, synchronously: TPCG_EINVAL when any of nsys x n values is NaN or
// outside [0, 1].
int check_rho_sync(Handle* h, const double* rho, int64_t n, int nsys) {
  int* hf = h->hpoll + 2 * kMaxSys;
  hipMemsetAsync(h->dflag + 1, 0, sizeof(int), h->stream);
  launch_check_rho(rho, n, nsys, h->dflag + 1, 0, 1, h->stream);
  hipMemcpyAsync(hf, h->dflag + 1, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  hipStreamSynchronize(h->stream);
  int rc = check_hip(h, "density check");
  if (rc != TPCG_OK) return rc;
  if (*hf) return fail(reinterpret_cast<tpcg_handle*>(h), TPCG_EINVAL,
                       "densities must lie in [0, 1] (NaN or out-of-range value found)");
  return TPCG_OK;
}

// Minimum bytes one system's share of a local-solve launch must move, per
// subdomain: the lower triangles of the inverted diagonal factor blocks D_b
// (read in the forward and the backward pass of the twisted solve: the
// middle block once, the lower half's innermost block once), the moduli of
// the inner element layers, the right-hand side (FP64) and the support flags
// read once, the forward result written and read back and the solution
// written.
double local_solve_bytes(const Geometry& g, int elem, int big) {
  const double tri = 0.5 * g.nb * (g.nb + 1.0);
  const double sw = g.dim == 3 ? (g.bn + 1.0) * (g.bn + 1.0) : g.bn + 1.0;
  const int mid = g.nblk / 2, nbot = g.nblk - 1 - mid;
  // the HBM-resident solves run the forward and backward passes as separate
  // launches, so the innermost block of the lower half is read twice too
  const double reads = big ? 2.0 * g.nblk - 1.0
                           : 2.0 * mid + 1.0 + (nbot > 0 ? 2.0 * nbot - 1.0 : 0.0);
  const double per = reads * tri * elem + (g.nblk - 1.0) * sw * elem +
                     (double)g.nloc * (8.0 + 1.0 + 3.0 * elem);
  return g.nsub * per;
}

// the summary values [nsys][4] (iterations, status, recursive and true
// relative residual) as tpcg_info records in device memory
__global__ void k_info_pack(const double* __restrict__ dout, int nsys, tpcg_info* __restrict__ info) {
  const int sys = threadIdx.x;
  if (sys >= nsys) return;
  info[sys].iters = (int32_t)dout[4 * sys + 0];
  info[sys].status = (int32_t)dout[4 * sys + 1];
  info[sys].relres = dout[4 * sys + 2];
  info[sys].true_relres = dout[4 * sys + 3];
  info[sys].seconds = 0.0;
}

Gate make_gate(const Handle* h, int rr_slot, int it, int maxit, double tol2, int enabled) {
  Gate g;
  g.parts = h->parts;
  g.istate = h->istate;
  g.np = parts_for(h->g.nnodes);
  g.rr_slot = rr_slot;
  g.it = it;
  g.maxit = maxit;
  g.tol2 = tol2;
  g.enabled = enabled;
  g.test = 0;
  g.itbase = nullptr;
  return g;
}

}  // namespace

namespace tpcg {
bool device_alloc(void** p, size_t bytes) {
  *p = nullptr;
  ++g_alloc_count;
  if (g_fail_at > 0 && g_alloc_count == g_fail_at) return false;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();   // no stale error for the next check
    *p = nullptr;
    return false;
  }
  return true;
}
}  // namespace tpcg

// ---------------------------------------------------------------------------
// Scratch of the entry point that allocates nothing
// (tpcg_compliance_and_sensitivity_noalloc): the element matrix, then the
// f^T u partials of up to kMaxSys systems. Every device holds its own copy
// of this array until the process ends. Host code must not use the array's
// name as a device address: its address on the current device comes from
// hipGetSymbolAddress, looked up once per device.
// ---------------------------------------------------------------------------
namespace {
constexpr int kNaK0 = 576;                                   // 24 x 24 (H8) at most
constexpr size_t kNaElems = kNaK0 + (size_t)kMaxSys * kMaxParts;
constexpr int kNaMaxDev = 64;
}  // namespace

static __device__ __align__(256) double scratch[kNaElems];

namespace {

std::mutex g_na_mu;
double* g_na_ptr[kNaMaxDev] = {};

// Address of `scratch` on the current device (looked up on the first call
// on that device).
int scratch_on_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNaMaxDev) {
    (void)hipGetLastError();
    return TPCG_EHIP;
  }
  std::lock_guard<std::mutex> lock(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return TPCG_EHIP;
    }
    g_na_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_na_ptr[dev];
  return TPCG_OK;
}

// 64 values passed by value in the kernel arguments (no staging buffer):
// dst[i] = v[i] for i < n; thread 0 of the first chunk also clears `flag`
struct Vals64 {
  double v[64];
};

__global__ void k_na_put(double* __restrict__ dst, Vals64 v, int n, int* __restrict__ flag) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = v.v[i];
  if (flag && i == 0) *flag = 0;
}

}  // namespace

extern "C" int tpcg_compliance_and_sensitivity_noalloc(const tpcg_problem* prob,
                                                       const uint8_t* fixed, const double* rho_phys,
                                                       const double* u, const double* f,
                                                       int32_t nsys, double* c, double* dc,
                                                       int32_t* status, void* stream) {
  if (!prob || !fixed || !rho_phys || !u || !f || !c) return TPCG_EINVAL;
  if (nsys < 1 || nsys > kMaxSys) {
    fprintf(stderr, "tpcg_compliance_and_sensitivity_noalloc: nsys must lie in 1..%d\n", kMaxSys);
    return TPCG_EINVAL;
  }
  Geometry g;
  const char* msg = make_geometry(*prob, g);
  if (msg) {
    fprintf(stderr, "tpcg_compliance_and_sensitivity_noalloc: %s\n", msg);
    return TPCG_EINVAL;
  }
  double* ws = nullptr;
  int rc = scratch_on_current_device(&ws);
  if (rc != TPCG_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  double K0[kNaK0];
  element_stiffness(g.dim, prob->nu, K0);
  const int nk = g.ndpe * g.ndpe;
  for (int o = 0; o < nk; o += 64) {
    Vals64 v;
    const int n = std::min(64, nk - o);
    for (int i = 0; i < n; ++i) v.v[i] = K0[o + i];
    hipLaunchKernelGGL(k_na_put, dim3(1), dim3(64), 0, st, ws + o, v, n,
                       o == 0 ? reinterpret_cast<int*>(status) : nullptr);
  }
  if (status) launch_check_rho(rho_phys, g.nel, nsys, reinterpret_cast<int*>(status), 0, 1, st);
  launch_compliance_sens_raw(g, fixed, ws, prob->E0, prob->Emin, prob->penal, ws + kNaK0, rho_phys,
                             u, f, nsys, c, dc, st);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    fprintf(stderr, "tpcg_compliance_and_sensitivity_noalloc: %s\n", hipGetErrorString(e));
    return TPCG_EHIP;
  }
  return TPCG_OK;
}

// GMRES storage: the small arrays once, the Krylov basis grown to (m + 1)
// nsys vectors when a call needs more (all or nothing each time)
int ensure_gmres(Handle* h, int m, int nsys) {
  if (!h->gm_w) {
    AllocGroup a;
    a.add(h->gm_w, gmres_small_elems());
    a.add(h->gm_i, (size_t)(kNumState + 4) * kMaxSys);
    a.add(h->gm_flags, (size_t)2 * kMaxSys);
    a.add(h->gm_out, (size_t)4 * kMaxSys);
    if (a.commit() != TPCG_OK) {
      (void)hipGetLastError();
      return TPCG_ENOMEM;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&h->gm_host), sizeof(int) * 2 * kMaxSys) != hipSuccess ||
        hipEventCreateWithFlags(&h->gm_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->gm_ev[1], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return TPCG_ENOMEM;
    }
  }
  if ((size_t)(m + 1) * nsys > (size_t)(h->gm_m + 1) * h->gm_nsys || !h->gm_V) {
    if (h->gm_V) hipFree(h->gm_V);
    h->gm_V = nullptr;
    h->gm_m = h->gm_nsys = 0;
    AllocGroup a;
    a.add(h->gm_V, (size_t)(m + 1) * nsys * h->g.ndof);
    if (a.commit() != TPCG_OK) {
      (void)hipGetLastError();
      return TPCG_ENOMEM;
    }
    h->gm_m = m;
    h->gm_nsys = nsys;
  }
  return TPCG_OK;
}

extern "C" {

int tpcg_build_partition(const tpcg_problem* prob, const uint8_t* fixed_mask, void* stream,
                         tpcg_handle** out) {
  if (!prob || !fixed_mask || !out) return TPCG_EINVAL;
  *out = nullptr;
  Geometry g;
  const char* msg = make_geometry(*prob, g);
  if (msg) {
    fprintf(stderr, "tpcg_build_partition: %s\n", msg);
    return TPCG_EINVAL;
  }
  if (prob->nsys_max < 1 || prob->nsys_max > kMaxSys) {
    fprintf(stderr, "tpcg_build_partition: nsys_max must lie in 1..%d\n", kMaxSys);
    return TPCG_EINVAL;
  }
  if (prob->precision != TPCG_FP64 && prob->precision != TPCG_MIXED) return TPCG_EINVAL;
  Handle* h = new (std::nothrow) Handle();
  if (!h) return TPCG_ENOMEM;
  h->prob = *prob;
  h->g = g;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  h->mixed = prob->precision == TPCG_MIXED;
  h->big = local_is_big(g, prob->big_min_nb);
  h->msub = std::min(kMaxSub, g.k + (prob->eig_extra > 0 ? prob->eig_extra : g.k));
  if (h->msub > g.nloc) h->msub = g.nloc;
  const int ns = prob->nsys_max;
  int e = TPCG_OK;
  e |= alloc(h->fixed, g.ndof);
  e |= alloc(h->K0, (size_t)g.ndpe * g.ndpe);
  e |= alloc(h->r, ns * (size_t)g.ndof);
  e |= alloc(h->z, ns * (size_t)g.ndof);
  e |= alloc(h->p, ns * (size_t)g.ndof);
  e |= alloc(h->p2, ns * (size_t)g.ndof);
  e |= alloc(h->q, ns * (size_t)g.ndof);
  e |= alloc(h->fscratch, (size_t)kMaxSys * g.nel);
  e |= alloc(h->parts, kPartsElems);
  e |= alloc(h->istate, (size_t)kNumState * kMaxSys);
  e |= alloc(h->dflag, 4);
  if (e != TPCG_OK) {
    release(h);
    delete h;
    fprintf(stderr, "tpcg_build_partition: out of device memory\n");
    return TPCG_ENOMEM;
  }
  hipMemset(h->dflag, 0, 4 * sizeof(int));
  if (hipHostMalloc(reinterpret_cast<void**>(&h->hpoll), (2 * kMaxSys + 1) * sizeof(int)) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev[1], hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&h->t0) != hipSuccess || hipEventCreate(&h->t1) != hipSuccess ||
      hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->join, hipEventDisableTiming) != hipSuccess) {
    release(h);
    delete h;
    return TPCG_EHIP;
  }
  std::vector<double> K0((size_t)g.ndpe * g.ndpe);
  element_stiffness(g.dim, prob->nu, K0.data());
  hipMemcpy(h->K0, K0.data(), sizeof(double) * K0.size(), hipMemcpyHostToDevice);
  if (g.dim == 2) {
    std::copy(K0.begin(), K0.end(), h->K0q4);
    if (!q4_structured(h->K0q4)) {
      fprintf(stderr, "tpcg_build_partition: Q4 element matrix without the square's structure\n");
      release(h);
      delete h;
      return TPCG_EINVAL;
    }
  } else if (!h8_structured(K0.data(), h->K0h8)) {
    fprintf(stderr, "tpcg_build_partition: H8 element matrix without the cube's structure\n");
    release(h);
    delete h;
    return TPCG_EINVAL;
  }
  hipMemcpy(h->fixed, fixed_mask, g.ndof, hipMemcpyHostToDevice);
  hipMemset(h->istate, 0, sizeof(int) * kNumState * kMaxSys);
  hipMemset(h->parts, 0, sizeof(double) * kPartsElems);
  if (check_hip(h, "tpcg_build_partition") != TPCG_OK) {
    fprintf(stderr, "%s\n", h->err.c_str());
    release(h);
    delete h;
    return TPCG_EHIP;
  }
  *out = reinterpret_cast<tpcg_handle*>(h);
  return TPCG_OK;
}

size_t tpcg_workspace_bytes(const tpcg_problem* prob, int32_t nsys) {
  if (!prob) return 0;
  Geometry g;
  if (make_geometry(*prob, g)) return 0;
  Sizes s = sizes(*prob, g, nsys);
  return s.persistent + s.setup_peak;
}

int tpcg_build_coarse_basis(tpcg_handle* hh, const double* rho_phys, int32_t nsys, int32_t rep) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!rho_phys) return fail(hh, TPCG_EINVAL, "rho_phys is NULL");
  if (nsys < 1 || nsys > h->prob.nsys_max) return fail(hh, TPCG_EINVAL, "nsys out of range");
  if (rep < 0 || rep >= nsys) return fail(hh, TPCG_EINVAL, "rep out of range");
  const Geometry& g = h->g;
  std::string lim = precond_limits(g, h->big);
  if (!lim.empty()) return fail(hh, TPCG_EINVAL, lim);
  int rc = check_rho_sync(h, rho_phys, g.nel, nsys);
  if (rc != TPCG_OK) return rc;
  h->basis_ready = 0;
  if (!h->phi) {
    // preconditioner storage for nsys_max systems, allocated on the first
    // build, all or nothing (a failed build leaves the handle as it was)
    const int ns = h->prob.nsys_max;
    const size_t fsz = h->big ? (size_t)g.nblk * big_shape(g).rec_dir
                              : (size_t)g.nblk * tile_shape(g.nb).tstride;
    const size_t cfsz = (size_t)g.nblkc * g.bstridec;
    const size_t ts = h->mixed ? 4 : 8;
    AllocGroup a;
    a.add(h->phi, (size_t)g.nsub * g.nloc * g.k);
    a.add_bytes(h->phim, ts * (size_t)g.nsub * g.nloc * g.k);
    a.add(h->lam, (size_t)g.nsub * h->msub);
    a.add(h->kj, (size_t)g.nsub);
    a.add(h->cell_sig, (size_t)g.nsub);
    a.add(h->submap_d, (size_t)g.nsub);
    a.add(h->dedup_pairs, (size_t)2 * g.nsub);
    a.add(h->dedup_flag, (size_t)g.nsub);
    a.add(h->eres, (size_t)g.nsub * h->msub);
    a.add_bytes(h->lfac, ts * ns * g.nsub * fsz);
    a.add_bytes(h->emod, ts * ns * (size_t)g.nel);
    if (!h->big) a.add(h->twist, (size_t)ns * g.nsub * g.nb * (g.nb + 1) / 2);
    if (h->mixed) a.add(h->emod64, (size_t)ns * g.nel);
    if (g.nt <= g.dense_max && !g.cband) {
      const size_t T = coarse_tiles(g.nt);
      a.add(h->cpk, (size_t)ns * T * (T + 1) / 2 * kCT * kCT);
      a.add(h->cpart, (size_t)ns * T * T * kCT);
    }
    if (!g.cband && (g.nt > g.dense_max || coarse_btri_fits(g))) a.add(h->cfac, ns * cfsz);
    if (g.cband) {
      a.add(h->cband, (size_t)ns * coarse_band_elems(g));
      a.add(h->cband_w, (size_t)ns * g.nt);
    }
    a.add_bytes(h->zloc, ts * ns * (size_t)g.nsub * g.nloc);
    a.add(h->yc, ns * (size_t)g.nt);
    a.add(h->xc, ns * (size_t)g.nt);
    if (restrict_splits(g) > 1) a.add(h->ycp, (size_t)restrict_splits(g) * kMaxSys * g.nt);
    if (a.commit() != TPCG_OK)
      return fail(hh, TPCG_ENOMEM, "out of device memory for the preconditioner");
  }
  ++h->build_gen;
  return build_preconditioner(*h, rho_phys, nsys, rep, 1);
}

int tpcg_refactor(tpcg_handle* hh, const double* rho_phys, int32_t nsys) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!h->basis_ready) return fail(hh, TPCG_ESTATE, "no coarse basis to keep: build it first");
  if (!rho_phys) return fail(hh, TPCG_EINVAL, "rho_phys is NULL");
  if (nsys < 1 || nsys > h->prob.nsys_max) return fail(hh, TPCG_EINVAL, "nsys out of range");
  int rc = check_rho_sync(h, rho_phys, h->g.nel, nsys);
  if (rc != TPCG_OK) return rc;
  h->basis_ready = 0;
  ++h->build_gen;
  return build_preconditioner(*h, rho_phys, nsys, 0, 0);
}

int tpcg_apply_K(tpcg_handle* hh, const double* rho_phys, const double* x, double* y, int32_t nsys) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!rho_phys || !x || !y) return fail(hh, TPCG_EINVAL, "NULL array");
  if (!aligned16(x) || !aligned16(y)) return fail(hh, TPCG_EINVAL, "vectors must be 16-byte aligned");
  if (nsys < 1 || nsys > h->prob.nsys_max) return fail(hh, TPCG_EINVAL, "nsys out of range");
  int rc = check_rho_sync(h, rho_phys, h->g.nel, nsys);
  if (rc != TPCG_OK) return rc;
  Gate nog = make_gate(h, kPartRR0, 0, 1, 0.0, 0);
  launch_apply_K(*h, rho_phys, x, y, nsys, -1, nog, h->stream);
  return check_hip(h, "tpcg_apply_K");
}

int tpcg_apply_precond(tpcg_handle* hh, const double* r, double* z, int32_t nsys) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!h->basis_ready) return fail(hh, TPCG_ESTATE, "preconditioner not built");
  if (!r || !z) return fail(hh, TPCG_EINVAL, "NULL array");
  if (nsys != h->nsys_built) return fail(hh, TPCG_EINVAL, "nsys differs from the build");
  Gate nog = make_gate(h, kPartRR0, 0, 1, 0.0, 0);
  launch_precond(*h, r, z, nsys, nog, kPartAux, -2, 0, h->stream);
  return check_hip(h, "tpcg_apply_precond");
}

// info -> host results after polling (the synchronous solve); dinfo ->
// device results, every iteration up to maxit enqueued with no host wait
static int pcg_solve_impl(tpcg_handle* hh, const double* rho_phys, const double* f, double* u,
                          int32_t nsys, double rtol, int32_t maxit, tpcg_info* info,
                          tpcg_info* dinfo) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!h->basis_ready) return fail(hh, TPCG_ESTATE, "preconditioner not built");
  if (!rho_phys || !f || !u || (!info && !dinfo)) return fail(hh, TPCG_EINVAL, "NULL argument");
  if (!aligned16(f) || !aligned16(u)) return fail(hh, TPCG_EINVAL, "vectors must be 16-byte aligned");
  if (nsys != h->nsys_built) return fail(hh, TPCG_EINVAL, "nsys differs from the build");
  if (!(rtol > 0.0) || maxit < 0) return fail(hh, TPCG_EINVAL, "rtol must be > 0 and maxit >= 0");
  if (!dinfo) tune_before_solve(*h);
  hipStream_t st = h->stream;
  const double tol2 = rtol * rtol;
  const int flexible = h->mixed;
  const int pe = std::min(std::max(h->poll_every, 1), kMaxPoll);   // iterations per chunk
  const auto wall0 = std::chrono::steady_clock::now();
  hipEventRecord(h->t0, st);
  // r0 = P (f - K u0); z0 = M^-1 r0; p0 = z0
  Gate g0 = make_gate(h, kPartRR0, 0, maxit, tol2, 1);
  Gate nog = g0;
  nog.enabled = 0;
  launch_apply_K(*h, rho_phys, u, h->q, nsys, -1, nog, st);
  launch_residual_init(*h, f, u, h->q, nsys, st);
  // a system with invalid densities never starts and reports TPCG_EINVAL
  launch_check_rho(rho_phys, h->g.nel, nsys, h->istate + kStBreak * kMaxSys, 1, 2, st);
  launch_gate(*h, nsys, g0, st);
  h->prof_n = 0;
  launch_precond(*h, h->r, h->z, nsys, g0, kPartRZ0, -1, flexible, st);
  launch_beta(*h, nsys, g0, kPartRZ0, flexible, 1, st);
  // the direction update p = z + beta p runs inside the next operator
  // launch, alternating between two buffers
  double* pcur = h->p;
  double* pnext = h->p2;
  int* itbase = h->istate + kStIter * kMaxSys;
  // one PCG iteration; `itg` is the gates' iteration (absolute, or an offset
  // from the device counter when `rel`), its parity picks the partial slots
  auto iteration = [&](int itg, bool rel, int first, int prof_it, double*& pc, double*& pn,
                       hipStream_t st) {
    const int rr_now = (itg & 1) ? kPartRR1 : kPartRR0;
    const int rr_next = (itg & 1) ? kPartRR0 : kPartRR1;
    const int rz_next = (itg & 1) ? kPartRZ0 : kPartRZ1;
    Gate gi = make_gate(h, rr_now, itg, maxit, tol2, 1);
    Gate gn = make_gate(h, rr_next, itg + 1, maxit, tol2, 1);
    if (rel) gi.itbase = gn.itbase = itbase;
    launch_apply_K_dir(*h, rho_phys, h->z, pc, pn, h->q, nsys, kPartPQ, gi, first, st);
    std::swap(pc, pn);
    launch_update_xr(*h, u, pc, nsys, gi, st);
    Gate gt = gn;   // the restriction takes this iteration's residual test
    gt.test = 1;
    launch_precond(*h, h->r, h->z, nsys, gt, rz_next, prof_it, flexible, st);
    launch_beta(*h, nsys, gn, rz_next, flexible, 0, st);
  };
  if (dinfo) {
    // asynchronous: every iteration enqueued (the gates stop each system at
    // its own convergence; the launches after it return at once), then the
    // summary into device memory
    for (int it = 0; it < maxit; ++it) iteration(it, false, it == 0, -2, pcur, pnext, st);
    Gate gf = make_gate(h, (maxit & 1) ? kPartRR1 : kPartRR0, maxit, maxit, tol2, 1);
    launch_apply_K(*h, rho_phys, u, h->q, nsys, -1, nog, st);
    double* dout = h->parts + (size_t)kNumPartSlots * kMaxSys * kMaxParts;
    launch_summary(*h, f, nsys, gf, dout, st);
    hipLaunchKernelGGL(k_info_pack, dim3(1), dim3(64), 0, st, dout, nsys, dinfo);
    return check_hip(h, "tpcg_pcg_solve_async");
  }
  // Chunks after the first replay a captured graph of poll_every iterations
  // (a chunk starts at an even iteration with the direction buffers in their
  // initial order, so one graph serves every chunk); the block coarse solve
  // on the side stream stays eager, and so do solves that time their local
  // solves with events (events recorded inside a graph cannot be timed).
  const bool use_graphs = h->graphs_on && h->graphs_ok && h->cpk != nullptr && !h->prof_on;
  if (use_graphs) {
    std::vector<double> key = {(double)reinterpret_cast<uintptr_t>(rho_phys),
                               (double)reinterpret_cast<uintptr_t>(f),
                               (double)reinterpret_cast<uintptr_t>(u),
                               (double)nsys, (double)maxit, tol2, (double)flexible,
                               (double)h->prof_on, (double)h->build_gen, (double)pe};
    if (key != h->gkey) {
      drop_graphs(h);
      h->gkey = key;
    }
  }
  // captured on the handle's side stream (a stream of its own, which can be
  // captured even when the handle's stream is the legacy default stream),
  // replayed on the handle's stream
  hipStream_t cs = h->side;
  auto capture = [&](int g) {
    if (h->prof_on)
      for (auto& e : h->gprof_ev[g])
        if (!e && hipEventCreate(&e) != hipSuccess) return false;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      fprintf(stderr, "tpcg_pcg_solve: graph capture not available (%s); eager launches\n",
              hipGetErrorString(e));
      return false;
    }
    h->cap_ev = h->prof_on ? h->gprof_ev[g] : nullptr;
    h->cap_n = 0;
    double* pc = h->p;
    double* pn = h->p2;
    for (int off = 0; off < pe; ++off) iteration(off, true, 0, off, pc, pn, cs);
    h->cap_ev = nullptr;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess || !graph) {
      fprintf(stderr, "tpcg_pcg_solve: graph capture failed (%s); eager launches\n",
              hipGetErrorString(e));
      return false;
    }
    e = hipGraphInstantiate(&h->gexec[g], graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
      fprintf(stderr, "tpcg_pcg_solve: graph instantiation failed (%s); eager launches\n",
              hipGetErrorString(e));
      h->gexec[g] = nullptr;
      return false;
    }
    return true;
  };
  int it = 0;
  int chunk = 0;
  int graph_it0[2] = {-1, -1};   // first iteration of the unharvested chunk of each graph
  std::vector<std::pair<int, float>> gprof;   // (iteration, ms) of graph-timed local solves
  auto harvest = [&](int g) {
    if (graph_it0[g] < 0) return;
    if (h->prof_on)
      for (int k = 0; k < pe; ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, h->gprof_ev[g][2 * k], h->gprof_ev[g][2 * k + 1]) == hipSuccess)
          gprof.emplace_back(graph_it0[g] + k, ms);
      }
    graph_it0[g] = -1;
  };
  h->last_graph_chunks = 0;
  bool done = maxit == 0;
  while (!done) {
    const int it0 = it;
    bool graphed = false;
    if (use_graphs && h->graphs_ok && chunk >= 1) {
      const int g = chunk & 1;
      if (!h->gexec[g] && !capture(g)) {
        (void)hipGetLastError();
        hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(cs, &cst) == hipSuccess && cst != hipStreamCaptureStatusNone) {
          hipGraph_t junk = nullptr;
          hipStreamEndCapture(cs, &junk);
          if (junk) hipGraphDestroy(junk);
        }
        (void)hipGetLastError();
        h->cap_ev = nullptr;
        h->graphs_ok = 0;
        drop_graphs(h);
      }
      if (h->gexec[g] && hipGraphLaunch(h->gexec[g], st) == hipSuccess) {
        graphed = true;
        graph_it0[g] = it0;
        it = it0 + pe;
        ++h->last_graph_chunks;
      }
    }
    if (!graphed)
      for (int c = 0; c < pe && it < maxit; ++c, ++it)
        iteration(it, false, it == 0, it, pcur, pnext, st);
    const int slot = chunk & 1;
    Gate gp = make_gate(h, (it & 1) ? kPartRR1 : kPartRR0, it, maxit, tol2, 1);
    launch_poll(*h, nsys, gp, it - it0, st);
    hipMemcpyAsync(h->hpoll + slot * kMaxSys, h->istate + kStPoll * kMaxSys, sizeof(int) * kMaxSys,
                   hipMemcpyDeviceToHost, st);
    hipEventRecord(h->ev[slot], st);
    if (it >= maxit) break;
    if (chunk > 0) {
      const int prev = slot ^ 1;
      if (hipEventSynchronize(h->ev[prev]) != hipSuccess) break;
      harvest(prev);
      int running = 0;
      for (int s = 0; s < nsys; ++s) running |= h->hpoll[prev * kMaxSys + s];
      if (!running) done = true;
    }
    ++chunk;
  }
  // summary: true residual with a fresh K u
  Gate gf = make_gate(h, (it & 1) ? kPartRR1 : kPartRR0, it, maxit, tol2, 1);
  launch_apply_K(*h, rho_phys, u, h->q, nsys, -1, nog, st);
  double* dout = h->parts + (size_t)kNumPartSlots * kMaxSys * kMaxParts;   // 4 * kMaxSys spare
  launch_summary(*h, f, nsys, gf, dout, st);
  hipEventRecord(h->t1, st);
  double hout[4 * kMaxSys];
  hipMemcpyAsync(hout, dout, sizeof(double) * 4 * nsys, hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  harvest(0);
  harvest(1);
  int rc = check_hip(h, "tpcg_pcg_solve");
  if (rc != TPCG_OK) return rc;
  float ms = 0.0f;
  hipEventElapsedTime(&ms, h->t0, h->t1);
  (void)wall0;
  int worst = TPCG_OK;
  for (int s = 0; s < nsys; ++s) {
    info[s].iters = (int)hout[4 * s + 0];
    info[s].status = (int)hout[4 * s + 1];
    info[s].relres = hout[4 * s + 2];
    info[s].true_relres = hout[4 * s + 3];
    info[s].seconds = ms * 1e-3;
    const int st_s = info[s].status;
    if (st_s < 0 && (worst >= 0 || st_s < worst)) worst = st_s;
    else if (worst == TPCG_OK && st_s > 0) worst = st_s;
  }
  if (h->prof_on) {
    // attribute each timed block-solve launch its algorithmic bytes: only the
    // systems still running at that iteration did work
    const Geometry& g = h->g;
    const double per_sys = local_solve_bytes(g, h->mixed ? 4 : 8, h->big);
    auto account = [&](int pit, float lms) {
      int running = 0;
      for (int s = 0; s < nsys; ++s) running += info[s].iters >= pit + 2;
      if (!running) return;
      h->prof_ms += lms;
      h->prof_bytes += running * per_sys;
      h->prof_launches += 1;
    };
    for (int i = 0; i < h->prof_n; ++i) {
      float lms = 0.0f;
      hipEventElapsedTime(&lms, h->prof_ev[2 * i], h->prof_ev[2 * i + 1]);
      account(h->prof_it[i], lms);
    }
    for (const auto& e : gprof) account(e.first, e.second);
  }
  {
    int most = 0;
    for (int s = 0; s < nsys; ++s) most = std::max(most, info[s].iters);
    tune_after_solve(*h, ms, most);
  }
  if (worst == TPCG_EINVAL) h->err = "densities must lie in [0, 1] (NaN or out-of-range value found)";
  else if (worst == TPCG_EBREAKDOWN) h->err = "PCG breakdown (p^T K p <= 0, r^T z <= 0 or NaN)";
  else if (worst == TPCG_ENOCONV) h->err = "maxit reached before rtol";
  return worst;
}

int tpcg_apply_msfem(tpcg_handle* hh, const double* rho_phys, const double* r, double* z,
                     int32_t nsys) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!h->basis_ready) return fail(hh, TPCG_ESTATE, "preconditioner not built");
  if (!rho_phys || !r || !z) return fail(hh, TPCG_EINVAL, "NULL array");
  if (r == z) return fail(hh, TPCG_EINVAL, "r and z must be distinct");
  if (!aligned16(r) || !aligned16(z)) return fail(hh, TPCG_EINVAL, "vectors must be 16-byte aligned");
  if (nsys != h->nsys_built) return fail(hh, TPCG_EINVAL, "nsys differs from the build");
  int rc = check_rho_sync(h, rho_phys, h->g.nel, nsys);
  if (rc != TPCG_OK) return rc;
  Gate nog = make_gate(h, kPartRR0, 0, 1, 0.0, 0);
  launch_msfem_cycle(*h, rho_phys, r, z, nsys, nog, h->stream);
  return check_hip(h, "tpcg_apply_msfem");
}

int tpcg_gmres_solve(tpcg_handle* hh, const double* rho_phys, const double* f, double* u,
                     int32_t nsys, double rtol, int32_t maxit, int32_t restart, int32_t precond,
                     tpcg_info* info) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!h->basis_ready) return fail(hh, TPCG_ESTATE, "preconditioner not built");
  if (!rho_phys || !f || !u || !info) return fail(hh, TPCG_EINVAL, "NULL argument");
  if (!aligned16(f) || !aligned16(u)) return fail(hh, TPCG_EINVAL, "vectors must be 16-byte aligned");
  if (nsys != h->nsys_built) return fail(hh, TPCG_EINVAL, "nsys differs from the build");
  if (!(rtol > 0.0) || maxit < 0) return fail(hh, TPCG_EINVAL, "rtol must be > 0 and maxit >= 0");
  if (restart < 1 || restart > kGmMaxRestart)
    return fail(hh, TPCG_EINVAL, "restart must lie in 1..64");
  if (precond != TPCG_PC_ADDITIVE && precond != TPCG_PC_MSFEM_SGS)
    return fail(hh, TPCG_EINVAL, "unknown preconditioner kind");
  int rc = check_rho_sync(h, rho_phys, h->g.nel, nsys);
  if (rc != TPCG_OK) return rc;
  if (ensure_gmres(h, restart, nsys) != TPCG_OK)
    return fail(hh, TPCG_ENOMEM, "GMRES basis allocation failed");
  tune_gmres(*h, nsys, restart);
  hipStream_t st = h->stream;
  hipEventRecord(h->t0, st);
  double hout[4 * kMaxSys];
  rc = gmres_solve(*h, rho_phys, f, u, nsys, rtol, maxit, restart, precond, hout);
  hipEventRecord(h->t1, st);
  hipEventSynchronize(h->t1);
  const int hrc = check_hip(h, "tpcg_gmres_solve");
  if (hrc != TPCG_OK) return hrc;
  if (rc != TPCG_OK) return fail(hh, rc, "GMRES: HIP error while polling");
  float ms = 0.0f;
  hipEventElapsedTime(&ms, h->t0, h->t1);
  int worst = TPCG_OK;
  for (int s = 0; s < nsys; ++s) {
    info[s].iters = (int)hout[4 * s + 0];
    info[s].status = (int)hout[4 * s + 1];
    info[s].relres = hout[4 * s + 2];
    info[s].true_relres = hout[4 * s + 3];
    info[s].seconds = ms * 1e-3;
    const int st_s = info[s].status;
    if (st_s < 0 && (worst >= 0 || st_s < worst)) worst = st_s;
    else if (worst == TPCG_OK && st_s > 0) worst = st_s;
  }
  if (worst == TPCG_EBREAKDOWN) h->err = "GMRES breakdown (NaN or a zero rotation)";
  else if (worst == TPCG_ENOCONV) h->err = "maxit reached before rtol";
  return worst;
}

int tpcg_pcg_solve(tpcg_handle* hh, const double* rho_phys, const double* f, double* u,
                   int32_t nsys, double rtol, int32_t maxit, tpcg_info* info) {
  return pcg_solve_impl(hh, rho_phys, f, u, nsys, rtol, maxit, info, nullptr);
}

int tpcg_pcg_solve_async(tpcg_handle* hh, const double* rho_phys, const double* f, double* u,
                         int32_t nsys, double rtol, int32_t maxit, tpcg_info* info_dev) {
  if (!info_dev) return fail(hh, TPCG_EINVAL, "NULL info");
  return pcg_solve_impl(hh, rho_phys, f, u, nsys, rtol, maxit, nullptr, info_dev);
}

int tpcg_compliance_and_sensitivity(tpcg_handle* hh, const double* rho_phys, const double* u,
                                    const double* f, int32_t nsys, double* c, double* dc) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!rho_phys || !u || !f || !c) return fail(hh, TPCG_EINVAL, "NULL argument");
  if (nsys < 1 || nsys > h->prob.nsys_max) return fail(hh, TPCG_EINVAL, "nsys out of range");
  if (dc) {
    int rc = check_rho_sync(h, rho_phys, h->g.nel, nsys);
    if (rc != TPCG_OK) return rc;
  }
  launch_compliance_sens(*h, rho_phys, u, f, nsys, c, dc, h->stream);
  return check_hip(h, "tpcg_compliance_and_sensitivity");
}

int tpcg_filter_project(tpcg_handle* hh, const double* rho, double rmin, double beta,
                        const double* eta, int32_t nsys, double* rho_tilde, double* rho_phys) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!rho || !eta || !rho_tilde || !rho_phys) return fail(hh, TPCG_EINVAL, "NULL argument");
  if (nsys < 1 || nsys > kMaxSys) return fail(hh, TPCG_EINVAL, "nsys out of range");
  if (!(beta > 0.0)) return fail(hh, TPCG_EINVAL, "beta must be > 0");
  if (rmin > 8.0) return fail(hh, TPCG_EINVAL, "rmin above 8 elements is not supported");
  int rc = check_rho_sync(h, rho, h->g.nel, 1);
  if (rc != TPCG_OK) return rc;
  launch_filter_project(*h, rho, rmin, beta, eta, nsys, rho_tilde, rho_phys, h->stream);
  return check_hip(h, "tpcg_filter_project");
}

int tpcg_robust_objective(tpcg_handle* hh, const double* c, const double* dc, int32_t nsys,
                          double kappa, const double* weights, double* out3, double* df) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!c || !out3 || (dc && !df)) return fail(hh, TPCG_EINVAL, "NULL argument");
  if (nsys < 1 || nsys > kMaxSys) return fail(hh, TPCG_EINVAL, "nsys out of range");
  if (!(kappa >= 0.0)) return fail(hh, TPCG_EINVAL, "kappa must be >= 0");
  double w[kMaxSys];
  for (int s = 0; s < nsys; ++s) {
    w[s] = weights ? weights[s] : 1.0 / nsys;
    if (!(w[s] >= 0.0)) return fail(hh, TPCG_EINVAL, "weights must be >= 0");
  }
  launch_robust(*h, c, dc, nsys, kappa, w, out3, df, h->stream);
  return check_hip(h, "tpcg_robust_objective");
}

int tpcg_nondiscreteness(tpcg_handle* hh, const double* rho_phys, double* out) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!rho_phys || !out) return fail(hh, TPCG_EINVAL, "NULL argument");
  launch_nondiscreteness(*h, rho_phys, out, h->stream);
  return check_hip(h, "tpcg_nondiscreteness");
}

int tpcg_periodic_sum(tpcg_handle* hh, const double* g, int32_t nsys, const int32_t* cell,
                      double* gcell) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!g || !cell || !gcell) return fail(hh, TPCG_EINVAL, "NULL argument");
  if (nsys < 1 || nsys > kMaxSys) return fail(hh, TPCG_EINVAL, "nsys out of range");
  const int cz = h->g.dim == 3 ? cell[2] : 1;
  if (cell[0] < 1 || cell[1] < 1 || cz < 1 || cell[0] > h->g.nelx || cell[1] > h->g.nely ||
      cz > h->g.nelz)
    return fail(hh, TPCG_EINVAL, "unit cell must lie within the mesh");
  launch_periodic_sum(*h, g, nsys, cell[0], cell[1], cz, gcell, h->stream);
  return check_hip(h, "tpcg_periodic_sum");
}

int tpcg_filter_project_adjoint(tpcg_handle* hh, const double* rho_tilde, double rmin, double beta,
                                const double* eta, int32_t nsys, const double* dc_drho_phys,
                                double* dc_drho) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (h->sticky) return fail(hh, TPCG_EHIP, "handle has a sticky HIP error");
  if (!rho_tilde || !eta || !dc_drho_phys || !dc_drho) return fail(hh, TPCG_EINVAL, "NULL argument");
  if (nsys < 1 || nsys > kMaxSys) return fail(hh, TPCG_EINVAL, "nsys out of range");
  if (!(beta > 0.0)) return fail(hh, TPCG_EINVAL, "beta must be > 0");
  if (rmin > 8.0) return fail(hh, TPCG_EINVAL, "rmin above 8 elements is not supported");
  launch_filter_project_adjoint(*h, rho_tilde, rmin, beta, eta, nsys, dc_drho_phys, dc_drho,
                                h->stream);
  return check_hip(h, "tpcg_filter_project_adjoint");
}

int tpcg_export_coarse_basis(tpcg_handle* hh, double* phi, double* lambda, double* resid) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (!h->basis_ready) return fail(hh, TPCG_ESTATE, "preconditioner not built");
  const Geometry& g = h->g;
  hipStreamSynchronize(h->stream);
  if (phi)
    hipMemcpy(phi, h->phi, sizeof(double) * (size_t)g.nsub * g.nloc * g.k, hipMemcpyDeviceToDevice);
  std::vector<double> tmp((size_t)g.nsub * h->msub);
  for (int which = 0; which < 2; ++which) {
    double* dst = which == 0 ? lambda : resid;
    if (!dst) continue;
    hipMemcpy(tmp.data(), which == 0 ? h->lam : h->eres, sizeof(double) * tmp.size(),
              hipMemcpyDeviceToHost);
    for (int j = 0; j < g.nsub; ++j)
      for (int i = 0; i < g.k; ++i) dst[(size_t)j * g.k + i] = tmp[(size_t)j * h->msub + i];
  }
  return check_hip(h, "tpcg_export_coarse_basis");
}

int tpcg_export_local_record(tpcg_handle* hh, int32_t sys, int32_t sub, int32_t blk, double* out) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (!h->basis_ready) return fail(hh, TPCG_ESTATE, "preconditioner not built");
  const Geometry& g = h->g;
  if (!h->big) return fail(hh, TPCG_EINVAL, "records of the on-chip path are not exported");
  if (!out || sys < 0 || sys >= h->nsys_built || sub < 0 || sub >= g.nsub || blk < 0 ||
      blk >= g.nblk)
    return fail(hh, TPCG_EINVAL, "record index out of range");
  const BigShape bs = big_shape(g);
  const size_t off = ((size_t)(sys * g.nsub + sub) * g.nblk + blk) * bs.rec_dir;
  std::vector<double> rec(bs.rec_dir);
  hipStreamSynchronize(h->stream);
  if (h->mixed) {
    std::vector<float> tmp(bs.rec_dir);
    hipMemcpy(tmp.data(), reinterpret_cast<float*>(h->lfac) + off, sizeof(float) * tmp.size(),
              hipMemcpyDeviceToHost);
    for (size_t i = 0; i < tmp.size(); ++i) rec[i] = tmp[i];
  } else {
    hipMemcpy(rec.data(), reinterpret_cast<double*>(h->lfac) + off, sizeof(double) * rec.size(),
              hipMemcpyDeviceToHost);
  }
  const int nb = g.nb;
  for (int r = 0; r < nb; ++r)
    for (int c = 0; c < nb; ++c) {
      const int R = r >= c ? r : c, C = r >= c ? c : r;   // lower tiles hold the symmetric matrix
      const int I = R / kBT, J = C / kBT;
      int rr = R % kBT, cc = C % kBT;
      if (I == J) { rr = r % kBT; cc = c % kBT; }          // diagonal tiles are stored in full
      out[(size_t)r * nb + c] = rec[(size_t)big_ltile(I, J) * kBTE + big_cofs(rr, cc)];
    }
  return check_hip(h, "tpcg_export_local_record");
}

int tpcg_query(const tpcg_handle* hh, int64_t* out) {
  const Handle* h = H(hh);
  if (!h || !out) return TPCG_EINVAL;
  const Geometry& g = h->g;
  int64_t v[9] = {g.ndof, g.nel, g.nsub, g.nloc, g.k, g.nb, g.nblk, g.nbc, g.nblkc};
  std::memcpy(out, v, sizeof(v));
  return TPCG_OK;
}

int tpcg_set_profiling(tpcg_handle* hh, int32_t on) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  h->prof_on = on ? 1 : 0;
  h->prof_ms = 0.0;
  h->prof_bytes = 0.0;
  h->prof_launches = 0;
  return TPCG_OK;
}

int tpcg_profile_block_solves(const tpcg_handle* hh, double* out3) {
  const Handle* h = H(hh);
  if (!h || !out3) return TPCG_EINVAL;
  out3[0] = (double)h->prof_launches;
  out3[1] = h->prof_ms;
  out3[2] = h->prof_bytes;
  return TPCG_OK;
}

int tpcg_export_eigenvalues(tpcg_handle* hh, double* lambda, int32_t m, int32_t* kj) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  if (!h->basis_ready) return fail(hh, TPCG_ESTATE, "preconditioner not built");
  if (m < 0 || m > h->msub) return fail(hh, TPCG_EINVAL, "m exceeds the eigensolver's subspace");
  const Geometry& g = h->g;
  hipStreamSynchronize(h->stream);
  if (lambda && m > 0) {
    std::vector<double> tmp((size_t)g.nsub * h->msub);
    hipMemcpy(tmp.data(), h->lam, sizeof(double) * tmp.size(), hipMemcpyDeviceToHost);
    for (int j = 0; j < g.nsub; ++j)
      for (int i = 0; i < m; ++i) lambda[(size_t)j * m + i] = tmp[(size_t)j * h->msub + i];
  }
  if (kj) hipMemcpy(kj, h->kj, sizeof(int) * g.nsub, hipMemcpyDeviceToHost);
  return check_hip(h, "tpcg_export_eigenvalues");
}

int tpcg_query_unique_cells(const tpcg_handle* hh) {
  const Handle* h = H(hh);
  return h ? h->nrep : TPCG_EINVAL;
}

int tpcg_query_subspace(const tpcg_handle* hh) {
  const Handle* h = H(hh);
  return h ? h->msub : TPCG_EINVAL;
}

int tpcg_set_graphs(tpcg_handle* hh, int32_t on) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  h->graphs_on = on ? 1 : 0;
  if (!on) drop_graphs(h);
  return TPCG_OK;
}

int tpcg_set_autotune(tpcg_handle* hh, int32_t on) {
  Handle* h = H(hh);
  if (!h) return TPCG_EINVAL;
  h->tune_on = on ? 1 : 0;
  return TPCG_OK;
}

int tpcg_query_tune(const tpcg_handle* hh, int32_t* out) {
  const Handle* h = H(hh);
  if (!h || !out) return TPCG_EINVAL;
  out[0] = h->tune_on;
  out[1] = h->tune_decided;
  out[2] = h->tune_from_cache;
  out[3] = h->graphs_on;
  out[4] = h->poll_every;
  out[5] = h->tune_gm_decided;
  out[6] = h->gm_chunk;
  out[7] = h->tune_seen;
  return TPCG_OK;
}

int tpcg_last_solve_graph_chunks(const tpcg_handle* hh) {
  const Handle* h = H(hh);
  return h ? h->last_graph_chunks : TPCG_EINVAL;
}

void tpcg_test_fail_alloc(int32_t nth) {
  g_fail_at = nth > 0 ? nth : 0;
  g_alloc_count = 0;
}

const char* tpcg_last_error(const tpcg_handle* hh) {
  const Handle* h = H(hh);
  return h ? h->err.c_str() : "null handle";
}

void tpcg_destroy(tpcg_handle* hh) {
  Handle* h = H(hh);
  if (!h) return;
  hipStreamSynchronize(h->stream);
  release(h);
  delete h;
}

}  // extern "C"

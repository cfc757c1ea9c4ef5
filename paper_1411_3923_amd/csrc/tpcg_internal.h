// Internal declarations of the tpcg library: geometry, handle state, device
// helpers and the kernel launchers shared between translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "tpcg.h"

namespace tpcg {

constexpr int kThreads = 256;        // threads per workgroup (4 wave64)
constexpr int kMaxParts = 2048;      // reduction partials per system and vector kernel
constexpr int kMaxSys = 4;           // systems solved together
constexpr int kMaxK = 16;            // coarse vectors per subdomain
constexpr int kMaxPoll = 8;          // longest PCG chunk between convergence polls
constexpr int kGmMaxRestart = 64;    // GMRES: longest cycle
constexpr int kGmMaxVec = kGmMaxRestart + 1;
constexpr int kMaxSub = 16;          // eigensolver subspace width
constexpr int kMaxNb = 96;           // largest block of the block-tridiagonal kernels
constexpr int kDenseCoarse = 12288;  // coarse dimensions up to this keep a dense K_c^-1
constexpr int kCT = 64;              // tile edge of the packed K_c^-1
__host__ __device__ inline int coarse_tiles(int nt) { return (nt + kCT - 1) / kCT; }

// Structured-mesh and partition sizes. Everything is derived from the problem.
struct Geometry {
  int dim;
  int nelx, nely, nelz;              // elements per axis (nelz = 1 in 2D)
  int nnx, nny, nnz;                 // nodes per axis (nnz = 1 in 2D)
  int64_t nnodes, ndof, nel;
  int s;                             // subdomain edge in elements
  int gx, gy, gz;                    // subdomains per axis (gz = 1 in 2D)
  int nsub;
  int bn;                            // nodes per box edge (s + 1)
  int nbox;                          // nodes per subdomain box
  int nloc;                          // DOFs per subdomain box
  int nb, nblk;                      // local block-tridiagonal: block size, block count
  int k;                             // coarse vectors per subdomain
  int caxis;                         // coarse blocks run along this subdomain axis
  int pe, bstride;                   // local packed factor: band diagonals of B, record length
  int nbc, nblkc;                    // coarse block size, block count
  int pec, bstridec;                 // coarse packed factor
  int nt;                            // coarse dimension nsub * k
  int dense_max;                     // coarse dimensions up to this keep a dense K_c^-1
  int ebn;                           // nodes per extended box edge (s + 3)
  int nebox;                         // nodes per extended box
  int ndpe;                          // DOFs per element (8 or 24)
  int cband;                         // coarse level as the HBM-resident block-tridiagonal factor
  const int* submap;                 // eigen phase over distinct cells only: the subdomain of
                                     // each launch index (device array; nullptr: identity)
};

// subdomain of launch index c of the eigen phase
__device__ inline int phys_sub(const Geometry& g, int c) { return g.submap ? g.submap[c] : c; }

// Coarse index of (subdomain j, mode m): block-major along `caxis`.
__host__ __device__ inline int coarse_index(const Geometry& g, int jx, int jy, int jz, int m) {
  int blk, w;
  if (g.caxis == 0) { blk = jx; w = jy + g.gy * jz; }
  else if (g.caxis == 1) { blk = jy; w = jx + g.gx * jz; }
  else { blk = jz; w = jx + g.gx * jy; }
  return blk * g.nbc + w * g.k + m;
}

// global DOF of local DOF l (box order) of subdomain (jx, jy, jz)
__device__ inline int64_t box_dof(const Geometry& g, int jx, int jy, int jz, int l) {
  const int d = g.dim;
  const int ln = l / d, c = l - ln * d;
  const int lx = ln % g.bn;
  const int rest = ln / g.bn;
  const int ly = rest % g.bn;
  const int lz = rest / g.bn;
  const int64_t n = (int64_t)(g.s * jx + lx) +
                    (int64_t)g.nnx * ((g.s * jy + ly) + (int64_t)g.nny * (g.s * jz + lz));
  return d * n + c;
}

__host__ __device__ inline void sub_coords(const Geometry& g, int j, int& jx, int& jy, int& jz) {
  jx = j % g.gx;
  jy = (j / g.gx) % g.gy;
  jz = j / (g.gx * g.gy);
}

struct Handle {
  tpcg_problem prob;
  Geometry g;
  hipStream_t stream = nullptr;
  std::string err;
  int sticky = 0;
  int mixed = 0;

  // problem data
  uint8_t* fixed = nullptr;          // [ndof]
  double* K0 = nullptr;              // [ndpe * ndpe]
  double K0q4[64] = {};              // host copy of the Q4 element matrix (2-d)
  double K0h8[12] = {};              // the H8 element matrix's twelve class values (3-d)

  // preconditioner state
  int basis_ready = 0;
  int big = 0;                       // subdomain blocks take the HBM-resident factors (big.h)
  int nsys_built = 0;
  int msub = 0;                      // eigensolver subspace width
  double* phi = nullptr;             // [nsub][nloc][k]
  void* phim = nullptr;              // mode-major copy [nsub][k][nloc], double (FP32 when mixed)
  double* lam = nullptr;             // [nsub][msub] Ritz values
  int* kj = nullptr;                 // [nsub] coarse vectors in use (the rest of the k columns are zero)
  double* eres = nullptr;            // [nsub][msub] residual norms
  void* lfac = nullptr;              // tiled D_b [nsys][nsub][nblk][tstride], double or float
  void* emod = nullptr;              // moduli the local factors were built from [nsys][nel], same type
  double* twist = nullptr;           // Schur terms of the lower halves, [nsys][nsub][nb (nb + 1) / 2]
  double* emod64 = nullptr;          // FP64 moduli (mixed precision), [nsys][nel]
  double* cfac = nullptr;            // block-tridiagonal coarse factor [nsys][nblkc][bstridec]
                                     // (coarse dimensions above dense_max only)
  double* cpk = nullptr;             // lower 64 x 64 tiles of the dense K_c^-1 (nt <= dense_max)
                                     // [nsys][T (T + 1) / 2][64][64]
  double* cpart = nullptr;           // tile partials of K_c^-1 y_c [nsys][T][T][64]
  double* build_ws = nullptr;        // work arrays of the preconditioner build
  double* fscratch = nullptr;        // [kMaxSys][nel] element factors of the filter adjoint
  double* cband = nullptr;           // HBM-resident coarse factor [nsys][coarse_band_elems]
  double* cband_w = nullptr;         // its solve's forward-chain vector [nsys][nt]
  // one eigenproblem per distinct cell (tpcg_problem.dedup): signatures, the
  // distinct cells' subdomains, (duplicate, representative) pairs, flags of
  // the exact comparison; nrep = eigenproblems solved by the last build
  unsigned long long* cell_sig = nullptr;   // [nsub]
  int* submap_d = nullptr;                  // [nsub]
  int* dedup_pairs = nullptr;               // [nsub][2]
  int* dedup_flag = nullptr;                // [nsub]
  int nrep = 0;
  size_t build_elems = 0;
  hipStream_t side = nullptr;        // second stream: the block coarse solve, the setup's local factors
  hipEvent_t fork = nullptr, join = nullptr;

  // workspace
  double* r = nullptr;               // [nsys_max][ndof]
  double* z = nullptr;
  double* p = nullptr;
  double* p2 = nullptr;              // second direction buffer (fused update)
  double* q = nullptr;
  void* zloc = nullptr;              // [nsys][nsub][nloc], double or float
  double* yc = nullptr;              // [nsys][nt]
  double* ycp = nullptr;             // [restrict_splits][kMaxSys][nt] restriction parts (or null)
  double* xc = nullptr;              // [nsys][nt]
  double* parts = nullptr;           // reduction partials, see kParts* offsets
  int* istate = nullptr;             // per-system integer state, see kSt*
  int* hpoll = nullptr;              // pinned host [2][kMaxSys], then one validation flag
  int* dflag = nullptr;              // device error flags [4]
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t t0 = nullptr, t1 = nullptr;

  // PCG chunks replayed from HIP graphs: two instantiated graphs of
  // poll_every iterations (chunks alternate between them, so that a chunk's
  // timing events can be read while the next one runs), captured for the
  // arguments in gkey and recaptured when they change
  int poll_every = 4;                // PCG iterations between convergence polls
  int graphs_on = 0;                 // off by default: measured slower than eager launches
  int graphs_ok = 1;                 // 0 after a capture failed: eager launches only
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::vector<double> gkey;
  hipEvent_t gprof_ev[2][2 * kMaxPoll] = {};   // per graph: event pairs around its local solves

  // autotuning of launch choices that leave every result bit for bit the
  // same (tune.hip): the PCG launch mode and poll interval, measured over
  // the handle's first solves, and the GMRES dot-product grouping; the
  // choices are kept in an on-disk cache keyed by device and problem
  int tune_on = 0;
  int tune_decided = 0;              // the PCG choice is in force
  int tune_from_cache = 0;
  int tune_seen = 0;                 // solves seen while measuring
  int tune_cand = -1;                // candidate of the running solve (-1: warm-up or none)
  double tune_ms[4] = {0.0, 0.0, 0.0, 0.0};   // best ms per iteration of each candidate
  int tune_gm_decided = 0;
  int gm_chunk = 8;                  // Krylov vectors per workgroup of the GMRES dot products
  hipEvent_t* cap_ev = nullptr;      // during a capture: the events the marks record
  int cap_n = 0;
  int last_graph_chunks = 0;
  int build_gen = 0;                 // preconditioner builds so far (part of the graphs' key)

  // restarted GMRES: the Krylov basis [gm_m + 1][gm_nsys][ndof] (allocated by
  // the first solve, grown when a longer cycle or more systems ask for it),
  // the small arrays (Hessenberg matrix, rotations, partial sums), per-system
  // ints (the gate state, then counters), the flags the host polls
  double* gm_V = nullptr;
  int gm_m = 0, gm_nsys = 0;
  double* gm_w = nullptr;
  int* gm_i = nullptr;
  int* gm_flags = nullptr;           // device [2][kMaxSys]
  int* gm_host = nullptr;            // pinned host [2][kMaxSys]
  double* gm_out = nullptr;          // device [4][kMaxSys]
  hipEvent_t gm_ev[2] = {nullptr, nullptr};

  // optional event timing of the block-solve launches inside pcg_solve
  int prof_on = 0;
  int prof_n = 0;                    // launches recorded in the current solve
  std::vector<hipEvent_t> prof_ev;   // [2 * capacity]
  std::vector<int> prof_it;          // PCG iteration of each recorded launch (-1: initial)
  double prof_ms = 0.0, prof_bytes = 0.0;
  int64_t prof_launches = 0;
};

// Partial-sum slots, each [kMaxSys][kMaxParts] doubles.
enum {
  kPartPQ = 0,
  kPartRR0 = 1,     // parity buffers for r.r
  kPartRR1 = 2,
  kPartRZ0 = 3,     // parity buffers for r.z
  kPartRZ1 = 4,
  kPartRZO = 5,     // r_new . z_old (flexible beta)
  kPartFF = 6,      // ||P f||^2
  kPartAux = 7,
  kNumPartSlots = 8
};

// Per-system scalars of the iteration, [kNumScal][kMaxSys] doubles after the
// partial slots and the four summary values per system: beta of the latest
// direction update and r.z of the latest preconditioned residual, each
// reduced once (k_beta) instead of by every workgroup that needs it, and
// ||P f||^2 (stored by the first residual test).
enum { kScBeta = 0, kScRZ = 1, kScFF = 2, kNumScal = 3 };
constexpr size_t kPartsElems = (size_t)kNumPartSlots * kMaxSys * kMaxParts + 4 * kMaxSys +
                               (size_t)kNumScal * kMaxSys;

__host__ __device__ inline double* scal_slot(double* parts, int which) {
  return parts + (size_t)kNumPartSlots * kMaxSys * kMaxParts + 4 * kMaxSys + which * kMaxSys;
}

// Per-system integer state [kNumState][kMaxSys]. kStBreak: 1 breakdown, 2
// invalid densities (the system never starts).
// kStIter: one counter (at istate[kStIter * kMaxSys]) of the iterations
// issued before the current chunk; the poll kernel advances it, and the
// kernels of a replayed chunk add it to their gate's iteration offset.
enum { kStLastIt = 0, kStBreak = 1, kStPoll = 2, kStRun = 3, kStIter = 4, kNumState = 5 };

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the threads of a workgroup (blockDim.x a multiple of 64, at most
// 256); every thread gets the same value. `sh` needs 4 doubles of LDS. Fixed
// reduction tree: deterministic.
// value of v in lane `lane` (uniform index) for every lane
__device__ inline double bcast_lane(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = sh[0];
  if (nw == 4) s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  else
    for (int i = 1; i < nw; ++i) s += sh[i];
  return s;
}

// Sum of n partials in a fixed order (identical in every workgroup of a
// launch).
__device__ inline double sum_parts(const double* __restrict__ p, int n, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += p[i];
  return block_sum(v, sh);
}

// element-local node of the corner at offset (dx, dy, dz) from the element's
// first node: counter-clockwise in the x-y plane, bottom face first
__host__ __device__ inline int corner_of(int dx, int dy, int dz) {
  return (dy ? (dx ? 2 : 3) : (dx ? 1 : 0)) + 4 * dz;
}

__device__ inline double simp_modulus(double rho, double E0, double Emin, double penal) {
  double rp = (penal == 3.0) ? rho * rho * rho : pow(rho, penal);
  return Emin + (E0 - Emin) * rp;
}

// Convergence gate of a batched PCG kernel. A system keeps running while
// its recursive residual r.r (partials in slot rr_slot) exceeds tol2 * ||Pf||^2,
// no breakdown was flagged and the iteration index is below maxit. The
// residual test is taken once per iteration by k_gate (launch_gate), which
// stores it in the kStRun state; the kernels read that flag.
struct Gate {
  const double* parts;
  const int* istate;
  int np;          // partials per system
  int rr_slot;     // kPartRR0 or kPartRR1
  int it;          // iteration index the gated work belongs to
  int maxit;
  double tol2;
  int enabled;     // 0: always run
  int test;        // 1: the restriction takes the residual test itself
  const int* itbase;   // null: `it` is absolute; else it is an offset from *itbase
};

// absolute iteration index of the gated work
__device__ inline int gate_it(const Gate& gt) { return gt.it + (gt.itbase ? *gt.itbase : 0); }

__device__ inline bool gate_running(const Gate& gt, int sys) {
  if (!gt.enabled) return true;
  if (gate_it(gt) >= gt.maxit) return false;
  if (gt.istate[kStBreak * kMaxSys + sys]) return false;
  return gt.istate[kStRun * kMaxSys + sys] != 0;
}

inline int parts_for(int64_t work) {
  int64_t b = (work + kThreads - 1) / kThreads;
  return (int)(b < 1 ? 1 : (b > kMaxParts ? kMaxParts : b));
}

__host__ __device__ inline double* part_slot(double* parts, int slot, int sys) {
  return parts + ((size_t)slot * kMaxSys + sys) * kMaxParts;
}



// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files). All node-parallel kernels use
// parts_for(nnodes) workgroups per system, so their partials line up.
// ---------------------------------------------------------------------------

// matvec.hip: y = P K(rho) P x; optional partials of x.y into slot `dot_slot` (-1: none),
// apply_parts(g) of them per system
int apply_parts(const Geometry& g);
// whether a Q4 element matrix has the eight-value structure of the unit
// square's element, which the Q4 product relies on
// workgroups per subdomain of the coarse restriction
int restrict_splits(const Geometry& g);
bool q4_structured(const double* K0);
// true when K0 (24 x 24, row-major) has the trilinear cube's structure; then
// q holds its twelve class values
bool h8_structured(const double* K0, double* q);
void launch_apply_K(const Handle& h, const double* rho, const double* x, double* y, int nsys,
                    int dot_slot, const Gate& gate, hipStream_t st);
// 2-d only: y = P K P p with the direction update fused, p = z + beta x (beta
// from launch_beta; p = z when first), p written to pnew (pnew != x)
void launch_apply_K_dir(const Handle& h, const double* rho, const double* z, const double* x,
                        double* pnew, double* y, int nsys, int dot_slot, const Gate& gate,
                        int first, hipStream_t st);

// vectors.hip
void launch_residual_init(const Handle& h, const double* f, double* u, const double* q, int nsys,
                          hipStream_t st);
void launch_update_xr(const Handle& h, double* u, const double* p, int nsys, const Gate& gate,
                      hipStream_t st);
// beta and r.z of the preconditioned residual whose r.z partials are in
// rz_slot (first: beta = 0), into the scalar slots; flags a breakdown
void launch_beta(const Handle& h, int nsys, const Gate& gate, int rz_slot, int flexible,
                 int first, hipStream_t st);
// running flags into kStPoll; advances the kStIter counter by `advance`
void launch_poll(const Handle& h, int nsys, const Gate& gate, int advance, hipStream_t st);
// residual test of gate.rr_slot into the kStRun flags
void launch_gate(const Handle& h, int nsys, const Gate& gate, hipStream_t st);
// true residual of P(f - q) (q must hold K u) and out[sys] = {iters, status, relres, true_relres}
void launch_summary(const Handle& h, const double* f, int nsys, const Gate& gate,
                    double* out /*dev [nsys][4]*/, hipStream_t st);
void launch_copy(double* dst, const double* src, int64_t n, hipStream_t st);

// tune.hip: the autotuner's hooks around a PCG solve, and its choice of the
// GMRES dot-product grouping (a short measurement on the handle's stream)
void tune_before_solve(Handle& h);
void tune_after_solve(Handle& h, double ms, int iters);
void tune_gmres(Handle& h, int nsys, int m);
// gmres.hip: ms per launch of the dot-product kernel with `chunk` vectors
// per workgroup on nv basis vectors (for the autotuner)
double gmres_time_dots(Handle& h, int nsys, int nv, int chunk);
// gmres.hip: restarted GMRES (cycle length m) with the MsFEM cycle or the
// additive Schwarz preconditioner; hout [4][nsys]: iterations, status,
// preconditioned relative residual estimate, true relative residual
size_t gmres_small_elems();
int gmres_solve(Handle& h, const double* rho, const double* f, double* u, int nsys, double rtol,
                int maxit, int m, int precond, double* hout);
// gmres.hip: xout = B rin with the MsFEM cycle (h.q and h.z are work vectors)
void launch_msfem_cycle(Handle& h, const double* rho, const double* rin, double* xout, int nsys,
                        const Gate& gate, hipStream_t st);
// precond.hip: x_c = K_c^-1 Phi^T r into h.xc for every running system (the
// coarse branch alone, on stream st)
void launch_coarse_only(Handle& h, const double* r, int nsys, const Gate& gate, hipStream_t st);
// precond.hip: z = M^-1 r, gated; partials of r.z into rz_slot (and r.z_old into kPartRZO)
// prof_it >= -1 records events around the block-solve launch when profiling is on
void launch_precond(Handle& h, const double* r, double* z, int nsys, const Gate& gate,
                    int rz_slot, int prof_it, int flexible, hipStream_t st);

// local.hip: zloc = A_j^-1 R_j r for every running (system, subdomain)
void launch_local_solves(Handle& h, const double* r, int nsys, const Gate& gate, hipStream_t st);

// setup.hip
// with_basis = 0: keep the spectral basis, rebuild the local and coarse factors
int build_preconditioner(Handle& h, const double* rho, int nsys, int rep, int with_basis);
// work arrays (doubles) the preconditioner build keeps in the handle
size_t build_ws_elems(const tpcg_problem& pr, const Geometry& g, int big, int msub);

// density.hip
void launch_filter_project(const Handle& h, const double* rho, double rmin, double beta,
                           const double* eta, int nsys, double* rho_tilde, double* rho_phys,
                           hipStream_t st);
void launch_filter_project_adjoint(const Handle& h, const double* rho_tilde, double rmin,
                                   double beta, const double* eta, int nsys, const double* g,
                                   double* out, hipStream_t st);
void launch_compliance_sens(const Handle& h, const double* rho, const double* u, const double* f,
                            int nsys, double* c, double* dc, hipStream_t st);
// robust objective {E + kappa std, E, std} of c [nsys] (weights w, host) and,
// if dc, its gradient df [n_el] from dc [nsys][n_el]
void launch_robust(const Handle& h, const double* c, const double* dc, int nsys, double kappa,
                   const double* w, double* out, double* df, hipStream_t st);
// out[0] = sum_e 4 rho_e (1 - rho_e) / n_el (one density field)
void launch_nondiscreteness(const Handle& h, const double* rho, double* out, hipStream_t st);
// gcell [nsys][cx cy cz] = sums of gin [nsys][n_el] over the copies of a unit cell
void launch_periodic_sum(const Handle& h, const double* gin, int nsys, int cx, int cy, int cz,
                         double* gcell, hipStream_t st);
// the same without a handle: supports, element matrix and partials
// (part[sys * kMaxParts + i], i < parts_for(nnodes)) given as device pointers
void launch_compliance_sens_raw(const Geometry& g, const uint8_t* fixed, const double* K0,
                                double E0, double Emin, double penal, double* part,
                                const double* rho, const double* u, const double* f, int nsys,
                                double* c, double* dc, hipStream_t st);

// element.cpp
void element_stiffness(int dim, double nu, double* K0 /* [ndpe*ndpe] */);

// capi.hip: device allocation through the library's fault-injection counter
// (tpcg_test_fail_alloc); false when the allocation failed
bool device_alloc(void** p, size_t bytes);

// vectors.hip: densities outside [0, 1] or NaN. Per system s of [nsys][n]
// with a bad entry: flag[s * stride] = value.
void launch_check_rho(const double* rho, int64_t n, int nsys, int* flag, int stride, int value,
                      hipStream_t st);

}  // namespace tpcg

// Host side of the C ABI declared in include/lb_chiral.h.
//
// A context owns the device state of one periodic box (ping-pong population,
// Q and phi buffers, scratch fields, reduction partials) and enqueues every
// kernel on the stream it was given.  The arithmetic type and the storage
// types are template parameters of the backend: float64 throughout, float32
// throughout, or float16 population storage with float32 arithmetic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lb_chiral.h"
#include "kernels_adjoint.hpp"
#include "kernels_fused.hpp"
#include "kernels_pc.hpp"
#include "kernels_pc_adjoint.hpp"
#include "kernels_reduce.hpp"
#include "kernels_step.hpp"

namespace {

thread_local std::string g_last_error;

struct LbError {
  lb_status st;
  std::string msg;
};

[[noreturn]] void fail(lb_status st, const std::string& msg) { throw LbError{st, msg}; }

#define HIPCHECK(expr)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) fail(LB_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int TPB = 256;

template <class T>
T* dalloc(size_t n) {
  void* p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(LB_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  return static_cast<T*>(p);
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// sums[k] = sum over nblocks block partials (nv values each) in a fixed
// order: one workgroup for few blocks, else kSumChunks chunk sums (into mids)
// first.  mids holds kSumChunks * nv doubles, sums nv.
constexpr int kSumChunks = 64;
void final_sum_into(hipStream_t stream, const double* part, int nblocks, int nv, double* mids, double* sums) {
  if (nblocks <= 4096) {
    lbc::k_final_sum<<<1, TPB, 0, stream>>>(part, nblocks, nv, sums);
    return;
  }
  const int chunk = (nblocks + kSumChunks - 1) / kSumChunks;
  lbc::k_final_sum<<<kSumChunks, TPB, 0, stream>>>(part, nblocks, nv, mids, chunk);
  lbc::k_final_sum<<<1, TPB, 0, stream>>>(mids, kSumChunks, nv, sums);
}

// x-y tiles of the fused kernels.  The stress kernel computes the stress on
// the (TX+2) x (TY+2) frame of a TX x TY tile; LDS per workgroup is about
// 20 (TX+4)(TY+4) + 10 (TX+2)(TY+2) values.  The variant is chosen at context
// creation (lb_tuning selects another one; in double, the 32 x 16 stress
// tile is replaced by 16 x 16 and the 64 x 16 order tile by 64 x 8).
struct TileCfg {
  int tx, ty;
};
constexpr TileCfg kLbTiles[] = {{32, 8}, {32, 16}, {64, 4}, {16, 16}, {16, 8}};
constexpr TileCfg kOrTiles[] = {{32, 8}, {64, 4}, {32, 16}, {64, 8}, {64, 16}};
// tiles of the z-marching predictor-corrector stage and mu kernels
constexpr TileCfg kPcTiles[] = {{32, 8}, {32, 16}, {16, 16}, {64, 8}};

// Deepest z-slab of at most tz_max planes (halved down to tz_min) that still
// gives per_cu workgroups per CU for a grid of ntx x nty tiles.  Small boxes
// get shallow slabs: a deep slab on few tiles leaves most CUs idle while a
// handful of workgroups march through the planes one after another.
int cu_count() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
    ncu = 256;
  return ncu;
}
int auto_slab(int ntx, int nty, int nz, int tz_max, int tz_min, int per_cu) {
  const int ncu = cu_count();
  int tz = tz_max;
  while (tz > tz_min && size_t(ntx) * nty * ((nz + tz - 1) / tz) < size_t(per_cu) * ncu) tz /= 2;
  return tz;
}

// Default tiles and slab depths per storage (measured on the 128^3 and
// 256^3 droplets): stress kernel float 32 x 8 with slabs of up to 16 planes,
// half populations 32 x 8 with up to 11, double 16 x 8 with up to 16 (its
// register and LDS footprint leaves one or two small workgroups per CU); the
// slab is the deepest that still gives a workgroup per CU.  Order kernel
// 64 x 8 with the deepest slab of at most 16 planes that gives two
// workgroups per CU.  lb_tuning can fix each depth instead.
template <class R, class GS>
struct DefaultTile {
  static constexpr int lb = 0, order = 3, tz_lb_max = 16;
};
template <>
struct DefaultTile<float, __half> {
  static constexpr int lb = 0, order = 3, tz_lb_max = 11;
};
template <>
struct DefaultTile<double, double> {
  static constexpr int lb = 4, order = 3, tz_lb_max = 16;
};

bool finite_params(const lb_params& p) {
  const double v[] = {p.tau, p.rho0, p.a, p.phi0, p.phi_cr, p.k_phi, p.M, p.A0, p.chi0, p.chi_s, p.K,
                      p.q0, p.W, p.Gamma, p.xi, p.zeta, p.body_force[0], p.body_force[1], p.body_force[2]};
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

void validate(const lb_params& p) {
  if (p.nx < 3 || p.ny < 3 || p.nz < 3) fail(LB_EINVAL, "box sides must be >= 3");
  if (p.prec < LB_FP64 || p.prec > LB_FP16S) fail(LB_EINVAL, "unknown precision");
  if (p.lattice != LB_D3Q19 && p.lattice != LB_D3Q15) fail(LB_EINVAL, "unknown lattice");
  if (p.fd_scheme != LB_FD_EULER2 && p.fd_scheme != LB_FD_PC4) fail(LB_EINVAL, "unknown fd_scheme");
  if (!finite_params(p)) fail(LB_EINVAL, "non-finite parameter");
  if (!(p.tau > 0.5)) fail(LB_EINVAL, "tau must be > 0.5");
  if (!(p.rho0 > 0.0)) fail(LB_EINVAL, "rho0 must be > 0");
  if (!(p.phi_cr != 0.0)) fail(LB_EINVAL, "phi_cr must be nonzero");
  const double n = double(p.nx) * double(p.ny) * double(p.nz);
  if (n > double(1 << 29)) fail(LB_ENOMEM, "box exceeds 2^29 sites");
}

// tiles of the one-launch step kernel (each keeps one halo stress slot or
// edge job per thread and plane)
constexpr TileCfg kStTiles[] = {{32, 8}, {32, 16}, {64, 8}};
constexpr int kNStTiles = int(sizeof(kStTiles) / sizeof(kStTiles[0]));
constexpr int kNLbTiles = int(sizeof(kLbTiles) / sizeof(kLbTiles[0]));
constexpr int kNOrTiles = int(sizeof(kOrTiles) / sizeof(kOrTiles[0]));
constexpr int kNPcTiles = int(sizeof(kPcTiles) / sizeof(kPcTiles[0]));

// The one-launch step applies to the explicit Euler integrator.  It is never
// the default: its halo recompute (the stress on a frame two sites wide, the
// moments of the tile's edge sites) costs more than the u, mu round trip and
// the second read of Q, phi that it saves (measured at 128^3 and 256^3).
bool one_launch_applies(const lb_params& p) { return p.fd_scheme == LB_FD_EULER2; }

void validate_tuning(const lb_params& p, const lb_tuning& t) {
  if (t.path < LB_PATH_DEFAULT || t.path > LB_PATH_SITE) fail(LB_EINVAL, "unknown lb_path");
  if (t.path == LB_PATH_ONE_LAUNCH && !one_launch_applies(p))
    fail(LB_EINVAL, "LB_PATH_ONE_LAUNCH needs LB_FD_EULER2");
  if (t.lb_tile < 0 || t.lb_tile > kNLbTiles) fail(LB_EINVAL, "lb_tile out of range");
  if (t.order_tile < 0 || t.order_tile > kNOrTiles) fail(LB_EINVAL, "order_tile out of range");
  if (t.pc_tile < 0 || t.pc_tile > kNPcTiles) fail(LB_EINVAL, "pc_tile out of range");
  if (t.pcmu_tile < 0 || t.pcmu_tile > kNPcTiles) fail(LB_EINVAL, "pcmu_tile out of range");
  if (t.step_tile < 0 || t.step_tile > kNStTiles) fail(LB_EINVAL, "step_tile out of range");
  if (t.adj_tile < 0 || t.adj_tile > 2) fail(LB_EINVAL, "adj_tile out of range");
  if (t.adj_order_tile < 0 || t.adj_order_tile > 2) fail(LB_EINVAL, "adj_order_tile out of range");
  if (t.pc_adj < 0 || t.pc_adj > 1) fail(LB_EINVAL, "pc_adj out of range");
  const int32_t tz[] = {t.tz_step, t.tz_lb, t.tz_order, t.tz_pc, t.tz_pcmu, t.tz_adj, t.tz_adj_order, t.tz_pc_adj};
  for (int32_t v : tz)
    if (v < 0) fail(LB_EINVAL, "negative slab depth");
}

template <class R>
lbc::Params<R> make_params(const lb_params& p) {
  lbc::Params<R> P;
  P.omega = R(1.0 / p.tau);
  P.guo = R(1.0 - 0.5 / p.tau);
  P.rho0 = R(p.rho0);
  P.a = R(p.a);
  P.phi0 = R(p.phi0);
  P.inv_phicr2 = R(1.0 / (p.phi_cr * p.phi_cr));
  P.k_phi = R(p.k_phi);
  P.M = R(p.M);
  P.A0 = R(p.A0);
  P.chi0 = R(p.chi0);
  P.chi_s = R(p.chi_s);
  P.K = R(p.K);
  P.q0 = R(p.q0);
  P.W = R(p.W);
  P.Gamma = R(p.Gamma);
  P.xi = R(p.xi);
  P.zeta = R(p.zeta);
  for (int a = 0; a < 3; ++a) P.bf[a] = R(p.body_force[a]);
  return P;
}

struct Backend {
  virtual ~Backend() = default;
  virtual void set_params(const lb_params& p) = 0;
  virtual void upload(const double* phi, const double* q5, const double* u0) = 0;
  virtual void set_fields(const double* g19, const double* phi, const double* q5) = 0;
  virtual void step(int n) = 0;
  virtual void profile(int n, double* ms, int* count) = 0;
  virtual const char* kernel_name(int i) const = 0;
  virtual void moments(double* rho, double* u3, double* phi, double* q5) = 0;
  virtual void populations(double* g19) = 0;
  virtual void totals(double out[lbc::NTOT]) = 0;
  virtual void centre(double out[lbc::NCEN]) = 0;
  virtual size_t state_bytes() const = 0;
  virtual void get_state(void* dst, int64_t step) = 0;
  virtual int64_t set_state(const void* src) = 0;
  virtual size_t adjoint_bytes() const = 0;
  virtual size_t record_bytes() const = 0;
  virtual void step_record(const void* state_in, void* state_out, void* rec_out) = 0;
  virtual void adjoint_step(const void* state, const void* rec, const void* adj_in, void* adj_out,
                            double* zeta_bar, double* q0_bar) = 0;
  virtual size_t lean_record_bytes() const = 0;
  virtual void step_record_lean(void* rec_out) = 0;
  virtual void adjoint_step_lean(const void* rec, const void* adj_in, void* adj_out, double* zeta_bar,
                                 double* q0_bar) = 0;
  virtual double seed_centre(double z_ref, void* adj) = 0;
};

template <class R, class GS, class FS, class L>
struct BackendT final : Backend {
  static constexpr int NQ = L::Q;  // populations per site
  lbc::Box box;
  hipStream_t stream;
  lbc::Params<R> P;
  lbc::Params<double> Pd;
  size_t N;
  unsigned nblk;
  GS* B[2] = {nullptr, nullptr};
  FS* Q[2] = {nullptr, nullptr};
  FS* Ph[2] = {nullptr, nullptr};
  int cur = 0;
  R* mu = nullptr;
  R* H = nullptr;
  R* sig = nullptr;
  R* u = nullptr;
  double* partial = nullptr;
  double* sums = nullptr;
  double* mids = nullptr;  // chunk sums of the two-stage total over many blocks
  // adjoint scratch (allocated on first use)
  R* aF = nullptr;
  R* amub = nullptr;
  R* aWb = nullptr;
  R* aubp = nullptr;
  R* aqbp = nullptr;
  R* aphibp = nullptr;
  R* aFb = nullptr;
  R* agbar = nullptr;
  R* ahx = nullptr;  // face terms and edge-column adjoints of the fused stress + gather adjoint (x tiles > 1)
  R* ahy = nullptr;  // the same along y
  R* aSb = nullptr;  // D3Q15: adjoint of the symmetric stress S_ab in the collision, [6][N]
  R* apb = nullptr;    // pc4 reverse: per-site adjoints of one product's stencil data [NPB][N]
  R* axs = nullptr;    // pc4 reverse: X*_bar [6][N]
  R* aupc = nullptr;   // pc4 reverse: u_bar [3][N]
  int gz_tz = 0, gz_blocks = 0;  // pc4 reverse: slab depth and grid of k_pcb_gather_z
  // pc4 reverse product in one z-march (k_pcb_fused) on kPfTX x 16 tiles, where
  // every tile along a split axis is at least two sites wide; else the
  // site-parallel k_pcb_local / k_pcb_v / k_pcb_gather
  static constexpr int kPfTX = sizeof(R) == 4 ? 32 : 16, kPfTY = 16;
  bool pf_fused = false;
  int pf_ntx = 1, pf_nty = 1, pf_tz = 1, pf_blocks = 1;
  int mb_ntx = 1, mb_nty = 1, mb_blocks = 1;  // its mu_bar kernel (k_pcb_mub: 32 x 8 tiles of eight planes)
  R* apfx = nullptr;  // its face terms along x ([2][2][pf_ntx][nz][ny][kRec])
  R* apfy = nullptr;  // along y ([9][2][2][pf_nty][nz][nx])
  double* apart = nullptr;   // per-block (zeta, q0) adjoint partials, kept across reverse steps
  size_t apart_n = 0;        // doubles in apart
  bool apart_live = false;   // apart holds sums not yet fetched by the caller
  bool site_path = false;  // three site-parallel kernels instead of the fused pair
  bool one_launch = false;  // the whole step in k_step_fused
  int st_tile = 0, st_ntx = 1, st_nty = 1, st_tz = 1, st_blocks = 1;  // k_step_fused
  // predictor-corrector integrator of the order parameters: X* (Q then phi, in
  // FS) and the anchoring vector v [3][N]
  bool pc4 = false;
  FS* pcs = nullptr;
  R* pcv = nullptr;
  int pc_tile = 0, tz_pc = 0, pc_ntx = 1, pc_nty = 1, pc_blocks = 1;          // stage kernel
  int pm_tile = 0, tz_pm = 0, pm_ntx = 1, pm_nty = 1, pm_blocks = 1;          // mu kernel
  int tz_lb = 8, tz_or = 8;
  int lb_tile = 0, or_tile = 0;
  int lb_ntx, lb_nty, lb_blocks, or_ntx, or_nty, or_blocks;
  static constexpr int kAoTX = 32;  // tile of the z-marching adjoint order kernel: 32 x ao_ty
  int ao_ty = 8, ao_ntx, ao_nty, ao_tz, ao_blocks;
  // tile of the fused stress + gather adjoint (double: 16 x 8, whose LDS frame is half as large)
  static constexpr int kAsTX = sizeof(R) == 4 ? 32 : 16;
  // rows of the stress + gather adjoint's tile: 16 in float (half the y tile faces
  // of 8 rows, whose terms k_adj_faces adds: checkpointed adjoint/forward 3.21 ->
  // 3.13 at 256^3, 3.00 -> 2.91 at 128^3), 8 in double
  int as_ty = 8;
  int as_ntx, as_nty, as_tz, as_blocks;

  BackendT(const lb_params& p, const lb_tuning& t, hipStream_t s) : stream(s) {
    box.nx = p.nx;
    box.ny = p.ny;
    box.nz = p.nz;
    N = size_t(p.nx) * p.ny * p.nz;
    box.N = int(N);
    nblk = unsigned((N + TPB - 1) / TPB);
    set_params(p);
    site_path = t.path == LB_PATH_SITE;
    pc4 = p.fd_scheme == LB_FD_PC4;
    one_launch = !pc4 && t.path == LB_PATH_ONE_LAUNCH;
    pc_tile = t.pc_tile > 0 ? t.pc_tile - 1 : 0;
    tz_pc = t.tz_pc;
    // mu kernel: 64 x 8 in float; in double that frame needs 150 KB of LDS, so 32 x 8
    const int pm_default = sizeof(R) == 4 ? 3 : 0;
    pm_tile = t.pcmu_tile > 0 ? t.pcmu_tile - 1 : pm_default;
    tz_pm = t.tz_pcmu;
    using D = DefaultTile<R, GS>;
    tz_lb = t.tz_lb;
    tz_or = t.tz_order;
    lb_tile = t.lb_tile > 0 ? t.lb_tile - 1 : D::lb;
    or_tile = t.order_tile > 0 ? t.order_tile - 1 : D::order;
    if (sizeof(R) == 8 && lb_tile == 1) lb_tile = 3;  // 32 x 16 needs more than 160 KB of LDS in double
    if (sizeof(R) == 8 && or_tile == 4) or_tile = 3;  // 64 x 16 would spill in double
    st_tile = (t.step_tile > 0 && sizeof(R) == 4) ? t.step_tile - 1 : 0;  // float64: 32 x 8 only
    const TileCfg stt = kStTiles[st_tile];
    st_ntx = (p.nx + stt.tx - 1) / stt.tx;
    st_nty = (p.ny + stt.ty - 1) / stt.ty;
    // workgroups per CU the LDS frame allows: two for the 32 x 8 tile in float, else one
    const int st_per_cu = (sizeof(R) == 4 && st_tile == 0) ? 2 : 1;
    st_tz = t.tz_step > 0 ? t.tz_step : auto_slab(st_ntx, st_nty, p.nz, 32, 1, st_per_cu);
    st_blocks = st_ntx * st_nty * ((p.nz + st_tz - 1) / st_tz);
    const TileCfg lt = kLbTiles[lb_tile], ot = kOrTiles[or_tile];
    lb_ntx = (p.nx + lt.tx - 1) / lt.tx;
    lb_nty = (p.ny + lt.ty - 1) / lt.ty;
    if (tz_lb == 0) tz_lb = auto_slab(lb_ntx, lb_nty, p.nz, D::tz_lb_max, 1, 1);
    lb_blocks = lb_ntx * lb_nty * ((p.nz + tz_lb - 1) / tz_lb);
    or_ntx = (p.nx + ot.tx - 1) / ot.tx;
    or_nty = (p.ny + ot.ty - 1) / ot.ty;
    if (tz_or == 0) tz_or = auto_slab(or_ntx, or_nty, p.nz, 16, 1, 2);
    or_blocks = or_ntx * or_nty * ((p.nz + tz_or - 1) / tz_or);
    pc_ntx = (p.nx + kPcTiles[pc_tile].tx - 1) / kPcTiles[pc_tile].tx;
    pc_nty = (p.ny + kPcTiles[pc_tile].ty - 1) / kPcTiles[pc_tile].ty;
    if (tz_pc == 0) tz_pc = auto_slab(pc_ntx, pc_nty, p.nz, 16, 1, 2);
    pc_blocks = pc_ntx * pc_nty * ((p.nz + tz_pc - 1) / tz_pc);
    pm_ntx = (p.nx + kPcTiles[pm_tile].tx - 1) / kPcTiles[pm_tile].tx;
    pm_nty = (p.ny + kPcTiles[pm_tile].ty - 1) / kPcTiles[pm_tile].ty;
    if (tz_pm == 0) tz_pm = auto_slab(pm_ntx, pm_nty, p.nz, 16, 1, 2);
    pm_blocks = pm_ntx * pm_nty * ((p.nz + tz_pm - 1) / tz_pm);
    // order adjoint tile: float 32 x 16 (two workgroups of 512 threads per
    // CU at 124 registers), double 32 x 8 (32 x 16 spills there)
    ao_ty = t.adj_order_tile == 2 || (t.adj_order_tile == 0 && sizeof(R) == 4) ? 16 : 8;
    ao_ntx = (p.nx + kAoTX - 1) / kAoTX;
    ao_nty = (p.ny + ao_ty - 1) / ao_ty;
    ao_tz = t.tz_adj_order;
    // float holds four waves per SIMD (124 registers: four workgroups of a
    // 32 x 8 tile per CU, or two of 32 x 16): slabs of up to 16 planes, deep
    // enough to fill them (8 planes at 128^3, 16 at 256^3)
    if (ao_tz == 0)
      ao_tz = sizeof(R) == 4 ? auto_slab(ao_ntx, ao_nty, p.nz, 16, 1, ao_ty == 16 ? 2 : 4)
                             : auto_slab(ao_ntx, ao_nty, p.nz, 32, 1, ao_ty == 16 ? 1 : 2);
    ao_blocks = ao_ntx * ao_nty * ((p.nz + ao_tz - 1) / ao_tz);
    as_ty = t.adj_tile == 2 || (t.adj_tile == 0 && sizeof(R) == 4) ? 16 : 8;
    as_ntx = (p.nx + kAsTX - 1) / kAsTX;
    as_nty = (p.ny + as_ty - 1) / as_ty;
    as_tz = t.tz_adj;
    // the deepest slab of up to 128 planes that still gives every CU a
    // workgroup (8 waves): each slab marches two planes more than it owns, and
    // its LDS footprint allows one such workgroup per CU at a time
    if (as_tz == 0) as_tz = auto_slab(as_ntx, as_nty, p.nz, 128, 1, as_ty == 16 ? 1 : 2);
    as_blocks = as_ntx * as_nty * ((p.nz + as_tz - 1) / as_tz);
    pf_ntx = (p.nx + kPfTX - 1) / kPfTX;
    pf_nty = (p.ny + kPfTY - 1) / kPfTY;
    pf_fused = pc4 && t.pc_adj == 0 && (pf_ntx == 1 || p.nx % kPfTX != 1) && (pf_nty == 1 || p.ny % kPfTY != 1);
    pf_tz = t.tz_pc_adj;
    if (pf_tz == 0) pf_tz = auto_slab(pf_ntx, pf_nty, p.nz, 16, 1, 1);  // one workgroup per CU fits its LDS
    pf_blocks = pf_ntx * pf_nty * ((p.nz + pf_tz - 1) / pf_tz);
    mb_ntx = (p.nx + 31) / 32;
    mb_nty = (p.ny + 7) / 8;
    mb_blocks = mb_ntx * mb_nty * ((p.nz + 7) / 8);
    size_t need = 2 * (NQ * N * sizeof(GS) + 6 * N * sizeof(FS)) + 4 * N * sizeof(R);
    if (pc4) need += 6 * N * sizeof(FS) + (site_path ? 3 * N * sizeof(R) : 0);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && need > free_b)
      fail(LB_ENOMEM, "state needs " + std::to_string(need) + " bytes, " + std::to_string(free_b) + " free");
    try {
      for (int k = 0; k < 2; ++k) {
        B[k] = dalloc<GS>(NQ * N);
        Q[k] = dalloc<FS>(5 * N);
        Ph[k] = dalloc<FS>(N);
      }
      mu = dalloc<R>(N);
      u = dalloc<R>(3 * N);
      partial = dalloc<double>(size_t(nblk) * 16);
      sums = dalloc<double>(16);
      mids = dalloc<double>(size_t(kSumChunks) * 16);
      if (site_path) ensure_thermo();
      if (pc4) {
        pcs = dalloc<FS>(6 * N);
        if (site_path) pcv = dalloc<R>(3 * N);
      }
    } catch (...) {
      release();
      throw;
    }
  }
  // H [5][N] and sigma [9][N]: used by the site-parallel step, by observation
  // (u and rho need the force) and by the adjoint's recomputation of u and F,
  // never by the fused step; allocated on first use.
  void ensure_thermo() {
    if (H) return;
    R* h = dalloc<R>(5 * N);
    try {
      sig = dalloc<R>(9 * N);
    } catch (...) {
      dfree(h);
      throw;
    }
    H = h;
  }
  ~BackendT() override { release(); }
  void release() {
    for (int k = 0; k < 2; ++k) {
      dfree(B[k]);
      dfree(Q[k]);
      dfree(Ph[k]);
      B[k] = nullptr;
      Q[k] = nullptr;
      Ph[k] = nullptr;
    }
    dfree(mu);
    dfree(H);
    dfree(sig);
    dfree(u);
    dfree(partial);
    dfree(sums);
    dfree(mids);
    dfree(pcs);
    dfree(pcv);
    pcs = nullptr;
    pcv = nullptr;
    mu = H = sig = u = nullptr;
    partial = sums = mids = nullptr;
    R** adj[] = {&aF, &amub, &aWb, &aubp, &aqbp, &aphibp, &aFb, &agbar, &ahx, &ahy, &aSb, &apb, &axs, &aupc, &apfx, &apfy};
    for (R** a : adj) {
      dfree(*a);
      *a = nullptr;
    }
    dfree(apart);
    apart = nullptr;
  }

  void set_params(const lb_params& p) override {
    P = make_params<R>(p);
    Pd = make_params<double>(p);
  }

  void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(LB_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  }

  // host float64 -> device FS (via a float64 staging buffer)
  template <class T>
  void h2d_convert(const double* host, T* dev, size_t n) {
    double* tmp = dalloc<double>(n);
    try {
      HIPCHECK(hipMemcpyAsync(tmp, host, n * sizeof(double), hipMemcpyHostToDevice, stream));
      lbc::k_convert<T, double><<<unsigned((n + TPB - 1) / TPB), TPB, 0, stream>>>(n, tmp, dev);
      check_launch();
      HIPCHECK(hipStreamSynchronize(stream));
    } catch (...) {
      dfree(tmp);
      throw;
    }
    dfree(tmp);
  }
  template <class T>
  void d2h_convert(const T* dev, double* host, size_t n) {
    double* tmp = dalloc<double>(n);
    try {
      lbc::k_convert<double, T><<<unsigned((n + TPB - 1) / TPB), TPB, 0, stream>>>(n, dev, tmp);
      check_launch();
      HIPCHECK(hipMemcpyAsync(host, tmp, n * sizeof(double), hipMemcpyDeviceToHost, stream));
      HIPCHECK(hipStreamSynchronize(stream));
    } catch (...) {
      dfree(tmp);
      throw;
    }
    dfree(tmp);
  }

  void upload(const double* phi, const double* q5, const double* u0) override {
    h2d_convert(phi, Ph[cur], N);
    h2d_convert(q5, Q[cur], 5 * N);
    double* du0 = nullptr;
    double* g = dalloc<double>(NQ * N);
    try {
      if (u0) {
        du0 = dalloc<double>(3 * N);
        HIPCHECK(hipMemcpyAsync(du0, u0, 3 * N * sizeof(double), hipMemcpyHostToDevice, stream));
      }
      lbc::k_equilibrium<L><<<nblk, TPB, 0, stream>>>(box, double(Pd.rho0), du0, g);
      lbc::k_push<GS, L><<<nblk, TPB, 0, stream>>>(box, g, B[cur]);
      check_launch();
      HIPCHECK(hipStreamSynchronize(stream));
    } catch (...) {
      dfree(du0);
      dfree(g);
      throw;
    }
    dfree(du0);
    dfree(g);
  }

  void set_fields(const double* g19, const double* phi, const double* q5) override {
    if (phi) h2d_convert(phi, Ph[cur], N);
    if (q5) h2d_convert(q5, Q[cur], 5 * N);
    if (g19) {
      double* g = dalloc<double>(NQ * N);
      try {
        HIPCHECK(hipMemcpyAsync(g, g19, NQ * N * sizeof(double), hipMemcpyHostToDevice, stream));
        lbc::k_push<GS, L><<<nblk, TPB, 0, stream>>>(box, g, B[cur]);
        check_launch();
        HIPCHECK(hipStreamSynchronize(stream));
      } catch (...) {
        dfree(g);
        throw;
      }
      dfree(g);
    }
  }

  // --- the step -----------------------------------------------------------
  // launches of one step: the LB part (two site kernels or the fused stress /
  // collide kernel), then the order-parameter update (one kernel, or the six
  // launches of the predictor-corrector)
  int n_lb() const { return site_path ? 2 : 1; }
  int n_pc() const { return site_path ? 6 : 4; }
  int nkernels() const { return one_launch ? 1 : n_lb() + (pc4 ? n_pc() : 1); }
  const char* kernel_name(int i) const override {
    if (one_launch) return i == 0 ? "k_step_fused" : nullptr;
    static const char* site_names[3] = {"k_thermo", "k_collide", "k_order"};
    static const char* fused_names[2] = {"k_lb_fused", "k_order_fused"};
    static const char* pc_names[6] = {"k_pc_v", "k_pc_mu", "k_pc_predict", "k_pc_v (X*)", "k_pc_mu (X*)",
                                      "k_pc_correct"};
    static const char* pcz_names[4] = {"k_pc_mu_z", "k_pc_stage_z (predict)", "k_pc_mu_z (X*)",
                                       "k_pc_stage_z (correct)"};
    if (i < 0 || i >= nkernels()) return nullptr;
    if (i >= n_lb() && pc4) return (site_path ? pc_names : pcz_names)[i - n_lb()];
    return site_path ? site_names[i] : fused_names[i];
  }
  void launch_pc(int k) {
    const int nx = cur ^ 1;
    FS* qs = pcs;
    FS* phs = pcs + 5 * N;
    if (!site_path) {
      switch (k) {
        case 0: launch_pc_mu(Ph[cur], Q[cur]); break;
        case 1: launch_pc_stage<true>(Ph[cur], Q[cur], nullptr, nullptr, phs, qs); break;
        case 2: launch_pc_mu(phs, qs); break;
        default:
          launch_pc_stage<false>(phs, qs, Ph[cur], Q[cur], Ph[nx], Q[nx]);
          cur = nx;
          break;
      }
      return;
    }
    switch (k) {
      case 0: lbc::k_pc_v<R, FS><<<nblk, TPB, 0, stream>>>(box, Ph[cur], Q[cur], pcv); break;
      case 1: lbc::k_pc_mu<R, FS><<<nblk, TPB, 0, stream>>>(box, P, Ph[cur], Q[cur], pcv, mu); break;
      case 2: lbc::k_pc_predict<R, FS><<<nblk, TPB, 0, stream>>>(box, P, Ph[cur], Q[cur], u, mu, phs, qs); break;
      case 3: lbc::k_pc_v<R, FS><<<nblk, TPB, 0, stream>>>(box, phs, qs, pcv); break;
      case 4: lbc::k_pc_mu<R, FS><<<nblk, TPB, 0, stream>>>(box, P, phs, qs, pcv, mu); break;
      default:
        lbc::k_pc_correct<R, FS><<<nblk, TPB, 0, stream>>>(box, P, phs, qs, u, mu, Ph[cur], Q[cur], Ph[nx], Q[nx]);
        cur = nx;
        break;
    }
  }
  void launch_pc_mu(const FS* phi_i, const FS* q_i) {
    switch (pm_tile) {
      case 0: launch_pc_mu_tile<32, 8, 2>(phi_i, q_i); break;
      case 1: launch_pc_mu_tile<32, 16, 2>(phi_i, q_i); break;
      case 2: launch_pc_mu_tile<16, 16, 2>(phi_i, q_i); break;
      default: launch_pc_mu_tile<64, 8, 2>(phi_i, q_i); break;
    }
  }
  template <int TX, int TY, int MINW>
  void launch_pc_mu_tile(const FS* phi_i, const FS* q_i) {
    lbc::k_pc_mu_z<R, FS, TX, TY, MINW><<<pm_blocks, TX * TY, 0, stream>>>(box, P, tz_pm, pm_ntx, pm_nty, phi_i,
                                                                           q_i, mu);
  }
  // one Heun stage on explicit buffers with the velocity uu (the context's u by default)
  template <bool PRED>
  void launch_pc_stage(const FS* phi_i, const FS* q_i, const FS* phi_x, const FS* q_x, FS* phi_o, FS* q_o,
                       const R* uu = nullptr) {
    if (!uu) uu = u;
    switch (pc_tile) {
      case 0: launch_pc_tile<32, 8, 2, PRED>(phi_i, q_i, phi_x, q_x, phi_o, q_o, uu); break;
      case 1: launch_pc_tile<32, 16, 2, PRED>(phi_i, q_i, phi_x, q_x, phi_o, q_o, uu); break;
      case 2: launch_pc_tile<16, 16, 2, PRED>(phi_i, q_i, phi_x, q_x, phi_o, q_o, uu); break;
      default: launch_pc_tile<64, 8, 2, PRED>(phi_i, q_i, phi_x, q_x, phi_o, q_o, uu); break;
    }
  }
  template <int TX, int TY, int MINW, bool PRED>
  void launch_pc_tile(const FS* phi_i, const FS* q_i, const FS* phi_x, const FS* q_x, FS* phi_o, FS* q_o,
                      const R* uu) {
    lbc::k_pc_stage_z<R, FS, TX, TY, MINW, PRED><<<pc_blocks, TX * TY, 0, stream>>>(
        box, P, tz_pc, pc_ntx, pc_nty, phi_i, q_i, uu, mu, phi_x, q_x, phi_o, q_o);
  }
  void launch(int k) {
    const int nx = cur ^ 1;
    if (pc4 && k >= n_lb()) {
      launch_pc(k - n_lb());
      return;
    }
    if (site_path) {
      switch (k) {
        case 0:
          lbc::k_thermo<R, FS><<<nblk, TPB, 0, stream>>>(box, P, Ph[cur], Q[cur], mu, H, sig);
          break;
        case 1:
          lbc::k_collide<R, GS, L><<<nblk, TPB, 0, stream>>>(box, P, B[cur], B[nx], sig, u);
          break;
        case 2:
          lbc::k_order<R, FS><<<nblk, TPB, 0, stream>>>(box, P, Ph[cur], Q[cur], u, H, mu, Ph[nx], Q[nx]);
          cur = nx;
          break;
      }
      return;
    }
    if (one_launch) {
      launch_step1(Io{B[cur], B[nx], Ph[cur], Q[cur], Ph[nx], Q[nx], nullptr, nullptr, nullptr});
      cur = nx;
      return;
    }
    const Io io = cur_io();
    if (k == 0) {
      launch_lb_tile(io);
    } else {
      launch_or_tile(io);
      cur = nx;
    }
  }
  // buffers of one step: in / out state, u (and optionally F) output
  struct Io {
    const GS* Bi;
    GS* Bo;
    const FS* phi_i;
    const FS* q_i;
    FS* phi_o;
    FS* q_o;
    R* u;
    R* F;
    R* drho;
    const int64_t* step_in = nullptr;  // step counters of a recording step's states
    int64_t* step_out = nullptr;
    FS* xs_q = nullptr;  // pc4 recording step: the predictor's X* goes here (record) instead of pcs
    FS* xs_phi = nullptr;
  };
  Io cur_io() { return Io{B[cur], B[cur ^ 1], Ph[cur], Q[cur], Ph[cur ^ 1], Q[cur ^ 1], u, nullptr, nullptr}; }
  void launch_lb_tile(const Io& io) {
    constexpr int W2 = sizeof(R) == 4 ? 2 : 1;  // double's registers allow one wave per SIMD on these tiles
    switch (lb_tile) {
      case 0: launch_lb<32, 8, W2>(io); break;
      case 1:  // float only: the double 32 x 16 frame does not fit the LDS (mapped to 16 x 16 at creation)
        if constexpr (sizeof(R) == 4) launch_lb<32, 16, 2>(io);
        break;
      case 2: launch_lb<64, 4, W2>(io); break;
      case 3: launch_lb<16, 16, W2>(io); break;
      default: launch_lb<16, 8, 1>(io); break;
    }
  }
  template <int TX, int TY, int MINW>
  void launch_lb(const Io& io) {
    lbc::k_lb_fused<R, GS, FS, L, TX, TY, MINW><<<lb_blocks, TX * TY, 0, stream>>>(
        box, P, tz_lb, lb_ntx, lb_nty, io.Bi, io.Bo, io.phi_i, io.q_i, io.u, mu, io.F, io.drho, io.step_in,
        io.step_out);
  }
  void launch_or_tile(const Io& io) {
    switch (or_tile) {
      case 0: launch_or<32, 8, 2>(io); break;
      case 1: launch_or<64, 4, 2>(io); break;
      case 2: launch_or<32, 16, 2>(io); break;
      case 3: launch_or<64, 8, 2>(io); break;
      default:  // float only: 1024 threads need <= 128 VGPRs (double: mapped to 64 x 8 at creation)
        if constexpr (sizeof(R) == 4) launch_or<64, 16, 4>(io);
        break;
    }
  }
  template <int TX, int TY, int MINW>
  void launch_or(const Io& io) {
    lbc::k_order_fused<R, FS, TX, TY, MINW><<<or_blocks, TX * TY, 0, stream>>>(
        box, P, tz_or, or_ntx, or_nty, io.phi_i, io.q_i, io.u, mu, io.phi_o, io.q_o);
  }
  // the fused pair on explicit buffers
  // the whole Heun update of one step on the buffers of io (z-marching kernels)
  void pc_update(const Io& io) {
    FS* qs = io.xs_q ? io.xs_q : pcs;
    FS* phs = io.xs_phi ? io.xs_phi : pcs + 5 * N;
    launch_pc_mu(io.phi_i, io.q_i);
    launch_pc_stage<true>(io.phi_i, io.q_i, nullptr, nullptr, phs, qs, io.u);
    launch_pc_mu(phs, qs);
    launch_pc_stage<false>(phs, qs, io.phi_i, io.q_i, io.phi_o, io.q_o, io.u);
  }
  // the whole step in one launch (u, F, drho written only where io asks for them)
  void launch_step1(const Io& io) {
    if constexpr (sizeof(R) == 8) {  // 158 KB of LDS on the 32 x 8 tile: one workgroup per CU
      launch_step1_tile<32, 8, 1>(io);
    } else {
      switch (st_tile) {
        case 1: launch_step1_tile<32, 16, 2>(io); break;
        case 2: launch_step1_tile<64, 8, 2>(io); break;
        default: launch_step1_tile<32, 8, 2>(io); break;
      }
    }
  }
  template <int TX, int TY, int MINW>
  void launch_step1_tile(const Io& io) {
    lbc::k_step_fused<R, GS, FS, L, TX, TY, MINW><<<st_blocks, TX * TY, 0, stream>>>(
        box, P, st_tz, st_ntx, st_nty, io.Bi, io.Bo, io.phi_i, io.q_i, io.phi_o, io.q_o, io.u, io.F, io.drho,
        io.step_in, io.step_out);
  }
  void fused_step(const Io& io) {
    if (one_launch) {
      launch_step1(io);
      return;
    }
    launch_lb_tile(io);
    if (pc4)
      pc_update(io);
    else
      launch_or_tile(io);
  }
  void step(int n) override {
    const int nk = nkernels();
    for (int s = 0; s < n; ++s)
      for (int k = 0; k < nk; ++k) launch(k);
    check_launch();
  }
  void profile(int n, double* ms, int* count) override {
    const int NK = nkernels();
    *count = NK;
    for (int k = 0; k < NK; ++k) ms[k] = 0.0;
    const int chunk = 32;
    std::vector<hipEvent_t> ev(size_t(chunk) * (NK + 1));
    for (auto& e : ev) HIPCHECK(hipEventCreate(&e));
    int done = 0;
    try {
      while (done < n) {
        const int m = std::min(chunk, n - done);
        for (int s = 0; s < m; ++s) {
          for (int k = 0; k < NK; ++k) {
            HIPCHECK(hipEventRecord(ev[size_t(s) * (NK + 1) + k], stream));
            launch(k);
          }
          HIPCHECK(hipEventRecord(ev[size_t(s) * (NK + 1) + NK], stream));
        }
        check_launch();
        HIPCHECK(hipStreamSynchronize(stream));
        for (int s = 0; s < m; ++s)
          for (int k = 0; k < NK; ++k) {
            float t = 0.f;
            HIPCHECK(hipEventElapsedTime(&t, ev[size_t(s) * (NK + 1) + k], ev[size_t(s) * (NK + 1) + k + 1]));
            ms[k] += t;
          }
        done += m;
      }
    } catch (...) {
      for (auto& e : ev) (void)hipEventDestroy(e);
      throw;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (int k = 0; k < NK; ++k) ms[k] /= (n > 0 ? n : 1);
  }

  // --- observation -----------------------------------------------------------
  void thermo_now() {
    ensure_thermo();
    lbc::k_thermo<R, FS><<<nblk, TPB, 0, stream>>>(box, P, Ph[cur], Q[cur], mu, H, sig);
    check_launch();
  }
  void moments(double* rho, double* u3, double* phi, double* q5) override {
    if (rho || u3) {
      thermo_now();
      R* r = dalloc<R>(N);
      R* uu = nullptr;
      try {
        uu = dalloc<R>(3 * N);
        lbc::k_moments<R, GS, L><<<nblk, TPB, 0, stream>>>(box, P, B[cur], sig, r, uu);
        check_launch();
        if (rho) d2h_convert(r, rho, N);
        if (u3) d2h_convert(uu, u3, 3 * N);
      } catch (...) {
        dfree(r);
        dfree(uu);
        throw;
      }
      dfree(r);
      dfree(uu);
    }
    if (phi) d2h_convert(Ph[cur], phi, N);
    if (q5) d2h_convert(Q[cur], q5, 5 * N);
  }
  void populations(double* g19) override {
    R* g = dalloc<R>(NQ * N);
    try {
      lbc::k_pull<R, GS, L><<<nblk, TPB, 0, stream>>>(box, B[cur], g);
      check_launch();
      d2h_convert(g, g19, NQ * N);
    } catch (...) {
      dfree(g);
      throw;
    }
    dfree(g);
  }
  void final_sum(const double* part, int nblocks, int nv) { final_sum_into(stream, part, nblocks, nv, mids, sums); }
  void totals(double out[lbc::NTOT]) override {
    thermo_now();
    lbc::k_totals<R, GS, FS, L><<<nblk, TPB, 0, stream>>>(box, Pd, B[cur], Ph[cur], Q[cur], sig, partial);
    final_sum(partial, int(nblk), lbc::NTOT);
    check_launch();
    HIPCHECK(hipMemcpyAsync(out, sums, lbc::NTOT * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHECK(hipStreamSynchronize(stream));
  }
  void centre(double out[lbc::NCEN]) override {
    lbc::k_centre<FS><<<nblk, TPB, 0, stream>>>(box, Ph[cur], partial);
    final_sum(partial, int(nblk), lbc::NCEN);
    check_launch();
    HIPCHECK(hipMemcpyAsync(out, sums, lbc::NCEN * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHECK(hipStreamSynchronize(stream));
  }

  // --- checkpoint --------------------------------------------------------------
  size_t off_q() const { return align256(NQ * N * sizeof(GS)); }
  size_t off_phi() const { return off_q() + align256(5 * N * sizeof(FS)); }
  size_t off_step() const { return off_phi() + align256(N * sizeof(FS)); }
  size_t state_bytes() const override { return off_step() + sizeof(int64_t); }
  void get_state(void* dst, int64_t stepno) override {
    char* d = static_cast<char*>(dst);
    HIPCHECK(hipMemcpyAsync(d, B[cur], NQ * N * sizeof(GS), hipMemcpyDeviceToDevice, stream));
    HIPCHECK(hipMemcpyAsync(d + off_q(), Q[cur], 5 * N * sizeof(FS), hipMemcpyDeviceToDevice, stream));
    HIPCHECK(hipMemcpyAsync(d + off_phi(), Ph[cur], N * sizeof(FS), hipMemcpyDeviceToDevice, stream));
    HIPCHECK(hipMemcpyAsync(d + off_step(), &stepno, sizeof(int64_t), hipMemcpyHostToDevice, stream));
    HIPCHECK(hipStreamSynchronize(stream));
  }
  int64_t set_state(const void* src) override {
    const char* s = static_cast<const char*>(src);
    HIPCHECK(hipMemcpyAsync(B[cur], s, NQ * N * sizeof(GS), hipMemcpyDeviceToDevice, stream));
    HIPCHECK(hipMemcpyAsync(Q[cur], s + off_q(), 5 * N * sizeof(FS), hipMemcpyDeviceToDevice, stream));
    HIPCHECK(hipMemcpyAsync(Ph[cur], s + off_phi(), N * sizeof(FS), hipMemcpyDeviceToDevice, stream));
    int64_t stepno = 0;
    HIPCHECK(hipMemcpyAsync(&stepno, s + off_step(), sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    HIPCHECK(hipStreamSynchronize(stream));
    return stepno;
  }

  // --- adjoint ---------------------------------------------------------------
  // adjoint buffer: g_bar [NQ][N], q_bar [5][N], phi_bar [N] in R.  The
  // reverses of the D3Q15 scheme and of the pc4 integrator exist for the
  // fused kernels only.
  bool has_adjoint() const { return !(site_path && (pc4 || L::kStressInEq)); }
  void need_adjoint() const {
    if (!has_adjoint())
      fail(LB_EINVAL, "the adjoint of the D3Q15 scheme and of the pc4 integrator needs the fused kernels");
  }
  size_t adjoint_bytes() const override { return has_adjoint() ? (NQ + 6) * N * sizeof(R) : 0; }
  void ensure_adjoint() {
    if (aF) return;
    try {
      aF = dalloc<R>(3 * N);
      amub = dalloc<R>(N);
      if (site_path) aWb = dalloc<R>(9 * N);  // the fused order kernel forms the whole u_bar
      aubp = dalloc<R>(3 * N);
      aqbp = dalloc<R>(5 * N);
      aphibp = dalloc<R>(N);
      aFb = dalloc<R>(3 * N);
      if (site_path) agbar = dalloc<R>(size_t(lbc::NGB) * N);  // the fused kernel keeps it on chip
      if (L::kStressInEq) aSb = dalloc<R>(6 * N);  // adjoint of the symmetric stress in the collision
      if (pc4) {
        apb = dalloc<R>(size_t(lbc::NPB) * N);  // per-site scratch of one R'^T V product
        if (pf_fused && pf_ntx > 1) apfx = dalloc<R>(4 * lbc::kRec * size_t(pf_ntx) * box.nz * box.ny);
        if (pf_fused && pf_nty > 1) apfy = dalloc<R>(36 * size_t(pf_nty) * box.nz * box.nx);
        axs = dalloc<R>(6 * N);                 // X*_bar: q [5][N], phi [N]
        aupc = dalloc<R>(3 * N);                // u_bar of both Heun stages
        const int ncb = (box.nx * box.ny + 255) / 256;  // column blocks of a plane
        gz_tz = auto_slab(ncb, 1, box.nz, 16, 1, 2);
        gz_blocks = ncb * ((box.nz + gz_tz - 1) / gz_tz);
      }
      if (!site_path && as_ntx > 1) ahx = dalloc<R>(24 * size_t(as_ntx) * box.nz * box.ny);
      if (!site_path && as_nty > 1) ahy = dalloc<R>(12 * size_t(as_nty) * box.nz * box.nx);
      // one (zeta, q0) pair per block of whichever reverse kernel writes them
      // pc4: the stress kernel's blocks, then those of k_pcb_local
      const int pc_part = std::max<int>(int(nblk), pf_blocks);  // the pc4 product kernel's blocks
      const size_t npart = size_t(pc4 ? as_blocks + pc_part : std::max<int>(int(nblk), as_blocks)) * 2;
      apart = dalloc<double>(npart);
      apart_n = npart;
      HIPCHECK(hipMemsetAsync(apart, 0, npart * sizeof(double), stream));
      apart_live = false;
    } catch (...) {
      R** adj[] = {&aF, &amub, &aWb, &aubp, &aqbp, &aphibp, &aFb, &agbar, &ahx, &ahy, &aSb, &apb, &axs, &aupc, &apfx, &apfy};
      for (R** a : adj) {
        dfree(*a);
        *a = nullptr;
      }
      dfree(apart);
      apart = nullptr;
      throw;
    }
  }
  // record buffer: u [3][N] and F [3][N] of the step that leaves the state
  // step record: u [3][N], F [3][N] and drho [N] of the step that leaves the state
  // pc4: then the predictor's X* = (Q* [5][N], phi* [N]) in the storage type, which the
  // reverse of the step reads instead of recomputing the predictor
  size_t record_bytes() const override {
    return has_adjoint() ? 7 * N * sizeof(R) + (pc4 ? 6 * N * sizeof(FS) : 0) : 0;
  }
  FS* rec_xs(void* rec) const { return pc4 ? reinterpret_cast<FS*>(static_cast<char*>(rec) + 7 * N * sizeof(R)) : nullptr; }
  const FS* rec_xs(const void* rec) const {
    return pc4 ? reinterpret_cast<const FS*>(static_cast<const char*>(rec) + 7 * N * sizeof(R)) : nullptr;
  }
  struct StateView {
    const GS* B;
    const FS* q;
    const FS* phi;
    const int64_t* step;
  };
  StateView view(const void* st) const {
    const char* c = static_cast<const char*>(st);
    return StateView{reinterpret_cast<const GS*>(c), reinterpret_cast<const FS*>(c + off_q()),
                     reinterpret_cast<const FS*>(c + off_phi()), reinterpret_cast<const int64_t*>(c + off_step())};
  }
  // One forward step from a state buffer into another, recording u, F and
  // drho of the input time (the replay of a checkpoint segment for the adjoint).
  void step_record(const void* state_in, void* state_out, void* rec_out) override {
    need_adjoint();
    const StateView vi = view(state_in);
    R* ru = static_cast<R*>(rec_out);
    R* rF = ru + 3 * N;
    R* rd = ru + 6 * N;
    FS* xs = rec_xs(rec_out);
    if (!state_out) {  // the record only
      record_only(vi, ru, rF, rd, xs);
      check_launch();
      return;
    }
    char* co = static_cast<char*>(state_out);
    GS* Bo = reinterpret_cast<GS*>(co);
    FS* qo = reinterpret_cast<FS*>(co + off_q());
    FS* po = reinterpret_cast<FS*>(co + off_phi());
    int64_t* step_out = reinterpret_cast<int64_t*>(co + off_step());
    if (site_path) {
      ensure_thermo();
      lbc::k_thermo<R, FS><<<nblk, TPB, 0, stream>>>(box, P, vi.phi, vi.q, mu, H, sig);
      lbc::k_fwd_force<R, GS, L><<<nblk, TPB, 0, stream>>>(box, P, vi.B, sig, rF, ru, rd);
      lbc::k_collide<R, GS, L><<<nblk, TPB, 0, stream>>>(box, P, vi.B, Bo, sig, ru);
      lbc::k_order<R, FS><<<nblk, TPB, 0, stream>>>(box, P, vi.phi, vi.q, ru, H, mu, po, qo);
      lbc::k_step_count<<<1, 64, 0, stream>>>(vi.step, step_out);
    } else {
      fused_step(Io{vi.B, Bo, vi.phi, vi.q, po, qo, ru, rF, rd, vi.step, step_out, xs, xs ? xs + 5 * N : nullptr});
    }
    check_launch();
  }
  // u, F and drho of the state at vi without forming the next state: the
  // site path's force kernel, or the stress + collision kernel with no
  // population output and no order-parameter update
  void record_only(const StateView& vi, R* ru, R* rF, R* rd, FS* xs = nullptr) {
    if (site_path) {
      ensure_thermo();
      lbc::k_thermo<R, FS><<<nblk, TPB, 0, stream>>>(box, P, vi.phi, vi.q, mu, H, sig);
      lbc::k_fwd_force<R, GS, L><<<nblk, TPB, 0, stream>>>(box, P, vi.B, sig, rF, ru, rd);
    } else if (one_launch) {
      launch_step1(Io{vi.B, nullptr, vi.phi, vi.q, nullptr, nullptr, ru, rF, rd});
    } else {
      launch_lb_tile(Io{vi.B, nullptr, vi.phi, vi.q, nullptr, nullptr, ru, rF, rd});
      if (xs) {  // pc4: the predictor stage of the step (its X* is what the reverse reads)
        launch_pc_mu(vi.phi, vi.q);
        launch_pc_stage<true>(vi.phi, vi.q, nullptr, nullptr, xs + 5 * N, xs, ru);
      }
    }
  }
  // lean step record: Q [5][N], phi [N] (storage type) of time t, then drho,
  // u [3][N], F [3][N] of that step (arithmetic type), each 256-byte aligned
  size_t lr_phi() const { return align256(5 * N * sizeof(FS)); }
  size_t lr_drho() const { return lr_phi() + align256(N * sizeof(FS)); }
  size_t lr_u() const { return lr_drho() + align256(N * sizeof(R)); }
  size_t lr_F() const { return lr_u() + align256(3 * N * sizeof(R)); }
  size_t lr_xs() const { return lr_F() + align256(3 * N * sizeof(R)); }  // pc4: Q* [5][N], then phi* [N]
  size_t lean_record_bytes() const override {
    return has_adjoint() ? lr_xs() + (pc4 ? align256(5 * N * sizeof(FS)) + align256(N * sizeof(FS)) : 0) : 0;
  }
  // Record time t into a lean record and advance the context's state by one step.
  void step_record_lean(void* rec_out) override {
    need_adjoint();
    char* c = static_cast<char*>(rec_out);
    R* rd = reinterpret_cast<R*>(c + lr_drho());
    R* ru = reinterpret_cast<R*>(c + lr_u());
    R* rF = reinterpret_cast<R*>(c + lr_F());
    HIPCHECK(hipMemcpyAsync(c, Q[cur], 5 * N * sizeof(FS), hipMemcpyDeviceToDevice, stream));
    HIPCHECK(hipMemcpyAsync(c + lr_phi(), Ph[cur], N * sizeof(FS), hipMemcpyDeviceToDevice, stream));
    const int nx = cur ^ 1;
    if (site_path) {
      ensure_thermo();
      lbc::k_thermo<R, FS><<<nblk, TPB, 0, stream>>>(box, P, Ph[cur], Q[cur], mu, H, sig);
      lbc::k_fwd_force<R, GS, L><<<nblk, TPB, 0, stream>>>(box, P, B[cur], sig, rF, ru, rd);
      lbc::k_collide<R, GS, L><<<nblk, TPB, 0, stream>>>(box, P, B[cur], B[nx], sig, ru);
      lbc::k_order<R, FS><<<nblk, TPB, 0, stream>>>(box, P, Ph[cur], Q[cur], ru, H, mu, Ph[nx], Q[nx]);
    } else {
      FS* xq = pc4 ? reinterpret_cast<FS*>(c + lr_xs()) : nullptr;
      FS* xp = pc4 ? reinterpret_cast<FS*>(c + lr_xs() + align256(5 * N * sizeof(FS))) : nullptr;
      fused_step(Io{B[cur], B[nx], Ph[cur], Q[cur], Ph[nx], Q[nx], ru, rF, rd, nullptr, nullptr, xq, xp});
    }
    cur = nx;
    check_launch();
  }
  void adjoint_step_lean(const void* rec, const void* adj_in, void* adj_out, double* zeta_bar,
                         double* q0_bar) override {
    need_adjoint();
    ensure_adjoint();
    const char* c = static_cast<const char*>(rec);
    const FS* rq = reinterpret_cast<const FS*>(c);
    const FS* rphi = reinterpret_cast<const FS*>(c + lr_phi());
    const R* rd = reinterpret_cast<const R*>(c + lr_drho());
    const R* ru = reinterpret_cast<const R*>(c + lr_u());
    const R* rF = reinterpret_cast<const R*>(c + lr_F());
    const FS* xq = pc4 ? reinterpret_cast<const FS*>(c + lr_xs()) : nullptr;
    const FS* xp = pc4 ? reinterpret_cast<const FS*>(c + lr_xs() + align256(5 * N * sizeof(FS))) : nullptr;
    reverse_kernels(rphi, rq, ru, rF, nullptr, rd, adj_in, adj_out, zeta_bar, q0_bar, xq, xp);
  }
  // the z-marching order adjoint: mu_bar, the whole u_bar and the site-local Q, phi adjoints
  void launch_adj_order(const FS* phi_t, const FS* q_t, const R* uu, const R* pi, const R* qi) {
    if (ao_ty == 16)
      lbc::k_adj_order_fused<R, FS, kAoTX, 16><<<ao_blocks, kAoTX * 16, 0, stream>>>(
          box, P, ao_tz, ao_ntx, ao_nty, phi_t, q_t, uu, pi, qi, amub, aubp, aqbp, aphibp);
    else
      lbc::k_adj_order_fused<R, FS, kAoTX, 8><<<ao_blocks, kAoTX * 8, 0, stream>>>(
          box, P, ao_tz, ao_ntx, ao_nty, phi_t, q_t, uu, pi, qi, amub, aubp, aqbp, aphibp);
  }
  // the fused stress + gather adjoint and its tile-face terms; aq: Q_bar(t+1)
  // for the Euler update's H_bar (zeros under pc4), mb: mu_bar
  // aq == mb == nullptr: no Q_bar(t+1) or mu_bar seeds (the pc4 reverse)
  void stress_gather(const FS* phi_t, const FS* q_t, const R* aq, const R* mb, R* po, R* qo) {
    const int acc = apart_live ? 1 : 0;
    if (as_ty == 16) {
      if (aq)
        lbc::k_adj_sg_fused<R, FS, kAsTX, 16, L::kStressInEq><<<as_blocks, kAsTX * 16, 0, stream>>>(
            box, P, as_tz, as_ntx, as_nty, phi_t, q_t, aFb, aq, mb, aqbp, aphibp, aSb, po, qo, ahx, ahy, apart, acc);
      else
        lbc::k_adj_sg_fused<R, FS, kAsTX, 16, L::kStressInEq, false><<<as_blocks, kAsTX * 16, 0, stream>>>(
            box, P, as_tz, as_ntx, as_nty, phi_t, q_t, aFb, nullptr, nullptr, aqbp, aphibp, aSb, po, qo, ahx, ahy,
            apart, acc);
    } else {
      if (aq)
        lbc::k_adj_sg_fused<R, FS, kAsTX, 8, L::kStressInEq><<<as_blocks, kAsTX * 8, 0, stream>>>(
            box, P, as_tz, as_ntx, as_nty, phi_t, q_t, aFb, aq, mb, aqbp, aphibp, aSb, po, qo, ahx, ahy, apart, acc);
      else
        lbc::k_adj_sg_fused<R, FS, kAsTX, 8, L::kStressInEq, false><<<as_blocks, kAsTX * 8, 0, stream>>>(
            box, P, as_tz, as_ntx, as_nty, phi_t, q_t, aFb, nullptr, nullptr, aqbp, aphibp, aSb, po, qo, ahx, ahy,
            apart, acc);
    }
    // blocks of up to 256 rows (columns) per plane and per (field, x face),
    // then per (field, y face)
    const unsigned gy = (as_ntx > 1 ? 6u * unsigned(as_ntx) : 0u) + (as_nty > 1 ? 6u * unsigned(as_nty) : 0u);
    if (gy > 0) {
      const int line = std::max(box.nx, box.ny);
      const unsigned tpb = unsigned(std::min(256, (line + 63) / 64 * 64));
      const dim3 grid(unsigned((line + int(tpb) - 1) / int(tpb)), gy, unsigned(box.nz));
      lbc::k_adj_faces<R><<<grid, tpb, 0, stream>>>(box, kAsTX, as_ntx, as_ty, as_nty, ahx, ahy, po, qo);
    }
  }
  // Reverse of a step of the pc4 integrator: the predictor is replayed from
  // X = (phi_t, q_t) with the step's velocity uu, the two Heun products
  // R'(X*)^T (X_bar(t+1)/2) and R'(X)^T X*_bar give the order parameters' part
  // of X_bar(t) (in aqbp, aphibp) and u_bar (aupc); then the collision and
  // the stress reverses (the stress kernel without the Euler update's H_bar
  // and mu_bar, which pc4 does not use).
  void reverse_pc4(const FS* phi_t, const FS* q_t, const R* uu, const R* FF, const GS* Bt, const R* drho,
                   const R* gi, const R* qi, const R* pi, R* go, R* qo, R* po, const FS* xs_q, const FS* xs_phi) {
    const FS* qs = xs_q;
    const FS* phs = xs_phi;
    if (!qs) {  // no recorded X*: replay the predictor
      launch_pc_mu(phi_t, q_t);
      launch_pc_stage<true>(phi_t, q_t, nullptr, nullptr, pcs + 5 * N, pcs, uu);
      qs = pcs;
      phs = pcs + 5 * N;
    }
    double* pl = apart + size_t(as_blocks) * 2;  // the product kernel's block partials follow the stress kernel's
    R* xsq = axs;
    R* xsp = axs + 5 * N;
    if (pf_fused) {
      R* zf = apb;          // z-stencil adjoints [9][N]
      R* mb = apb + 9 * N;  // mu_bar of the product
      auto product = [&](const FS* ph, const FS* qq, const R* vq, const R* vp, R vs, R c2, const R* x2q,
                         const R* x2p, R* oq, R* op, int acc, int pacc) {
        lbc::k_pcb_mub<R, 32, 8, 8><<<mb_blocks, 256, 0, stream>>>(box, P, mb_ntx, mb_nty, vp, vs, mb);
        lbc::k_pcb_fused<R, FS, kPfTX, kPfTY><<<pf_blocks, kPfTX * kPfTY, 0, stream>>>(
            box, P, pf_tz, pf_ntx, pf_nty, ph, qq, uu, vq, vp, vs, mb, qi, pi, R(0.5), x2q, x2p, c2, oq, op, aupc,
            acc, zf, apfx, apfy, pl, pacc);
        lbc::k_pcb_gather_z<R, FS, true><<<gz_blocks, 256, 0, stream>>>(box, P, gz_tz, ph, uu, vq, vp, vs, nullptr,
                                                                         oq, op, aupc, zf, mb, kPfTX, kPfTY, pf_ntx,
                                                                         pf_nty, apfx, apfy);
      };
      // X*_bar = X_bar(t+1)/2 + R'(X*)^T (X_bar(t+1)/2)
      product(phs, qs, qi, pi, R(0.5), R(0), nullptr, nullptr, xsq, xsp, 0, apart_live ? 1 : 0);
      // X_bar = X_bar(t+1)/2 + X*_bar + R'(X)^T X*_bar
      product(phi_t, q_t, xsq, xsp, R(1), R(1), xsq, xsp, aqbp, aphibp, 1, 1);
    } else {
      // X*_bar = X_bar(t+1)/2 + R'(X*)^T (X_bar(t+1)/2)
      lbc::k_pcb_local<R, FS><<<nblk, TPB, 0, stream>>>(box, P, phs, qs, uu, qi, pi, R(0.5), apb, pl,
                                                         apart_live ? 1 : 0);
      lbc::k_pcb_v<R, FS><<<nblk, TPB, 0, stream>>>(box, phs, qs, apb);
      lbc::k_pcb_gather<R, FS, 2><<<nblk, TPB, 0, stream>>>(box, phs, uu, qi, pi, R(0.5), apb, qi, pi, R(0.5),
                                                             nullptr, nullptr, R(0), xsq, xsp, aupc, 0);
      lbc::k_pcb_gather_z<R, FS, false><<<gz_blocks, 256, 0, stream>>>(box, P, gz_tz, phs, uu, qi, pi, R(0.5), apb, xsq, xsp,
                                                                 aupc, nullptr, nullptr, 0, 0, 1, 1, nullptr, nullptr);
      // X_bar = X_bar(t+1)/2 + X*_bar + R'(X)^T X*_bar
      lbc::k_pcb_local<R, FS><<<nblk, TPB, 0, stream>>>(box, P, phi_t, q_t, uu, xsq, xsp, R(1), apb, pl, 1);
      lbc::k_pcb_v<R, FS><<<nblk, TPB, 0, stream>>>(box, phi_t, q_t, apb);
      lbc::k_pcb_gather<R, FS, 2><<<nblk, TPB, 0, stream>>>(box, phi_t, uu, xsq, xsp, R(1), apb, qi, pi, R(0.5),
                                                             xsq, xsp, R(1), aqbp, aphibp, aupc, 1);
      lbc::k_pcb_gather_z<R, FS, false><<<gz_blocks, 256, 0, stream>>>(box, P, gz_tz, phi_t, uu, xsq, xsp, R(1), apb, aqbp,
                                                                 aphibp, aupc, nullptr, nullptr, 0, 0, 1, 1, nullptr, nullptr);
    }
    lbc::UbarIn<R> ubin{nullptr, aupc, 1};
    if (Bt)
      lbc::k_adj_collide<R, GS, L><<<nblk, TPB, 0, stream>>>(box, P, Bt, FF, ubin, gi, go, aFb, aSb);
    else
      lbc::k_adj_collide_lean<R, L><<<nblk, TPB, 0, stream>>>(box, P, drho, uu, FF, ubin, gi, go, aFb, aSb);
    stress_gather(phi_t, q_t, nullptr, nullptr, po, qo);
  }
  // the reverse kernels of one step; the collision adjoint reads the
  // populations B, or (B == nullptr) the recorded density deviation drho
  void reverse_kernels(const FS* phi_t, const FS* q_t, const R* uu, const R* FF, const GS* Bt, const R* drho,
                       const void* adj_in, void* adj_out, double* zeta_bar, double* q0_bar,
                       const FS* xs_q = nullptr, const FS* xs_phi = nullptr) {
    const R* gi = static_cast<const R*>(adj_in);
    const R* qi = gi + NQ * N;
    const R* pi = gi + (NQ + 5) * N;
    R* go = static_cast<R*>(adj_out);
    R* qo = go + NQ * N;
    R* po = go + (NQ + 5) * N;
    const int npart_blocks =
        site_path ? int(nblk) : (pc4 ? as_blocks + std::max<int>(int(nblk), pf_blocks) : as_blocks);
    if (size_t(npart_blocks) * 2 > apart_n) fail(LB_EDEVICE, "adjoint partial buffer smaller than the grid");
    if (pc4) {
      reverse_pc4(phi_t, q_t, uu, FF, Bt, drho, gi, qi, pi, go, qo, po, xs_q, xs_phi);
    } else {
      // site path: W_bar [9][N] and the local u_bar part; fused: the whole u_bar (in aubp)
      lbc::UbarIn<R> ubin{aWb, aubp, site_path ? 0 : 1};
      if (site_path)
        lbc::k_adj_order<R, FS><<<nblk, TPB, 0, stream>>>(box, P, phi_t, q_t, uu, pi, qi, amub, aWb, aubp, aqbp,
                                                           aphibp);
      else
        launch_adj_order(phi_t, q_t, uu, pi, qi);
      if (Bt)
        lbc::k_adj_collide<R, GS, L><<<nblk, TPB, 0, stream>>>(box, P, Bt, FF, ubin, gi, go, aFb, aSb);
      else
        lbc::k_adj_collide_lean<R, L><<<nblk, TPB, 0, stream>>>(box, P, drho, uu, FF, ubin, gi, go, aFb, aSb);
      if (site_path) {
        lbc::k_adj_stress<R, FS><<<nblk, TPB, 0, stream>>>(box, P, phi_t, q_t, aFb, qi, amub, aqbp, aphibp, agbar,
                                                            apart, apart_live ? 1 : 0);
        lbc::k_adj_gather<R><<<nblk, TPB, 0, stream>>>(box, agbar, po, qo);
      } else {
        stress_gather(phi_t, q_t, qi, amub, po, qo);
      }
    }
    apart_live = true;
    check_launch();
    if (!zeta_bar && !q0_bar) return;  // the parameter sums stay on the device
    final_sum(apart, npart_blocks, 2);
    check_launch();
    apart_live = false;
    double pv[2] = {0.0, 0.0};
    HIPCHECK(hipMemcpyAsync(pv, sums, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHECK(hipStreamSynchronize(stream));
    if (zeta_bar) *zeta_bar += pv[0];
    if (q0_bar) *q0_bar += pv[1];
  }
  void adjoint_step(const void* state, const void* rec, const void* adj_in, void* adj_out, double* zeta_bar,
                    double* q0_bar) override {
    need_adjoint();
    ensure_adjoint();
    const StateView v = view(state);
    if (rec) {  // the collision adjoint reads the recorded drho and u, not the populations
      const R* uu = static_cast<const R*>(rec);
      const FS* xs = rec_xs(rec);
      reverse_kernels(v.phi, v.q, uu, uu + 3 * N, nullptr, uu + 6 * N, adj_in, adj_out, zeta_bar, q0_bar, xs,
                      xs ? xs + 5 * N : nullptr);
      return;
    }
    // recompute u and F of time t
    ensure_thermo();
    lbc::k_thermo<R, FS><<<nblk, TPB, 0, stream>>>(box, P, v.phi, v.q, mu, H, sig);
    lbc::k_fwd_force<R, GS, L><<<nblk, TPB, 0, stream>>>(box, P, v.B, sig, aF, u, nullptr);
    reverse_kernels(v.phi, v.q, u, aF, v.B, nullptr, adj_in, adj_out, zeta_bar, q0_bar);
  }
  double seed_centre(double z_ref, void* adj) override {
    need_adjoint();
    double v[lbc::NCEN];
    centre(v);
    const double zc = v[2] / v[3];
    lbc::k_seed_centre<R><<<nblk, TPB, 0, stream>>>(box, NQ, zc, z_ref, v[3], static_cast<R*>(adj));
    check_launch();
    HIPCHECK(hipStreamSynchronize(stream));
    return (zc - z_ref) * (zc - z_ref);
  }
};

}  // namespace

struct lb_ctx {
  lb_params p{};
  hipStream_t stream = nullptr;
  int64_t step = 0;
  std::unique_ptr<Backend> be;
};

namespace {

template <class F>
lb_status guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return LB_OK;
  } catch (const LbError& e) {
    g_last_error = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return LB_ENOMEM;
  } catch (...) {
    g_last_error = "unknown error";
    return LB_EDEVICE;
  }
}

void need_ctx(const lb_ctx* c) {
  if (!c || !c->be) fail(LB_EINVAL, "null context");
}

void need_adjoint_ctx(const lb_ctx* c) {
  need_ctx(c);
  if (c->be->adjoint_bytes() == 0) fail(LB_EINVAL, "no adjoint for this context (D3Q15: fused kernels only)");
}

std::unique_ptr<Backend> make_backend(const lb_params& p, const lb_tuning& t, hipStream_t s) {
  switch (p.prec) {
    case LB_FP64:
      if (p.lattice == LB_D3Q15) return std::unique_ptr<Backend>(new BackendT<double, double, double, lbc::D3Q15>(p, t, s));
      return std::unique_ptr<Backend>(new BackendT<double, double, double, lbc::D3Q19>(p, t, s));
    case LB_FP32:
      if (p.lattice == LB_D3Q15) return std::unique_ptr<Backend>(new BackendT<float, float, float, lbc::D3Q15>(p, t, s));
      return std::unique_ptr<Backend>(new BackendT<float, float, float, lbc::D3Q19>(p, t, s));
    default:
      if (p.lattice == LB_D3Q15) return std::unique_ptr<Backend>(new BackendT<float, __half, float, lbc::D3Q15>(p, t, s));
      return std::unique_ptr<Backend>(new BackendT<float, __half, float, lbc::D3Q19>(p, t, s));
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free centre.  Its block partials, chunk sums and final sums live
// in `scratch`, a static device array of fixed size that each GPU the library
// runs on holds until the process ends.  In host code `scratch` names only a
// host-side stand-in: its device address on the current GPU is looked up once
// per device with hipGetSymbolAddress and kept in g_na_ptr, and only that
// address is ever passed to a kernel.
constexpr int kNaMaxBlocks = LB_NOALLOC_MAX_SITES / 256;  // k_centre: one site per thread, 256 per block
constexpr size_t kNaPartial = size_t(kNaMaxBlocks) * lbc::NCEN;
constexpr size_t kNaMids = size_t(kSumChunks) * lbc::NCEN;
constexpr size_t kNaDoubles = kNaPartial + kNaMids + lbc::NCEN;
static_assert(kNaDoubles * sizeof(double) <= LB_NOALLOC_SCRATCH_BYTES, "scratch size stated in the header");
static __device__ __align__(256) double scratch[kNaDoubles];

namespace {
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
double* g_na_ptr[kNaMaxDevices] = {};

// Device address of `scratch` on the current GPU (looked up on first use).
double* noalloc_scratch() {
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNaMaxDevices) fail(LB_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(LB_EDEVICE, "no device address for the scratch array");
    g_na_ptr[dev] = static_cast<double*>(p);
  }
  return g_na_ptr[dev];
}

template <class FS>
void centre_noalloc(const lbc::Box& box, const FS* phi, double* out, hipStream_t stream) {
  double* base = noalloc_scratch();
  double* partial = base;
  double* mids = base + kNaPartial;
  double* sums = mids + kNaMids;
  const int nblk = int((size_t(box.N) + TPB - 1) / TPB);
  lbc::k_centre<FS><<<nblk, TPB, 0, stream>>>(box, phi, partial);
  final_sum_into(stream, partial, nblk, lbc::NCEN, mids, sums);
  lbc::k_centre_finish<<<1, 64, 0, stream>>>(box, sums, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(LB_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}
}  // namespace

extern "C" {

lb_status lb_init_tuned(const lb_params* p, const lb_tuning* t, const double* phi, const double* q5,
                        const double* u0, void* hip_stream, lb_ctx** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!p || !phi || !q5 || !out) fail(LB_EINVAL, "null argument");
    validate(*p);
    lb_tuning tt{};
    if (t) tt = *t;
    validate_tuning(*p, tt);
    std::unique_ptr<lb_ctx> c(new lb_ctx);
    c->p = *p;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->be = make_backend(*p, tt, c->stream);
    c->be->upload(phi, q5, u0);
    *out = c.release();
  });
}

lb_status lb_init(const lb_params* p, const double* phi, const double* q5, const double* u0, void* hip_stream,
                  lb_ctx** out) {
  return lb_init_tuned(p, nullptr, phi, q5, u0, hip_stream, out);
}

lb_status lb_step(lb_ctx* c, int32_t nsteps) {
  return guarded([&] {
    need_ctx(c);
    if (nsteps < 0) fail(LB_EINVAL, "nsteps < 0");
    c->be->step(nsteps);
    c->step += nsteps;
  });
}

lb_status lb_set_params(lb_ctx* c, const lb_params* p) {
  return guarded([&] {
    need_ctx(c);
    if (!p) fail(LB_EINVAL, "null params");
    validate(*p);
    if (p->nx != c->p.nx || p->ny != c->p.ny || p->nz != c->p.nz || p->prec != c->p.prec ||
        p->lattice != c->p.lattice || p->fd_scheme != c->p.fd_scheme)
      fail(LB_EINVAL, "box size, precision, lattice and integrator cannot change");
    c->p = *p;
    c->be->set_params(*p);
  });
}

lb_status lb_moments(lb_ctx* c, double* rho, double* u3, double* phi, double* q5) {
  return guarded([&] {
    need_ctx(c);
    c->be->moments(rho, u3, phi, q5);
  });
}

lb_status lb_populations(lb_ctx* c, double* g19) {
  return guarded([&] {
    need_ctx(c);
    if (!g19) fail(LB_EINVAL, "null output");
    c->be->populations(g19);
  });
}

lb_status lb_set_fields(lb_ctx* c, const double* g19, const double* phi, const double* q5) {
  return guarded([&] {
    need_ctx(c);
    c->be->set_fields(g19, phi, q5);
  });
}

lb_status lb_free_energy(lb_ctx* c, lb_totals* out) {
  return guarded([&] {
    need_ctx(c);
    if (!out) fail(LB_EINVAL, "null output");
    double v[lbc::NTOT];
    c->be->totals(v);
    const double N = double(c->p.nx) * c->p.ny * c->p.nz;
    out->mass = N * c->p.rho0 + v[0];
    out->momentum[0] = v[1];
    out->momentum[1] = v[2];
    out->momentum[2] = v[3];
    out->phi_total = v[4];
    out->free_energy = v[5];
    out->kinetic_energy = v[6];
    out->step = c->step;
    bool finite = v[7] == 0.0;
    for (int k = 0; k < 7; ++k) finite = finite && std::isfinite(v[k]);
    if (!finite) fail(LB_ENONFINITE, "non-finite value in the state");
  });
}

lb_status lb_centre(lb_ctx* c, double out[6], double* phi_total) {
  return guarded([&] {
    need_ctx(c);
    if (!out) fail(LB_EINVAL, "null output");
    double v[lbc::NCEN];
    c->be->centre(v);
    const int n[3] = {c->p.nx, c->p.ny, c->p.nz};
    for (int a = 0; a < 3; ++a) {
      out[a] = v[a] / v[3];
      double ang = std::atan2(v[4 + 2 * a], v[5 + 2 * a]);
      double cc = ang * n[a] / (2.0 * M_PI);
      if (cc < 0) cc += n[a];
      out[3 + a] = cc;
    }
    if (phi_total) *phi_total = v[3];
  });
}

lb_status lb_centre_noalloc(int32_t nx, int32_t ny, int32_t nz, int32_t prec, const void* dev_phi,
                            double* dev_out, void* hip_stream) {
  return guarded([&] {
    if (nx < 1 || ny < 1 || nz < 1) fail(LB_EINVAL, "box sides must be >= 1");
    if (prec < LB_FP64 || prec > LB_FP16S) fail(LB_EINVAL, "unknown precision");
    if (!dev_phi || !dev_out) fail(LB_EINVAL, "null device pointer");
    const double n = double(nx) * double(ny) * double(nz);
    if (n > double(LB_NOALLOC_MAX_SITES))
      fail(LB_EINVAL, "box of " + std::to_string(int64_t(n)) + " sites exceeds the allocation-free maximum of " +
                          std::to_string(LB_NOALLOC_MAX_SITES) + " sites");
    lbc::Box box;
    box.nx = nx;
    box.ny = ny;
    box.nz = nz;
    box.N = int(size_t(nx) * ny * nz);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (prec == LB_FP64)
      centre_noalloc(box, static_cast<const double*>(dev_phi), dev_out, s);
    else
      centre_noalloc(box, static_cast<const float*>(dev_phi), dev_out, s);
  });
}

size_t lb_state_bytes(const lb_ctx* c) { return (c && c->be) ? c->be->state_bytes() : 0; }

lb_status lb_get_state(lb_ctx* c, void* dev_dst, size_t bytes) {
  return guarded([&] {
    need_ctx(c);
    if (!dev_dst) fail(LB_EINVAL, "null buffer");
    if (bytes != c->be->state_bytes()) fail(LB_ESTATE, "state buffer size mismatch");
    c->be->get_state(dev_dst, c->step);
  });
}

lb_status lb_set_state(lb_ctx* c, const void* dev_src, size_t bytes) {
  return guarded([&] {
    need_ctx(c);
    if (!dev_src) fail(LB_EINVAL, "null buffer");
    if (bytes != c->be->state_bytes()) fail(LB_ESTATE, "state buffer size mismatch");
    c->step = c->be->set_state(dev_src);
  });
}

size_t lb_adjoint_bytes(const lb_ctx* c) { return (c && c->be) ? c->be->adjoint_bytes() : 0; }

size_t lb_record_bytes(const lb_ctx* c) { return (c && c->be) ? c->be->record_bytes() : 0; }

lb_status lb_step_record(lb_ctx* c, const void* dev_state_in, void* dev_state_out, void* dev_rec_out,
                         size_t state_bytes, size_t rec_bytes) {
  return guarded([&] {
    need_adjoint_ctx(c);
    if (!dev_state_in || !dev_rec_out) fail(LB_EINVAL, "null buffer");
    if (dev_state_in == dev_state_out) fail(LB_EINVAL, "state_in and state_out must differ");
    if (state_bytes != c->be->state_bytes()) fail(LB_ESTATE, "state buffer size mismatch");
    if (rec_bytes != c->be->record_bytes()) fail(LB_ESTATE, "record buffer size mismatch");
    c->be->step_record(dev_state_in, dev_state_out, dev_rec_out);
  });
}

lb_status lb_adjoint_step(lb_ctx* c, const void* dev_state_t, size_t state_bytes, const void* dev_rec_t,
                          size_t rec_bytes, const void* dev_adj_in, void* dev_adj_out, size_t adj_bytes,
                          double* zeta_bar, double* q0_bar) {
  return guarded([&] {
    need_adjoint_ctx(c);
    if (!dev_state_t || !dev_adj_in || !dev_adj_out) fail(LB_EINVAL, "null buffer");
    if (dev_adj_in == dev_adj_out) fail(LB_EINVAL, "adj_in and adj_out must differ");
    if (state_bytes != c->be->state_bytes()) fail(LB_ESTATE, "state buffer size mismatch");
    if (dev_rec_t && rec_bytes != c->be->record_bytes()) fail(LB_ESTATE, "record buffer size mismatch");
    if (adj_bytes != c->be->adjoint_bytes()) fail(LB_ESTATE, "adjoint buffer size mismatch");
    c->be->adjoint_step(dev_state_t, dev_rec_t, dev_adj_in, dev_adj_out, zeta_bar, q0_bar);
  });
}

size_t lb_lean_record_bytes(const lb_ctx* c) {
  if (!c || !c->be) return 0;
  return c->be->lean_record_bytes();
}

lb_status lb_step_record_lean(lb_ctx* c, void* dev_rec_out, size_t rec_bytes) {
  return guarded([&] {
    need_adjoint_ctx(c);
    if (!dev_rec_out) fail(LB_EINVAL, "null buffer");
    if (rec_bytes != c->be->lean_record_bytes()) fail(LB_ESTATE, "lean record buffer size mismatch");
    c->be->step_record_lean(dev_rec_out);
    c->step += 1;
  });
}

lb_status lb_adjoint_step_lean(lb_ctx* c, const void* dev_rec_t, size_t rec_bytes, const void* dev_adj_in,
                               void* dev_adj_out, size_t adj_bytes, double* zeta_bar, double* q0_bar) {
  return guarded([&] {
    need_adjoint_ctx(c);
    if (!dev_rec_t || !dev_adj_in || !dev_adj_out) fail(LB_EINVAL, "null buffer");
    if (dev_adj_in == dev_adj_out) fail(LB_EINVAL, "adj_in and adj_out must differ");
    if (rec_bytes != c->be->lean_record_bytes()) fail(LB_ESTATE, "lean record buffer size mismatch");
    if (adj_bytes != c->be->adjoint_bytes()) fail(LB_ESTATE, "adjoint buffer size mismatch");
    c->be->adjoint_step_lean(dev_rec_t, dev_adj_in, dev_adj_out, zeta_bar, q0_bar);
  });
}

lb_status lb_adjoint_seed_centre(lb_ctx* c, double z_ref, void* dev_adj, size_t adj_bytes, double* loss) {
  return guarded([&] {
    need_adjoint_ctx(c);
    if (!dev_adj) fail(LB_EINVAL, "null buffer");
    if (adj_bytes != c->be->adjoint_bytes()) fail(LB_ESTATE, "adjoint buffer size mismatch");
    const double L = c->be->seed_centre(z_ref, dev_adj);
    if (loss) *loss = L;
  });
}

lb_status lb_profile_step(lb_ctx* c, int32_t nsteps, double* kernel_ms, int32_t* count) {
  return guarded([&] {
    need_ctx(c);
    if (!kernel_ms || !count || nsteps <= 0) fail(LB_EINVAL, "bad profile arguments");
    int n = 0;
    c->be->profile(nsteps, kernel_ms, &n);
    *count = n;
    c->step += nsteps;
  });
}

const char* lb_kernel_name(const lb_ctx* c, int32_t i) { return (c && c->be) ? c->be->kernel_name(i) : nullptr; }

lb_status lb_sync(lb_ctx* c) {
  return guarded([&] {
    need_ctx(c);
    HIPCHECK(hipStreamSynchronize(c->stream));
  });
}

void lb_destroy(lb_ctx* c) {
  if (!c) return;
  if (c->be) (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char* lb_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

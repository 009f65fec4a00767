// Host side of the C ABI declared in include/lb_nematic2d.h: the 2D bulk
// active nematic on D2Q9.  A context owns ping-pong population and Q buffers
// and u, and enqueues the two kernels of the step (kernels_2d.hpp) on its
// stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "kernels_2d.hpp"
#include "lb_nematic2d.h"

namespace {

thread_local std::string g2_last_error;

struct Err2 {
  lb_status st;
  std::string msg;
};

[[noreturn]] void fail2(lb_status st, const std::string& msg) { throw Err2{st, msg}; }

#define HIPCHECK2(expr)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) fail2(LB_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int TPB2 = 256;
constexpr int kTX = 32, kTY = 8;

template <class T>
T* dalloc2(size_t n) {
  void* p = nullptr;
  if (hipMalloc(&p, (n ? n : 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    fail2(LB_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  return static_cast<T*>(p);
}

void check_launch2() { HIPCHECK2(hipGetLastError()); }

void validate2(const lb2d_params& p) {
  if (p.nx < 3 || p.ny < 3) fail2(LB_EINVAL, "box sides must be >= 3");
  if (double(p.nx) * double(p.ny) > double(1 << 28)) fail2(LB_ENOMEM, "box exceeds 2^28 sites");
  if (p.prec != LB_FP64 && p.prec != LB_FP32) fail2(LB_EINVAL, "precision must be LB_FP64 or LB_FP32");
  const double v[] = {p.tau, p.rho0, p.A0, p.chi, p.K, p.Gamma, p.xi, p.zeta, p.body_force[0], p.body_force[1]};
  for (double x : v)
    if (!std::isfinite(x)) fail2(LB_EINVAL, "non-finite parameter");
  if (!(p.tau > 0.5)) fail2(LB_EINVAL, "tau must be > 0.5");
  if (!(p.rho0 > 0.0)) fail2(LB_EINVAL, "rho0 must be > 0");
}

template <class R>
lbc2::Params2<R> params2(const lb2d_params& p) {
  lbc2::Params2<R> P;
  P.omega = R(1.0 / p.tau);
  P.guo = R(1.0 - 0.5 / p.tau);
  P.rho0 = R(p.rho0);
  P.A0 = R(p.A0);
  P.chi = R(p.chi);
  P.K = R(p.K);
  P.Gamma = R(p.Gamma);
  P.xi = R(p.xi);
  P.zeta = R(p.zeta);
  P.bf[0] = R(p.body_force[0]);
  P.bf[1] = R(p.body_force[1]);
  return P;
}

struct Backend2 {
  virtual ~Backend2() = default;
  virtual void step(int n) = 0;
  virtual void moments(double* rho, double* u, double* q2) = 0;
  virtual void populations(double* g9) = 0;
  virtual void set_fields(const double* g9, const double* q2) = 0;
  virtual void totals(lb2d_totals* t) = 0;
  virtual void profile(int n, double* ms, int* count) = 0;
};

template <class R>
struct Backend2T final : Backend2 {
  lbc2::Box2 box;
  hipStream_t stream;
  lbc2::Params2<R> P;
  lbc2::Params2<double> Pd;
  size_t N;
  unsigned nblk;
  int ntx, nty;
  R* B[2] = {nullptr, nullptr};
  R* Q[2] = {nullptr, nullptr};
  R* u = nullptr;
  int cur = 0;

  Backend2T(const lb2d_params& p, hipStream_t s, const double* q2, const double* u0) : stream(s) {
    box.nx = p.nx;
    box.ny = p.ny;
    N = size_t(p.nx) * p.ny;
    box.N = int(N);
    nblk = unsigned((N + TPB2 - 1) / TPB2);
    ntx = (p.nx + kTX - 1) / kTX;
    nty = (p.ny + kTY - 1) / kTY;
    P = params2<R>(p);
    Pd = params2<double>(p);
    try {
      for (int k = 0; k < 2; ++k) {
        B[k] = dalloc2<R>(9 * N);
        Q[k] = dalloc2<R>(2 * N);
      }
      u = dalloc2<R>(2 * N);
      upload_q(q2, Q[0]);
      double* du = nullptr;
      double* g = dalloc2<double>(9 * N);
      try {
        if (u0) {
          du = dalloc2<double>(2 * N);
          HIPCHECK2(hipMemcpyAsync(du, u0, 2 * N * sizeof(double), hipMemcpyHostToDevice, stream));
        }
        lbc2::k2_equilibrium<<<nblk, TPB2, 0, stream>>>(box, p.rho0, du, g);
        lbc2::k2_push<R><<<nblk, TPB2, 0, stream>>>(box, g, B[0]);
        check_launch2();
        HIPCHECK2(hipStreamSynchronize(stream));
      } catch (...) {
        (void)hipFree(g);
        if (du) (void)hipFree(du);
        throw;
      }
      (void)hipFree(g);
      if (du) (void)hipFree(du);
    } catch (...) {
      release();
      throw;
    }
  }
  ~Backend2T() override { release(); }
  void release() {
    for (int k = 0; k < 2; ++k) {
      if (B[k]) (void)hipFree(B[k]);
      if (Q[k]) (void)hipFree(Q[k]);
      B[k] = Q[k] = nullptr;
    }
    if (u) (void)hipFree(u);
    u = nullptr;
  }
  void upload_q(const double* q2, R* dst) {
    std::vector<R> h(2 * N);
    for (size_t k = 0; k < 2 * N; ++k) h[k] = R(q2[k]);
    HIPCHECK2(hipMemcpyAsync(dst, h.data(), 2 * N * sizeof(R), hipMemcpyHostToDevice, stream));
    HIPCHECK2(hipStreamSynchronize(stream));
  }
  void launch(int k) {
    const int nx = cur ^ 1;
    if (k == 0) {
      lbc2::k2_lb<R, kTX, kTY><<<ntx * nty, kTX * kTY, 0, stream>>>(box, P, ntx, B[cur], B[nx], Q[cur], u);
    } else {
      lbc2::k2_order<R><<<nblk, TPB2, 0, stream>>>(box, P, Q[cur], u, Q[nx]);
      cur = nx;
    }
  }
  void step(int n) override {
    for (int s = 0; s < n; ++s) {
      launch(0);
      launch(1);
    }
    check_launch2();
  }
  void observe(std::vector<double>& out) {
    double* d = dalloc2<double>(6 * N);
    try {
      lbc2::k2_observe<R><<<nblk, TPB2, 0, stream>>>(box, Pd, B[cur], Q[cur], d);
      check_launch2();
      out.resize(6 * N);
      HIPCHECK2(hipMemcpyAsync(out.data(), d, 6 * N * sizeof(double), hipMemcpyDeviceToHost, stream));
      HIPCHECK2(hipStreamSynchronize(stream));
    } catch (...) {
      (void)hipFree(d);
      throw;
    }
    (void)hipFree(d);
  }
  void moments(double* rho, double* u2, double* q2) override {
    if (rho || u2) {
      std::vector<double> o;
      observe(o);
      if (rho) std::copy(o.begin(), o.begin() + N, rho);
      if (u2) std::copy(o.begin() + N, o.begin() + 3 * N, u2);
    }
    if (q2) {
      std::vector<R> h(2 * N);
      HIPCHECK2(hipMemcpyAsync(h.data(), Q[cur], 2 * N * sizeof(R), hipMemcpyDeviceToHost, stream));
      HIPCHECK2(hipStreamSynchronize(stream));
      for (size_t k = 0; k < 2 * N; ++k) q2[k] = double(h[k]);
    }
  }
  void populations(double* g9) override {
    double* d = dalloc2<double>(9 * N);
    try {
      lbc2::k2_pull<R><<<nblk, TPB2, 0, stream>>>(box, B[cur], d);
      check_launch2();
      HIPCHECK2(hipMemcpyAsync(g9, d, 9 * N * sizeof(double), hipMemcpyDeviceToHost, stream));
      HIPCHECK2(hipStreamSynchronize(stream));
    } catch (...) {
      (void)hipFree(d);
      throw;
    }
    (void)hipFree(d);
  }
  void set_fields(const double* g9, const double* q2) override {
    if (q2) upload_q(q2, Q[cur]);
    if (g9) {
      double* d = dalloc2<double>(9 * N);
      try {
        HIPCHECK2(hipMemcpyAsync(d, g9, 9 * N * sizeof(double), hipMemcpyHostToDevice, stream));
        lbc2::k2_push<R><<<nblk, TPB2, 0, stream>>>(box, d, B[cur]);
        check_launch2();
        HIPCHECK2(hipStreamSynchronize(stream));
      } catch (...) {
        (void)hipFree(d);
        throw;
      }
      (void)hipFree(d);
    }
  }
  void totals(lb2d_totals* t) override {
    std::vector<double> o;
    observe(o);
    double m = 0, px = 0, py = 0, fe = 0, ke = 0;
    for (size_t s = 0; s < N; ++s) {
      m += o[3 * N + s];
      px += o[s] * o[N + s];
      py += o[s] * o[2 * N + s];
      fe += o[4 * N + s];
      ke += o[5 * N + s];
    }
    if (!std::isfinite(m) || !std::isfinite(fe) || !std::isfinite(ke)) fail2(LB_ENONFINITE, "non-finite state");
    t->mass = double(N) * Pd.rho0 + m;
    t->momentum[0] = px;
    t->momentum[1] = py;
    t->free_energy = fe;
    t->kinetic_energy = ke;
  }
  void profile(int n, double* ms, int* count) override {
    *count = 2;
    ms[0] = ms[1] = 0.0;
    hipEvent_t ev[3];
    for (auto& e : ev) HIPCHECK2(hipEventCreate(&e));
    try {
      for (int s = 0; s < n; ++s) {
        for (int k = 0; k < 2; ++k) {
          HIPCHECK2(hipEventRecord(ev[k], stream));
          launch(k);
        }
        HIPCHECK2(hipEventRecord(ev[2], stream));
        check_launch2();
        HIPCHECK2(hipEventSynchronize(ev[2]));
        for (int k = 0; k < 2; ++k) {
          float t = 0.f;
          HIPCHECK2(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
          ms[k] += t;
        }
      }
    } catch (...) {
      for (auto& e : ev) (void)hipEventDestroy(e);
      throw;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (int k = 0; k < 2; ++k) ms[k] /= (n > 0 ? n : 1);
  }
};

template <class F>
lb_status guarded2(F&& f) {
  try {
    f();
    return LB_OK;
  } catch (const Err2& e) {
    g2_last_error = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    g2_last_error = "host allocation failed";
    return LB_ENOMEM;
  } catch (...) {
    g2_last_error = "unknown error";
    return LB_EDEVICE;
  }
}

}  // namespace

struct lb2d_ctx {
  lb2d_params p{};
  hipStream_t stream = nullptr;
  int64_t step = 0;
  std::unique_ptr<Backend2> be;
};

namespace {
void need2(const lb2d_ctx* c) {
  if (!c || !c->be) fail2(LB_EINVAL, "null context");
}
}  // namespace

extern "C" {

lb_status lb2d_init(const lb2d_params* p, const double* q2, const double* u0, void* stream, lb2d_ctx** out) {
  if (out) *out = nullptr;
  return guarded2([&] {
    if (!p || !q2 || !out) fail2(LB_EINVAL, "null argument");
    validate2(*p);
    auto c = std::make_unique<lb2d_ctx>();
    c->p = *p;
    c->stream = static_cast<hipStream_t>(stream);
    if (p->prec == LB_FP64)
      c->be.reset(new Backend2T<double>(*p, c->stream, q2, u0));
    else
      c->be.reset(new Backend2T<float>(*p, c->stream, q2, u0));
    *out = c.release();
  });
}

lb_status lb2d_step(lb2d_ctx* c, int32_t nsteps) {
  return guarded2([&] {
    need2(c);
    if (nsteps < 0) fail2(LB_EINVAL, "negative step count");
    c->be->step(nsteps);
    c->step += nsteps;
  });
}

lb_status lb2d_sync(lb2d_ctx* c) {
  return guarded2([&] {
    need2(c);
    HIPCHECK2(hipStreamSynchronize(c->stream));
  });
}

lb_status lb2d_moments(lb2d_ctx* c, double* rho, double* u, double* q2) {
  return guarded2([&] {
    need2(c);
    c->be->moments(rho, u, q2);
  });
}

lb_status lb2d_populations(lb2d_ctx* c, double* g9) {
  return guarded2([&] {
    need2(c);
    if (!g9) fail2(LB_EINVAL, "null buffer");
    c->be->populations(g9);
  });
}

lb_status lb2d_set_fields(lb2d_ctx* c, const double* g9, const double* q2) {
  return guarded2([&] {
    need2(c);
    c->be->set_fields(g9, q2);
  });
}

lb_status lb2d_free_energy(lb2d_ctx* c, lb2d_totals* t) {
  return guarded2([&] {
    need2(c);
    if (!t) fail2(LB_EINVAL, "null totals");
    c->be->totals(t);
    t->step = c->step;
  });
}

lb_status lb2d_profile_step(lb2d_ctx* c, int32_t nsteps, double* kernel_ms, int32_t* count) {
  return guarded2([&] {
    need2(c);
    if (!kernel_ms || !count || nsteps <= 0) fail2(LB_EINVAL, "bad profile arguments");
    int n = 0;
    c->be->profile(nsteps, kernel_ms, &n);
    *count = n;
    c->step += nsteps;
  });
}

const char* lb2d_kernel_name(const lb2d_ctx* c, int32_t i) {
  static const char* names[2] = {"k2_lb", "k2_order"};
  if (!c || i < 0 || i > 1) return nullptr;
  return names[i];
}

void lb2d_destroy(lb2d_ctx* c) { delete c; }

const char* lb2d_last_error(void) { return g2_last_error.c_str(); }

}  // extern "C"

// Shared device helpers of libdpgmg: complex arithmetic on double2 / float2,
// device buffers, launch checks.  gfx950 only (wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dpgmg.h"

namespace dpg {

constexpr int kWave = 64;

// ---- complex helpers (x = real, y = imaginary) -----------------------------
template <typename T> struct cplx;
template <> struct cplx<double> { using type = double2; };
template <> struct cplx<float> { using type = float2; };
template <typename T> using cplx_t = typename cplx<T>::type;

__host__ __device__ inline double2 mk(double re, double im) { return make_double2(re, im); }
__host__ __device__ inline float2 mkf(float re, float im) { return make_float2(re, im); }

template <typename C> __host__ __device__ inline C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __host__ __device__ inline C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __host__ __device__ inline C cmul(C a, C b) {
  C r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
template <typename C> __host__ __device__ inline C cconj(C a) { C r; r.x = a.x; r.y = -a.y; return r; }
// c + a * b
template <typename C> __host__ __device__ inline C cfma(C a, C b, C c) {
  C r; r.x = c.x + a.x * b.x - a.y * b.y; r.y = c.y + a.x * b.y + a.y * b.x; return r;
}
// c + conj(a) * b
template <typename C> __host__ __device__ inline C cfmaconj(C a, C b, C c) {
  C r; r.x = c.x + a.x * b.x + a.y * b.y; r.y = c.y + a.x * b.y - a.y * b.x; return r;
}
template <typename C> __host__ __device__ inline C cscale(C a, decltype(a.x) s) { C r; r.x = a.x * s; r.y = a.y * s; return r; }

// ---- errors ------------------------------------------------------------------
struct DpgError : std::runtime_error {
  int code;
  DpgError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      throw ::dpg::DpgError(-7, std::string(#expr) + ": " + hipGetErrorString(_e));    \
  } while (0)

#define LAUNCH_OK() HIP_OK(hipGetLastError())

// ---- device buffer -------------------------------------------------------------
struct Budget {
  int64_t limit = 0, used = 0;
};

template <typename T> struct DevBuf {
  T *p = nullptr;
  int64_t n = 0;
  Budget *bud = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; bud = o.bud;
      o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      (void)hipFree(p);
      if (bud) bud->used -= n * (int64_t)sizeof(T);
    }
    p = nullptr;
    n = 0;
  }
  void alloc(int64_t count, Budget *b) {
    release();
    bud = b;
    if (count <= 0) return;
    int64_t bytes = count * (int64_t)sizeof(T);
    if (b && b->limit > 0 && b->used + bytes > b->limit)
      throw DpgError(-2, "device memory budget exceeded (" + std::to_string(b->used + bytes) +
                             " > " + std::to_string(b->limit) + " bytes)");
    hipError_t e = hipMalloc((void **)&p, bytes);
    if (e != hipSuccess) {
      p = nullptr;
      throw DpgError(-2, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    n = count;
    if (b) b->used += bytes;
  }
  // alloc unless the buffer already has exactly count elements (contents kept)
  void ensure(int64_t count, Budget *b) {
    if (!(p && n == count)) alloc(count, b);
  }
  void upload(const std::vector<T> &h, Budget *b, hipStream_t s) {
    alloc((int64_t)h.size(), b);
    if (n) HIP_OK(hipMemcpyAsync(p, h.data(), n * sizeof(T), hipMemcpyHostToDevice, s));
  }
  std::vector<T> download(hipStream_t s) const {
    std::vector<T> h(n);
    if (n) {
      HIP_OK(hipMemcpyAsync(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
    }
    return h;
  }
};

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// ---- kernel timing with HIP events (optional, per context) -------------------------
// Classes match the kernel symbols, so that averages can be compared with a
// rocprofv3 kernel trace of the same run.  `work` is algorithmic bytes for the
// HBM-bound apply kernels and algorithmic flops for the dense kernels.
constexpr int kProfClasses = 32;
struct Prof {
  bool on = false;
  struct Rec { int cls; hipEvent_t a, b; double work; };
  struct Stat { int64_t n = 0; double ms = 0.0, work = 0.0; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  Stat stat[kProfClasses];
  hipEvent_t ev() {
    if (pool.empty()) {
      hipEvent_t e;
      HIP_OK(hipEventCreate(&e));
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  void flush() {
    for (Rec &r : pending) {
      HIP_OK(hipEventSynchronize(r.b));
      float ms = 0.0f;
      HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
      stat[r.cls].n += 1;
      stat[r.cls].ms += ms;
      stat[r.cls].work += r.work;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    flush();
    for (auto &s : stat) s = Stat{};
  }
  ~Prof() {
    for (Rec &r : pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// Records one launch (or one batch call) of class cls between construction and
// destruction.
struct ProfScope {
  Prof *p;
  Prof::Rec rec{};
  hipStream_t s;
  ProfScope(Prof *p_, int cls, double work, hipStream_t s_) : p(p_), s(s_) {
    if (!p || !p->on) return;
    rec.cls = cls;
    rec.work = work;
    rec.a = p->ev();
    rec.b = p->ev();
    HIP_OK(hipEventRecord(rec.a, s));
  }
  ~ProfScope() {
    if (!p || !p->on) return;
    if (hipEventRecord(rec.b, s) == hipSuccess) p->pending.push_back(rec);
  }
};

}  // namespace dpg

#pragma once
// Per-thread sums of the kernels' terms: plain in double; in float, runs of
// plain float additions folded into a compensated (Kahan) sum. The value is
// handed on in double to the fixed-order FP64 reductions.
#include <hip/hip_runtime.h>

namespace kde {

template <typename T>
struct Acc;

// Terms a float sum adds in plain float before folding them into its
// compensated sum (a power of two).
constexpr int kRun = 8;

template <>
struct Acc<double> {
  double s;
  __device__ __forceinline__ void zero() { s = 0.0; }
  __device__ __forceinline__ void add(double v) { s += v; }
  __device__ __forceinline__ void fold() {}
  __device__ __forceinline__ double value() const { return s; }
};

// Float terms in a compensated float sum: kRun consecutive terms are added
// in plain float into r, and each such run is folded into a Kahan sum
// (s, c), c carrying the part of each addition that s lost, taken off the
// next run. For terms of one sign a thread's sum is within about
// (kRun + 1) units of float rounding (5.4e-7 relative for runs of 8) of
// the exact sum of its terms; for terms of both signs (a field times a
// kernel) the bound holds relative to the sum of their magnitudes. The
// value is handed on in double (s - c + r) to the fixed-order FP64
// reductions. Per term that is one float add and a fifth of a fold,
// against four operations and a register move for a Kahan step per term:
// on MI355X the float pair kernel at the paper-scale scan takes 17.2 ms
// instead of 19.9 ms, and its CV and sums move by less than 1e-9 relative
// (the error of the float terms themselves, about 7e-8, dominates).
template <>
struct Acc<float> {
  float s, c, r;
  __device__ __forceinline__ void zero() {
    s = 0.0f;
    c = 0.0f;
    r = 0.0f;
  }
  __device__ __forceinline__ void add(float v) { r += v; }
  __device__ __forceinline__ void fold() {
    const float y = r - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
    r = 0.0f;
  }
  __device__ __forceinline__ double value() const { return double(s) - double(c) + double(r); }
};

template <typename T, int BC>
__device__ __forceinline__ void fold_all(Acc<T> (&a1)[BC], Acc<T> (&a2)[BC]) {
#pragma unroll
  for (int bb = 0; bb < BC; ++bb) {
    a1[bb].fold();
    a2[bb].fold();
  }
}

}  // namespace kde

#pragma once
// Device pieces of the grid density, field gather and adaptive widths with
// von Mises kernels, shared by density.hip and the batched engine.
//
// Deposit (Sec. II.B Eq. kde; Sec. II.C step 3 for per-particle widths):
//   rho[g] = (1/N) sum_i w_i exp(-2 kappa_i s_ig^2),
//   s_ig = sin(pi (x_g - x_i) / L),  w_i = 1 / (L I0e(kappa_i)).
// The grid is small (M <= 4096) and every particle touches every node, so
// a workgroup owns the whole grid for one contiguous chunk of particles:
// the chunk is staged in LDS (half-angle vector, exponent scale, weight)
// and read by all lanes at the same address (broadcast), each thread
// accumulating its own node(s). Per-chunk grids go to fixed slots and are
// summed in a fixed order. The cost is one exponential per (particle, node):
// transcendental-bound, not HBM-bound, at every grid size used here.
//
// Gather (field interpolation of Sec. III.A with the same kernels):
//   out[i] = (L/M) w_i sum_g F_g exp(-2 kappa_i s_ig^2),
// one thread per particle with the node table in LDS.
//
// Adaptive widths (Sec. II.C, Eq. adaptive_width): the pilot grid is
// interpolated linearly at each particle, its logarithms are averaged in
// double (fixed-order reduction), and kappa_i = kappa* exp(2 alpha (log f_i
// - log g)) is written per particle.
#include <cfloat>

#include "dev_sum.hpp"
#include "device_bessel.hpp"
#include "kde_internal.hpp"

namespace kde {


template <typename T>
struct Flt;
// ex(a, tab): exp of a kernel exponent a <= 0 (natural in double, with the
// exponential's table `tab` in LDS; base 2 in float, where tab is unused).
// ex_in(a, tab): the same for an exponent known to lie in the table
// exponential's own domain (a >= kExpTableMin), without the clamp.
constexpr double kExpTableMin = -17592186044416.0;  // -2^44
template <>
struct Flt<double> {
  static __device__ __forceinline__ double ex(double a, const double* tab) { return exp_nonpos_table_any(a, tab); }
  static __device__ __forceinline__ double ex_in(double a, const double* tab) { return exp_nonpos_table(a, tab); }
  static constexpr double unit = 1.0;
  static constexpr double tiny = DBL_MIN;
};
template <>
struct Flt<float> {
  static __device__ __forceinline__ float ex(float a, const double*) { return __builtin_amdgcn_exp2f(a); }
  static __device__ __forceinline__ float ex_in(float a, const double*) { return __builtin_amdgcn_exp2f(a); }
  static constexpr double unit = 1.4426950408889634;
  static constexpr float tiny = FLT_MIN;
};

template <typename T>
struct SumOf;
template <>
struct SumOf<double> {
  double s = 0.0;
  __device__ __forceinline__ void zero() { s = 0.0; }
  __device__ __forceinline__ void add(double v) { s += v; }
  __device__ __forceinline__ void fold() {}
  __device__ __forceinline__ double value() const { return s; }
};
// Float terms in a compensated float sum (Kahan, one step per term); the
// value is handed on in double for the FP64 reductions. Two registers per
// sum against the three of Acc<float>, for loops that hold many sums.
template <>
struct SumOf<float> {
  float s = 0.0f, c = 0.0f;
  __device__ __forceinline__ void zero() { s = c = 0.0f; }
  __device__ __forceinline__ void add(float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ __forceinline__ void fold() {}
  __device__ __forceinline__ double value() const { return double(s) - double(c); }
};

constexpr int kDepMaxChunk = 512;

// Geometry of a (node, particle) pair. Both forms give s = sin(pi (x_g - x_i) / L):
//   double: global half-angle vectors, s = sin(pi g/M) a_i - cos(pi g/M) b_i with
//           (a_i, b_i) = (cos(pi x_i/L), sin(pi x_i/L));
//   float : node-relative, with the particle at v = x_i M / L split as v = g0 + d
//           (g0 the nearest node, |d| <= 1/2) and beta = pi d / M:
//           s = sin(pi k/M) cos(beta) - cos(pi k/M) sin(beta), k = (g - g0) mod M,
//           from a table over k. Near nodes have small k and small beta, so s
//           keeps float relative accuracy where the kernel is largest (the
//           global form would carry the absolute rounding of a_i, b_i).
// In double that absolute rounding (about one unit) matters only for a sharp
// kernel close to a node: through the exponent -2 kappa s^2 it is a term
// error up to about 6 sqrt(372 kappa) units. So for a particle with
// kappa_i > kNearKappa, a node with |s| < 2^-8 takes s = sin(pi d / L) from
// the exact difference d = x_g - w_i (node x_g = g (L/M), w_i the wrapped
// position; the periodic image by an exact shift of the larger one), by
// its Taylor series.
template <typename T>
struct PGeo;
template <>
struct PGeo<double> {
  double a, b, w;
};

constexpr double kNearKappa = 50.0;
constexpr double kNearS2 = 0.00390625;  // 2^-8

// s for node g (position g dx, dx = L / M) and particle position w in
// [0, L) when |s0| (the table form) is below 2^-8; s0 otherwise. Only s^2
// is used. The node position must be the rounded product that defines the
// grid, so the product and the difference are not fused into one FMA.
__device__ __forceinline__ double near_node_s(double s0, int g, double dx, double w, double L) {
#pragma clang fp contract(off)
  if (!(fabs(s0) < kNearS2)) return s0;
  const double xg = double(g) * dx;
  double d = xg - w;
  d = (d > 0.5 * L) ? (xg - L) - w : ((d < -0.5 * L) ? xg - (w - L) : d);
  const double ph = d * (3.141592653589793 / L);
  const double p2 = ph * ph;
  return ph * fma(p2, fma(p2, fma(p2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), 1.0);
}
template <>
struct PGeo<float> {
  int g0;
  float cb, sb;
};

// The LDS node table: sin and cos of pi k / M side by side, so that one
// read (8 or 16 bytes) gives both.
template <typename T>
struct __align__(2 * sizeof(T)) SinCos {
  T s, c;
};

__device__ __forceinline__ void make_geo(double xw, double L, int M, PGeo<double>& p) {
  double sp, cp;
  sincospi(xw / L, &sp, &cp);
  p.a = cp;
  p.b = sp;
  p.w = xw;
}

__device__ __forceinline__ void make_geo(double xw, double L, int M, PGeo<float>& p) {
  const double v = xw * (double(M) / L);
  double g0 = floor(v + 0.5);
  const double d = v - g0;
  if (g0 >= double(M)) g0 -= double(M);
  double sb, cb;
  sincospi(d / double(M), &sb, &cb);
  p.g0 = int(g0);
  p.cb = float(cb);
  p.sb = float(sb);
}

// A deposit chunk's particle as the node loops read it: geometry and the
// exponent factor in one record (16 bytes in float, one LDS read), the
// weight apart (read only with per-particle widths).
template <typename T>
struct __align__(16) DepRec {
  PGeo<T> g;
  T A;
};

template <typename T, bool PER>
__device__ __forceinline__ void particle_terms(const T* __restrict__ x, const T* __restrict__ kap, double kappa_g,
                                               int64_t i, double L, int M, DepRec<T>& r, T& w) {
  const double xi = double(x[i]);
  const double xw = xi - L * floor(xi / L);
  make_geo(xw, L, M, r.g);
  const double k = PER ? double(kap[i]) : kappa_g;
  r.A = T(-2.0 * k * Flt<T>::unit);
  w = PER ? T(1.0 / (L * i0e_f64(k))) : T(1);
}

// s for node g of a particle; `t` holds sin/cos(pi g/M) (double form,
// indexed by g) or sin/cos(pi k/M) (float form, indexed by k = g - g0 mod M).
__device__ __forceinline__ double node_s(const PGeo<double>& p, int g, int M, const SinCos<double>* t) {
  const SinCos<double> e = t[g];
  return e.s * p.a - e.c * p.b;
}
__device__ __forceinline__ float node_s(const PGeo<float>& p, int g, int M, const SinCos<float>* t) {
  int k = g - p.g0;
  k += (k < 0) ? M : 0;
  const SinCos<float> e = t[k];
  return e.s * p.cb - e.c * p.sb;
}

// Shared memory of one deposit chunk (the node table is separate: dynamic
// LDS of M SinCos<T>).
template <typename T>
struct DepSmem {
  DepRec<T> rec[kDepMaxChunk];
  T pw[kDepMaxChunk];
  double red[kBlock];
  double etab[std::is_same<T, double>::value ? 256 : 1];  // exponential table (double form)
};

// Stage the double exponential's table (KDE_EXP_TABLE) in LDS; no-op in float.
template <typename T>
__device__ __forceinline__ void exp_table_fill(double* etab) {
  if constexpr (std::is_same<T, double>::value) {
    constexpr double src[256] = KDE_EXP_TABLE;
    for (int k = threadIdx.x; k < 256; k += kBlock) etab[k] = src[k];
  }
}

// Fill the node table: t[k] = (sin(pi k/M), cos(pi k/M)).
template <typename T>
__device__ __forceinline__ void node_table(int M, SinCos<T>* t) {
  for (int k = threadIdx.x; k < M; k += kBlock) {
    double sv, cv;
    sincospi(double(k) / double(M), &sv, &cv);
    t[k] = SinCos<T>{T(sv), T(cv)};
  }
}

// One deposit chunk: particles [lo, lo + cnt) onto all M nodes, written to
// out[M] (the chunk's partial grid, unnormalised by N). The node table must
// be filled and visible. Non-finite positions and per-particle
// concentrations that are non-finite or negative are noted in `status`
// (may be null). Ends with a barrier.
// M <= 256: S = 256 / M sub-streams share a node, thread t -> node t % M,
//           sub-stream t / M (threads beyond S*M idle);
// M  > 256: thread t -> nodes t, t + 256, ... (G per thread).
// Sum over the chunk's particles p = sub, sub + S, ... at node g. NEAR: the
// chunk holds a sharp kernel (kappa > kNearKappa), whose near nodes take the
// exact separation; CLAMP: it holds an exponent factor beyond the table
// exponential's domain, so exponents are clamped first. Chunks without
// either (every chunk of ordinary widths) run the plain loop.
template <typename T, bool PER, bool NEAR, bool CLAMP>
__device__ __forceinline__ T dep_term(int g, int p, int M, double L, const SinCos<T>* tab, const DepSmem<T>& sm) {
  const DepRec<T> r = sm.rec[p];
  T s = node_s(r.g, g, M, tab);
  if constexpr (NEAR) {
    if (r.A < T(-2.0 * kNearKappa)) s = near_node_s(s, g, L / double(M), r.g.w, L);
  }
  const T e = CLAMP ? Flt<T>::ex(r.A * (s * s), sm.etab) : Flt<T>::ex_in(r.A * (s * s), sm.etab);
  return PER ? sm.pw[p] * e : e;
}

// The particles in groups of eight without a bound test inside a group, so
// that their LDS reads (the record, then the table entry it points to) are
// in flight together, then the rest one by one. The sum's run folds fall
// after every kRun terms either way, so the result is that of the plain
// loop. (Groups of four: float deposit 9 % slower, double 3 %.)
template <typename T, bool PER, bool NEAR, bool CLAMP>
__device__ __forceinline__ double dep_node_sum(int g, int sub, int S, int cnt, int M, double L,
                                               const SinCos<T>* tab, const DepSmem<T>& sm) {
  static_assert(kRun % 8 == 0, "a run holds whole groups");
  Acc<T> acc;
  acc.zero();
  int p = sub, q = 0;
  for (; p + 7 * S < cnt; p += 8 * S, q += 8) {
    T e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = dep_term<T, PER, NEAR, CLAMP>(g, p + u * S, M, L, tab, sm);
#pragma unroll
    for (int u = 0; u < 8; ++u) acc.add(e[u]);
    if (((q + 8) & (kRun - 1)) == 0) acc.fold();
  }
  for (; p < cnt; p += S, ++q) {
    acc.add(dep_term<T, PER, NEAR, CLAMP>(g, p, M, L, tab, sm));
    if ((q & (kRun - 1)) == kRun - 1) acc.fold();
  }
  return acc.value();
}

// The same for G nodes per thread (g = tid + k kBlock), all particles.
template <typename T, bool PER, int G, bool NEAR, bool CLAMP, typename Sum>
__device__ __forceinline__ void dep_node_sums(int tid, int cnt, int M, double L, const SinCos<T>* tab,
                                              const DepSmem<T>& sm, Sum (&acc)[G]) {
  const double dx = L / double(M);
  for (int p = 0; p < cnt; ++p) {
    const DepRec<T> r = sm.rec[p];
    const T w = PER ? sm.pw[p] : T(1);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int g = tid + k * kBlock;
      if (g < M) {
        T s = node_s(r.g, g, M, tab);
        if constexpr (NEAR) {
          if (r.A < T(-2.0 * kNearKappa)) s = near_node_s(s, g, dx, r.g.w, L);
        }
        const T e = CLAMP ? Flt<T>::ex(r.A * (s * s), sm.etab) : Flt<T>::ex_in(r.A * (s * s), sm.etab);
        acc[k].add(PER ? w * e : e);
      }
    }
    if ((p & (kRun - 1)) == kRun - 1) {
#pragma unroll
      for (int k = 0; k < G; ++k) acc[k].fold();
    }
  }
}

template <typename T, bool PER, int G>
__device__ __forceinline__ void deposit_block(const T* __restrict__ x, const T* __restrict__ kap, double kappa_g,
                                              int M, double L, int64_t lo, int cnt, double* __restrict__ out,
                                              const SinCos<T>* tab, DepSmem<T>& sm, uint32_t* status) {
  const int tid = threadIdx.x;
  int sharp = 0, huge = 0;
  for (int k = tid; k < cnt; k += kBlock) {
    const double xi = double(x[lo + k]);
    const double ki = PER ? double(kap[lo + k]) : 0.0;
    note_numeric(status, !isfinite(xi), PER && !(isfinite(ki) && ki >= 0.0));
    particle_terms<T, PER>(x, kap, kappa_g, lo + k, L, M, sm.rec[k], sm.pw[k]);
    if (std::is_same<T, double>::value && sm.rec[k].A < T(-2.0 * kNearKappa)) sharp = 1;
    if (std::is_same<T, double>::value && !(sm.rec[k].A >= T(kExpTableMin))) huge = 1;
  }
  exp_table_fill<T>(sm.etab);
  // one barrier that also tells every thread whether the chunk holds a
  // sharp kernel or an exponent factor beyond the table's domain
  const int flags = __syncthreads_or(sharp | (huge << 1)) ? (__syncthreads_or(huge) ? 3 : 1) : 0;
  if (M <= kBlock) {
    const int S = kBlock / M;
    const int g = tid % M, sub = tid / M;
    double tot = 0.0;
    if (sub < S) {
      if constexpr (std::is_same<T, double>::value) {
        if (flags == 0)
          tot = dep_node_sum<T, PER, false, false>(g, sub, S, cnt, M, L, tab, sm);
        else if (flags == 1)
          tot = dep_node_sum<T, PER, true, false>(g, sub, S, cnt, M, L, tab, sm);
        else
          tot = dep_node_sum<T, PER, true, true>(g, sub, S, cnt, M, L, tab, sm);
      } else {
        tot = dep_node_sum<T, PER, false, false>(g, sub, S, cnt, M, L, tab, sm);
      }
    }
    sm.red[tid] = tot;
    __syncthreads();
    if (tid < M) {
      double v = 0.0;
      for (int q = 0; q < S; ++q) v += sm.red[q * M + tid];
      out[tid] = PER ? v : v * (1.0 / (L * i0e_f64(kappa_g)));
    }
  } else {
    // runs folded into Kahan sums, or for 16 nodes per thread a Kahan step
    // per term (the runs' third register per sum would cost two waves)
    using Sum = typename std::conditional<(G <= 8), Acc<T>, SumOf<T>>::type;
    Sum acc[G];
#pragma unroll
    for (int k = 0; k < G; ++k) acc[k].zero();
    if constexpr (std::is_same<T, double>::value) {
      if (flags == 0)
        dep_node_sums<T, PER, G, false, false>(tid, cnt, M, L, tab, sm, acc);
      else if (flags == 1)
        dep_node_sums<T, PER, G, true, false>(tid, cnt, M, L, tab, sm, acc);
      else
        dep_node_sums<T, PER, G, true, true>(tid, cnt, M, L, tab, sm, acc);
    } else {
      dep_node_sums<T, PER, G, false, false>(tid, cnt, M, L, tab, sm, acc);
    }
    const double scale = PER ? 1.0 : 1.0 / (L * i0e_f64(kappa_g));
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int g = tid + k * kBlock;
      if (g < M) out[g] = acc[k].value() * scale;
    }
  }
  __syncthreads();
}

// Particles per deposit chunk for N particles (the chunk grid is what the
// fixed-order reduction sums, so every user must cut the same chunks).
__host__ __device__ inline int deposit_chunk(int64_t n) {
  int64_t c = (n + 2047) / 2048;
  if (c < 64) c = 64;
  if (c > kDepMaxChunk) c = kDepMaxChunk;
  return int(c);
}

// Pilot density at a particle: periodic linear interpolation between the
// two nodes around it, floored at the smallest normal number of T. A
// non-finite position yields NaN (and is not counted as floored). The
// arithmetic is double in both precisions: this step reads and writes a
// few bytes per particle and is bound by memory traffic, not arithmetic.
template <typename T>
__device__ __forceinline__ double pilot_at(T xv, double L, int M, const double* __restrict__ pilot, bool& floored) {
  const double xi = double(xv);
  floored = false;
  if (!isfinite(xi)) return NAN;
  const double xw = xi - L * floor(xi / L);
  double u = xw * (double(M) / L);
  if (!(u >= 0.0)) u = 0.0;
  int j = int(floor(u));
  double t = u - double(j);
  if (j >= M) {  // x rounded up to L: the node at 0
    j = 0;
    t = 0.0;
  }
  const int j1 = (j + 1 == M) ? 0 : j + 1;
  double f = (1.0 - t) * pilot[j] + t * pilot[j1];
  if (f < double(Flt<T>::tiny)) {  // NaN stays NaN
    floored = true;
    f = double(Flt<T>::tiny);
  }
  return f;
}

// Block b of the log-sum pass: particles [256 b, 256 b + 256); writes
// (sum of log f, floored count) to out[0..2). `r0`, `r1`: kBlock/64 doubles
// of LDS each. Non-finite positions are noted in `status` (may be null).
template <typename T>
__device__ __forceinline__ void adapt_logsum_block(const T* __restrict__ x, int64_t n, int M, double L,
                                                   const double* __restrict__ pilot, int64_t b,
                                                   double* __restrict__ out, double* r0, double* r1,
                                                   uint32_t* status) {
  const int64_t i = b * kBlock + threadIdx.x;
  double lsum = 0.0, fl = 0.0;
  if (i < n) {
    bool floored;
    const T xv = x[i];
    lsum = log(pilot_at<T>(xv, L, M, pilot, floored));
    fl = floored ? 1.0 : 0.0;
    note_numeric(status, !isfinite(double(xv)), false);
  }
  lsum = wave_sum(lsum);
  fl = wave_sum(fl);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    r0[wave] = lsum;
    r1[wave] = fl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      a += r0[w];
      c += r1[w];
    }
    out[0] = a;
    out[1] = c;
  }
  __syncthreads();
}

// Block b of the width pass: kappa_i = kappa* exp(2 alpha (log f_i - log g))
// with log g = sums[0] / n.
template <typename T>
__device__ __forceinline__ void adapt_apply_block(const T* __restrict__ x, int64_t n, int M, double L,
                                                  const double* __restrict__ pilot, double kappa_star, double alpha,
                                                  const double* __restrict__ sums, int64_t b, T* __restrict__ kout) {
  const double log_g = sums[0] / double(n);
  const int64_t i = b * kBlock + threadIdx.x;
  if (i < n) {
    bool floored;
    const double lf = log(pilot_at<T>(x[i], L, M, pilot, floored));
    kout[i] = T(kappa_star * exp(2.0 * alpha * (lf - log_g)));
  }
}

}  // namespace kde

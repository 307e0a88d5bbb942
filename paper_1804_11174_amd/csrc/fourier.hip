// Fourier-moment route of the von Mises CV objective (Sec. II.B, Eq.
// cv_def), its Newton refinement in concentration, and the exact pilot at
// the particles for the adaptive widths (Sec. II.C); see kde.h.
//
// On the circle the kernel's Fourier coefficients are rho_m = I_m/I_0, and
// a double sum over pairs of any function of the separation collapses onto
// the sample's moments S_m = sum_j exp(i m theta_j):
//   sum_{i,j} cos(m (theta_i - theta_j)) = |S_m|^2 = P_m.
// So the two sums of the objective cost O(N M) for the moments plus O(M)
// per concentration, instead of O(N^2) per concentration.
//
// Kernels:
//   moments_kernel   -- block (particle chunk, 16 consecutive m): per
//                       particle the phase exp(i m0 theta) with the product
//                       m0 * (x/L) reduced mod 1 exactly (its rounding error
//                       recovered by an FMA), then 15 rotations by
//                       exp(i theta); per-m sums reduced in the workgroup in
//                       a fixed order into the chunk's slot; the chunks are
//                       summed by the shared fixed-order column sum.
//   series_kernel    -- one workgroup per concentration: the backward
//                       recurrence of the ratios r_m = I_m/I_{m-1},
//                       r_m = kappa / (2 m + kappa r_{m+1}) (stable downwards,
//                       started where the neglected tail has decayed below
//                       e^-40), as a scan of Mobius maps over the workgroup
//                       (bessel_series), the ratios multiplied up to rho_m by
//                       a prefix scan; then all threads form the series in a
//                       fixed order.
//   newton_start_kernel -- three workgroups side by side: the objective
//                       and its derivatives at the two ends of the bracket
//                       around the scan's first minimum and at the first
//                       iterate (the vertex of the parabola through the three
//                       grid values there).
//   newton_kernel    -- one workgroup: from those, Newton's method on
//                       u = log(kappa) with bisection as the safeguard.
//                       The derivatives come from the same
//                       recurrence differentiated in kappa:
//                         r'_k  = r_k^2 (2k / kappa^2 - r'_{k+1}),
//                         r''_k = 2 r'_k^2 / r_k - r_k^2 (4k / kappa^3 + r''_{k+1}),
//                         rho'_m = rho_m D_m, D_m = sum_{k<=m} r'_k / r_k,
//                         rho''_m = rho_m (D_m^2 + sum_{k<=m} (r''_k / r_k - (r'_k / r_k)^2)).
//                       Each r'_k is positive (I_k/I_{k-1} grows with kappa),
//                       so D_m is a sum of positive terms; the textbook form
//                       rho_{m+1} + (m/kappa) rho_m - rho_1 rho_m is the same
//                       value computed as a difference of O(rho_m) terms,
//                       which loses 2 kappa^2/m^2 rounding units at small m.
//   pilot kernels    -- weights w_m = rho_m(kappa*) S_m (one workgroup), then
//                       one thread per particle sums Re(conj(w_m) e^{i m
//                       theta}) over m in runs of 64 rotations, each run
//                       started from an exactly reduced phase; logs of the
//                       floored pilot go to a workspace array, their sum
//                       through the fixed-order column sums, then the widths.
// Every reduction has a fixed order: results are deterministic.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <limits>

#include "dev_layout.hpp"
#include "kde_internal.hpp"

namespace kde {

namespace {

constexpr double kFourierTail = 1e-18;  // rho_M below this ends the series
constexpr int kMomM = 16;               // consecutive m per moment block
constexpr int kMomChunks = 64;          // moment partials' budget: kMomChunks x kMaxOrder (re, im) pairs
constexpr int64_t kMomBlocks = 4096;    // workgroups a moment launch aims for
constexpr int kMomPerThread = 8;        // fewest particles per thread of a moment workgroup
constexpr int kPilotRun = 64;           // rotations between exact phase restarts
constexpr int kMaxNewton = 100;
constexpr int kStartEvals = 3;          // refine: bracket ends and first iterate, evaluated side by side

// Concentrations with their series orders (fourier_order of each; the
// order grows with kappa, so a bracket's upper end bounds it inside).
struct FKappas {
  double k[KDE_MAX_KAPPAS];
  int order[KDE_MAX_KAPPAS];
};

// Smallest m at which the product of Amos's upper bounds
//   I_nu(k) / I_{nu-1}(k) <= k / (nu - 1/2 + sqrt((nu - 1/2)^2 + k^2))
// falls below kFourierTail: rho_m(kmax) is below it from there on, and
// rho_m grows with kappa, so the series for every kappa <= kmax is cut there.
int fourier_order(double kmax) {
  if (!(kmax > 0.0)) return 1;
  const double lim = std::log(kFourierTail);
  double lg = 0.0;
  for (int m = 1;; ++m) {
    const double nu = double(m) - 0.5;
    lg += std::log(kmax / (nu + std::sqrt(nu * nu + kmax * kmax)));
    if (lg < lim) return m;
  }
}

const int kMaxOrder = fourier_order(KDE_MAX_FOURIER_KAPPA);

// Moment partials' budget for N particles, in units of kMaxOrder (re, im)
// pairs: one per kBlock x kMomPerThread particles, at least 1, at most
// kMomChunks.
int64_t moment_budget(int64_t n) {
  return std::max<int64_t>(1, std::min<int64_t>(kMomChunks, n / (int64_t(kBlock) * kMomPerThread)));
}

// Particle chunks of the moments of N particles to order M: about
// kMomBlocks workgroups over the ceil(M / kMomM) mode groups (a low order
// still fills the GPU), at least kMomPerThread particles per thread (so the
// workgroup's fixed-order reduction of 2 kMomM sums stays a small part of
// its work), and chunks x M within the partials' budget.
int64_t moment_chunks(int64_t n, int M) {
  int64_t c = ceil_div(kMomBlocks, ceil_div(M, kMomM));
  c = std::min<int64_t>(c, n / (int64_t(kBlock) * kMomPerThread));
  c = std::min<int64_t>(c, moment_budget(n) * kMaxOrder / M);
  return std::max<int64_t>(1, c);
}

struct FourierBufs {
  double* partials;  // [chunks][2 M]
  double* colsum;    // column-sum scratch
  double* S;         // [2 M] moments (re, im)
  double* rho;       // [B][M + 1] (scan) or [3][M + 1] (refine, pilot)
  double* cvgrid;    // [B]
  double* start;     // refine: (cv, g, g') at the bracket ends and the first iterate, then that iterate's u
  double* w;         // [2 M] pilot weights
  double* lf;        // [N] log pilot
  double* bpart;     // [blocks][2]
  double* colsum2;
  double* sums2;     // [2]
};

FourierBufs carve_fourier(Carver& c, int op, int64_t n, int B) {
  FourierBufs b{};
  const int M = kMaxOrder;
  // any order's chunks x 2 M partials fit the budget; its column-sum
  // scratch, ceil(chunks / R) x 2 M for R rows per level-1 block, is at
  // most (chunks x 2 M) / R + 2 M
  const int64_t budget = moment_budget(n);
  b.partials = c.take<double>(size_t(budget) * 2 * M);
  b.colsum = c.take<double>((column_sum_scratch(budget * M, 2) + column_sum_scratch(1, 2 * M)) / sizeof(double) + 1);
  b.S = c.take<double>(size_t(2) * M);
  const int slots = (op == KDE_OP_CV_FOURIER) ? B : (op == KDE_OP_CV_REFINE ? std::max(B, 3 * kStartEvals) : 1);
  b.rho = c.take<double>(size_t(slots) * (M + 1));
  if (op == KDE_OP_CV_REFINE) {
    b.cvgrid = c.take<double>(size_t(B));
    b.start = c.take<double>(3 * kStartEvals + 1);
  }
  if (op == KDE_OP_ADAPT_EXACT) {
    const int64_t blocks = ceil_div(n, kBlock);
    b.w = c.take<double>(size_t(2) * M);
    b.lf = c.take<double>(size_t(n));
    b.bpart = c.take<double>(size_t(blocks) * 2);
    b.colsum2 = c.take<double>(column_sum_scratch(blocks, 2) / sizeof(double) + 1);
    b.sums2 = c.take<double>(2);
  }
  return b;
}

// Phase exp(i 2 pi m f) for f in [0, 1]: m f reduced mod 1 with its
// rounding error recovered, so the angle is exact to a few units of f's
// last place times m.
__device__ __forceinline__ void phase(int m, double f, double& c, double& s) {
  const double t = double(m) * f;
  const double e = fma(double(m), f, -t);
  const double fr = (t - floor(t)) + e;
  sincospi(2.0 * fr, &s, &c);
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) t += red[w];
  return t;
}

// Six workgroup sums at once, each in block_sum's order (wave sums, then
// the waves in order), with one exchange through LDS.
__device__ __forceinline__ void block_sum6(double (&v)[6], double (*red)[6]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) red[wave][k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += red[w][k];
    v[k] = t;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) moments_kernel(const T* __restrict__ x, int64_t n, double L, int M,
                                                        int64_t per_chunk, double* __restrict__ partials,
                                                        uint32_t* status) {
  __shared__ double red[kBlock / 64][2 * kMomM];
  const int64_t ch = blockIdx.x;
  const int m0 = 1 + int(blockIdx.y) * kMomM;
  double re[kMomM], im[kMomM];
#pragma unroll
  for (int k = 0; k < kMomM; ++k) re[k] = im[k] = 0.0;
  const int64_t lo = ch * per_chunk, hi = min(n, lo + per_chunk);
  uint32_t* const st = blockIdx.y == 0 ? status : nullptr;  // one column of blocks notes the positions
  for (int64_t j = lo + threadIdx.x; j < hi; j += kBlock) {
    note_numeric(st, !isfinite(double(x[j])), false);
    const double f = wrap_d(double(x[j]), L) / L;
    double c, s, c1, s1;
    phase(m0, f, c, s);
    sincospi(2.0 * f, &s1, &c1);
#pragma unroll
    for (int k = 0; k < kMomM; ++k) {
      re[k] += c;
      im[k] += s;
      const double nc = c * c1 - s * s1;
      s = fma(s, c1, c * s1);
      c = nc;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kMomM; ++k) {
    const double a = wave_sum(re[k]);
    const double b = wave_sum(im[k]);
    if (lane == 0) {
      red[wave][2 * k] = a;
      red[wave][2 * k + 1] = b;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * kMomM) {
    const int m = m0 + (t >> 1);
    if (m <= M) {
      double v = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) v += red[w][t];
      partials[ch * 2 * int64_t(M) + 2 * (m - 1) + (t & 1)] = v;
    }
  }
}

// Shared memory of the workgroup-wide series (double-buffered scans).
struct SeriesSmem {
  double mat[2][kBlock][4];  // Mobius matrices (row-major 2x2)
  double aff[2][kBlock][2];  // affine maps x -> a + b x
  double pre[2][kBlock][3];  // segment totals (product, sum, sum)
  double red[kBlock / 64];
  double red6[kBlock / 64][6];
};

__device__ __forceinline__ void mat_mul_norm(const double* a, const double* b, double* c) {
  double c0 = fma(a[0], b[0], a[1] * b[2]);
  double c1 = fma(a[0], b[1], a[1] * b[3]);
  double c2 = fma(a[2], b[0], a[3] * b[2]);
  double c3 = fma(a[2], b[1], a[3] * b[3]);
  const double mx = fmax(fmax(fabs(c0), fabs(c1)), fmax(fabs(c2), fabs(c3)));
  const int e = (mx > 0.0) ? ilogb(mx) : 0;  // exact rescaling by a power of two
  c[0] = ldexp(c0, -e);
  c[1] = ldexp(c1, -e);
  c[2] = ldexp(c2, -e);
  c[3] = ldexp(c3, -e);
}

// rho_m(kappa) for m = 0..M into rho[]; with DER also rho'_m, rho''_m into
// d1[], d2[] (kappa > 0 then). All threads of the workgroup take part.
//
// The backward recurrence r_m = kappa / (2m + kappa r_{m+1}), r_{Ms+1} = 0,
// applies the Mobius maps with matrices [[0, kappa], [kappa, 2m]] to the
// homogeneous vector (0, 1): thread t composes the maps of its segment of m
// (non-negative matrices, rescaled by powers of two, so no cancellation), a
// suffix scan over the threads gives every segment the vector entering it
// from above, and each thread walks its segment. r'_m and r''_m obey affine
// recurrences in r'_{m+1} and r''_{m+1} (coefficients from r_m, r'_m), done
// the same way with affine maps; rho_m, D_m and E_m are prefix products and
// sums over m (a combined prefix scan). The composition is a reassociation
// of the recurrence; its rounding grows with the tree depth instead of the
// length of the chain.
template <bool DER>
__device__ void bessel_series(double kappa, int M, double* __restrict__ rho, double* __restrict__ d1,
                              double* __restrict__ d2, SeriesSmem& sm) {
  const int t = threadIdx.x;
  const int Ms = int(ceil(sqrt(double(M) * double(M) + 40.0 * kappa))) + 16;
  const int len = (Ms + kBlock - 1) / kBlock;
  const int lo = 1 + t * len, hi = min(Ms, (t + 1) * len);  // empty when lo > hi
  const double ik2 = DER ? 1.0 / (kappa * kappa) : 0.0;
  const double ik3 = DER ? ik2 / kappa : 0.0;

  // 1. Mobius composition of the segment, suffix scan, then the walk.
  double P[4] = {1.0, 0.0, 0.0, 1.0};
  for (int m = hi; m >= lo; --m) {
    const double Mm[4] = {0.0, kappa, kappa, 2.0 * double(m)};
    double Q[4];
    mat_mul_norm(Mm, P, Q);
    P[0] = Q[0]; P[1] = Q[1]; P[2] = Q[2]; P[3] = Q[3];
  }
  int cur = 0;
  for (int k = 0; k < 4; ++k) sm.mat[0][t][k] = P[k];
  __syncthreads();
  for (int d = 1; d < kBlock; d <<= 1) {
    if (t + d < kBlock)
      mat_mul_norm(sm.mat[cur][t], sm.mat[cur][t + d], sm.mat[cur ^ 1][t]);
    else
      for (int k = 0; k < 4; ++k) sm.mat[cur ^ 1][t][k] = sm.mat[cur][t][k];
    __syncthreads();
    cur ^= 1;
  }
  const double r_top = (t + 1 < kBlock) ? sm.mat[cur][t + 1][1] / sm.mat[cur][t + 1][3] : 0.0;
  {
    double r = r_top;
    for (int m = hi; m >= lo; --m) {
      r = kappa / (2.0 * double(m) + kappa * r);
      if (m <= M) rho[m] = r;
    }
  }
  double rp_top = 0.0, rpp_top = 0.0;
  if (DER) {
    // 2. r'_m = 2m r_m^2 / kappa^2 - r_m^2 r'_{m+1}.
    double a = 0.0, b = 1.0;
    {
      double r = r_top;
      for (int m = hi; m >= lo; --m) {
        r = kappa / (2.0 * double(m) + kappa * r);
        const double r2 = r * r;
        a = fma(-r2, a, 2.0 * double(m) * r2 * ik2);
        b = -r2 * b;
      }
    }
    __syncthreads();  // the matrix scan's reads are done
    sm.aff[0][t][0] = a;
    sm.aff[0][t][1] = b;
    __syncthreads();
    cur = 0;
    for (int d = 1; d < kBlock; d <<= 1) {
      if (t + d < kBlock) {
        sm.aff[cur ^ 1][t][0] = fma(sm.aff[cur][t][1], sm.aff[cur][t + d][0], sm.aff[cur][t][0]);
        sm.aff[cur ^ 1][t][1] = sm.aff[cur][t][1] * sm.aff[cur][t + d][1];
      } else {
        sm.aff[cur ^ 1][t][0] = sm.aff[cur][t][0];
        sm.aff[cur ^ 1][t][1] = sm.aff[cur][t][1];
      }
      __syncthreads();
      cur ^= 1;
    }
    rp_top = (t + 1 < kBlock) ? sm.aff[cur][t + 1][0] : 0.0;
    // 3. r''_m = 2 r'_m^2 / r_m - r_m^2 (4m / kappa^3 + r''_{m+1}).
    a = 0.0;
    b = 1.0;
    {
      double r = r_top, rp = rp_top;
      for (int m = hi; m >= lo; --m) {
        r = kappa / (2.0 * double(m) + kappa * r);
        const double r2 = r * r;
        rp = r2 * (2.0 * double(m) * ik2 - rp);
        const double A = 2.0 * rp * rp / r - 4.0 * double(m) * r2 * ik3;
        a = fma(-r2, a, A);
        b = -r2 * b;
        if (m <= M) d1[m] = rp;
      }
    }
    __syncthreads();
    sm.aff[0][t][0] = a;
    sm.aff[0][t][1] = b;
    __syncthreads();
    cur = 0;
    for (int d = 1; d < kBlock; d <<= 1) {
      if (t + d < kBlock) {
        sm.aff[cur ^ 1][t][0] = fma(sm.aff[cur][t][1], sm.aff[cur][t + d][0], sm.aff[cur][t][0]);
        sm.aff[cur ^ 1][t][1] = sm.aff[cur][t][1] * sm.aff[cur][t + d][1];
      } else {
        sm.aff[cur ^ 1][t][0] = sm.aff[cur][t][0];
        sm.aff[cur ^ 1][t][1] = sm.aff[cur][t][1];
      }
      __syncthreads();
      cur ^= 1;
    }
    rpp_top = (t + 1 < kBlock) ? sm.aff[cur][t + 1][0] : 0.0;
    {
      double r = r_top, rp = rp_top, rpp = rpp_top;
      for (int m = hi; m >= lo; --m) {
        r = kappa / (2.0 * double(m) + kappa * r);
        const double r2 = r * r;
        rp = r2 * (2.0 * double(m) * ik2 - rp);
        rpp = 2.0 * rp * rp / r - r2 * (4.0 * double(m) * ik3 + rpp);
        if (m <= M) d2[m] = rpp;
      }
    }
  }
  // 4. Prefix products and sums over m = 1..M (segments clipped to M).
  const int hm = min(hi, M);
  double sp = 1.0, sD = 0.0, sE = 0.0;
  for (int m = lo; m <= hm; ++m) {
    sp *= rho[m];
    if (DER) {
      const double q = d1[m] / rho[m];
      sD += q;
      sE += d2[m] / rho[m] - q * q;
    }
  }
  __syncthreads();
  sm.pre[0][t][0] = sp;
  sm.pre[0][t][1] = sD;
  sm.pre[0][t][2] = sE;
  __syncthreads();
  cur = 0;
  for (int d = 1; d < kBlock; d <<= 1) {
    if (t >= d) {
      sm.pre[cur ^ 1][t][0] = sm.pre[cur][t - d][0] * sm.pre[cur][t][0];
      sm.pre[cur ^ 1][t][1] = sm.pre[cur][t - d][1] + sm.pre[cur][t][1];
      sm.pre[cur ^ 1][t][2] = sm.pre[cur][t - d][2] + sm.pre[cur][t][2];
    } else {
      sm.pre[cur ^ 1][t][0] = sm.pre[cur][t][0];
      sm.pre[cur ^ 1][t][1] = sm.pre[cur][t][1];
      sm.pre[cur ^ 1][t][2] = sm.pre[cur][t][2];
    }
    __syncthreads();
    cur ^= 1;
  }
  double p = (t > 0) ? sm.pre[cur][t - 1][0] : 1.0;
  double D = (t > 0) ? sm.pre[cur][t - 1][1] : 0.0;
  double E = (t > 0) ? sm.pre[cur][t - 1][2] : 0.0;
  if (t == 0) rho[0] = 1.0;
  if (DER && t == 0) {
    d1[0] = 0.0;
    d2[0] = 0.0;
  }
  for (int m = lo; m <= hm; ++m) {
    const double rm = rho[m];
    p *= rm;
    rho[m] = p;
    if (DER) {
      const double q = d1[m] / rm;
      D += q;
      E += d2[m] / rm - q * q;
      d1[m] = p * D;
      d2[m] = p * (D * D + E);
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kBlock) series_kernel(const double* __restrict__ S, int M, double n, double L,
                                                       FKappas kap, int B, double* __restrict__ rho_all,
                                                       double* __restrict__ cv, double* __restrict__ sums) {
  __shared__ SeriesSmem sm;
  double* red = sm.red;
  const int b = blockIdx.x;
  double* rho = rho_all + int64_t(b) * (M + 1);
  const int Mb = min(M, kap.order[b]);
  bessel_series<false>(kap.k[b], Mb, rho, nullptr, nullptr, sm);
  double a = 0.0, a0 = 0.0, c = 0.0;
  for (int m = 1 + threadIdx.x; m <= Mb; m += kBlock) {
    const double sr = S[2 * (m - 1)], si = S[2 * (m - 1) + 1];
    const double P = fma(sr, sr, si * si);
    const double q = P - n;
    const double r = rho[m];
    const double r2 = r * r;
    a = fma(r2, P, a);
    a0 = fma(r2, q, a0);
    c = fma(r, q, c);
  }
  a = block_sum(a, red);
  a0 = block_sum(a0, red);
  c = block_sum(c, red);
  if (threadIdx.x == 0) {
    cv[b] = (2.0 * a / (n * n) - 4.0 * c / (n * (n - 1.0)) - 1.0) / L;
    if (sums) {
      sums[b] = (n * n - n + 2.0 * a0) / (2.0 * L);
      sums[B + b] = (n * n - n + 2.0 * c) / (2.0 * L);
    }
  }
}

__device__ __forceinline__ int first_min(const double* v, int B) {
  int best = 0;
  for (int t = 1; t < B; ++t)
    if (v[t] < v[best]) best = t;
  return best;
}

__global__ void argmin_kernel(const double* __restrict__ cv, int B, int32_t* __restrict__ argmin) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *argmin = first_min(cv, B);
}

struct Eval {
  double cv, g, gp;
};

// Objective and its first two derivatives in u = log(kappa), all threads,
// with the series cut at order Mk (that of a kappa at least as large).
__device__ Eval eval_u(double u, const double* __restrict__ S, int Mk, double n, double L, double* rho, double* d1,
                       double* d2, SeriesSmem& sm) {
  const double kappa = exp(u);
  bessel_series<true>(kappa, Mk, rho, d1, d2, sm);
  double A = 0.0, C = 0.0, A1 = 0.0, C1 = 0.0, A2 = 0.0, C2 = 0.0;
  for (int m = 1 + threadIdx.x; m <= Mk; m += kBlock) {
    const double sr = S[2 * (m - 1)], si = S[2 * (m - 1) + 1];
    const double P = fma(sr, sr, si * si);
    const double q = P - n;
    const double r = rho[m], r1 = d1[m], r2 = d2[m];
    A = fma(r * r, P, A);
    C = fma(r, q, C);
    A1 = fma(2.0 * r * r1, P, A1);
    C1 = fma(r1, q, C1);
    A2 = fma(2.0 * fma(r1, r1, r * r2), P, A2);
    C2 = fma(r2, q, C2);
  }
  double v[6] = {A, C, A1, C1, A2, C2};
  block_sum6(v, sm.red6);
  A = v[0];
  C = v[1];
  A1 = v[2];
  C1 = v[3];
  A2 = v[4];
  C2 = v[5];
  const double n2 = n * n, nn = n * (n - 1.0);
  Eval e;
  e.cv = (2.0 * A / n2 - 4.0 * C / nn - 1.0) / L;
  const double ck = (2.0 * A1 / n2 - 4.0 * C1 / nn) / L;
  const double ckk = (2.0 * A2 / n2 - 4.0 * C2 / nn) / L;
  e.g = kappa * ck;
  e.gp = kappa * kappa * ckk + kappa * ck;
  __syncthreads();  // rho, d1, d2 are rewritten by the next evaluation
  return e;
}

// The refinement's bracket: the list neighbours of the scan's first
// minimum bs (the lower one replaced by the first positive kappa when it is
// 0), the series order Mk of its upper end, and the first Newton iterate:
// the vertex of the parabola through the three grid values around bs in
// u = log(kappa) when it lies inside the bracket, else log(kappa_bs), else
// the bracket's middle. valid is false when there is no bracket of
// positive concentrations.
struct Bracket {
  int bs, Mk;
  double klo, khi, ul, uh, u0;
  bool valid;
};

__device__ Bracket make_bracket(const double* __restrict__ cvgrid, int B, const FKappas& kap, int M) {
  Bracket r;
  r.bs = first_min(cvgrid, B);
  r.Mk = min(M, kap.order[min(r.bs + 1, B - 1)]);
  double klo = kap.k[max(r.bs - 1, 0)];
  const double khi = kap.k[min(r.bs + 1, B - 1)];
  if (!(klo > 0.0)) {
    double kp = 0.0;
    for (int t = 0; t < B; ++t)
      if (kap.k[t] > 0.0) {
        kp = kap.k[t];
        break;
      }
    klo = kp;
  }
  r.valid = (klo > 0.0) && (khi > klo);
  r.klo = klo;
  r.khi = khi;
  r.ul = r.valid ? log(klo) : 0.0;
  r.uh = r.valid ? log(khi) : 0.0;
  r.u0 = 0.5 * (r.ul + r.uh);
  const int b = r.bs;
  if (r.valid && b > 0 && b < B - 1 && kap.k[b] > klo && kap.k[b] < khi) {
    const double ub = log(kap.k[b]);
    r.u0 = ub;
    if (kap.k[b - 1] > 0.0) {
      const double ua = log(kap.k[b - 1]), uc = log(kap.k[b + 1]);
      const double p = (ub - ua) * (cvgrid[b] - cvgrid[b + 1]);
      const double q = (ub - uc) * (cvgrid[b] - cvgrid[b - 1]);
      const double den = p - q;
      if (den != 0.0) {
        const double uv = ub - 0.5 * ((ub - ua) * p - (ub - uc) * q) / den;
        if (uv > r.ul && uv < r.uh) r.u0 = uv;
      }
    }
  }
  return r;
}

// Workgroup w evaluates the objective at the bracket's lower end (w = 0),
// upper end (1) and first iterate (2), each with its own series arrays
// (slots 3w .. 3w + 2 of rho); start[3w..3w+2] = (cv, g, g'),
// start[9] = the first iterate's u.
__global__ void __launch_bounds__(kBlock) newton_start_kernel(const double* __restrict__ S, int M, double n,
                                                             double L, FKappas kap, int B,
                                                             const double* __restrict__ cvgrid,
                                                             double* __restrict__ rho, double* __restrict__ start) {
  __shared__ SeriesSmem sm;
  const Bracket br = make_bracket(cvgrid, B, kap, M);
  if (!br.valid) return;
  const int w = blockIdx.x;
  const double u = (w == 0) ? br.ul : (w == 1) ? br.uh : br.u0;
  double* r = rho + size_t(3 * w) * (M + 1);
  const Eval e = eval_u(u, S, br.Mk, n, L, r, r + (M + 1), r + 2 * (M + 1), sm);
  if (threadIdx.x == 0) {
    start[3 * w] = e.cv;
    start[3 * w + 1] = e.g;
    start[3 * w + 2] = e.gp;
    if (w == 2) start[3 * kStartEvals] = u;
  }
}

// result: [kappa*, cv(kappa*), dCV/du at kappa*, steps, b*], continuing
// from newton_start_kernel's evaluations. Every thread runs the same
// control flow on the same values (block sums reach all).
__global__ void __launch_bounds__(kBlock) newton_kernel(const double* __restrict__ S, int M, double n, double L,
                                                       FKappas kap, int B, const double* __restrict__ cvgrid,
                                                       const double* __restrict__ start, double* __restrict__ rho3,
                                                       double* __restrict__ result, int32_t* __restrict__ argmin) {
  __shared__ SeriesSmem sm;
  double* rho = rho3;
  double* d1 = rho3 + (M + 1);
  double* d2 = rho3 + 2 * (M + 1);
  const Bracket br = make_bracket(cvgrid, B, kap, M);
  const int bs = br.bs;
  if (argmin && threadIdx.x == 0) *argmin = bs;
  double k_best = 0.0, cv_best = 0.0, g_best = 0.0;
  int steps = 0;
  if (!br.valid) {
    // no bracket of positive concentrations: the scan's value
    k_best = kap.k[bs];
    cv_best = cvgrid[bs];
    g_best = 0.0;
  } else {
    double ul = br.ul, uh = br.uh;
    const Eval el{start[0], start[1], start[2]};
    const Eval eh{start[3], start[4], start[5]};
    steps = 2;
    if (!(el.g < 0.0 && eh.g > 0.0)) {
      const bool lo_wins = el.cv <= eh.cv;
      k_best = lo_wins ? br.klo : br.khi;
      cv_best = lo_wins ? el.cv : eh.cv;
      g_best = lo_wins ? el.g : eh.g;
    } else {
      double u = start[3 * kStartEvals];
      Eval e{start[6], start[7], start[8]};
      ++steps;
      for (int it = 0; it < kMaxNewton && e.g != 0.0; ++it) {
        if (e.g < 0.0)
          ul = u;
        else
          uh = u;
        double un = u - e.g / e.gp;
        if (!(e.gp > 0.0) || !(un > ul && un < uh)) un = 0.5 * (ul + uh);
        const bool done = fabs(un - u) <= 1e-14 * fmax(1.0, fabs(un)) || (uh - ul) <= 1e-14 * fmax(1.0, fabs(un));
        u = un;
        e = eval_u(u, S, br.Mk, n, L, rho, d1, d2, sm);
        ++steps;
        if (done) break;
      }
      k_best = exp(u);
      cv_best = e.cv;
      g_best = e.g;
    }
  }
  if (threadIdx.x == 0) {
    result[0] = k_best;
    result[1] = cv_best;
    result[2] = g_best;
    result[3] = double(steps);
    result[4] = double(bs);
  }
}

// w_m = rho_m(kappa) S_m, m = 1..M (one workgroup).
__global__ void __launch_bounds__(kBlock) pilot_weights_kernel(const double* __restrict__ S, int M, double kappa,
                                                              double* __restrict__ rho, double* __restrict__ w) {
  __shared__ SeriesSmem sm;
  bessel_series<false>(kappa, M, rho, nullptr, nullptr, sm);
  for (int m = 1 + threadIdx.x; m <= M; m += kBlock) {
    w[2 * (m - 1)] = rho[m] * S[2 * (m - 1)];
    w[2 * (m - 1) + 1] = rho[m] * S[2 * (m - 1) + 1];
  }
}

// Per particle: f = (1/L)(1 + (2/N) sum_m Re(conj(w_m) e^{i m theta})),
// floored at `floor`; lf[i] = log f; block sums of (log f, floored).
template <typename T>
__global__ void __launch_bounds__(kBlock) pilot_kernel(const T* __restrict__ x, int64_t n, double L, int M,
                                                      const double* __restrict__ w, double floor_v,
                                                      double* __restrict__ lf, double* __restrict__ bpart,
                                                      uint32_t* status) {
  __shared__ double red[kBlock / 64];
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  double lsum = 0.0, fl = 0.0;
  if (i < n) {
    note_numeric(status, !isfinite(double(x[i])), false);
    const double f = wrap_d(double(x[i]), L) / L;
    double c1, s1;
    sincospi(2.0 * f, &s1, &c1);
    double acc = 0.0;
    for (int m0 = 1; m0 <= M; m0 += kPilotRun) {
      double c, s;
      phase(m0, f, c, s);
      const int m1 = min(M, m0 + kPilotRun - 1);
      for (int m = m0; m <= m1; ++m) {
        acc = fma(w[2 * (m - 1)], c, acc);
        acc = fma(w[2 * (m - 1) + 1], s, acc);
        const double nc = c * c1 - s * s1;
        s = fma(s, c1, c * s1);
        c = nc;
      }
    }
    double p = (1.0 + 2.0 * acc / double(n)) / L;
    if (!(p >= floor_v)) {  // also catches NaN: floored and counted
      fl = 1.0;
      p = isnan(p) ? p : floor_v;
    }
    const double l = log(p);
    lf[i] = l;
    lsum = l;
  }
  lsum = block_sum(lsum, red);
  fl = block_sum(fl, red);
  if (threadIdx.x == 0) {
    bpart[2 * int64_t(blockIdx.x)] = lsum;
    bpart[2 * int64_t(blockIdx.x) + 1] = fl;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) pilot_apply_kernel(const double* __restrict__ lf, int64_t n,
                                                            double kappa_star, double alpha,
                                                            const double* __restrict__ sums, T* __restrict__ kout,
                                                            double* __restrict__ log_g_out,
                                                            int64_t* __restrict__ nfl_out) {
  const double log_g = sums[0] / double(n);
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) kout[i] = T(kappa_star * exp(2.0 * alpha * (lf[i] - log_g)));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (log_g_out) *log_g_out = log_g;
    if (nfl_out) *nfl_out = int64_t(sums[1]);
  }
}

template <typename T>
kde_status launch_moments(const T* x, int64_t n, double L, int M, const FourierBufs& b, hipStream_t s) {
  const int64_t chunks = moment_chunks(n, M);
  const int64_t per = ceil_div(n, chunks);
  const dim3 grid{unsigned(chunks), unsigned(ceil_div(M, kMomM))};
  {
    TimedLaunch timed(KDE_KERNEL_MOMENTS, s);
    hipExtLaunchKernelGGL((moments_kernel<T>), grid, dim3(kBlock), 0, s, timed.start(), timed.stop(), 0, x, n, L,
                          M, per, b.partials, plain_numeric_word());
  }
  KDE_CHECK_LAUNCH();
  return launch_column_sum(b.partials, chunks, 2 * M, b.colsum, b.S, s);
}

kde_status moments_any(const kde_domain* dom, int64_t n, const void* x, int M, const FourierBufs& b,
                       hipStream_t s) {
  if (dom->prec == KDE_F64) return launch_moments(static_cast<const double*>(x), n, dom->L, M, b, s);
  return launch_moments(static_cast<const float*>(x), n, dom->L, M, b, s);
}

kde_status check_fourier_common(const kde_domain* dom, int64_t N, const void* x, int64_t nmin) {
  KDE_RETURN_IF(check_domain(dom, false));
  if (dom->shape != KDE_SHAPE_VONMISES) return fail(KDE_E_INVALID_ARG, "the Fourier route is defined for the von Mises shape");
  if (N < nmin || N > kMaxN) return fail(KDE_E_INVALID_ARG, "N must lie in [%lld, %lld] (got %lld)", (long long)nmin, (long long)kMaxN, (long long)N);
  if (!x) return fail(KDE_E_INVALID_ARG, "x must not be NULL");
  return KDE_OK;
}

kde_status check_fourier_kappas(int B, const double* kappas_h) {
  if (B < 1 || B > KDE_MAX_KAPPAS) return fail(KDE_E_INVALID_ARG, "B must lie in [1, %d] (got %d)", KDE_MAX_KAPPAS, B);
  if (!kappas_h) return fail(KDE_E_INVALID_ARG, "kappas_h is NULL");
  for (int b = 0; b < B; ++b) {
    const double k = kappas_h[b];
    if (!std::isfinite(k) || k < 0.0 || k > KDE_MAX_FOURIER_KAPPA)
      return fail(KDE_E_INVALID_ARG, "every kappa must lie in [0, %g] (got %g at %d)", KDE_MAX_FOURIER_KAPPA, k, b);
    if (b > 0 && !(k > kappas_h[b - 1])) return fail(KDE_E_INVALID_ARG, "kappas must be strictly ascending (index %d)", b);
  }
  return KDE_OK;
}

FKappas to_list(const double* k, int B) {
  FKappas f{};
  for (int b = 0; b < B; ++b) {
    f.k[b] = k[b];
    f.order[b] = fourier_order(k[b]);
  }
  return f;
}

}  // namespace

size_t fourier_workspace_bytes(int op, int64_t n, int B) {
  Carver c(nullptr, 0);
  carve_fourier(c, op, n, B);
  return c.used;
}

}  // namespace kde

using namespace kde;

extern "C" {

kde_status kde_cv_scan_fourier(const kde_domain* dom, int64_t N, const void* x, int32_t B, const double* kappas_h,
                               double* cv, double* sums, int32_t* argmin, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  KDE_RETURN_IF(check_fourier_common(dom, N, x, 2));
  KDE_RETURN_IF(check_fourier_kappas(B, kappas_h));
  if (!cv) return fail(KDE_E_INVALID_ARG, "cv must not be NULL");
  KDE_RETURN_IF(check_workspace(ws, ws_bytes, fourier_workspace_bytes(KDE_OP_CV_FOURIER, N, B)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws, ws_bytes);
  const FourierBufs b = carve_fourier(c, KDE_OP_CV_FOURIER, N, B);
  const int M = fourier_order(kappas_h[B - 1]);
  KDE_RETURN_IF(moments_any(dom, N, x, M, b, s));
  hipLaunchKernelGGL(series_kernel, dim3(B), dim3(kBlock), 0, s, (const double*)b.S, M, double(N), dom->L,
                     to_list(kappas_h, B), B, b.rho, cv, sums);
  KDE_CHECK_LAUNCH();
  if (argmin) {
    hipLaunchKernelGGL(argmin_kernel, dim3(1), dim3(64), 0, s, (const double*)cv, B, argmin);
    KDE_CHECK_LAUNCH();
  }
  return KDE_OK;
}

kde_status kde_cv_refine(const kde_domain* dom, int64_t N, const void* x, int32_t B, const double* kappas_h,
                         double* result, double* cv, int32_t* argmin, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  KDE_RETURN_IF(check_fourier_common(dom, N, x, 2));
  KDE_RETURN_IF(check_fourier_kappas(B, kappas_h));
  if (!result) return fail(KDE_E_INVALID_ARG, "result must not be NULL");
  KDE_RETURN_IF(check_workspace(ws, ws_bytes, fourier_workspace_bytes(KDE_OP_CV_REFINE, N, B)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws, ws_bytes);
  const FourierBufs b = carve_fourier(c, KDE_OP_CV_REFINE, N, B);
  const int M = fourier_order(kappas_h[B - 1]);
  KDE_RETURN_IF(moments_any(dom, N, x, M, b, s));
  double* grid = cv ? cv : b.cvgrid;
  const FKappas kl = to_list(kappas_h, B);
  hipLaunchKernelGGL(series_kernel, dim3(B), dim3(kBlock), 0, s, (const double*)b.S, M, double(N), dom->L, kl, B,
                     b.rho, grid, (double*)nullptr);
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL(newton_start_kernel, dim3(kStartEvals), dim3(kBlock), 0, s, (const double*)b.S, M, double(N),
                     dom->L, kl, B, (const double*)grid, b.rho, b.start);
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL(newton_kernel, dim3(1), dim3(kBlock), 0, s, (const double*)b.S, M, double(N), dom->L, kl, B,
                     (const double*)grid, (const double*)b.start, b.rho, result, argmin);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

kde_status kde_adapt_widths_exact(const kde_domain* dom, int64_t N, const void* x, double kappa_star, double alpha,
                                  void* kappa_out, double* log_geomean, int64_t* n_floored, void* ws, size_t ws_bytes,
                                  void* stream) {
  clear_error();
  KDE_RETURN_IF(check_fourier_common(dom, N, x, 1));
  if (!kappa_out) return fail(KDE_E_INVALID_ARG, "kappa_out must not be NULL");
  if (!std::isfinite(kappa_star) || !(kappa_star > 0.0) || kappa_star > KDE_MAX_FOURIER_KAPPA)
    return fail(KDE_E_INVALID_ARG, "kappa_star must lie in (0, %g] (got %g)", KDE_MAX_FOURIER_KAPPA, kappa_star);
  if (!std::isfinite(alpha) || alpha < 0.0) return fail(KDE_E_INVALID_ARG, "alpha must be finite and >= 0 (got %g)", alpha);
  KDE_RETURN_IF(check_workspace(ws, ws_bytes, fourier_workspace_bytes(KDE_OP_ADAPT_EXACT, N, 0)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws, ws_bytes);
  const FourierBufs b = carve_fourier(c, KDE_OP_ADAPT_EXACT, N, 0);
  const int M = fourier_order(kappa_star);
  KDE_RETURN_IF(moments_any(dom, N, x, M, b, s));
  hipLaunchKernelGGL(pilot_weights_kernel, dim3(1), dim3(kBlock), 0, s, (const double*)b.S, M, kappa_star, b.rho, b.w);
  KDE_CHECK_LAUNCH();
  const int64_t blocks = ceil_div(N, kBlock);
  const dim3 grid{unsigned(blocks)};
  TimedLaunch timed(KDE_KERNEL_ADAPT, s);  // from the pilot values' start to the widths' end
  if (dom->prec == KDE_F64)
    hipExtLaunchKernelGGL(pilot_kernel<double>, grid, dim3(kBlock), 0, s, timed.start(), nullptr, 0,
                          static_cast<const double*>(x), N, dom->L, M, (const double*)b.w,
                          double(std::numeric_limits<double>::min()), b.lf, b.bpart, plain_numeric_word());
  else
    hipExtLaunchKernelGGL(pilot_kernel<float>, grid, dim3(kBlock), 0, s, timed.start(), nullptr, 0,
                          static_cast<const float*>(x), N, dom->L, M, (const double*)b.w,
                          double(std::numeric_limits<float>::min()), b.lf, b.bpart, plain_numeric_word());
  KDE_CHECK_LAUNCH();
  KDE_RETURN_IF(launch_column_sum(b.bpart, blocks, 2, b.colsum2, b.sums2, s));
  if (dom->prec == KDE_F64)
    hipExtLaunchKernelGGL(pilot_apply_kernel<double>, grid, dim3(kBlock), 0, s, nullptr, timed.stop(), 0,
                          (const double*)b.lf, N, kappa_star, alpha, (const double*)b.sums2,
                          static_cast<double*>(kappa_out), log_geomean, n_floored);
  else
    hipExtLaunchKernelGGL(pilot_apply_kernel<float>, grid, dim3(kBlock), 0, s, nullptr, timed.stop(), 0,
                          (const double*)b.lf, N, kappa_star, alpha, (const double*)b.sums2,
                          static_cast<float*>(kappa_out), log_geomean, n_floored);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

}  // extern "C"

// Vector kernels of BiCGSTAB (van der Vorst 1992), the second iterative
// workload of Sec. 5.5.2, around the plan's fused SpMV.  Iteration i:
//   update_p : rho_i = (r^, r_i); beta = (rho_i / rho_{i-1}) (alpha_{i-1} / omega_{i-1});
//              p = r + beta (p - omega_{i-1} v)          (p = r at i = 0)
//   SpMV     : v = A p
//   dot1     : (r^, v)
//   update_s : alpha_i = rho_i / (r^, v);  s = r - alpha_i v
//   SpMV     : t = A s
//   dot2     : (t, s), (t, t)
//   update_xr: omega_i = (t, s) / (t, t);  x += alpha_i p + omega_i s;
//              r = s - omega_i t;  (r^, r), (r, r) for the next iteration
// Every dot product is reduced per block into a (first, second) pair of
// doubles; each consumer kernel sums the pairs itself in block order, so the
// scalars are bit-identical in every block and across runs, and no scalar
// crosses a kernel boundary through a device-scope fence.  The pair arrays of
// consecutive iterations alternate, so iteration i still sees i - 1's.
// Divisions by zero are guarded (the quotient is taken as 0): omega = 0 when
// t = 0 (s = 0, x + alpha p is exact), alpha = 0 when (r^, v) = 0 and
// beta = 0 when rho_{i-1} or omega_{i-1} is 0; the host reports a breakdown
// when rho reaches 0 before convergence.
#include "merbit_internal.hpp"

namespace merbit {

// Totals of both components of G pairs, identical in every block.
__device__ __forceinline__ void sum_pairs(const double* __restrict__ part, int G, double& a,
                                          double& b) {
  __shared__ double ta, tb;
  double x = 0.0, y = 0.0;
  for (int k = threadIdx.x; k < G; k += kReduceThreads) {
    x += part[2 * k];
    y += part[2 * k + 1];
  }
  block_sum2(x, y);
  if (threadIdx.x == 0) {
    ta = x;
    tb = y;
  }
  __syncthreads();
  a = ta;
  b = tb;
  __syncthreads();  // ta / tb may be rewritten by a later call
}

__device__ __forceinline__ double safe_div(double a, double b) { return b != 0.0 ? a / b : 0.0; }

__device__ __forceinline__ void write_pair(double* part, double a, double b) {
  block_sum2(a, b);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

#define BICG_LOOP(i) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; \
       i += (int64_t)gridDim.x * blockDim.x)

// r = b - Ax0 (ax = A x0), r^ = r; pairs (r^.r, r.r) and (b.b, 0)
template <typename V>
__global__ __launch_bounds__(kReduceThreads) void bicg_init_kernel(
    const V* __restrict__ b, const V* __restrict__ ax, V* __restrict__ r, V* __restrict__ rh,
    int64_t n, double* __restrict__ part_r, double* __restrict__ part_b) {
  double rr = 0.0, bb = 0.0;
  BICG_LOOP(i) {
    const V bi = b[i];
    const V ri = bi - ax[i];
    r[i] = ri;
    rh[i] = ri;
    rr += (double)ri * (double)ri;
    bb += (double)bi * (double)bi;
  }
  double rr2 = rr, z = 0.0;
  write_pair(part_r, rr, rr2);
  write_pair(part_b, bb, z);
}

template <typename V>
__global__ __launch_bounds__(kReduceThreads) void bicg_update_p_kernel(
    const V* __restrict__ r, V* __restrict__ p, const V* __restrict__ v, int64_t n, int first,
    const double* __restrict__ pa_cur, const double* __restrict__ pa_prev,
    const double* __restrict__ pb_prev, const double* __restrict__ pc_prev, int G) {
  if (first) {
    BICG_LOOP(i) p[i] = r[i];
    return;
  }
  double rho, rr, rho_prev, d0, rhv_prev, d1, ts_prev, tt_prev;
  sum_pairs(pa_cur, G, rho, rr);
  sum_pairs(pa_prev, G, rho_prev, d0);
  sum_pairs(pb_prev, G, rhv_prev, d1);
  sum_pairs(pc_prev, G, ts_prev, tt_prev);
  const double alpha_prev = safe_div(rho_prev, rhv_prev);
  const double omega_prev = safe_div(ts_prev, tt_prev);
  const double beta = safe_div(rho, rho_prev) * safe_div(alpha_prev, omega_prev);
  const V bt = (V)beta, om = (V)omega_prev;
  BICG_LOOP(i) p[i] = r[i] + bt * (p[i] - om * v[i]);
}

// pairs (a.b, 0)
template <typename V>
__global__ __launch_bounds__(kReduceThreads) void bicg_dot1_kernel(
    const V* __restrict__ a, const V* __restrict__ b, int64_t n, double* __restrict__ part) {
  double d = 0.0, z = 0.0;
  BICG_LOOP(i) d += (double)a[i] * (double)b[i];
  write_pair(part, d, z);
}

template <typename V>
__global__ __launch_bounds__(kReduceThreads) void bicg_update_s_kernel(
    const V* __restrict__ r, const V* __restrict__ v, V* __restrict__ s, int64_t n,
    const double* __restrict__ pa_cur, const double* __restrict__ pb_cur, int G) {
  double rho, rr, rhv, d;
  sum_pairs(pa_cur, G, rho, rr);
  sum_pairs(pb_cur, G, rhv, d);
  const V al = (V)safe_div(rho, rhv);
  BICG_LOOP(i) s[i] = r[i] - al * v[i];
}

// pairs (t.s, t.t)
template <typename V>
__global__ __launch_bounds__(kReduceThreads) void bicg_dot2_kernel(
    const V* __restrict__ t, const V* __restrict__ s, int64_t n, double* __restrict__ part) {
  double ts = 0.0, tt = 0.0;
  BICG_LOOP(i) {
    const double ti = (double)t[i];
    ts += ti * (double)s[i];
    tt += ti * ti;
  }
  write_pair(part, ts, tt);
}

template <typename V>
__global__ __launch_bounds__(kReduceThreads) void bicg_update_xr_kernel(
    V* __restrict__ x, const V* __restrict__ p, const V* __restrict__ s, const V* __restrict__ t,
    V* __restrict__ r, const V* __restrict__ rh, int64_t n, const double* __restrict__ pa_cur,
    const double* __restrict__ pb_cur, const double* __restrict__ pc_cur, int G,
    double* __restrict__ pa_next) {
  double rho, rr, rhv, d, ts, tt;
  sum_pairs(pa_cur, G, rho, rr);
  sum_pairs(pb_cur, G, rhv, d);
  sum_pairs(pc_cur, G, ts, tt);
  const V al = (V)safe_div(rho, rhv);
  const V om = (V)safe_div(ts, tt);
  double rhr = 0.0, rr2 = 0.0;
  BICG_LOOP(i) {
    const V si = s[i];
    x[i] = x[i] + al * p[i] + om * si;
    const V ri = si - om * t[i];
    r[i] = ri;
    rhr += (double)rh[i] * (double)ri;
    rr2 += (double)ri * (double)ri;
  }
  write_pair(pa_next, rhr, rr2);
}

#undef BICG_LOOP

int bicg_grid(int64_t n) { return pr_reduce_grid(n); }

template <typename V>
static hipError_t bicg_step_t(const BicgArgs& a, int stage, hipStream_t st) {
  const dim3 g((unsigned)a.G), b(kReduceThreads);
  const int64_t n = a.n;
  V* x = static_cast<V*>(a.x);
  V* r = static_cast<V*>(a.r);
  V* rh = static_cast<V*>(a.rh);
  V* p = static_cast<V*>(a.p);
  V* v = static_cast<V*>(a.v);
  V* s = static_cast<V*>(a.s);
  V* t = static_cast<V*>(a.t);
  switch (stage) {
    case kBicgInit:
      hipLaunchKernelGGL(bicg_init_kernel<V>, g, b, 0, st, static_cast<const V*>(a.b), t, r, rh,
                         n, a.pa_next, a.pb_norm);
      break;
    case kBicgUpdateP:
      hipLaunchKernelGGL(bicg_update_p_kernel<V>, g, b, 0, st, r, p, v, n, a.first, a.pa_cur,
                         a.pa_prev, a.pb_prev, a.pc_prev, a.G);
      break;
    case kBicgDot1:
      hipLaunchKernelGGL(bicg_dot1_kernel<V>, g, b, 0, st, rh, v, n, a.pb_cur);
      break;
    case kBicgUpdateS:
      hipLaunchKernelGGL(bicg_update_s_kernel<V>, g, b, 0, st, r, v, s, n, a.pa_cur, a.pb_cur,
                         a.G);
      break;
    case kBicgDot2:
      hipLaunchKernelGGL(bicg_dot2_kernel<V>, g, b, 0, st, t, s, n, a.pc_cur);
      break;
    case kBicgUpdateXR:
      hipLaunchKernelGGL(bicg_update_xr_kernel<V>, g, b, 0, st, x, p, s, t, r, rh, n, a.pa_cur,
                         a.pb_cur, a.pc_cur, a.G, a.pa_next);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bicg(int dtype, const BicgArgs& a, int stage, hipStream_t st) {
  return dtype == 0 ? bicg_step_t<float>(a, stage, st) : bicg_step_t<double>(a, stage, st);
}

}  // namespace merbit

// The pseudofermion force and the momentum update of the molecular dynamics.
//
// For S_f = eta^dag (D^dag D)^{-1} eta, X = (D^dag D)^{-1} eta and Y = D X,
// a link change U_mu(x) -> exp(eps T) U_mu(x) (T traceless antihermitian)
// changes the action by eps Re tr[T F_mu(x)] with
//   F_mu(x) = 2 kappa s_mu(x) U_mu(x) [ M + N^dag ],
//   M = sum over the 4 spins of ((1 - g_mu) X(x+mu))_s Y(x)_s^dag,
//   N = sum over the 4 spins of ((1 + g_mu) X(x))_s Y(x+mu)_s^dag,
// s_mu(x) the boundary sign of the link.  The projectors have rank two: with
// h = upper((1 - g_mu) psi) the lower spins are -A^dag h, and the 4-spin sum
// of outer products equals the 2-spin sum of the projected upper halves,
// M = sum_{s<2} h[X(x+mu)]_s h[Y(x)]_s^dag (and N likewise with 1 + g_mu).
// So each term costs two half-spinor projections and 2 x 9 complex products.
#include "wd_kcommon.h"
#include "wd_kernels.h"

namespace wd {

template <int R, int MU>
__device__ __forceinline__ void force_link(const char* __restrict__ X, const char* __restrict__ Y, size_t pstride,
                                           const char* __restrict__ gauge, const Geom& g, const Coord& k,
                                           int parity, int s, float bc_mu, double two_kappa,
                                           double2* __restrict__ out) {
  const size_t n = (size_t)g.n;
  const int nb = neighbour_cb(g, k, MU, +1);
  const char* Xo = X + (size_t)parity * pstride;
  const char* Xn = X + (size_t)(1 - parity) * pstride;
  const char* Yo = Y + (size_t)parity * pstride;
  const char* Yn = Y + (size_t)(1 - parity) * pstride;
  cplx<double> q[9];
  {
    spinor<double> a, b;
    SpinorFmt<F64>::load(Xn, n, (size_t)nb, a);
    SpinorFmt<F64>::load(Yo, n, (size_t)s, b);
    half_spinor<double> ha, hb;
    project<MU, +1>(a, ha);
    project<MU, +1>(b, hb);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        q[3 * r + c] = cadd(cjmul(hb.c[c], ha.c[r]), cjmul(hb.c[3 + c], ha.c[3 + r]));
  }
  {
    spinor<double> a, b;
    SpinorFmt<F64>::load(Xo, n, (size_t)s, a);
    SpinorFmt<F64>::load(Yn, n, (size_t)nb, b);
    half_spinor<double> ha, hb;
    project<MU, -1>(a, ha);
    project<MU, -1>(b, hb);
    // + N^dag: (N^dag)_{rc} = sum_s h[Y(x+mu)]_{s r} conj(h[X(x)]_{s c})
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        q[3 * r + c] = cadd(q[3 * r + c], cadd(cjmul(ha.c[c], hb.c[r]), cjmul(ha.c[3 + c], hb.c[3 + r])));
  }
  su3<double> u;
  LinkFmt<F64, R>::load_nt(gauge + (size_t)(parity * 4 + MU) * link_dir_bytes<F64, R>(n), n, (size_t)s, u);
  const double f = (k.c[MU] == g.L[MU] - 1 && bc_mu < 0.f) ? -two_kappa : two_kappa;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cplx<double> v = cmul(u.e[3 * r], q[c]);
      v = cadd(v, cmul(u.e[3 * r + 1], q[3 + c]));
      v = cadd(v, cmul(u.e[3 * r + 2], q[6 + c]));
      out[3 * r + c] = make_double2(f * v.re, f * v.im);
    }
}

// One thread per (mu, lexicographic site); X and Y are FP64 internal fields
// (one rhs, both parity blocks pstride bytes apart); F is complex128
// [mu][t][z][y][x][3][3].
template <int R>
__global__ void __launch_bounds__(256) force_kernel(const char* __restrict__ X, const char* __restrict__ Y,
                                                    size_t pstride, const char* __restrict__ gauge, Geom g,
                                                    float4 bc, double two_kappa, double2* __restrict__ F) {
  const long long V = 2LL * g.n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 4 * V) return;
  const int mu = (int)(idx / V);
  const int i = (int)(idx - (long long)mu * V);
  Coord k;
  k.c[0] = i % g.L[0];
  k.rest = i / g.L[0];
  k.c[1] = k.rest % g.L[1];
  const int r2 = k.rest / g.L[1];
  k.c[2] = r2 % g.L[2];
  k.c[3] = r2 / g.L[2];
  const int parity = (k.c[0] + k.c[1] + k.c[2] + k.c[3]) & 1;
  const int s = i >> 1;
  double2* out = F + ((size_t)mu * V + i) * 9;
  switch (mu) {
    case 0: force_link<R, 0>(X, Y, pstride, gauge, g, k, parity, s, bc.x, two_kappa, out); break;
    case 1: force_link<R, 1>(X, Y, pstride, gauge, g, k, parity, s, bc.y, two_kappa, out); break;
    case 2: force_link<R, 2>(X, Y, pstride, gauge, g, k, parity, s, bc.z, two_kappa, out); break;
    default: force_link<R, 3>(X, Y, pstride, gauge, g, k, parity, s, bc.w, two_kappa, out); break;
  }
}

hipError_t launch_force(const void* X, const void* Y, size_t pstride, const void* gauge, int recon, const Geom& g,
                        const float bc[4], double kappa, void* F, hipStream_t stream) {
  const long long total = 8LL * g.n;
  const unsigned grid = (unsigned)((total + 255) / 256);
  const float4 b = make_float4(bc[0], bc[1], bc[2], bc[3]);
  if (recon == 12)
    hipLaunchKernelGGL((force_kernel<12>), dim3(grid), dim3(256), 0, stream, (const char*)X, (const char*)Y, pstride,
                       (const char*)gauge, g, b, 2.0 * kappa, (double2*)F);
  else
    hipLaunchKernelGGL((force_kernel<18>), dim3(grid), dim3(256), 0, stream, (const char*)X, (const char*)Y, pstride,
                       (const char*)gauge, g, b, 2.0 * kappa, (double2*)F);
  return hipGetLastError();
}

// p += factor * TA(F) per link matrix, TA(M) = (M - M^dag)/2 - tr(M - M^dag)/6.
__global__ void __launch_bounds__(256) ta_add_kernel(double2* __restrict__ p, const double2* __restrict__ F,
                                                     double factor, long long nmat) {
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nmat) return;
  const double2* f = F + m * 9;
  double2* q = p + m * 9;
  double2 a[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) a[k] = f[k];
  // antihermitian part A = (M - M^dag)/2: A_rc = (M_rc - conj(M_cr)) / 2
  double2 A[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      A[3 * r + c] = make_double2(0.5 * (a[3 * r + c].x - a[3 * c + r].x), 0.5 * (a[3 * r + c].y + a[3 * c + r].y));
  const double tr_im = (A[0].y + A[4].y + A[8].y) / 3.0;  // the trace of A is imaginary
#pragma unroll
  for (int d = 0; d < 3; ++d) A[4 * d].y -= tr_im;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double2 v = q[k];
    q[k] = make_double2(v.x + factor * A[k].x, v.y + factor * A[k].y);
  }
}

hipError_t launch_ta_add(void* p, const void* F, double factor, long long nmat, hipStream_t stream) {
  if (nmat <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((nmat + 255) / 256);
  hipLaunchKernelGGL(ta_add_kernel, dim3(grid), dim3(256), 0, stream, (double2*)p, (const double2*)F, factor, nmat);
  return hipGetLastError();
}

}  // namespace wd

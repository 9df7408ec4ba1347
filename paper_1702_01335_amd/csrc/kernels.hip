// HIP kernels for gfx950 (MI355X) of the mixed-quadrature lattice Boltzmann time step
// for 3D Couette flow (Ambrus & Sofonea, arXiv:1702.01335).
//
// One RK3 stage (Eq. rk3) is two launches:
//   closure_kernel  per node: sum the moment partials of the stage input, form n, u, the
//                   pressure tensor, T and q (Eq. qdef), tau (Eq. mw_tau / power law /
//                   Eq. sutherland_tau), and the Hermite-projected equilibrium factors
//                   (Sec. III direct product) into a per-node record; one extra block per
//                   instance computes the wall density from the outgoing wall fluxes
//                   (App. A.4).
//   stage_kernel    per (velocity block x node chunk): each thread owns one velocity and
//                   marches a chunk of nodes along x with the stencil in registers,
//                   synthesising the ghost nodes in place (bounce-back, extrapolation,
//                   wall Maxwellian), computes the WENO-5 / upwind interface fluxes
//                   (App. A.3), the derivative of Eq. flux, the Shakhov relaxation
//                   (Eq. L_def with Eq. sdef) and the RK3 combination, stores the result
//                   and reduces its moment partials (and, at stage 3, residual partials)
//                   for the next closure.
// Populations: FP64 [B][S][V], v fastest, so a wave reads 64 consecutive velocities of
// one node (coalesced 512-byte rows).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "hrlb_internal.h"

namespace hrlb {

// ---------------------------------------------------------------------------------------
// helpers

// Map the hardware block index to a tile so that consecutive tiles (neighbouring node
// chunks of one velocity block, which share halo rows) land on the same XCD: blocks are
// dealt round-robin to the 8 XCDs, so XCD x receives block ids x, x+8, x+16, ...
__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int xcd = bid & 7, idx = bid >> 3;
  return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// a pointer into device memory re-typed to the global address space.  Pointers that reach
// a kernel through memory (the batched kernels' group descriptors) are generic to the
// compiler, which would otherwise access them with flat instructions; flat accesses count
// on both wait counters, so a wait for a scalar load would also wait for them.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// WENO-5 reconstruction at the interface downstream of c from the upwind-ordered
// stencil (a, b, c, d, e) (App. A.3; candidates of Eq. weno5_flux, indicators of
// Eq. weno_sigma, weights of Eq. weno5_omega without epsilon).  The candidates are carried
// as 6 f_q and the indicators as 12 s_q, so every coefficient is a small integer; the
// weights (d_q / s_q^2) / sum_r (d_r / s_r^2) do not change under a common factor of the
// indicators.  They are evaluated as N_q / sum N with N_q = d_q prod_{r != q} t_r^2, the
// ideal weights d as 1 : 6 : 3 and t_q = s_q / 2^e, 2^e the binade of max s: one quotient,
// exact power-of-two scaling (so the scheme stays homogeneous of degree one), and vanishing
// indicators give the Table II rows directly (one vanishing: N_q alone survives; two: the
// sum vanishes and the pair row is taken; three: ideal weights).
__device__ __forceinline__ double weno5(double a, double b, double c, double d, double e) {
  const double f1 = 2.0 * a - 7.0 * b + 11.0 * c;
  const double f2 = -b + 5.0 * c + 2.0 * d;
  const double f3 = 2.0 * c + 5.0 * d - e;
  const double r1 = a - 2.0 * b + c, q1 = a - 4.0 * b + 3.0 * c;
  const double r2 = b - 2.0 * c + d, q2 = b - d;
  const double r3 = c - 2.0 * d + e, q3 = 3.0 * c - 4.0 * d + e;
  const double s1 = 13.0 * r1 * r1 + 3.0 * q1 * q1;
  const double s2 = 13.0 * r2 * r2 + 3.0 * q2 * q2;
  const double s3 = 13.0 * r3 * r3 + 3.0 * q3 * q3;
  const double smax = fmax(s1, fmax(s2, s3));
  int ex;
  (void)frexp(smax, &ex);  // 0 for smax = 0: then every t_q is 0
  const double t1 = ldexp(s1, -ex), t2 = ldexp(s2, -ex), t3 = ldexp(s3, -ex);
  const double u1 = t1 * t1, u2 = t2 * t2, u3 = t3 * t3;
  const double n1 = u2 * u3, n2 = 6.0 * (u1 * u3), n3 = 3.0 * (u1 * u2);
  const double den = n1 + n2 + n3;
  const double num = n1 * f1 + n2 * f2 + n3 * f3;
  // one branch on the common path.  Above 2^-1000 the quotient is num times the
  // reciprocal of 6 den refined by one Newton step, then one residual correction
  // (v_rcp_f64 has no range trouble there); the few lanes below take the division itself.
  // Measured on gfx950 over 2^20 quotients with operands across [2^-900, 2^900]: the
  // estimate is good to ~2^-25, one Newton step to 11 ulp, and the corrected quotient
  // equals the correctly rounded one in every case (as it does with a second step)
  if (den > 0x1p-1000) {
    const double x = 6.0 * den;
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    const double q = num * r;
    return fma(r, fma(-x, q, num), q);
  }
  if (den > 0.0) return num / (6.0 * den);
  if (smax == 0.0) return (f1 + 6.0 * f2 + 3.0 * f3) * (1.0 / 60.0);
  if (u1 == 0.0 && u2 == 0.0) return (f1 + 6.0 * f2) * (1.0 / 42.0);
  if (u1 == 0.0 && u3 == 0.0) return (f1 + 3.0 * f3) * (1.0 / 24.0);
  return (2.0 * f2 + f3) * (1.0 / 18.0);
}

// the WENO-5 candidates with the ideal weights: the linear fifth-order upwind flux,
// (0.1 f1 + 0.6 f2 + 0.3 f3) with the candidates expanded
__device__ __forceinline__ double linear5(double a, double b, double c, double d, double e) {
  return (2.0 * a - 13.0 * b + 47.0 * c + 27.0 * d - 3.0 * e) * (1.0 / 60.0);
}

template <int SCHEME>
__device__ __forceinline__ double interp(double a, double b, double c, double d, double e) {
  if constexpr (SCHEME == 1) {
    return weno5(a, b, c, d, e);
  } else if constexpr (SCHEME == 2) {
    return linear5(a, b, c, d, e);
  } else {
    (void)a;
    (void)d;
    (void)e;
    return 1.5 * c - 0.5 * b;  // second-order upwind: (3 F_s - F_{s-1}) / 2
  }
}

// Half-range Gaussian moments I_k(u, T) = int_0^inf p^k G(p; u, T) dp, k <= NX_MAX:
// I_0 = erfc(-u / sqrt(2T)) / 2, I_1 = u I_0 + T G(0), I_k = u I_{k-1} + (k-1) T I_{k-2}.
// The square root and divisions are the correctly rounded ones, so that at rest (u = 0) the
// moments are the same doubles on any IEEE machine.
__device__ __forceinline__ void half_gauss_moments(double u, double T, double* I) {
  const double G0 = exp(-u * u / (2.0 * T)) / sqrt(2.0 * M_PI * T);
  I[0] = 0.5 * erfc(-u / sqrt(2.0 * T));
  I[1] = u * I[0] + T * G0;
#pragma unroll
  for (int k = 2; k <= NX_MAX; ++k) I[k] = u * I[k - 1] + (k - 1) * T * I[k - 2];
}

// Coefficients J_l = int G h_l over one semi-axis (monic half-range h_l, l <= Nx), as the
// dot product sum_k C_lk I_k of the monomial coefficients with the half-range moments.  The
// terms cancel (at rest J_l vanishes for l >= 1 while the terms reach 1e3), and the outer
// half-range nodes multiply what is left of J_l by up to 1e7 (Qx = 50), so the product is
// summed by the compensated algorithm Dot2 of Ogita, Rump and Oishi (2005): exact products
// (fma), exact two-term sums, the rounding errors summed on the side; the result is as
// accurate as a dot product in twice the precision.  The compiler must not contract the
// two-term sums into fused multiply-adds, which would break their exactness.
__device__ __forceinline__ void half_projection(const double* __restrict__ cx, int Nx, const double* I, double* J) {
#pragma clang fp contract(off)
#pragma unroll
  for (int l = 0; l <= NX_MAX; ++l) {
    double p = 0.0, s = 0.0;
    if (l <= Nx) {
      const double* c = cx + l * (Nx + 1);
      p = c[0] * I[0];
      s = fma(c[0], I[0], -p);
#pragma unroll
      for (int k = 1; k <= l; ++k) {
        const double h = c[k] * I[k];
        const double r = fma(c[k], I[k], -h);
        const double t = p + h;
        const double bb = t - p;
        const double q = (p - (t - bb)) + (h - bb);
        p = t;
        s = s + (q + r);
      }
    }
    J[l] = p + s;
  }
}

// g_x at axis node i (ascending over both semi-axes): w_m sum_l h_l(p_m) J^{+-}_l / gamma_l.
__device__ __forceinline__ double gx_node(const double* __restrict__ phix, int Qx, int Nx, int i, const double* Jp,
                                          const double* Jm) {
  const bool pos = i >= Qx;
  const int m = pos ? i - Qx : Qx - 1 - i;
  double s = 0.0;
#pragma unroll
  for (int l = 0; l <= NX_MAX; ++l)
    if (l <= Nx) s += phix[m * (Nx + 1) + l] * (pos ? Jp[l] : Jm[l]);
  return s;
}

// Full-range Hermite coefficients of the 1D Maxwellian: a_l = int G He_l dp,
// a_0 = 1, a_1 = u, a_{l+1} = u a_l + l (T - 1) a_{l-1} (generating function
// exp(u t + (T-1) t^2 / 2) of E[He_l(X)], X ~ N(u, T)).
__device__ __forceinline__ void full_coeffs(double u, double T, double* a) {
  a[0] = 1.0;
  a[1] = u;
#pragma unroll
  for (int l = 1; l < NYZ_MAX; ++l) a[l + 1] = u * a[l] + l * (T - 1.0) * a[l - 1];
}

__device__ __forceinline__ double full_node(const double* __restrict__ phi, int N, int j, const double* a) {
  double s = 0.0;
#pragma unroll
  for (int l = 0; l <= NYZ_MAX; ++l)
    if (l <= N) s += phi[j * (N + 1) + l] * a[l];
  return s;
}

// ---------------------------------------------------------------------------------------
// setup: equilibrium at rest and wall Maxwellian per unit density, wall denominator

__global__ void __launch_bounds__(256) setup_tables_kernel(Shape sh, DevPtrs d) {
  const int b = blockIdx.x;
  const InstDev in = d.inst[b];
  __shared__ double gx0[2 * QX_MAX], gy0[QYZ_MAX], gyw[QYZ_MAX], gz0[QYZ_MAX];
  __shared__ double red[256];
  double I[NX_MAX + 1], Jp[NX_MAX + 1], Jm[NX_MAX + 1];
  half_gauss_moments(0.0, in.T_w, I);
  half_projection(d.cx, sh.Nx, I, Jp);
  half_gauss_moments(-0.0, in.T_w, I);
  half_projection(d.cx, sh.Nx, I, Jm);
  double a0[NYZ_MAX + 1], aw[NYZ_MAX + 1];
  full_coeffs(0.0, in.T_w, a0);
  full_coeffs(in.u_w, in.T_w, aw);
  for (int i = threadIdx.x; i < 2 * sh.Qx; i += blockDim.x) gx0[i] = gx_node(d.phix, sh.Qx, sh.Nx, i, Jp, Jm);
  for (int j = threadIdx.x; j < sh.Qy; j += blockDim.x) {
    gy0[j] = full_node(d.phiy, sh.Ny, j, a0);
    gyw[j] = full_node(d.phiy, sh.Ny, j, aw);
  }
  // reduced (phi, chi) model: the z factor is 1 for phi and T for chi (chi^eq = T phi^eq)
  for (int k = threadIdx.x; k < sh.Qz; k += blockDim.x)
    gz0[k] = sh.reduced ? (k == 0 ? 1.0 : in.T_w) : full_node(d.phiz, sh.Nz, k, a0);
  if (b == 0) {
    // moment multipliers of each velocity (1, p, p_a p_b, p^2 p), the A operand of the
    // moment contraction, in operand order: for the wave of velocities 64 w .. 64 w + 63,
    // operand t of lane l is multiplier l % 16 of velocity 64 w + 4 t + l / 16, stored
    // [w][t / 2][l][t % 2] so that a lane reads two operands with one 16-byte load; zero
    // past V (and for MAX_WAVES - 1 waves more, which whole idle waves read)
    const int n = ptab_blocks(sh.V) * 1024;
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
      const int w = idx >> 10, rem = idx & 1023, t = 2 * (rem >> 7) + (rem & 1), l = (rem >> 1) & 63;
      const int v = 64 * w + 4 * t + (l >> 4), q = l & 15;
      double val = 0.0;
      if (v < sh.V && q < NMOM) {
        const int i = v / sh.QyQz, jk = v - i * sh.QyQz, j = jk / sh.Qz, k = jk - j * sh.Qz;
        const double px = d.px[i], py = d.py[j], pz = d.pz[k], p2 = px * px + py * py + pz * pz;
        const double m[NMOM] = {1.0, px, py, pz, px * px, py * py, pz * pz, px * py, px * pz, py * pz,
                                p2 * px, p2 * py, p2 * pz};
        // in the reduced model (p_z = 0) phi takes the multipliers above, and chi = int f p_z^2
        // dp_z carries p_z^2 (for P_zz) and p_z^2 p_a (for q_a), Eq. qdef with p_z integrated out
        const double mchi[NMOM] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, px, py, 0.0};
        val = (sh.reduced && k == 1) ? mchi[q] : m[q];
      }
      d.ptab[idx] = val;
    }
  }
  __syncthreads();
  double acc = 0.0;
  for (int v = threadIdx.x; v < sh.V; v += blockDim.x) {
    const int i = v / sh.QyQz, jk = v - i * sh.QyQz, j = jk / sh.Qz, k = jk - j * sh.Qz;
    const double gr = gx0[i] * gy0[j] * gz0[k];
    const double gw = gx0[i] * gyw[j] * gz0[k];
    d.g_rest[(size_t)b * sh.V + v] = gr;
    d.g_wall[(size_t)b * sh.V + v] = gw;
    if (i < sh.Qx && !(sh.reduced && k == 1)) acc += d.px[i] * gw;  // mass flux: phi only
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) d.inst[b].wall_den = red[0];
}

// F = n0 F^eq_rest (1 + eps r)
__global__ void init_state_kernel(Shape sh, DevPtrs d, const double* __restrict__ r, double eps) {
  const size_t total = (size_t)sh.B * sh.S * sh.V;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / ((size_t)sh.S * sh.V));
    const int v = (int)(idx % sh.V);
    double f = d.inst[b].n0 * d.g_rest[(size_t)b * sh.V + v];
    if (r) f *= 1.0 + eps * r[idx];
    d.F[0][idx] = f;
  }
}

// the free-molecular steady state of diffuse walls (the collisionless limit of Sec. IV, whose
// shear stress is Eq. Txy_bal): the populations leaving the wall at x = L/2 (p_x < 0) are
// n0 times its Maxwellian, those with p_x > 0 the bounce-back images of these (the
// Maxwellian of the wall at -L/2), the same at every node
__global__ void fm_state_kernel(Shape sh, DevPtrs d) {
  const size_t total = (size_t)sh.B * sh.S * sh.V;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / ((size_t)sh.S * sh.V));
    const int v = (int)(idx % sh.V);
    const int i = v / sh.QyQz, jk = v - i * sh.QyQz, j = jk / sh.Qz, k = jk - j * sh.Qz;
    const int vm = ((2 * sh.Qx - 1 - i) * sh.Qy + (sh.Qy - 1 - j)) * sh.Qz + k;
    d.F[0][idx] = d.inst[b].n0 * d.g_wall[(size_t)b * sh.V + (i < sh.Qx ? v : vm)];
  }
}

// ---------------------------------------------------------------------------------------
// warm-start seed from a moment table (per node: n, ux, uy, uz, T, Pxx, Pyy, Pzz, Pxy, Pxz,
// Pyz, qx, qy, qz):  F = c F^eq(n, u, T) (1 + Pi_ab xi_a xi_b / (2 n T^2)
//                                       + (xi^2 / (5T) - 1) xi.q / (n T^2)),
// Pi_ab = P_ab - n T delta_ab, xi = p - u.  F^eq is the projected discrete equilibrium
// (Sec. III) and the heat-flux polynomial is that of the Shakhov factor (Eq. sdef) with
// 1 - Pr replaced by 1.  c = 1, or with preserve_mass the per-instance factor that gives
// the seed the mass of the equilibrium start, c = n0 sum_s dx_s / sum_s n_s dx_s (the
// scheme conserves mass, so the steady state is fixed by it).  An instance with a node that
// is not finite or has n <= 0 or T <= 0 is seeded with the equilibrium at rest instead
// (flags[b] = 1).  The factor c travels in nw[b], which the first closure of the next step
// recomputes before anything reads it.

constexpr int TAB = 14;

__global__ void __launch_bounds__(256) seed_check_kernel(Shape sh, DevPtrs d, const double* __restrict__ tab,
                                                         int preserve_mass) {
  const int b = blockIdx.x;
  int bad = 0;
  for (int idx = threadIdx.x; idx < sh.S * TAB; idx += blockDim.x) {
    const double x = tab[(size_t)b * sh.S * TAB + idx];
    const int c = idx % TAB;
    if (!isfinite(x) || ((c == 0 || c == 4) && !(x > 0.0))) bad = 1;
  }
  bad = __syncthreads_or(bad);
  __shared__ double red[2][256];
  double m = 0.0, len = 0.0;
  for (int s = threadIdx.x; s < sh.S; s += blockDim.x) {
    const double dx = 1.0 / d.inv_dx[(size_t)b * sh.S + s];
    m += tab[((size_t)b * sh.S + s) * TAB] * dx;
    len += dx;
  }
  red[0][threadIdx.x] = m;
  red[1][threadIdx.x] = len;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    d.flags[b] = bad;
    d.nw[b] = (preserve_mass && !bad) ? d.inst[b].n0 * red[1][0] / red[0][0] : 1.0;
  }
}

__global__ void __launch_bounds__(256) seed_kernel(Shape sh, DevPtrs d, const double* __restrict__ tab) {
  const int node = blockIdx.x, b = node / sh.S;
  double* F = d.F[0] + (size_t)node * sh.V;
  if (d.flags[b]) {
    const double n0 = d.inst[b].n0;
    for (int v = threadIdx.x; v < sh.V; v += blockDim.x) F[v] = n0 * d.g_rest[(size_t)b * sh.V + v];
    return;
  }
  __shared__ double gx[2 * QX_MAX], gy[QYZ_MAX], gz[QYZ_MAX];
  const double* t = tab + (size_t)node * TAB;
  const double n = t[0], ux = t[1], uy = t[2], uz = t[3], T = t[4], scale = d.nw[b];
  {
    double I[NX_MAX + 1], Jp[NX_MAX + 1], Jm[NX_MAX + 1], ay[NYZ_MAX + 1], az[NYZ_MAX + 1];
    half_gauss_moments(ux, T, I);
    half_projection(d.cx, sh.Nx, I, Jp);
    half_gauss_moments(-ux, T, I);
    half_projection(d.cx, sh.Nx, I, Jm);
    full_coeffs(uy, T, ay);
    full_coeffs(uz, T, az);
    for (int i = threadIdx.x; i < 2 * sh.Qx; i += blockDim.x)
      gx[i] = scale * n * gx_node(d.phix, sh.Qx, sh.Nx, i, Jp, Jm);
    for (int j = threadIdx.x; j < sh.Qy; j += blockDim.x) gy[j] = full_node(d.phiy, sh.Ny, j, ay);
    for (int k = threadIdx.x; k < sh.Qz; k += blockDim.x) gz[k] = full_node(d.phiz, sh.Nz, k, az);
  }
  __syncthreads();
  const double nT = n * T, c2 = 0.5 / (nT * T), c3 = 1.0 / (nT * T), c5 = 1.0 / (5.0 * T);
  const double sxx = (t[5] - nT) * c2, syy = (t[6] - nT) * c2, szz = (t[7] - nT) * c2;
  const double sxy = 2.0 * t[8] * c2, sxz = 2.0 * t[9] * c2, syz = 2.0 * t[10] * c2;
  const double hx = t[11] * c3, hy = t[12] * c3, hz = t[13] * c3;
  for (int v = threadIdx.x; v < sh.V; v += blockDim.x) {
    const int i = v / sh.QyQz, jk = v - i * sh.QyQz, j = jk / sh.Qz, k = jk - j * sh.Qz;
    const double x = d.px[i] - ux, y = d.py[j] - uy, z = d.pz[k] - uz;
    const double stress = sxx * x * x + syy * y * y + szz * z * z + sxy * x * y + sxz * x * z + syz * y * z;
    const double heat = ((x * x + y * y + z * z) * c5 - 1.0) * (hx * x + hy * y + hz * z);
    F[v] = gx[i] * gy[j] * gz[k] * (1.0 + stress + heat);
  }
}

// fault flags and residuals of every instance to zero (a fill kernel rather than a memset,
// so a caller's graph capture records no memset node)
__global__ void clear_flags_kernel(int* flags, double* resid, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    flags[i] = 0;
    resid[i] = 0.0;
  }
}

// ---------------------------------------------------------------------------------------
// moment partials on the matrix cores
//
// The 13 moment sums of a node over a wave's 64 velocities are a dense contraction over
// the velocity axis: D[m][n] = sum_v P[v][m] F[n][v] for 16 nodes n at a time, with
// P[v][.] = {1, p_x, p_y, p_z, p_x^2, p_y^2, p_z^2, p_x p_y, p_x p_z, p_y p_z,
// |p|^2 p_x, |p|^2 p_y, |p|^2 p_z, 0, 0, 0}.  Each wave parks the 16 node rows of F it has
// produced in LDS and issues 16 v_mfma_f64_16x16x4 (K = 4 velocities each); the
// operand layouts are A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, and
// D[4r + l/16][l % 16] in lane l, result register r (checked on gfx950).

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int FT_LD = 65;                 // padded LDS row (doubles) of a wave's node tile
constexpr int FT_WAVE = 16 * FT_LD;       // doubles per wave tile
constexpr int RED_WAVE = 16 * 16;         // doubles per wave of reduced moments (moment x node)

// load this lane's A operands: a[t] = P[v0 + 4t + lane/16][lane % 16] (0 beyond V)
__device__ __forceinline__ void load_moment_operands(const double* __restrict__ ptab, int wave_v0, int V, int lane,
                                                     double* a) {
  (void)V;  // the table is zero past V
  typedef double pair_t __attribute__((ext_vector_type(2)));
  const auto p = gmem(reinterpret_cast<const pair_t*>(ptab) + (size_t)(wave_v0 >> 6) * 512 + lane);
#pragma unroll
  for (int t2 = 0; t2 < 8; ++t2) {
    const pair_t x = p[t2 * 64];
    a[2 * t2] = x.x;
    a[2 * t2 + 1] = x.y;
  }
}

// D[moment][node] = sum_v P[moment][v] F[v][node] over the wave's 64 velocities, in 16
// steps of 4: the multipliers are the A operand (lane l: moment l % 16, velocity
// 4 t + l / 16) and the node tile the B operand (lane l: velocity 4 t + l / 16, node
// l % 16), so register r of lane l ends up holding moment 4 r + l / 16 of node l % 16: the
// 16 lanes l / 16 = q of register r hold one moment of the group's 16 nodes
__device__ __forceinline__ dbl4 moment_mfma(const double* ft, const double* a, int lane) {
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  const int n = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int t = 0; t < 16; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], ft[n * FT_LD + 4 * t + kk], acc, 0, 0, 0);
  return acc;
}

// Moment sums of a group of 16 node rows, once every wave has stored its rows in its tile:
// the wave contracts its tile with the multipliers of its 64 velocities on the matrix
// cores (the multipliers loaded here; the stage kernel keeps them in registers instead);
// the 13 sums of node n end up in the lanes that hold D[.][n].  A block of one wave stores
// them straight from these registers; with more waves they are added across waves in LDS
// first.
__device__ __forceinline__ dbl4 moment_contract(const double* lds_ft, const double* __restrict__ ptab, int wave_v0,
                                                int V, int wave, int lane) {
  double a[16];
  load_moment_operands(ptab, wave_v0, V, lane, a);
  __syncthreads();
  return moment_mfma(lds_ft + wave * FT_WAVE, a, lane);
}

// park a wave's contraction in lds_red[wave][moment][node] (blocks of several waves)
__device__ __forceinline__ void park_moments(double* lds_red, const dbl4& acc, int wave, int lane) {
  double* r = lds_red + wave * RED_WAVE + lane;
  r[0] = acc[0];
  r[64] = acc[1];
  r[128] = acc[2];
  r[192] = acc[3];
}

// store the moment sums of the cnt nodes s, s + 1, .. of an instance into its partials
// (part: the instance's first group at this velocity block; gstride: doubles from one
// 16-node group to the next), from the registers of a one-wave block (register r of lane l
// holds moment 4 r + l / 16 of node l % 16) or from the waves' parked contractions summed
// in LDS.  Node s + n goes to slot (s + n) % 16 of group (s + n) / 16, so with s a multiple
// of 16 and cnt = 16 each moment is one whole 128-byte line and a store instruction writes
// four of them (lines written in part, or in several pieces, cost measurably more); 13
// lines per group, none of them padding.
__device__ __forceinline__ void store_moments(const dbl4& acc, const double* lds_red, int waves, int cnt,
                                              double* __restrict__ part, size_t gstride, int s) {
  if (waves == 1) {
    const int lane = threadIdx.x, n = lane & 15, m0 = lane >> 4;
    const int sn = s + n;
    auto o = gmem(part + (size_t)(sn >> 4) * gstride + 16 * m0 + (sn & 15));
    if (n < cnt) {
#pragma unroll
      for (int r = 0; r < 3; ++r) o[64 * r] = acc[r];
      if (m0 == 0) o[64 * 3] = acc[3];  // moment 12; 13..15 are zero
    }
    return;
  }
  for (int idx = threadIdx.x; idx < PART_GROUP; idx += blockDim.x) {
    const int m = idx >> 4, n = idx & 15, sn = s + n;
    if (n >= cnt) continue;
    double v = 0.0;
    for (int w = 0; w < waves; ++w) v += lds_red[w * RED_WAVE + idx];
    gmem(part)[(size_t)(sn >> 4) * gstride + 16 * m + (sn & 15)] = v;
  }
}

// the partials of instance b at velocity block vb (the first group's first line)
__device__ __forceinline__ double* part_base(const DevPtrs& d, int S, int b, int vb, int nvb) {
  return d.partials + ((size_t)b * part_groups(S) * nvb + vb) * PART_GROUP;
}

// LDS of the stage and partials kernels (doubles): the waves' node tiles, then (blocks of
// several waves) two buffers of parked contractions, then two residual sums per wave
__host__ __device__ inline int lds_red_offset(int waves) { return waves * FT_WAVE; }
__host__ __device__ inline int lds_res_offset(int waves) { return waves * FT_WAVE + (waves > 1 ? 2 * waves * RED_WAVE : 0); }

__global__ void __launch_bounds__(256) partials_kernel(Shape sh, DevPtrs d, const double* __restrict__ F, int nvb,
                                                       int nch, int cs) {
  extern __shared__ double lds[];
  const int waves = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* lds_ft = lds;
  double* lds_red = lds + lds_red_offset(waves);
  int t = xcd_tile(blockIdx.x, gridDim.x);
  const int ch = t % nch;
  t /= nch;
  const int vb = t % nvb, b = t / nvb;
  const int S = sh.S, V = sh.V;
  const int v = vb * blockDim.x + threadIdx.x;
  const bool active = v < V;
  const int wave_v0 = vb * blockDim.x + wave * 64;
  const int s0 = ch * cs;
  const int nloc = min(cs, S - s0);
  const double* Fb = F + (size_t)b * S * V;
  double* ft = lds_ft + wave * FT_WAVE;
  double* part = part_base(d, S, b, vb, nvb);
  const size_t gstride = (size_t)nvb * PART_GROUP;
  for (int g = 0; g < nloc; g += 16) {
    const int cnt = min(16, nloc - g);
    for (int u = 0; u < 16; ++u) ft[u * FT_LD + lane] = (u < cnt && active) ? Fb[(size_t)(s0 + g + u) * V + v] : 0.0;
    const dbl4 acc = moment_contract(lds_ft, d.ptab, wave_v0, V, wave, lane);
    if (waves > 1) {
      park_moments(lds_red, acc, wave, lane);
      __syncthreads();
    }
    store_moments(acc, lds_red, waves, cnt, part, gstride, s0 + g);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// closure: up to CL_NODES = 16 nodes per 64-lane block (one lane per node for the scalar
// closure, one per node and semi-axis for the half-range projections, four per node and
// moment for the partial sums), plus one wall block per instance


// one closure work item: node block `blk` (< node_blocks) or the wall of instance
// blk - node_blocks; 64 threads; cl_lds holds the closure LDS (size closure_lds_doubles)
__device__ __forceinline__ void closure_block(const Shape& sh, const DevPtrs& d, const double* __restrict__ Fin,
                                              int nvb, double* __restrict__ mom_out, int blk, int node_blocks, int nb,
                                              double* cl_lds) {
  const int S = sh.S;
  const int lane = threadIdx.x;
  if (blk >= node_blocks) {
    // wall density: zero net mass flux through x = L/2 (App. A.4); the outgoing fluxes
    // (p_x > 0) use the extrapolated ghosts, the incoming ones are p_x n_w F^eq_w exactly.
    const int b = blk - node_blocks;
    const auto in = gmem(d.inst + b);
    const int V = sh.V;
    const auto F = gmem(Fin + (size_t)b * S * V);
    double ex[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) ex[q] = in->ex[q];
    double acc = 0.0;
    // four velocities per lane and pass, their twelve loads issued before any is used
    for (int v0 = sh.Qx * sh.QyQz + lane; v0 < V; v0 += 256) {
      double px[4], f1[4], f2[4], f3[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int v = min(v0 + 64 * k, V - 1);
        // mass flux: every population, or phi alone in the reduced model (odd v are chi)
        px[k] = (v0 + 64 * k < V && !(sh.reduced && (v & 1))) ? gmem(d.px)[v / sh.QyQz] : 0.0;
        f3[k] = F[(size_t)(S - 3) * V + v];
        f2[k] = F[(size_t)(S - 2) * V + v];
        f1[k] = F[(size_t)(S - 1) * V + v];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double g0 = ex[0] * f1[k] + ex[1] * f2[k] + ex[2] * f3[k];
        const double g1 = ex[3] * g0 + ex[4] * f1[k] + ex[5] * f2[k];
        const double r = (sh.scheme == 1)   ? weno5(f3[k], f2[k], f1[k], g0, g1)
                         : (sh.scheme == 2) ? linear5(f3[k], f2[k], f1[k], g0, g1)
                                            : (1.5 * f1[k] - 0.5 * f2[k]);
        acc += px[k] * r;
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      const double nw = -acc / in->wall_den;
      gmem(d.nw)[b] = nw;
      if (!(nw > 0.0) || !isfinite(nw)) gmem(d.flags)[b] = 1;
    }
    return;
  }
  // LDS (sizes of this velocity set): moment sums, per-node coefficients, projection
  // tables, per-node g_y and g_z
  const int nphx = sh.Qx * (sh.Nx + 1), nphy = sh.Qy * (sh.Ny + 1), nphz = sh.Qz * (sh.Nz + 1);
  const int oJm = sh.Nx + 1, oay = 2 * (sh.Nx + 1), oaz = oay + sh.Ny + 1, SC = oaz + sh.Nz + 1;
  const int Qyz = sh.Qy + sh.Qz;
  const int ncx = (sh.Nx + 1) * (sh.Nx + 1);
  double* msum = cl_lds;
  double* scal = msum + nb * PART_STRIDE;
  double* phix = scal + nb * SC;
  double* phiy = phix + nphx;
  double* phiz = phiy + nphy;
  double* gyz = phiz + nphz;
  double* cxl = gyz + nb * Qyz;
  const int total = sh.B * S;
  const int g0 = blk * nb;
  const int nblk_nodes = min(nb, total - g0);
  // Every load of a phase is issued before any of its results is used: the block's time
  // is a chain of memory round trips, so each phase should cost one.  The parameters of
  // each lane's node (its instance's collision law, dt, and 1 / dx of the node) are loaded
  // first, so that they arrive with the partial sums.
  const bool live = lane < nblk_nodes;
  const int g = g0 + (live ? lane : 0), b = g / S;
  const auto in = gmem(d.inst + b);
  const double p_law = in->law, p_kn = in->kn, p_om = in->omega, p_su = in->suth;
  const double p_cl = in->collisionless, p_pr = in->pr, p_dt = in->dt;
  const double p_idx = gmem(d.inv_dx)[g];
  // 0) the projection tables (and the half-range monomial coefficients) into LDS.  The
  //    first 256 entries (all of them for Qx <= 28 at N = 6) are loaded into registers here
  //    and written to LDS only after the partial sums below, so their loads overlap
  //    those of the sums instead of costing a round trip of their own.
  const int n1 = nphx, n2 = n1 + nphy, n3 = n2 + nphz, n4 = n3 + ncx;
  auto table_entry = [&](int e) -> double {
    return (e < n1)   ? gmem(d.phix)[e]
           : (e < n2) ? gmem(d.phiy)[e - n1]
           : (e < n3) ? gmem(d.phiz)[e - n2]
           : (e < n4) ? gmem(d.cx)[e - n3]
                      : 0.0;
  };
  auto table_store = [&](int e, double x) {
    if (e < n3) phix[e] = x;  // phix, phiy, phiz are contiguous in LDS
    else if (e < n4) cxl[e - n3] = x;
  };
  double tab[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) tab[k] = table_entry(lane + 64 * k);
  for (int e0 = lane + 256; e0 < n4; e0 += 64) table_store(e0, table_entry(e0));
  // 1) sum the moment partials over velocity blocks: lane l owns node l % 16 of the block
  //    and its moments l / 16 + 4 j, and sums four velocity blocks per pass for all of them
  //    at once; the 16 lanes of one moment read one line when the block's nodes are one
  //    16-node group of an instance.  Each partial is read once, so the loads are
  //    nontemporal
  static_assert(CL_NODES <= 16, "one lane per node in the partial sums");
  {
    const int nd = lane & 15, m0 = lane >> 4;
    const bool okn = nd < nblk_nodes;
    const int gn = g0 + (okn ? nd : 0), bn = gn / S, sn = gn - bn * S;
    const auto src = gmem(part_base(d, S, bn, 0, nvb) + (size_t)(sn >> 4) * nvb * PART_GROUP + 16 * m0 + (sn & 15));
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int vb0 = 0; vb0 < nvb; vb0 += 4) {
      double x[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool ok = okn && m0 + 4 * j < NMOM;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          x[j][t] = (ok && vb0 + t < nvb) ? __builtin_nontemporal_load(&src[(size_t)(vb0 + t) * PART_GROUP + 64 * j]) : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] += (x[j][0] + x[j][1]) + (x[j][2] + x[j][3]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (nd < nb && m0 + 4 * j < NMOM) msum[nd * PART_STRIDE + m0 + 4 * j] = acc[j];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) table_store(lane + 64 * k, tab[k]);
  __syncthreads();
  // 2) one lane per node: moments, tau, Shakhov coefficients, full-range projection
  //    coefficients; n, u_x and T go to the three spare slots of the node's sum row
  static_assert(PART_STRIDE >= NMOM + 3, "the sum row carries n, u_x and T after the moments");
  double* M = msum + (live ? lane : 0) * PART_STRIDE;
  const double n = live ? M[0] : 1.0;
  const double ux = live ? M[1] / n : 0.0, uy = live ? M[2] / n : 0.0, uz = live ? M[3] / n : 0.0;
  const double Pxx = M[4] - n * ux * ux, Pyy = M[5] - n * uy * uy, Pzz = M[6] - n * uz * uz;
  const double Pxy = M[7] - n * ux * uy, Pxz = M[8] - n * ux * uz, Pyz = M[9] - n * uy * uz;
  const double T = live ? (Pxx + Pyy + Pzz) / (3.0 * n) : 1.0;
  // q_a = 1/2 sum F |p - u|^2 (p_a - u_a), expanded over the raw sums
  const double M2 = M[4] + M[5] + M[6];
  const double u2 = ux * ux + uy * uy + uz * uz;
  const double qx = 0.5 * (M[10] - ux * M2 - 2.0 * (ux * M[4] + uy * M[7] + uz * M[8]) + 2.0 * n * u2 * ux);
  const double qy = 0.5 * (M[11] - uy * M2 - 2.0 * (ux * M[7] + uy * M[5] + uz * M[9]) + 2.0 * n * u2 * uy);
  const double qz = 0.5 * (M[12] - uz * M2 - 2.0 * (ux * M[8] + uy * M[9] + uz * M[6]) + 2.0 * n * u2 * uz);
  const bool bad = !(n > 0.0) || !(T > 0.0) || !isfinite(n + T + ux + uy + uz + qx + qy + qz);
  double* sc = scal + lane * SC;
  if (live) {
    if (mom_out) {
      const auto o = gmem(mom_out + (size_t)g * 14);
      o[0] = n;
      o[1] = ux;
      o[2] = uy;
      o[3] = uz;
      o[4] = T;
      o[5] = Pxx;
      o[6] = Pyy;
      o[7] = Pzz;
      o[8] = Pxy;
      o[9] = Pxz;
      o[10] = Pyz;
      o[11] = qx;
      o[12] = qy;
      o[13] = qz;
    }
    if (bad) gmem(d.flags)[b] = 1;
    // relaxation time from mu = tau n T
    double tau;
    if (p_law == 0.0)
      tau = p_kn * pow(T, p_om - 1.0) / n;
    else if (p_law == 1.0)
      tau = p_kn * (1.0 + p_su) / (n * sqrt(T) * (1.0 + p_su / T));
    else
      tau = p_kn * M_SQRT1_2;  // linearised (low Mach) regime, Eq. knLuo: tau = k / sqrt(2)
    const double invtau = (p_cl != 0.0 || bad) ? 0.0 : 1.0 / tau;
    // Shakhov factor (Eq. sdef) S = (1 - Pr) (xi^2 / 5T - 1) xi.q / (n T^2), kept as
    // (xi^2 - 5T) xi.q' with q' = (1 - Pr) q / (5 n T^3); q' = 0 for Pr = 1 (BGK)
    // (zero at a node that failed the checks, whose populations then stay finite)
    const double a_sh = bad ? 0.0 : (1.0 - p_pr) / (n * T * T * (5.0 * T));
    const auto rec = gmem(d.rec + (size_t)g * sh.rec_len);
    rec[0] = ux;
    rec[1] = uy;
    rec[2] = uz;
    rec[3] = p_dt * invtau;
    rec[4] = bad ? 0.0 : 5.0 * T;
    rec[5] = 0.0;
    rec[6] = a_sh * qx;
    rec[7] = a_sh * qy;
    rec[8] = a_sh * qz;
    rec[9] = p_dt * p_idx;
    // projection coefficients of the 1D Maxwellian factors (Sec. III)
    double a[NYZ_MAX + 1];
    const double Tc = bad ? 1.0 : T;
    M[NMOM] = n;
    M[NMOM + 1] = ux;
    M[NMOM + 2] = Tc;
    full_coeffs(uy, Tc, a);
#pragma unroll
    for (int l = 0; l <= NYZ_MAX; ++l)
      if (l <= sh.Ny) sc[oay + l] = a[l];
    full_coeffs(uz, Tc, a);
#pragma unroll
    for (int l = 0; l <= NYZ_MAX; ++l)
      if (l <= sh.Nz) sc[oaz + l] = a[l];
  }
  __syncthreads();
  // 3) the half-range projection coefficients n J^+ and n J^-, one lane per node and
  //    semi-axis (the two share one pass through the exponential and erfc), and g_y and g_z
  //    of every node of the block
  //    (at most 2 x CL_NODES tasks, one pass of the block's 64 lanes)
  static_assert(2 * CL_NODES <= 64, "one pass covers every (node, semi-axis) task");
  auto half_pair = [&](int t) {
    if (t < 2 * nblk_nodes) {
      const int nd = t >> 1;
      const double* R = msum + nd * PART_STRIDE;
      double I[NX_MAX + 1], J[NX_MAX + 1];
      half_gauss_moments((t & 1) ? -R[NMOM + 1] : R[NMOM + 1], R[NMOM + 2], I);
      half_projection(cxl, sh.Nx, I, J);
      double* o = scal + nd * SC + ((t & 1) ? oJm : 0);
#pragma unroll
      for (int l = 0; l <= NX_MAX; ++l)
        if (l <= sh.Nx) o[l] = R[NMOM] * J[l];
    }
  };
  half_pair(lane);
  for (int idx = lane; idx < nblk_nodes * Qyz; idx += 64) {
    const int nd = idx / Qyz, e = idx - nd * Qyz;
    const double* sn = scal + nd * SC;
    gyz[nd * Qyz + e] = (e < sh.Qy)   ? full_node(phiy, sh.Ny, e, sn + oay)
                        : sh.reduced ? (e == sh.Qy ? 1.0 : msum[nd * PART_STRIDE + NMOM + 2])  // 1 for phi, T for chi
                                     : full_node(phiz, sh.Nz, e - sh.Qy, sn + oaz);
  }
  __syncthreads();
  // 4) the coalesced fill of the equilibrium tables, n g_x on the 2Qx nodes, then g_y g_z on
  //    the QyQz pairs (two loops, so that no pass mixes the two kinds of entry).  (node, entry)
  //    of lane l advance by 64 entries per pass without a division; the pair (j, k) of a
  //    g_y g_z entry comes from a float reciprocal, corrected to the exact quotient
  const int nx2 = 2 * sh.Qx, QyQz = sh.QyQz;
  {
    int nd = lane / nx2, e = lane - nd * nx2;
    while (nd < nblk_nodes) {
      const double* sn = scal + nd * SC;
      gmem(d.rec)[(size_t)(g0 + nd) * sh.rec_len + REC_HEAD + e] = gx_node(phix, sh.Qx, sh.Nx, e, sn, sn + oJm);
      e += 64;
      while (e >= nx2) {
        e -= nx2;
        ++nd;
      }
    }
  }
  {
    const float inv_qz = 1.0f / (float)sh.Qz;
    int nd = lane / QyQz, jk = lane - nd * QyQz;
    while (nd < nblk_nodes) {
      int j = (int)((float)jk * inv_qz);
      if (j * sh.Qz > jk) --j;
      if ((j + 1) * sh.Qz <= jk) ++j;
      const int k = jk - j * sh.Qz;
      gmem(d.rec)[(size_t)(g0 + nd) * sh.rec_len + REC_HEAD + nx2 + jk] = gyz[nd * Qyz + j] * gyz[nd * Qyz + sh.Qy + k];
      jk += 64;
      while (jk >= QyQz) {
        jk -= QyQz;
        ++nd;
      }
    }
  }
}

__global__ void __launch_bounds__(64) closure_kernel(Shape sh, DevPtrs d, const double* __restrict__ Fin, int nvb,
                                                     double* __restrict__ mom_out, int node_blocks, int nb) {
  extern __shared__ double cl_lds[];
  closure_block(sh, d, Fin, nvb, mom_out, blockIdx.x, node_blocks, nb, cl_lds);
}

// doubles of closure LDS for nb nodes per block
static inline size_t closure_lds_doubles(const Shape& sh, int nb) {
  return (size_t)nb * PART_STRIDE + (size_t)nb * (2 * (sh.Nx + 1) + sh.Ny + sh.Nz + 2) + (size_t)sh.Qx * (sh.Nx + 1) +
         (size_t)sh.Qy * (sh.Ny + 1) + (size_t)sh.Qz * (sh.Nz + 1) + (size_t)nb * (sh.Qy + sh.Qz) +
         (size_t)(sh.Nx + 1) * (sh.Nx + 1);
}

// nodes per closure block: CL_NODES, fewer when there are few nodes, so the grid keeps
// several thousand blocks.  Timed on the benchmark batch (65 536 nodes) and on the reduced
// model's (262 144 nodes): 16 is the fastest on both (8, 32 and 64 take 1.05-1.37x and
// 1.09-1.47x as long; a block of 64 nodes needs 27 KB of LDS, five blocks per CU)
static inline int closure_nodes_per_block(int total_nodes) {
  int nb = CL_NODES;
  while (nb > 4 && (total_nodes + nb - 1) / nb < 4096) nb >>= 1;
  return nb;
}

// ---------------------------------------------------------------------------------------
// the stage kernel

// value of node c for a thread's velocity before ghost completion: interior nodes are
// loaded, nodes left of the centre line are the bounce-back images of nodes 1..3
// (Eq. widetildei: F_{1-m; i j k} = F_{m; i~ j~ k}), nodes beyond the wall are 0 here.
// vcl is the thread's velocity clamped into [0, V).
__device__ __forceinline__ double raw_node(const double* __restrict__ Fb, int c, int S, int V, int vcl, int vm) {
  // branch- and select-free: every lane always issues one load from a valid address (nodes
  // beyond the wall read node S-1; ghost_node replaces them), so the number of outstanding
  // vector loads is the same on every path and prefetches stay in flight across iterations.
  // Lanes beyond V read a valid velocity; their results are never stored or summed.
  const int node = (c < 0) ? (-c - 1) : min(c, S - 1);
  const int vel = (c < 0) ? vm : vcl;
  return gmem(Fb)[(size_t)node * V + vel];
}

// buffer resource over an instance's array (raw, unbounded: every offset the kernels form is
// clamped into the array) and a load at a wave-uniform byte offset (scalar register) plus a
// fixed per-lane byte offset; both offsets are 32-bit, which holds because the host keeps
// one instance's state below 4 GiB
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const double* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, -1, 0x00020000);
}

__device__ __forceinline__ double ld_buf(__amdgpu_buffer_rsrc_t r, unsigned lane_off, unsigned row_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, row_off, 0));
}

// the same load marked nontemporal (cache-policy operand 2: the nt bit), for the streams a
// launch reads once: the caches then keep the node records and moment partials, which are
// read again
__device__ __forceinline__ double ld_buf_nt(__amdgpu_buffer_rsrc_t r, unsigned lane_off, unsigned row_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, row_off, 2));
}

// complete a node beyond the wall (App. A.4): p_x > 0 by quadratic extrapolation from the
// three nodes below (f1 nearest), p_x < 0 the wall Maxwellian n_w F^eq_w; nodes past
// the third ghost are never read.  The extrapolation weights (uniform) are read by scalar
// loads on the ghost path only, so they hold no registers on the interior march.
__device__ __forceinline__ double ghost_node(double raw, int c, int S, bool pos, double f1, double f2, double f3,
                                             const double* ex, double ghost_in) {
  typedef __attribute__((address_space(4))) const double cdouble;
  if (c < S) return raw;
  const cdouble* e = (const cdouble*)ex;
  if (c == S) return pos ? e[0] * f1 + e[1] * f2 + e[2] * f3 : ghost_in;
  if (c == S + 1) return pos ? e[3] * f1 + e[4] * f2 + e[5] * f3 : ghost_in;
  return pos ? 0.0 : ghost_in;
}

template <int SCHEME>
__device__ __forceinline__ double stencil_flux(bool pos, double px, double w0, double w1, double w2, double w3,
                                               double w4, double w5) {
  // upwind-ordered stencil of the interface between w2 and w3 (nodes c, c+1):
  // p_x > 0: (c-2 .. c+2); p_x < 0: mirrored (c+3 .. c-1)
  const double a = pos ? w0 : w5, b = pos ? w1 : w4, c = pos ? w2 : w3, dd = pos ? w3 : w2, e = pos ? w4 : w1;
  return px * interp<SCHEME>(a, b, c, dd, e);
}

// one tile: instance b, velocity block vb (64 * waves velocities), node chunk ch (cs nodes)
// depth of the stage kernel's load pipeline (nodes ahead); divides 16
constexpr int PIPE = 4;

// RED: the reduced (phi, chi) model of Sec. III (Eqs. reduced_def, boltz_red, sred_def), the
// z index being the component (0: phi, 1: chi) and p_z absent
template <int SCHEME, int STAGE, bool RED>
__device__ __forceinline__ void stage_tile(const Shape& sh, const DevPtrs& d, const double* __restrict__ Fin,
                                           const double* Fl, double* Fout, int b, int vb, int ch, int nvb, int nch,
                                           int cs, double* lds) {
  const int waves = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* lds_ft = lds;
  double* lds_red = lds + lds_red_offset(waves);
  double* lds_res = lds + lds_res_offset(waves);
  const int S = sh.S, V = sh.V, Qx = sh.Qx;
  const int v = vb * blockDim.x + threadIdx.x;
  const bool active = v < V;
  const int vv = active ? v : V - 1;
  const int i = vv / sh.QyQz, jk = vv - i * sh.QyQz, j = jk / sh.Qz, k = jk - j * sh.Qz;
  const double px = gmem(d.px)[i], py = gmem(d.py)[j], pz = gmem(d.pz)[k];
  // reduced Shakhov factors (Eq. sred_def): integrating (xi^2 / 5T - 1) over p_z against the
  // Maxwellian leaves xi_perp^2 / 5T - 4/5 for phi and xi_perp^2 / 5T - 2/5 for chi (the
  // p_z^2 and p_z^4 moments T and 3 T^2), so the constant term of Eq. sdef is scaled by
  // 4/5 or 2/5 (negated here: the factor is formed as xi_perp^2 + cneg 5T)
  const double cneg = RED ? (k == 0 ? -0.8 : -0.4) : -1.0;
  const bool pos = px > 0.0;
  const int vm = ((2 * Qx - 1 - i) * sh.Qy + (sh.Qy - 1 - j)) * sh.Qz + k;  // bounce-back partner
  const size_t base = (size_t)b * S * V;
  const double* Fb = Fin + base;
  const InstDev* in = d.inst + b;
  const double* ex = in->ex;
  const double ghost_in = active ? gmem(d.nw)[b] * gmem(d.g_wall)[(size_t)b * V + vv] : 0.0;
  const int wave_v0 = vb * blockDim.x + wave * 64;
  const int s0 = ch * cs;
  const int nloc = min(cs, S - s0);
  const double* recb = d.rec + (size_t)b * S * sh.rec_len;
  double* ft = lds_ft + wave * FT_WAVE;
  double* part = part_base(d, S, b, vb, nvb);
  const size_t gstride = (size_t)nvb * PART_GROUP;

  // window W0..W5 = nodes c-2 .. c+3, first for c = s0 - 1
  double W0 = raw_node(Fb, s0 - 3, S, V, vv, vm);
  double W1 = raw_node(Fb, s0 - 2, S, V, vv, vm);
  double W2 = raw_node(Fb, s0 - 1, S, V, vv, vm);
  double W3 = raw_node(Fb, s0, S, V, vv, vm);
  double W4 = raw_node(Fb, s0 + 1, S, V, vv, vm);
  double W5 = raw_node(Fb, s0 + 2, S, V, vv, vm);
  W3 = ghost_node(W3, s0, S, pos, W2, W1, W0, ex, ghost_in);
  W4 = ghost_node(W4, s0 + 1, S, pos, W3, W2, W1, ex, ghost_in);
  W5 = ghost_node(W5, s0 + 2, S, pos, W4, W3, W2, ex, ghost_in);
  double fl = stencil_flux<SCHEME>(pos, px, W0, W1, W2, W3, W4, W5);

  // Per-node operands, software-pipelined in rotating register sets (the node loop is
  // unrolled by PIPE, so no register with a load in flight is ever copied).  The two HBM
  // streams, the window node c+3 and F_l (nontemporal loads), and the two equilibrium-factor
  // gathers (which hit the cache) run PIPE nodes ahead.  All are unconditional vector loads with clamped
  // addresses, which complete in order; each is a wave-uniform row offset in a scalar
  // register plus a fixed 32-bit lane offset, so no address arithmetic is repeated per lane
  // and node.  The node's closure scalars are uniform and come by scalar loads (ld_sc).
  struct Far {
    double raw, fl0;
  };
  struct Near {
    double gx, gyz;
  };
  // the node's closure scalars (record head: u, dt / tau, 5T, unused, the scaled heat flux
  // q', dt / dx), wave-uniform, read by scalar loads
  struct Sc {
    double ux, uy, uz, itau, t5, unused, qx, qy, qz, idx;
  };
  typedef __attribute__((address_space(4))) const double cdouble;
  const int clast = s0 + nloc - 1;
  // the last window row the chunk needs: the prefetches issued for nodes past the chunk's
  // end (never computed) re-read it instead of fetching the next chunk's rows from HBM
  const int rtop = min(clast + 3, S - 1);
  const int gx_off = REC_HEAD + i, gyz_off = REC_HEAD + 2 * Qx + jk;
  const unsigned vv8 = 8u * vv, gx8 = 8u * gx_off, gyz8 = 8u * gyz_off;
  const __amdgpu_buffer_rsrc_t r_in = raw_rsrc(Fb), r_rec = raw_rsrc(recb);
  const __amdgpu_buffer_rsrc_t r_l = raw_rsrc(STAGE != 1 ? Fl + base : Fb);
  const unsigned row8 = 8u * V, rec8 = 8u * sh.rec_len;
  auto ld_far = [&](int c, Far& o) {
    // c + 3 >= 3 on the march: never a bounce-back image
    o.raw = ld_buf_nt(r_in, vv8, row8 * min(c + 3, rtop));
    if constexpr (STAGE != 1)
      o.fl0 = ld_buf_nt(r_l, vv8, row8 * min(c, clast));
    else
      o.fl0 = 0.0;
  };
  auto ld_near = [&](int c, Near& o) {
    const unsigned ro = rec8 * min(c, clast);
    o.gx = ld_buf(r_rec, gx8, ro);
    o.gyz = ld_buf(r_rec, gyz8, ro);
  };
  auto ld_sc = [&](int c, Sc& o) {
    cdouble* r = (cdouble*)(recb + (size_t)min(c, clast) * sh.rec_len);
    o = Sc{r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7], r[8], r[9]};
  };
  double rd = 0.0, rf = 0.0;
  const double act = active ? 1.0 : 0.0;
  // one node: complete the window, flux, collision, RK combine, store; returns F_out
  auto node = [&](int c, const Far& o, const Near& p, const Sc& z, bool valid) -> double {
    const double Wn = ghost_node(o.raw, c + 3, S, pos, W5, W4, W3, ex, ghost_in);
    W0 = W1;
    W1 = W2;
    W2 = W3;
    W3 = W4;
    W4 = W5;
    W5 = Wn;
    const double fr = stencil_flux<SCHEME>(pos, px, W0, W1, W2, W3, W4, W5);
    const double D = (fr - fl) * z.idx;  // dt times Eq. flux
    fl = fr;
    const double F = W2;
    const double feq = p.gx * p.gyz;
    // F^eq (1 + S), Eq. sdef, with S = (xi^2 - 5T) xi.q' (the record holds 5T and q'); no
    // branch for BGK, whose q' = 0 gives FS = F^eq exactly
    double FS;
    if constexpr (RED) {
      (void)pz;
      const double xx = px - z.ux, xy = py - z.uy;
      const double xi2 = xx * xx + xy * xy;
      const double qxi = z.qx * xx + z.qy * xy;
      FS = feq + feq * (fma(cneg, z.t5, xi2) * qxi);  // phi^eq (1 + S_phi), T phi^eq (1 + S_chi)
    } else {
      (void)cneg;
      const double xx = px - z.ux, xy = py - z.uy, xz = pz - z.uz;
      const double xi2 = xx * xx + xy * xy + xz * xz;
      const double qxi = z.qx * xx + z.qy * xy + z.qz * xz;
      FS = feq + feq * ((xi2 - z.t5) * qxi);
    }
    const double G = F + (FS - F) * z.itau - D;  // F + dt L[F], Eq. L_def
    double out;
    if constexpr (STAGE == 1) {
      out = G;
    } else if constexpr (STAGE == 2) {
      out = 0.75 * o.fl0 + 0.25 * G;
    } else {
      // F_{l+1} = F_l / 3 + 2 G / 3, with the step's change F_{l+1} - F_l formed directly;
      // the residual sums take lanes below V at the chunk's nodes only (weight w = 1, else 0)
      const double dlt = (2.0 / 3.0) * (G - o.fl0);
      out = o.fl0 + dlt;
      const double w = act * (valid ? 1.0 : 0.0);  // the condition is uniform: no select per lane
      const double dm = dlt * w, flm = o.fl0 * w;
      rd += dm * dm;
      rf += flm * flm;
      // keep each node's update here: sunk to the end of the 16-node group, the updates
      // would hold every node's terms live and cost a wave per SIMD of occupancy
      asm volatile("" : "+v"(rd), "+v"(rf));
    }
    // nodes past the chunk's end give finite values (clamped loads) that are neither
    // stored nor summed; so do lanes past V (velocity V - 1), whose moment multipliers
    // are zero
    return out;
  };
  Far far[PIPE];
  Near near[PIPE];
  Sc sc;
#pragma unroll
  for (int k = 0; k < PIPE; ++k) {
    ld_far(s0 + k, far[k]);
    ld_near(s0 + k, near[k]);
  }

  dbl4 acc;
  // the contraction's B operands (the multipliers of the wave's 64 velocities) stay in
  // registers for the whole tile: eight 16-byte loads once instead of per group
  double pa[16];
  load_moment_operands(d.ptab, wave_v0, V, lane, pa);
  for (int g = 0; g < nloc; g += 16) {
    const int cnt = min(16, nloc - g);
    // the 16 nodes of a group as straight-line code: the load counter's state is then known
    // exactly at every wait, which a loop back-edge inside the group would blur into a full
    // drain.  The nodes past the chunk's end in a last, partial group are computed too, from
    // clamped (valid) addresses, and give zero: a guard around them would merge the sliding
    // window at every node and cost a register copy per window entry.
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int c = s0 + g + u;
      ld_sc(c, sc);
      const double out = node(c, far[u % PIPE], near[u % PIPE], sc, u < cnt);
      ft[u * FT_LD + lane] = out;
      // the prefetches are issued on every path (clamped addresses): a load under a branch
      // would have to be merged into one register at the join, and that copy would wait
      // for the load
      ld_far(c + PIPE, far[u % PIPE]);
      ld_near(c + PIPE, near[u % PIPE]);
    }
    // Stores happen only here, once per 16 nodes: the group's results from the wave's LDS
    // tile, then its moment sums.  Loads and stores share one counter, so a wait
    // issued while a store is in flight drains everything; with the stores bunched here
    // the march starts each group with its next operands already loaded.  Blocks of several
    // waves add their contractions in LDS, in one of two buffers taken in turn, so a single
    // barrier per group orders the parking and the summing (a wave cannot get a whole
    // group ahead of the others); blocks of one wave need no barrier.  The rows are stored
    // nontemporal, as the two streams are loaded: the next launch reads them back at the
    // earliest, and a batch's arrays outgrow the last-level cache, which then keeps the
    // moment partials and node records that the closure and the next stage read (measured:
    // 5-8 % off stage and closure together).
    // Each store instruction writes two node rows of the wave's 64 velocities, 16 bytes (two
    // velocities) per lane: half the store instructions of one row per instruction.  V is
    // even (2 Qx nodes on x), so a pair that starts below V ends below V.
    {
      typedef double pair_t __attribute__((ext_vector_type(2)));
      const int pl = lane & 31, h = lane >> 5, vp = wave_v0 + 2 * pl;
      if (vp < V) {
        auto dst = gmem(reinterpret_cast<pair_t*>(Fout + base + (size_t)(s0 + g + h) * V + vp));
        for (int u2 = 0; 2 * u2 + h < cnt; ++u2) {
          const int u = 2 * u2 + h;
          pair_t x;
          x.x = ft[u * FT_LD + 2 * pl];
          x.y = ft[u * FT_LD + 2 * pl + 1];
          __builtin_nontemporal_store(x, &dst[(size_t)u2 * V]);  // V pairs = two rows
        }
      }
    }
    acc = moment_mfma(lds_ft + wave * FT_WAVE, pa, lane);
    double* red = lds_red + ((g >> 4) & 1) * waves * RED_WAVE;
    if (waves > 1) {
      park_moments(red, acc, wave, lane);
      __syncthreads();
    }
    store_moments(acc, red, waves, cnt, part, gstride, s0 + g);
  }
  if constexpr (STAGE == 3) {
    rd = wave_sum(rd);
    rf = wave_sum(rf);
    if (lane == 0) {
      lds_res[2 * wave] = rd;
      lds_res[2 * wave + 1] = rf;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      double s = 0.0;
      for (int wv = 0; wv < waves; ++wv) s += lds_res[2 * wv + threadIdx.x];
      gmem(d.resid_part)[((size_t)b * nvb * nch + (size_t)vb * nch + ch) * 2 + threadIdx.x] = s;
    }
  }
}

// the stage kernels are held to three waves per SIMD (at most 168 VGPRs)
template <int SCHEME, int STAGE, bool RED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) stage_kernel(Shape sh, DevPtrs d, const double* __restrict__ Fin,
                                                    const double* Fl, double* Fout, int nvb, int nch, int cs) {
  extern __shared__ double lds[];
  int t = xcd_tile(blockIdx.x, gridDim.x);
  const int ch = t % nch;
  t /= nch;
  stage_tile<SCHEME, STAGE, RED>(sh, d, Fin, Fl, Fout, t / nvb, t % nvb, ch, nvb, nch, cs, lds);
}

// ---------------------------------------------------------------------------------------
// batched (ragged) launches: one grid serves the tiles of every group

template <int STAGE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) batch_stage_kernel(const GroupDesc* __restrict__ groups,
                                                          const int4* __restrict__ tiles, const int* __restrict__ ntiles) {
  extern __shared__ double lds[];
  // one block per tile; the grid is sized for every tile, blocks past the live count return
  const int t = blockIdx.x;
  if (t >= *ntiles) return;
  const int4 tl = tiles[t];
  const GroupDesc& g = groups[tl.x];
  const double* Fin = g.d.F[STAGE - 1];
  double* Fout = g.d.F[STAGE % 3];
  if (g.sh.reduced) {
    if (g.sh.scheme == 1)
      stage_tile<1, STAGE, true>(g.sh, g.d, Fin, g.d.F[0], Fout, tl.y, tl.z, tl.w, g.nvb, g.nch, g.cs, lds);
    else if (g.sh.scheme == 2)
      stage_tile<2, STAGE, true>(g.sh, g.d, Fin, g.d.F[0], Fout, tl.y, tl.z, tl.w, g.nvb, g.nch, g.cs, lds);
    else
      stage_tile<0, STAGE, true>(g.sh, g.d, Fin, g.d.F[0], Fout, tl.y, tl.z, tl.w, g.nvb, g.nch, g.cs, lds);
  } else if (g.sh.scheme == 1) {
    stage_tile<1, STAGE, false>(g.sh, g.d, Fin, g.d.F[0], Fout, tl.y, tl.z, tl.w, g.nvb, g.nch, g.cs, lds);
  } else if (g.sh.scheme == 2) {
    stage_tile<2, STAGE, false>(g.sh, g.d, Fin, g.d.F[0], Fout, tl.y, tl.z, tl.w, g.nvb, g.nch, g.cs, lds);
  } else {
    stage_tile<0, STAGE, false>(g.sh, g.d, Fin, g.d.F[0], Fout, tl.y, tl.z, tl.w, g.nvb, g.nch, g.cs, lds);
  }
}

__global__ void __launch_bounds__(64) batch_closure_kernel(const GroupDesc* __restrict__ groups,
                                                           const int2* __restrict__ items, const int* __restrict__ nitems,
                                                           int stage) {
  extern __shared__ double cl_lds[];
  // one block per item; the grid is sized for every item, blocks past the live count return
  const int t = blockIdx.x;
  if (t >= *nitems) return;
  const int2 it = items[t];
  const GroupDesc& g = groups[it.x];
  closure_block(g.sh, g.d, g.d.F[stage - 1], g.nvb, nullptr, it.y, g.node_blocks, g.nb, cl_lds);
}

__global__ void __launch_bounds__(256) residual_kernel(DevPtrs d, int nres) {
  const int b = blockIdx.x;
  __shared__ double r0[256], r1[256];
  double a = 0.0, f = 0.0;
  for (int k = threadIdx.x; k < nres; k += blockDim.x) {
    a += d.resid_part[((size_t)b * nres + k) * 2];
    f += d.resid_part[((size_t)b * nres + k) * 2 + 1];
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = f;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      r0[threadIdx.x] += r0[threadIdx.x + o];
      r1[threadIdx.x] += r1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) d.resid[b] = (r1[0] > 0.0) ? sqrt(r0[0]) / (d.inst[b].dt * sqrt(r1[0])) : 0.0;
}

// ---------------------------------------------------------------------------------------
// launchers

static inline int grid_tiles(const Shape& sh, int cells, int waves, int* nvb, int* nch) {
  *nvb = (sh.V + 64 * waves - 1) / (64 * waves);
  *nch = (sh.S + cells - 1) / cells;
  return sh.B * (*nvb) * (*nch);
}

int launch_setup_tables(const Shape& sh, const DevPtrs& d, void* stream) {
  hipLaunchKernelGGL(setup_tables_kernel, dim3(sh.B), dim3(256), 0, (hipStream_t)stream, sh, d);
  return (int)hipGetLastError();
}

int launch_init_state(const Shape& sh, const DevPtrs& d, const double* perturb, double eps, void* stream) {
  const size_t total = (size_t)sh.B * sh.S * sh.V;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(init_state_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, sh, d, perturb, eps);
  return (int)hipGetLastError();
}

int launch_fm_state(const Shape& sh, const DevPtrs& d, void* stream) {
  const size_t total = (size_t)sh.B * sh.S * sh.V;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(fm_state_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, sh, d);
  return (int)hipGetLastError();
}

int launch_seed(const Shape& sh, const DevPtrs& d, const double* tab, int preserve_mass, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(seed_check_kernel, dim3(sh.B), dim3(256), 0, st, sh, d, tab, preserve_mass);
  hipLaunchKernelGGL(seed_kernel, dim3(sh.B * sh.S), dim3(256), 0, st, sh, d, tab);
  return (int)hipGetLastError();
}

int launch_clear_flags(const Shape& sh, const DevPtrs& d, void* stream) {
  hipLaunchKernelGGL(clear_flags_kernel, dim3((sh.B + 255) / 256), dim3(256), 0, (hipStream_t)stream, d.flags, d.resid,
                     sh.B);
  return (int)hipGetLastError();
}

static size_t stage_lds_bytes(int waves) { return ((size_t)lds_res_offset(waves) + 2 * waves) * sizeof(double); }

int launch_partials(const Shape& sh, const DevPtrs& d, const double* F, int cells, int waves, void* stream) {
  int nvb, nch;
  const int nblk = grid_tiles(sh, cells, waves, &nvb, &nch);
  hipLaunchKernelGGL(partials_kernel, dim3(nblk), dim3(64 * waves), stage_lds_bytes(waves), (hipStream_t)stream, sh, d,
                     F, nvb, nch, cells);
  return (int)hipGetLastError();
}

int launch_closure(const Shape& sh, const DevPtrs& d, const double* Fin, int nvb, double* mom_out, void* stream) {
  const int total = sh.B * sh.S;
  const int nb = closure_nodes_per_block(total);
  const int node_blocks = (total + nb - 1) / nb;
  hipLaunchKernelGGL(closure_kernel, dim3(node_blocks + sh.B), dim3(64), closure_lds_doubles(sh, nb) * sizeof(double),
                     (hipStream_t)stream, sh, d, Fin, nvb, mom_out, node_blocks, nb);
  return (int)hipGetLastError();
}

template <int SCHEME, int STAGE, bool RED>
static int launch_stage_t(const Shape& sh, const DevPtrs& d, const double* Fin, const double* Fl, double* Fout,
                          int cells, int waves, void* stream) {
  int nvb, nch;
  const int nblk = grid_tiles(sh, cells, waves, &nvb, &nch);
  hipLaunchKernelGGL((stage_kernel<SCHEME, STAGE, RED>), dim3(nblk), dim3(64 * waves), stage_lds_bytes(waves),
                     (hipStream_t)stream, sh, d, Fin, Fl, Fout, nvb, nch, cells);
  return (int)hipGetLastError();
}

template <bool RED>
static int launch_stage_r(const Shape& sh, const DevPtrs& d, int stage, const double* Fin, const double* Fl,
                          double* Fout, int cells, int waves, void* stream) {
  if (sh.scheme == 1) {
    if (stage == 1) return launch_stage_t<1, 1, RED>(sh, d, Fin, Fl, Fout, cells, waves, stream);
    if (stage == 2) return launch_stage_t<1, 2, RED>(sh, d, Fin, Fl, Fout, cells, waves, stream);
    return launch_stage_t<1, 3, RED>(sh, d, Fin, Fl, Fout, cells, waves, stream);
  }
  if (sh.scheme == 2) {
    if (stage == 1) return launch_stage_t<2, 1, RED>(sh, d, Fin, Fl, Fout, cells, waves, stream);
    if (stage == 2) return launch_stage_t<2, 2, RED>(sh, d, Fin, Fl, Fout, cells, waves, stream);
    return launch_stage_t<2, 3, RED>(sh, d, Fin, Fl, Fout, cells, waves, stream);
  }
  if (stage == 1) return launch_stage_t<0, 1, RED>(sh, d, Fin, Fl, Fout, cells, waves, stream);
  if (stage == 2) return launch_stage_t<0, 2, RED>(sh, d, Fin, Fl, Fout, cells, waves, stream);
  return launch_stage_t<0, 3, RED>(sh, d, Fin, Fl, Fout, cells, waves, stream);
}

int launch_stage(const Shape& sh, const DevPtrs& d, int stage, const double* Fin, const double* Fl, double* Fout,
                 int cells, int waves, void* stream) {
  if (sh.reduced) return launch_stage_r<true>(sh, d, stage, Fin, Fl, Fout, cells, waves, stream);
  return launch_stage_r<false>(sh, d, stage, Fin, Fl, Fout, cells, waves, stream);
}

int launch_residual(const Shape& sh, const DevPtrs& d, int nres, void* stream) {
  hipLaunchKernelGGL(residual_kernel, dim3(sh.B), dim3(256), 0, (hipStream_t)stream, d, nres);
  return (int)hipGetLastError();
}

size_t stage_lds_bytes_for(int waves) { return stage_lds_bytes(waves); }
size_t closure_lds_bytes_for(const Shape& sh, int nb) { return closure_lds_doubles(sh, nb) * sizeof(double); }
int closure_nodes_for(int total_nodes) { return closure_nodes_per_block(total_nodes); }
int batch_closure_blocks_per_cu(size_t lds_bytes) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_closure_kernel, 64, lds_bytes) != hipSuccess || n < 1)
    return 8;
  return n;
}

int launch_batch_stage(int stage, const GroupDesc* groups, const void* tiles, const int* ntiles, int grid, int waves,
                       size_t lds_bytes, void* stream) {
  const int4* t = (const int4*)tiles;
  if (stage == 1)
    hipLaunchKernelGGL(batch_stage_kernel<1>, dim3(grid), dim3(64 * waves), lds_bytes, (hipStream_t)stream, groups, t,
                       ntiles);
  else if (stage == 2)
    hipLaunchKernelGGL(batch_stage_kernel<2>, dim3(grid), dim3(64 * waves), lds_bytes, (hipStream_t)stream, groups, t,
                       ntiles);
  else
    hipLaunchKernelGGL(batch_stage_kernel<3>, dim3(grid), dim3(64 * waves), lds_bytes, (hipStream_t)stream, groups, t,
                       ntiles);
  return (int)hipGetLastError();
}

int launch_batch_closure(int stage, const GroupDesc* groups, const void* items, const int* nitems, int grid,
                         size_t lds_bytes, void* stream) {
  hipLaunchKernelGGL(batch_closure_kernel, dim3(grid), dim3(64), lds_bytes, (hipStream_t)stream, groups,
                     (const int2*)items, nitems, stage);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// fixed work memory of hrlb_step_noalloc, for callers that cannot allocate device memory:
// one array per GPU, held until the process ends.  In host code the name `scratch` is a
// host-side stand-in, not a device address; every host use goes through the address that
// hipGetSymbolAddress returns for the current device (each GPU has its own copy at its own
// address), taken once per device and kept.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

int scratch_pointer(void** out) {
  constexpr int MAX_DEVICES = 64;
  static std::mutex mu;
  static void* ptr[MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= MAX_DEVICES) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!p) return (int)hipErrorInvalidSymbol;
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return (int)hipSuccess;
}

}  // namespace hrlb

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

// WENO-5 reconstruction at the interface downstream of c from the upwind-ordered
// stencil (a, b, c, d, e) (App. A.3; candidates of Eq. weno5_flux, indicators of
// Eq. weno_sigma, weights of Eq. weno5_omega without epsilon).  The weights
// (d_q / s_q^2) / sum_r (d_r / s_r^2) are evaluated as N_q / sum N with
// N_q = d_q prod_{r != q} t_r^2 and t_q = s_q / 2^e, 2^e the binade of max s: one
// division, exact power-of-two scaling (so the scheme stays homogeneous of degree one),
// and vanishing indicators give the Table II rows directly (one vanishing: N_q alone
// survives; two: the sum vanishes and the pair row is taken; three: ideal weights).
__device__ __forceinline__ double weno5(double a, double b, double c, double d, double e) {
  const double f1 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
  const double f2 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
  const double f3 = (2.0 * c + 5.0 * d - e) * (1.0 / 6.0);
  const double r1 = a - 2.0 * b + c, q1 = a - 4.0 * b + 3.0 * c;
  const double r2 = b - 2.0 * c + d, q2 = b - d;
  const double r3 = c - 2.0 * d + e, q3 = 3.0 * c - 4.0 * d + e;
  const double s1 = (13.0 / 12.0) * r1 * r1 + 0.25 * q1 * q1;
  const double s2 = (13.0 / 12.0) * r2 * r2 + 0.25 * q2 * q2;
  const double s3 = (13.0 / 12.0) * r3 * r3 + 0.25 * q3 * q3;
  const double smax = fmax(s1, fmax(s2, s3));
  if (smax == 0.0) return 0.1 * f1 + 0.6 * f2 + 0.3 * f3;
  int ex;
  (void)frexp(smax, &ex);
  const double t1 = ldexp(s1, -ex), t2 = ldexp(s2, -ex), t3 = ldexp(s3, -ex);
  const double u1 = t1 * t1, u2 = t2 * t2, u3 = t3 * t3;
  const double n1 = 0.1 * (u2 * u3), n2 = 0.6 * (u1 * u3), n3 = 0.3 * (u1 * u2);
  const double den = n1 + n2 + n3;
  if (den > 0.0) return (n1 * f1 + n2 * f2 + n3 * f3) / den;
  if (u1 == 0.0 && u2 == 0.0) return (1.0 / 7.0) * f1 + (6.0 / 7.0) * f2;
  if (u1 == 0.0 && u3 == 0.0) return 0.25 * f1 + 0.75 * f3;
  return (2.0 / 3.0) * f2 + (1.0 / 3.0) * f3;
}

template <int SCHEME>
__device__ __forceinline__ double interp(double a, double b, double c, double d, double e) {
  if constexpr (SCHEME == 1) {
    return weno5(a, b, c, d, e);
  } else {
    (void)a;
    (void)d;
    (void)e;
    return 1.5 * c - 0.5 * b;  // second-order upwind: (3 F_s - F_{s-1}) / 2
  }
}

// Half-range Gaussian moments I_k(u, T) = int_0^inf p^k G(p; u, T) dp, k <= NX_MAX:
// I_0 = erfc(-u / sqrt(2T)) / 2, I_1 = u I_0 + T G(0), I_k = u I_{k-1} + (k-1) T I_{k-2}.
__device__ __forceinline__ void half_gauss_moments(double u, double T, double* I) {
  const double G0 = exp(-u * u / (2.0 * T)) * rsqrt(2.0 * M_PI * T);
  I[0] = 0.5 * erfc(-u * rsqrt(2.0 * T));
  I[1] = u * I[0] + T * G0;
#pragma unroll
  for (int k = 2; k <= NX_MAX; ++k) I[k] = u * I[k - 1] + (k - 1) * T * I[k - 2];
}

// Coefficients J_l = int G h_l over one semi-axis (monic half-range h_l, l <= Nx).
__device__ __forceinline__ void half_projection(const double* __restrict__ cx, int Nx, const double* I, double* J) {
#pragma unroll
  for (int l = 0; l <= NX_MAX; ++l) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k <= NX_MAX; ++k)
      if (k <= l && l <= Nx) s += cx[l * (Nx + 1) + k] * I[k];
    J[l] = s;
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
  for (int k = threadIdx.x; k < sh.Qz; k += blockDim.x) gz0[k] = full_node(d.phiz, sh.Nz, k, a0);
  __syncthreads();
  double acc = 0.0;
  for (int v = threadIdx.x; v < sh.V; v += blockDim.x) {
    const int i = v / sh.QyQz, jk = v - i * sh.QyQz, j = jk / sh.Qz, k = jk - j * sh.Qz;
    const double gr = gx0[i] * gy0[j] * gz0[k];
    const double gw = gx0[i] * gyw[j] * gz0[k];
    d.g_rest[(size_t)b * sh.V + v] = gr;
    d.g_wall[(size_t)b * sh.V + v] = gw;
    if (i < sh.Qx) acc += d.px[i] * gw;
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

// ---------------------------------------------------------------------------------------
// moment partials: per (block, node) the 13 sums over the block's velocities of
// F {1, p_x, p_y, p_z, p_x^2, p_y^2, p_z^2, p_x p_y, p_x p_z, p_y p_z, |p|^2 p_x, |p|^2 p_y, |p|^2 p_z}

struct VelMul {
  double m[NMOM];
};

__device__ __forceinline__ VelMul velocity_multipliers(double px, double py, double pz, bool active) {
  VelMul r;
  const double p2 = px * px + py * py + pz * pz;
  r.m[0] = active ? 1.0 : 0.0;
  r.m[1] = active ? px : 0.0;
  r.m[2] = active ? py : 0.0;
  r.m[3] = active ? pz : 0.0;
  r.m[4] = active ? px * px : 0.0;
  r.m[5] = active ? py * py : 0.0;
  r.m[6] = active ? pz * pz : 0.0;
  r.m[7] = active ? px * py : 0.0;
  r.m[8] = active ? px * pz : 0.0;
  r.m[9] = active ? py * pz : 0.0;
  r.m[10] = active ? p2 * px : 0.0;
  r.m[11] = active ? p2 * py : 0.0;
  r.m[12] = active ? p2 * pz : 0.0;
  return r;
}

// wave-reduce the 13 weighted sums of f for node slot u and stash them in LDS
__device__ __forceinline__ void stash_moments(double f, const VelMul& vm, double* red, int wave, int u, int cs,
                                              int lane) {
#pragma unroll
  for (int q = 0; q < NMOM; ++q) {
    const double s = wave_sum(f * vm.m[q]);
    if (lane == 0) red[(wave * cs + u) * NMOM + q] = s;
  }
}

// sum the per-wave stashes over the block's waves and write the block's partials
__device__ __forceinline__ void flush_moments(const double* red, int waves, int cs, int nloc, double* __restrict__ out) {
  for (int idx = threadIdx.x; idx < nloc * NMOM; idx += blockDim.x) {
    const int u = idx / NMOM, q = idx - u * NMOM;
    double s = 0.0;
    for (int w = 0; w < waves; ++w) s += red[(w * cs + u) * NMOM + q];
    out[(size_t)u * PART_STRIDE + q] = s;
  }
}

template <int CS>
__global__ void __launch_bounds__(1024) partials_kernel(Shape sh, DevPtrs d, const double* __restrict__ F, int nvb,
                                                        int nch) {
  extern __shared__ double red[];
  int t = xcd_tile(blockIdx.x, gridDim.x);
  const int ch = t % nch;
  t /= nch;
  const int vb = t % nvb, b = t / nvb;
  const int S = sh.S, V = sh.V;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, waves = blockDim.x >> 6;
  const int v = vb * blockDim.x + threadIdx.x;
  const bool active = v < V;
  const int vv = active ? v : V - 1;
  const int i = vv / sh.QyQz, jk = vv - i * sh.QyQz, j = jk / sh.Qz, k = jk - j * sh.Qz;
  const VelMul vm = velocity_multipliers(d.px[i], d.py[j], d.pz[k], active);
  const int s0 = ch * CS;
  const int nloc = min(CS, S - s0);
  const double* Fb = F + (size_t)b * S * V;
#pragma unroll
  for (int u = 0; u < CS; ++u) {
    if (u < nloc) {
      const double f = active ? Fb[(size_t)(s0 + u) * V + v] : 0.0;
      stash_moments(f, vm, red, wave, u, CS, lane);
    }
  }
  __syncthreads();
  flush_moments(red, waves, CS, nloc, d.partials + (((size_t)b * nvb + vb) * S + s0) * PART_STRIDE);
}

// ---------------------------------------------------------------------------------------
// closure: one 64-lane block per (instance, node), plus one wall block per instance

__global__ void __launch_bounds__(64) closure_kernel(Shape sh, DevPtrs d, const double* __restrict__ Fin, int nvb,
                                                     double* __restrict__ mom_out) {
  const int S = sh.S;
  const int b = blockIdx.x / (S + 1), c = blockIdx.x - b * (S + 1);
  const int lane = threadIdx.x;
  const InstDev in = d.inst[b];
  if (c == S) {
    // wall density: zero net mass flux through x = L/2 (App. A.4); the outgoing fluxes
    // (p_x > 0) use the extrapolated ghosts, the incoming ones are p_x n_w F^eq_w exactly.
    const int V = sh.V;
    const double* F = Fin + (size_t)b * S * V;
    double acc = 0.0;
    for (int v = sh.Qx * sh.QyQz + lane; v < V; v += 64) {
      const double px = d.px[v / sh.QyQz];
      const double f3 = F[(size_t)(S - 3) * V + v], f2 = F[(size_t)(S - 2) * V + v], f1 = F[(size_t)(S - 1) * V + v];
      const double g0 = in.ex[0] * f1 + in.ex[1] * f2 + in.ex[2] * f3;
      const double g1 = in.ex[3] * g0 + in.ex[4] * f1 + in.ex[5] * f2;
      const double r = (sh.scheme == 1) ? weno5(f3, f2, f1, g0, g1) : (1.5 * f1 - 0.5 * f2);
      acc += px * r;
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      const double nw = -acc / in.wall_den;
      d.nw[b] = nw;
      if (!(nw > 0.0) || !isfinite(nw)) d.flags[b] = 1;
    }
    return;
  }
  __shared__ double Msh[NMOM];
  if (lane < NMOM) {
    double acc = 0.0;
    for (int vb = 0; vb < nvb; ++vb) acc += d.partials[(((size_t)b * nvb + vb) * S + c) * PART_STRIDE + lane];
    Msh[lane] = acc;
  }
  __syncthreads();
  const double n = Msh[0];
  const double ux = Msh[1] / n, uy = Msh[2] / n, uz = Msh[3] / n;
  const double Pxx = Msh[4] - n * ux * ux, Pyy = Msh[5] - n * uy * uy, Pzz = Msh[6] - n * uz * uz;
  const double Pxy = Msh[7] - n * ux * uy, Pxz = Msh[8] - n * ux * uz, Pyz = Msh[9] - n * uy * uz;
  const double T = (Pxx + Pyy + Pzz) / (3.0 * n);
  // q_a = 1/2 sum F |p - u|^2 (p_a - u_a), expanded over the raw sums
  const double M2 = Msh[4] + Msh[5] + Msh[6];
  const double u2 = ux * ux + uy * uy + uz * uz;
  const double qx = 0.5 * (Msh[10] - ux * M2 - 2.0 * (ux * Msh[4] + uy * Msh[7] + uz * Msh[8]) + 2.0 * n * u2 * ux);
  const double qy = 0.5 * (Msh[11] - uy * M2 - 2.0 * (ux * Msh[7] + uy * Msh[5] + uz * Msh[9]) + 2.0 * n * u2 * uy);
  const double qz = 0.5 * (Msh[12] - uz * M2 - 2.0 * (ux * Msh[8] + uy * Msh[9] + uz * Msh[6]) + 2.0 * n * u2 * uz);
  if (mom_out && lane == 0) {
    double* o = mom_out + ((size_t)b * S + c) * 14;
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
  const bool bad = !(n > 0.0) || !(T > 0.0) || !isfinite(n + T + ux + uy + uz + qx + qy + qz);
  if (bad) {
    if (lane == 0) d.flags[b] = 1;
  }
  // relaxation time from mu = tau n T
  double tau;
  if (in.law == 0.0)
    tau = in.kn * pow(T, in.omega - 1.0) / n;
  else
    tau = in.kn * (1.0 + in.suth) / (n * sqrt(T) * (1.0 + in.suth / T));
  const double invtau = (in.collisionless != 0.0 || bad) ? 0.0 : 1.0 / tau;
  const double Cs = (1.0 - in.pr) / (n * T * T);
  double* rec = d.rec + ((size_t)b * S + c) * sh.rec_len;
  if (lane == 0) {
    rec[0] = ux;
    rec[1] = uy;
    rec[2] = uz;
    rec[3] = invtau;
    rec[4] = Cs;
    rec[5] = Cs / (5.0 * T);
    rec[6] = qx;
    rec[7] = qy;
    rec[8] = qz;
    rec[9] = n;
    rec[10] = T;
  }
  // Hermite-projected equilibrium factors (Sec. III): n g_x on the 2Qx nodes, g_y g_z
  double I[NX_MAX + 1], Jp[NX_MAX + 1], Jm[NX_MAX + 1];
  const double Tc = bad ? 1.0 : T;
  half_gauss_moments(ux, Tc, I);
  half_projection(d.cx, sh.Nx, I, Jp);
  half_gauss_moments(-ux, Tc, I);
  half_projection(d.cx, sh.Nx, I, Jm);
  for (int i = lane; i < 2 * sh.Qx; i += 64) rec[REC_HEAD + i] = n * gx_node(d.phix, sh.Qx, sh.Nx, i, Jp, Jm);
  double ay[NYZ_MAX + 1], az[NYZ_MAX + 1];
  full_coeffs(uy, Tc, ay);
  full_coeffs(uz, Tc, az);
  for (int jk = lane; jk < sh.QyQz; jk += 64) {
    const int j = jk / sh.Qz, k = jk - j * sh.Qz;
    rec[REC_HEAD + 2 * sh.Qx + jk] = full_node(d.phiy, sh.Ny, j, ay) * full_node(d.phiz, sh.Nz, k, az);
  }
}

// ---------------------------------------------------------------------------------------
// the stage kernel

template <int SCHEME, int STAGE, int CS>
__global__ void __launch_bounds__(1024) stage_kernel(Shape sh, DevPtrs d, const double* __restrict__ Fin,
                                                     const double* Fl, double* Fout, int nvb, int nch) {
  extern __shared__ double red[];
  int t = xcd_tile(blockIdx.x, gridDim.x);
  const int ch = t % nch;
  t /= nch;
  const int vb = t % nvb, b = t / nvb;
  const int S = sh.S, V = sh.V, Qx = sh.Qx;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, waves = blockDim.x >> 6;
  const int v = vb * blockDim.x + threadIdx.x;
  const bool active = v < V;
  const int vv = active ? v : V - 1;
  const int i = vv / sh.QyQz, jk = vv - i * sh.QyQz, j = jk / sh.Qz, k = jk - j * sh.Qz;
  const double px = d.px[i], py = d.py[j], pz = d.pz[k];
  const bool pos = px > 0.0;
  // bounce-back partner (Eq. widetildei): p_x and p_y reversed, p_z kept
  const int vm = ((2 * Qx - 1 - i) * sh.Qy + (sh.Qy - 1 - j)) * sh.Qz + k;
  const size_t base = (size_t)b * S * V;
  const double* Fb = Fin + base;
  const InstDev& in = d.inst[b];
  const double dt = in.dt;
  const int s0 = ch * CS;
  const int nloc = min(CS, S - s0);

  // window of nodes s0-3 .. s0+CS+2 (0-based node c), ghosts synthesised in registers
  double w[CS + 6];
#pragma unroll
  for (int q = 0; q < CS + 6; ++q) {
    const int c = s0 - 3 + q;
    double val = 0.0;
    if (active) {
      if (c >= 0 && c < S)
        val = Fb[(size_t)c * V + v];
      else if (c < 0)
        val = Fb[(size_t)(-c - 1) * V + vm];  // F_{1-m; i j k} = F_{m; i~ j~ k}
    }
    w[q] = val;
  }
  if (s0 + CS + 2 >= S) {
    const double ghost_in = active ? d.nw[b] * d.g_wall[(size_t)b * V + vv] : 0.0;
#pragma unroll
    for (int q = 3; q < CS + 6; ++q) {
      const int c = s0 - 3 + q;
      if (c == S)
        w[q] = pos ? in.ex[0] * w[q - 1] + in.ex[1] * w[q - 2] + in.ex[2] * w[q - 3] : ghost_in;
      else if (c == S + 1)
        w[q] = pos ? in.ex[3] * w[q - 1] + in.ex[4] * w[q - 2] + in.ex[5] * w[q - 3] : ghost_in;
      else if (c == S + 2)
        w[q] = pos ? 0.0 : ghost_in;
    }
  }

  const VelMul vmul = velocity_multipliers(px, py, pz, active);
  const double* invdx = d.inv_dx + (size_t)b * S;
  double rd = 0.0, rf = 0.0;

  // interface flux between window slots q and q+1
  auto flux = [&](int q) -> double {
    const double r = pos ? interp<SCHEME>(w[q - 2], w[q - 1], w[q], w[q + 1], w[q + 2])
                         : interp<SCHEME>(w[q + 3], w[q + 2], w[q + 1], w[q], w[q - 1]);
    return px * r;
  };
  double fl = flux(2);
#pragma unroll
  for (int u = 0; u < CS; ++u) {
    if (u < nloc) {
      const int c = s0 + u;
      const double fr = flux(u + 3);
      const double D = (fr - fl) * invdx[c];
      fl = fr;
      const double F = w[u + 3];
      const double* rec = d.rec + ((size_t)b * S + c) * sh.rec_len;
      const double feq = rec[REC_HEAD + i] * rec[REC_HEAD + 2 * Qx + jk];
      const double Cs = rec[4];
      double FS = feq;
      if (Cs != 0.0) {
        const double xx = px - rec[0], xy = py - rec[1], xz = pz - rec[2];
        const double xi2 = xx * xx + xy * xy + xz * xz;
        const double qxi = rec[6] * xx + rec[7] * xy + rec[8] * xz;
        FS = feq + feq * ((rec[5] * xi2 - Cs) * qxi);  // F^eq (1 + S), Eq. sdef
      }
      const double L = (FS - F) * rec[3] - D;  // Eq. L_def
      const double G = F + dt * L;
      double out;
      if constexpr (STAGE == 1) {
        out = G;
      } else {
        const double fl0 = active ? Fl[base + (size_t)c * V + v] : 0.0;
        if constexpr (STAGE == 2)
          out = 0.75 * fl0 + 0.25 * G;
        else
          out = (1.0 / 3.0) * fl0 + (2.0 / 3.0) * G;
        if constexpr (STAGE == 3) {
          const double dlt = out - fl0;
          rd += dlt * dlt;
          rf += fl0 * fl0;
        }
      }
      if (active) Fout[base + (size_t)c * V + v] = out;
      stash_moments(active ? out : 0.0, vmul, red, wave, u, CS, lane);
    }
  }
  if constexpr (STAGE == 3) {
    rd = wave_sum(rd);
    rf = wave_sum(rf);
    if (lane == 0) {
      red[waves * CS * NMOM + 2 * wave] = rd;
      red[waves * CS * NMOM + 2 * wave + 1] = rf;
    }
  }
  __syncthreads();
  flush_moments(red, waves, CS, nloc, d.partials + (((size_t)b * nvb + vb) * S + s0) * PART_STRIDE);
  if constexpr (STAGE == 3) {
    if (threadIdx.x < 2) {
      double s = 0.0;
      for (int wv = 0; wv < waves; ++wv) s += red[waves * CS * NMOM + 2 * wv + threadIdx.x];
      d.resid_part[((size_t)b * nvb * nch + (size_t)vb * nch + ch) * 2 + threadIdx.x] = s;
    }
  }
}

__global__ void __launch_bounds__(256) residual_kernel(Shape sh, DevPtrs d, int nres) {
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

template <int CS>
static int launch_partials_cs(const Shape& sh, const DevPtrs& d, const double* F, int waves, void* stream) {
  int nvb, nch;
  const int nblk = grid_tiles(sh, CS, waves, &nvb, &nch);
  const size_t lds = (size_t)waves * CS * NMOM * sizeof(double);
  hipLaunchKernelGGL(partials_kernel<CS>, dim3(nblk), dim3(64 * waves), lds, (hipStream_t)stream, sh, d, F, nvb, nch);
  return (int)hipGetLastError();
}

int launch_partials(const Shape& sh, const DevPtrs& d, const double* F, int cells, int waves, void* stream) {
  switch (cells) {
    case 1: return launch_partials_cs<1>(sh, d, F, waves, stream);
    case 2: return launch_partials_cs<2>(sh, d, F, waves, stream);
    case 4: return launch_partials_cs<4>(sh, d, F, waves, stream);
    case 8: return launch_partials_cs<8>(sh, d, F, waves, stream);
    case 16: return launch_partials_cs<16>(sh, d, F, waves, stream);
    case 32: return launch_partials_cs<32>(sh, d, F, waves, stream);
  }
  return (int)hipErrorInvalidValue;
}

int launch_closure(const Shape& sh, const DevPtrs& d, const double* Fin, int nvb, double* mom_out, void* stream) {
  hipLaunchKernelGGL(closure_kernel, dim3(sh.B * (sh.S + 1)), dim3(64), 0, (hipStream_t)stream, sh, d, Fin, nvb,
                     mom_out);
  return (int)hipGetLastError();
}

template <int SCHEME, int STAGE, int CS>
static int launch_stage_t(const Shape& sh, const DevPtrs& d, const double* Fin, const double* Fl, double* Fout,
                          int waves, void* stream) {
  int nvb, nch;
  const int nblk = grid_tiles(sh, CS, waves, &nvb, &nch);
  const size_t lds = ((size_t)waves * CS * NMOM + 2 * waves) * sizeof(double);
  hipLaunchKernelGGL((stage_kernel<SCHEME, STAGE, CS>), dim3(nblk), dim3(64 * waves), lds, (hipStream_t)stream, sh,
                     d, Fin, Fl, Fout, nvb, nch);
  return (int)hipGetLastError();
}

template <int SCHEME, int STAGE>
static int launch_stage_s(const Shape& sh, const DevPtrs& d, const double* Fin, const double* Fl, double* Fout,
                          int cells, int waves, void* stream) {
  switch (cells) {
    case 1: return launch_stage_t<SCHEME, STAGE, 1>(sh, d, Fin, Fl, Fout, waves, stream);
    case 2: return launch_stage_t<SCHEME, STAGE, 2>(sh, d, Fin, Fl, Fout, waves, stream);
    case 4: return launch_stage_t<SCHEME, STAGE, 4>(sh, d, Fin, Fl, Fout, waves, stream);
    case 8: return launch_stage_t<SCHEME, STAGE, 8>(sh, d, Fin, Fl, Fout, waves, stream);
    case 16: return launch_stage_t<SCHEME, STAGE, 16>(sh, d, Fin, Fl, Fout, waves, stream);
    case 32: return launch_stage_t<SCHEME, STAGE, 32>(sh, d, Fin, Fl, Fout, waves, stream);
  }
  return (int)hipErrorInvalidValue;
}

int launch_stage(const Shape& sh, const DevPtrs& d, int stage, const double* Fin, const double* Fl, double* Fout,
                 int cells, int waves, void* stream) {
  if (sh.scheme == 1) {
    if (stage == 1) return launch_stage_s<1, 1>(sh, d, Fin, Fl, Fout, cells, waves, stream);
    if (stage == 2) return launch_stage_s<1, 2>(sh, d, Fin, Fl, Fout, cells, waves, stream);
    return launch_stage_s<1, 3>(sh, d, Fin, Fl, Fout, cells, waves, stream);
  }
  if (stage == 1) return launch_stage_s<0, 1>(sh, d, Fin, Fl, Fout, cells, waves, stream);
  if (stage == 2) return launch_stage_s<0, 2>(sh, d, Fin, Fl, Fout, cells, waves, stream);
  return launch_stage_s<0, 3>(sh, d, Fin, Fl, Fout, cells, waves, stream);
}

int launch_residual(const Shape& sh, const DevPtrs& d, int nres, void* stream) {
  hipLaunchKernelGGL(residual_kernel, dim3(sh.B), dim3(256), 0, (hipStream_t)stream, sh, d, nres);
  return (int)hipGetLastError();
}

}  // namespace hrlb

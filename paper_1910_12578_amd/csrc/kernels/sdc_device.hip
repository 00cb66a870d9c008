// Hand-written HIP kernels of the SDC reactive-flow update for gfx950.
//
// This source is compiled at sdc_init together with the network code that
// netgen.cpp generates for the caller's reaction network (it defines SDC_NS,
// SDC_NR, SDC_NX, SDC_NNZ, NetParams and the net_* functions) and with
// SDC_DIM.  Every kernel works on structure-of-arrays state, U[comp][zone]
// with the zone index x-fastest; the components are
//   0: rho,  1..DIM: rho u_d,  DIM+1: rho E,  DIM+2+s: rho X_s,
// and reacting-variable arrays (sources R, Newton vectors) are [NX][zone]
// with x = (rho X_1..rho X_Ns, rho e).
//
// Paper: Zingale et al., Castro, Sec. 2.  Eq. 1 splits U_t = A(U) + R(U);
// Eq. 2 is the node-to-node SDC correction, whose implicit part
// U^{m+1} - dt_m R(U^{m+1}) = rhs is solved here per zone by Newton.
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "sdc_args.h"

#ifndef SDC_DIM
#error "SDC_DIM must be defined"
#endif
#define SDC_NC (2 + SDC_DIM + SDC_NS)
#define SDC_NH (2 + SDC_DIM)

typedef long long i64;
typedef unsigned long long u64;

// ------------------------------------------------------------------ launch
// Blocks are dealt round-robin to the 8 XCDs; remap so that each XCD works on
// a contiguous range of zones and neighbouring stencil blocks share its L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned nx = 8u;
  const unsigned per = nb / nx, rem = nb % nx;
  const unsigned x = b % nx, i = b / nx;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + i;
}

// ------------------------------------------------------------ statistics
// counters: [0..15] histogram of Newton iterations (bin 15 = 15 or more),
// [16] failed solves, [17] total Newton iterations, [18] non-finite results,
// [19] solves, [20] pivot fallbacks.
#define SDC_NSTAT 21
__device__ __forceinline__ void stats_block(unsigned long long* __restrict__ stats, int nu, bool valid, bool nonfinite, int fallbacks) {
  __shared__ unsigned sh[SDC_NSTAT];
  if (threadIdx.x < SDC_NSTAT) sh[threadIdx.x] = 0u;
  __syncthreads();
  if (valid) {
    if (nu > 0) {
      atomicAdd(&sh[nu < 15 ? nu : 15], 1u);
      atomicAdd(&sh[17], (unsigned)nu);
    } else {
      atomicAdd(&sh[16], 1u);
    }
    if (nonfinite) atomicAdd(&sh[18], 1u);
    atomicAdd(&sh[19], 1u);
    if (fallbacks) atomicAdd(&sh[20], (unsigned)fallbacks);
  }
  __syncthreads();
  if (threadIdx.x < SDC_NSTAT && sh[threadIdx.x] != 0u) atomicAdd(&stats[threadIdx.x], (u64)sh[threadIdx.x]);
}

// ------------------------------------------------------------ parameters
// Copy the network parameters (NetParams, a flat array of doubles) from
// device memory into LDS.  Every thread of the block must call it before any
// divergence: it ends with a barrier.
__device__ __forceinline__ ParamPtr stage_params(const void* gp) {
  __shared__ NetParams sh_params;
  const double* src = (const double*)gp;
  double* dst = (double*)&sh_params;
  for (int i = threadIdx.x; i < (int)(sizeof(NetParams) / sizeof(double)); i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  return (ParamPtr)&sh_params;
}

// ------------------------------------------------------------ advection
// A(U) = -sum_d (F_{i+1/2} - F_{i-1/2}) / dx_d: method of lines, piecewise-
// linear reconstruction of the conserved variables (central or monotonized-
// central slopes), Rusanov face flux with the local max(|u_d| + c) of the two
// face states or a frozen speed, periodic grid.

// Written with selects rather than branches: 2 min(|a|, |b|) equals
// min(2|a|, 2|b|) exactly, and the sign comes from a.
__device__ __forceinline__ double mc_slope_of(double um, double u0, double up) {
  const double a = u0 - um, b = up - u0;
  const double m = fmin(2.0 * fmin(fabs(a), fabs(b)), 0.5 * fabs(a + b));
  return a * b > 0.0 ? copysign(m, a) : 0.0;
}

__device__ __forceinline__ double slope_of(double um, double u0, double up, int slope) {
  return slope == 0 ? 0.5 * (up - um) : mc_slope_of(um, u0, up);
}

// Face state pair (left/right of one face) of the hydro components.
struct FaceHydro {
  double uL, uR, a;  // normal velocities, Rusanov speed
};

__device__ __forceinline__ void hydro_flux(const double* W, int d, double gamma, double* F, double& un, double& p, double& c) {
  const double rho = W[0];
  const double ir = 1.0 / rho;
  double ke = 0.0;
#pragma unroll
  for (int e = 0; e < SDC_DIM; ++e) ke = fma(W[1 + e], W[1 + e], ke);
  ke = 0.5 * ke * ir;
  un = W[1 + d] * ir;
  p = (gamma - 1.0) * (W[1 + SDC_DIM] - ke);
  c = sqrt(gamma * p * ir);
#pragma unroll
  for (int q = 0; q < SDC_NH; ++q) F[q] = W[q] * un;
  // multiply-adds written out, so every kernel rounds a face the same way
  F[1 + d] = fma(W[1 + d], un, p);
  F[1 + SDC_DIM] = fma(p, un, F[1 + SDC_DIM]);
}

// Rusanov flux of the hydro components through one face from the two
// reconstructed states, plus the face data the species fluxes need.
__device__ __forceinline__ void hydro_face(const double* WL, const double* WR, int d, double gamma, double alpha,
                                           double* F, FaceHydro& fh) {
  double FL[SDC_NH], FR[SDC_NH], pL, pR, cL, cR;
  hydro_flux(WL, d, gamma, FL, fh.uL, pL, cL);
  hydro_flux(WR, d, gamma, FR, fh.uR, pR, cR);
  fh.a = alpha > 0.0 ? alpha : fmax(fabs(fh.uL) + cL, fabs(fh.uR) + cR);
  const double ha = -0.5 * fh.a;
#pragma unroll
  for (int q = 0; q < SDC_NH; ++q) F[q] = fma(ha, WR[q] - WL[q], 0.5 * (FL[q] + FR[q]));
}

__device__ __forceinline__ double species_face(double L, double R, const FaceHydro& f) {
  return fma(-0.5 * f.a, R - L, 0.5 * fma(L, f.uL, R * f.uR));
}

extern "C" __global__ __launch_bounds__(256) void sdc_advect(AdvArgs a) {
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const i64 z = (i64)b * blockDim.x + threadIdx.x;
  if (z >= a.Z) return;
  // grid (or box) extents and the zone's coordinates inside it; with batched
  // boxes every box is its own periodic grid, so neighbours stay in the box
  int n[3] = {a.n[0], a.n[1], a.n[2]};
  i64 local = z;
  if (a.nbox > 0) {
    int bx = a.blk_box[b];
    while (z >= a.box_off[bx + 1]) ++bx;  // a block may straddle boxes
    n[0] = a.box_ext[3 * bx];
    n[1] = a.box_ext[3 * bx + 1];
    n[2] = a.box_ext[3 * bx + 2];
    local = z - a.box_off[bx];
  }
  int c3[3] = {0, 0, 0};
  {
    i64 t = local;
    c3[0] = (int)(t % n[0]);
    t /= n[0];
    if (SDC_DIM > 1) {
      c3[1] = (int)(t % n[1]);
      t /= n[1];
    }
    if (SDC_DIM > 2) c3[2] = (int)t;
  }
  const double* __restrict__ U = a.U;
  // periodic neighbour offsets i-2..i+2 (without the centre) per direction
  i64 off[SDC_DIM][4];
  {
    i64 stride = 1;
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) {
      const int nd = n[d], cd = c3[d];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int sh = s < 2 ? s - 2 : s - 1;
        int cc = cd + sh;
        cc = cc < 0 ? cc + nd : (cc >= nd ? cc - nd : cc);
        off[d][s] = (i64)(cc - cd) * stride;
      }
      stride *= nd;
    }
  }
  // ---- hydro components, face velocities and speeds per direction
  FaceHydro fh[SDC_DIM][2];
  double acc[SDC_NH];
#pragma unroll
  for (int q = 0; q < SDC_NH; ++q) acc[q] = 0.0;
#pragma unroll
  for (int d = 0; d < SDC_DIM; ++d) {
    double WL[2][SDC_NH], WR[2][SDC_NH];  // face 0 = i-1/2, face 1 = i+1/2
#pragma unroll
    for (int q = 0; q < SDC_NH; ++q) {
      const double* Uq = U + (i64)q * a.Z + z;
      const double h0 = Uq[off[d][0]], h1 = Uq[off[d][1]], h2 = Uq[0], h3 = Uq[off[d][2]], h4 = Uq[off[d][3]];
      const double sm = slope_of(h0, h1, h2, a.slope);
      const double s0 = slope_of(h1, h2, h3, a.slope);
      const double sp = slope_of(h2, h3, h4, a.slope);
      WL[0][q] = h1 + 0.5 * sm;
      WR[0][q] = h2 - 0.5 * s0;
      WL[1][q] = h2 + 0.5 * s0;
      WR[1][q] = h3 - 0.5 * sp;
    }
    double Fh[2][SDC_NH];
#pragma unroll
    for (int f = 0; f < 2; ++f) hydro_face(WL[f], WR[f], d, a.gamma, a.alpha, Fh[f], fh[d][f]);
    const double id = a.idx[d];
#pragma unroll
    for (int q = 0; q < SDC_NH; ++q) acc[q] -= (Fh[1][q] - Fh[0][q]) * id;
  }
#pragma unroll
  for (int q = 0; q < SDC_NH; ++q) a.A[(i64)q * a.Z + z] = acc[q];
  // ---- passive species, one at a time, with the hydro faces' u and speed
#pragma unroll 1
  for (int s = 0; s < SDC_NS; ++s) {
    const double* Us = U + (i64)(SDC_NH + s) * a.Z + z;
    const double v2 = Us[0];
    double A = 0.0;
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) {
      const double v0 = Us[off[d][0]], v1 = Us[off[d][1]], v3 = Us[off[d][2]], v4 = Us[off[d][3]];
      const double sm = slope_of(v0, v1, v2, a.slope);
      const double s0 = slope_of(v1, v2, v3, a.slope);
      const double sp = slope_of(v2, v3, v4, a.slope);
      const double F0 = species_face(v1 + 0.5 * sm, v2 - 0.5 * s0, fh[d][0]);
      const double F1 = species_face(v2 + 0.5 * s0, v3 - 0.5 * sp, fh[d][1]);
      A -= (F1 - F0) * a.idx[d];
    }
    a.A[(i64)(SDC_NH + s) * a.Z + z] = A;
  }
}

#if SDC_DIM == 3
// ---- 3D advective term: complete x-rows per block, marching in z.
// A 256-thread block holds R = 256 / n0 complete x-rows of one periodic grid
// (the domain, or one of the batched boxes; a per-block descriptor says which
// rows and z chunk), periodic in x, so
// every x-face flux is computed once (by the zone to its right) and handed to
// the zone on its left through LDS.  Each row marches up a chunk of planes in
// z carrying, per component, the left state of the face above the current
// plane and the flux through the face below it, so z-faces are computed once
// as well.  The y stencil (both faces of a zone) is read from memory, where
// the neighbouring rows of the same plane sit in L2.  Offsets inside one
// component array are 32-bit byte offsets (the host guarantees 8 Z < 2^32).
// Loads and stores through one buffer resource per array: 32-bit byte
// offsets, the component's offset in a scalar register (the host guarantees
// that every array is below 4 GiB), and out-of-range accesses return zero
// instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t array_rsrc(const double* p, i64 bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(unsigned)bytes, 0x00020000);
}

__device__ __forceinline__ double ld_at(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

typedef unsigned u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned))));

// Non-temporal (cache policy nt): the output is not read again in this
// launch and should not evict the neighbour rows that are.
__device__ __forceinline__ void st_at(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 2);
}

__device__ __forceinline__ int wrap_index(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// One component's values at a zone, its y neighbours y-2..y+2 and the two
// planes above.
struct Stencil7 {
  double c, ym2, ym1, yp1, yp2, z1, z2;
};

template <int SLOPE>
__device__ __forceinline__ double slope_t(double um, double u0, double up) {
  return SLOPE == 0 ? 0.5 * (up - um) : mc_slope_of(um, u0, up);
}

// BW: threads per block (256, or 512 for rows of 257..512 zones).
template <int SLOPE, int BW>
__device__ __forceinline__ void advect_rows_body(const AdvArgs& a) {
  __shared__ double sh_u[SDC_NH][BW];   // hydro components of the current plane
  __shared__ double sh_fh[SDC_NH][BW];  // hydro x-face fluxes
  __shared__ double sh_s[2][BW];        // one species component (alternating)
  __shared__ double sh_fs[2][BW];       // its x-face flux (alternating)
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const RowDesc d = a.rows[b];
  const int n0 = d.n0, n1 = d.n1, n2 = d.n2, ZC = d.zc;
  const int R = BW / n0;
  const int t = threadIdx.x;
  const int r = t / n0, x = t - r * n0;
  const int slot = d.slot0 + r;
  const bool row_ok = r < R && slot < d.nslot;
  const int y = row_ok ? slot % n1 : 0;
  const int k0 = row_ok ? (slot / n1) * ZC : 0;
  const int k1 = row_ok ? min(k0 + ZC, n2) : 0;
  // LDS slots of the x neighbours; idle lanes (r >= R) only touch their own slot
  const int rb = (r < R ? r : 0) * n0, xx = r < R ? x : 0;
  const int lxm2 = r < R ? rb + wrap_index(xx - 2, n0) : t;
  const int lxm1 = r < R ? rb + wrap_index(xx - 1, n0) : t;
  const int lxp1 = r < R ? rb + wrap_index(xx + 1, n0) : t;
  const unsigned P8 = (unsigned)n0 * (unsigned)n1 * 8u;  // plane stride in bytes
  const unsigned row8 = ((unsigned)d.base + (unsigned)y * (unsigned)n0 + (unsigned)xx) * 8u;
  unsigned oy[4];  // byte offsets of rows y-2, y-1, y+1, y+2 relative to row y
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int dy = j < 2 ? j - 2 : j - 1;
    oy[j] = (unsigned)((wrap_index(y + dy, n1) - y) * n0) * 8u;
  }
  const i64 Z = a.Z;
  // one buffer resource per component array (each below 4 GiB)
  auto rU = [&](int c) { return array_rsrc(a.U + (i64)c * Z, Z * 8); };
  auto rA = [&](int c) { return array_rsrc(a.A + (i64)c * Z, Z * 8); };
  const double idx = a.idx[0], idy = a.idx[1], idz = a.idx[2];

  // prologue: the face below plane k0 and the left state of the face above it
  double WLz[SDC_NC], Fz[SDC_NC];
  {
    const unsigned o0 = (unsigned)wrap_index(k0 - 2, n2) * P8 + row8, o1 = (unsigned)wrap_index(k0 - 1, n2) * P8 + row8;
    const unsigned o2 = (unsigned)k0 * P8 + row8, o3 = (unsigned)wrap_index(k0 + 1, n2) * P8 + row8;
    double WL[SDC_NH], WR[SDC_NH];
#pragma unroll
    for (int q = 0; q < SDC_NH; ++q) {
      const __amdgpu_buffer_rsrc_t rq = rU(q);
      const double v0 = ld_at(rq, o0, 0), v1 = ld_at(rq, o1, 0), v2 = ld_at(rq, o2, 0), v3 = ld_at(rq, o3, 0);
      const double sA = slope_t<SLOPE>(v0, v1, v2), sB = slope_t<SLOPE>(v1, v2, v3);
      WL[q] = v1 + 0.5 * sA;
      WR[q] = v2 - 0.5 * sB;
      WLz[q] = v2 + 0.5 * sB;
    }
    FaceHydro fzm;
    hydro_face(WL, WR, 2, a.gamma, a.alpha, Fz, fzm);
#pragma unroll
    for (int s = 0; s < SDC_NS; ++s) {
      const __amdgpu_buffer_rsrc_t rq = rU(SDC_NH + s);
      const double v0 = ld_at(rq, o0, 0), v1 = ld_at(rq, o1, 0), v2 = ld_at(rq, o2, 0), v3 = ld_at(rq, o3, 0);
      const double sA = slope_t<SLOPE>(v0, v1, v2), sB = slope_t<SLOPE>(v1, v2, v3);
      Fz[SDC_NH + s] = species_face(v1 + 0.5 * sA, v2 - 0.5 * sB, fzm);
      WLz[SDC_NH + s] = v2 + 0.5 * sB;
    }
  }

  // the trip count is the same for every thread of the block (barriers)
  for (int k = k0; k < k0 + ZC; ++k) {
    const bool act = row_ok && k < k1;
    const int kc = k < n2 ? k : k - n2;
    const unsigned oc = (unsigned)kc * P8 + row8;
    const unsigned oz1 = (unsigned)wrap_index(kc + 1, n2) * P8 + row8;
    const unsigned oz2 = (unsigned)wrap_index(kc + 2, n2) * P8 + row8;
    auto load7 = [&](int comp) {
      const __amdgpu_buffer_rsrc_t rq = rU(comp);
      Stencil7 v;
      v.c = ld_at(rq, oc, 0);
      v.ym2 = ld_at(rq, oc + oy[0], 0);
      v.ym1 = ld_at(rq, oc + oy[1], 0);
      v.yp1 = ld_at(rq, oc + oy[2], 0);
      v.yp2 = ld_at(rq, oc + oy[3], 0);
      v.z1 = ld_at(rq, oz1, 0);
      v.z2 = ld_at(rq, oz2, 0);
      return v;
    };
    // ---- hydro: y and z faces from memory, stage the plane for x
    __builtin_amdgcn_s_setprio(2);
    double Ay[SDC_NH], Az[SDC_NH];
    FaceHydro fy0, fy1, fz, fx;
    {
      double WLy0[SDC_NH], WRy0[SDC_NH], WLy1[SDC_NH], WRy1[SDC_NH], WRz[SDC_NH], WLzn[SDC_NH];
#pragma unroll
      for (int q = 0; q < SDC_NH; ++q) {
        const __amdgpu_buffer_rsrc_t rq = rU(q);
        const double c = ld_at(rq, oc, 0);
        sh_u[q][t] = c;
        const double ym2 = ld_at(rq, oc + oy[0], 0), ym1 = ld_at(rq, oc + oy[1], 0);
        const double yp1 = ld_at(rq, oc + oy[2], 0), yp2 = ld_at(rq, oc + oy[3], 0);
        const double z1 = ld_at(rq, oz1, 0), z2 = ld_at(rq, oz2, 0);
        const double sm = slope_t<SLOPE>(ym2, ym1, c), s0 = slope_t<SLOPE>(ym1, c, yp1);
        const double sp = slope_t<SLOPE>(c, yp1, yp2), s1 = slope_t<SLOPE>(c, z1, z2);
        WLy0[q] = ym1 + 0.5 * sm;
        WRy0[q] = c - 0.5 * s0;
        WLy1[q] = c + 0.5 * s0;
        WRy1[q] = yp1 - 0.5 * sp;
        WRz[q] = z1 - 0.5 * s1;
        WLzn[q] = z1 + 0.5 * s1;
      }
      double F0[SDC_NH], F1[SDC_NH];
      hydro_face(WLy0, WRy0, 1, a.gamma, a.alpha, F0, fy0);
      hydro_face(WLy1, WRy1, 1, a.gamma, a.alpha, F1, fy1);
#pragma unroll
      for (int q = 0; q < SDC_NH; ++q) Ay[q] = (F1[q] - F0[q]) * idy;
      hydro_face(WLz, WRz, 2, a.gamma, a.alpha, F1, fz);
#pragma unroll
      for (int q = 0; q < SDC_NH; ++q) {
        Az[q] = (F1[q] - Fz[q]) * idz;
        Fz[q] = F1[q];
        WLz[q] = WLzn[q];
      }
    }
    Stencil7 nxt = load7(SDC_NH);  // first species, in flight across the hydro barriers
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    double Fx[SDC_NH];
    {
      double WLx[SDC_NH], WRx[SDC_NH];
#pragma unroll
      for (int q = 0; q < SDC_NH; ++q) {
        const double xm2 = sh_u[q][lxm2], xm1 = sh_u[q][lxm1], c = sh_u[q][t], xp1 = sh_u[q][lxp1];
        const double sA = slope_t<SLOPE>(xm2, xm1, c), sB = slope_t<SLOPE>(xm1, c, xp1);
        WLx[q] = xm1 + 0.5 * sA;
        WRx[q] = c - 0.5 * sB;
      }
      hydro_face(WLx, WRx, 0, a.gamma, a.alpha, Fx, fx);
    }
#pragma unroll
    for (int q = 0; q < SDC_NH; ++q) sh_fh[q][t] = Fx[q];
    // ---- species, with the hydro faces' velocities and speeds.  One barrier
    // per species: the barrier of species s publishes its staged values and
    // the x-face flux of species s - 1 (the hydro fluxes for s = 0), in
    // alternating LDS buffers; the loads of species s + 1 are issued before it.
    double pf = 0.0, pay = 0.0, paz = 0.0;  // species s - 1: x flux, y and z parts
#pragma unroll
    for (int s = 0; s <= SDC_NS; ++s) {
      double c = 0.0, ay = 0.0, az = 0.0;
      if (s < SDC_NS) {
        const Stencil7 cur = nxt;
        if (s + 1 < SDC_NS) nxt = load7(SDC_NH + s + 1);
        c = cur.c;
        sh_s[s & 1][t] = c;
        const double sm = slope_t<SLOPE>(cur.ym2, cur.ym1, c), s0 = slope_t<SLOPE>(cur.ym1, c, cur.yp1);
        const double sp = slope_t<SLOPE>(c, cur.yp1, cur.yp2), s1 = slope_t<SLOPE>(c, cur.z1, cur.z2);
        ay = (species_face(c + 0.5 * s0, cur.yp1 - 0.5 * sp, fy1) - species_face(cur.ym1 + 0.5 * sm, c - 0.5 * s0, fy0)) * idy;
        const double fzn = species_face(WLz[SDC_NH + s], cur.z1 - 0.5 * s1, fz);
        az = (fzn - Fz[SDC_NH + s]) * idz;
        Fz[SDC_NH + s] = fzn;
        WLz[SDC_NH + s] = cur.z1 + 0.5 * s1;
      }
      __syncthreads();
      if (s == 0) {
#pragma unroll
        for (int q = 0; q < SDC_NH; ++q) {
          double acc = -((sh_fh[q][lxp1] - Fx[q]) * idx);
          acc -= Ay[q];
          acc -= Az[q];
          if (act) st_at(rA(q), oc, 0, acc);
        }
      } else {
        double acc = -((sh_fs[(s - 1) & 1][lxp1] - pf) * idx);
        acc -= pay;
        acc -= paz;
        if (act) st_at(rA(SDC_NH + s - 1), oc, 0, acc);
      }
      if (s < SDC_NS) {
        const double xm2 = sh_s[s & 1][lxm2], xm1 = sh_s[s & 1][lxm1], xp1 = sh_s[s & 1][lxp1];
        const double sA = slope_t<SLOPE>(xm2, xm1, c), sB = slope_t<SLOPE>(xm1, c, xp1);
        pf = species_face(xm1 + 0.5 * sA, c - 0.5 * sB, fx);
        sh_fs[s & 1][t] = pf;
        pay = ay;
        paz = az;
      }
    }
  }
}
extern "C" __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void sdc_advect_rows(AdvArgs a) {
  advect_rows_body<1, 256>(a);
}
extern "C" __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void sdc_advect_rows_c(AdvArgs a) {
  advect_rows_body<0, 256>(a);
}
// rows of 257..512 zones: one 512-thread block per CU, two waves per SIMD
extern "C" __global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void sdc_advect_rows_w(AdvArgs a) {
  advect_rows_body<1, 512>(a);
}
extern "C" __global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void sdc_advect_rows_wc(AdvArgs a) {
  advect_rows_body<0, 512>(a);
}
#endif

// ------------------------------------------------------------ reactions
// Newton's stopping test on the scaled step sizes e_k = err and e_{k-1} =
// perr (0 before the first step): the step is at most tol, or the steps
// contract and the contraction bounds the new iterate's distance from the
// root, theta / (1 - theta) e_k with theta = e_k / e_{k-1}, by tol (Hairer and
// Wanner, Solving ODEs II, Sec. IV.8).
__device__ __forceinline__ bool newton_done(double err, double perr, double tol) {
  return err <= tol || (err < perr && err * err <= tol * (perr - err));
}

struct VecX {
  double v[SDC_NX];
};

struct DenseResult {
  VecX x;
  int it;  // iteration count at exit, or -1
};

// Dense Newton matrix M = I - dt_m dR/dx (row-major) and r = -(x - dt_m R - b),
// assembled with rolled loops over the topology tables (scratch resident).
__device__ __forceinline__ void dense_newton_matrix(const double* x, const double* b, double irho, double dtm,
                                                    ParamPtr P, double gm1, double* M, double* r) {
  const int e = SDC_NX - 1;
  for (int i = 0; i < SDC_NX * SDC_NX; ++i) M[i] = 0.0;
  for (int i = 0; i < SDC_NX; ++i) {
    M[i * SDC_NX + i] = 1.0;
    r[i] = b[i] - x[i];
  }
  const double T = gm1 * x[e] * irho, lnT = log(T), invT = 1.0 / T, dTdxe = gm1 * irho;
  for (int q = 0; q < SDC_NR; ++q) {
    const double k = exp(fma(P->b[q], lnT, P->lnA[q]) - P->E[q] * invT);
    const int a = kRxA[q], c = kRxC[q];
    const double mono = c < 0 ? x[a] : x[a] * x[c];
    const double v = k * mono;
    const double da = c < 0 ? k : (a == c ? 2.0 * k * x[a] : k * x[c]);
    const double dc = c < 0 ? 0.0 : (a == c ? 0.0 : k * x[a]);
    const double de = v * fma(P->E[q], invT * invT, P->b[q] * invT) * dTdxe;
    for (int s = 0; s <= kRxN[q]; ++s) {
      const int i = s < kRxN[q] ? kRxSp[q][s] : e;
      const double w = (s < kRxN[q] ? kRxS[q][s] : P->Q[q]) * dtm;  // row weight
      r[i] = fma(w, v, r[i]);
      M[i * SDC_NX + a] -= w * da;
      if (c >= 0) M[i * SDC_NX + c] -= w * dc;
      M[i * SDC_NX + e] -= w * de;
    }
  }
}

// Newton with a dense, partially pivoted LU of M = I - dt_m dR/dx, continued
// from iterate x after `it0` iterations.  Used only for zones whose fixed-
// order factorisation met a pivot below tau times its column maximum.  It is
// kept out of line and written with rolled loops over the topology tables, so
// that its arrays live in scratch memory and the fast path's register budget
// does not pay for it.
__device__ __attribute__((noinline)) DenseResult dense_newton(VecX xv, VecX bv, double rho, double dtm, ParamPtr P,
                                                              double gm1, double tol, int it0, int maxiter,
                                                              double perr) {
  DenseResult out;
  double x[SDC_NX], b[SDC_NX];
  for (int i = 0; i < SDC_NX; ++i) {
    x[i] = xv.v[i];
    b[i] = bv.v[i];
  }
  const double irho = 1.0 / rho;
  const double ise = 1.0 / fabs(b[SDC_NX - 1]);
  const int e = SDC_NX - 1;
  out.it = -1;
  for (int it = it0; it <= maxiter; ++it) {
    double M[SDC_NX * SDC_NX];
    double r[SDC_NX];
    dense_newton_matrix(x, b, irho, dtm, P, gm1, M, r);
    for (int k = 0; k < SDC_NX; ++k) {
      int p = k;
      double best = fabs(M[k * SDC_NX + k]);
      for (int i = k + 1; i < SDC_NX; ++i) {
        const double v = fabs(M[i * SDC_NX + k]);
        if (v > best) {
          best = v;
          p = i;
        }
      }
      if (p != k) {
        for (int j = k; j < SDC_NX; ++j) {
          const double t = M[k * SDC_NX + j];
          M[k * SDC_NX + j] = M[p * SDC_NX + j];
          M[p * SDC_NX + j] = t;
        }
        const double t = r[k];
        r[k] = r[p];
        r[p] = t;
      }
      const double inv = 1.0 / M[k * SDC_NX + k];
      for (int i = k + 1; i < SDC_NX; ++i) {
        const double l = M[i * SDC_NX + k] * inv;
        for (int j = k + 1; j < SDC_NX; ++j) M[i * SDC_NX + j] = fma(-l, M[k * SDC_NX + j], M[i * SDC_NX + j]);
        r[i] = fma(-l, r[k], r[i]);
      }
    }
    double err = 0.0, inf_or_nan = ise * 0.0;
    for (int k = SDC_NX - 1; k >= 0; --k) {
      double s = r[k];
      for (int j = k + 1; j < SDC_NX; ++j) s = fma(-M[k * SDC_NX + j], r[j], s);
      r[k] = s / M[k * SDC_NX + k];
      x[k] += r[k];
      err = fmax(err, fabs(r[k]) * (k == e ? ise : irho));
      inf_or_nan += r[k] * 0.0;
    }
    if (!(inf_or_nan == 0.0)) break;
    if (newton_done(err, perr, tol)) {
      out.it = it;
      break;
    }
    perr = err;
  }
  for (int i = 0; i < SDC_NX; ++i) out.x.v[i] = x[i];
  return out;
}

// One zone's vector in a block-shared [SDC_NX][256] LDS array.
struct LdsVec {
  __attribute__((address_space(3))) double* p;  // &array[0][threadIdx.x]
  __device__ double get(int i) const { return p[i * 256]; }
  __device__ void set(int i, double v) const { p[i * 256] = v; }
  __device__ double operator[](int i) const { return p[i * 256]; }
};

// Fast Newton pass for x - dt_m R(x; rho) = b from the iterate in x, running
// iterations it0..itmax.  Measures each step by max_i |delta_i| / s_i (s = rho
// for species, |b_e| for energy) and stops by newton_done.  Returns the last
// iteration index and a status:
// 0 converged, 1 no convergence by itmax, 2 the pivot guard stopped iteration
// `it` before it changed x, 3 non-finite step.  MT is the type of the Newton
// matrix and its LU factors (double, or float in the mixed mode where the
// residual and the update stay in double).  No calls.  b is read back
// unchanged from LDS at the end.  perr: size of the step before iteration it0
// (0: none); on return that of the last step taken (a step the pivot guard
// rejected does not count).
template <class MT>
__device__ __forceinline__ int newton_fast(double* x, double* b, double irho, double ise, double dtm,
                                           ParamPtr P, double gm1, double tol, double tau, int it0, int itmax,
                                           int& st, double& perr) {
  // x and b wait in LDS while the Newton matrix and its factors hold the
  // registers; each iteration reads them back where it needs them
  __shared__ double sh_x[SDC_NX][256], sh_b[SDC_NX][256];
  const LdsVec xs{(__attribute__((address_space(3))) double*)&sh_x[0][threadIdx.x]};
  const LdsVec bs{(__attribute__((address_space(3))) double*)&sh_b[0][threadIdx.x]};
#pragma unroll
  for (int i = 0; i < SDC_NX; ++i) {
    xs.set(i, x[i]);
    bs.set(i, b[i]);
  }
  int it = it0;
  st = 1;
  for (; it <= itmax; ++it) {
    // keep the parameter and x/b reads inside the iteration: hoisted out of
    // the loop they would pin registers for its whole length
    asm volatile("" ::: "memory");
    double G[SDC_NX];
    MT M[SDC_NNZ];
    net_residual_matrix<MT>(xs, bs, irho, dtm, P, gm1, G, M);
    // the right-hand side rides along the factorisation, which drops each
    // multiplier once it is applied (mixed mode: rounded to the matrix type)
    MT r[SDC_NX];
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) r[i] = (MT)(-G[i]);
    // A failed pivot guard zeroes the step instead of leaving the loop here:
    // a branch between the factorisation and the update splits them into
    // separately scheduled blocks and costs about a hundred registers.
    const bool ok = net_lu_solve<MT>(M, r, (MT)tau);
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) r[i] = ok ? r[i] : (MT)0;
    asm volatile("" ::: "memory");
    double err = 0.0, inf_or_nan = ise * 0.0;  // fmax drops NaN, so track it apart
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) {
      const double d = (double)r[i];
      xs.set(i, xs.get(i) + d);
      err = fmax(err, fabs(d) * (i == SDC_NX - 1 ? ise : irho));
      inf_or_nan += d * 0.0;
    }
    if (!ok) {  // x is unchanged: x + 0 == x
      st = 2;
      break;
    }
    if (!(inf_or_nan == 0.0)) {
      st = 3;
      break;
    }
    if (newton_done(err, perr, tol)) {
      st = 0;
      break;
    }
    perr = err;
  }
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < SDC_NX; ++i) {
    x[i] = xs.get(i);
    b[i] = bs.get(i);
  }
  return it > itmax ? itmax : it;
}

// Queue slot for lanes that defer their zone: one atomic per wavefront.
__device__ __forceinline__ long long defer_slot(unsigned* count, bool want) {
  const unsigned long long mask = __ballot(want);
  if (mask == 0ull) return -1;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  unsigned base = 0u;
  if (lane == leader) base = atomicAdd(count, (unsigned)__popcll(mask));
  base = __shfl(base, leader, 64);
  const unsigned rank = (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
  return want ? (long long)(base + rank) : -1;
}

// Finish a deferred solve: the fast pass from iteration it0 + 1 (it0 > 0) or
// the dense pivoted Newton from iteration -it0 (it0 < 0, guard failure);
// perr is the size of the last step taken before.
template <class MT>
__device__ __forceinline__ int newton_finish(double* x, double* b, double rho, double dtm, ParamPtr P, double gm1,
                                             const NewtonCtl& ctl, int it0, double perr, int& fallbacks) {
  const double irho = 1.0 / rho;
  const double ise = 1.0 / fabs(b[SDC_NX - 1]);
  int start = -it0;
  if (it0 > 0) {
    int st = 1;
    const int it = newton_fast<MT>(x, b, irho, ise, dtm, P, gm1, ctl.tol, ctl.tau, it0 + 1, ctl.maxiter, st, perr);
    if (st == 0) return it;
    if (st != 2) return -1;
    start = it;
  }
  fallbacks = 1;
  VecX xv, bv;
#pragma unroll
  for (int i = 0; i < SDC_NX; ++i) {
    xv.v[i] = x[i];
    bv.v[i] = b[i];
  }
  const DenseResult r = dense_newton(xv, bv, rho, dtm, P, gm1, ctl.tol, start, ctl.maxiter, perr);
#pragma unroll
  for (int i = 0; i < SDC_NX; ++i) x[i] = r.x.v[i];
  return r.it;
}

__device__ __forceinline__ bool all_finite(const double* x) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < SDC_NX; ++i) ok = ok && (fabs(x[i]) <= 1.7976931348623157e308);
  return ok;
}


// ---- sdc_reaction_solve: the implicit part of Eq. 2 alone.
template <class MT>
__device__ __forceinline__ void reaction_solve_body(const SolveArgs& a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = z < a.Z;
  ParamPtr P = stage_params(a.P);
  double x[SDC_NX], b[SDC_NX], rho = 1.0;
  int it = 0, st = 3;
  double perr = 0.0;
  if (valid) {
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) {
      x[i] = a.x[(i64)i * a.Z + z];
      b[i] = a.b[(i64)i * a.Z + z];
    }
    rho = a.rho[z];
    const double ise = 1.0 / fabs(b[SDC_NX - 1]);
    it = newton_fast<MT>(x, b, 1.0 / rho, ise, a.dtm, P, a.gm1, a.ctl.tol, a.ctl.tau, 1,
                         min(a.ctl.cap, a.ctl.maxiter), st, perr);
  }
  const bool defer = valid && (st == 2 || (st == 1 && a.ctl.cap < a.ctl.maxiter));
  const long long slot = defer_slot(a.q.count, defer);
  int nu = 0;
  bool nonfinite = false;
  if (defer) {
    const i64 cap = a.q.capacity;
    a.q.z[slot] = z;
    a.q.it[slot] = st == 2 ? -it : it;
    a.q.perr[slot] = perr;
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) {
      a.q.x[(i64)i * cap + slot] = x[i];
      a.q.b[(i64)i * cap + slot] = b[i];
    }
    a.q.aux[slot] = rho;
  } else if (valid) {
    nu = st == 0 ? it : -1;
    double R[SDC_NX];
    net_source(x, 1.0 / rho, P, a.gm1, R);
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) {
      a.x[(i64)i * a.Z + z] = x[i];
      a.R[(i64)i * a.Z + z] = R[i];
    }
    a.iters[z] = nu;
    nonfinite = !all_finite(x);
  }
  stats_block(a.stats, nu, valid && !defer, nonfinite, 0);
}

template <class MT>
__device__ __forceinline__ void reaction_finish_body(const SolveArgs& a) {
  ParamPtr P = stage_params(a.P);
  // a bounded grid strides over the queue; the trip count is uniform per
  // block (the barriers of stats_block)
  const i64 count = (i64)*a.q.count, stride = (i64)gridDim.x * blockDim.x;
  for (i64 base = (i64)blockIdx.x * blockDim.x; base < count; base += stride) {
    const i64 i = base + threadIdx.x;
    const bool valid = i < count;
    int nu = 0, fb = 0;
    bool nonfinite = false;
    if (valid) {
      const i64 cap = a.q.capacity;
      const i64 z = a.q.z[i];
      double x[SDC_NX], b[SDC_NX];
#pragma unroll
      for (int k = 0; k < SDC_NX; ++k) {
        x[k] = a.q.x[(i64)k * cap + i];
        b[k] = a.q.b[(i64)k * cap + i];
      }
      const double rho = a.q.aux[i];
      nu = newton_finish<MT>(x, b, rho, a.dtm, P, a.gm1, a.ctl, a.q.it[i], a.q.perr[i], fb);
      double R[SDC_NX];
      net_source(x, 1.0 / rho, P, a.gm1, R);
#pragma unroll
      for (int k = 0; k < SDC_NX; ++k) {
        a.x[(i64)k * a.Z + z] = x[k];
        a.R[(i64)k * a.Z + z] = R[k];
      }
      a.iters[z] = nu;
      nonfinite = !all_finite(x);
    }
    stats_block(a.stats, nu, valid, nonfinite, fb);
  }
}

#ifndef SDC_MIXED
typedef double SdcMT;
#else
typedef float SdcMT;
#endif
// Two register budgets of the hot kernels: the compiler's choice (occupancy 1
// for the larger networks) and one that targets two waves per SIMD; the
// autotuner picks between them.
#define SDC_OCC2 __attribute__((amdgpu_waves_per_eu(2, 2)))
extern "C" __global__ __launch_bounds__(256) void sdc_reaction_solve(SolveArgs a) { reaction_solve_body<SdcMT>(a); }
extern "C" __global__ __launch_bounds__(256) SDC_OCC2 void sdc_reaction_solve_o2(SolveArgs a) {
  reaction_solve_body<SdcMT>(a);
}
extern "C" __global__ __launch_bounds__(256) void sdc_reaction_finish(SolveArgs a) { reaction_finish_body<SdcMT>(a); }

// ---- R(U): the reactive source of a full state, on the reacting variables.

extern "C" __global__ __launch_bounds__(256) void sdc_source(SourceArgs a) {
  ParamPtr P = stage_params(a.P);
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= a.Z) return;
  const double rho = a.U[z];
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < SDC_DIM; ++d) {
    const double m = a.U[(i64)(1 + d) * a.Z + z];
    ke = fma(m, m, ke);
  }
  ke = 0.5 * ke / rho;
  double x[SDC_NX], R[SDC_NX];
#pragma unroll
  for (int s = 0; s < SDC_NS; ++s) x[s] = a.U[(i64)(SDC_NH + s) * a.Z + z];
  x[SDC_NX - 1] = a.U[(i64)(1 + SDC_DIM) * a.Z + z] - ke;
  net_source(x, 1.0 / rho, P, a.gm1, R);
#pragma unroll
  for (int i = 0; i < SDC_NX; ++i) a.R[(i64)i * a.Z + z] = R[i];
}

// ------------------------------------------------------------ transition
// One node transition m -> m+1 of Eq. 2 for every zone, fused:
//   rhs = U^{m,(k+1)} + dt_m A^{m,(k+1)} + C_m,
//   C_m = dt sum_j S_mj (A^{j,(k)} + R^{j,(k)}) - dt_m A^{m,(k)} - dt_m R^{m+1,(k)}
// with C_m = 0 on the first sweep (every iteration-0 node holds U^n), and for
// m = 0 the A^0 terms cancelling exactly.  rho and rho u are final after the
// explicit part; (rho X, rho e) solve x - dt_m R(x) = b by Newton from the
// previous iterate of node m+1; R^{m+1} is re-evaluated at the root.  The
// m = 0 transition also forms C_1..C_{M-1} for the later transitions, before
// anything of iteration k is overwritten.
#ifndef SDC_NNODES
#error "SDC_NNODES (number of Gauss-Lobatto nodes) must be defined"
#endif
#define SDC_M (SDC_NNODES - 1)
enum { KIND_FIRST = 0, KIND_NODE0 = 1, KIND_LATER = 2 };

// component c of the full state -> reacting index, or -1
__device__ __forceinline__ constexpr int react_index(int c) {
  return c == 1 + SDC_DIM ? SDC_NX - 1 : (c >= SDC_NH ? c - SDC_NH : -1);
}

// Streaming accesses of the transition kernels: every value is read or
// written once per launch, so they are marked non-temporal and leave the
// caches to what is reused (the Newton kernels' register spill).
__device__ __forceinline__ double ld_s(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_s(double* p, double v) { __builtin_nontemporal_store(v, p); }

// Finalise node m+1 of zone z: rho, rho u from the explicit part, rho E =
// x_e + KE, rho X = x_s, and R^{m+1} re-evaluated at the root.
// (FULL = false: rho and rho u were written by the explicit-part kernel.)
template <bool FULL = true>
__device__ __forceinline__ void transition_store(const TransArgs& a, i64 z, double rho, double ke, const double* mom,
                                                 const double* x, ParamPtr P) {
  const i64 Z = a.Z;
  double R[SDC_NX];
  net_source(x, 1.0 / rho, P, a.gm1, R);
  double* __restrict__ Uo = a.Uout;
  if (FULL) {
    st_s(&Uo[z], rho);
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) st_s(&Uo[(i64)(1 + d) * Z + z], mom[d]);
  }
  st_s(&Uo[(i64)(1 + SDC_DIM) * Z + z], x[SDC_NX - 1] + ke);
#pragma unroll
  for (int s = 0; s < SDC_NS; ++s) st_s(&Uo[(i64)(SDC_NH + s) * Z + z], x[s]);
#pragma unroll
  for (int i = 0; i < SDC_NX; ++i) st_s(&a.Rout[(i64)i * Z + z], R[i]);
}

// Right-hand side of Eq. 2 for zone z (all components), with the quadrature
// of every node and the C_m outputs for m = 0.
template <int KIND>
__device__ __forceinline__ void transition_rhs(const TransArgs& a, i64 z, double* rhs) {
  const i64 Z = a.Z;
  if (KIND == KIND_FIRST) {
#pragma unroll
    for (int c = 0; c < SDC_NC; ++c) rhs[c] = fma(a.dtm, ld_s(&a.Am[(i64)c * Z + z]), ld_s(&a.Um[(i64)c * Z + z]));
  } else if (KIND == KIND_NODE0) {
#pragma unroll
    for (int c = 0; c < SDC_NC; ++c) {
      const int ri = c == 1 + SDC_DIM ? SDC_NX - 1 : (c >= SDC_NH ? c - SDC_NH : -1);
      double f[SDC_NNODES];
#pragma unroll
      for (int j = 0; j <= SDC_M; ++j) {
        f[j] = ld_s(&a.Aold[j][(i64)c * Z + z]);
        if (ri >= 0) f[j] += ld_s(&a.Rold[j][(i64)ri * Z + z]);
      }
      double i0 = 0.0;
#pragma unroll
      for (int j = 0; j <= SDC_M; ++j) i0 = fma(a.S[0][j], f[j], i0);
      double r = fma(a.dt, i0, ld_s(&a.Um[(i64)c * Z + z]));
      if (ri >= 0) r = fma(-a.dtm, ld_s(&a.Rold[1][(i64)ri * Z + z]), r);
      rhs[c] = r;
#pragma unroll
      for (int mm = 1; mm < SDC_M; ++mm) {
        double im = 0.0;
#pragma unroll
        for (int j = 0; j <= SDC_M; ++j) im = fma(a.S[mm][j], f[j], im);
        double cm = fma(-a.dtj[mm], ld_s(&a.Aold[mm][(i64)c * Z + z]), a.dt * im);
        if (ri >= 0) cm = fma(-a.dtj[mm], ld_s(&a.Rold[mm + 1][(i64)ri * Z + z]), cm);
        st_s(&a.Cout[mm - 1][(i64)c * Z + z], cm);
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < SDC_NC; ++c)
      rhs[c] = fma(a.dtm, ld_s(&a.Am[(i64)c * Z + z]), ld_s(&a.Um[(i64)c * Z + z])) + ld_s(&a.Cin[(i64)c * Z + z]);
  }
}

// Explicit part of the transition of zone z: the right-hand side of Eq. 2
// (with the quadrature of every node and the C_m outputs for m = 0), the final
// rho and rho u, KE at m+1, the reacting right-hand side b and the energy
// component of the Newton guess (from the previous iterate of node m+1).
template <int KIND>
__device__ __forceinline__ void transition_explicit(const TransArgs& a, i64 z, double& rho, double& ke, double* mom,
                                                    double* b, double& xe_guess) {
  const i64 Z = a.Z;
  {
    double rhs[SDC_NC];
    transition_rhs<KIND>(a, z, rhs);
    // explicit part: rho and rho u are final
    rho = rhs[0];
    ke = 0.0;
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) {
      mom[d] = rhs[1 + d];
      ke = fma(rhs[1 + d], rhs[1 + d], ke);
    }
    ke = 0.5 * ke / rho;
#pragma unroll
    for (int s = 0; s < SDC_NS; ++s) b[s] = rhs[SDC_NH + s];
    b[SDC_NX - 1] = rhs[1 + SDC_DIM] - ke;
    // energy part of the Newton guess: previous iterate of node m+1
    {
      const double* __restrict__ g = a.guess;
      const double grho = ld_s(&g[z]);
      double gke = 0.0;
#pragma unroll
      for (int d = 0; d < SDC_DIM; ++d) {
        const double mo = ld_s(&g[(i64)(1 + d) * Z + z]);
        gke = fma(mo, mo, gke);
      }
      gke = 0.5 * gke / grho;
      xe_guess = ld_s(&g[(i64)(1 + SDC_DIM) * Z + z]) - gke;
    }
  }
}

template <class MT, int KIND>
__device__ __forceinline__ void transition_body(const TransArgs& a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = z < a.Z;
  ParamPtr P = stage_params(a.P);
  const i64 Z = a.Z;
  double rho = 1.0, ke = 0.0, mom[SDC_DIM];
  double b[SDC_NX], x[SDC_NX];
  int it = 0, st = 3;
  double perr = 0.0;
  if (valid) {
    // the m = 0 prologue (the quadrature inputs of every node) issues its
    // loads ahead of the other wave's Newton work (measured: helps the m = 0
    // transition, slows the lighter ones)
    if (KIND == KIND_NODE0) __builtin_amdgcn_s_setprio(2);
    transition_explicit<KIND>(a, z, rho, ke, mom, b, x[SDC_NX - 1]);
    // species part of the Newton guess
#pragma unroll
    for (int s = 0; s < SDC_NS; ++s) x[s] = ld_s(&a.guess[(i64)(SDC_NH + s) * Z + z]);
    if (KIND == KIND_NODE0) __builtin_amdgcn_s_setprio(0);
    it = newton_fast<MT>(x, b, 1.0 / rho, 1.0 / fabs(b[SDC_NX - 1]), a.dtm, P, a.gm1, a.ctl.tol, a.ctl.tau, 1,
                         min(a.ctl.cap, a.ctl.maxiter), st, perr);
  }
  const bool defer = valid && (st == 2 || (st == 1 && a.ctl.cap < a.ctl.maxiter));
  const long long slot = defer_slot(a.q.count, defer);
  int nu = 0;
  bool nonfinite = false;
  if (defer) {
    const i64 cap = a.q.capacity;
    a.q.z[slot] = z;
    a.q.it[slot] = st == 2 ? -it : it;
    a.q.perr[slot] = perr;
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) {
      a.q.x[(i64)i * cap + slot] = x[i];
      a.q.b[(i64)i * cap + slot] = b[i];
    }
    a.q.aux[slot] = rho;
    a.q.aux[cap + slot] = ke;
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) a.q.aux[(i64)(2 + d) * cap + slot] = mom[d];
  } else if (valid) {
    nu = st == 0 ? it : -1;
    transition_store(a, z, rho, ke, mom, x, P);
    nonfinite = !all_finite(x);
  }
  stats_block(a.stats, nu, valid && !defer, nonfinite, 0);
}

template <class MT>
__device__ __forceinline__ void transition_finish_body(const TransArgs& a) {
  ParamPtr P = stage_params(a.P);
  // a bounded grid strides over the queue; the trip count is uniform per
  // block (the barriers of stats_block)
  const i64 count = (i64)*a.q.count, stride = (i64)gridDim.x * blockDim.x;
  for (i64 base = (i64)blockIdx.x * blockDim.x; base < count; base += stride) {
    const i64 i = base + threadIdx.x;
    const bool valid = i < count;
    int nu = 0, fb = 0;
    bool nonfinite = false;
    if (valid) {
      const i64 cap = a.q.capacity;
      const i64 z = a.q.z[i];
      double x[SDC_NX], b[SDC_NX], mom[SDC_DIM];
#pragma unroll
      for (int k = 0; k < SDC_NX; ++k) {
        x[k] = a.q.x[(i64)k * cap + i];
        b[k] = a.q.b[(i64)k * cap + i];
      }
      const double rho = a.q.aux[i], ke = a.q.aux[cap + i];
#pragma unroll
      for (int d = 0; d < SDC_DIM; ++d) mom[d] = a.q.aux[(i64)(2 + d) * cap + i];
      nu = newton_finish<MT>(x, b, rho, a.dtm, P, a.gm1, a.ctl, a.q.it[i], a.q.perr[i], fb);
      transition_store(a, z, rho, ke, mom, x, P);
      nonfinite = !all_finite(x);
    }
    stats_block(a.stats, nu, valid, nonfinite, fb);
  }
}

// ---- split schedule.  The explicit part (quadrature, rhs, final rho and
// rho u) of a zone batch runs in its own kernel, which streams through memory
// with few registers, while the Newton kernel of the previous batch runs
// beside it on another stream; the right-hand side b, KE and the energy part
// of the guess pass through a [NX + 2][Z] array.  Same arithmetic as the
// fused kernel, so the same bits.
template <int KIND>
__device__ __forceinline__ void transition_pre_body(const TransArgs& a) {
  const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.zcount) return;
  const i64 z = a.zbeg + t, Z = a.Z;
  double rho, ke, mom[SDC_DIM], b[SDC_NX], xe;
  transition_explicit<KIND>(a, z, rho, ke, mom, b, xe);
  // the guess (previous iterate of node m+1, possibly this very array) has
  // been read: rho and rho u of node m+1 are final
  double* __restrict__ Uo = a.Uout;
  Uo[z] = rho;
#pragma unroll
  for (int d = 0; d < SDC_DIM; ++d) Uo[(i64)(1 + d) * Z + z] = mom[d];
#pragma unroll
  for (int i = 0; i < SDC_NX; ++i) a.split[(i64)i * Z + z] = b[i];
  a.split[(i64)SDC_NX * Z + z] = ke;
  a.split[(i64)(SDC_NX + 1) * Z + z] = xe;
}

template <class MT>
__device__ __forceinline__ void transition_newton_body(const TransArgs& a) {
  const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < a.zcount;
  const i64 z = a.zbeg + (valid ? t : 0), Z = a.Z;
  ParamPtr P = stage_params(a.P);
  double rho = 1.0, ke = 0.0;
  double b[SDC_NX], x[SDC_NX];
  int it = 0, st = 3;
  double perr = 0.0;
  if (valid) {
    rho = a.Uout[z];
    ke = a.split[(i64)SDC_NX * Z + z];
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) b[i] = a.split[(i64)i * Z + z];
#pragma unroll
    for (int s = 0; s < SDC_NS; ++s) x[s] = a.guess[(i64)(SDC_NH + s) * Z + z];
    x[SDC_NX - 1] = a.split[(i64)(SDC_NX + 1) * Z + z];
    it = newton_fast<MT>(x, b, 1.0 / rho, 1.0 / fabs(b[SDC_NX - 1]), a.dtm, P, a.gm1, a.ctl.tol, a.ctl.tau, 1,
                         min(a.ctl.cap, a.ctl.maxiter), st, perr);
  }
  const bool defer = valid && (st == 2 || (st == 1 && a.ctl.cap < a.ctl.maxiter));
  const long long slot = defer_slot(a.q.count, defer);
  int nu = 0;
  bool nonfinite = false;
  if (defer) {
    const i64 cap = a.q.capacity;
    a.q.z[slot] = z;
    a.q.it[slot] = st == 2 ? -it : it;
    a.q.perr[slot] = perr;
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) {
      a.q.x[(i64)i * cap + slot] = x[i];
      a.q.b[(i64)i * cap + slot] = b[i];
    }
    a.q.aux[slot] = rho;
    a.q.aux[cap + slot] = ke;
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) a.q.aux[(i64)(2 + d) * cap + slot] = a.Uout[(i64)(1 + d) * Z + z];
  } else if (valid) {
    nu = st == 0 ? it : -1;
    transition_store<false>(a, z, rho, ke, nullptr, x, P);
    nonfinite = !all_finite(x);
  }
  stats_block(a.stats, nu, valid && !defer, nonfinite, 0);
}

// the explicit-part kernels share the CUs with the Newton kernel: few registers
#define SDC_PRE __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
extern "C" __global__ SDC_PRE void sdc_transition_pre_first(TransArgs a) { transition_pre_body<KIND_FIRST>(a); }
extern "C" __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void sdc_transition_pre_node0(
    TransArgs a) {
  transition_pre_body<KIND_NODE0>(a);
}
extern "C" __global__ SDC_PRE void sdc_transition_pre_later(TransArgs a) { transition_pre_body<KIND_LATER>(a); }
extern "C" __global__ __launch_bounds__(256) void sdc_transition_newton(TransArgs a) { transition_newton_body<SdcMT>(a); }
extern "C" __global__ __launch_bounds__(256) SDC_OCC2 void sdc_transition_newton_o2(TransArgs a) {
  transition_newton_body<SdcMT>(a);
}

extern "C" __global__ __launch_bounds__(256) void sdc_transition_first(TransArgs a) { transition_body<SdcMT, KIND_FIRST>(a); }
extern "C" __global__ __launch_bounds__(256) void sdc_transition_node0(TransArgs a) { transition_body<SdcMT, KIND_NODE0>(a); }
extern "C" __global__ __launch_bounds__(256) void sdc_transition_later(TransArgs a) { transition_body<SdcMT, KIND_LATER>(a); }
extern "C" __global__ __launch_bounds__(256) SDC_OCC2 void sdc_transition_first_o2(TransArgs a) {
  transition_body<SdcMT, KIND_FIRST>(a);
}
extern "C" __global__ __launch_bounds__(256) SDC_OCC2 void sdc_transition_node0_o2(TransArgs a) {
  transition_body<SdcMT, KIND_NODE0>(a);
}
extern "C" __global__ __launch_bounds__(256) SDC_OCC2 void sdc_transition_later_o2(TransArgs a) {
  transition_body<SdcMT, KIND_LATER>(a);
}
extern "C" __global__ __launch_bounds__(256) void sdc_transition_finish(TransArgs a) { transition_finish_body<SdcMT>(a); }

// reset of the deferred-zone counter (a kernel, so captured graphs stay valid)
// ------------------------------------------------------------ fourth order
// The fourth-order method in space (Sec. 2: Simpson in time with McCorquodale
// and Colella's reconstruction), on zone averages of a periodic grid:
//  - face average along d of the face at i+1/2: 7/12 (u_i + u_{i+1})
//    - 1/12 (u_{i-1} + u_{i+2});
//  - face-centre value: face average minus 1/24 of its second differences
//    across the face (the other directions); the flux at the face centre is
//    the Euler flux of that value, and the face-averaged flux adds 1/24 of the
//    second differences across the face of the flux of the face averages;
//  - no limiter: both face states coincide, the Rusanov term vanishes;
//  - zone centres u_c = <u> - lap/24 and zone averages <f> = f_c + lap/24,
//    lap the sum over directions of second differences.
// Zone-per-thread kernels: stencil values come through L1/L2.

__device__ __forceinline__ void zone_coords(i64 z, const int* n, int* c) {
  const i64 plane = (i64)n[0] * n[1];
  c[2] = (int)(z / plane);
  const i64 r = z - (i64)c[2] * plane;
  c[1] = (int)(r / n[0]);
  c[0] = (int)(r - (i64)c[1] * n[0]);
}

// zone (c + o0 e_d0 + o1 e_d1), periodic, for offsets of any size
__device__ __forceinline__ i64 zone_off(const int* c, const int* n, int d0, int o0, int d1, int o1) {
  int q[3] = {c[0], c[1], c[2]};
  q[d0] += o0;
  q[d1] += o1;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    q[e] %= n[e];
    if (q[e] < 0) q[e] += n[e];
  }
  return (i64)q[0] + (i64)n[0] * ((i64)q[1] + (i64)n[1] * q[2]);
}

// the 2 DIM neighbour zones (+d, -d per direction) of the zone at c
struct Nbr {
  i64 p[SDC_DIM], m[SDC_DIM];
};
__device__ __forceinline__ Nbr neighbours(const int* c, const int* n) {
  Nbr b;
#pragma unroll
  for (int d = 0; d < SDC_DIM; ++d) {
    b.p[d] = zone_off(c, n, d, 1, d, 0);
    b.m[d] = zone_off(c, n, d, -1, d, 0);
  }
  return b;
}

// second differences of u summed over directions: sum_d (u_{+d} - 2 u) + u_{-d}
__device__ __forceinline__ double lap_sum(const double* u, const Nbr& b, double u0) {
  double l = 0.0;
#pragma unroll
  for (int d = 0; d < SDC_DIM; ++d) l += (u[b.p[d]] - 2.0 * u0) + u[b.m[d]];
  return l;
}

// Transverse positions of a face normal to D: the face itself, then +/- one
// zone along every other direction, in increasing direction order.
#define SDC_NT (2 * SDC_DIM - 1)
template <int D>
__device__ __forceinline__ void transverse(int t, int& dd, int& o) {
  // t = 0: the face; t = 1 + 2 j (+) and 2 + 2 j (-) for the j-th other direction
  dd = D;
  o = 0;
  if (t > 0) {
    const int j = (t - 1) >> 1;
    dd = j < D ? j : j + 1;
    o = (t & 1) ? 1 : -1;
  }
}

// Face averages along D of every zone's face i+1/2, all components: a pass of
// its own, so that the flux kernel reads each face average once per
// transverse position instead of re-forming it from four zone averages.
template <int D>
__device__ __forceinline__ void faceavg4_body(const Flux4Args& a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= a.Z) return;
  int c[3];
  zone_coords(z, a.n, c);
  const i64 zm = zone_off(c, a.n, D, -1, D, 0), zp = zone_off(c, a.n, D, 1, D, 0), zpp = zone_off(c, a.n, D, 2, D, 0);
  for (int q = 0; q < SDC_NC; ++q) {
    const double* u = a.U + (i64)q * a.Z;
    a.Uf[(i64)q * a.Z + z] = (7.0 / 12.0) * (u[z] + u[zp]) - (1.0 / 12.0) * (u[zm] + u[zpp]);
  }
}
extern "C" __global__ __launch_bounds__(256) void sdc_faceavg4_0(Flux4Args a) { faceavg4_body<0>(a); }
#if SDC_DIM >= 2
extern "C" __global__ __launch_bounds__(256) void sdc_faceavg4_1(Flux4Args a) { faceavg4_body<1>(a); }
#endif
#if SDC_DIM >= 3
extern "C" __global__ __launch_bounds__(256) void sdc_faceavg4_2(Flux4Args a) { faceavg4_body<2>(a); }
#endif



// 1/24 of the second differences across the face from the face values v[t]
__device__ __forceinline__ double cross_lap24(const double* v) {
  double l = 0.0;
#pragma unroll
  for (int j = 0; j < SDC_DIM - 1; ++j) l += (v[1 + 2 * j] - 2.0 * v[0]) + v[2 + 2 * j];
  return l / 24.0;
}

template <int D>
__device__ __forceinline__ void flux4_body(const Flux4Args& a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= a.Z) return;
  const i64 Z = a.Z;
  int c[3];
  zone_coords(z, a.n, c);
  // hydro components: face averages at the transverse positions, their
  // fluxes and velocities, the face-centre value and its flux
  double W[SDC_NT][SDC_NH], un[SDC_NT];
  double F[SDC_NH], Fc[SDC_NH], Wc[SDC_NH], unc, p, cs;
  i64 zt[SDC_NT];  // zones of the transverse positions (the same for every component)
#pragma unroll
  for (int t = 0; t < SDC_NT; ++t) {
    int dd, o;
    transverse<D>(t, dd, o);
    zt[t] = zone_off(c, a.n, dd, o, dd, 0);
  }
#pragma unroll
  for (int t = 0; t < SDC_NT; ++t) {
#pragma unroll
    for (int q = 0; q < SDC_NH; ++q) W[t][q] = a.Uf[(i64)q * Z + zt[t]];
  }
#pragma unroll
  for (int q = 0; q < SDC_NH; ++q) {
    double v[SDC_NT];
#pragma unroll
    for (int t = 0; t < SDC_NT; ++t) v[t] = W[t][q];
    Wc[q] = W[0][q] - cross_lap24(v);
  }
  hydro_flux(Wc, D, a.gamma, Fc, unc, p, cs);
  {
    double Ft[SDC_NT][SDC_NH];
#pragma unroll
    for (int t = 0; t < SDC_NT; ++t) hydro_flux(W[t], D, a.gamma, Ft[t], un[t], p, cs);
#pragma unroll
    for (int q = 0; q < SDC_NH; ++q) {
      double v[SDC_NT];
#pragma unroll
      for (int t = 0; t < SDC_NT; ++t) v[t] = Ft[t][q];
      F[q] = Fc[q] + cross_lap24(v);
    }
  }
#pragma unroll
  for (int q = 0; q < SDC_NH; ++q) a.F[(i64)q * Z + z] = F[q];
  // species: passive, flux u_n times the species density
  for (int s = 0; s < SDC_NS; ++s) {
    const double* us = a.Uf + (i64)(SDC_NH + s) * Z;
    double v[SDC_NT], f[SDC_NT];
#pragma unroll
    for (int t = 0; t < SDC_NT; ++t) {
      v[t] = us[zt[t]];
      f[t] = v[t] * un[t];
    }
    const double vc = v[0] - cross_lap24(v);
    a.F[(i64)(SDC_NH + s) * Z + z] = vc * unc + cross_lap24(f);
  }
}

extern "C" __global__ __launch_bounds__(256) void sdc_flux4_0(Flux4Args a) { flux4_body<0>(a); }
#if SDC_DIM >= 2
extern "C" __global__ __launch_bounds__(256) void sdc_flux4_1(Flux4Args a) { flux4_body<1>(a); }
#endif
#if SDC_DIM >= 3
extern "C" __global__ __launch_bounds__(256) void sdc_flux4_2(Flux4Args a) { flux4_body<2>(a); }
#endif

// A (=, or -=) (F_{i+1/2} - F_{i-1/2}) / dx_d for the face fluxes F along d
template <int D>
__device__ __forceinline__ void div4_body(const Flux4Args& a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= a.Z) return;
  const i64 Z = a.Z;
  int c[3];
  zone_coords(z, a.n, c);
  const i64 zm = zone_off(c, a.n, D, -1, D, 0);
  for (int q = 0; q < SDC_NC; ++q) {
    const double dv = (a.F[(i64)q * Z + z] - a.F[(i64)q * Z + zm]) * a.idx;
    a.A[(i64)q * Z + z] = (a.first ? 0.0 : a.A[(i64)q * Z + z]) - dv;
  }
}
extern "C" __global__ __launch_bounds__(256) void sdc_div4_0(Flux4Args a) { div4_body<0>(a); }
#if SDC_DIM >= 2
extern "C" __global__ __launch_bounds__(256) void sdc_div4_1(Flux4Args a) { div4_body<1>(a); }
#endif
#if SDC_DIM >= 3
extern "C" __global__ __launch_bounds__(256) void sdc_div4_2(Flux4Args a) { div4_body<2>(a); }
#endif

// dst = src + sign * lap / 24 on ncomp components (src and dst distinct)
extern "C" __global__ __launch_bounds__(256) void sdc_convert4(ConvArgs a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= a.Z) return;
  int c[3];
  zone_coords(z, a.n, c);
  const Nbr nb = neighbours(c, a.n);
  for (int q = 0; q < a.ncomp; ++q) {
    const double* u = a.src + (i64)q * a.Z;
    const double u0 = u[z];
    a.dst[(i64)q * a.Z + z] = u0 + a.sign * (lap_sum(u, nb, u0) / 24.0);
  }
}

// R at the zone-centre values of U, into R [NX][Z]
extern "C" __global__ __launch_bounds__(256) void sdc_source4_centre(O4Args a) {
  ParamPtr P = stage_params(a.P);
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= a.Z) return;
  const i64 Z = a.Z;
  int c[3];
  zone_coords(z, a.n, c);
  const Nbr nb = neighbours(c, a.n);
  double uc[SDC_NC];
  for (int q = 0; q < SDC_NC; ++q) {
    const double* u = a.U + (i64)q * Z;
    const double u0 = u[z];
    uc[q] = u0 - lap_sum(u, nb, u0) / 24.0;
  }
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < SDC_DIM; ++d) ke = fma(uc[1 + d], uc[1 + d], ke);
  ke = 0.5 * ke / uc[0];
  double x[SDC_NX], R[SDC_NX];
#pragma unroll
  for (int s = 0; s < SDC_NS; ++s) x[s] = uc[SDC_NH + s];
  x[SDC_NX - 1] = uc[1 + SDC_DIM] - ke;
  net_source(x, 1.0 / uc[0], P, a.gm1, R);
#pragma unroll
  for (int i = 0; i < SDC_NX; ++i) a.R[(i64)i * Z + z] = R[i];
}

// Right-hand side of the transition into Uout (zone averages) and the Newton
// guess into x4; the guess is read before Uout is written (they may share
// the node array).
template <int KIND>
__device__ __forceinline__ void rhs4_body(const TransArgs& a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= a.Z) return;
  const i64 Z = a.Z;
  double rhs[SDC_NC];
  transition_rhs<KIND>(a, z, rhs);
  {
    const double* __restrict__ g = a.guess;
    const double grho = g[z];
    double gke = 0.0;
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) {
      const double mo = g[(i64)(1 + d) * Z + z];
      gke = fma(mo, mo, gke);
    }
    gke = 0.5 * gke / grho;
    double xg[SDC_NX];
#pragma unroll
    for (int s = 0; s < SDC_NS; ++s) xg[s] = g[(i64)(SDC_NH + s) * Z + z];
    xg[SDC_NX - 1] = g[(i64)(1 + SDC_DIM) * Z + z] - gke;
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) a.x4[(i64)i * Z + z] = xg[i];
  }
#pragma unroll
  for (int q = 0; q < SDC_NC; ++q) a.Uout[(i64)q * Z + z] = rhs[q];
}
extern "C" __global__ __launch_bounds__(256) void sdc_rhs4_first(TransArgs a) { rhs4_body<KIND_FIRST>(a); }
extern "C" __global__ __launch_bounds__(256) void sdc_rhs4_node0(TransArgs a) { rhs4_body<KIND_NODE0>(a); }
extern "C" __global__ __launch_bounds__(256) void sdc_rhs4_later(TransArgs a) { rhs4_body<KIND_LATER>(a); }

// Newton inputs at zone centres: rho_c and b_c = (rhs_c X, rhs_c E - KE_c)
extern "C" __global__ __launch_bounds__(256) void sdc_newton_inputs4(O4Args a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= a.Z) return;
  const i64 Z = a.Z;
  int c[3];
  zone_coords(z, a.n, c);
  const Nbr nb = neighbours(c, a.n);
  double rc[SDC_NC];
  for (int q = 0; q < SDC_NC; ++q) {
    const double* u = a.U + (i64)q * Z;
    const double u0 = u[z];
    rc[q] = u0 - lap_sum(u, nb, u0) / 24.0;
  }
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < SDC_DIM; ++d) ke = fma(rc[1 + d], rc[1 + d], ke);
  ke = 0.5 * ke / rc[0];
  a.rho_c[z] = rc[0];
#pragma unroll
  for (int s = 0; s < SDC_NS; ++s) a.b_c[(i64)s * Z + z] = rc[SDC_NH + s];
  a.b_c[(i64)(SDC_NX - 1) * Z + z] = rc[1 + SDC_DIM] - ke;
}

// <R> = R_c + lap(R_c) / 24; U^{m+1} = rhs + dt_m <R> (reacting components;
// rho and rho u are the rhs); R^{m+1} = <R>
extern "C" __global__ __launch_bounds__(256) void sdc_average_store4(O4Args a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= a.Z) return;
  const i64 Z = a.Z;
  int c[3];
  zone_coords(z, a.n, c);
  const Nbr nb = neighbours(c, a.n);
  for (int i = 0; i < SDC_NX; ++i) {
    const double* r = a.R_c + (i64)i * Z;
    const double r0 = r[z];
    const double ravg = r0 + lap_sum(r, nb, r0) / 24.0;
    a.R[(i64)i * Z + z] = ravg;
    const int q = i == SDC_NX - 1 ? 1 + SDC_DIM : SDC_NH + i;
    a.U[(i64)q * Z + z] = fma(a.dtm, ravg, a.U[(i64)q * Z + z]);
  }
}

// ------------------------------------------------------------ refined patches
// Two-level hierarchy around the SDC step (extension to refinement with
// subcycling, Sec. 2 and Sec. 5): the patches are padded boxes whose G = 2
// ghost zones are filled from the coarse level before every evaluation of A,
// interpolated in time with the Lagrange weights of the coarse nodes and in
// space conservatively and piecewise-linearly (central coarse slopes).

__device__ __forceinline__ i64 coarse_zone(const int* c, const int* n, int e, int o) {
  int q[3] = {c[0], c[1], c[2]};
  q[e] += o;
  q[e] = q[e] < 0 ? q[e] + n[e] : (q[e] >= n[e] ? q[e] - n[e] : q[e]);
  return (i64)q[0] + (i64)n[0] * ((i64)q[1] + (i64)n[1] * q[2]);
}

// time-interpolated coarse value of component array offset `off` at zone z
__device__ __forceinline__ double coarse_at(const AmrFillArgs& a, i64 off, i64 z) {
  double v = 0.0;
  for (int j = 0; j < a.nnodes; ++j) v += a.w[j] * a.Uc[j][off + z];
  return v;
}

extern "C" __global__ __launch_bounds__(256) void sdc_amr_fill(AmrFillArgs a) {
  const i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.count) return;
  const AmrGhost e = a.list[g];
  const i64 zp = coarse_zone(e.pc, a.nc, 0, 0);
  for (int q = 0; q < SDC_NC; ++q) {
    const i64 off = (i64)q * a.Zc;
    double v = coarse_at(a, off, zp);
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) {
      const double slope = 0.5 * (coarse_at(a, off, coarse_zone(e.pc, a.nc, d, 1)) -
                                  coarse_at(a, off, coarse_zone(e.pc, a.nc, d, -1)));
      v += ((e.sig >> d) & 1 ? 0.25 : -0.25) * slope;
    }
    a.Uf[(i64)q * a.Zf + e.zf] = v;
  }
}

// A = 0 in the ghost zones (their transitions are then reaction-only)
extern "C" __global__ __launch_bounds__(256) void sdc_amr_zero(AmrFillArgs a) {
  const i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.count) return;
  const i64 z = a.list[g].zf;
  for (int q = 0; q < SDC_NC; ++q) a.Uf[(i64)q * a.Zf + z] = 0.0;
}

// Face flux (the reconstruction and Rusanov flux of the advective term) at
// listed faces, accumulated into a register: reg += coef * F.
template <int D>
__device__ __forceinline__ void amr_face_flux(const AmrFluxArgs& a, const AmrFace& f, i64 g) {
  i64 z[4];
#pragma unroll
  for (int o = 0; o < 4; ++o) z[o] = f.base + coarse_zone(f.c, f.n, D, o - 1);
  double WL[SDC_NH], WR[SDC_NH], F[SDC_NH];
  auto states = [&](int q, double& L, double& R) {
    const double* u = a.U + (i64)q * a.Z;
    const double um = u[z[0]], u0 = u[z[1]], u1 = u[z[2]], u2 = u[z[3]];
    L = u0 + 0.5 * slope_of(um, u0, u1, a.slope);
    R = u1 - 0.5 * slope_of(u0, u1, u2, a.slope);
  };
#pragma unroll
  for (int q = 0; q < SDC_NH; ++q) states(q, WL[q], WR[q]);
  FaceHydro fh;
  hydro_face(WL, WR, D, a.gamma, a.alpha, F, fh);
#pragma unroll
  for (int q = 0; q < SDC_NH; ++q) a.reg[(i64)q * a.count + g] += a.coef * F[q];
  for (int s = 0; s < SDC_NS; ++s) {
    double L, R;
    states(SDC_NH + s, L, R);
    a.reg[(i64)(SDC_NH + s) * a.count + g] += a.coef * species_face(L, R, fh);
  }
}

extern "C" __global__ __launch_bounds__(256) void sdc_amr_flux(AmrFluxArgs a) {
  const i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.count) return;
  const AmrFace f = a.faces[g];
  if (f.d == 0) amr_face_flux<0>(a, f, g);
#if SDC_DIM >= 2
  else if (f.d == 1) amr_face_flux<1>(a, f, g);
#endif
#if SDC_DIM >= 3
  else amr_face_flux<2>(a, f, g);
#endif
}

// Refluxing: the uncovered coarse zones next to a patch replace the coarse
// flux through the shared face by the fine fluxes averaged over it.
extern "C" __global__ __launch_bounds__(256) void sdc_amr_reflux(AmrSyncArgs a) {
  const i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.nreflux) return;
  const AmrReflux r = a.reflux[g];
  for (int q = 0; q < SDC_NC; ++q) {
    const double* ff = a.regf + (i64)q * a.nregf;
    double f;
    if (SDC_DIM == 1) f = ff[r.ff[0]];
    else if (SDC_DIM == 2) f = 0.5 * (ff[r.ff[0]] + ff[r.ff[1]]);
    else f = 0.5 * (0.5 * (ff[r.ff[0]] + ff[r.ff[1]]) + 0.5 * (ff[r.ff[2]] + ff[r.ff[3]]));
    const double corr = (f - a.regc[(i64)q * a.nregc + r.fc]) / r.h;
    a.Uc[(i64)q * a.Zc + r.zu] += r.sign * corr;
  }
}

// Average-down: every covered coarse zone takes the mean of its fine zones.
extern "C" __global__ __launch_bounds__(256) void sdc_amr_average(AmrSyncArgs a) {
  const i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.ncover) return;
  const AmrCover c = a.cover[g];
  for (int q = 0; q < SDC_NC; ++q) {
    const double* u = a.Uf + (i64)q * a.Zf + c.f0;
    double acc = 0.0;
    for (int cz = 0; cz < (SDC_DIM >= 3 ? 2 : 1); ++cz)
      for (int cy = 0; cy < (SDC_DIM >= 2 ? 2 : 1); ++cy)
        for (int cx = 0; cx < 2; ++cx) acc += u[cz * c.sz + cy * c.sy + cx];
    a.Uc[(i64)q * a.Zc + c.zc] = acc / (double)(1 << SDC_DIM);
  }
}

extern "C" __global__ void sdc_reset_counter(unsigned* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0u;
}


// ---- constant fill (used instead of memset so that captured graphs stay valid)
extern "C" __global__ __launch_bounds__(256) void sdc_fill(FillArgs a) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n) a.p[i] = a.v;
}

// zeroes a.count arrays, every thread striding over each in turn
extern "C" __global__ __launch_bounds__(256) void sdc_zero_list(ZeroListArgs a) {
  const i64 stride = (i64)gridDim.x * blockDim.x;
  for (int j = 0; j < a.count; ++j) {
    double* __restrict__ p = a.p[j];
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < a.n[j]; i += stride) p[i] = 0.0;
  }
}

// ====================================================================== adjoint
// Reverse mode of the SDC step for gradients of a scalar objective with respect
// to the state and the rate parameters theta = (lnA_r, E_r).  Each implicit
// reaction solve is differentiated with the implicit-function theorem at its
// converged root: with M = I - dt_m dR/dx, mu = M^{-T} xbar gives bbar = mu and
// the parameter and density adjoints dt_m (dR/dtheta)^T mu, dt_m (dR/drho)^T mu.
// The advective term is differentiated in its smooth mode (central slopes,
// frozen Rusanov speed), where it is a differentiable function of U.

// (dF/dU)^T w for the Euler flux plus passive species in direction d at state W.
__device__ __forceinline__ void flux_jt(const double* W, int d, double gamma, const double* w, double* v) {
  const double g = gamma - 1.0;
  const double rho = W[0], ir = 1.0 / rho;
  double u[SDC_DIM], q2 = 0.0, wmu = 0.0;
#pragma unroll
  for (int k = 0; k < SDC_DIM; ++k) {
    u[k] = W[1 + k] * ir;
    q2 = fma(u[k], u[k], q2);
    wmu = fma(w[1 + k], u[k], wmu);
  }
  const double E = W[1 + SDC_DIM];
  const double p = g * (E - 0.5 * rho * q2);
  const double H = (E + p) * ir;
  const double ud = u[d], wmd = w[1 + d], wE = w[1 + SDC_DIM];
  double wsX = 0.0;
#pragma unroll
  for (int s = 0; s < SDC_NS; ++s) wsX = fma(w[SDC_NH + s], W[SDC_NH + s] * ir, wsX);
  const double hq = 0.5 * g * q2;
  v[0] = -ud * wmu + wmd * hq + wE * ud * (hq - H) - ud * wsX;
#pragma unroll
  for (int k = 0; k < SDC_DIM; ++k) {
    double t = w[1 + k] * ud - g * u[k] * wmd - g * u[k] * ud * wE;
    if (k == d) t += w[0] + wmu + H * wE + wsX;
    v[1 + k] = t;
  }
  v[1 + SDC_DIM] = g * wmd + (1.0 + g) * ud * wE;
#pragma unroll
  for (int s = 0; s < SDC_NS; ++s) v[SDC_NH + s] = ud * w[SDC_NH + s];
}

extern "C" __global__ __launch_bounds__(256) void sdc_advect_vjp(AdvVjpArgs a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= a.Z) return;
  int c3[3] = {0, 0, 0};
  {
    i64 t = z;
    c3[0] = (int)(t % a.n[0]);
    t /= a.n[0];
    if (SDC_DIM > 1) {
      c3[1] = (int)(t % a.n[1]);
      t /= a.n[1];
    }
    if (SDC_DIM > 2) c3[2] = (int)t;
  }
  double ub[SDC_NC];
#pragma unroll
  for (int c = 0; c < SDC_NC; ++c) ub[c] = 0.0;
  i64 stride = 1;
  for (int d = 0; d < SDC_DIM; ++d) {
    const int nd = a.n[d], cd = c3[d];
    i64 off[7];  // zones j-3 .. j+3 along d
    for (int s = -3; s <= 3; ++s) {
      int cc = cd + s;
      while (cc < 0) cc += nd;
      while (cc >= nd) cc -= nd;
      off[s + 3] = z + (i64)(cc - cd) * stride;
    }
    // faces i+1/2 for i = j-2 .. j+1 (r = i - j = -2 .. 1)
    for (int r = -2; r <= 1; ++r) {
      const double cL = r == 1 ? -0.25 : (r == 0 ? 1.0 : (r == -1 ? 0.25 : 0.0));
      const double cR = r == 0 ? 0.25 : (r == -1 ? 1.0 : (r == -2 ? -0.25 : 0.0));
      const i64 im1 = off[r + 2], i0 = off[r + 3], ip1 = off[r + 4], ip2 = off[r + 5];
      double Fb[SDC_NC], W[SDC_NC], v[SDC_NC];
#pragma unroll
      for (int c = 0; c < SDC_NC; ++c) Fb[c] = (a.Abar[(i64)c * a.Z + ip1] - a.Abar[(i64)c * a.Z + i0]) * a.idx[d];
      if (cL != 0.0) {
#pragma unroll
        for (int c = 0; c < SDC_NC; ++c) {
          const double* Uc = a.U + (i64)c * a.Z;
          W[c] = Uc[i0] + 0.25 * (Uc[ip1] - Uc[im1]);
        }
        flux_jt(W, d, a.gamma, Fb, v);
#pragma unroll
        for (int c = 0; c < SDC_NC; ++c) ub[c] = fma(cL, 0.5 * v[c] + 0.5 * a.alpha * Fb[c], ub[c]);
      }
      if (cR != 0.0) {
#pragma unroll
        for (int c = 0; c < SDC_NC; ++c) {
          const double* Uc = a.U + (i64)c * a.Z;
          W[c] = Uc[ip1] - 0.25 * (Uc[ip2] - Uc[i0]);
        }
        flux_jt(W, d, a.gamma, Fb, v);
#pragma unroll
        for (int c = 0; c < SDC_NC; ++c) ub[c] = fma(cR, 0.5 * v[c] - 0.5 * a.alpha * Fb[c], ub[c]);
      }
    }
    stride *= nd;
  }
#pragma unroll
  for (int c = 0; c < SDC_NC; ++c) a.Ubar[(i64)c * a.Z + z] += ub[c];
}

// Dense transposed solve M^T y = c with a partially pivoted LU of M (used when
// the fixed-order factorisation meets a small pivot).
__device__ __attribute__((noinline)) VecX dense_solve_t(VecX xv, VecX cv, double irho, double dtm, ParamPtr P,
                                                        double gm1) {
  double x[SDC_NX], M[SDC_NX * SDC_NX], r[SDC_NX], y[SDC_NX];
  int piv[SDC_NX];
  for (int i = 0; i < SDC_NX; ++i) x[i] = xv.v[i];
  dense_newton_matrix(x, x, irho, dtm, P, gm1, M, r);
  for (int k = 0; k < SDC_NX; ++k) {
    int p = k;
    double best = fabs(M[k * SDC_NX + k]);
    for (int i = k + 1; i < SDC_NX; ++i)
      if (fabs(M[i * SDC_NX + k]) > best) {
        best = fabs(M[i * SDC_NX + k]);
        p = i;
      }
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < SDC_NX; ++j) {
        const double t = M[k * SDC_NX + j];
        M[k * SDC_NX + j] = M[p * SDC_NX + j];
        M[p * SDC_NX + j] = t;
      }
    const double inv = 1.0 / M[k * SDC_NX + k];
    for (int i = k + 1; i < SDC_NX; ++i) {
      const double l = M[i * SDC_NX + k] * inv;
      M[i * SDC_NX + k] = l;
      for (int j = k + 1; j < SDC_NX; ++j) M[i * SDC_NX + j] = fma(-l, M[k * SDC_NX + j], M[i * SDC_NX + j]);
    }
  }
  // P M = L U  =>  M^T = U^T L^T P:  U^T w = c, L^T v = w, y = P^T v
  for (int k = 0; k < SDC_NX; ++k) {
    double s = cv.v[k];
    for (int j = 0; j < k; ++j) s = fma(-M[j * SDC_NX + k], y[j], s);
    y[k] = s / M[k * SDC_NX + k];
  }
  for (int k = SDC_NX - 1; k >= 0; --k) {
    double s = y[k];
    for (int i = k + 1; i < SDC_NX; ++i) s = fma(-M[i * SDC_NX + k], y[i], s);
    y[k] = s;
  }
  for (int k = SDC_NX - 1; k >= 0; --k)
    if (piv[k] != k) {
      const double t = y[k];
      y[k] = y[piv[k]];
      y[piv[k]] = t;
    }
  VecX out;
  for (int i = 0; i < SDC_NX; ++i) out.v[i] = y[i];
  return out;
}

// Deterministic block sum of the per-zone parameter adjoints into part[block][*].
__device__ __forceinline__ void theta_block_sum(double* gl, double* gE, double* part) {
  __shared__ double sh[4];
  for (int p = 0; p < 2 * SDC_NR; ++p) {
    double v = p < SDC_NR ? gl[p] : gE[p - SDC_NR];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
      part[(i64)blockIdx.x * (2 * SDC_NR) + p] = t;
    }
    __syncthreads();
  }
}

template <int FIRST>
__device__ __forceinline__ void transition_adjoint_body(const TransAdjArgs& a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = z < a.Z;
  ParamPtr P = stage_params(a.P);
  double gl[SDC_NRA], gE[SDC_NRA];
#pragma unroll
  for (int r = 0; r < SDC_NRA; ++r) gl[r] = gE[r] = 0.0;
  if (valid) {
    const i64 Z = a.Z;
    const double rho = a.Uout[z];
    const double irho = 1.0 / rho;
    double mom[SDC_DIM], ke = 0.0;
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) {
      mom[d] = a.Uout[(i64)(1 + d) * Z + z];
      ke = fma(mom[d], mom[d], ke);
    }
    ke = 0.5 * ke * irho;
    double x[SDC_NX], w[SDC_NX], xb[SDC_NX], mu[SDC_NX];
#pragma unroll
    for (int s = 0; s < SDC_NS; ++s) x[s] = a.Uout[(i64)(SDC_NH + s) * Z + z];
    x[SDC_NX - 1] = a.Uout[(i64)(1 + SDC_DIM) * Z + z] - ke;
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) w[i] = a.Routbar[(i64)i * Z + z];
    // R^{m+1} = R(x; rho): its adjoint feeds x, rho and theta
    double rhob;
    net_vjp(x, irho, P, a.gm1, w, xb, &rhob, gl, gE);
#pragma unroll
    for (int s = 0; s < SDC_NS; ++s) mu[s] = a.Uoutbar[(i64)(SDC_NH + s) * Z + z] + xb[s];
    const double UbE = a.Uoutbar[(i64)(1 + SDC_DIM) * Z + z];
    mu[SDC_NX - 1] = UbE + xb[SDC_NX - 1];
    rhob += a.Uoutbar[z];
    // implicit solve: mu = M^{-T} xbar at the converged root
    {
      double G[SDC_NX], Mtx[SDC_NNZ];
      net_residual_matrix<double, const double*>(x, x, irho, a.dtm, P, a.gm1, G, Mtx);
      if (net_lu<double>(Mtx, a.tau)) {
        net_solve_t<double>(Mtx, mu);
      } else {
        VecX xv, cv;
#pragma unroll
        for (int i = 0; i < SDC_NX; ++i) {
          xv.v[i] = x[i];
          cv.v[i] = mu[i];
        }
        const VecX y = dense_solve_t(xv, cv, irho, a.dtm, P, a.gm1);
#pragma unroll
        for (int i = 0; i < SDC_NX; ++i) mu[i] = y.v[i];
      }
    }
    // parameters and density through the solve: dt_m (dR/d.)^T mu
    {
      double wm[SDC_NX], xb2[SDC_NX], rhob2;
#pragma unroll
      for (int i = 0; i < SDC_NX; ++i) wm[i] = a.dtm * mu[i];
      net_vjp(x, irho, P, a.gm1, wm, xb2, &rhob2, gl, gE);
      rhob += rhob2;
    }
    // bbar = mu; rho E = x_e + KE and b_e = rhs_E - KE
    const double keb = UbE - mu[SDC_NX - 1];
    double rb[SDC_NC];
    rb[0] = rhob - keb * ke * irho;
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) rb[1 + d] = a.Uoutbar[(i64)(1 + d) * Z + z] + keb * mom[d] * irho;
    rb[1 + SDC_DIM] = mu[SDC_NX - 1];
#pragma unroll
    for (int s = 0; s < SDC_NS; ++s) rb[SDC_NH + s] = mu[s];
    // transposes of the right-hand side assembly
#pragma unroll
    for (int c = 0; c < SDC_NC; ++c) {
      const i64 o = (i64)c * Z + z;
      const int ri = c == 1 + SDC_DIM ? SDC_NX - 1 : (c >= SDC_NH ? c - SDC_NH : -1);
      a.Umbar[o] += rb[c];
      if (a.Ambar) a.Ambar[o] += a.dtm * rb[c];
      if (!FIRST) {
        for (int j = 0; j <= a.M; ++j) {
          const double f = a.dt * a.S[a.m][j] * rb[c];
          a.Aoldbar[j][o] += f;
          if (ri >= 0) a.Roldbar[j][(i64)ri * Z + z] += f;
        }
        if (a.m >= 1) a.Aoldbar[a.m][o] -= a.dtm * rb[c];
        if (ri >= 0) a.Roldbar[a.m + 1][(i64)ri * Z + z] -= a.dtm * rb[c];
      }
    }
  }
  theta_block_sum(gl, gE, a.theta_part);
}

extern "C" __global__ __launch_bounds__(256) void sdc_transition_adjoint_first(TransAdjArgs a) {
  transition_adjoint_body<1>(a);
}
extern "C" __global__ __launch_bounds__(256) void sdc_transition_adjoint(TransAdjArgs a) {
  transition_adjoint_body<0>(a);
}

// Ubar += (dR(U)/dU)^T Rbar at U, with x = (rho X, rho E - KE); parameter partials.
extern "C" __global__ __launch_bounds__(256) void sdc_source_vjp(SourceVjpArgs a) {
  const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = z < a.Z;
  ParamPtr P = stage_params(a.P);
  double gl[SDC_NRA], gE[SDC_NRA];
#pragma unroll
  for (int r = 0; r < SDC_NRA; ++r) gl[r] = gE[r] = 0.0;
  if (valid) {
    const i64 Z = a.Z;
    const double rho = a.U[z], irho = 1.0 / rho;
    double mom[SDC_DIM], ke = 0.0;
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) {
      mom[d] = a.U[(i64)(1 + d) * Z + z];
      ke = fma(mom[d], mom[d], ke);
    }
    ke = 0.5 * ke * irho;
    double x[SDC_NX], w[SDC_NX], xb[SDC_NX], rhob;
#pragma unroll
    for (int s = 0; s < SDC_NS; ++s) x[s] = a.U[(i64)(SDC_NH + s) * Z + z];
    x[SDC_NX - 1] = a.U[(i64)(1 + SDC_DIM) * Z + z] - ke;
#pragma unroll
    for (int i = 0; i < SDC_NX; ++i) w[i] = a.Rbar[(i64)i * Z + z];
    net_vjp(x, irho, P, a.gm1, w, xb, &rhob, gl, gE);
    const double keb = -xb[SDC_NX - 1];
    a.Ubar[z] += rhob - keb * ke * irho;
#pragma unroll
    for (int d = 0; d < SDC_DIM; ++d) a.Ubar[(i64)(1 + d) * Z + z] += keb * mom[d] * irho;
    a.Ubar[(i64)(1 + SDC_DIM) * Z + z] += xb[SDC_NX - 1];
#pragma unroll
    for (int s = 0; s < SDC_NS; ++s) a.Ubar[(i64)(SDC_NH + s) * Z + z] += xb[s];
  }
  theta_block_sum(gl, gE, a.theta_part);
}

// thetabar[p] += sum over blocks of part[b][p], in block order (one block per p).
extern "C" __global__ __launch_bounds__(256) void sdc_theta_reduce(ThetaReduceArgs a) {
  __shared__ double sh[256];
  const int p = blockIdx.x;
  double t = 0.0;
  for (i64 b = threadIdx.x; b < a.nblocks; b += blockDim.x) t += a.part[b * a.nparam + p];
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.thetabar[p] += sh[0];
}

extern "C" __global__ __launch_bounds__(256) void sdc_axpy(AxpyArgs a) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n) a.y[i] = fma(a.a, a.x[i], a.y[i]);
}

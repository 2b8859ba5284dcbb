// lbrx: one coupled reactive-transport lattice Boltzmann step per kernel launch
// on gfx950 (MI355X), behind the C ABI of include/lbrx.h.
//
// Method: arXiv:1410.3464, Sec. 3-4 (Eq. 6-35, A2), procedure of Sec. 4.7.
//
// Kernel structure (one launch per time step):
//   * A workgroup owns a 62 x TY tile of nodes and runs one thread per node of
//     the tile plus a one-node ring (64 x (TY+2) threads, one wavefront per row).
//   * Phase 1: every thread reads its node's streamed populations (SoA, push
//     layout, coalesced along x), forms the moments (Eq. 9, 23) and the
//     effective masses psi_1, phi_1, phi_2 (Eq. 13, 15) and stages them in LDS.
//     Node types of the tile plus two rings go to LDS as bytes.
//   * Phase 2: tile threads form the forces (Eq. 11, 14, 16) from the LDS
//     stencil, the velocities (Eq. 17-19), reaction sources (Eq. 5, 27, 28),
//     both collisions (Eq. 6, 20), the status-change amendments (Sec. 4.5),
//     the volume-of-pixel update (Eq. 33, 35) and push-stream their
//     populations with halfway bounce-back and the reactive link flux.
//   * Nothing is read back in the same launch, so there is no grid-wide sync;
//     the liquid threshold uses the previous step's maximum (atomic max on the
//     bit pattern of a non-negative double), and balances accumulate into one
//     FP64 record per tile (no floating-point atomics in global memory).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbrx.h"

namespace {

// ---------------------------------------------------------------- lattice
// D2Q9 (Eq. 7): 0 rest, 1..4 axes (+x, +y, -x, -y), 5..8 diagonals.
// D2Q5 uses directions 0..4.
__host__ __device__ constexpr int ex(int a) { return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0); }
__host__ __device__ constexpr int ey(int a) { return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0); }
__host__ __device__ constexpr int opp(int a) { return a == 0 ? 0 : (a < 5 ? ((a + 1) & 3) + 1 : ((a - 3) & 3) + 5); }
// equilibrium weights (text after Eq. 8) and pseudopotential weights w(1)=1/3, w(2)=1/12 (Eq. 11)
__host__ __device__ constexpr double w9(int a) { return a == 0 ? 4.0 / 9 : (a < 5 ? 1.0 / 9 : 1.0 / 36); }
__host__ __device__ constexpr double wf(int a) { return a == 0 ? 0.0 : (a < 5 ? 1.0 / 3 : 1.0 / 12); }
static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp axes");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp diagonals");

// node-type byte: bits 0-1 type, bit 2 liquid this step, bit 3 liquid last
// step, bit 4 stranded (became SOLID_F at the end of the last step; its
// streamed-in populations are still stored).  Bit 7 marks "outside a
// non-periodic boundary" in LDS only.
constexpr uint8_t TB_T = 0x3, TB_LIQ = 0x4, TB_LIQP = 0x8, TB_STR = 0x10, TB_WALL = 0x80;
constexpr int T_FLUID = 0, T_INERT = 1, T_D = 2, T_F = 3;

constexpr int TW = 62;  // tile width: a 64-lane row minus the two ring lanes

// ledger slots, same order as lbrx_ledger
constexpr int L_MSRC = 0, L_MINJ = 2, L_MREM = 4, L_SSRC = 6, L_SHET = 14, L_SREM = 22, L_VDV = 30,
              L_VCLIP = 31, L_CLAMP = 32, L_NDIS = 33, L_NPRE = 34, L_NL2G = 35, L_NG2L = 36;
constexpr int NLED = 38;  // + steps (host)
// LDS slots of the rarely non-zero balances: 0-1 mass_inj, 2-3 mass_rem, 4 vol_clip,
// 5 psi clamps, 6 dissolved, 7 precipitated, 8-15 sol_rem, 16 liquid->gas, 17 gas->liquid
constexpr int NRARE_SLOTS = 18;
__host__ __device__ constexpr int rare_dst(int i) {
  return i == 0 ? L_MINJ : i == 1 ? L_MINJ + 1 : i == 2 ? L_MREM : i == 3 ? L_MREM + 1 : i == 4 ? L_VCLIP
       : i == 5 ? L_CLAMP : i == 6 ? L_NDIS : i == 7 ? L_NPRE : i < 16 ? L_SREM + (i - 8) : i == 16 ? L_NL2G : L_NG2L;
}

enum { HOM_FIRST = 0, HOM_R1 = 1, HOM_BI = 2 };
enum { HET_CONSUMES = 0, HET_GROWS = 1, HET_MINERAL = 2 };

struct KConst {
  int nx, ny, pitch, per_x, per_y, tiles_x, tiles_y, nblocks, ns;
  long long plane;
  double om[2], tau[2], RT, a, b, G11, psi_pre, G12, G21, w1, w2, gx, gy, a0, rho10, rho20, lfrac;
  int has_psi, has_phi1, has_phi2;
  double J[LBRX_MAX_SPECIES][5];
  double omg[LBRX_MAX_SPECIES];
  int nhom;
  int hkind[LBRX_MAX_RXN], hre0[LBRX_MAX_RXN], hre1[LBRX_MAX_RXN], hpr0[LBRX_MAX_RXN], hpr1[LBRX_MAX_RXN];
  double hk[LBRX_MAX_RXN], hKeq[LBRX_MAX_RXN], hMgas[LBRX_MAX_RXN];
  int nhet;
  int xre[LBRX_MAX_RXN], xpr[LBRX_MAX_RXN], xsurf[LBRX_MAX_RXN], xmode[LBRX_MAX_RXN], xirrev[LBRX_MAX_RXN];
  double xkap[LBRX_MAX_RXN], xCeq[LBRX_MAX_RXN], xmvol[LBRX_MAX_RXN];
};

struct KArgs {
  KConst c;
  const void* f_in;
  void* f_out;
  const void* g_in;
  void* g_out;
  const uint8_t* t_in;
  uint8_t* t_out;
  double* V;
  unsigned long long* rmax;  // 3 rotating slots
  int slot_prev, slot_cur, slot_next;
  double* led;               // [nblocks][NLED]
  unsigned int* err;         // [0] flags, [1] first failing node (min index)
  double *o_r1, *o_r2, *o_ux, *o_uy, *o_C;  // export outputs (plane-sized)
};

enum { ERR_DENSITY = 1u, ERR_EOS = 2u };

__device__ inline bool wrap(int& X, int n, int per) {
  if (X >= 0 && X < n) return true;
  if (!per) return false;
  X %= n;
  if (X < 0) X += n;
  return true;
}

template <typename T> __device__ inline T dexp(T x);
template <> __device__ inline double dexp<double>(double x) { return exp(x); }
template <> __device__ inline float dexp<float>(float x) { return expf(x); }
template <typename T> __device__ inline T dsqrt(T x);
template <> __device__ inline double dsqrt<double>(double x) { return sqrt(x); }
template <> __device__ inline float dsqrt<float>(float x) { return sqrtf(x); }

template <int NS, typename T> __device__ inline T sel(const T (&v)[NS > 0 ? NS : 1], int i) {
  T r = T(0);
#pragma unroll
  for (int k = 0; k < NS; ++k)
    if (k == i) r = v[k];
  return r;
}
template <int NS, typename T> __device__ inline void addto(T (&v)[NS > 0 ? NS : 1], int i, T x) {
#pragma unroll
  for (int k = 0; k < NS; ++k)
    if (k == i) v[k] += x;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Carnahan-Starling pressure (Eq. 12), same operation order as the text.
template <typename T> __device__ inline T p_cs(const KConst& c, T rho) {
  const T e = T(0.25) * T(c.b) * rho;
  const T om = T(1) - e;
  const T num = T(1) + e + e * e - e * e * e;
  return rho * T(c.RT) * num / (om * om * om) - T(c.a) * rho * rho;
}

// ---------------------------------------------------------------- step kernel
template <typename T, int NS, int TY, bool EXPORT>
__global__ __launch_bounds__(64 * (TY + 2)) void k_step(const KArgs A) {
  constexpr int BY = TY + 2;
  constexpr int NSA = NS > 0 ? NS : 1;
  const KConst& c = A.c;
  __shared__ uint8_t s_t[TY + 4][68];
  __shared__ T s_r1[BY][64], s_r2[BY][64], s_ps[BY][64], s_q1[BY][64], s_q2[BY][64];
  __shared__ T s_C[NSA][BY][64];
  __shared__ double s_red[BY][4 + 2 * NSA];
  __shared__ double s_rare[NRARE_SLOTS];
  __shared__ double s_rmax[BY];

  // XCD-aware tile order: consecutive workgroups are dealt round-robin to the
  // 8 XCDs; give each XCD a contiguous band of tiles so that the halo rows two
  // neighbouring tiles share sit in the same L2.
  const int nb = c.nblocks;
  const int bid = blockIdx.x;
  const int xcd = bid & 7, loc = bid >> 3;
  const int tile = xcd * (nb >> 3) + min(xcd, nb & 7) + loc;
  const int tyi = tile / c.tiles_x, txi = tile - tyi * c.tiles_x;
  const int x0 = txi * TW, y0 = tyi * TY;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int nx = c.nx, ny = c.ny, pitch = c.pitch;
  const long long plane = c.plane;

  if (!EXPORT && ty == 0 && tx < NRARE_SLOTS) s_rare[tx] = 0.0;
  for (int k = ty * 64 + tx; k < (TY + 4) * 68; k += 64 * BY) {
    const int j = k / 68, i = k - j * 68;
    int X = x0 - 2 + i, Y = y0 - 2 + j;
    uint8_t v = TB_WALL;
    if (wrap(X, nx, c.per_x) && wrap(Y, ny, c.per_y)) v = A.t_in[(long long)Y * pitch + X];
    s_t[j][i] = v;
  }

  // ------------------------------------------------------------ phase 1
  const int X = x0 - 1 + tx, Y = y0 - 1 + ty;
  const bool own = tx >= 1 && tx <= TW && ty >= 1 && ty <= TY && X < nx && Y < ny;
  int Xw = X, Yw = Y;
  const bool indom = wrap(Xw, nx, c.per_x) && wrap(Yw, ny, c.per_y);
  const long long idx = (long long)Yw * pitch + Xw;
  const uint8_t tb = indom ? A.t_in[idx] : TB_WALL;
  const int t = tb & TB_T;
  const bool fluid = indom && t == T_FLUID;
  const bool validf = indom && (t == T_FLUID || (tb & TB_STR));
  const bool liq = indom && (tb & TB_LIQ);
  const bool liqp = indom && (tb & TB_LIQP);

  const T* fi = static_cast<const T*>(A.f_in);
  const T* gi = static_cast<const T*>(A.g_in);
  T f[2][9];
  T g[NSA][5];
  T rho[2] = {T(0), T(0)}, jx[2] = {T(0), T(0)}, jy[2] = {T(0), T(0)};
  T Ck[NSA];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int a = 0; a < 9; ++a) f[s][a] = validf ? fi[(s * 9 + a) * plane + idx] : T(0);
  }
  if (validf) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        rho[s] += f[s][a];
        jx[s] += f[s][a] * T(ex(a));
        jy[s] += f[s][a] * T(ey(a));
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    T cs = T(0);
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      g[k][a] = liqp ? gi[(k * 5 + a) * plane + idx] : T(0);
      cs += g[k][a];
    }
    Ck[k] = liqp ? cs : T(0);
  }
  T ps = T(0), q1 = T(0), q2 = T(0);
  unsigned errf = 0;
  if (validf) {
    if (!(rho[0] >= T(0)) || !(rho[1] >= T(0)) || (fluid && !(rho[0] + rho[1] > T(0)))) errf |= ERR_DENSITY;
  }
  bool clamped = false;
  if (fluid) {
    if (c.has_psi) {
      if (!(T(0.25) * T(c.b) * rho[0] < T(1))) errf |= ERR_EOS;
      T arg = T(c.psi_pre) * (p_cs<T>(c, rho[0]) - rho[0] / T(3)) / T(c.G11);
      if (arg < T(0)) {
        arg = T(0);
        clamped = true;
      }
      ps = dsqrt<T>(arg);
    }
    if (c.has_phi1) q1 = T(1) - dexp<T>(-rho[1] / T(c.rho20));
    if (c.has_phi2) q2 = T(c.a0) - dexp<T>(-rho[0] / T(c.rho10));
  }
  s_r1[ty][tx] = rho[0];
  s_r2[ty][tx] = rho[1];
  s_ps[ty][tx] = ps;
  s_q1[ty][tx] = q1;
  s_q2[ty][tx] = q2;
#pragma unroll
  for (int k = 0; k < NS; ++k) s_C[k][ty][tx] = Ck[k];
  if (own && errf && !EXPORT) {
    atomicOr(&A.err[0], errf);
    atomicMin(&A.err[1], (unsigned)(Yw * nx + Xw));
  }
  __syncthreads();

  // ------------------------------------------------------------ phase 2
  auto TT = [&](int dx, int dy) -> uint8_t { return s_t[ty + 1 + dy][tx + 1 + dx]; };
  auto nb_idx = [&](int a) -> long long {
    int Xn = Xw + ex(a), Yn = Yw + ey(a);
    if (Xn < 0) Xn += nx; else if (Xn >= nx) Xn -= nx;
    if (Yn < 0) Yn += ny; else if (Yn >= ny) Yn -= ny;
    return (long long)Yn * pitch + Xn;
  };
  auto is_fluid = [](uint8_t v) { return (v & (TB_WALL | TB_T)) == 0; };
  auto is_rsolid = [](uint8_t v) { return !(v & TB_WALL) && (v & TB_T) >= T_D; };

  // per-thread balance contributions (common ones in registers, rare ones via LDS)
  T l_msrc[2] = {T(0), T(0)};
  T l_ssrc[NSA], l_shet[NSA];
#pragma unroll
  for (int k = 0; k < NSA; ++k) l_ssrc[k] = l_shet[k] = T(0);
  double l_vdv = 0.0;
  double my_rmax = 0.0;
  bool precip = false;
  const double thr = c.lfrac * __longlong_as_double((long long)A.rmax[A.slot_prev]);

  if (own && fluid) {
    my_rmax = (double)rho[0];
    // forces: Eq. 11 (cohesion), 14 (inter-component), 16 (adhesion), body force.
    // Non-fluid neighbours carry the centre's own psi / phi and s = 1.
    T c1x = 0, c1y = 0, c12x = 0, c12y = 0, c21x = 0, c21y = 0, swx = 0, swy = 0;
#pragma unroll
    for (int a = 1; a < 9; ++a) {
      const uint8_t nt = TT(ex(a), ey(a));
      const bool fl = is_fluid(nt);
      const int ly = ty + ey(a), lx = tx + ex(a);
      const T psn = fl ? s_ps[ly][lx] : ps;
      const T q2n = fl ? s_q2[ly][lx] : q2;
      const T q1n = fl ? s_q1[ly][lx] : q1;
      const T sw = fl ? T(0) : T(1);
      c1x += T(wf(a)) * psn * T(ex(a));
      c1y += T(wf(a)) * psn * T(ey(a));
      c12x += T(wf(a)) * q2n * T(ex(a));
      c12y += T(wf(a)) * q2n * T(ey(a));
      c21x += T(wf(a)) * q1n * T(ex(a));
      c21y += T(wf(a)) * q1n * T(ey(a));
      swx += T(wf(a)) * sw * T(ex(a));
      swy += T(wf(a)) * sw * T(ey(a));
    }
    const T r1 = rho[0], r2 = rho[1];
    T Fx[2], Fy[2];
    Fx[0] = -T(c.G11) * ps * c1x - T(c.G12) * q1 * c12x - T(c.w1) * ps * swx + r1 * T(c.gx);
    Fy[0] = -T(c.G11) * ps * c1y - T(c.G12) * q1 * c12y - T(c.w1) * ps * swy + r1 * T(c.gy);
    Fx[1] = -T(c.G21) * q2 * c21x - T(c.w2) * r2 * swx + r2 * T(c.gx);
    Fy[1] = -T(c.G21) * q2 * c21y - T(c.w2) * r2 * swy + r2 * T(c.gy);
    // velocities: Eq. 18 (common), 17 (shifted equilibrium), 19 (physical)
    const T t1 = T(c.tau[0]), t2 = T(c.tau[1]);
    const T den = r1 / t1 + r2 / t2;
    const T upx = (jx[0] / t1 + jx[1] / t2) / den;
    const T upy = (jy[0] / t1 + jy[1] / t2) / den;
    T ux[2], uy[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T r = rho[s], ts = T(c.tau[s]);
      ux[s] = upx;
      uy[s] = upy;
      if (r > T(1e-12)) {
        ux[s] = upx + ts * Fx[s] / r;
        uy[s] = upy + ts * Fy[s] / r;
      }
    }
    const T rt = r1 + r2;
    const T urx = (jx[0] + jx[1] + T(0.5) * (Fx[0] + Fx[1])) / rt;
    const T ury = (jy[0] + jy[1] + T(0.5) * (Fy[0] + Fy[1])) / rt;

    if (EXPORT) {
      A.o_ux[idx] = (double)urx;
      A.o_uy[idx] = (double)ury;
    } else {
      // homogeneous reactions at liquid nodes (Eq. 5a, 5c, 27, 28)
      T Sk[NSA];
#pragma unroll
      for (int k = 0; k < NSA; ++k) Sk[k] = T(0);
      T Ss[2] = {T(0), T(0)};
      if (liq) {
        for (int r = 0; r < c.nhom; ++r) {
          const int re0 = c.hre0[r], re1 = c.hre1[r], pr0 = c.hpr0[r], pr1 = c.hpr1[r];
          T R;
          if (c.hkind[r] == HOM_FIRST) {
            R = T(c.hk[r]) * sel<NS>(Ck, re0);
          } else if (c.hkind[r] == HOM_BI) {
            R = T(c.hk[r]) * sel<NS>(Ck, re0) * sel<NS>(Ck, re1);
          } else {
            T cg = r2 / T(c.hMgas[r]);
            if (cg < T(0)) cg = T(0);
            R = T(c.hk[r]) * (sel<NS>(Ck, re0) - sel<NS>(Ck, pr0) * dsqrt<T>(cg) / T(c.hKeq[r]));
            Ss[0] -= T(0.5) * R * T(c.hMgas[r]);
            Ss[1] += T(0.5) * R * T(c.hMgas[r]);
          }
          addto<NS>(Sk, re0, -R);
          if (re1 >= 0) addto<NS>(Sk, re1, -R);
          if (pr0 >= 0) addto<NS>(Sk, pr0, R);
          if (pr1 >= 0) addto<NS>(Sk, pr1, R);
        }
        l_msrc[0] = Ss[0];
        l_msrc[1] = Ss[1];
#pragma unroll
        for (int k = 0; k < NS; ++k) l_ssrc[k] = Sk[k];
      }
      // flow collision (Eq. 6, 8)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const T om = T(c.om[s]);
        const T usq = ux[s] * ux[s] + uy[s] * uy[s];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
          const T eu = T(ex(a)) * ux[s] + T(ey(a)) * uy[s];
          const T feq = T(w9(a)) * rho[s] * (T(1) + T(3) * eu + T(4.5) * eu * eu - T(1.5) * usq);
          f[s][a] = f[s][a] - om * (f[s][a] - feq) + T(w9(a)) * Ss[s];
        }
      }
      // (a) populations stranded in a node that became SOLID_F last step go,
      // at rest, equally to that node's fluid D2Q9 neighbours
      T don[2] = {T(0), T(0)};
#pragma unroll
      for (int a = 1; a < 9; ++a) {
        const uint8_t nt = TT(ex(a), ey(a));
        if (!(nt & TB_WALL) && (nt & TB_STR)) {
          int m = 0;
#pragma unroll
          for (int b = 1; b < 9; ++b) m += is_fluid(TT(ex(a) + ex(b), ey(a) + ey(b))) ? 1 : 0;
          don[0] += s_r1[ty + ey(a)][tx + ex(a)] / T(m);
          don[1] += s_r2[ty + ey(a)][tx + ex(a)] / T(m);
        }
      }
#pragma unroll
      for (int s = 0; s < 2; ++s)
        if (don[s] != T(0)) {
#pragma unroll
          for (int a = 0; a < 9; ++a) f[s][a] += T(w9(a)) * don[s];
        }
      // flow push-streaming with halfway bounce-back
      T* fo = static_cast<T*>(A.f_out);
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        const bool tf = a == 0 ? true : is_fluid(TT(ex(a), ey(a)));
        const long long dst = tf ? (a * plane + (a == 0 ? idx : nb_idx(a))) : (opp(a) * plane + idx);
        fo[dst] = f[0][a];
        fo[9 * plane + dst] = f[1][a];
      }

      if (NS > 0 && liq) {
        // solute collision (Eq. 20-22) with the physical velocity u_r
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const T om = T(c.omg[k]);
#pragma unroll
          for (int a = 0; a < 5; ++a) {
            const T J = T(c.J[k][a]);
            const T geq = Ck[k] * (J + T(0.5) * (T(ex(a)) * urx + T(ey(a)) * ury));
            g[k][a] = g[k][a] - om * (g[k][a] - geq) + J * Sk[k];
          }
        }
        // (b) solute of a node that left the liquid set goes, at rest, equally
        // to its liquid D2Q5 neighbours
        T donk[NSA];
#pragma unroll
        for (int k = 0; k < NSA; ++k) donk[k] = T(0);
        bool any = false;
#pragma unroll
        for (int a = 1; a < 5; ++a) {
          const uint8_t nt = TT(ex(a), ey(a));
          if (!(nt & TB_WALL) && (nt & TB_LIQP) && !(nt & TB_LIQ)) {
            int m = 0;
#pragma unroll
            for (int b = 1; b < 5; ++b) {
              const uint8_t q = TT(ex(a) + ex(b), ey(a) + ey(b));
              m += (!(q & TB_WALL) && (q & TB_LIQ)) ? 1 : 0;
            }
#pragma unroll
            for (int k = 0; k < NS; ++k) donk[k] += s_C[k][ty + ey(a)][tx + ex(a)] / T(m);
            any = true;
          }
        }
        if (any) {
#pragma unroll
          for (int k = 0; k < NS; ++k)
#pragma unroll
            for (int a = 0; a < 5; ++a) g[k][a] += T(c.J[k][a]) * donk[k];
        }
        // heterogeneous link fluxes (Eq. 29-31, A2) and the precipitate the
        // node collects from GROWS reactions (Eq. 35)
        T phi[LBRX_MAX_RXN];
        for (int r = 0; r < c.nhet; ++r) {
          T v = T(c.xkap[r]) * (sel<NS>(Ck, c.xre[r]) - T(c.xCeq[r]));
          if (c.xirrev[r] && v < T(0)) v = T(0);
          phi[r] = v;
        }
        T* go = static_cast<T*>(A.g_out);
        double dv = 0.0;
        bool touched = false;
#pragma unroll
        for (int a = 0; a < 5; ++a) {
          const uint8_t nt = a == 0 ? tb : TT(ex(a), ey(a));
          const bool tl = a == 0 ? true : (!(nt & TB_WALL) && (nt & TB_LIQ));
          if (tl) {
            const long long dst = a * plane + (a == 0 ? idx : nb_idx(a));
#pragma unroll
            for (int k = 0; k < NS; ++k) go[k * 5 * plane + dst] = g[k][a];
          } else {
            const bool rs = is_rsolid(nt);
            const int tj = nt & TB_T;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
              T v = g[k][a];
              if (rs) {
                for (int r = 0; r < c.nhet; ++r) {
                  if (!(c.xsurf[r] & (1 << tj))) continue;
                  if (c.xre[r] == k) {
                    v -= phi[r];
                    l_shet[k] -= phi[r];
                  }
                  if (c.xpr[r] == k) {
                    v += phi[r];
                    l_shet[k] += phi[r];
                  }
                }
              }
              go[k * 5 * plane + opp(a) * plane + idx] = v;
            }
            if (rs && a > 0) {
              for (int r = 0; r < c.nhet; ++r)
                if ((c.xsurf[r] & (1 << tj)) && c.xmode[r] == HET_GROWS) {
                  dv += c.xmvol[r] * (double)phi[r];
                  touched = true;
                }
            }
          }
        }
        if (touched) {
          const double Vn = A.V[idx] + dv;
          A.V[idx] = Vn;
          l_vdv += dv;
          precip = Vn >= 1.0;  // the precipitate fills the node: SOLID_F next step
        }
      }
    }
  }

  // ---------------------------------------------------------- node status
  if (!EXPORT && own) {
    uint8_t tnew = (uint8_t)t;
    bool lnew = false;
    if (t == T_FLUID) {
      if (precip) tnew = T_F;
      else lnew = (double)rho[0] > thr;
    } else if (t == T_D || t == T_F) {
      // volume of pixel at a reactive solid node (Eq. 33; A2): sum of the
      // fluxes on its D2Q5 links to liquid nodes, in direction then reaction order
      double dv = 0.0;
      bool touched = false;
      if (NS > 0) {
#pragma unroll
        for (int a = 1; a < 5; ++a) {
          const uint8_t nt = TT(ex(a), ey(a));
          if ((nt & TB_WALL) || !(nt & TB_LIQ)) continue;
          for (int r = 0; r < c.nhet; ++r) {
            if (!(c.xsurf[r] & (1 << t))) continue;
            const int md = c.xmode[r];
            if (md != HET_CONSUMES && md != HET_MINERAL) continue;
            T cn = T(0);
#pragma unroll
            for (int k = 0; k < NS; ++k)
              if (k == c.xre[r]) cn = s_C[k][ty + ey(a)][tx + ex(a)];
            T v = T(c.xkap[r]) * (cn - T(c.xCeq[r]));
            if (c.xirrev[r] && v < T(0)) v = T(0);
            if (md == HET_CONSUMES) dv -= c.xmvol[r] * (double)v;
            else dv += c.xmvol[r] * (double)v;
            touched = true;
          }
        }
      }
      double Vn = A.V[idx];
      if (touched) {
        Vn += dv;
        A.V[idx] = Vn;
        l_vdv += dv;
      }
      if (Vn <= 0.0) {
        int nf = 0;
        T sum0 = T(0), sum1 = T(0);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
          const uint8_t nt = TT(ex(a), ey(a));
          if (!is_fluid(nt)) continue;
          sum0 += s_r1[ty + ey(a)][tx + ex(a)];
          sum1 += s_r2[ty + ey(a)][tx + ex(a)];
          ++nf;
        }
        if (nf > 0) {
          // (c) dissolved: fluid from the next step, at rest with the mean
          // density of its fluid neighbours; no solute yet
          const T rb0 = sum0 / T(nf), rb1 = sum1 / T(nf);
          T* fo = static_cast<T*>(A.f_out);
#pragma unroll
          for (int a = 0; a < 9; ++a) {
            fo[a * plane + idx] = T(w9(a)) * rb0;
            fo[(9 + a) * plane + idx] = T(w9(a)) * rb1;
          }
          atomicAdd(&s_rare[0], (double)rb0);
          atomicAdd(&s_rare[1], (double)rb1);
          atomicAdd(&s_rare[4], Vn);
          atomicAdd(&s_rare[6], 1.0);
          A.V[idx] = 0.0;
          tnew = T_FLUID;
          lnew = (double)rb0 > thr;
        }
      }
      if (tb & TB_STR) {
        int m = 0;
#pragma unroll
        for (int b = 1; b < 9; ++b) m += is_fluid(TT(ex(b), ey(b))) ? 1 : 0;
        if (m == 0) {
          atomicAdd(&s_rare[2], (double)rho[0]);
          atomicAdd(&s_rare[3], (double)rho[1]);
        }
      }
    }
    if (clamped) atomicAdd(&s_rare[5], 1.0);
    // a node leaving the liquid set with no liquid neighbour to take its solute
    if (liqp && !liq) {
      int m = 0;
#pragma unroll
      for (int b = 1; b < 5; ++b) {
        const uint8_t q = TT(ex(b), ey(b));
        m += (!(q & TB_WALL) && (q & TB_LIQ)) ? 1 : 0;
      }
      if (m == 0) {
#pragma unroll
        for (int k = 0; k < NS; ++k) atomicAdd(&s_rare[8 + k], (double)Ck[k]);
      }
      if (t == T_FLUID) atomicAdd(&s_rare[16], 1.0);
    }
    if (liq && !liqp) atomicAdd(&s_rare[17], 1.0);
    const bool to_f = (t == T_FLUID && tnew == T_F);
    if (to_f) atomicAdd(&s_rare[7], 1.0);
    uint8_t nbyte = (uint8_t)(tnew | (lnew ? TB_LIQ : 0) | (liq ? TB_LIQP : 0) | (to_f ? TB_STR : 0));
    A.t_out[idx] = nbyte;
  }

  if (EXPORT) {
    if (own) {
      A.o_r1[idx] = (double)rho[0];
      A.o_r2[idx] = (double)rho[1];
      if (!fluid) {
        A.o_ux[idx] = 0.0;
        A.o_uy[idx] = 0.0;
      }
#pragma unroll
      for (int k = 0; k < NS; ++k) A.o_C[k * plane + idx] = (double)Ck[k];
    }
    return;
  }

  // ---------------------------------------------------------- reductions
  // step maximum of rho_1 over fluid nodes
  {
    const double wm = wave_max(my_rmax);
    if (tx == 0) s_rmax[ty] = wm;
  }
  // common balances: per-wave sums in registers, then per tile in fixed order
  {
    double v;
    v = wave_sum((double)l_msrc[0]);
    if (tx == 0) s_red[ty][0] = v;
    v = wave_sum((double)l_msrc[1]);
    if (tx == 0) s_red[ty][1] = v;
    v = wave_sum(l_vdv);
    if (tx == 0) s_red[ty][2] = v;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      v = wave_sum((double)l_ssrc[k]);
      if (tx == 0) s_red[ty][4 + k] = v;
      v = wave_sum((double)l_shet[k]);
      if (tx == 0) s_red[ty][4 + NSA + k] = v;
    }
  }
  __syncthreads();
  if (ty == 0) {
    double* L = A.led + (long long)tile * NLED;
    if (tx == 0) {
      double m = 0.0;
      for (int w = 0; w < BY; ++w) m = fmax(m, s_rmax[w]);
      if (m > 0.0) atomicMax(&A.rmax[A.slot_cur], (unsigned long long)__double_as_longlong(m));
      if (bid == 0) A.rmax[A.slot_next] = 0ull;
    }
    // lane -> ledger slot
    int src = -1, dst = -1;
    if (tx < 2) { src = tx; dst = L_MSRC + tx; }
    else if (tx == 2) { src = 2; dst = L_VDV; }
    else if (tx >= 3 && tx < 3 + NS) { src = 4 + (tx - 3); dst = L_SSRC + (tx - 3); }
    else if (tx >= 3 + NS && tx < 3 + 2 * NS) { src = 4 + NSA + (tx - 3 - NS); dst = L_SHET + (tx - 3 - NS); }
    if (src >= 0) {
      double s = 0.0;
      for (int w = 0; w < BY; ++w) s += s_red[w][src];
      if (s != 0.0) L[dst] += s;
    }
    // rare balances accumulated in LDS
    if (tx >= 32 && tx < 32 + NRARE_SLOTS) {
      const int i = tx - 32;
      const double s = s_rare[i];
      if (s != 0.0) L[rare_dst(i)] += s;
    }
  }
}


// ---------------------------------------------------------------- ledger sum
// Fixed-order sum of the per-tile balance records (one block, one field per thread).
__global__ void k_ledger_sum(const double* led, int nblocks, double* out) {
  const int f = threadIdx.x;
  if (f >= NLED) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += led[(long long)b * NLED + f];
  out[f] = s;
}

// ---------------------------------------------------------------- host side
constexpr int TY64 = 6;   // FP64 tile height: 64 x 8 threads
constexpr int TY32 = 14;  // FP32 tile height: 64 x 16 threads

using KFn = void (*)(const KArgs);

template <typename T, int TY, bool EXPORT>
KFn pick(int ns) {
  switch (ns) {
    case 0: return k_step<T, 0, TY, EXPORT>;
    case 1: return k_step<T, 1, TY, EXPORT>;
    case 2: return k_step<T, 2, TY, EXPORT>;
    case 3: return k_step<T, 3, TY, EXPORT>;
    case 4: return k_step<T, 4, TY, EXPORT>;
    case 5: return k_step<T, 5, TY, EXPORT>;
    case 6: return k_step<T, 6, TY, EXPORT>;
    case 7: return k_step<T, 7, TY, EXPORT>;
    default: return k_step<T, 8, TY, EXPORT>;
  }
}

thread_local std::string g_create_err;

}  // namespace

struct lbrx_ctx {
  KConst c{};
  int precision = LBRX_F64;
  int ty = TY64;
  size_t esz = 8;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  void* f[2] = {nullptr, nullptr};
  void* g[2] = {nullptr, nullptr};
  uint8_t* t[2] = {nullptr, nullptr};
  double* V = nullptr;
  unsigned long long* rmax = nullptr;
  double* led = nullptr;
  double* ledsum = nullptr;
  unsigned int* err = nullptr;
  double* out = nullptr;  // export scratch: (4 + ns) planes
  int cur = 0;
  int64_t steps = 0;
  bool failed = false;
  std::string msg;
  KFn step_fn = nullptr, export_fn = nullptr;
};

namespace {

lbrx_status set_err(lbrx_ctx* c, lbrx_status s, const std::string& m) {
  if (c) {
    c->msg = m;
    if (s == LBRX_E_UNSTABLE || s == LBRX_E_DEVICE) c->failed = true;
  }
  return s;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return set_err(ctx, LBRX_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

std::string validate(const lbrx_params* p) {
  if (!p) return "params is NULL";
  if (p->abi_version != LBRX_ABI_VERSION) return "abi_version mismatch";
  if (p->nx < 1 || p->ny < 1) return "nx and ny must be >= 1";
  if ((long long)p->nx * p->ny > (1ll << 31) - 1) return "lattice too large";
  if (p->precision != LBRX_F64 && p->precision != LBRX_F32) return "unknown precision";
  for (int s = 0; s < 2; ++s)
    if (!(p->tau[s] > 0.5)) return "tau must exceed 1/2";
  if (p->n_species < 0 || p->n_species > LBRX_MAX_SPECIES) return "n_species out of range";
  const int ns = p->n_species;
  for (int k = 0; k < ns; ++k) {
    if (!(p->tau_g[k] > 0.5)) return "tau_g must exceed 1/2";
    if (!(p->J0[k] >= 0.0 && p->J0[k] < 1.0)) return "J0 must lie in [0,1)";
  }
  if (!(p->liquid_frac >= 0.0 && p->liquid_frac < 1.0)) return "liquid_frac must lie in [0,1)";
  if (p->n_hom < 0 || p->n_hom > LBRX_MAX_RXN || p->n_het < 0 || p->n_het > LBRX_MAX_RXN)
    return "reaction count out of range";
  for (int r = 0; r < p->n_hom; ++r) {
    const lbrx_hom_rxn& h = p->hom[r];
    if (h.kind < 0 || h.kind > 2) return "unknown homogeneous reaction kind";
    for (int i = 0; i < 2; ++i)
      if (h.re[i] < -1 || h.re[i] >= ns || h.pr[i] < -1 || h.pr[i] >= ns) return "species index out of range";
    if (h.re[0] < 0) return "homogeneous reaction needs a first reactant";
    if (h.kind == LBRX_HOM_BIMOLECULAR && h.re[1] < 0) return "bimolecular reaction needs two reactants";
    if (h.kind == LBRX_HOM_R1_GAS && (h.pr[0] < 0 || !(h.M_gas > 0.0) || !(h.K_eq > 0.0)))
      return "R1 reaction needs an aqueous product, M_gas > 0 and K_eq > 0";
    if (!(h.k >= 0.0)) return "rate constants must be >= 0";
  }
  for (int r = 0; r < p->n_het; ++r) {
    const lbrx_het_rxn& h = p->het[r];
    if (h.reactant < 0 || h.reactant >= ns || h.product < -1 || h.product >= ns) return "species index out of range";
    if (h.mode < 0 || h.mode > 2) return "unknown heterogeneous mode";
    if (h.surface & ~((1u << LBRX_SOLID_D) | (1u << LBRX_SOLID_F))) return "surface may only name SOLID_D / SOLID_F";
    if (!(h.k >= 0.0)) return "rate constants must be >= 0";
  }
  if (!p->node_type || !p->rho1 || !p->rho2) return "node_type, rho1 and rho2 are required";
  if (ns > 0 && !p->C0) return "C0 is required when n_species > 0";
  const long long N = (long long)p->nx * p->ny;
  for (long long i = 0; i < N; ++i) {
    const uint8_t t = p->node_type[i];
    if (t > 3) return "node type out of range";
    if (t == LBRX_FLUID) {
      if (!(p->rho1[i] > 0.0) || !(p->rho2[i] >= 0.0)) return "fluid node needs rho1 > 0 and rho2 >= 0";
      if (p->V0 && !(p->V0[i] >= 0.0 && p->V0[i] < 1.0)) return "fluid node precipitate volume must lie in [0,1)";
    } else if (t != LBRX_SOLID_INERT && p->V0 && !(p->V0[i] > 0.0)) {
      return "reactive solid needs V > 0";
    }
  }
  return "";
}

template <typename T>
void fill_populations(const lbrx_params* p, const KConst& c, const std::vector<uint8_t>& tb,
                      std::vector<T>& f, std::vector<T>& g) {
  const int nx = p->nx, ny = p->ny, ns = p->n_species;
  const long long plane = c.plane;
  f.assign((size_t)18 * plane, T(0));
  g.assign((size_t)5 * ns * plane + 1, T(0));
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const long long i = (long long)y * nx + x, d = (long long)y * c.pitch + x;
      if ((tb[d] & TB_T) != T_FLUID) continue;
      for (int a = 0; a < 9; ++a) {
        f[a * plane + d] = T(w9(a) * p->rho1[i]);
        f[(9 + a) * plane + d] = T(w9(a) * p->rho2[i]);
      }
      if (tb[d] & TB_LIQ)
        for (int k = 0; k < ns; ++k)
          for (int a = 0; a < 5; ++a) g[((long long)k * 5 + a) * plane + d] = T(c.J[k][a] * p->C0[(long long)k * nx * ny + i]);
    }
}

lbrx_status launch_step(lbrx_ctx* x) {
  KArgs A{};
  A.c = x->c;
  const int nxt = 1 - x->cur;
  A.f_in = x->f[x->cur];
  A.f_out = x->f[nxt];
  A.g_in = x->g[x->cur];
  A.g_out = x->g[nxt];
  A.t_in = x->t[x->cur];
  A.t_out = x->t[nxt];
  A.V = x->V;
  A.rmax = x->rmax;
  const int s = (int)(x->steps % 3);
  A.slot_prev = (s + 2) % 3;
  A.slot_cur = s;
  A.slot_next = (s + 1) % 3;
  A.led = x->led;
  A.err = x->err;
  dim3 block(64, x->ty + 2);
  hipLaunchKernelGGL(x->step_fn, dim3(x->c.nblocks), block, 0, x->stream, A);
  HIPCHK(x, hipGetLastError());
  x->cur = nxt;
  x->steps += 1;
  return LBRX_OK;
}

}  // namespace

extern "C" {

const char* lbrx_status_string(lbrx_status s) {
  switch (s) {
    case LBRX_OK: return "LBRX_OK";
    case LBRX_E_INVAL: return "LBRX_E_INVAL";
    case LBRX_E_NOMEM: return "LBRX_E_NOMEM";
    case LBRX_E_DEVICE: return "LBRX_E_DEVICE";
    case LBRX_E_UNSTABLE: return "LBRX_E_UNSTABLE";
    case LBRX_E_STATE: return "LBRX_E_STATE";
  }
  return "unknown";
}

const char* lbrx_create_error(void) { return g_create_err.c_str(); }

lbrx_status lbrx_create(const lbrx_params* p, void* hip_stream, lbrx_ctx** out) {
  g_create_err.clear();
  if (!out) {
    g_create_err = "out is NULL";
    return LBRX_E_INVAL;
  }
  *out = nullptr;
  const std::string v = validate(p);
  if (!v.empty()) {
    g_create_err = v;
    return LBRX_E_INVAL;
  }
  lbrx_ctx* x = new lbrx_ctx();
  KConst& c = x->c;
  c.nx = p->nx;
  c.ny = p->ny;
  c.pitch = (p->nx + 63) / 64 * 64;
  c.per_x = (p->periodic & 1u) ? 1 : 0;
  c.per_y = (p->periodic & 2u) ? 1 : 0;
  c.plane = (long long)c.pitch * p->ny;
  c.ns = p->n_species;
  x->precision = p->precision;
  x->ty = p->precision == LBRX_F64 ? TY64 : TY32;
  x->esz = p->precision == LBRX_F64 ? 8 : 4;
  c.tiles_x = (p->nx + TW - 1) / TW;
  c.tiles_y = (p->ny + x->ty - 1) / x->ty;
  c.nblocks = c.tiles_x * c.tiles_y;
  for (int s = 0; s < 2; ++s) {
    c.tau[s] = p->tau[s];
    c.om[s] = 1.0 / p->tau[s];
  }
  c.RT = p->R * p->T;
  c.a = p->a;
  c.b = p->b;
  c.G11 = p->G11;
  c.psi_pre = 2.0;
  c.G12 = p->G12;
  c.G21 = p->G21;
  c.w1 = p->w_adh[0];
  c.w2 = p->w_adh[1];
  c.gx = p->gbody[0];
  c.gy = p->gbody[1];
  c.a0 = p->a0;
  c.rho10 = p->rho10;
  c.rho20 = p->rho20;
  c.lfrac = p->liquid_frac;
  c.has_psi = p->G11 != 0.0;
  c.has_phi1 = p->rho20 > 0.0;
  c.has_phi2 = p->rho10 > 0.0;
  double D[LBRX_MAX_SPECIES] = {0};
  for (int k = 0; k < c.ns; ++k) {
    c.omg[k] = 1.0 / p->tau_g[k];
    c.J[k][0] = p->J0[k];
    for (int a = 1; a < 5; ++a) c.J[k][a] = 0.25 * (1.0 - p->J0[k]);
    D[k] = 0.5 * (1.0 - p->J0[k]) * (p->tau_g[k] - 0.5);  // Eq. 24
  }
  c.nhom = p->n_hom;
  for (int r = 0; r < p->n_hom; ++r) {
    c.hkind[r] = p->hom[r].kind;
    c.hre0[r] = p->hom[r].re[0];
    c.hre1[r] = p->hom[r].re[1];
    c.hpr0[r] = p->hom[r].pr[0];
    c.hpr1[r] = p->hom[r].pr[1];
    c.hk[r] = p->hom[r].k;
    c.hKeq[r] = p->hom[r].K_eq;
    c.hMgas[r] = p->hom[r].M_gas;
  }
  c.nhet = p->n_het;
  for (int r = 0; r < p->n_het; ++r) {
    const lbrx_het_rxn& h = p->het[r];
    c.xre[r] = h.reactant;
    c.xpr[r] = h.product;
    c.xsurf[r] = (int)h.surface;
    c.xmode[r] = h.mode;
    c.xirrev[r] = h.irreversible ? 1 : 0;
    const double Dk = D[h.reactant];
    // link flux coefficient of the halfway-wall Robin condition
    c.xkap[r] = (2.0 * Dk + h.k) > 0.0 ? 2.0 * Dk * h.k / (2.0 * Dk + h.k) : 0.0;
    c.xCeq[r] = h.C_eq;
    c.xmvol[r] = h.molar_volume;
  }
  x->step_fn = p->precision == LBRX_F64 ? pick<double, TY64, false>(c.ns) : pick<float, TY32, false>(c.ns);
  x->export_fn = p->precision == LBRX_F64 ? pick<double, TY64, true>(c.ns) : pick<float, TY32, true>(c.ns);

  auto fail = [&](lbrx_status s, const std::string& m) {
    g_create_err = m;
    lbrx_destroy(x);
    return s;
  };
  if (hipGetDevice(&x->device) != hipSuccess) return fail(LBRX_E_DEVICE, "hipGetDevice failed");
  if (hip_stream) {
    x->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&x->stream, hipStreamNonBlocking) != hipSuccess)
      return fail(LBRX_E_DEVICE, "hipStreamCreate failed");
    x->own_stream = true;
  }
  const size_t plane = (size_t)c.plane;
  const size_t fbytes = 18 * plane * x->esz, gbytes = (5 * (size_t)c.ns * plane + 1) * x->esz;
  for (int i = 0; i < 2; ++i) {
    if (hipMalloc(&x->f[i], fbytes) != hipSuccess || hipMalloc(&x->g[i], gbytes) != hipSuccess ||
        hipMalloc((void**)&x->t[i], plane) != hipSuccess)
      return fail(LBRX_E_NOMEM, "device allocation of the populations failed");
  }
  if (hipMalloc((void**)&x->V, plane * 8) != hipSuccess || hipMalloc((void**)&x->rmax, 3 * 8) != hipSuccess ||
      hipMalloc((void**)&x->led, (size_t)c.nblocks * NLED * 8) != hipSuccess ||
      hipMalloc((void**)&x->ledsum, NLED * 8) != hipSuccess || hipMalloc((void**)&x->err, 2 * 4) != hipSuccess)
    return fail(LBRX_E_NOMEM, "device allocation of the state failed");

  // initial state (host staging, then one copy each)
  const int nx = p->nx, ny = p->ny;
  double rmax0 = 0.0;
  for (long long i = 0; i < (long long)nx * ny; ++i)
    if (p->node_type[i] == LBRX_FLUID && p->rho1[i] > rmax0) rmax0 = p->rho1[i];
  const double thr0 = p->liquid_frac * rmax0;
  std::vector<uint8_t> tb(plane, (uint8_t)T_INERT);
  std::vector<double> V(plane, 0.0);
  for (int y = 0; y < ny; ++y)
    for (int xx = 0; xx < nx; ++xx) {
      const long long i = (long long)y * nx + xx, d = (long long)y * c.pitch + xx;
      const uint8_t t = p->node_type[i];
      uint8_t b = t;
      if (t == LBRX_FLUID && p->rho1[i] > thr0) b |= TB_LIQ | TB_LIQP;
      tb[d] = b;
      V[d] = p->V0 ? p->V0[i] : ((t == LBRX_SOLID_D || t == LBRX_SOLID_F) ? 1.0 : 0.0);
    }
  hipError_t e = hipSuccess;
  if (p->precision == LBRX_F64) {
    std::vector<double> f, g;
    fill_populations<double>(p, c, tb, f, g);
    e = hipMemcpy(x->f[0], f.data(), fbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(x->g[0], g.data(), gbytes, hipMemcpyHostToDevice);
  } else {
    std::vector<float> f, g;
    fill_populations<float>(p, c, tb, f, g);
    e = hipMemcpy(x->f[0], f.data(), fbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(x->g[0], g.data(), gbytes, hipMemcpyHostToDevice);
  }
  // the second buffers start as copies so that never-written slots hold defined values
  if (e == hipSuccess) e = hipMemcpy(x->f[1], x->f[0], fbytes, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->g[1], x->g[0], gbytes, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->t[0], tb.data(), plane, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->t[1], tb.data(), plane, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->V, V.data(), plane * 8, hipMemcpyHostToDevice);
  unsigned long long rm[3] = {0ull, 0ull, 0ull};
  std::memcpy(&rm[2], &rmax0, 8);
  if (e == hipSuccess) e = hipMemcpy(x->rmax, rm, sizeof rm, hipMemcpyHostToDevice);
  unsigned int er[2] = {0u, 0xffffffffu};
  if (e == hipSuccess) e = hipMemcpy(x->err, er, sizeof er, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(x->led, 0, (size_t)c.nblocks * NLED * 8);
  if (e != hipSuccess) return fail(LBRX_E_DEVICE, std::string("initial copy failed: ") + hipGetErrorString(e));
  *out = x;
  return LBRX_OK;
}

lbrx_status lbrx_step(lbrx_ctx* x, int64_t n) {
  if (!x) return LBRX_E_INVAL;
  if (x->failed) return set_err(x, LBRX_E_STATE, "context failed earlier: " + x->msg);
  if (n < 0) return set_err(x, LBRX_E_INVAL, "n_steps must be >= 0");
  HIPCHK(x, hipSetDevice(x->device));
  for (int64_t i = 0; i < n; ++i) {
    const lbrx_status s = launch_step(x);
    if (s != LBRX_OK) return s;
  }
  return LBRX_OK;
}

lbrx_status lbrx_sync(lbrx_ctx* x) {
  if (!x) return LBRX_E_INVAL;
  if (x->failed) return set_err(x, LBRX_E_STATE, "context failed earlier: " + x->msg);
  HIPCHK(x, hipSetDevice(x->device));
  HIPCHK(x, hipStreamSynchronize(x->stream));
  unsigned int er[2];
  HIPCHK(x, hipMemcpy(er, x->err, sizeof er, hipMemcpyDeviceToHost));
  if (er[0]) {
    char buf[256];
    snprintf(buf, sizeof buf, "unstable: %s%s at node (%u,%u) within the first %lld steps",
             (er[0] & ERR_DENSITY) ? "negative or NaN density " : "",
             (er[0] & ERR_EOS) ? "b*rho/4 >= 1 " : "", er[1] % (unsigned)x->c.nx, er[1] / (unsigned)x->c.nx,
             (long long)x->steps);
    return set_err(x, LBRX_E_UNSTABLE, buf);
  }
  return LBRX_OK;
}

lbrx_status lbrx_fields(lbrx_ctx* x, lbrx_fields_out* o) {
  if (!x || !o) return LBRX_E_INVAL;
  const lbrx_status st = lbrx_sync(x);
  if (st != LBRX_OK) return st;
  const KConst& c = x->c;
  const size_t plane = (size_t)c.plane;
  if (!x->out) HIPCHK(x, hipMalloc((void**)&x->out, (4 + (size_t)c.ns) * plane * 8));
  HIPCHK(x, hipMemsetAsync(x->out, 0, (4 + (size_t)c.ns) * plane * 8, x->stream));
  KArgs A{};
  A.c = c;
  A.f_in = x->f[x->cur];
  A.g_in = x->g[x->cur];
  A.t_in = x->t[x->cur];
  A.V = x->V;
  A.rmax = x->rmax;
  const int s = (int)(x->steps % 3);
  A.slot_prev = (s + 2) % 3;
  A.slot_cur = s;
  A.slot_next = (s + 1) % 3;
  A.err = x->err;
  A.o_r1 = x->out;
  A.o_r2 = x->out + plane;
  A.o_ux = x->out + 2 * plane;
  A.o_uy = x->out + 3 * plane;
  A.o_C = x->out + 4 * plane;
  hipLaunchKernelGGL(x->export_fn, dim3(c.nblocks), dim3(64, x->ty + 2), 0, x->stream, A);
  HIPCHK(x, hipGetLastError());
  hipLaunchKernelGGL(k_ledger_sum, dim3(1), dim3(64), 0, x->stream, x->led, c.nblocks, x->ledsum);
  HIPCHK(x, hipGetLastError());
  HIPCHK(x, hipStreamSynchronize(x->stream));
  const size_t sp = (size_t)c.pitch * 8, dp = (size_t)c.nx * 8;
  auto get2d = [&](double* dst, const double* src) -> hipError_t {
    return hipMemcpy2D(dst, dp, src, sp, dp, c.ny, hipMemcpyDeviceToHost);
  };
  if (o->rho1) HIPCHK(x, get2d(o->rho1, x->out));
  if (o->rho2) HIPCHK(x, get2d(o->rho2, x->out + plane));
  if (o->ux) HIPCHK(x, get2d(o->ux, x->out + 2 * plane));
  if (o->uy) HIPCHK(x, get2d(o->uy, x->out + 3 * plane));
  if (o->C)
    for (int k = 0; k < c.ns; ++k) HIPCHK(x, get2d(o->C + (size_t)k * c.nx * c.ny, x->out + (4 + k) * plane));
  if (o->V) HIPCHK(x, get2d(o->V, x->V));
  if (o->type || o->liquid) {
    std::vector<uint8_t> tb((size_t)c.nx * c.ny);
    HIPCHK(x, hipMemcpy2D(tb.data(), c.nx, x->t[x->cur], c.pitch, c.nx, c.ny, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < tb.size(); ++i) {
      if (o->type) o->type[i] = tb[i] & TB_T;
      if (o->liquid) o->liquid[i] = (tb[i] & TB_LIQ) ? 1 : 0;
    }
  }
  if (o->ledger) {
    double l[NLED];
    HIPCHK(x, hipMemcpy(l, x->ledsum, sizeof l, hipMemcpyDeviceToHost));
    static_assert(sizeof(lbrx_ledger) == NLED * sizeof(double), "ledger layout");
    l[NLED - 1] = (double)x->steps;
    std::memcpy(o->ledger, l, sizeof l);
  }
  if (o->rho_max) {
    unsigned long long v;
    const int last = (int)((x->steps + 2) % 3);
    HIPCHK(x, hipMemcpy(&v, x->rmax + last, 8, hipMemcpyDeviceToHost));
    std::memcpy(o->rho_max, &v, 8);
  }
  return LBRX_OK;
}

int64_t lbrx_step_count(const lbrx_ctx* x) { return x ? x->steps : -1; }

void* lbrx_stream(const lbrx_ctx* x) { return x ? (void*)x->stream : nullptr; }

const char* lbrx_last_error(const lbrx_ctx* x) { return x ? x->msg.c_str() : "NULL context"; }

lbrx_status lbrx_destroy(lbrx_ctx* x) {
  if (!x) return LBRX_OK;
  (void)hipSetDevice(x->device);
  if (x->stream) (void)hipStreamSynchronize(x->stream);
  for (int i = 0; i < 2; ++i) {
    if (x->f[i]) (void)hipFree(x->f[i]);
    if (x->g[i]) (void)hipFree(x->g[i]);
    if (x->t[i]) (void)hipFree(x->t[i]);
  }
  if (x->V) (void)hipFree(x->V);
  if (x->rmax) (void)hipFree(x->rmax);
  if (x->led) (void)hipFree(x->led);
  if (x->ledsum) (void)hipFree(x->ledsum);
  if (x->err) (void)hipFree(x->err);
  if (x->out) (void)hipFree(x->out);
  if (x->own_stream && x->stream) (void)hipStreamDestroy(x->stream);
  delete x;
  return LBRX_OK;
}

}  // extern "C"

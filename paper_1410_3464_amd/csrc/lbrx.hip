// lbrx: one coupled reactive-transport lattice Boltzmann step per kernel launch
// on gfx950 (MI355X), behind the C ABI of include/lbrx.h.
//
// Method: arXiv:1410.3464, Sec. 3-4 (Eq. 6-35, A2), procedure of Sec. 4.7.
//
// Kernel structure (one launch per time step):
//   * State between steps: post-collision populations f*, g* of every node in
//     its own slots (row-interleaved structure of arrays: population q of row
//     y at (y * NP + q) * pitch + x), one 32-bit status word per node (type,
//     the solute it holds, and which neighbours were fluid / liquid when the
//     populations were written), the FP64 solid / precipitate volume.
//   * One wavefront owns a 62-column by H-row item (its 64 lanes also hold
//     the column on either side) and marches down it.  Per
//     row it pulls the next row's populations along the links (halfway
//     bounce-back where the status word names no fluid neighbour), forms the
//     moments (Eq. 9, 23) and effective masses psi_1, phi_1, phi_2 (Eq. 13,
//     15) into a three-row LDS ring, then for the current row forms the forces
//     (Eq. 11, 14, 16) from the ring, the velocities (Eq. 17-19), reaction
//     sources (Eq. 5, 27, 28), both collisions (Eq. 6, 20), the status-change
//     amendments (Sec. 4.5), the volume-of-pixel update (Eq. 33, 35) and the
//     reactive link flux (Eq. 29-31, A2), and stores the results in place.
//   * Nothing is read back in the same launch, so there is no grid-wide sync;
//     the liquid threshold uses the previous step's maximum (atomic max on the
//     bit pattern of a non-negative double), and balances accumulate into one
//     FP64 record per item (no floating-point atomics in global memory).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
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

// Node status word (32 bits): bits 0-1 type, bits 2-3 the solute the node
// holds (SF_*), bit 4 stranded (became SOLID_F at the end of the last step;
// its incoming populations are still to be pulled and given away), bits 8-15
// neighbour b = 1..8 was fluid last step, bits 16-19 D2Q5 neighbour b = 1..4 was
// liquid last step (set at liquid nodes only).  A node with none of bits 8-19
// set reads its own slots back; that is how the initial state, a node freed by
// dissolution (both at rest, whose populations are equal in opposite
// directions) and a node keeping solute at rest enter the pull.  Bit 7 marks
// "outside a non-periodic boundary" in the kernel only.
constexpr uint32_t TB_T = 0x3, TB_SF = 0xC, TB_STR = 0x10, TB_WALL = 0x80;
constexpr int NBF_SHIFT = 8, NBL_SHIFT = 16, SF_SHIFT = 2;
// Solute a node holds at the start of a step (Sec. 4.5 amendments):
//   SF_STREAM  liquid in the previous step: its slots get the populations
//              streamed into it
//   SF_HOLD    not liquid; keeps its content at rest in its own slots (it had
//              no liquid D2Q5 neighbour to give it to)
//   SF_SHARE   left the liquid set last step; its own slots hold, at rest, one
//              equal share of its content per D2Q5 neighbour that was liquid
//              then, which those neighbours take during this step
enum { SF_NONE = 0, SF_STREAM = 1, SF_HOLD = 2, SF_SHARE = 3 };
__host__ __device__ inline int sf_of(uint32_t w) { return (int)((w & TB_SF) >> SF_SHIFT); }

// FP32 and 16-bit population storage keep each flow population as a
// deviation from w_a times a reference density of the node that will pull it
// (FP32 divides the deviation by w_a; 16-bit storage also keeps solute as a
// deviation from J_a times a reference concentration).  A reference is coded in a few
// bits: the float's bit pattern above bit `sh` (exponent and top mantissa
// bits), counted from a base, and decoded to the middle of its bucket.  The
// codes are integer operations on both sides, so the writer of a population
// and its reader always agree on the reference.  The flow codes of a node
// (rho_1: 8 bits, rho_2: 7 bits) ride in bits 24-31 and 20-23, 5-7 of its
// status word; the solute codes (8 bits per species) in one 32-bit word per
// four species.
constexpr int SH1 = 19, SH2 = 20, SHC = 19;  // 16, 16 and 16 binades of range
constexpr uint32_t MAX1 = 255, MAX2 = 127, MAXC = 255;
__host__ __device__ inline uint32_t ref_code(float v, uint32_t base, int sh, uint32_t maxc) {
  const uint32_t b = __builtin_bit_cast(uint32_t, v);
  if (b == 0u || (b >> 31)) return 0u;  // zero or negative: the lowest reference
  const uint32_t q = b >> sh;
  if (q <= base) return 0u;
  return (q - base) < maxc ? (q - base) : maxc;
}
__host__ __device__ inline float ref_value(uint32_t code, uint32_t base, int sh) {
  return __builtin_bit_cast(float, ((code + base) << sh) | (1u << (sh - 1)));
}
__host__ __device__ inline uint32_t put_codes(uint32_t c1, uint32_t c2) {
  return (c1 << 24) | ((c2 & 15u) << 20) | ((c2 >> 4) << 5);
}
__host__ __device__ inline uint32_t code1_of(uint32_t w) { return w >> 24; }
__host__ __device__ inline uint32_t code2_of(uint32_t w) { return ((w >> 20) & 15u) | (((w >> 5) & 7u) << 4); }
constexpr int T_FLUID = 0, T_INERT = 1, T_D = 2, T_F = 3;


// ledger slots, same order as lbrx_ledger
constexpr int L_MSRC = 0, L_MINJ = 2, L_MREM = 4, L_SSRC = 6, L_SHET = 14, L_SREM = 22, L_VDV = 30,
              L_VCLIP = 31, L_CLAMP = 32, L_NDIS = 33, L_NPRE = 34, L_NL2G = 35, L_NG2L = 36;
constexpr int NLED = 38;  // + steps (host)
// LDS slots of the rarely non-zero balances (a wavefront's sums, added by
// lane 0 in row order): 0-1 mass_inj, 2-3 mass_rem, 4 vol_clip, 5 psi clamps,
// 6 dissolved, 7 precipitated, 8 liquid->gas, 9 gas->liquid.  Solute is never
// dropped, so sol_rem stays zero.
constexpr int NRARE_SLOTS = 10;
__host__ __device__ constexpr int rare_dst(int i) {
  return i == 0 ? L_MINJ : i == 1 ? L_MINJ + 1 : i == 2 ? L_MREM : i == 3 ? L_MREM + 1 : i == 4 ? L_VCLIP
       : i == 5 ? L_CLAMP : i == 6 ? L_NDIS : i == 7 ? L_NPRE : i == 8 ? L_NL2G : L_NG2L;
}

// rho_max slots: 3 rotating step slots x 8 partial maxima (one per XCD), each
// partial on its own 128-byte line so that workgroups on different XCDs never
// contend for one address
constexpr int RM_STRIDE = 16;  // u64 per partial
constexpr int RM_SLOT = 8 * RM_STRIDE;
constexpr int RM_WORDS = 3 * RM_SLOT;

enum { HOM_FIRST = 0, HOM_R1 = 1, HOM_BI = 2 };
enum { HET_CONSUMES = 0, HET_GROWS = 1, HET_MINERAL = 2 };

struct KConst {
  int nx, ny, pitch, per_x, per_y, strips, seg_rows, nitems, nblocks, ns;
  unsigned fbytes, gbytes, tbytes, cbytes;  // array sizes (buffer ranges)
  int ncw;                                  // solute code words per node (16-bit storage)
  int sg;                                   // species per solute slot (species_group)
  long long plane;
  double om[2], tau[2], RT, a, b, G11, rG11, psi_pre, G12, G21, w1, w2, gx, gy, a0, rho10, rho20, lfrac;
  int has_psi, has_phi1, has_phi2;
  double J[LBRX_MAX_SPECIES][5];
  double omg[LBRX_MAX_SPECIES];
  int nhom;
  int hkind[LBRX_MAX_RXN], hre0[LBRX_MAX_RXN], hre1[LBRX_MAX_RXN], hpr0[LBRX_MAX_RXN], hpr1[LBRX_MAX_RXN];
  double hk[LBRX_MAX_RXN], hKeq[LBRX_MAX_RXN], hMgas[LBRX_MAX_RXN];
  int hsurf[LBRX_MAX_RXN], any_hsurf;  // surface-enhanced rates: solid-type bits, any at all
  double hks[LBRX_MAX_RXN];            // rate constant times the surface factor
  int nhet;
  int xre[LBRX_MAX_RXN], xpr[LBRX_MAX_RXN], xsurf[LBRX_MAX_RXN], xmode[LBRX_MAX_RXN], xirrev[LBRX_MAX_RXN];
  double xkap[LBRX_MAX_RXN], xCeq[LBRX_MAX_RXN], xmvol[LBRX_MAX_RXN];
  // per reactive solid type (q = 0: SOLID_D, 1: SOLID_F) and reaction: the
  // precipitate volume per unit flux a liquid node collects on a link to it
  // (GROWS reactions on that surface, else 0), and the solid volume change per
  // unit flux on a link from a liquid node (-Vbar CONSUMES, +Vbar MINERAL, else 0)
  double xgv[2][LBRX_MAX_RXN], xsv[2][LBRX_MAX_RXN];
  int sub;        // the species taken by subtraction at liquid nodes (Sec. 4.1), -1: none
  double sub_tot; // total liquid concentration per unit rho_1
  int xgrow[2], xsolid[2];  // some reaction of that kind runs on that surface
};

// Per-precision copies of the real constants (and reciprocals, used by the FP32
// path in place of divisions by constants).
template <typename T> struct KT {
  T om[2], tau[2], r_tau[2], RT, a, b, G11, r_G11, psi_pre, G12, G21, w1, w2, gx, gy, a0, rho10, r_rho10,
      rho20, r_rho20;
  T J[LBRX_MAX_SPECIES][5];
  T omg[LBRX_MAX_SPECIES];
  T hk[LBRX_MAX_RXN], hks[LBRX_MAX_RXN], hKeq[LBRX_MAX_RXN], r_hKeq[LBRX_MAX_RXN], hMgas[LBRX_MAX_RXN],
      r_hMgas[LBRX_MAX_RXN];
  T xkap[LBRX_MAX_RXN], xCeq[LBRX_MAX_RXN];
  T hnu[LBRX_MAX_RXN][LBRX_MAX_SPECIES];  // net stoichiometric coefficient of species k in reaction r
  // link flux of a heterogeneous reaction: +1 for its product, -1 for its
  // reactant, per reactive solid type whose surface it runs on (else 0)
  T xnu[2][LBRX_MAX_RXN][LBRX_MAX_SPECIES];
  // FP32 solute weights of Eq. 22 as stored: J1' on a 2^-26 grid and
  // J0' = 1 - 4 J1', so that the weights sum to one exactly; 1 / (2 J1'), 1 / J1'
  T Jp0[LBRX_MAX_SPECIES], Jp1[LBRX_MAX_SPECIES], hJ[LBRX_MAX_SPECIES], iJ1[LBRX_MAX_SPECIES];
  T sub_tot;
  // 16-bit storage: deviation scales (powers of two) and reference-code bases
  T sc[2], isc[2], wsc[2][3];               // flow: scale, 1/scale, w (rest, axis, diagonal) x scale
  T scg[LBRX_MAX_SPECIES], iscg[LBRX_MAX_SPECIES], Jsc[LBRX_MAX_SPECIES][2];
  T wc[3], Jc[LBRX_MAX_SPECIES][2];         // the weights themselves
  uint32_t rb1, rb2, rbc[LBRX_MAX_SPECIES];
};

// Everything a launch needs about one simulation, kept in device memory for
// the simulation's lifetime: the buffer pair of each array (which one is read
// follows from the step count), constants, and state.
template <typename T> struct KArgs {
  KConst c;
  KT<T> k;
  void* f[2];
  void* g[2];
  uint32_t* t[2];
  uint32_t* cw[2];           // solute reference codes (16-bit storage)
  double* V;
  unsigned long long* rmax;  // 3 rotating slots
  double* led;               // [nitems][NLED]
  unsigned int* err;         // [0] flags, [1] first failing node (min index)
};

// constant address space: data no store of a running kernel can change
#define KAS __attribute__((address_space(4)))

// The kernel arguments of one launch: one simulation (ninst == 0), or a batch
// whose workgroups each look up their simulation, item block and step phase
// in a table.  The phase of a simulation is its step count modulo 6: bit 0
// picks the buffer that is read, the count modulo 3 the rho_max slot.
struct LaunchArgs {
  const void* single;       // KArgs of the simulation (ninst == 0)
  const void* const* inst;  // batch: KArgs of every simulation
  const uint32_t* table;    // batch: per workgroup, simulation << 20 | base phase << 17 | block
  int ninst;
  int phase0;  // single: step count mod 6
  int launch;  // batch: launches since the table was built, mod 6
  double* out;  // read-out launches: planes rho1, rho2, ux, uy, C_0.., liquid (pitch-strided)
};
constexpr int TAB_INST_SHIFT = 20, TAB_PHASE_SHIFT = 17;
constexpr uint32_t TAB_BLOCK_MASK = (1u << TAB_PHASE_SHIFT) - 1u;

enum { ERR_DENSITY = 1u, ERR_EOS = 2u };

// Coordinate X inside [0, n) (periodic) or "outside" (false).  The callers'
// coordinates lie at most 66 nodes outside, so a few additions or
// subtractions wrap them (one unless n is tiny); no integer division.
__device__ inline bool wrap(int& X, int n, int per) {
  if (X >= 0 && X < n) return true;
  if (!per) return false;
  while (X < 0) X += n;
  while (X >= n) X -= n;
  return true;
}

// Row Y with a free outlet beyond row n - 1 (a wall below row 0): the ghost
// rows beyond the outlet repeat row n - 1 (zero gradient of every variable,
// Sec. 5.1), so such a row becomes n - 1.
__device__ inline bool wrap_out(int& Y, int n) {
  if (Y < 0) return false;
  if (Y >= n) Y = n - 1;
  return true;
}

template <typename T> __device__ inline T dexp(T x);
template <> __device__ inline double dexp<double>(double x) { return exp(x); }
template <> __device__ inline float dexp<float>(float x) { return __expf(x); }
template <typename T> __device__ inline T dsqrt(T x);
template <> __device__ inline double dsqrt<double>(double x) { return sqrt(x); }
template <> __device__ inline float dsqrt<float>(float x) { return sqrtf(x); }

// a / b: IEEE division in FP64 (same rounding as the plain expression); in FP32
// the hardware reciprocal (1 ulp) times a.
template <typename T> __device__ inline T qdiv(T a, T b);
template <> __device__ inline double qdiv<double>(double a, double b) { return a / b; }
template <> __device__ inline float qdiv<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// a / c for a constant c with precomputed reciprocal rc
template <typename T> __device__ inline T cdiv(T a, T c, T rc);
template <> __device__ inline double cdiv<double>(double a, double c, double) { return a / c; }
template <> __device__ inline float cdiv<float>(float a, float, float rc) { return a * rc; }

// loads and stores at a uniform base plus a 32-bit byte offset
template <typename T> __device__ inline T ldb(const T* base, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T> __device__ inline void stb(T* base, unsigned off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off) = v;
}

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

// Wave (64-lane) reductions; a wave whose values are all zero skips the shuffles.
template <typename T> __device__ inline T wave_sum_t(T v) {
  if (__ballot(v != T(0)) == 0ull) return T(0);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T> __device__ inline T wave_max_t(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const T w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// Carnahan-Starling pressure (Eq. 12), same operation order as the text.
template <typename T, typename K> __device__ inline T p_cs(const K& k, T rho) {
  const T e = T(0.25) * k.b * rho;
  const T om = T(1) - e;
  const T num = T(1) + e + e * e - e * e * e;
  return qdiv<T>(rho * k.RT * num, om * om * om) - k.a * rho * rho;
}

// ---------------------------------------------------------------- step kernel
// One launch = one time step n.  Populations are stored after collision
// (f*(n-1), g*(n-1)) in the slots of the node that produced them; the kernel
// first pulls them along the lattice links (the streaming of step n-1, with
// halfway bounce-back against the previous step's masks, which each node keeps
// in its status word), then runs step n and writes f*(n), g*(n) back into the
// node's own slots.  Own-slot stores let every written 128-byte line be
// complete: every lane of a group that shares a line and holds a valid
// population stores (lanes without one store values that are never read).
//
// Work decomposition: one wavefront per item of IW = 62 columns by H rows.
// Its 64 lanes hold columns x0 - 1 .. x0 + 62: the item's own columns and one
// halo column on each side, which the horizontally adjacent items own.  The
// wavefront marches down its rows: at row R it pulls row R + 1 on every lane,
// stages that row's psi, phi, node flags, densities and concentrations in a
// three-row LDS ring, and collides row R on its own lanes against the ring.
// The halo lanes pull the same lines as the neighbouring item's edge lanes,
// at about the same time (adjacent items are dispatched one after the other),
// so those lines are read once from memory.  Wavefronts never wait for each
// other, so one wavefront's loads overlap another's arithmetic.
//
// Memory access is through raw buffer descriptors: a per-lane 32-bit offset
// (one per link direction, shared by both components and all species) plus a
// uniform offset for the population plane.
constexpr int SW = 64;       // lanes: one column each
constexpr int IW = SW - 2;   // columns an item owns (lanes 1 .. 62)
constexpr int HMAX = 30;     // most rows per item
// wavefronts per workgroup, each with its own item
#ifndef LBRX_WPB
#define LBRX_WPB 1
#endif
constexpr int WPB = LBRX_WPB;
// lower bound on resident wavefronts per SIMD asked of the FP32 register
// allocator (0: the compiler's choice)
#ifndef LBRX_F32_WAVES
#define LBRX_F32_WAVES 0
#endif
template <typename T> constexpr int min_waves() {
  return (std::is_same<T, float>::value && LBRX_F32_WAVES > 0) ? LBRX_F32_WAVES : 1;
}

// node flags as staged in LDS: status bits 0-4 of the word, plus
constexpr uint32_t LF_LIQN = 0x20;  // liquid at this step (in the domain)
constexpr uint32_t LF_FLU = 0x40;   // fluid at this step (in the domain)
// (TB_WALL = 0x80: outside a non-periodic side)

template <typename T> struct alignas(4 * sizeof(T)) PQ {
  T ps, q1, q2, fl;  // psi_1, phi_1, phi_2 (zero at non-fluid nodes), node flags (bit pattern)
};

template <typename T> __device__ inline T flags_as(uint32_t v) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, v);
  else return __builtin_bit_cast(T, (unsigned long long)v);
}
template <typename T> __device__ inline uint32_t flags_of(T v) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(uint32_t, v);
  else return (uint32_t)__builtin_bit_cast(unsigned long long, v);
}

// Population storage: the working precision itself, or 16-bit deviations
// (FP16 or BF16, with FP32 arithmetic) from the coded references above.
// SM_OUT: plain storage, kernels built with the free-outlet rows (a separate
// instantiation, so that the other kernels carry none of its code)
enum { SM_PLAIN = 0, SM_F16 = 1, SM_BF16 = 2, SM_OUT = 3 };
__host__ __device__ constexpr bool sm_dev(int sm) { return sm == SM_F16 || sm == SM_BF16; }
template <typename T, int SM> struct StoreT { using type = T; };
template <> struct StoreT<float, SM_F16> { using type = uint16_t; };
template <> struct StoreT<float, SM_BF16> { using type = uint16_t; };
template <int SM> __device__ inline float dev_in(uint16_t h) {
  if constexpr (SM == SM_F16) return (float)__builtin_bit_cast(_Float16, h);
  else return __builtin_bit_cast(float, (uint32_t)h << 16);
}
template <int SM> __device__ inline uint16_t dev_out(float v) {
  if constexpr (SM == SM_F16) return __builtin_bit_cast(uint16_t, (_Float16)v);
  else return __builtin_bit_cast(uint16_t, (__bf16)v);
}
// weight class of a direction: rest, axis, diagonal
__host__ __device__ constexpr int wcls(int a) { return a == 0 ? 0 : (a < 5 ? 1 : 2); }

template <typename T> struct alignas(2 * sizeof(T)) RF {
  T r1, r2;  // reference densities a population written to this node is coded against
};

// the change of a reactive solid's volume over one link from a liquid node
// (Eq. 33, A2), for a SOLID_D and a SOLID_F node at the other end
struct alignas(16) VS {
  double d, f;
};

template <typename T, int NS, int SM> struct WaveLds {
  static constexpr int NSA = NS > 0 ? NS : 1;
  // flow reference rows (FP32 and 16-bit storage), solute reference rows (16-bit storage)
  static constexpr bool REFS = sm_dev(SM) || std::is_same<T, float>::value;
  static constexpr int NRF = REFS ? 3 : 1;
  static constexpr int NCF = sm_dev(SM) ? 3 : 1;
  // ring rows (R - 1, R, R + 1 in rotation) x lanes; lane l at index l + 1
  // (indices 0 and SW + 1 are read only by the halo lanes, whose row-R
  // results are not used)
  PQ<T> pq[3][SW + 2];
  T r1[3][SW + 2], r2[3][SW + 2];
  T C[NSA][3][SW + 2];
  RF<T> rf[NRF][SW + 2];
  VS vs[3][SW + 2];
  T Cf[NSA][NCF][SW + 2];
  double rare[NRARE_SLOTS];
};

typedef unsigned int v2u_t __attribute__((ext_vector_type(2)));
__device__ inline __amdgpu_buffer_rsrc_t rsrc_of(const void* p, unsigned bytes) {
  // raw buffer: stride 0, a byte range, 32-bit data format in word 3
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T> __device__ inline T bload(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  if constexpr (sizeof(T) == 2) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0));
  else if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
  else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
}
// Stores are non-temporal (cache policy bit "nt"): nothing reads the written
// lines in the same launch, and keeping them out of the way leaves the L2 to
// the rows the pulls of neighbouring rows read again.
constexpr int STORE_NT = 2;
// A buffer offset past the end of every array (each stays below it, checked
// when a simulation is created).  Buffer accesses out of range read zero and
// drop stores, so a lane with nothing to load or store still issues every
// memory instruction with this offset: the wavefront's count of memory
// operations is then the same on every path, and the compiler's waits for a
// load do not also wait for loads and stores issued after it.
constexpr unsigned OOB_OFF = 0xFFFFFF00u;
__device__ inline unsigned gate(bool on, unsigned off) { return off | (on ? 0u : OOB_OFF); }
// sel ? a : b on offsets, as integer arithmetic (a conditional expression
// there can be compiled into a branch around each load)
__device__ inline unsigned pick_off(bool sel, unsigned a, unsigned b) { return b + ((a - b) & (0u - (unsigned)sel)); }
template <typename T> __device__ inline void bstore(T v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  if constexpr (sizeof(T) == 2) __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, (int)vo, (int)so, STORE_NT);
  else if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)vo, (int)so, STORE_NT);
  else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u_t, v), r, (int)vo, (int)so, STORE_NT);
}

// Slots hold pairs: both flow components of one direction, or two species of
// one direction, so that one load or store moves both (16-bit pairs make one
// 32-bit word per lane).
template <typename ST> struct Pair {
  ST lo, hi;
};
typedef unsigned int v4u_t __attribute__((ext_vector_type(4)));
template <typename ST> __device__ inline Pair<ST> bload2(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  if constexpr (sizeof(ST) == 2) {
    const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0);
    return Pair<ST>{(ST)(u & 0xffffu), (ST)(u >> 16)};
  } else {
    // The loaded vector is reinterpreted as a whole (two-element vector of
    // ST): taking its integer elements apart one by one let the compiler
    // shrink the load to the low dword.
    typedef ST v2s_t __attribute__((ext_vector_type(2)));
    v2s_t u;
    if constexpr (sizeof(ST) == 4) u = __builtin_bit_cast(v2s_t, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
    else u = __builtin_bit_cast(v2s_t, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0));
    return Pair<ST>{u.x, u.y};
  }
}
template <typename ST> __device__ inline void bstore2(ST lo, ST hi, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  if constexpr (sizeof(ST) == 2) {
    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)lo | ((uint32_t)hi << 16), r, (int)vo, (int)so, STORE_NT);
  } else if constexpr (sizeof(ST) == 4) {
    __builtin_amdgcn_raw_buffer_store_b64(v2u_t{__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi)}, r,
                                          (int)vo, (int)so, STORE_NT);
  } else {
    const v2u_t a = __builtin_bit_cast(v2u_t, lo), b = __builtin_bit_cast(v2u_t, hi);
    __builtin_amdgcn_raw_buffer_store_b128(v4u_t{a.x, a.y, b.x, b.y}, r, (int)vo, (int)so, STORE_NT);
  }
}

// Species per solute slot: the four species of a group share one slot of a
// direction (16 bytes in FP32, 8 in 16-bit storage) when the species count is
// a multiple of four, else pairs (FP64 always: 16 bytes).  A wider slot puts
// fewer nodes in a 128-byte line, so fewer lines are only partly used where
// liquid meets gas or solid, and one load or store moves the whole group.
__host__ __device__ constexpr int species_group(int ns, int esz) { return (ns > 0 && ns % 4 == 0 && esz <= 4) ? 4 : 2; }

template <typename ST, int SG> struct Grp {
  ST v[SG];
};
template <typename ST, int SG> __device__ inline Grp<ST, SG> bloadg(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  Grp<ST, SG> g;
  if constexpr (SG == 2) {
    const Pair<ST> q = bload2<ST>(r, vo, so);
    g.v[0] = q.lo;
    g.v[1] = q.hi;
  } else {
    // reinterpreted as a whole vector of ST, as for pairs
    typedef ST vs_t __attribute__((ext_vector_type(SG)));
    vs_t u;
    if constexpr (sizeof(ST) * SG == 8) u = __builtin_bit_cast(vs_t, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
    else u = __builtin_bit_cast(vs_t, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0));
#pragma unroll
    for (int i = 0; i < SG; ++i) g.v[i] = u[i];
  }
  return g;
}
template <typename ST, int SG> __device__ inline void bstoreg(const Grp<ST, SG>& g, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  if constexpr (SG == 2) {
    bstore2<ST>(g.v[0], g.v[1], r, vo, so);
  } else {
    typedef ST vs_t __attribute__((ext_vector_type(SG)));
    vs_t u;
#pragma unroll
    for (int i = 0; i < SG; ++i) u[i] = g.v[i];
    if constexpr (sizeof(ST) * SG == 8) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u_t, u), r, (int)vo, (int)so, STORE_NT);
    else __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u_t, u), r, (int)vo, (int)so, STORE_NT);
  }
}

template <typename T, int NS> struct Mom {
  T rho[2], jx[2], jy[2], C[NS > 0 ? NS : 1];
  T drho[2];  // FP32 storage: rho - the decoding reference (the mass the deviations carry)
};

// deterministic sum over the wavefront (a fixed butterfly; lane 0's result)
__device__ inline double wave_sum_det(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return __builtin_bit_cast(double, ((unsigned long long)__builtin_amdgcn_readfirstlane(
                                         (unsigned)(__builtin_bit_cast(unsigned long long, v) >> 32)) << 32) |
                                        (unsigned)__builtin_amdgcn_readfirstlane(
                                            (unsigned)__builtin_bit_cast(unsigned long long, v)));
}

template <typename T, int SM, int NS, bool EXPORT>
__global__ __launch_bounds__(64 * WPB, min_waves<T>()) void k_step(const LaunchArgs LA_arg) {
  // The launch arguments are read where the launch put them (the kernarg
  // segment): a reference to the by-value parameter itself would make the
  // compiler copy it to private memory first.
  (void)LA_arg;
  const LaunchArgs& LA = *(const LaunchArgs*)__builtin_amdgcn_kernarg_segment_ptr();

  // XCD-aware order: consecutive workgroups are dealt round-robin to the 8
  // XCDs; each XCD gets a contiguous band of items (of a batch's table), so
  // that horizontally adjacent items (whose halo lanes read each other's
  // edge columns) run at about the same time, and the rows two vertically
  // neighbouring items share sit in the same L2.
  const int nb = gridDim.x;
  const int bid = blockIdx.x;
  const int xcd = bid & 7, loc = bid >> 3;
  const int gblk = xcd * (nb >> 3) + min(xcd, nb & 7) + loc;
  // the simulation, block and phase are the same for the whole workgroup:
  // kept in scalar registers (readfirstlane), so that its KArgs are read with
  // scalar loads
  const void* Ap;
  int phase, blk;
  if (LA.ninst == 0) {
    Ap = LA.single;
    phase = LA.phase0;
    blk = gblk;
  } else {
    const uint32_t e = __builtin_amdgcn_readfirstlane(LA.table[gblk]);
    const unsigned long long pa = (unsigned long long)LA.inst[e >> TAB_INST_SHIFT];
    Ap = (const void*)(((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(pa >> 32)) << 32) |
                       (unsigned)__builtin_amdgcn_readfirstlane((unsigned)pa));
    phase = ((int)((e >> TAB_PHASE_SHIFT) & 7u) + LA.launch) % 6;
    blk = (int)(e & TAB_BLOCK_MASK);
  }
  // The simulation's KArgs never change while a kernel runs: reading them
  // through the constant address space lets the compiler keep them in scalar
  // registers and scalar loads (through a plain pointer it would reload them
  // with vector loads after every store).
  const KAS KArgs<T>& A = *(const KAS KArgs<T>*)Ap;
  const int cur = phase & 1;
  const int slot_cur = phase % 3, slot_prev = (slot_cur + 2) % 3, slot_next = (slot_cur + 1) % 3;
  constexpr int NSA = NS > 0 ? NS : 1;
  using ST = typename StoreT<T, SM>::type;  // stored population type
  constexpr unsigned ES = sizeof(ST);
  constexpr bool DEV = sm_dev(SM);
  // FP32 storage: a flow slot holds s_a = f_a / w_a - R (R the reader's
  // reference density) and a solute slot g_a / J'_a, and the arithmetic works
  // on these (mass carried by the small deviations, weights that sum to one
  // exactly), so that rounding does not drift the balances step after step
  constexpr bool SFORM = std::is_same<T, float>::value && !DEV;
  constexpr bool REFS = DEV || SFORM;  // flow reference codes in the status words
  // row R's homogeneous reaction sources formed while row R + 1 is pulled
  constexpr bool EARLY_RX = !std::is_same<T, double>::value && SM != SM_OUT;
  // this simulation's top side is a free outlet (only in SM_OUT kernels; a
  // batch of mixed simulations runs them all in one)
  const bool outy = SM == SM_OUT && A.c.per_y == 2;
  static_assert(!DEV || std::is_same<T, float>::value, "16-bit storage computes in FP32");
  const KAS KConst& c = A.c;
  const KAS KT<T>& k = A.k;
  // the wavefront's index in the workgroup (one row of 64 lanes each), kept
  // uniform so that the item's rows, bounds and phases stay in scalar
  // registers and its control flow in scalar branches
  const int wv = WPB == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)threadIdx.y);
  __shared__ WaveLds<T, NS, SM> s_all[WPB];
  WaveLds<T, NS, SM>& L = s_all[wv];
  const int lane = threadIdx.x;

  const int item = blk * WPB + wv;
  if (item >= c.nitems) return;  // whole wavefront
  const int sx = item % c.strips, sy = item / c.strips;
  const int x0 = sx * IW, y0 = sy * c.seg_rows;
  const int y1 = min(y0 + c.seg_rows, c.ny);
  const int nrow = y1 - y0;
  const int nx = c.nx, ny = c.ny;
  // a row coordinate inside the lattice, or a ghost row of the free outlet
  // (as the row it repeats), or "outside"
  auto wrap_y = [&](int& Y) -> bool { return outy ? wrap_out(Y, ny) : wrap(Y, ny, c.per_y); };
  const unsigned upitch = (unsigned)c.pitch;
  constexpr unsigned PE = 2 * ES;      // bytes per flow slot (a pair)
  const unsigned PS = upitch * PE;     // bytes per flow slot plane row
  const unsigned RSF = 9u * PS;        // bytes per lattice row, flow: 9 directions x (component 1, 2)
  constexpr int SG = species_group(NS, (int)ES);  // species per solute slot
  constexpr int NGR = (NS + SG - 1) / SG;         // species groups
  constexpr unsigned PEG = SG * ES;               // bytes per solute slot
  constexpr int GSH = SG == 4 ? 1 : 0;            // PEG = PE << GSH
  const unsigned PSG = upitch * PEG;              // bytes per solute slot plane row
  const unsigned RSG = 5u * NGR * PSG;            // bytes per lattice row, solute: groups x 5 directions

  const __amdgpu_buffer_rsrc_t rf = rsrc_of(A.f[cur], c.fbytes);
  const __amdgpu_buffer_rsrc_t rg = rsrc_of(A.g[cur], c.gbytes);
  const __amdgpu_buffer_rsrc_t rt = rsrc_of(A.t[cur], c.tbytes);
  const __amdgpu_buffer_rsrc_t rcw = rsrc_of(A.cw[cur], c.cbytes);
  // written this step: the other buffer of each pair, and the volumes
  const __amdgpu_buffer_rsrc_t wf_ = rsrc_of(A.f[1 - cur], c.fbytes);
  const __amdgpu_buffer_rsrc_t wg_ = rsrc_of(A.g[1 - cur], c.gbytes);
  const __amdgpu_buffer_rsrc_t wt_ = rsrc_of(A.t[1 - cur], c.tbytes);
  const __amdgpu_buffer_rsrc_t wc_ = rsrc_of(A.cw[1 - cur], c.cbytes);
  const __amdgpu_buffer_rsrc_t rv = rsrc_of(A.V, (unsigned)(c.plane * 8));
  const unsigned ncw = (unsigned)c.ncw;

  if (!EXPORT && lane < NRARE_SLOTS) L.rare[lane] = 0.0;

  auto is_fluid = [](uint32_t v) { return (v & LF_FLU) != 0; };
  auto is_liq = [](uint32_t v) { return (v & LF_LIQN) != 0; };
  auto is_rsolid = [](uint32_t v) { return !(v & TB_WALL) && (v & TB_T) >= T_D; };
  // LDS flags of an in-domain node's status word; its liquid mark of this step
  // is added where its density is known
  auto flags_w = [](uint32_t w) -> uint32_t { return (w & 0x1fu) | ((w & TB_T) == T_FLUID ? LF_FLU : 0u); };

  // Liquid threshold of this step (Sec. 4.5): liquid_frac times the largest
  // liquid-component density of the previous step (the partial maxima of its
  // slot; the current step's is known only once every node is updated).
  double rprev = 0.0;
#pragma unroll
  for (int xc = 0; xc < 8; ++xc)
    rprev = fmax(rprev, __longlong_as_double((long long)A.rmax[slot_prev * RM_SLOT + xc * RM_STRIDE]));
  const double thr = c.lfrac * rprev;

  // status word of node (X, Y), TB_WALL outside a non-periodic side
  auto word_at = [&](int X, int Y) -> uint32_t {
    if (wrap(X, nx, c.per_x) && wrap_y(Y)) return bload<uint32_t>(rt, (unsigned)X * 4u, (unsigned)Y * upitch * 4u);
    return TB_WALL;
  };
  // the flow references a node decodes its pulled populations with (FP32 and
  // 16-bit storage): coded in its status word when they were written
  auto refs_of = [&](uint32_t w, T& r1, T& r2) {
    if constexpr (REFS) {
      r1 = ref_value(code1_of(w), k.rb1, SH1);
      r2 = ref_value(code2_of(w), k.rb2, SH2);
    } else {
      r1 = r2 = T(0);
    }
  };

  // Pull (streaming of the previous step): population a arrives from
  // x - e_a = x + e_b (b = opp(a)) if that node was fluid (liquid) then,
  // otherwise it is this node's own population b bounced back at the halfway
  // wall.  co[] are the byte offsets of columns x-1, x, x+1 (wrapped); Yw is
  // the wrapped row of an in-domain node.  withg: the node holds solute.
  auto pull = [&](const unsigned (&co)[3], int Yw, uint32_t w, bool validf, bool withg, T(&f)[2][9], T(&g)[NSA][5]) {
    // (beyond a wall the neighbour bit is clear and the row is never read;
    // beyond the outlet the ghost row is row ny - 1 itself)
    int ym = Yw - 1, yp = Yw + 1;
    if (ym < 0) ym += ny;
    if (yp >= ny) yp = outy ? ny - 1 : yp - ny;
    const unsigned ur[3] = {(unsigned)ym, (unsigned)Yw, (unsigned)yp};
    // a stored value becomes a population: itself (FP64; FP32 keeps the
    // normalised deviation), or (16-bit storage) deviation / scale + weight x
    // this node's reference
    T fb[2][3];
    if constexpr (DEV) {
      T r1, r2;
      refs_of(w, r1, r2);
      if (!validf) r1 = r2 = T(0);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        fb[0][q] = k.wc[q] * r1;
        fb[1][q] = k.wc[q] * r2;
      }
    }
    auto fin = [&](int a, unsigned vo) {
      const Pair<ST> q = bload2<ST>(rf, vo, 0u);
      if constexpr (DEV) {
        f[0][a] = __builtin_fmaf(dev_in<SM>(q.lo), k.isc[0], fb[0][wcls(a)]);
        f[1][a] = __builtin_fmaf(dev_in<SM>(q.hi), k.isc[1], fb[1][wcls(a)]);
      } else {
        f[0][a] = q.lo;
        f[1][a] = q.hi;
      }
    };
    // Every lane issues every load; a node without flow populations (or
    // solute) reads out of range, which gives zero.  16-bit storage: its
    // references are taken as zero too, so that its populations stay zero.
    {
      const unsigned own = co[1] + ur[1] * RSF;
      fin(0, gate(validf, own));
#pragma unroll
      for (int b = 1; b < 9; ++b) {
        const int a = opp(b);
        const bool src = (w >> (NBF_SHIFT + b - 1)) & 1u;
        const unsigned nb = co[ex(b) + 1] + (ur[ey(b) + 1] * RSF + (unsigned)a * PS);
        fin(a, gate(validf, pick_off(src, nb, own + (unsigned)b * PS)));
      }
      if constexpr (SFORM) {
        // Free outlet: the downward populations of the top row have two
        // readers (the row below, and the top row through the ghost row), so
        // they are stored with reference zero; re-reference them here
        if (outy && Yw >= ny - 2) {
          T r1, r2;
          refs_of(w, r1, r2);
          if (!validf) r1 = r2 = T(0);
#pragma unroll
          for (int b = 1; b < 9; ++b) {
            const int a = opp(b);
            const bool src = (w >> (NBF_SHIFT + b - 1)) & 1u;
            // the value read is slot a of the row above (pulled), or own slot b
            const bool zref = src ? (ey(a) < 0) : (ey(b) < 0 && Yw == ny - 1);
            f[0][a] -= zref ? r1 : T(0);
            f[1][a] -= zref ? r2 : T(0);
          }
        }
      }
    }
    if constexpr (NS == 0) {
#pragma unroll
      for (int a = 0; a < 5; ++a) g[0][a] = T(0);
    } else {
      const unsigned own = (co[1] << GSH) + ur[1] * RSG;
      T gb[NSA][2];
      if constexpr (DEV) {
        // this node's solute reference codes, one word per four species
        const unsigned cwo = gate(withg, (co[1] / PE) * 4u + ur[1] * ncw * upitch * 4u);
        const uint32_t cw0 = bload<uint32_t>(rcw, cwo, 0u);
        const uint32_t cw1 = NS > 4 ? bload<uint32_t>(rcw, cwo, upitch * 4u) : 0u;
#pragma unroll
        for (int kk = 0; kk < NS; ++kk) {
          T cr = ref_value(((kk < 4 ? cw0 : cw1) >> (8 * (kk & 3))) & 255u, k.rbc[kk], SHC);
          if (!withg) cr = T(0);
          gb[kk][0] = k.Jc[kk][0] * cr;
          gb[kk][1] = k.Jc[kk][1] * cr;
        }
      }
      auto gcv = [&](int kk, int a, ST v) -> T {
        if constexpr (DEV) return __builtin_fmaf(dev_in<SM>(v), k.iscg[kk], gb[kk][a == 0 ? 0 : 1]);
        else return v;
      };
      // species group j holds species SG j .. SG j + SG - 1
      auto gin = [&](int a, unsigned vo) {
#pragma unroll
        for (int j = 0; j < NGR; ++j) {
          const Grp<ST, SG> q = bloadg<ST, SG>(rg, vo, (unsigned)(j * 5) * PSG);
#pragma unroll
          for (int i = 0; i < SG; ++i)
            if (j * SG + i < NS) g[j * SG + i][a] = gcv(j * SG + i, a, q.v[i]);
        }
      };
      gin(0, gate(withg, own));
      // On the top row at a free outlet the ghost row above sends slot 2, not
      // slot 4, of the node itself: the writer keeps its post-collision
      // population 4 there (slot 4 may carry a reactive bounce-back).  The
      // shift is zero in every other kernel, which keeps their address
      // arithmetic (and load schedule) as it is.
      const bool gtop = outy && Yw == ny - 1;
#pragma unroll
      for (int b = 1; b < 5; ++b) {
        const int a = opp(b);
        const bool src = (w >> (NBL_SHIFT + b - 1)) & 1u;
        const unsigned sh = (b == 2 && gtop) ? 2u * PSG : 0u;
        const unsigned nb = (co[ex(b) + 1] << GSH) + (ur[ey(b) + 1] * RSG + (unsigned)a * PSG - sh);
        gin(a, gate(withg, pick_off(src, nb, own + (unsigned)b * PSG)));
      }
    }
  };

  // moments (Eq. 9, 23); terms with a zero velocity component are skipped:
  // adding +-0 to the running sum would not change it.  FP32 storage: the
  // deviations s_a = f_a / w_a - R give rho - R = sum w_a s_a and j = sum w_a
  // s_a e_a (the w_a are 16, 4 and 1 over 36); solute C = J0' t_0 + J1' (t_1 +
  // .. + t_4) with t_a = g_a / J'_a.
  auto moments = [&](const T(&f)[2][9], const T(&g)[NSA][5], uint32_t w, bool validf, Mom<T, NS>& m) {
    if constexpr (SFORM) {
      T r[2] = {T(0), T(0)};  // a node without flow populations has none
      if (validf) refs_of(w, r[0], r[1]);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const T ax = ((f[s][1] + f[s][2]) + f[s][3]) + f[s][4];
        const T dg = ((f[s][5] + f[s][6]) + f[s][7]) + f[s][8];
        m.drho[s] = (T(16) * f[s][0] + T(4) * ax + dg) * T(1.0 / 36.0);
        m.rho[s] = r[s] + m.drho[s];
        m.jx[s] = (T(4) * (f[s][1] - f[s][3]) + ((f[s][5] - f[s][6]) - f[s][7] + f[s][8])) * T(1.0 / 36.0);
        m.jy[s] = (T(4) * (f[s][2] - f[s][4]) + ((f[s][5] + f[s][6]) - f[s][7] - f[s][8])) * T(1.0 / 36.0);
      }
#pragma unroll
      for (int kk = 0; kk < NSA; ++kk)
        m.C[kk] = k.Jp0[kk] * g[kk][0] + k.Jp1[kk] * (((g[kk][1] + g[kk][2]) + g[kk][3]) + g[kk][4]);
    } else {
      (void)w;
      (void)validf;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        m.rho[s] = T(0);
        m.jx[s] = T(0);
        m.jy[s] = T(0);
        m.drho[s] = T(0);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
          m.rho[s] += f[s][a];
          if (ex(a) != 0) m.jx[s] += f[s][a] * T(ex(a));
          if (ey(a) != 0) m.jy[s] += f[s][a] * T(ey(a));
        }
      }
#pragma unroll
      for (int kk = 0; kk < NSA; ++kk) {
        T cs = T(0);
#pragma unroll
        for (int a = 0; a < 5; ++a) cs += g[kk][a];
        m.C[kk] = cs;
      }
    }
  };

  // effective masses: psi_1 from the CS EOS (Eq. 12, 13), phi_1, phi_2 (Eq. 15)
  auto effmass = [&](bool fluid, const T(&rho)[2], T& ps, T& q1, T& q2, bool& clamped, unsigned& errf) {
    ps = q1 = q2 = T(0);
    clamped = false;
    if (fluid) {
      if (c.has_psi) {
        if (!(T(0.25) * k.b * rho[0] < T(1))) errf |= ERR_EOS;
        if constexpr (SFORM) {
          // FP32 storage: the two terms of Eq. 12 nearly cancel in the liquid
          // (the pressure is a few hundredths of each), so psi_1 is formed in
          // FP64 from the node's density and rounded once
          const double r0 = (double)rho[0];
          const double e = 0.25 * c.b * r0, om = 1.0 - e;
          const double pcs = r0 * c.RT * (1.0 + e + e * e - e * e * e) / (om * om * om) - c.a * r0 * r0;
          double arg = c.psi_pre * (pcs - r0 * (1.0 / 3.0)) * c.rG11;
          if (arg < 0.0) {
            arg = 0.0;
            clamped = true;
          }
          ps = (T)sqrt(arg);
        } else {
          T arg = cdiv<T>(k.psi_pre * (p_cs<T>(k, rho[0]) - cdiv<T>(rho[0], T(3), T(1.0 / 3.0))), k.G11, k.r_G11);
          if (arg < T(0)) {
            arg = T(0);
            clamped = true;
          }
          ps = dsqrt<T>(arg);
        }
      }
      if (c.has_phi1) q1 = T(1) - dexp<T>(-cdiv<T>(rho[1], k.rho20, k.r_rho20));
      if (c.has_phi2) q2 = k.a0 - dexp<T>(-cdiv<T>(rho[0], k.rho10, k.r_rho10));
    }
  };

  // the references this node's populations are coded against when they are
  // written this step (from the current moments; stored in its status and
  // solute words for the reader)
  auto wref = [&](const Mom<T, NS>& m, RF<T>& r, T(&cf)[NSA]) {
    if constexpr (REFS) {
      r.r1 = ref_value(ref_code(m.rho[0], k.rb1, SH1, MAX1), k.rb1, SH1);
      r.r2 = ref_value(ref_code(m.rho[1], k.rb2, SH2, MAX2), k.rb2, SH2);
    }
    if constexpr (DEV) {
#pragma unroll
      for (int kk = 0; kk < NSA; ++kk) cf[kk] = ref_value(ref_code(m.C[kk], k.rbc[kk], SHC, MAXC), k.rbc[kk], SHC);
    }
  };

  // A liquid node's contribution to the volume of a reactive solid D2Q5
  // neighbour (Eq. 33, A2): the flux of every reaction on that solid's surface
  // from the node's concentration (zero for a liquid node without content),
  // times -Vbar (CONSUMES) or +Vbar (MINERAL), summed in reaction order.
  // Formed once per node where its moments are staged, so that a solid node
  // adds up its neighbours' values.
  // Sec. 4.1: with a subtracted species m, a liquid node's C_m is the total
  // liquid concentration (sub_tot rho_1) minus the other species, in species
  // order (the same operations as the plain definition)
  auto subtract = [&](T (&C)[NS > 0 ? NS : 1], T rho1) {
    if (NS > 1 && c.sub >= 0) {
      T cs = k.sub_tot * rho1;
#pragma unroll
      for (int kk = 0; kk < NS; ++kk) cs -= kk != c.sub ? C[kk] : T(0);
#pragma unroll
      for (int kk = 0; kk < NS; ++kk) C[kk] = kk == c.sub ? cs : C[kk];
    }
  };
  const bool any_xsolid = NS > 0 && (c.xsolid[0] || c.xsolid[1]);
  auto solid_dv = [&](bool liqn, uint32_t w, const Mom<T, NS>& m) -> VS {
    VS o{0.0, 0.0};
    if (any_xsolid) {
      const int nsf = sf_of(w);
      const bool has = nsf == SF_STREAM || nsf == SF_HOLD;
      // the concentrations the node's own collision sees (none if it has
      // just become liquid without content; the subtracted species derived)
      T ce[NS > 0 ? NS : 1];
#pragma unroll
      for (int kk = 0; kk < (NS > 0 ? NS : 1); ++kk) ce[kk] = has ? m.C[kk] : T(0);
      subtract(ce, m.rho[0]);
      for (int r = 0; r < c.nhet; ++r) {
        const T cr = sel<NS>(ce, c.xre[r]);
        T v = k.xkap[r] * (cr - k.xCeq[r]);
        if (c.xirrev[r] && v < T(0)) v = T(0);
        o.d += c.xsv[0][r] * (double)v;
        o.f += c.xsv[1][r] * (double)v;
      }
      if (!liqn) o.d = o.f = 0.0;
    }
    return o;
  };

  auto col_offsets = [&](int Xw, unsigned (&co)[3]) {
    int xm = Xw - 1, xp = Xw + 1;
    if (xm < 0) xm += nx;
    if (xp >= nx) xp -= nx;
    co[0] = (unsigned)xm * PE;
    co[1] = (unsigned)Xw * PE;
    co[2] = (unsigned)xp * PE;
  };

  // this lane's column: the item's own columns on lanes 1 .. IW, a halo
  // column on lanes 0 and SW - 1
  int Xw = x0 - 1 + lane;
  const bool colin = wrap(Xw, nx, c.per_x);
  const int X = x0 - 1 + lane;
  const bool colown = lane >= 1 && lane <= IW && X < nx;
  unsigned co[3];
  col_offsets(colin ? Xw : 0, co);

  // status word of this lane's column in row Y (the column is wrapped once)
  auto word_row = [&](int Y) -> uint32_t {
    const bool in = colin && wrap_y(Y);
    const uint32_t v = bload<uint32_t>(rt, gate(in, (unsigned)Xw * 4u + (unsigned)Y * upitch * 4u), 0u);
    return in ? v : (uint32_t)TB_WALL;
  };
  uint32_t w_cur = 0, w_next = word_row(y0 - 1);
  // per-lane balance contributions over the item's rows, in FP64: the gas
  // component's homogeneous source (the liquid component's is its exact
  // negative), the solute sources and the heterogeneous exchange
  double l_msrc = 0.0;
  double l_ssrc[NSA], l_shet[NSA];
#pragma unroll
  for (int kk = 0; kk < NSA; ++kk) l_ssrc[kk] = l_shet[kk] = 0.0;
  double l_vdv = 0.0;
  T my_rmax = T(0);

  // Homogeneous reactions at a liquid node (Eq. 5a, 5c, 27, 28): the species
  // sources Sk (net stoichiometric coefficients times the rates) and the gas
  // component's source Sg (the liquid component's is -Sg), added to the
  // node's balances.  nbt: the solid types among its D2Q5 neighbours, for
  // surface-enhanced rates.
  auto hom_sources = [&](const Mom<T, NS>& m, uint32_t nbt, T (&Sk)[NSA], T& Sg) {
    const T r2 = m.rho[1];
    for (int r = 0; r < c.nhom; ++r) {
      T Rr;
      // (behind the uniform test, the rate stays a scalar operand)
      T kr = k.hk[r];
      if (c.any_hsurf && (c.hsurf[r] & nbt)) kr = k.hks[r];
      if (c.hkind[r] == HOM_FIRST) {
        Rr = kr * sel<NS>(m.C, c.hre0[r]);
      } else if (c.hkind[r] == HOM_BI) {
        Rr = kr * sel<NS>(m.C, c.hre0[r]) * sel<NS>(m.C, c.hre1[r]);
      } else {
        T cg = cdiv<T>(r2, k.hMgas[r], k.r_hMgas[r]);
        if (cg < T(0)) cg = T(0);
        Rr = kr * (sel<NS>(m.C, c.hre0[r]) -
                   cdiv<T>(sel<NS>(m.C, c.hpr0[r]) * dsqrt<T>(cg), k.hKeq[r], k.r_hKeq[r]));
        Sg += T(0.5) * Rr * k.hMgas[r];
      }
#pragma unroll
      for (int kk = 0; kk < NS; ++kk) Sk[kk] += k.hnu[r][kk] * Rr;
    }
    l_msrc += (double)Sg;
#pragma unroll
    for (int kk = 0; kk < NS; ++kk) l_ssrc[kk] += (double)Sk[kk];
  };

  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");

  // The march: iteration R pulls row R + 1 into the ring and collides row R.
  // The first two iterations (R = y0 - 2, y0 - 1) only fill the ring.
  T fc[2][9], gc[NSA][5];
  Mom<T, NS> mc;
  // The FP64 volume of this lane's node is loaded one iteration before its row
  // is collided where it may be needed: at a reactive solid node, and at a
  // fluid node next to a non-fluid one (a liquid node collects precipitate on
  // its links to reactive solid).  A load in the middle of a row would wait for
  // every memory operation the wavefront has in flight.
  auto vol_pre = [](uint32_t w) -> bool {
    const int t = (int)(w & TB_T);
    return t == T_D || t == T_F || (t == T_FLUID && ((w >> NBF_SHIFT) & 0xFu) != 0xFu);
  };
  double v_cur = 0.0;
  int sm = 1, s0 = 2, sp = 0;
  for (int R = y0 - 2; R < y1; ++R) {
    const int Rn = R + 1;
    const uint32_t w_nn = word_row(R + 2);  // next iteration's row, loaded ahead
    const bool vpre = !EXPORT && colown && Rn >= y0 && Rn < y1 && vol_pre(w_next);
    const double v_nn = EXPORT ? 0.0 : bload<double>(rv, gate(vpre, ((unsigned)Rn * upitch + (unsigned)X) * 8u), 0u);
    T fn[2][9], gn[NSA][5];
    Mom<T, NS> mn;
    // row R's node-local results formed while the pull of row R + 1 is in
    // flight (see below)
    T e_Sk[NSA], e_Sg = T(0);
#pragma unroll
    for (int kk = 0; kk < NSA; ++kk) e_Sk[kk] = T(0);
    uint32_t e_cwc0 = 0u, e_cwc1 = 0u;
    {
      // ---------------------------------------------------- phase 1, row R + 1
      int Yw = Rn;
      const bool rowin = wrap_y(Yw);
      const bool indom = colin && rowin;
      const uint32_t w = w_next;
      const int t = (int)(w & TB_T);
      const bool fluid = indom && t == T_FLUID;
      const bool validf = indom && (t == T_FLUID || (w & TB_STR));
      const bool withg = indom && sf_of(w) != SF_NONE;
      pull(co, rowin ? Yw : 0, w, validf, withg, fn, gn);
      // While those loads are in flight: row R's work that needs nothing of
      // row R + 1 (its own status word, its liquid mark staged in the ring
      // last iteration, its moments).  16-bit storage: the node's solute
      // reference codes for its own pull next step, from its staged moments
      // (the references its neighbours code the populations they send it
      // against).  Solute amendments (Sec. 4.5; Step 2): a node that turns
      // liquid without content starts at zero (a node that was sending shares
      // has handed its content over), and a subtracted species is derived
      // (Sec. 4.1).  Then the homogeneous reaction sources, unless a rate
      // depends on the solid types around the node (row R + 1 among them);
      // the FP64 and free-outlet kernels form the sources in phase 2 (in the
      // FP64 outlet kernel with two species, forming them here gave wrong
      // product concentrations that came and went with unrelated code
      // changes; its cause was not found).
      if (R >= y0) {
        Mom<T, NS>& m = mc;
        T(&g)[NSA][5] = gc;
        const uint32_t w0 = w_cur;
        const bool fluid0 = colin && (int)(w0 & TB_T) == T_FLUID;
        const int sf0 = colin ? sf_of(w0) : SF_NONE;
        const bool liq0 = colin && is_liq(flags_of<T>(L.pq[s0][lane + 1].fl));
        if constexpr (DEV) {
#pragma unroll
          for (int kk = 0; kk < NS; ++kk) {
            const uint32_t cc = ref_code(m.C[kk], k.rbc[kk], SHC, MAXC) << (8 * (kk & 3));
            if (kk < 4) e_cwc0 |= cc;
            else e_cwc1 |= cc;
          }
        }
        if (NS > 0) {
          if (liq0 && (sf0 == SF_NONE || sf0 == SF_SHARE)) {
#pragma unroll
            for (int kk = 0; kk < NSA; ++kk) {
              m.C[kk] = T(0);
#pragma unroll
              for (int a = 0; a < 5; ++a) g[kk][a] = T(0);
            }
          }
          if (NS > 1 && c.sub >= 0) {
            T cd[NSA];
#pragma unroll
            for (int kk = 0; kk < NSA; ++kk) cd[kk] = m.C[kk];
            subtract(cd, m.rho[0]);
#pragma unroll
            for (int kk = 0; kk < NSA; ++kk) m.C[kk] = liq0 ? cd[kk] : m.C[kk];
          }
        }
        if (EARLY_RX && !EXPORT && !c.any_hsurf && colown && fluid0 && liq0) hom_sources(m, 0u, e_Sk, e_Sg);
      }
      moments(fn, gn, w, validf, mn);
      unsigned errf = 0;
      const bool bad = validf && (!(mn.rho[0] >= T(0)) || !(mn.rho[1] >= T(0)) || (fluid && !(mn.rho[0] + mn.rho[1] > T(0))));
      errf |= bad ? (unsigned)ERR_DENSITY : 0u;
      T ps, q1, q2;
      bool clamped;
      effmass(fluid, mn.rho, ps, q1, q2, clamped, errf);
      const bool mine = !EXPORT && colown && Rn >= y0 && Rn < y1;
      if (mine && errf) {
        atomicOr(&A.err[0], errf);
        atomicMin(&A.err[1], (unsigned)(Rn * nx + X));
      }
      if (!EXPORT) {
        const unsigned long long bc = __ballot(mine && clamped);
        if (bc && lane == 0) L.rare[5] += (double)__popcll(bc);
      }
      const int cl = lane + 1;
      const uint32_t fl = indom ? (flags_w(w) | ((fluid && (double)mn.rho[0] > thr) ? LF_LIQN : 0u)) : (uint32_t)TB_WALL;
      L.pq[sp][cl] = PQ<T>{ps, q1, q2, flags_as<T>(fl)};
      if (!EXPORT) L.vs[sp][cl] = solid_dv((fl & LF_LIQN) != 0, w, mn);
      L.r1[sp][cl] = mn.rho[0];
      L.r2[sp][cl] = mn.rho[1];
#pragma unroll
      for (int kk = 0; kk < NSA; ++kk) L.C[kk][sp][cl] = mn.C[kk];
      if constexpr (REFS) {
        RF<T> r;
        T cf[NSA];
        wref(mn, r, cf);
        L.rf[sp][cl] = r;
        if constexpr (DEV) {
#pragma unroll
          for (int kk = 0; kk < NSA; ++kk) L.Cf[kk][sp][cl] = cf[kk];
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");

    // what row R stores, and where (out of range: nothing)
    unsigned so_f = OOB_OFF, so_g = OOB_OFF, so_t = OOB_OFF, so_c = OOB_OFF, so_v = OOB_OFF;
    uint32_t wst = 0u, cws0 = 0u, cws1 = 0u;
    double vnew = 0.0;
    if (R >= y0) {
      // ---------------------------------------------------- phase 2, row R
      const uint32_t w = w_cur;
      const int t = (int)(w & TB_T);
      const bool own = colown;  // R < y1 <= ny
      const bool fluid = colin && t == T_FLUID;
      const int sf = colin ? sf_of(w) : SF_NONE;
      const unsigned idx = (unsigned)R * upitch + (unsigned)X;
      auto slot = [&](int dy) { return dy < 0 ? sm : (dy > 0 ? sp : s0); };
      // the flags of the eight neighbours (and their psi, phi)
      // (their records are read from the ring where they are used)
      auto nq = [&](int a) -> const PQ<T>& { return L.pq[slot(ey(a))][lane + 1 + ex(a)]; };
      uint32_t nt[9];
#pragma unroll
      for (int a = 0; a < 9; ++a) nt[a] = flags_of<T>(nq(a).fl);
      const bool liq = colin && is_liq(nt[0]);  // liquid mark of this step (Sec. 4.5)
      // The amendments of Sec. 4.5 move content between lattice nodes only:
      // beyond the free outlet there is no node to give, take or be counted,
      // so their neighbour flags (am) see a wall there; transport and forces
      // (nt) see the ghost row.
      const bool top_out = outy && R == ny - 1;
      auto am = [&](int a) -> uint32_t { return (top_out && ey(a) > 0) ? (uint32_t)TB_WALL : nt[a]; };
      // node flags two links away (the rare stranded-population path)
      auto far_flags = [&](int dx, int dy) -> uint32_t {
        if (outy && R + dy >= ny) return TB_WALL;
        const uint32_t v = word_at(X + dx, R + dy);
        return (v & TB_WALL) ? (uint32_t)TB_WALL : flags_w(v);
      };
      Mom<T, NS>& m = mc;
      const T ps = nq(0).ps, q1 = nq(0).q1, q2 = nq(0).q2;
      T(&f)[2][9] = fc;
      T(&g)[NSA][5] = gc;

      // Solute amendments (Sec. 4.5; Step 2): the shares in transit from D2Q5
      // neighbours that left the liquid set last step reach this node if it
      // was liquid then (the node's own amendments were made while the pull
      // was in flight).
      const uint32_t cwc0 = e_cwc0, cwc1 = e_cwc1;
      T Cin[NSA];
#pragma unroll
      for (int kk = 0; kk < NSA; ++kk) Cin[kk] = T(0);
      bool any_in_w = false;  // some lane of this row takes shares
      if (NS > 0) {
        bool any_in = false;
#pragma unroll
        for (int a = 1; a < 5; ++a) any_in |= !(am(a) & TB_WALL) && sf_of(am(a)) == SF_SHARE;
        any_in = any_in && sf == SF_STREAM;
        any_in_w = __ballot(any_in) != 0ull;
        if (any_in) {
#pragma unroll
          for (int a = 1; a < 5; ++a)
            if (!(am(a) & TB_WALL) && sf_of(am(a)) == SF_SHARE) {
              const int sl = slot(ey(a)), lx = lane + 1 + ex(a);
#pragma unroll
              for (int kk = 0; kk < NS; ++kk) Cin[kk] += L.C[kk][sl][lx];
            }
        }
      }

      bool precip = false;
      bool storef = false, storeg = false;  // this lane holds valid post-collision populations

      if (own && fluid) {
        my_rmax = m.rho[0] > my_rmax ? m.rho[0] : my_rmax;
        // forces: Eq. 11 (cohesion), 14 (inter-component), 16 (adhesion), body
        // force.  A non-fluid neighbour has s = 1 and, in the cohesion and
        // inter-component sums, the psi / phi of its mirror image in the wall
        // within the 3x3 block: the centre node for an axis link; for a
        // diagonal link the fluid axis neighbour(s) sharing its column or row
        // (their mean when both are fluid), else the centre.  The ring holds
        // zero psi / phi at non-fluid nodes, so an axis link's share is the
        // centre's value times the axis solid-neighbour sum.
        // In FP32 the sums take each neighbour's difference from the centre
        // value (the weighted link vectors sum to zero, so this is the same
        // sum): in a smooth region the differences are small and exact, and
        // the sum keeps its accuracy instead of cancelling large terms.
        T c1x = 0, c1y = 0, c12x = 0, c12y = 0, c21x = 0, c21y = 0, swx = 0, swy = 0, sax = 0, say = 0;
        const T ps0 = SFORM ? ps : T(0), q10 = SFORM ? q1 : T(0), q20 = SFORM ? q2 : T(0);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
          const bool nf = !is_fluid(nt[a]);
          const T sw = nf ? T(1) : T(0);
          T vps = nq(a).ps - ps0, vq1 = nq(a).q1 - q10, vq2 = nq(a).q2 - q20;
          if (SFORM && nf && a < 5) vps = vq1 = vq2 = T(0);  // the centre's mirror image
          if (a >= 5) {
            const int ax = ex(a) > 0 ? 1 : 3, ay = ey(a) > 0 ? 2 : 4;
            const bool fx = is_fluid(nt[ax]), fy = is_fluid(nt[ay]);
            const T h = (fx && fy) ? T(0.5) : T(1);
            const bool ownm = !fx && !fy;
            // (formed on every lane and selected: a branch per diagonal
            // costs more than the arithmetic)
            T mps, mq1, mq2;
            if constexpr (SFORM) {
              const T dxp = fx ? nq(ax).ps - ps : T(0), dyp = fy ? nq(ay).ps - ps : T(0);
              const T dx1 = fx ? nq(ax).q1 - q1 : T(0), dy1 = fy ? nq(ay).q1 - q1 : T(0);
              const T dx2 = fx ? nq(ax).q2 - q2 : T(0), dy2 = fy ? nq(ay).q2 - q2 : T(0);
              mps = (dxp + dyp) * h;
              mq1 = (dx1 + dy1) * h;
              mq2 = (dx2 + dy2) * h;
            } else {
              mps = ownm ? ps : (nq(ax).ps + nq(ay).ps) * h;
              mq1 = ownm ? q1 : (nq(ax).q1 + nq(ay).q1) * h;
              mq2 = ownm ? q2 : (nq(ax).q2 + nq(ay).q2) * h;
            }
            vps = nf ? mps : vps;
            vq1 = nf ? mq1 : vq1;
            vq2 = nf ? mq2 : vq2;
          }
          if (ex(a) != 0) {
            c1x += T(wf(a) * ex(a)) * vps;
            c12x += T(wf(a) * ex(a)) * vq2;
            c21x += T(wf(a) * ex(a)) * vq1;
            swx += T(wf(a) * ex(a)) * sw;
            if (a < 5) sax += T(wf(a) * ex(a)) * sw;
          }
          if (ey(a) != 0) {
            c1y += T(wf(a) * ey(a)) * vps;
            c12y += T(wf(a) * ey(a)) * vq2;
            c21y += T(wf(a) * ey(a)) * vq1;
            swy += T(wf(a) * ey(a)) * sw;
            if (a < 5) say += T(wf(a) * ey(a)) * sw;
          }
        }
        if constexpr (!SFORM) {
          c1x += ps * sax;
          c1y += ps * say;
          c12x += q2 * sax;
          c12y += q2 * say;
          c21x += q1 * sax;
          c21y += q1 * say;
        }
        const T r1 = m.rho[0], r2 = m.rho[1];
        T Fx[2], Fy[2];
        Fx[0] = -k.G11 * ps * c1x - k.G12 * q1 * c12x - k.w1 * ps * swx + r1 * k.gx;
        Fy[0] = -k.G11 * ps * c1y - k.G12 * q1 * c12y - k.w1 * ps * swy + r1 * k.gy;
        Fx[1] = -k.G21 * q2 * c21x - k.w2 * r2 * swx + r2 * k.gx;
        Fy[1] = -k.G21 * q2 * c21y - k.w2 * r2 * swy + r2 * k.gy;
        // velocities: Eq. 18 (common), 17 (shifted equilibrium), 19 (physical)
        const T den = cdiv<T>(r1, k.tau[0], k.r_tau[0]) + cdiv<T>(r2, k.tau[1], k.r_tau[1]);
        const T upx = qdiv<T>(cdiv<T>(m.jx[0], k.tau[0], k.r_tau[0]) + cdiv<T>(m.jx[1], k.tau[1], k.r_tau[1]), den);
        const T upy = qdiv<T>(cdiv<T>(m.jy[0], k.tau[0], k.r_tau[0]) + cdiv<T>(m.jy[1], k.tau[1], k.r_tau[1]), den);
        T ux[2], uy[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const T r = m.rho[s];
          ux[s] = upx;
          uy[s] = upy;
          const T vx = upx + qdiv<T>(k.tau[s] * Fx[s], r), vy = upy + qdiv<T>(k.tau[s] * Fy[s], r);
          ux[s] = r > T(1e-12) ? vx : ux[s];
          uy[s] = r > T(1e-12) ? vy : uy[s];
        }
        const T rt_ = r1 + r2;
        const T urx = qdiv<T>(m.jx[0] + m.jx[1] + T(0.5) * (Fx[0] + Fx[1]), rt_);
        const T ury = qdiv<T>(m.jy[0] + m.jy[1] + T(0.5) * (Fy[0] + Fy[1]), rt_);

        if (EXPORT) {
          LA.out[2 * c.plane + idx] = (double)urx;
          LA.out[3 * c.plane + idx] = (double)ury;
        } else {
          // homogeneous reaction sources: formed while the pull was in
          // flight, or here where a rate depends on the neighbours' solid
          // types (surface-enhanced rates) and in the FP64 and outlet kernels
          T Sk[NSA];
#pragma unroll
          for (int kk = 0; kk < NSA; ++kk) Sk[kk] = e_Sk[kk];
          T Sg = e_Sg;
          if (liq && (!EARLY_RX || c.any_hsurf)) {
            uint32_t nbt = 0u;
            if (c.any_hsurf) {
#pragma unroll
              for (int a = 1; a < 5; ++a)
                if (!(nt[a] & TB_WALL)) nbt |= 1u << (nt[a] & TB_T);
            }
            hom_sources(m, nbt, Sk, Sg);
          }
          const T Ss[2] = {T(0) - Sg, Sg};
          // flow collision (Eq. 6, 8)
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const T om = k.om[s];
            const T usq = ux[s] * ux[s] + uy[s] * uy[s];
            if constexpr (std::is_same<T, double>::value) {
              // literal Eq. 6 and 8
#pragma unroll
              for (int a = 0; a < 9; ++a) {
                const T eu = (ex(a) == 0 ? T(0) : T(ex(a)) * ux[s]) + (ey(a) == 0 ? T(0) : T(ey(a)) * uy[s]);
                const T feq = T(w9(a)) * m.rho[s] * (T(1) + T(3) * eu + T(4.5) * eu * eu - T(1.5) * usq);
                f[s][a] = f[s][a] - om * (f[s][a] - feq) + T(w9(a)) * Ss[s];
              }
            } else if constexpr (SFORM) {
              // Eq. 6 and 8 divided by w_a, on the deviations from the decoding
              // reference R: s* = (1-om) s + om (rho - R + rho P_a) + S, with
              // P_a = 3 e.u + 4.5 (e.u)^2 - 1.5 u^2
              const T oneom = T(1) - om;
#pragma unroll
              for (int a = 0; a < 9; ++a) {
                const T eu = (ex(a) == 0 ? T(0) : T(ex(a)) * ux[s]) + (ey(a) == 0 ? T(0) : T(ey(a)) * uy[s]);
                const T P = eu * (T(3) + T(4.5) * eu) - T(1.5) * usq;
                f[s][a] = oneom * f[s][a] + om * (m.drho[s] + m.rho[s] * P) + Ss[s];
              }
            } else {
              // the same update factored: f* = (1-om) f + om w rho (1 - 1.5 u^2 + eu (3 + 4.5 eu)) + w S
              const T oneom = T(1) - om;
              const T base = T(1) - T(1.5) * usq;
#pragma unroll
              for (int a = 0; a < 9; ++a) {
                const T eu = (ex(a) == 0 ? T(0) : T(ex(a)) * ux[s]) + (ey(a) == 0 ? T(0) : T(ey(a)) * uy[s]);
                const T wr = T(w9(a)) * om * m.rho[s];
                f[s][a] = oneom * f[s][a] + wr * (base + eu * (T(3) + T(4.5) * eu)) + T(w9(a)) * Ss[s];
              }
            }
          }
          // (a) populations stranded in a node that became SOLID_F last step go,
          // at rest, equally to that node's fluid D2Q9 neighbours
          bool any_str = false;
#pragma unroll
          for (int a = 1; a < 9; ++a) any_str |= !(nt[a] & TB_WALL) && (nt[a] & TB_STR);
          if (any_str) {
            T don[2] = {T(0), T(0)};
#pragma unroll
            for (int a = 1; a < 9; ++a) {
              if (!(am(a) & TB_WALL) && (am(a) & TB_STR)) {
                int mm = 0;
#pragma unroll 1
                for (int b = 1; b < 9; ++b) mm += is_fluid(far_flags(ex(a) + ex(b), ey(a) + ey(b))) ? 1 : 0;
                const int sl = slot(ey(a)), lx = lane + 1 + ex(a);
                don[0] += L.r1[sl][lx] / T(mm);
                don[1] += L.r2[sl][lx] / T(mm);
              }
            }
#pragma unroll
            for (int s = 0; s < 2; ++s)
              if (don[s] != T(0)) {
#pragma unroll
                for (int a = 0; a < 9; ++a) f[s][a] += SFORM ? don[s] : T(w9(a)) * don[s];
              }
          }
          storef = true;

          if (NS > 0 && liq) {
            // solute collision (Eq. 20-22) with the physical velocity u_r
#pragma unroll
            for (int kk = 0; kk < NS; ++kk) {
              const T om = k.omg[kk];
              if constexpr (std::is_same<T, double>::value) {
                // literal Eq. 20 and 21
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                  const T J = k.J[kk][a];
                  const T eu = (ex(a) == 0 ? T(0) : T(ex(a)) * urx) + (ey(a) == 0 ? T(0) : T(ey(a)) * ury);
                  const T geq = m.C[kk] * (J + T(0.5) * eu);
                  g[kk][a] = g[kk][a] - om * (g[kk][a] - geq) + J * Sk[kk];
                }
              } else if constexpr (SFORM) {
                // Eq. 20-21 divided by J'_a: t* = (1-om) t + om C + S + (om C / (2 J'_a)) e.u
                const T oneom = T(1) - om;
                const T b = om * m.C[kk] + Sk[kk];
                const T hc = om * m.C[kk] * k.hJ[kk];
                const T hx = hc * urx, hy = hc * ury;
                g[kk][0] = oneom * g[kk][0] + b;
                g[kk][1] = oneom * g[kk][1] + b + hx;
                g[kk][2] = oneom * g[kk][2] + b + hy;
                g[kk][3] = oneom * g[kk][3] + b - hx;
                g[kk][4] = oneom * g[kk][4] + b - hy;
              } else {
                // factored: g* = (1-om) g + J (om C + S) + (om C / 2) e.u
                const T oneom = T(1) - om;
                const T omC = om * m.C[kk];
                const T hx = T(0.5) * omC * urx, hy = T(0.5) * omC * ury;
                const T b0 = k.J[kk][0] * (omC + Sk[kk]);
                const T b1 = k.J[kk][1] * (omC + Sk[kk]);
                g[kk][0] = oneom * g[kk][0] + b0;
                g[kk][1] = oneom * g[kk][1] + b1 + hx;
                g[kk][2] = oneom * g[kk][2] + b1 + hy;
                g[kk][3] = oneom * g[kk][3] + b1 - hx;
                g[kk][4] = oneom * g[kk][4] + b1 - hy;
              }
            }
            // (b) the shares taken this step, at rest
            // (zero at nodes that take none)
            if (any_in_w) {
#pragma unroll
              for (int kk = 0; kk < NS; ++kk)
#pragma unroll
                for (int a = 0; a < 5; ++a) g[kk][a] += SFORM ? Cin[kk] : k.J[kk][a] * Cin[kk];
            }
            // heterogeneous link fluxes (Eq. 29-31, A2): a population heading into a
            // reactive solid comes back next step minus the reactant's (plus the
            // product's) link flux; the node also collects the precipitate of GROWS
            // reactions (Eq. 35)
            // Free outlet: the ghost row above a top-row node sends it that
            // node's post-collision population 4, which slot 4 may not keep (a
            // reactive link below bounces it back with its flux); slot 2 heads
            // out through the outlet and is read by nobody, so it keeps the copy.
            if (top_out) {
#pragma unroll
              for (int kk = 0; kk < NSA; ++kk) g[kk][2] = g[kk][4];
            }
            bool any_rs = false;
#pragma unroll
            for (int a = 1; a < 5; ++a) any_rs |= is_rsolid(nt[a]);
            if (any_rs) {
              // every reaction's flux from this node's concentration, summed
              // per reactive solid type into each species' net link flux (a
              // product gains, a reactant loses it) and the precipitate
              // volume one link collects
              T dq[2][NSA];
              double vq[2] = {0.0, 0.0};
#pragma unroll
              for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int kk = 0; kk < NSA; ++kk) dq[q][kk] = T(0);
              for (int r = 0; r < c.nhet; ++r) {
                T v = k.xkap[r] * (sel<NS>(m.C, c.xre[r]) - k.xCeq[r]);
                if (c.xirrev[r] && v < T(0)) v = T(0);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
#pragma unroll
                  for (int kk = 0; kk < NS; ++kk) dq[q][kk] += k.xnu[q][r][kk] * v;
                  vq[q] += c.xgv[q][r] * (double)v;
                }
              }
              // the links: the population heading into the solid comes back
              // with the net flux of its species
              int nlk[2] = {0, 0};
#pragma unroll
              for (int a = 1; a < 5; ++a) {
                const bool rs = is_rsolid(nt[a]);
                const bool sF = (nt[a] & TB_T) == T_F;
                nlk[0] += rs && !sF ? 1 : 0;
                nlk[1] += rs && sF ? 1 : 0;
#pragma unroll
                for (int kk = 0; kk < NS; ++kk) {
                  // (zero on a link to anything but reactive solid)
                  const T d = rs ? (sF ? dq[1][kk] : dq[0][kk]) : T(0);
                  g[kk][a] += SFORM ? d * k.iJ1[kk] : d;
                }
              }
#pragma unroll
              for (int kk = 0; kk < NS; ++kk)
                l_shet[kk] += (double)nlk[0] * (double)dq[0][kk] + (double)nlk[1] * (double)dq[1][kk];
              const double dv = (double)nlk[0] * vq[0] + (double)nlk[1] * vq[1];
              const bool touched = (nlk[0] > 0 && c.xgrow[0]) || (nlk[1] > 0 && c.xgrow[1]);
              if (touched) {
                // (a fluid node whose neighbour turned solid in the last step
                // may not have its volume loaded ahead)
                const double Vn = (vol_pre(w) ? v_cur : A.V[idx]) + dv;
                vnew = Vn;
                so_v = idx * 8u;
                l_vdv += dv;
                precip = Vn >= 1.0;  // the precipitate fills the node: SOLID_F next step
              }
            }
            storeg = true;
          }
        }
      }

      // ------------------------------------------------------ node status
      uint32_t wout = 0;
      bool dissolved = false;
      T rdis[2] = {T(0), T(0)};  // density given to a dissolved node
      bool r_diss = false, r_strand = false, r_l2g = false, r_g2l = false, r_pre = false;
      double r_v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // mass_inj 1, 2, mass_rem 1, 2, vol_clip
      if (!EXPORT && own) {
        uint32_t tnew = (uint32_t)t;
        if (t == T_FLUID) {
          if (precip) tnew = T_F;
        } else if (t == T_D || t == T_F) {
          // volume of pixel at a reactive solid node (Eq. 33; A2): sum of the
          // fluxes on its D2Q5 links to liquid nodes, in direction then reaction order
          double dv = 0.0;
          bool touched = false;
          const int q = t - T_D;
          if (any_xsolid) {
#pragma unroll
            for (int a = 1; a < 5; ++a) {
              const bool lq = is_liq(nt[a]);
              const bool on = (q ? c.xsolid[1] : c.xsolid[0]) != 0;
              touched = touched | (lq & on);
              const VS nv = L.vs[slot(ey(a))][lane + 1 + ex(a)];
              const double nvq = q ? nv.f : nv.d;
              dv += lq ? nvq : 0.0;
            }
          }
          double Vn = v_cur;  // (loaded ahead)
          if (touched) {
            Vn += dv;
            vnew = Vn;
            so_v = idx * 8u;
            l_vdv += dv;
          }
          if (Vn <= 0.0) {
            int nf = 0;
            T sum0 = T(0), sum1 = T(0);
#pragma unroll
            for (int a = 1; a < 9; ++a) {
              if (!is_fluid(am(a))) continue;
              const int sl = slot(ey(a)), lx = lane + 1 + ex(a);
              sum0 += L.r1[sl][lx];
              sum1 += L.r2[sl][lx];
              ++nf;
            }
            if (nf > 0) {
              // (c) dissolved: fluid from the next step, at rest with the mean
              // density of its fluid neighbours.  Its next status word names
              // no fluid neighbour, so the next pull reads its own slots back
              // (slot opp(a) for direction a: the rest populations are the
              // same in opposite directions).
              const T rb0 = sum0 / T(nf), rb1 = sum1 / T(nf);
              rdis[0] = rb0;
              rdis[1] = rb1;
#pragma unroll
              for (int a = 0; a < 9; ++a) {
                f[0][a] = SFORM ? rb0 : T(w9(a)) * rb0;
                f[1][a] = SFORM ? rb1 : T(w9(a)) * rb1;
              }
              storef = true;
              dissolved = true;
              r_diss = true;
              r_v[0] = (double)rb0;
              r_v[1] = (double)rb1;
              r_v[4] = Vn;
              vnew = 0.0;
              so_v = idx * 8u;
              tnew = T_FLUID;
            }
          }
          if (w & TB_STR) {
            int mm = 0;
#pragma unroll
            for (int b = 1; b < 9; ++b) mm += is_fluid(am(b)) ? 1 : 0;
            if (mm == 0) {
              r_strand = true;
              r_v[2] = (double)m.rho[0];
              r_v[3] = (double)m.rho[1];
            }
          }
        }
        // (b) a node that holds solute but is not liquid now passes its content
        // (and the shares it took) in equal shares, at rest, to its D2Q5
        // neighbours that are liquid now, which take them next step; with no
        // such neighbour it keeps the content at rest in its own slots
        int sfn = liq ? SF_STREAM : SF_NONE;
        if (NS > 0 && !liq && (sf == SF_STREAM || sf == SF_HOLD)) {
          int mm = 0;
#pragma unroll
          for (int b = 1; b < 5; ++b) mm += is_liq(am(b)) ? 1 : 0;
          bool any = false;
#pragma unroll
          for (int kk = 0; kk < NS; ++kk) {
            T cv = m.C[kk];
            if (sf == SF_STREAM) cv += Cin[kk];
            if (mm > 0) cv = cv / T(mm);
            any |= cv != T(0);
#pragma unroll
            for (int a = 0; a < 5; ++a) g[kk][a] = SFORM ? cv : k.J[kk][a] * cv;
          }
          if (any) {
            sfn = mm > 0 ? SF_SHARE : SF_HOLD;
            storeg = true;
          }
        }
        r_l2g = sf == SF_STREAM && !liq && t == T_FLUID;
        r_g2l = liq && sf != SF_STREAM;
        const bool to_f = (t == T_FLUID && tnew == T_F);
        r_pre = to_f;
        // status word of the next step: type, solute state, stranded flag, and
        // which neighbours are fluid / liquid now (the next pull follows them)
        wout = tnew | ((uint32_t)sfn << SF_SHIFT) | (to_f ? TB_STR : 0u);
        if constexpr (REFS) {
          // reference codes of the populations stored now (the node's own
          // density, or the one a dissolved node is given)
          const T d0 = dissolved ? rdis[0] : m.rho[0], d1 = dissolved ? rdis[1] : m.rho[1];
          const uint32_t codes = put_codes(ref_code(d0, k.rb1, SH1, MAX1), ref_code(d1, k.rb2, SH2, MAX2));
          wout |= (fluid || dissolved) ? codes : 0u;
        }
        uint32_t nbf = 0u, nbl = 0u;
#pragma unroll
        for (int b = 1; b < 9; ++b) nbf |= (nt[b] & LF_FLU) << (NBF_SHIFT + b - 1 - 6);
#pragma unroll
        for (int b = 1; b < 5; ++b) nbl |= (nt[b] & LF_LIQN) << (NBL_SHIFT + b - 1 - 5);
        wout |= dissolved ? 0u : (nbf | (liq ? nbl : 0u));
      }
      // the rare balances of this row: wave sums in a fixed order, added by
      // lane 0 (one test for the whole row first: most rows have none)
      if (!EXPORT && __ballot(r_diss | r_strand | r_l2g | r_g2l | r_pre) != 0ull) {
        const unsigned long long bd = __ballot(r_diss), bs = __ballot(r_strand);
        const unsigned long long bl = __ballot(r_l2g), bgl = __ballot(r_g2l), bp = __ballot(r_pre);
        if (bd) {
          const double s0_ = wave_sum_det(r_v[0]), s1_ = wave_sum_det(r_v[1]), s4_ = wave_sum_det(r_v[4]);
          if (lane == 0) {
            L.rare[0] += s0_;
            L.rare[1] += s1_;
            L.rare[4] += s4_;
            L.rare[6] += (double)__popcll(bd);
          }
        }
        if (bs) {
          const double s2_ = wave_sum_det(r_v[2]), s3_ = wave_sum_det(r_v[3]);
          if (lane == 0) {
            L.rare[2] += s2_;
            L.rare[3] += s3_;
          }
        }
        if (lane == 0) {
          if (bp) L.rare[7] += (double)__popcll(bp);
          if (bl) L.rare[8] += (double)__popcll(bl);
          if (bgl) L.rare[9] += (double)__popcll(bgl);
        }
      }

      if (EXPORT) {
        if (own) {
          double* const o = LA.out;
          o[idx] = (double)m.rho[0];
          o[c.plane + idx] = (double)m.rho[1];
          if (!fluid) {
            o[2 * c.plane + idx] = 0.0;
            o[3 * c.plane + idx] = 0.0;
          }
          // the solute each node holds once the shares in transit are
          // delivered (a subtracted species derived from the others there)
          T cv[NSA];
#pragma unroll
          for (int kk = 0; kk < NSA; ++kk) cv[kk] = sf == SF_STREAM ? m.C[kk] + Cin[kk] : (sf == SF_HOLD ? m.C[kk] : T(0));
          if (liq) subtract(cv, m.rho[0]);
#pragma unroll
          for (int kk = 0; kk < NS; ++kk) o[(size_t)(4 + kk) * c.plane + idx] = (double)cv[kk];
          o[(size_t)(4 + NS) * c.plane + idx] = liq ? 1.0 : 0.0;
        }
      } else {
        // -------------------------------------------------- own-slot stores
        // The item's own lanes (columns below nx) write their nodes' slots;
        // the halo lanes' columns belong to the neighbouring items.  Own
        // lanes whose columns share a 128-byte line write all of them when
        // any holds valid populations, so that lines are written whole; a
        // lane without valid populations writes values nobody reads (its
        // slots are not pulled from next step).  Here the values are put in
        // the form they are stored in and the offsets set; the stores follow
        // the row (every lane, every iteration, out of range where nothing
        // is stored).
        so_t = gate(own, (unsigned)X * 4u + (unsigned)R * upitch * 4u);
        wst = wout;
        const unsigned long long bf = __ballot(storef);
        const unsigned long long bg = __ballot(storeg);
        // a 128-byte line holds the flow slots of 128 / PE columns (32 for
        // 16-bit pairs, 16 for FP32, 8 for FP64), the solute slots of
        // 128 / PEG columns; the solute code words, 32 columns.  The lanes
        // whose columns share this lane's line (lanes are columns x0 - 1 ..):
        auto line_lanes = [&](int lg) -> unsigned long long {
          const int lo = ((X >> lg) << lg) - (x0 - 1);
          const int a0 = lo < 0 ? 0 : lo, a1 = lo + (1 << lg) - 1 > SW - 1 ? SW - 1 : lo + (1 << lg) - 1;
          return (~0ull >> (SW - 1 - a1)) & (~0ull << a0);
        };
        constexpr int LGF = __builtin_ctz(128 / PE), LGG = __builtin_ctz(128 / PEG);
        const bool gf = own && (bf & line_lanes(LGF)) != 0ull;
        const bool gg = own && (bg & line_lanes(LGG)) != 0ull;
        const bool gw = own && (bg & line_lanes(5)) != 0ull;
        const unsigned xo = (unsigned)X * PE;
        so_f = gate(gf, xo + (unsigned)R * RSF);
        if constexpr (REFS) {
          // deviation from w_a x the reference of the node that pulls the
          // population next step: the neighbour it heads to if that one is
          // fluid now, else this node (bounce-back; a dissolved node reads
          // all its slots back)
          RF<T> ro;
          if (dissolved) {
            ro.r1 = ref_value(ref_code(rdis[0], k.rb1, SH1, MAX1), k.rb1, SH1);
            ro.r2 = ref_value(ref_code(rdis[1], k.rb2, SH2, MAX2), k.rb2, SH2);
          } else {
            ro = L.rf[s0][lane + 1];
          }
          if constexpr (DEV) {
#pragma unroll
            for (int a = 0; a < 9; ++a) {
              RF<T> rd = ro;
              if (a != 0) {
                const RF<T> rn = L.rf[slot(ey(a))][lane + 1 + ex(a)];
                const bool use = !dissolved && is_fluid(nt[a]);
                rd.r1 = use ? rn.r1 : rd.r1;
                rd.r2 = use ? rn.r2 : rd.r2;
              }
              f[0][a] = __builtin_fmaf(f[0][a], k.sc[0], -(k.wsc[0][wcls(a)] * rd.r1));
              f[1][a] = __builtin_fmaf(f[1][a], k.sc[1], -(k.wsc[1][wcls(a)] * rd.r2));
            }
          } else {
            // FP32: s_a is a deviation from the decoding reference of this
            // step (zero for a dissolved node, which holds rest populations
            // w_a rho); re-referenced to the reader's, an exact difference of
            // two coded values.  The top row's downward populations at a free
            // outlet keep reference zero (they have two readers).
            T o1 = T(0), o2 = T(0);
            if (!dissolved) refs_of(w, o1, o2);
#pragma unroll
            for (int a = 0; a < 9; ++a) {
              RF<T> rd = ro;
              if (a != 0) {
                const RF<T> rn = L.rf[slot(ey(a))][lane + 1 + ex(a)];
                const bool use = !dissolved && is_fluid(nt[a]);
                rd.r1 = use ? rn.r1 : rd.r1;
                rd.r2 = use ? rn.r2 : rd.r2;
              }
              if (top_out && ey(a) < 0) rd = RF<T>{T(0), T(0)};
              f[0][a] += o1 - rd.r1;
              f[1][a] += o2 - rd.r2;
            }
          }
        }
        if constexpr (NS > 0) {
          so_g = gate(gg, (xo << GSH) + (unsigned)R * RSG);
          if constexpr (DEV) {
            // deviation from J_a x the reference concentration of the reader:
            // the liquid neighbour it heads to, else this node
            T co_[NSA];
#pragma unroll
            for (int kk = 0; kk < NSA; ++kk) co_[kk] = L.Cf[kk][s0][lane + 1];
            const bool donor = !liq;  // a node sending shares or keeping content reads its own slots
#pragma unroll
            for (int a = 0; a < 5; ++a) {
              const bool nbr = a != 0 && !donor && is_liq(nt[a]);
#pragma unroll
              for (int kk = 0; kk < NS; ++kk) {
                // (read on every lane and selected: a read under the condition
                // is a branch per direction and species)
                const T cn = a != 0 ? L.Cf[kk][slot(ey(a))][lane + 1 + ex(a)] : co_[kk];
                const T cr = nbr ? cn : co_[kk];
                g[kk][a] = __builtin_fmaf(g[kk][a], k.scg[kk], -(k.Jsc[kk][a == 0 ? 0 : 1] * cr));
              }
            }
            // the node's solute reference codes, for its own pull next step
            so_c = gate(gw, (unsigned)X * 4u + (unsigned)R * ncw * upitch * 4u);
            cws0 = cwc0;
            cws1 = cwc1;
          }
        }
      }
    }

    if constexpr (!EXPORT) {
      // the stores of row R (out of range in the two ring-filling iterations)
      auto cvt = [](T v) -> ST {
        if constexpr (DEV) return dev_out<SM>(v);
        else return v;
      };
      bstore<uint32_t>(wst, wt_, so_t, 0u);
#pragma unroll
      for (int a = 0; a < 9; ++a) bstore2<ST>(cvt(fc[0][a]), cvt(fc[1][a]), wf_, so_f, (unsigned)a * PS);
      if constexpr (NS > 0) {
#pragma unroll
        for (int j = 0; j < NGR; ++j)
#pragma unroll
          for (int a = 0; a < 5; ++a) {
            Grp<ST, SG> q;
#pragma unroll
            for (int i = 0; i < SG; ++i) q.v[i] = j * SG + i < NS ? cvt(gc[j * SG + i][a]) : ST(0);
            bstoreg<ST, SG>(q, wg_, so_g, (unsigned)(j * 5 + a) * PSG);
          }
        if constexpr (DEV) {
          bstore<uint32_t>(cws0, wc_, so_c, 0u);
          if (NS > 4) bstore<uint32_t>(cws1, wc_, so_c, upitch * 4u);
        }
      }
      bstore<double>(vnew, rv, so_v, 0u);
    }

    // next row
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int a = 0; a < 9; ++a) fc[s][a] = fn[s][a];
#pragma unroll
    for (int kk = 0; kk < NSA; ++kk)
#pragma unroll
      for (int a = 0; a < 5; ++a) gc[kk][a] = gn[kk][a];
    mc = mn;
    w_cur = w_next;
    w_next = w_nn;
    v_cur = v_nn;
    const int s_old = sm;
    sm = s0;
    s0 = sp;
    sp = s_old;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  if (EXPORT) return;

  // ---------------------------------------------------------- item balances
  // Wave sums in FP64 in a fixed order (lane 0's butterfly), added to this
  // item's FP64 record (the item is this wavefront's alone, so plain
  // read-modify-write).
  const T wm = wave_max_t(my_rmax);
  const double vg = __ballot(l_msrc != 0.0) ? wave_sum_det(l_msrc) : 0.0;
  const double vd = __ballot(l_vdv != 0.0) ? wave_sum_det(l_vdv) : 0.0;
  double vs[NSA], vh[NSA];
#pragma unroll
  for (int kk = 0; kk < NSA; ++kk) {
    vs[kk] = __ballot(l_ssrc[kk] != 0.0) ? wave_sum_det(l_ssrc[kk]) : 0.0;
    vh[kk] = __ballot(l_shet[kk] != 0.0) ? wave_sum_det(l_shet[kk]) : 0.0;
  }
  double* Lg = A.led + (size_t)item * NLED;
  if (lane == 0) {
    const double md = (double)wm;
    unsigned long long* part = &A.rmax[slot_cur * RM_SLOT + xcd * RM_STRIDE];
    const unsigned long long mb = (unsigned long long)__double_as_longlong(md);
    // the partial only grows during a step, so a value already at least as
    // large makes this wavefront's atomic unnecessary
    const unsigned long long seen = __hip_atomic_load(part, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (md > 0.0 && mb > seen) atomicMax(part, mb);
    if (item == 0)
      for (int xc = 0; xc < 8; ++xc) A.rmax[slot_next * RM_SLOT + xc * RM_STRIDE] = 0ull;
    if (vg != 0.0) {
      Lg[L_MSRC] += -vg;
      Lg[L_MSRC + 1] += vg;
    }
    if (vd != 0.0) Lg[L_VDV] += vd;
#pragma unroll
    for (int kk = 0; kk < NS; ++kk) {
      if (vs[kk] != 0.0) Lg[L_SSRC + kk] += vs[kk];
      if (vh[kk] != 0.0) Lg[L_SHET + kk] += vh[kk];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (lane < NRARE_SLOTS) {
    const double s = L.rare[lane];
    if (s != 0.0) Lg[rare_dst(lane)] += s;
  }
}

// ---------------------------------------------------------------- ledger sum
// Fixed-order sum of the per-item balance records: one workgroup per ledger
// field; thread t adds items t, t + 256, ... in order, then a fixed tree adds
// the 256 partial sums (the same result on every call).
constexpr int LSUM_THREADS = 256;
__global__ __launch_bounds__(LSUM_THREADS) void k_ledger_sum(const double* led, int nitems, double* out) {
  __shared__ double part[LSUM_THREADS];
  const int f = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int b = t; b < nitems; b += LSUM_THREADS) s += led[(long long)b * NLED + f];
  part[t] = s;
  __syncthreads();
  for (int h = LSUM_THREADS / 2; h > 0; h >>= 1) {
    if (t < h) part[t] += part[t + h];
    __syncthreads();
  }
  if (t == 0) out[f] = part[0];
}

// ---------------------------------------------------------------- host side
constexpr int SEG_ROWS = 16;      // default rows per item (LBRX_SEG_ROWS overrides, 1..HMAX)
constexpr int SEG_ROWS_F64 = 16;  // FP64 storage (one wavefront per SIMD): taller items
// Rows per item when the caller names none: SEG_ROWS, halved (down to 2) while
// the lattice has fewer items than the device holds wavefronts at once (2 per
// SIMD on 256 CUs, 1 with FP64 storage).  A lattice that does not fill the
// device takes as long per step as one item's march down its rows, so shorter
// items finish sooner even though each pulls two ring rows more per H rows.
int default_seg_rows(int nx, int ny, int precision) {
  const bool f64 = precision == LBRX_F64;
  const long long slots = f64 ? 1024 : 2048;
  const long long strips = (nx + IW - 1) / IW;
  int h = f64 ? SEG_ROWS_F64 : SEG_ROWS;
  while (h > 2 && strips * ((ny + h - 1) / h) < slots) h /= 2;
  return h;
}
// Steps per captured HIP graph of launches: a multiple of 6, the period of
// the step phases (buffer parity and rho_max slot), so that one graph serves
// every replay that starts at a step count divisible by 6.
constexpr int GRAPH_LEN = 30;

template <typename T> using KFnT = void (*)(const LaunchArgs);

template <typename T, int SM, bool EXPORT>
KFnT<T> pick(int ns) {
  switch (ns) {
    case 0: return k_step<T, SM, 0, EXPORT>;
    case 1: return k_step<T, SM, 1, EXPORT>;
    case 2: return k_step<T, SM, 2, EXPORT>;
    case 3: return k_step<T, SM, 3, EXPORT>;
    case 4: return k_step<T, SM, 4, EXPORT>;
    case 5: return k_step<T, SM, 5, EXPORT>;
    case 6: return k_step<T, SM, 6, EXPORT>;
    case 7: return k_step<T, SM, 7, EXPORT>;
    default: return k_step<T, SM, 8, EXPORT>;
  }
}

int storage_mode(int precision) {
  return precision == LBRX_F16DEV ? SM_F16 : precision == LBRX_BF16DEV ? SM_BF16 : SM_PLAIN;
}
size_t storage_bytes(int precision) {
  return precision == LBRX_F64 ? 8 : precision == LBRX_F32 ? 4 : 2;
}

thread_local std::string g_create_err;

}  // namespace

struct lbrx_ctx {
  KConst c{};
  int precision = LBRX_F64;
  size_t esz = 8;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  void* f[2] = {nullptr, nullptr};
  void* g[2] = {nullptr, nullptr};
  uint32_t* t[2] = {nullptr, nullptr};
  uint32_t* cw[2] = {nullptr, nullptr};  // solute reference codes (16-bit storage)
  double* V = nullptr;
  unsigned long long* rmax = nullptr;
  double* led = nullptr;
  double* ledsum = nullptr;
  unsigned int* err = nullptr;
  double* out = nullptr;  // read-out staging (read_out_doubles), allocated by the first lbrx_fields
  void* dargs = nullptr;  // this simulation's KArgs in device memory
  int cur = 0;
  int64_t steps = 0;
  bool failed = false;
  std::string msg;
  KT<double> kd{};
  KT<float> kf{};
  KFnT<double> step64 = nullptr, export64 = nullptr;
  KFnT<float> step32 = nullptr, export32 = nullptr;
  void* (*dev_alloc)(uint64_t, void*) = nullptr;  // caller's device allocator (else hipMalloc)
  void (*dev_free)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
  hipGraph_t graph = nullptr;  // GRAPH_LEN single launches, captured on first use
  hipGraphExec_t gexec = nullptr;
};

namespace {

// Device memory of a context: the caller's allocator when one was given, else
// hipMalloc / hipFree.  A zero-byte request yields a null pointer.
bool ctx_alloc(lbrx_ctx* x, void** p, size_t n) {
  *p = nullptr;
  if (n == 0) return true;
  if (x->dev_alloc) {
    *p = x->dev_alloc((uint64_t)n, x->alloc_user);
    return *p != nullptr;
  }
  return hipMalloc(p, n) == hipSuccess;
}
void ctx_free(lbrx_ctx* x, void* p) {
  if (!p) return;
  if (x->dev_free) x->dev_free(p, x->alloc_user);
  else (void)hipFree(p);
}

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
  if (p->periodic & ~7u) return "unknown bits in periodic";
  if ((p->periodic & 4u) && ((p->periodic & 2u) || p->ny < 2)) return "a free outlet needs walls in y and ny >= 2";
  // A 16-bit population is a deviation from the reference of the one node
  // that pulls it; beyond the outlet the top row's downward populations have
  // two readers (the row below, and the top row through the ghost row).
  if ((p->periodic & 4u) && (p->precision == LBRX_F16DEV || p->precision == LBRX_BF16DEV))
    return "a free outlet needs FP64 or FP32 storage";
  if (p->seg_rows < 0 || p->seg_rows > HMAX) return "seg_rows must lie in 0..30";
  if ((long long)p->nx * p->ny > (1ll << 31) - 1) return "lattice too large";
  if (p->precision != LBRX_F64 && p->precision != LBRX_F32 && p->precision != LBRX_F16DEV &&
      p->precision != LBRX_BF16DEV)
    return "unknown precision";
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
    if (h.surface & ~((1u << LBRX_SOLID_INERT) | (1u << LBRX_SOLID_D) | (1u << LBRX_SOLID_F)))
      return "a homogeneous reaction's surface may only name solid types";
    if (h.surface && !(h.surface_factor > 0.0 && h.surface_factor < 1e300))
      return "surface_factor must be positive and finite";
  }
  if (!(p->psi_prefactor >= 0.0 && p->psi_prefactor < 1e300)) return "psi_prefactor must be 0 (default) or positive";
  if (p->subtract_species < -1 || p->subtract_species >= p->n_species) return "subtract_species must be -1 or a species index";
  if (p->subtract_species >= 0 && !(p->subtract_total > 0.0 && p->subtract_total < 1e300))
    return "subtract_total must be > 0 when a species is subtracted";
  if (!p->dev_alloc != !p->dev_free) return "dev_alloc and dev_free must be given together";
  for (int r = 0; r < p->n_het; ++r) {
    const lbrx_het_rxn& h = p->het[r];
    if (h.reactant < 0 || h.reactant >= ns || h.product < -1 || h.product >= ns) return "species index out of range";
    if (h.mode < 0 || h.mode > 2) return "unknown heterogeneous mode";
    if (h.surface & ~((1u << LBRX_SOLID_D) | (1u << LBRX_SOLID_F))) return "surface may only name SOLID_D / SOLID_F";
    if (!(h.k >= 0.0)) return "rate constants must be >= 0";
  }
  if (!p->node_type || !p->rho1 || !p->rho2) return "node_type, rho1 and rho2 are required";
  {
    // the kernels address each population array with 32-bit byte offsets
    const unsigned long long pitch = ((unsigned long long)p->nx + 63) / 64 * 64;
    const unsigned long long esz = storage_bytes(p->precision);
    // elements per node: 9 flow pairs; 5 slots per species group
    const unsigned long long sg = (unsigned long long)species_group(p->n_species, (int)esz);
    const unsigned long long ge = 5ull * ((p->n_species + sg - 1) / sg) * sg;
    const unsigned long long np = 18ull > ge ? 18ull : ge;
    if (np * pitch * (unsigned long long)p->ny * esz >= (unsigned long long)OOB_OFF)
      return "lattice too large: a population array must stay below 4 GiB (use FP32 or fewer species)";
  }
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

// Element index of the slot layout: row-interleaved planes of slots.  Flow:
// plane a of row y holds (component 1, component 2) of direction a; solute:
// plane 5j + a holds species sg j .. sg j + sg - 1 of direction a (sg from
// species_group: 4 or 2).
inline long long fslot(const KConst& c, int y, int a, int x, int s) {
  return (((long long)y * 9 + a) * c.pitch + x) * 2 + s;
}
inline int n_groups(const KConst& c) { return (c.ns + c.sg - 1) / c.sg; }
inline long long gslot(const KConst& c, int y, int k, int a, int x) {
  return (((long long)y * 5 * n_groups(c) + (k / c.sg) * 5 + a) * c.pitch + x) * c.sg + (k % c.sg);
}
size_t f_elems(const KConst& c) { return (size_t)18 * c.plane; }
size_t g_elems(const KConst& c) { return (size_t)5 * n_groups(c) * c.sg * c.plane + c.sg; }

template <typename T>
void fill_populations(const lbrx_params* p, const KConst& c, const std::vector<uint32_t>& tb,
                      std::vector<T>& f, std::vector<T>& g) {
  const int nx = p->nx, ny = p->ny, ns = p->n_species;
  f.assign(f_elems(c), T(0));
  g.assign(g_elems(c), T(0));
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const long long i = (long long)y * nx + x, d = (long long)y * c.pitch + x;
      if ((tb[d] & TB_T) != T_FLUID) continue;
      for (int a = 0; a < 9; ++a) {
        f[fslot(c, y, a, x, 0)] = T(w9(a) * p->rho1[i]);
        f[fslot(c, y, a, x, 1)] = T(w9(a) * p->rho2[i]);
      }
      if (sf_of(tb[d]) == SF_STREAM)
        for (int k = 0; k < ns; ++k)
          for (int a = 0; a < 5; ++a) g[gslot(c, y, k, a, x)] = T(c.J[k][a] * p->C0[(long long)k * nx * ny + i]);
    }
}

// FP32 storage: the rest equilibria of Eq. 8 and 21 as the kernels keep them.
// A flow slot holds f_a / w_a - R = rho - R, R the reference density coded in
// the node's status word (every node reads its own slots at step 0); at a
// free outlet the top row's downward slots keep reference zero (they have two
// readers).  A solute slot holds g_a / J'_a = C.
void fill_sform_populations(const lbrx_params* p, const KConst& c, const KT<float>& k, std::vector<uint32_t>& tb,
                            std::vector<float>& f, std::vector<float>& g) {
  const int nx = p->nx, ny = p->ny, ns = p->n_species;
  const bool outlet = c.per_y == 2;
  f.assign(f_elems(c), 0.0f);
  g.assign(g_elems(c), 0.0f);
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const long long i = (long long)y * nx + x, d = (long long)y * c.pitch + x;
      if ((tb[d] & TB_T) != T_FLUID) continue;
      const double r[2] = {p->rho1[i], p->rho2[i]};
      const uint32_t c1 = ref_code((float)r[0], k.rb1, SH1, MAX1), c2 = ref_code((float)r[1], k.rb2, SH2, MAX2);
      tb[d] |= put_codes(c1, c2);
      const double ref[2] = {(double)ref_value(c1, k.rb1, SH1), (double)ref_value(c2, k.rb2, SH2)};
      for (int s = 0; s < 2; ++s)
        for (int a = 0; a < 9; ++a) {
          const bool zref = outlet && y == ny - 1 && ey(a) < 0;
          f[fslot(c, y, a, x, s)] = (float)(zref ? r[s] : r[s] - ref[s]);
        }
      if (sf_of(tb[d]) == SF_STREAM)
        for (int q = 0; q < ns; ++q)
          for (int a = 0; a < 5; ++a) g[gslot(c, y, q, a, x)] = (float)p->C0[(long long)q * nx * ny + i];
    }
}

// 16-bit storage: the deviation scales are powers of two such that a stored
// deviation stays far below the FP16 maximum even if every population of a
// node held six times the largest initial density (or concentration sum);
// the reference codes cover sixteen binades from an eighth of the smallest
// initial density (2^-14 of the concentration sum) upward.
double pow2_scale(double vmax) {
  if (!(vmax > 0.0)) vmax = 1.0;
  int e = (int)std::floor(std::log2(65504.0 / (6.0 * vmax)));
  e = e < -60 ? -60 : (e > 60 ? 60 : e);
  return std::ldexp(1.0, e);
}
uint32_t code_base(double v, int sh) {
  const float f = (float)(v > 1e-30 ? v : 1e-30);
  return __builtin_bit_cast(uint32_t, f) >> sh;
}

// Bases of the flow reference codes (FP32 and 16-bit storage): sixteen
// binades upward from an eighth of the smallest initial density.
void fill_ref_bases(KT<float>& k, const lbrx_params* p) {
  const long long N = (long long)p->nx * p->ny;
  double mx[2] = {0.0, 0.0}, mn[2] = {1e300, 1e300};
  for (long long i = 0; i < N; ++i) {
    if (p->node_type[i] != LBRX_FLUID) continue;
    const double r[2] = {p->rho1[i], p->rho2[i]};
    for (int s = 0; s < 2; ++s) {
      mx[s] = std::max(mx[s], r[s]);
      if (r[s] > 0.0) mn[s] = std::min(mn[s], r[s]);
    }
  }
  k.rb1 = code_base((mn[0] < 1e300 ? mn[0] : 1.0) / 8.0, SH1);
  k.rb2 = code_base(std::max(mn[1] < 1e300 ? mn[1] : 0.0, 1e-3 * mx[1]) / 8.0, SH2);
}

void fill_dev_constants(KT<float>& k, const lbrx_params* p, const KConst& c) {
  const long long N = (long long)p->nx * p->ny;
  double mx[2] = {0.0, 0.0}, mn[2] = {1e300, 1e300};
  for (long long i = 0; i < N; ++i) {
    if (p->node_type[i] != LBRX_FLUID) continue;
    const double r[2] = {p->rho1[i], p->rho2[i]};
    for (int s = 0; s < 2; ++s) {
      mx[s] = std::max(mx[s], r[s]);
      if (r[s] > 0.0) mn[s] = std::min(mn[s], r[s]);
    }
  }
  double csum = 0.0;
  for (int q = 0; q < c.ns; ++q) {
    double m = 0.0;
    for (long long i = 0; i < N; ++i) m = std::max(m, p->C0[(long long)q * N + i]);
    csum += m;
  }
  if (!(csum > 0.0)) csum = 1.0;
  const double wv[3] = {4.0 / 9, 1.0 / 9, 1.0 / 36};
  for (int s = 0; s < 2; ++s) {
    const double sc = pow2_scale(mx[s]);
    k.sc[s] = (float)sc;
    k.isc[s] = (float)(1.0 / sc);
    for (int q = 0; q < 3; ++q) k.wsc[s][q] = (float)(wv[q] * sc);
  }
  for (int q = 0; q < 3; ++q) k.wc[q] = (float)wv[q];
  const double scg = pow2_scale(csum);
  for (int q = 0; q < LBRX_MAX_SPECIES; ++q) {
    k.scg[q] = (float)scg;
    k.iscg[q] = (float)(1.0 / scg);
    const double J0 = q < c.ns ? c.J[q][0] : 0.0, J1 = q < c.ns ? c.J[q][1] : 0.0;
    k.Jc[q][0] = (float)J0;
    k.Jc[q][1] = (float)J1;
    k.Jsc[q][0] = (float)(J0 * scg);
    k.Jsc[q][1] = (float)(J1 * scg);
    k.rbc[q] = code_base(csum * std::ldexp(1.0, -14), SHC);
  }
}

uint16_t dev_store_host(float v, int sm) {
  if (sm == SM_F16) return __builtin_bit_cast(uint16_t, (_Float16)v);
  // BF16, round to nearest even (finite values)
  uint32_t u = __builtin_bit_cast(uint32_t, v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Initial state in 16-bit form: the rest equilibria of Eq. 8 and 21 as
// deviations from the references coded in the status and solute words (every
// node reads its own slots at step 0).
void fill_dev_populations(const lbrx_params* p, const KConst& c, const KT<float>& k, int sm,
                          std::vector<uint32_t>& tb, std::vector<uint16_t>& f, std::vector<uint16_t>& g,
                          std::vector<uint32_t>& cw) {
  const int nx = p->nx, ny = p->ny, ns = p->n_species;
  const long long plane = c.plane;
  f.assign(f_elems(c), 0);
  g.assign(g_elems(c), 0);
  cw.assign((size_t)(c.ncw > 0 ? c.ncw : 0) * plane, 0u);
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const long long i = (long long)y * nx + x, d = (long long)y * c.pitch + x;
      if ((tb[d] & TB_T) != T_FLUID) continue;
      const float r[2] = {(float)p->rho1[i], (float)p->rho2[i]};
      const uint32_t c1 = ref_code(r[0], k.rb1, SH1, MAX1), c2 = ref_code(r[1], k.rb2, SH2, MAX2);
      tb[d] |= put_codes(c1, c2);
      const float ref[2] = {ref_value(c1, k.rb1, SH1), ref_value(c2, k.rb2, SH2)};
      for (int s = 0; s < 2; ++s)
        for (int a = 0; a < 9; ++a) {
          const float f0 = (float)(w9(a) * (s == 0 ? p->rho1[i] : p->rho2[i]));
          f[fslot(c, y, a, x, s)] = dev_store_host(std::fma(f0, k.sc[s], -(k.wsc[s][wcls(a)] * ref[s])), sm);
        }
      if (sf_of(tb[d]) == SF_STREAM && ns > 0) {
        for (int q = 0; q < ns; ++q) {
          const float C = (float)p->C0[(long long)q * nx * ny + i];
          const uint32_t cc = ref_code(C, k.rbc[q], SHC, MAXC);
          cw[(size_t)((long long)y * c.ncw + (q >> 2)) * c.pitch + x] |= cc << (8 * (q & 3));
          const float cr = ref_value(cc, k.rbc[q], SHC);
          for (int a = 0; a < 5; ++a) {
            const float g0 = (float)(c.J[q][a] * p->C0[(long long)q * nx * ny + i]);
            g[gslot(c, y, q, a, x)] = dev_store_host(std::fma(g0, k.scg[q], -(k.Jsc[q][a == 0 ? 0 : 1] * cr)), sm);
          }
        }
      }
    }
}

template <typename T>
void make_args(const lbrx_ctx* x, KArgs<T>& A, const KT<T>& kt) {
  A.c = x->c;
  A.k = kt;
  for (int i = 0; i < 2; ++i) {
    A.f[i] = x->f[i];
    A.g[i] = x->g[i];
    A.t[i] = x->t[i];
    A.cw[i] = x->cw[i];
  }
  A.V = x->V;
  A.rmax = x->rmax;
  A.led = x->led;
  A.err = x->err;
}

// (re)writes the simulation's device-resident KArgs (synchronous copy)
hipError_t upload_args(lbrx_ctx* x) {
  if (x->precision == LBRX_F64) {
    KArgs<double> A{};
    make_args(x, A, x->kd);
    return hipMemcpy(x->dargs, &A, sizeof A, hipMemcpyHostToDevice);
  }
  KArgs<float> A{};
  make_args(x, A, x->kf);
  return hipMemcpy(x->dargs, &A, sizeof A, hipMemcpyHostToDevice);
}

size_t args_bytes(int precision) { return precision == LBRX_F64 ? sizeof(KArgs<double>) : sizeof(KArgs<float>); }

void launch_one(lbrx_ctx* x, bool exporting, double* out = nullptr) {
  LaunchArgs L{};
  L.single = x->dargs;
  L.ninst = 0;
  L.phase0 = (int)(x->steps % 6);
  L.out = out;
  const dim3 grid(x->c.nblocks), block(64, WPB);
  if (x->precision == LBRX_F64)
    hipLaunchKernelGGL(exporting ? x->export64 : x->step64, grid, block, 0, x->stream, L);
  else
    hipLaunchKernelGGL(exporting ? x->export32 : x->step32, grid, block, 0, x->stream, L);
}

lbrx_status launch_step(lbrx_ctx* x) {
  launch_one(x, false);
  HIPCHK(x, hipGetLastError());
  x->steps += 1;
  x->cur = (int)(x->steps & 1);
  return LBRX_OK;
}

template <typename T>
void fill_kt(KT<T>& k, const lbrx_params* p, const KConst& c, const double* D) {
  for (int s = 0; s < 2; ++s) {
    k.om[s] = (T)c.om[s];
    k.tau[s] = (T)p->tau[s];
    k.r_tau[s] = (T)(1.0 / p->tau[s]);
  }
  k.RT = (T)c.RT;
  k.a = (T)c.a;
  k.b = (T)c.b;
  k.G11 = (T)c.G11;
  k.r_G11 = (T)(c.G11 != 0.0 ? 1.0 / c.G11 : 0.0);
  k.psi_pre = (T)c.psi_pre;
  k.G12 = (T)c.G12;
  k.G21 = (T)c.G21;
  k.w1 = (T)c.w1;
  k.w2 = (T)c.w2;
  k.gx = (T)c.gx;
  k.gy = (T)c.gy;
  k.a0 = (T)c.a0;
  k.rho10 = (T)c.rho10;
  k.r_rho10 = (T)(c.rho10 > 0.0 ? 1.0 / c.rho10 : 0.0);
  k.rho20 = (T)c.rho20;
  k.sub_tot = (T)c.sub_tot;
  k.r_rho20 = (T)(c.rho20 > 0.0 ? 1.0 / c.rho20 : 0.0);
  for (int q = 0; q < LBRX_MAX_SPECIES; ++q) {
    k.omg[q] = (T)c.omg[q];
    for (int a = 0; a < 5; ++a) k.J[q][a] = (T)c.J[q][a];
    // J1' = J1 rounded to a multiple of 2^-26, J0' = 1 - 4 J1' (both exact in
    // FP32, so that they sum to one); used by FP32 storage only
    const double j1 = q < c.ns ? std::nearbyint(c.J[q][1] * 67108864.0) / 67108864.0 : 0.25;
    k.Jp1[q] = (T)j1;
    k.Jp0[q] = (T)(1.0 - 4.0 * j1);
    k.hJ[q] = (T)(j1 > 0.0 ? 0.5 / j1 : 0.0);
    k.iJ1[q] = (T)(j1 > 0.0 ? 1.0 / j1 : 0.0);
  }
  for (int r = 0; r < LBRX_MAX_RXN; ++r) {
    k.hk[r] = (T)c.hk[r];
    k.hks[r] = (T)c.hks[r];
    k.hKeq[r] = (T)c.hKeq[r];
    k.r_hKeq[r] = (T)(c.hKeq[r] != 0.0 ? 1.0 / c.hKeq[r] : 0.0);
    k.hMgas[r] = (T)c.hMgas[r];
    k.r_hMgas[r] = (T)(c.hMgas[r] != 0.0 ? 1.0 / c.hMgas[r] : 0.0);
    k.xkap[r] = (T)c.xkap[r];
    k.xCeq[r] = (T)c.xCeq[r];
    for (int q = 0; q < LBRX_MAX_SPECIES; ++q) k.hnu[r][q] = T(0);
    if (r < c.nhom) {
      // reactants consumed, products formed (Eq. 27)
      if (c.hre0[r] >= 0) k.hnu[r][c.hre0[r]] -= T(1);
      if (c.hre1[r] >= 0) k.hnu[r][c.hre1[r]] -= T(1);
      if (c.hpr0[r] >= 0) k.hnu[r][c.hpr0[r]] += T(1);
      if (c.hpr1[r] >= 0) k.hnu[r][c.hpr1[r]] += T(1);
    }
    for (int q = 0; q < 2; ++q) {
      for (int sp = 0; sp < LBRX_MAX_SPECIES; ++sp) k.xnu[q][r][sp] = T(0);
      if (r < c.nhet && (c.xsurf[r] & (1 << (T_D + q)))) {
        k.xnu[q][r][c.xre[r]] -= T(1);
        if (c.xpr[r] >= 0) k.xnu[q][r][c.xpr[r]] += T(1);
      }
    }
  }
  (void)D;
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
  x->dev_alloc = p->dev_alloc;
  x->dev_free = p->dev_free;
  x->alloc_user = p->alloc_user;
  KConst& c = x->c;
  c.nx = p->nx;
  c.ny = p->ny;
  c.pitch = (p->nx + 63) / 64 * 64;
  c.per_x = (p->periodic & 1u) ? 1 : 0;
  c.per_y = (p->periodic & 2u) ? 1 : ((p->periodic & 4u) ? 2 : 0);
  c.plane = (long long)c.pitch * p->ny;
  c.ns = p->n_species;
  x->precision = p->precision;
  x->esz = storage_bytes(p->precision);
  c.sg = species_group(c.ns, (int)x->esz);
  c.seg_rows = p->seg_rows > 0 ? p->seg_rows : default_seg_rows(p->nx, p->ny, p->precision);
  if (const char* e = getenv("LBRX_SEG_ROWS")) {
    const int v = atoi(e);
    if (v >= 1 && v <= HMAX) c.seg_rows = v;
  }
  c.strips = (c.nx + IW - 1) / IW;
  c.nitems = c.strips * ((p->ny + c.seg_rows - 1) / c.seg_rows);
  c.nblocks = (c.nitems + WPB - 1) / WPB;
  // byte sizes of the population and status arrays (below 4 GiB, checked in validate)
  c.fbytes = (unsigned)(f_elems(c) * x->esz);
  c.gbytes = (unsigned)(g_elems(c) * x->esz);
  c.tbytes = (unsigned)((unsigned long long)c.plane * 4ull);
  const int sm = storage_mode(p->precision);
  c.ncw = (sm_dev(sm) && c.ns > 0) ? (c.ns + 3) / 4 : 0;
  c.cbytes = (unsigned)((unsigned long long)(c.ncw > 0 ? c.ncw : 1) * c.plane * 4ull);
  for (int s = 0; s < 2; ++s) {
    c.tau[s] = p->tau[s];
    c.om[s] = 1.0 / p->tau[s];
  }
  c.RT = p->R * p->T;
  c.a = p->a;
  c.b = p->b;
  c.G11 = p->G11;
  c.rG11 = p->G11 != 0.0 ? 1.0 / p->G11 : 0.0;
  c.psi_pre = p->psi_prefactor > 0.0 ? p->psi_prefactor : 2.0;
  c.sub = p->subtract_species;
  c.sub_tot = p->subtract_species >= 0 ? p->subtract_total : 0.0;
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
    c.hsurf[r] = (int)p->hom[r].surface;
    c.hks[r] = p->hom[r].surface ? p->hom[r].k * p->hom[r].surface_factor : p->hom[r].k;
    c.any_hsurf |= c.hsurf[r] != 0;
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
    for (int q = 0; q < 2; ++q) {
      const bool on = (h.surface & (1u << (T_D + q))) != 0;
      c.xgv[q][r] = on && h.mode == HET_GROWS ? h.molar_volume : 0.0;
      c.xsv[q][r] = !on ? 0.0 : h.mode == HET_CONSUMES ? -h.molar_volume : h.mode == HET_MINERAL ? h.molar_volume : 0.0;
      c.xgrow[q] |= on && h.mode == HET_GROWS;
      c.xsolid[q] |= on && (h.mode == HET_CONSUMES || h.mode == HET_MINERAL);
    }
  }
  fill_kt(x->kd, p, c, D);
  fill_kt(x->kf, p, c, D);
  fill_ref_bases(x->kf, p);
  if (sm_dev(sm)) fill_dev_constants(x->kf, p, c);
  const bool outlet = c.per_y == 2;  // free outlet: the SM_OUT kernels (plain storage only)
  x->step64 = outlet ? pick<double, SM_OUT, false>(c.ns) : pick<double, SM_PLAIN, false>(c.ns);
  x->export64 = outlet ? pick<double, SM_OUT, true>(c.ns) : pick<double, SM_PLAIN, true>(c.ns);
  x->step32 = sm == SM_F16 ? pick<float, SM_F16, false>(c.ns)
             : sm == SM_BF16 ? pick<float, SM_BF16, false>(c.ns)
             : outlet ? pick<float, SM_OUT, false>(c.ns) : pick<float, SM_PLAIN, false>(c.ns);
  x->export32 = sm == SM_F16 ? pick<float, SM_F16, true>(c.ns)
               : sm == SM_BF16 ? pick<float, SM_BF16, true>(c.ns)
               : outlet ? pick<float, SM_OUT, true>(c.ns) : pick<float, SM_PLAIN, true>(c.ns);

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
  const size_t fbytes = f_elems(c) * x->esz, gbytes = g_elems(c) * x->esz;
  for (int i = 0; i < 2; ++i) {
    if (!ctx_alloc(x, &x->f[i], fbytes) || !ctx_alloc(x, &x->g[i], gbytes) ||
        !ctx_alloc(x, (void**)&x->t[i], plane * 4) || !ctx_alloc(x, (void**)&x->cw[i], c.cbytes))
      return fail(LBRX_E_NOMEM, "device allocation of the populations failed");
  }
  if (!ctx_alloc(x, (void**)&x->V, plane * 8) || !ctx_alloc(x, (void**)&x->rmax, RM_WORDS * 8) ||
      !ctx_alloc(x, (void**)&x->led, (size_t)c.nitems * NLED * 8) || !ctx_alloc(x, (void**)&x->ledsum, NLED * 8) ||
      !ctx_alloc(x, (void**)&x->err, 2 * 4))
    return fail(LBRX_E_NOMEM, "device allocation of the state failed");

  // initial state (host staging, then one copy each)
  const int nx = p->nx, ny = p->ny;
  double rmax0 = 0.0;
  for (long long i = 0; i < (long long)nx * ny; ++i)
    if (p->node_type[i] == LBRX_FLUID && p->rho1[i] > rmax0) rmax0 = p->rho1[i];
  const double thr0 = p->liquid_frac * rmax0;
  std::vector<uint32_t> tb(plane, (uint32_t)T_INERT);
  std::vector<double> V(plane, 0.0);
  for (int y = 0; y < ny; ++y)
    for (int xx = 0; xx < nx; ++xx) {
      const long long i = (long long)y * nx + xx, d = (long long)y * c.pitch + xx;
      const uint8_t t = p->node_type[i];
      uint32_t b = t;
      // step 0: no neighbour bits, so every node reads its own slots, which
      // hold f(0) (and g(0) at liquid nodes)
      if (t == LBRX_FLUID && p->rho1[i] > thr0) b |= (uint32_t)SF_STREAM << SF_SHIFT;
      tb[d] = b;
      V[d] = p->V0 ? p->V0[i] : ((t == LBRX_SOLID_D || t == LBRX_SOLID_F) ? 1.0 : 0.0);
    }
  hipError_t e = hipSuccess;
  if (p->precision == LBRX_F64) {
    std::vector<double> f, g;
    fill_populations<double>(p, c, tb, f, g);
    e = hipMemcpy(x->f[0], f.data(), fbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(x->g[0], g.data(), gbytes, hipMemcpyHostToDevice);
  } else if (sm == SM_PLAIN) {
    std::vector<float> f, g;
    fill_sform_populations(p, c, x->kf, tb, f, g);
    e = hipMemcpy(x->f[0], f.data(), fbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(x->g[0], g.data(), gbytes, hipMemcpyHostToDevice);
  } else {
    std::vector<uint16_t> f, g;
    std::vector<uint32_t> cw;
    fill_dev_populations(p, c, x->kf, sm, tb, f, g, cw);
    e = hipMemcpy(x->f[0], f.data(), fbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(x->g[0], g.data(), gbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && !cw.empty()) e = hipMemcpy(x->cw[0], cw.data(), cw.size() * 4, hipMemcpyHostToDevice);
  }
  // the second buffers start as copies so that never-written slots hold defined values
  if (e == hipSuccess) e = hipMemcpy(x->f[1], x->f[0], fbytes, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->g[1], x->g[0], gbytes, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->t[0], tb.data(), plane * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->t[1], tb.data(), plane * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->V, V.data(), plane * 8, hipMemcpyHostToDevice);
  std::vector<unsigned long long> rm(RM_WORDS, 0ull);
  std::memcpy(&rm[2 * RM_SLOT], &rmax0, 8);  // the "previous step" of step 0
  if (e == hipSuccess) e = hipMemcpy(x->rmax, rm.data(), RM_WORDS * 8, hipMemcpyHostToDevice);
  unsigned int er[2] = {0u, 0xffffffffu};
  if (e == hipSuccess) e = hipMemcpy(x->err, er, sizeof er, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(x->led, 0, (size_t)c.nitems * NLED * 8);
  if (e == hipSuccess && !ctx_alloc(x, &x->dargs, args_bytes(x->precision)))
    return fail(LBRX_E_NOMEM, "device allocation of the kernel arguments failed");
  if (e == hipSuccess) e = upload_args(x);
  if (e != hipSuccess) return fail(LBRX_E_DEVICE, std::string("initial copy failed: ") + hipGetErrorString(e));
  *out = x;
  return LBRX_OK;
}

lbrx_status lbrx_step(lbrx_ctx* x, int64_t n) {
  if (!x) return LBRX_E_INVAL;
  if (x->failed) return set_err(x, LBRX_E_STATE, "context failed earlier: " + x->msg);
  if (n < 0) return set_err(x, LBRX_E_INVAL, "n_steps must be >= 0");
  HIPCHK(x, hipSetDevice(x->device));
  // a stream the caller is capturing gets plain launches (they become part
  // of the caller's graph)
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIPCHK(x, hipStreamIsCapturing(x->stream, &cap));
  const bool graphs = cap == hipStreamCaptureStatusNone;
  int64_t done = 0;
  while (done < n) {
    // runs of GRAPH_LEN steps starting at a step count divisible by 6 (the
    // period of the step phases) replay one captured graph of single launches
    if (graphs && x->steps % 6 == 0 && n - done >= GRAPH_LEN) {
      if (!x->gexec) {
        const int64_t s0 = x->steps;
        HIPCHK(x, hipStreamBeginCapture(x->stream, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < GRAPH_LEN; ++i) {
          launch_one(x, false);
          x->steps += 1;
        }
        x->steps = s0;
        const hipError_t le = hipGetLastError();  // a launch refused while capturing
        const hipError_t e = hipStreamEndCapture(x->stream, &x->graph);
        if (le != hipSuccess || e != hipSuccess ||
            hipGraphInstantiate(&x->gexec, x->graph, nullptr, nullptr, 0) != hipSuccess) {
          if (x->graph) (void)hipGraphDestroy(x->graph);
          x->graph = nullptr;
          x->gexec = nullptr;
          return set_err(x, LBRX_E_DEVICE, "graph capture failed");
        }
      }
      HIPCHK(x, hipGraphLaunch(x->gexec, x->stream));
      x->steps += GRAPH_LEN;
      x->cur = (int)(x->steps & 1);
      done += GRAPH_LEN;
    } else {
      const lbrx_status s = launch_step(x);
      if (s != LBRX_OK) return s;
      done += 1;
    }
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

}  // extern "C"

namespace {

// ------------------------------------------------------------ checkpoints
// State blob: a header naming the layout and the boundaries (the status words
// record which neighbours were fluid or liquid, which depends on them), then
// the current populations, status words, solute code words, solid volumes,
// rho_max partials and balance records.
struct StateHeader {
  char magic[8];
  uint32_t abi;
  int32_t nx, ny, pitch, precision, ns, seg_rows, nitems;
  int32_t per_x, per_y;  // 0 wall, 1 periodic; per_y 2: free outlet at the top
  int64_t steps;
  uint64_t fbytes, gbytes, tbytes, cbytes, vbytes, rbytes, lbytes;
};
static const char STATE_MAGIC[8] = {'L', 'B', 'R', 'X', 'S', 'T', '0', '2'};

StateHeader state_header(const lbrx_ctx* x) {
  const KConst& c = x->c;
  StateHeader h{};
  std::memcpy(h.magic, STATE_MAGIC, 8);
  h.abi = LBRX_ABI_VERSION;
  h.nx = c.nx;
  h.ny = c.ny;
  h.pitch = c.pitch;
  h.precision = x->precision;
  h.ns = c.ns;
  h.seg_rows = c.seg_rows;
  h.nitems = c.nitems;
  h.per_x = c.per_x;
  h.per_y = c.per_y;
  h.steps = x->steps;
  h.fbytes = c.fbytes;
  h.gbytes = c.gbytes;
  h.tbytes = c.tbytes;
  h.cbytes = x->cw[0] ? c.cbytes : 0;
  h.vbytes = (uint64_t)c.plane * 8;
  h.rbytes = (uint64_t)RM_WORDS * 8;
  h.lbytes = (uint64_t)c.nitems * NLED * 8;
  return h;
}
uint64_t state_size(const StateHeader& h) {
  return sizeof(StateHeader) + h.fbytes + h.gbytes + h.tbytes + h.cbytes + h.vbytes + h.rbytes + h.lbytes;
}

}  // namespace

extern "C" {

lbrx_status lbrx_state_bytes(const lbrx_ctx* x, uint64_t* bytes) {
  if (!x || !bytes) return LBRX_E_INVAL;
  *bytes = state_size(state_header(x));
  return LBRX_OK;
}

lbrx_status lbrx_save_state(lbrx_ctx* x, void* buf, uint64_t bytes) {
  if (!x || !buf) return LBRX_E_INVAL;
  const StateHeader h = state_header(x);
  if (bytes < state_size(h)) return set_err(x, LBRX_E_INVAL, "state buffer too small");
  const lbrx_status st = lbrx_sync(x);
  if (st != LBRX_OK) return st;
  char* p = (char*)buf;
  std::memcpy(p, &h, sizeof h);
  p += sizeof h;
  const int cur = x->cur;
  auto get = [&](const void* src, uint64_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    const hipError_t e = hipMemcpy(p, src, n, hipMemcpyDeviceToHost);
    p += n;
    return e;
  };
  HIPCHK(x, get(x->f[cur], h.fbytes));
  HIPCHK(x, get(x->g[cur], h.gbytes));
  HIPCHK(x, get(x->t[cur], h.tbytes));
  HIPCHK(x, get(x->cw[cur], h.cbytes));
  HIPCHK(x, get(x->V, h.vbytes));
  HIPCHK(x, get(x->rmax, h.rbytes));
  HIPCHK(x, get(x->led, h.lbytes));
  return LBRX_OK;
}

lbrx_status lbrx_load_state(lbrx_ctx* x, const void* buf, uint64_t bytes) {
  if (!x || !buf) return LBRX_E_INVAL;
  if (x->failed) return set_err(x, LBRX_E_STATE, "context failed earlier: " + x->msg);
  StateHeader h;
  if (bytes < sizeof h) return set_err(x, LBRX_E_INVAL, "state buffer too small");
  std::memcpy(&h, buf, sizeof h);
  StateHeader mine = state_header(x);
  mine.steps = h.steps;
  if (std::memcmp(&h, &mine, sizeof h) != 0)
    return set_err(x, LBRX_E_INVAL, "the state was saved from a context of another layout "
                                    "(lattice size, boundaries, precision, species count, seg_rows or ABI version)");
  if (h.steps < 0 || bytes < state_size(h)) return set_err(x, LBRX_E_INVAL, "state buffer too small");
  HIPCHK(x, hipSetDevice(x->device));
  HIPCHK(x, hipStreamSynchronize(x->stream));
  const char* p = (const char*)buf + sizeof h;
  const int cur = (int)(h.steps & 1);
  // the populations go into both buffers, as at create: slots that the next
  // steps do not write hold defined values
  auto put2 = [&](void* const (&dst)[2], uint64_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    hipError_t e = hipMemcpy(dst[cur], p, n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dst[1 - cur], p, n, hipMemcpyHostToDevice);
    p += n;
    return e;
  };
  auto put = [&](void* dst, uint64_t n) -> hipError_t {
    const hipError_t e = hipMemcpy(dst, p, n, hipMemcpyHostToDevice);
    p += n;
    return e;
  };
  void* const fb[2] = {x->f[0], x->f[1]};
  void* const gb[2] = {x->g[0], x->g[1]};
  void* const tb[2] = {x->t[0], x->t[1]};
  void* const cb[2] = {x->cw[0], x->cw[1]};
  HIPCHK(x, put2(fb, h.fbytes));
  HIPCHK(x, put2(gb, h.gbytes));
  HIPCHK(x, put2(tb, h.tbytes));
  HIPCHK(x, put2(cb, h.cbytes));
  HIPCHK(x, put(x->V, h.vbytes));
  HIPCHK(x, put(x->rmax, h.rbytes));
  HIPCHK(x, put(x->led, h.lbytes));
  x->steps = h.steps;
  x->cur = cur;
  return LBRX_OK;
}

}  // extern "C"

namespace {

// Read-out staging of a context, in doubles: the planes of lbrx_fields_out
// (rho1, rho2, ux, uy, every C_k, liquid marks; pitch-strided) and the summed
// balance records.
size_t read_out_doubles(const KConst& c) { return (5 + (size_t)c.ns) * (size_t)c.plane + NLED; }

// lbrx_fields into caller buffers, with the read-out kernels writing into
// `stage` (read_out_doubles(c) doubles of device memory).
lbrx_status fields_into(lbrx_ctx* x, lbrx_fields_out* o, double* stage) {
  const KConst& c = x->c;
  const size_t plane = (size_t)c.plane;
  double* const ledsum = stage + (5 + (size_t)c.ns) * plane;
  // the read-out kernel runs only for the fields it forms
  const bool moments = o->rho1 || o->rho2 || o->ux || o->uy || (o->C && c.ns > 0) || o->liquid;
  if (moments) {
    HIPCHK(x, hipMemsetAsync(stage, 0, (5 + (size_t)c.ns) * plane * 8, x->stream));
    launch_one(x, true, stage);
    HIPCHK(x, hipGetLastError());
  }
  if (o->ledger) {
    hipLaunchKernelGGL(k_ledger_sum, dim3(NLED), dim3(LSUM_THREADS), 0, x->stream, x->led, c.nitems, ledsum);
    HIPCHK(x, hipGetLastError());
  }
  HIPCHK(x, hipStreamSynchronize(x->stream));
  const size_t sp = (size_t)c.pitch * 8, dp = (size_t)c.nx * 8;
  auto get2d = [&](double* dst, const double* src) -> hipError_t {
    return hipMemcpy2D(dst, dp, src, sp, dp, c.ny, hipMemcpyDeviceToHost);
  };
  if (o->rho1) HIPCHK(x, get2d(o->rho1, stage));
  if (o->rho2) HIPCHK(x, get2d(o->rho2, stage + plane));
  if (o->ux) HIPCHK(x, get2d(o->ux, stage + 2 * plane));
  if (o->uy) HIPCHK(x, get2d(o->uy, stage + 3 * plane));
  if (o->C)
    for (int k = 0; k < c.ns; ++k) HIPCHK(x, get2d(o->C + (size_t)k * c.nx * c.ny, stage + (4 + k) * plane));
  if (o->V) HIPCHK(x, get2d(o->V, x->V));
  if (o->type) {
    std::vector<uint32_t> tb((size_t)c.nx * c.ny);
    HIPCHK(x, hipMemcpy2D(tb.data(), (size_t)c.nx * 4, x->t[x->cur], (size_t)c.pitch * 4, (size_t)c.nx * 4, c.ny,
                          hipMemcpyDeviceToHost));
    for (size_t i = 0; i < tb.size(); ++i) o->type[i] = tb[i] & TB_T;
  }
  if (o->liquid) {
    // this step's liquid marks, decided by the read-out kernel as by the step
    std::vector<double> lq((size_t)c.nx * c.ny);
    HIPCHK(x, get2d(lq.data(), stage + (4 + (size_t)c.ns) * plane));
    for (size_t i = 0; i < lq.size(); ++i) o->liquid[i] = lq[i] != 0.0 ? 1 : 0;
  }
  if (o->ledger) {
    double l[NLED];
    HIPCHK(x, hipMemcpy(l, ledsum, sizeof l, hipMemcpyDeviceToHost));
    static_assert(sizeof(lbrx_ledger) == NLED * sizeof(double), "ledger layout");
    l[NLED - 1] = (double)x->steps;
    std::memcpy(o->ledger, l, sizeof l);
  }
  if (o->rho_max) {
    std::vector<unsigned long long> v(RM_WORDS);
    const int last = (int)((x->steps + 2) % 3);
    HIPCHK(x, hipMemcpy(v.data(), x->rmax, RM_WORDS * 8, hipMemcpyDeviceToHost));
    double m = 0.0;
    for (int xc = 0; xc < 8; ++xc) {
      double d;
      std::memcpy(&d, &v[last * RM_SLOT + xc * RM_STRIDE], 8);
      m = d > m ? d : m;
    }
    *o->rho_max = m;
  }
  return LBRX_OK;
}

// Read-out staging for lbrx_fields_noalloc: one static array per GPU (each
// device holds its own copy from the time the library is loaded until the
// process ends).  Host code never uses the array's name as an address: its
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t NOALLOC_DOUBLES = LBRX_NOALLOC_SCRATCH_BYTES / sizeof(double);
__device__ __align__(256) double scratch[NOALLOC_DOUBLES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

double* scratch_of_device(int dev, hipError_t& e) {
  e = hipSuccess;
  if (dev < 0 || dev >= MAX_DEVICES) {
    e = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));  // the current device is `dev`
    if (e != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = (double*)ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

lbrx_status lbrx_fields(lbrx_ctx* x, lbrx_fields_out* o) {
  if (!x || !o) return LBRX_E_INVAL;
  const lbrx_status st = lbrx_sync(x);
  if (st != LBRX_OK) return st;
  if (!x->out && !ctx_alloc(x, (void**)&x->out, read_out_doubles(x->c) * 8))
    return set_err(x, LBRX_E_NOMEM, "device allocation of the read-out planes failed");
  return fields_into(x, o, x->out);
}

lbrx_status lbrx_fields_noalloc(lbrx_ctx* x, lbrx_fields_out* o) {
  if (!x || !o) return LBRX_E_INVAL;
  if (read_out_doubles(x->c) > NOALLOC_DOUBLES) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "lbrx_fields_noalloc: the read-out of this lattice needs %zu bytes, more than the %zu-byte static "
             "array (use lbrx_fields)", read_out_doubles(x->c) * 8, (size_t)LBRX_NOALLOC_SCRATCH_BYTES);
    return set_err(x, LBRX_E_INVAL, buf);
  }
  const lbrx_status st = lbrx_sync(x);  // (selects the context's device)
  if (st != LBRX_OK) return st;
  hipError_t e;
  double* stage = scratch_of_device(x->device, e);
  if (!stage) return set_err(x, LBRX_E_DEVICE, std::string("hipGetSymbolAddress of the read-out array: ") + hipGetErrorString(e));
  return fields_into(x, o, stage);
}

int64_t lbrx_step_count(const lbrx_ctx* x) { return x ? x->steps : -1; }

}  // extern "C"

// ---------------------------------------------------------------- batches
// Several simulations stepped by one launch per step: the workgroups of all
// of them in one grid, each looking up its simulation, item block and step
// phase in a table built on the host.  Runs of GRAPH_LEN steps replay a
// captured HIP graph.

struct lbrx_batch {
  std::vector<lbrx_ctx*> ctx;
  std::vector<int64_t> base;  // step counts when the table was built
  int precision = 0, device = 0;
  hipStream_t stream = nullptr;
  void** dinst = nullptr;
  uint32_t* dtable = nullptr;
  int nblocks = 0;
  int64_t launches = 0;  // since the table was built
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t done = nullptr;  // recorded after the batch's last launch
  std::string msg;
};

namespace {

lbrx_status batch_err(lbrx_batch* b, lbrx_status s, const std::string& m) {
  if (b) b->msg = m;
  return s;
}

void batch_drop_graph(lbrx_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
}

// table of workgroups: simulation-major, each simulation's blocks in order,
// with the simulation's step phase now
lbrx_status batch_build(lbrx_batch* b) {
  std::vector<uint32_t> tab;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    lbrx_ctx* x = b->ctx[i];
    for (int k = 0; k < x->c.nblocks; ++k)
      tab.push_back(((uint32_t)i << TAB_INST_SHIFT) | ((uint32_t)(x->steps % 6) << TAB_PHASE_SHIFT) | (uint32_t)k);
    b->base[i] = x->steps;
  }
  // launches still queued that read the old table (or replay the old graph)
  // finish before it is returned
  if (b->dtable) {
    (void)hipStreamSynchronize(b->stream);
    ctx_free(b->ctx[0], b->dtable);
  }
  b->dtable = nullptr;
  if (!ctx_alloc(b->ctx[0], (void**)&b->dtable, tab.size() * 4))
    return batch_err(b, LBRX_E_NOMEM, "device allocation of the batch table failed");
  if (hipMemcpy(b->dtable, tab.data(), tab.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return batch_err(b, LBRX_E_DEVICE, "copy of the batch table failed");
  b->nblocks = (int)tab.size();
  b->launches = 0;
  batch_drop_graph(b);
  return LBRX_OK;
}

void batch_launch(lbrx_batch* b, int lidx) {
  LaunchArgs L{};
  L.inst = b->dinst;
  L.table = b->dtable;
  L.ninst = (int)b->ctx.size();
  L.launch = lidx;
  const dim3 grid(b->nblocks), block(64, WPB);
  // the kernels of a simulation with a free outlet also run the others
  lbrx_ctx* x = b->ctx[0];
  for (lbrx_ctx* y : b->ctx)
    if (y->c.per_y == 2) x = y;
  if (b->precision == LBRX_F64)
    hipLaunchKernelGGL(x->step64, grid, block, 0, b->stream, L);
  else
    hipLaunchKernelGGL(x->step32, grid, block, 0, b->stream, L);
}

}  // namespace

extern "C" {

lbrx_status lbrx_batch_create(lbrx_ctx* const* ctxs, int n, lbrx_batch** out) {
  if (!out) return LBRX_E_INVAL;
  *out = nullptr;
  if (!ctxs || n < 1 || n >= (1 << (32 - TAB_INST_SHIFT))) return LBRX_E_INVAL;
  lbrx_ctx* x0 = ctxs[0];
  for (int i = 0; i < n; ++i) {
    lbrx_ctx* x = ctxs[i];
    if (!x || x->failed) return LBRX_E_INVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == x) return LBRX_E_INVAL;
    if (x->device != x0->device || x->stream != x0->stream || x->precision != x0->precision || x->c.ns != x0->c.ns)
      return LBRX_E_INVAL;
    if ((unsigned)x->c.nblocks > TAB_BLOCK_MASK + 1u) return LBRX_E_INVAL;
  }
  lbrx_batch* b = new lbrx_batch();
  b->ctx.assign(ctxs, ctxs + n);
  b->base.assign(n, 0);
  b->precision = x0->precision;
  b->device = x0->device;
  b->stream = x0->stream;
  if (hipSetDevice(b->device) != hipSuccess) {
    delete b;
    return LBRX_E_DEVICE;
  }
  std::vector<void*> inst(n);
  for (int i = 0; i < n; ++i) inst[i] = ctxs[i]->dargs;
  if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
    b->done = nullptr;
    delete b;
    return LBRX_E_DEVICE;
  }
  if (!ctx_alloc(b->ctx[0], (void**)&b->dinst, n * sizeof(void*))) {
    (void)hipEventDestroy(b->done);
    delete b;
    return LBRX_E_NOMEM;
  }
  const lbrx_status s = hipMemcpy(b->dinst, inst.data(), n * sizeof(void*), hipMemcpyHostToDevice) == hipSuccess
                            ? batch_build(b) : LBRX_E_DEVICE;
  if (s != LBRX_OK) {
    lbrx_batch_destroy(b);
    return s;
  }
  *out = b;
  return LBRX_OK;
}

lbrx_status lbrx_batch_step(lbrx_batch* b, int64_t n) {
  if (!b) return LBRX_E_INVAL;
  if (n < 0) return batch_err(b, LBRX_E_INVAL, "n_steps must be >= 0");
  for (size_t i = 0; i < b->ctx.size(); ++i)
    if (b->ctx[i]->failed) return batch_err(b, LBRX_E_STATE, "a simulation of the batch failed earlier");
  if (hipSetDevice(b->device) != hipSuccess) return batch_err(b, LBRX_E_DEVICE, "hipSetDevice failed");
  // a simulation stepped on its own since: the phases in the table are stale
  for (size_t i = 0; i < b->ctx.size(); ++i)
    if (b->ctx[i]->steps != b->base[i] + b->launches) {
      const lbrx_status s = batch_build(b);
      if (s != LBRX_OK) return s;
      break;
    }
  // every return after a launch records the batch's event (destroy waits on it)
  auto stop = [&](lbrx_status st, const char* m) {
    (void)hipEventRecord(b->done, b->stream);
    return batch_err(b, st, m);
  };
  int64_t done = 0;
  while (done < n) {
    const int lidx = (int)(b->launches % 6);
    if (lidx == 0 && n - done >= GRAPH_LEN) {
      if (!b->gexec) {
        if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
          return stop(LBRX_E_DEVICE, "graph capture failed to start");
        for (int i = 0; i < GRAPH_LEN; ++i) batch_launch(b, i % 6);
        if (hipStreamEndCapture(b->stream, &b->graph) != hipSuccess ||
            hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
          batch_drop_graph(b);
          return stop(LBRX_E_DEVICE, "graph capture failed");
        }
      }
      if (hipGraphLaunch(b->gexec, b->stream) != hipSuccess) return stop(LBRX_E_DEVICE, "graph launch failed");
      done += GRAPH_LEN;
      b->launches += GRAPH_LEN;
    } else {
      batch_launch(b, lidx);
      if (hipGetLastError() != hipSuccess) return stop(LBRX_E_DEVICE, "batched launch failed");
      done += 1;
      b->launches += 1;
    }
  }
  for (lbrx_ctx* x : b->ctx) {
    x->steps += n;
    x->cur = (int)(x->steps & 1);
  }
  if (hipEventRecord(b->done, b->stream) != hipSuccess) return batch_err(b, LBRX_E_DEVICE, "event record failed");
  return LBRX_OK;
}

const char* lbrx_batch_last_error(const lbrx_batch* b) { return b ? b->msg.c_str() : "NULL batch"; }

lbrx_status lbrx_batch_destroy(lbrx_batch* b) {
  if (!b) return LBRX_OK;
  (void)hipSetDevice(b->device);
  // wait for the batch's own launches only (work queued after them on the
  // stream, e.g. by another batch, keeps running)
  if (b->done) (void)hipEventSynchronize(b->done);
  else if (b->stream) (void)hipStreamSynchronize(b->stream);
  batch_drop_graph(b);
  ctx_free(b->ctx[0], b->dtable);
  ctx_free(b->ctx[0], b->dinst);
  if (b->done) (void)hipEventDestroy(b->done);
  delete b;
  return LBRX_OK;
}

void* lbrx_stream(const lbrx_ctx* x) { return x ? (void*)x->stream : nullptr; }

const char* lbrx_last_error(const lbrx_ctx* x) { return x ? x->msg.c_str() : "NULL context"; }

lbrx_status lbrx_destroy(lbrx_ctx* x) {
  if (!x) return LBRX_OK;
  (void)hipSetDevice(x->device);
  if (x->stream) (void)hipStreamSynchronize(x->stream);
  if (x->gexec) (void)hipGraphExecDestroy(x->gexec);
  if (x->graph) (void)hipGraphDestroy(x->graph);
  for (int i = 0; i < 2; ++i) {
    ctx_free(x, x->f[i]);
    ctx_free(x, x->g[i]);
    ctx_free(x, x->t[i]);
    ctx_free(x, x->cw[i]);
  }
  ctx_free(x, x->V);
  ctx_free(x, x->rmax);
  ctx_free(x, x->led);
  ctx_free(x, x->ledsum);
  ctx_free(x, x->err);
  ctx_free(x, x->out);
  ctx_free(x, x->dargs);
  if (x->own_stream && x->stream) (void)hipStreamDestroy(x->stream);
  delete x;
  return LBRX_OK;
}

}  // extern "C"

/*
 * Plain FP64 CPU oracle for one coupled time step of the two-phase
 * multi-mixture reactive-transport lattice Boltzmann model of
 * Chen, Kang, Tang, Robinson, He, Tao, "Pore-scale simulation of
 * multicomponent multiphase reactive transport with dissolution and
 * precipitation" (arXiv:1410.3464).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes,
 * links or calls this file; it is used by the tests, by the smoke check
 * and by the benchmark's CPU-baseline leg.  It shares no code, header,
 * table or constant with the GPU path.
 *
 * The oracle is deliberately slow: one full-lattice pass per sub-step of
 * the method, in the order of Sec. 4.7 (Steps 1-5), plain loops, double
 * precision everywhere.
 */
#ifndef LBRX_ORACLE_H
#define LBRX_ORACLE_H
#include <stdint.h>

#define ORC_MAX_SPECIES 8
#define ORC_MAX_RXN 8

/* node types */
#define ORC_FLUID 0
#define ORC_SOLID_INERT 1
#define ORC_SOLID_D 2
#define ORC_SOLID_F 3

/* homogeneous reaction kinds (Sec. 2 rate laws, Eq. 5) */
#define ORC_HOM_FIRST_ORDER 0   /* R = k C_re0                               */
#define ORC_HOM_R1_GAS 1        /* R = k (C_re0 - C_pr0 sqrt(rho2/M)/Keq)     */
#define ORC_HOM_BIMOLECULAR 2   /* R = k C_re0 C_re1                          */

/* heterogeneous reaction modes (Sec. 4.3 / 4.4 and Appendix A.3) */
#define ORC_HET_CONSUMES 0      /* solid node volume decreases by Vbar*Phi (R2-like, Eq. 33) */
#define ORC_HET_GROWS 1         /* liquid node precipitate volume increases by Vbar*Phi (R4-like, Eq. 35) */
#define ORC_HET_MINERAL 2       /* solid node volume increases by Vbar*Phi; Phi<0 dissolves (Eq. A2) */

typedef struct {
  int32_t nx, ny, periodic_x, periodic_y;
  double tau[2];          /* BGK relaxation times of the two flow components (Eq. 6, 10) */
  double w_adh[2];        /* fluid-solid interaction strengths (Eq. 16) */
  double gbody[2];        /* body acceleration (x, y); force = rho_sigma * g */
  double a, b, R, T;      /* Carnahan-Starling EOS (Eq. 12) */
  double G11, G12, G21;   /* interaction strengths (Eq. 11, 14) */
  double a0, rho10, rho20;/* inter-component effective masses (Eq. 15) */
  double liquid_frac;     /* liquid iff rho1 > liquid_frac * max rho1 (Sec. 4.5) */
  double psi_pre;         /* psi = sqrt(psi_pre (p - rho/3) / G11): 2 reproduces Eq. 12 with
                             the weights of Eq. 11; 6 is the printed prefactor of Eq. 13 */
  int32_t n_species;
  double tau_g[ORC_MAX_SPECIES];
  double J0[ORC_MAX_SPECIES];
  int32_t n_hom;
  int32_t hom_kind[ORC_MAX_RXN];
  int32_t hom_re[ORC_MAX_RXN][2];
  int32_t hom_pr[ORC_MAX_RXN][2];
  double hom_k[ORC_MAX_RXN];
  double hom_Keq[ORC_MAX_RXN];
  double hom_Mgas[ORC_MAX_RXN];
  int32_t hom_surface[ORC_MAX_RXN];  /* bit (1<<type): solid types whose D2Q5 adjacency enhances k */
  double hom_sfac[ORC_MAX_RXN];      /* factor on k next to such a solid (R1 at D(s), Sec. 2) */
  int32_t n_het;
  int32_t het_reactant[ORC_MAX_RXN];
  int32_t het_product[ORC_MAX_RXN];
  int32_t het_surface[ORC_MAX_RXN];  /* bit (1<<type) for each solid type the reaction acts on */
  int32_t het_mode[ORC_MAX_RXN];
  int32_t het_irrev[ORC_MAX_RXN];    /* 1: clamp the link flux at >= 0 */
  double het_k[ORC_MAX_RXN];
  double het_Ceq[ORC_MAX_RXN];
  double het_mvol[ORC_MAX_RXN];      /* molar volume x specific area per link */
  int32_t outlet_top;     /* 1: the side beyond y = ny - 1 is a free outlet with zero
                             gradient of every variable (Sec. 5.1); needs periodic_y = 0 */
  int32_t sub_species;    /* Sec. 4.1: the aqueous species whose concentration at a liquid
                             node is the total liquid concentration minus the others
                             (not transported in effect); -1: none */
  double sub_total;       /* the total liquid concentration per unit rho_1 (> 0 when
                             sub_species >= 0) */
} orc_params;

/* cumulative balance ledger, all FP64 */
typedef struct {
  double mass_src[2];   /* sum of homogeneous flow sources S_sigma (Eq. 27) */
  double mass_inj[2];   /* mass put into nodes freed by dissolution */
  double mass_rem[2];   /* stranded mass with no fluid neighbour to take it */
  double sol_src[ORC_MAX_SPECIES];  /* sum of homogeneous solute sources (Eq. 28) */
  double sol_het[ORC_MAX_SPECIES];  /* net heterogeneous boundary exchange (Eq. 29-31) */
  double sol_rem[ORC_MAX_SPECIES];  /* solute dropped: always 0 (content without a liquid
                                       neighbour is kept until it has one) */
  double vol_dv;        /* sum of all VOP volume increments (Eq. 33, 35) */
  double vol_clip;      /* sum of the (non-positive) volumes of removed solid nodes */
  double n_psi_clamp;   /* count of clamped negative psi arguments */
  double n_dissolved, n_precipitated, n_liq_to_gas, n_gas_to_liq;
  double steps;
} orc_ledger;

typedef struct orc_sim orc_sim;

/* Copies every input.  type0, V0, rho1, rho2: nx*ny, index y*nx+x.
 * C0: n_species*nx*ny.  V0 may be NULL (1.0 at solid D/F nodes, 0 elsewhere).
 * Returns NULL and fills err on invalid input. */
orc_sim* orc_create(const orc_params* p, const uint8_t* type0, const double* V0,
                    const double* rho1, const double* rho2, const double* C0,
                    char* err, int errlen);
/* Advances n steps; returns 0, or -1 on instability (message in orc_error). */
int orc_step(orc_sim* s, int n);
/* Macroscopic fields of the current state.  Any pointer may be NULL.
 * liquid: this step's liquid marks (Sec. 4.5).  C: the solute each node holds
 * once the shares in transit are delivered. */
void orc_fields(orc_sim* s, double* rho1, double* rho2, double* ux, double* uy,
                double* C, uint8_t* type, uint8_t* liquid, double* V,
                orc_ledger* ledger, double* rho_max_prev);
/* Raw state (populations, flags) for brute-force cross-checks.  Any pointer may be NULL.
 * f: 2*9*N, g: ns*5*N, flags: N bytes (bits 0-1 the solute a node holds: 0 none,
 * 1 streamed populations (liquid last step), 2 content kept at rest, 3 shares in
 * transit; bit 2 stranded). */
void orc_state(orc_sim* s, double* f, double* g, uint8_t* flags);
const char* orc_error(orc_sim* s);
/* Host threads for the node loops (OpenMP builds; 1 by default).  Every
 * balance sum stays serial in node order: results do not depend on n. */
void orc_set_threads(orc_sim* s, int n);
/* Diagnostics of the steps since the previous call (then reset): the smallest
 * relative distance |rho1 - threshold| / threshold of a liquid decision, and
 * the smallest distance of a changed solid or precipitate volume from its
 * threshold (0 or 1).  Decisions closer than a result's rounding may come out
 * the other way in another precision. */
void orc_margins(orc_sim* s, double* liq, double* vol);
int64_t orc_step_count(orc_sim* s);
void orc_destroy(orc_sim* s);

#endif

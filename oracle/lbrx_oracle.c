/*
 * Plain FP64 CPU oracle of the coupled reactive-transport LB step.
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
 * benchmark's CPU baseline.  The product library never includes or calls it.
 *
 * One step, in the order of Sec. 4.7 (Steps 1-5); every sub-step is one
 * full-lattice pass over plain arrays:
 *   1  moments of the streamed populations (Eq. 9, 23): the flow field of
 *      Step 1 is the result of the previous collision and streaming
 *   2  effective masses psi_1 (Eq. 12-13), phi_1, phi_2 (Eq. 15)
 *   3  liquid marks from this step's densities (Sec. 4.5; Step 2), and the
 *      maximum liquid-component density that sets the next step's threshold
 *   4  forces: cohesion (Eq. 11), inter-component (Eq. 14), adhesion (Eq. 16), body force
 *   5  velocities (Eq. 17-19)
 *   6  homogeneous reaction sources at liquid nodes (Eq. 5, 27, 28)
 *   7  flow collision (Eq. 6, 8) and solute collision (Eq. 20-22) (Step 3)
 *   8  heterogeneous link fluxes (Eq. 29-31, A2) in halfway-wall Robin form
 *   9  volume-of-pixel update (Eq. 33, 35) and the new node types (Step 4)
 *  10  amendments for nodes that changed status (Sec. 4.5; Steps 2 and 5)
 *  11  push streaming with halfway bounce-back and reactive flux
 * Readings of the places where the paper is silent are stated where used.
 * Parity unpinned (no closed form, invariant or printed value fixes them
 * beyond conservation, which the tests check): which density each phi of
 * Eq. 15 takes, the threshold's maximum density taken one step back, the
 * details of the status-change amendments of Sec. 4.5, and the time level
 * of the velocity in the solute equilibrium.
 */
#include "lbrx_oracle.h"
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Solute a node holds at the start of a step (Sec. 4.5 amendments):
 *   SF_STREAM  it was liquid in the previous step; its slots hold the
 *              populations streamed into it
 *   SF_HOLD    it is not liquid and keeps its content at rest in its own
 *              slots (no liquid D2Q5 neighbour could take it)
 *   SF_SHARE   it left the liquid set last step; its slots hold, at rest,
 *              the share of its content due to each D2Q5 neighbour that was
 *              liquid then, delivered during this step */
enum { SF_NONE = 0, SF_STREAM = 1, SF_HOLD = 2, SF_SHARE = 3 };

/* Loops whose iterations touch only their own node's results may run on
 * several host threads (orc_set_threads; OpenMP builds).  Every balance sum
 * stays in a serial loop in node order, so the results are bit for bit those
 * of one thread. */
#ifdef _OPENMP
#define PAR_FOR _Pragma("omp parallel for num_threads(s->nthreads) schedule(static)")
#else
#define PAR_FOR
#endif

/* D2Q9 velocities (Eq. 7); D2Q5 uses directions 0..4 of the same table (Sec. 3.2). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* equilibrium weights (text after Eq. 8) */
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
/* pseudopotential stencil weights w(1)=1/3, w(2)=1/12 (text after Eq. 11) */
static const double WF[9] = {0.0, 1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 3,
                             1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12};

struct orc_sim {
  orc_params p;
  int N, ns;
  int64_t step;
  /* state */
  double *f, *g;            /* f[s][a][N] (streamed, time n), g[k][a][N] */
  double *fs, *gs;          /* post-collision scratch */
  double *fn, *gn;          /* next-step buffers */
  uint8_t *type;            /* T(n) */
  uint8_t *liq;             /* liquid mark of this step, L(n) */
  uint8_t *sflag;           /* solute held at the start of the step (SF_*) */
  uint8_t *stranded;        /* node became SOLID_F at the end of the previous step */
  double *V;
  double rho_max_prev;
  orc_ledger led;
  /* per-step work arrays */
  double *rho, *jx, *jy;    /* [2][N] */
  double *C;                /* [ns][N] moments of the solute slots */
  double *Cin;              /* [ns][N] shares received from nodes that left the liquid */
  double *psi1, *phi1, *phi2;
  double *Fx, *Fy;          /* [2][N] */
  double *ueqx, *ueqy;      /* [2][N] */
  double *urx, *ury;
  double *Ss;               /* flow sources [2][N] */
  double *Sk;               /* solute sources [ns][N] */
  double *Phi;              /* link flux per het reaction [n_het][N] */
  uint8_t *tnext;           /* T(n+1) */
  uint8_t *snext;           /* solute held at the start of the next step */
  double *rbar;             /* [2][N] mean density put into dissolved nodes */
  double D[ORC_MAX_SPECIES];
  double kap[ORC_MAX_RXN];
  uint8_t *bad, *clamp;     /* per-node flags of sub-steps 1-2, examined in node order */
  double *dvv;              /* per-node volume increment of sub-step 9 */
  uint8_t *dvt;             /*   and whether the node had a reactive link */
  int nthreads;
  double margin_liq, margin_vol;  /* smallest decision margins since the last read-out */
  char err[256];
};

/* Neighbour of (x, y) in direction a; -1 outside a wall side.  Beyond a free
 * outlet (Sec. 5.1: zero gradient of every variable) lies a ghost row that
 * repeats the top row, so the neighbour there is the top-row node of the
 * same column: its type, potentials, concentrations and post-collision
 * populations stand for the ghost's. */
static int nb(const orc_sim* s, int x, int y, int a) {
  int X = x + EX[a], Y = y + EY[a];
  const int nx = s->p.nx, ny = s->p.ny;
  if (X < 0 || X >= nx) {
    if (!s->p.periodic_x) return -1;
    X = (X + nx) % nx;
  }
  if (Y >= ny && s->p.outlet_top) {
    Y = ny - 1;
  } else if (Y < 0 || Y >= ny) {
    if (!s->p.periodic_y) return -1;
    Y = (Y + ny) % ny;
  }
  return Y * nx + X;
}

/* Neighbour for the amendments of Sec. 4.5, which move content between
 * lattice nodes only: as nb(), but -1 beyond the free outlet (a ghost node
 * neither gives, takes nor counts). */
static int nb_node(const orc_sim* s, int x, int y, int a) {
  if (s->p.outlet_top && y + EY[a] >= s->p.ny) return -1;
  return nb(s, x, y, a);
}

/* 1 if the link from (x, y) in direction a crosses the free outlet */
static int crosses_outlet(const orc_sim* s, int y, int a) {
  return s->p.outlet_top && y + EY[a] >= s->p.ny;
}

static void* xcalloc(size_t n, size_t sz) {
  void* q = calloc(n ? n : 1, sz);
  if (!q) abort();
  return q;
}

static int fail(char* err, int errlen, const char* msg) {
  if (err && errlen > 0) snprintf(err, (size_t)errlen, "%s", msg);
  return 0;
}

static int validate(const orc_params* p, char* err, int errlen) {
  if (p->nx < 1 || p->ny < 1) return fail(err, errlen, "nx, ny must be >= 1");
  for (int s = 0; s < 2; ++s)
    if (!(p->tau[s] > 0.5)) return fail(err, errlen, "tau must exceed 1/2 (Eq. 10)");
  if (p->n_species < 0 || p->n_species > ORC_MAX_SPECIES) return fail(err, errlen, "bad n_species");
  for (int k = 0; k < p->n_species; ++k) {
    if (!(p->tau_g[k] > 0.5)) return fail(err, errlen, "tau_g must exceed 1/2 (Eq. 24)");
    if (!(p->J0[k] >= 0.0 && p->J0[k] < 1.0)) return fail(err, errlen, "J0 must be in [0,1) (Eq. 22)");
  }
  if (p->n_hom < 0 || p->n_hom > ORC_MAX_RXN || p->n_het < 0 || p->n_het > ORC_MAX_RXN)
    return fail(err, errlen, "bad reaction count");
  const int ns = p->n_species;
  for (int r = 0; r < p->n_hom; ++r) {
    int kind = p->hom_kind[r];
    if (kind < 0 || kind > 2) return fail(err, errlen, "bad homogeneous reaction kind");
    for (int i = 0; i < 2; ++i) {
      if (p->hom_re[r][i] < -1 || p->hom_re[r][i] >= ns) return fail(err, errlen, "bad reactant index");
      if (p->hom_pr[r][i] < -1 || p->hom_pr[r][i] >= ns) return fail(err, errlen, "bad product index");
    }
    if (p->hom_re[r][0] < 0) return fail(err, errlen, "reaction needs a first reactant");
    if (kind == ORC_HOM_BIMOLECULAR && p->hom_re[r][1] < 0) return fail(err, errlen, "bimolecular needs two reactants");
    if (kind == ORC_HOM_R1_GAS) {
      if (p->hom_pr[r][0] < 0) return fail(err, errlen, "R1 needs an aqueous product");
      if (!(p->hom_Mgas[r] > 0.0) || !(p->hom_Keq[r] > 0.0)) return fail(err, errlen, "R1 needs M_gas > 0 and K_eq > 0");
    }
    if (!(p->hom_k[r] >= 0.0)) return fail(err, errlen, "rate constants must be >= 0");
    if (p->hom_surface[r] && !(p->hom_sfac[r] > 0.0)) return fail(err, errlen, "surface factor must be > 0");
  }
  if (!(p->psi_pre > 0.0)) return fail(err, errlen, "psi prefactor must be > 0");
  for (int r = 0; r < p->n_het; ++r) {
    if (p->het_reactant[r] < 0 || p->het_reactant[r] >= ns) return fail(err, errlen, "bad het reactant");
    if (p->het_product[r] < -1 || p->het_product[r] >= ns) return fail(err, errlen, "bad het product");
    if (p->het_mode[r] < 0 || p->het_mode[r] > 2) return fail(err, errlen, "bad het mode");
    if (p->het_surface[r] & ~((1 << ORC_SOLID_D) | (1 << ORC_SOLID_F)))
      return fail(err, errlen, "het surface may only name SOLID_D / SOLID_F");
    if (!(p->het_k[r] >= 0.0)) return fail(err, errlen, "rate constants must be >= 0");
  }
  if (!(p->liquid_frac >= 0.0 && p->liquid_frac < 1.0)) return fail(err, errlen, "liquid_frac in [0,1)");
  if (p->outlet_top && (p->periodic_y || p->ny < 2)) return fail(err, errlen, "a free outlet needs walls in y and ny >= 2");
  if (p->sub_species < -1 || p->sub_species >= p->n_species) return fail(err, errlen, "bad subtracted species");
  if (p->sub_species >= 0 && !(p->sub_total > 0.0 && p->sub_total < 1e300))
    return fail(err, errlen, "the total liquid concentration per density must be > 0");
  return 1;
}

orc_sim* orc_create(const orc_params* p, const uint8_t* type0, const double* V0,
                    const double* rho1, const double* rho2, const double* C0,
                    char* err, int errlen) {
  if (!validate(p, err, errlen)) return NULL;
  const int N = p->nx * p->ny, ns = p->n_species;
  for (int i = 0; i < N; ++i) {
    if (type0[i] > 3) { fail(err, errlen, "node type out of range"); return NULL; }
    if (type0[i] == ORC_FLUID) {
      if (!(rho1[i] > 0.0) || !(rho2[i] >= 0.0)) { fail(err, errlen, "fluid node needs rho1 > 0, rho2 >= 0"); return NULL; }
      if (V0 && !(V0[i] >= 0.0 && V0[i] < 1.0)) { fail(err, errlen, "fluid node precipitate volume must be in [0,1)"); return NULL; }
    } else if (type0[i] != ORC_SOLID_INERT && V0 && !(V0[i] > 0.0)) {
      fail(err, errlen, "reactive solid needs V > 0"); return NULL;
    }
  }
  orc_sim* s = (orc_sim*)xcalloc(1, sizeof(orc_sim));
  s->p = *p;
  s->N = N;
  s->ns = ns;
  s->f = xcalloc((size_t)18 * N, sizeof(double));
  s->fs = xcalloc((size_t)18 * N, sizeof(double));
  s->fn = xcalloc((size_t)18 * N, sizeof(double));
  s->g = xcalloc((size_t)5 * ns * N + 1, sizeof(double));
  s->gs = xcalloc((size_t)5 * ns * N + 1, sizeof(double));
  s->gn = xcalloc((size_t)5 * ns * N + 1, sizeof(double));
  s->type = xcalloc(N, 1);
  s->liq = xcalloc(N, 1);
  s->sflag = xcalloc(N, 1);
  s->stranded = xcalloc(N, 1);
  s->tnext = xcalloc(N, 1);
  s->snext = xcalloc(N, 1);
  s->V = xcalloc(N, sizeof(double));
  s->rho = xcalloc((size_t)2 * N, sizeof(double));
  s->jx = xcalloc((size_t)2 * N, sizeof(double));
  s->jy = xcalloc((size_t)2 * N, sizeof(double));
  s->C = xcalloc((size_t)ns * N + 1, sizeof(double));
  s->Cin = xcalloc((size_t)ns * N + 1, sizeof(double));
  s->psi1 = xcalloc(N, sizeof(double));
  s->phi1 = xcalloc(N, sizeof(double));
  s->phi2 = xcalloc(N, sizeof(double));
  s->Fx = xcalloc((size_t)2 * N, sizeof(double));
  s->Fy = xcalloc((size_t)2 * N, sizeof(double));
  s->ueqx = xcalloc((size_t)2 * N, sizeof(double));
  s->ueqy = xcalloc((size_t)2 * N, sizeof(double));
  s->urx = xcalloc(N, sizeof(double));
  s->ury = xcalloc(N, sizeof(double));
  s->Ss = xcalloc((size_t)2 * N, sizeof(double));
  s->Sk = xcalloc((size_t)ns * N + 1, sizeof(double));
  s->Phi = xcalloc((size_t)ORC_MAX_RXN * N, sizeof(double));
  s->rbar = xcalloc((size_t)2 * N, sizeof(double));
  s->bad = xcalloc(N, 1);
  s->clamp = xcalloc(N, 1);
  s->dvv = xcalloc(N, sizeof(double));
  s->dvt = xcalloc(N, 1);
  s->nthreads = 1;
  s->margin_liq = s->margin_vol = INFINITY;

  /* Eq. 24: D = (1 - J0)(tau_g - 1/2)/2 */
  for (int k = 0; k < ns; ++k) s->D[k] = 0.5 * (1.0 - p->J0[k]) * (p->tau_g[k] - 0.5);
  /* Halfway-wall Robin link flux.  With the wall half a link from the node,
   * D dC/dn = 2 D (C - Cw) and the surface law D dC/dn = k (Cw - Ceq) give
   * Cw = (2 D C + k Ceq)/(2 D + k) and a flux into the wall per link of
   * k (Cw - Ceq) = kap (C - Ceq), kap = 2 D k / (2 D + k). */
  for (int r = 0; r < p->n_het; ++r) {
    double D = s->D[p->het_reactant[r]], k = p->het_k[r];
    s->kap[r] = (2.0 * D + k) > 0.0 ? 2.0 * D * k / (2.0 * D + k) : 0.0;
  }

  double rmax = 0.0;
  for (int i = 0; i < N; ++i) {
    s->type[i] = type0[i];
    if (V0) s->V[i] = V0[i];
    else s->V[i] = (type0[i] == ORC_SOLID_D || type0[i] == ORC_SOLID_F) ? 1.0 : 0.0;
    if (type0[i] == ORC_FLUID && rho1[i] > rmax) rmax = rho1[i];
  }
  /* Initial liquid set from the given densities and their own maximum. */
  s->rho_max_prev = rmax;
  const double thr = p->liquid_frac * rmax;
  for (int i = 0; i < N; ++i) {
    if (type0[i] != ORC_FLUID) continue;
    /* populations start at rest equilibrium, f = w rho (Eq. 8 with u = 0) */
    for (int a = 0; a < 9; ++a) {
      s->f[(0 * 9 + a) * N + i] = W9[a] * rho1[i];
      s->f[(1 * 9 + a) * N + i] = W9[a] * rho2[i];
    }
    if (rho1[i] > thr) {
      s->liq[i] = 1;
      s->sflag[i] = SF_STREAM;
      for (int k = 0; k < ns; ++k) {
        const double J1 = 0.25 * (1.0 - p->J0[k]);
        for (int a = 0; a < 5; ++a)
          s->g[(k * 5 + a) * N + i] = (a == 0 ? p->J0[k] : J1) * C0[k * N + i];
      }
    }
  }
  return s;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  void* ptrs[] = {s->f, s->fs, s->fn, s->g, s->gs, s->gn, s->type, s->liq, s->sflag, s->Cin, s->snext,
                  s->bad, s->clamp, s->dvv, s->dvt,
                  s->stranded, s->tnext, s->V, s->rho, s->jx, s->jy, s->C, s->psi1,
                  s->phi1, s->phi2, s->Fx, s->Fy, s->ueqx, s->ueqy, s->urx, s->ury,
                  s->Ss, s->Sk, s->Phi, s->rbar};
  for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) free(ptrs[i]);
  free(s);
}

const char* orc_error(orc_sim* s) { return s->err; }
void orc_set_threads(orc_sim* s, int n) { s->nthreads = n > 0 ? n : 1; }
void orc_margins(orc_sim* s, double* liq, double* vol) {
  if (liq) *liq = s->margin_liq;
  if (vol) *vol = s->margin_vol;
  s->margin_liq = s->margin_vol = INFINITY;
}
int64_t orc_step_count(orc_sim* s) { return s->step; }

static double J_of(const orc_params* p, int k, int a) {
  return a == 0 ? p->J0[k] : 0.25 * (1.0 - p->J0[k]);
}

/* Carnahan-Starling pressure, Eq. 12. */
static double p_cs(const orc_params* p, double rho) {
  const double e = 0.25 * p->b * rho;
  const double om = 1.0 - e;
  const double num = 1.0 + e + e * e - e * e * e;
  return rho * (p->R * p->T) * num / (om * om * om) - p->a * rho * rho;
}

/*
 * Sub-steps 1-5: moments, effective masses, forces, velocities of the
 * current state.  Used by the step and by the field export.
 * Returns 0 or -1 (unstable).
 */
static int macros(orc_sim* s) {
  const orc_params* p = &s->p;
  const int N = s->N, ns = s->ns, nx = p->nx;

  /* 1. moments (Eq. 9, 23).  f is valid at fluid nodes and at nodes that
   * turned solid at the end of the previous step (their streamed-in
   * populations are still there).  g is valid where the node holds solute
   * (SF_*); at an SF_SHARE node its moment is the share in transit. */
  PAR_FOR
  for (int i = 0; i < N; ++i) {
    const int validf = s->type[i] == ORC_FLUID || s->stranded[i];
    s->bad[i] = 0;
    for (int sg = 0; sg < 2; ++sg) {
      double r = 0.0, jx = 0.0, jy = 0.0;
      if (validf) {
        for (int a = 0; a < 9; ++a) {
          const double v = s->f[(sg * 9 + a) * N + i];
          r += v;
          jx += v * EX[a];
          jy += v * EY[a];
        }
      }
      s->rho[sg * N + i] = r;
      s->jx[sg * N + i] = jx;
      s->jy[sg * N + i] = jy;
    }
    if (validf) {
      const double r1 = s->rho[i], r2 = s->rho[N + i];
      if (!(r1 >= 0.0) || !(r2 >= 0.0) || (s->type[i] == ORC_FLUID && !(r1 + r2 > 0.0))) s->bad[i] = 1;
    }
    for (int k = 0; k < ns; ++k) {
      double c = 0.0;
      if (s->sflag[i] != SF_NONE)
        for (int a = 0; a < 5; ++a) c += s->g[(k * 5 + a) * N + i];
      s->C[k * N + i] = c;
    }
  }
  for (int i = 0; i < N; ++i)
    if (s->bad[i]) {
      snprintf(s->err, sizeof s->err, "unstable: bad density at node (%d,%d) step %lld",
               i % nx, i / nx, (long long)s->step);
      return -1;
    }

  /* 2. effective masses at fluid nodes.
   * psi_1: Eq. 13 with the prefactor that makes the stencil of Eq. 11
   * (weights 1/3, 1/12, whose second moment is the identity) reproduce the
   * EOS of Eq. 12: p = rho/3 + G11 psi^2 / 2, so psi = sqrt(2 (p - rho/3)/G11).
   * The printed 6/G11 belongs to weights whose second moment is c_s^2 I; it is
   * selected by psi_pre = 6.  A negative argument is clamped to zero and counted.
   * phi_1(rho_2), phi_2(rho_1): Eq. 15 with the natural logarithm in rho_10. */
  PAR_FOR
  for (int i = 0; i < N; ++i) {
    s->psi1[i] = s->phi1[i] = s->phi2[i] = 0.0;
    s->bad[i] = s->clamp[i] = 0;
    if (s->type[i] != ORC_FLUID) continue;
    const double r1 = s->rho[i], r2 = s->rho[N + i];
    if (p->G11 != 0.0) {
      if (!(0.25 * p->b * r1 < 1.0)) {
        s->bad[i] = 1;
        continue;
      }
      const double pre = p->psi_pre;
      double arg = pre * (p_cs(p, r1) - r1 / 3.0) / p->G11;
      if (arg < 0.0) {
        arg = 0.0;
        s->clamp[i] = 1;
      }
      s->psi1[i] = sqrt(arg);
    }
    if (p->rho20 > 0.0) s->phi1[i] = 1.0 - exp(-r2 / p->rho20);
    if (p->rho10 > 0.0) s->phi2[i] = p->a0 - exp(-r1 / p->rho10);
  }
  for (int i = 0; i < N; ++i) {
    if (s->bad[i]) {
      snprintf(s->err, sizeof s->err, "unstable: b*rho/4 >= 1 at node (%d,%d) step %lld",
               i % nx, i / nx, (long long)s->step);
      return -1;
    }
    if (s->clamp[i]) s->led.n_psi_clamp += 1.0;
  }

  /* 4. forces at fluid nodes (Eq. 11, 14, 16, body force).
   * A neighbour that is not fluid (solid, or outside a non-periodic
   * boundary) has wall density s = 1 in Eq. 16.  In the cohesion and
   * inter-component sums it carries the psi / phi of its mirror image in
   * the wall, taken inside the 3x3 block: for an axis link that is the
   * centre node itself; for a diagonal link, the fluid node(s) of the block
   * that share the diagonal neighbour's column or row (their mean when both
   * are fluid), else the centre node.  At a flat wall the sums then see the
   * reflected field, so with w = 0 the wall is neutral and a droplet meets
   * it at 90 degrees, as App. A.1 (Fig. A2) reports. */
  PAR_FOR
  for (int i = 0; i < N; ++i) {
    for (int sg = 0; sg < 2; ++sg) s->Fx[sg * N + i] = s->Fy[sg * N + i] = 0.0;
    if (s->type[i] != ORC_FLUID) continue;
    const int x = i % nx, y = i / nx;
    double c1x = 0, c1y = 0, c12x = 0, c12y = 0, c21x = 0, c21y = 0, swx = 0, swy = 0;
    for (int a = 1; a < 9; ++a) {
      const int j = nb(s, x, y, a);
      const int fl = j >= 0 && s->type[j] == ORC_FLUID;
      double ps, q1, q2;
      if (fl) {
        ps = s->psi1[j];
        q1 = s->phi1[j];
        q2 = s->phi2[j];
      } else {
        int m1 = i, m2 = -1;  /* mirror image node(s) */
        if (a >= 5) {
          const int jx = nb(s, x, y, EX[a] > 0 ? 1 : 3), jy = nb(s, x, y, EY[a] > 0 ? 2 : 4);
          const int fx = jx >= 0 && s->type[jx] == ORC_FLUID, fy = jy >= 0 && s->type[jy] == ORC_FLUID;
          if (fx && fy) {
            m1 = jx;
            m2 = jy;
          } else if (fx) {
            m1 = jx;
          } else if (fy) {
            m1 = jy;
          }
        }
        if (m2 >= 0) {
          ps = 0.5 * (s->psi1[m1] + s->psi1[m2]);
          q1 = 0.5 * (s->phi1[m1] + s->phi1[m2]);
          q2 = 0.5 * (s->phi2[m1] + s->phi2[m2]);
        } else {
          ps = s->psi1[m1];
          q1 = s->phi1[m1];
          q2 = s->phi2[m1];
        }
      }
      const double sw = fl ? 0.0 : 1.0;
      c1x += WF[a] * ps * EX[a];
      c1y += WF[a] * ps * EY[a];
      c12x += WF[a] * q2 * EX[a];
      c12y += WF[a] * q2 * EY[a];
      c21x += WF[a] * q1 * EX[a];
      c21y += WF[a] * q1 * EY[a];
      swx += WF[a] * sw * EX[a];
      swy += WF[a] * sw * EY[a];
    }
    const double r1 = s->rho[i], r2 = s->rho[N + i];
    const double ps = s->psi1[i], q1 = s->phi1[i], q2 = s->phi2[i];
    s->Fx[i] = -p->G11 * ps * c1x - p->G12 * q1 * c12x - p->w_adh[0] * ps * swx + r1 * p->gbody[0];
    s->Fy[i] = -p->G11 * ps * c1y - p->G12 * q1 * c12y - p->w_adh[0] * ps * swy + r1 * p->gbody[1];
    /* component 2: no self-interaction (G22 = 0); adhesion with psi_2 = rho_2 */
    s->Fx[N + i] = -p->G21 * q2 * c21x - p->w_adh[1] * r2 * swx + r2 * p->gbody[0];
    s->Fy[N + i] = -p->G21 * q2 * c21y - p->w_adh[1] * r2 * swy + r2 * p->gbody[1];
  }

  /* 5. velocities: common velocity (Eq. 18), shifted equilibrium velocity
   * (Eq. 17; a component with rho <= 1e-12 takes u' alone), physical
   * velocity (Eq. 19). */
  const double t1 = p->tau[0], t2 = p->tau[1];
  PAR_FOR
  for (int i = 0; i < N; ++i) {
    s->ueqx[i] = s->ueqy[i] = s->ueqx[N + i] = s->ueqy[N + i] = 0.0;
    s->urx[i] = s->ury[i] = 0.0;
    if (s->type[i] != ORC_FLUID) continue;
    const double r1 = s->rho[i], r2 = s->rho[N + i];
    const double den = r1 / t1 + r2 / t2;
    const double upx = (s->jx[i] / t1 + s->jx[N + i] / t2) / den;
    const double upy = (s->jy[i] / t1 + s->jy[N + i] / t2) / den;
    for (int sg = 0; sg < 2; ++sg) {
      const double r = s->rho[sg * N + i], t = p->tau[sg];
      double ux = upx, uy = upy;
      if (r > 1e-12) {
        ux = upx + t * s->Fx[sg * N + i] / r;
        uy = upy + t * s->Fy[sg * N + i] / r;
      }
      s->ueqx[sg * N + i] = ux;
      s->ueqy[sg * N + i] = uy;
    }
    const double rt = r1 + r2;
    s->urx[i] = (s->jx[i] + s->jx[N + i] + 0.5 * (s->Fx[i] + s->Fx[N + i])) / rt;
    s->ury[i] = (s->jy[i] + s->jy[N + i] + 0.5 * (s->Fy[i] + s->Fy[N + i])) / rt;
  }
  return 0;
}

/*
 * Step 2 of Sec. 4.7 (Sec. 4.5): the liquid marks of this step and the
 * solute shares that nodes which left the liquid set last step deliver now.
 * A fluid node is liquid when its liquid-component density exceeds
 * liquid_frac times the largest such density of the previous step (the
 * maximum of the current step is only known once every node is updated).
 * Cin of a node that was liquid last step (SF_STREAM) is the sum of the
 * shares of its SF_SHARE D2Q5 neighbours: they split their content equally
 * among the neighbours that were liquid when they left.  A ghost node beyond
 * a free outlet neither gives nor takes.
 */
static void mark_liquid(orc_sim* s) {
  const orc_params* p = &s->p;
  const int N = s->N, ns = s->ns, nx = p->nx;
  const double thr = p->liquid_frac * s->rho_max_prev;
  PAR_FOR
  for (int i = 0; i < N; ++i) s->liq[i] = s->type[i] == ORC_FLUID && s->rho[i] > thr;
  PAR_FOR
  for (int i = 0; i < N; ++i) {
    for (int k = 0; k < ns; ++k) s->Cin[k * N + i] = 0.0;
    if (s->sflag[i] != SF_STREAM) continue;
    for (int a = 1; a < 5; ++a) {
      const int j = nb_node(s, i % nx, i / nx, a);
      if (j < 0 || s->sflag[j] != SF_SHARE) continue;
      for (int k = 0; k < ns; ++k) s->Cin[k * N + i] += s->C[k * N + j];
    }
  }
}

/* Sec. 4.1 (and Sec. 2's liquid of A, B, E, F): with sub_species = m, only
 * the other aqueous species are transported in effect; at a liquid node
 * C_m = sub_total * rho_1 - sum of the others.  Applied to the
 * concentrations the step uses (after the amendments of step 3) and to the
 * exported ones. */
static double subtracted(const orc_sim* s, const double* C, int i) {
  double c = s->p.sub_total * s->rho[i];
  for (int k = 0; k < s->ns; ++k)
    if (k != s->p.sub_species) c -= C[k * s->N + i];
  return c;
}

int orc_step(orc_sim* s, int nsteps) {
  const orc_params* p = &s->p;
  const int N = s->N, ns = s->ns, nx = p->nx, ny = p->ny;
  for (int it = 0; it < nsteps; ++it) {
    if (macros(s) != 0) return -1;

    /* 3. liquid marks of this step; maximum rho_1 over fluid nodes, which
     * sets the threshold of the next step.  A node that has just become
     * liquid holds the content it kept, if any; otherwise it starts with no
     * solute (diffusion fills it). */
    mark_liquid(s);
    double rmax_now = 0.0, n_l2g = 0.0, n_g2l = 0.0, mliq = INFINITY;
    const double thr_now = p->liquid_frac * s->rho_max_prev;
#ifdef _OPENMP
#pragma omp parallel for num_threads(s->nthreads) schedule(static) reduction(max : rmax_now) reduction(+ : n_l2g, n_g2l) reduction(min : mliq)
#endif
    for (int i = 0; i < N; ++i) {
      if (s->type[i] == ORC_FLUID && s->rho[i] > rmax_now) rmax_now = s->rho[i];
      /* diagnostic: how close this liquid decision came to its threshold */
      if (s->type[i] == ORC_FLUID && thr_now > 0.0) {
        const double mg = fabs(s->rho[i] - thr_now) / thr_now;
        if (mg < mliq) mliq = mg;
      }
      if (s->liq[i] && (s->sflag[i] == SF_NONE || s->sflag[i] == SF_SHARE))
        for (int k = 0; k < ns; ++k) {
          s->C[k * N + i] = 0.0;
          for (int a = 0; a < 5; ++a) s->g[(k * 5 + a) * N + i] = 0.0;
        }
      if (s->sflag[i] == SF_STREAM && !s->liq[i] && s->type[i] == ORC_FLUID) n_l2g += 1.0;
      if (s->liq[i] && s->sflag[i] != SF_STREAM) n_g2l += 1.0;
    }
    if (mliq < s->margin_liq) s->margin_liq = mliq;
    /* 3b. the subtracted species at liquid nodes (Sec. 4.1) */
    if (p->sub_species >= 0) {
      PAR_FOR
      for (int i = 0; i < N; ++i)
        if (s->liq[i]) s->C[p->sub_species * N + i] = subtracted(s, s->C, i);
    }
    s->led.n_liq_to_gas += n_l2g;   /* counts: exact in any order */
    s->led.n_gas_to_liq += n_g2l;

    /* 6. homogeneous reaction sources at liquid nodes (Eq. 5a, 5c, 27, 28;
     * a first-order A -> B law is also available).  C_C = rho_2 / M_gas. */
    PAR_FOR
    for (int i = 0; i < N; ++i) {
      s->Ss[i] = s->Ss[N + i] = 0.0;
      for (int k = 0; k < ns; ++k) s->Sk[k * N + i] = 0.0;
      if (!s->liq[i]) continue;
      /* types of the D2Q5 neighbours inside the domain: a reaction with a
       * surface mask runs k * factor next to those solids (Sec. 2: R1 is
       * 1000 times faster at the D(s) surface than in the bulk) */
      int nbt = 0;
      for (int a = 1; a < 5; ++a) {
        const int j = nb(s, i % nx, i / nx, a);
        if (j >= 0) nbt |= 1 << s->type[j];
      }
      for (int r = 0; r < p->n_hom; ++r) {
        const int re0 = p->hom_re[r][0], re1 = p->hom_re[r][1];
        const int pr0 = p->hom_pr[r][0], pr1 = p->hom_pr[r][1];
        const double kr = (p->hom_surface[r] & nbt) ? p->hom_k[r] * p->hom_sfac[r] : p->hom_k[r];
        double R = 0.0;
        if (p->hom_kind[r] == ORC_HOM_FIRST_ORDER) {
          R = kr * s->C[re0 * N + i];
        } else if (p->hom_kind[r] == ORC_HOM_BIMOLECULAR) {
          R = kr * s->C[re0 * N + i] * s->C[re1 * N + i];
        } else {
          double cg = s->rho[N + i] / p->hom_Mgas[r];
          if (cg < 0.0) cg = 0.0;
          R = kr * (s->C[re0 * N + i] - s->C[pr0 * N + i] * sqrt(cg) / p->hom_Keq[r]);
          /* Eq. 27: half a mole of gas per mole of R1, moved from the liquid to the gas component */
          s->Ss[i] -= 0.5 * R * p->hom_Mgas[r];
          s->Ss[N + i] += 0.5 * R * p->hom_Mgas[r];
        }
        s->Sk[re0 * N + i] -= R;
        if (re1 >= 0) s->Sk[re1 * N + i] -= R;
        if (pr0 >= 0) s->Sk[pr0 * N + i] += R;
        if (pr1 >= 0) s->Sk[pr1 * N + i] += R;
      }
    }
    for (int i = 0; i < N; ++i) {
      if (!s->liq[i]) continue;
      s->led.mass_src[0] += s->Ss[i];
      s->led.mass_src[1] += s->Ss[N + i];
      for (int k = 0; k < ns; ++k) s->led.sol_src[k] += s->Sk[k * N + i];
    }

    /* 7a. flow collision (Eq. 6, 8) at fluid nodes */
    for (int sg = 0; sg < 2; ++sg) {
      const double om = 1.0 / p->tau[sg];
      PAR_FOR
      for (int i = 0; i < N; ++i) {
        if (s->type[i] != ORC_FLUID) continue;
        const double r = s->rho[sg * N + i];
        const double ux = s->ueqx[sg * N + i], uy = s->ueqy[sg * N + i];
        const double usq = ux * ux + uy * uy;
        for (int a = 0; a < 9; ++a) {
          const double eu = EX[a] * ux + EY[a] * uy;
          const double feq = W9[a] * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
          const double fv = s->f[(sg * 9 + a) * N + i];
          s->fs[(sg * 9 + a) * N + i] = fv - om * (fv - feq) + W9[a] * s->Ss[sg * N + i];
        }
      }
    }
    /* 7b. solute collision (Eq. 20-22) at liquid nodes with the physical velocity u_r */
    for (int k = 0; k < ns; ++k) {
      const double om = 1.0 / p->tau_g[k];
      PAR_FOR
      for (int i = 0; i < N; ++i) {
        if (!s->liq[i]) continue;
        const double c = s->C[k * N + i];
        for (int a = 0; a < 5; ++a) {
          const double J = J_of(p, k, a);
          const double geq = c * (J + 0.5 * (EX[a] * s->urx[i] + EY[a] * s->ury[i]));
          const double gv = s->g[(k * 5 + a) * N + i];
          s->gs[(k * 5 + a) * N + i] = gv - om * (gv - geq) + J * s->Sk[k * N + i];
        }
      }
    }

    /* 8. heterogeneous link flux per reaction at liquid nodes, from the
     * node's own concentration (halfway-wall Robin form, Eq. 31 / A2; Eq. 29
     * read with the same sign convention, so a positive flux consumes the
     * reactant).  Irreversible reactions cannot run backwards. */
    for (int r = 0; r < p->n_het; ++r) {
      PAR_FOR
      for (int i = 0; i < N; ++i) {
        double v = 0.0;
        if (s->liq[i]) {
          v = s->kap[r] * (s->C[p->het_reactant[r] * N + i] - p->het_Ceq[r]);
          if (p->het_irrev[r] && v < 0.0) v = 0.0;
        }
        s->Phi[r * N + i] = v;
      }
    }

    /* 9. volume of pixel (Eq. 33, 35).  A reactive solid node sums the fluxes
     * of its D2Q5 links to liquid nodes (directions 1..4, reactions in order);
     * CONSUMES reactions remove solid, MINERAL reactions add Vbar*Phi (a
     * negative flux dissolves).  A liquid node accumulates the precipitate of
     * GROWS reactions on its links to reactive solid.  A solid node whose
     * volume reaches 0 becomes fluid; a liquid node whose precipitate volume
     * reaches 1 becomes SOLID_F. */
    PAR_FOR
    for (int i = 0; i < N; ++i) {
      s->tnext[i] = s->type[i];
      s->dvt[i] = 0;
      const int t = s->type[i];
      const int x = i % nx, y = i / nx;
      if (t == ORC_SOLID_D || t == ORC_SOLID_F) {
        double dv = 0.0;
        int touched = 0;
        for (int a = 1; a < 5; ++a) {
          const int j = nb(s, x, y, a);
          if (j < 0 || s->type[j] != ORC_FLUID || !s->liq[j]) continue;
          for (int r = 0; r < p->n_het; ++r) {
            if (!(p->het_surface[r] & (1 << t))) continue;
            if (p->het_mode[r] == ORC_HET_CONSUMES) { dv -= p->het_mvol[r] * s->Phi[r * N + j]; touched = 1; }
            else if (p->het_mode[r] == ORC_HET_MINERAL) { dv += p->het_mvol[r] * s->Phi[r * N + j]; touched = 1; }
          }
        }
        if (touched) {
          s->V[i] += dv;
          s->dvv[i] = dv;
          s->dvt[i] = 1;
        }
        if (s->V[i] <= 0.0) {
          int nf = 0;
          for (int a = 1; a < 9; ++a) {
            const int j = nb_node(s, x, y, a);
            if (j >= 0 && s->type[j] == ORC_FLUID) ++nf;
          }
          if (nf > 0) s->tnext[i] = ORC_FLUID;
        }
      } else if (t == ORC_FLUID && s->liq[i]) {
        double dv = 0.0;
        int touched = 0;
        for (int a = 1; a < 5; ++a) {
          const int j = nb(s, x, y, a);
          if (j < 0) continue;
          const int tj = s->type[j];
          if (tj != ORC_SOLID_D && tj != ORC_SOLID_F) continue;
          for (int r = 0; r < p->n_het; ++r)
            if ((p->het_surface[r] & (1 << tj)) && p->het_mode[r] == ORC_HET_GROWS) {
              dv += p->het_mvol[r] * s->Phi[r * N + i];
              touched = 1;
            }
        }
        if (touched) {
          s->V[i] += dv;
          s->dvv[i] = dv;
          s->dvt[i] = 1;
        }
        if (s->V[i] >= 1.0) s->tnext[i] = ORC_SOLID_F;
      }
    }
    for (int i = 0; i < N; ++i)
      if (s->dvt[i]) {
        s->led.vol_dv += s->dvv[i];
        /* diagnostic: distance of a changed volume from its threshold (0 or 1) */
        const double mg = s->type[i] == ORC_FLUID ? fabs(s->V[i] - 1.0) : fabs(s->V[i]);
        if (mg < s->margin_vol) s->margin_vol = mg;
      }

    /* 10. amendments for nodes whose status changed (Sec. 4.5), applied to the
     * post-collision distributions before they stream, using this step's
     * pre-amendment moments.  All of them conserve mass and solute or put the
     * difference in the ledger:
     *  (a) stranded populations of a node that became SOLID_F last step are
     *      shared equally by its fluid D2Q9 neighbours, at rest;
     *  (b) the solute of a node that is not liquid now (it left the liquid
     *      set, to gas or to solid) goes in equal shares, at rest, to the
     *      D2Q5 neighbours that are liquid now; they take the shares one step
     *      later (so that every node involved is at most one link away); a
     *      node with no such neighbour keeps its content until it has one;
     *  (c) a node freed by dissolution this step starts, next step, at rest
     *      with the mean density of its fluid D2Q9 neighbours (the added mass
     *      is booked);
     *  (d) a node that has just turned liquid starts with the solute it kept,
     *      if any, else with none (done with the marks above); diffusion
     *      fills it. */
    PAR_FOR
    for (int i = 0; i < N; ++i) {
      const int x = i % nx, y = i / nx;
      if (s->type[i] == ORC_FLUID) {
        double don[2] = {0.0, 0.0};
        for (int a = 1; a < 9; ++a) {
          const int j = nb_node(s, x, y, a);
          if (j < 0 || !s->stranded[j]) continue;
          int m = 0;
          for (int b = 1; b < 9; ++b) {
            const int q = nb_node(s, j % nx, j / nx, b);
            if (q >= 0 && s->type[q] == ORC_FLUID) ++m;
          }
          for (int sg = 0; sg < 2; ++sg) don[sg] += s->rho[sg * N + j] / m;
        }
        for (int sg = 0; sg < 2; ++sg)
          if (don[sg] != 0.0)
            for (int a = 0; a < 9; ++a) s->fs[(sg * 9 + a) * N + i] += W9[a] * don[sg];
      }
      if (s->liq[i] && s->sflag[i] == SF_STREAM)
        for (int k = 0; k < ns; ++k)
          if (s->Cin[k * N + i] != 0.0)
            for (int a = 0; a < 5; ++a) s->gs[(k * 5 + a) * N + i] += J_of(p, k, a) * s->Cin[k * N + i];
    }
    /* donors with nobody to take their content */
    for (int i = 0; i < N; ++i) {
      if (!s->stranded[i]) continue;
      const int x = i % nx, y = i / nx;
      int m = 0;
      for (int b = 1; b < 9; ++b) {
        const int q = nb_node(s, x, y, b);
        if (q >= 0 && s->type[q] == ORC_FLUID) ++m;
      }
      if (m == 0)
        for (int sg = 0; sg < 2; ++sg) s->led.mass_rem[sg] += s->rho[sg * N + i];
    }
    PAR_FOR
    for (int i = 0; i < N; ++i) {
      const int x = i % nx, y = i / nx;
      /* (b) a node that holds solute but is not liquid now (it left the
       * liquid set, or kept its content earlier) passes its content, plus
       * the shares it received, to the D2Q5 neighbours that are liquid now:
       * its slots carry, at rest, one equal share per such neighbour, which
       * they take next step.  With no liquid neighbour it keeps the content
       * at rest.  Nothing is dropped. */
      s->snext[i] = s->liq[i] ? SF_STREAM : SF_NONE;
      if (!s->liq[i] && (s->sflag[i] == SF_STREAM || s->sflag[i] == SF_HOLD) && ns > 0) {
        int m = 0;
        for (int b = 1; b < 5; ++b) {
          const int q = nb_node(s, x, y, b);
          if (q >= 0 && s->liq[q]) ++m;
        }
        int any = 0;
        for (int k = 0; k < ns; ++k) {
          double c = s->C[k * N + i];
          if (s->sflag[i] == SF_STREAM) c += s->Cin[k * N + i];
          if (m > 0) c = c / m;
          if (c != 0.0) any = 1;
          for (int a = 0; a < 5; ++a) s->gn[(k * 5 + a) * N + i] = J_of(p, k, a) * c;
        }
        if (any) s->snext[i] = m > 0 ? SF_SHARE : SF_HOLD;
      }
    }
    /* (c) dissolved nodes: mean density of fluid neighbours */
    PAR_FOR
    for (int i = 0; i < N; ++i) {
      s->rbar[i] = s->rbar[N + i] = 0.0;
      if (!(s->type[i] != ORC_FLUID && s->tnext[i] == ORC_FLUID)) continue;
      const int x = i % nx, y = i / nx;
      double sum[2] = {0.0, 0.0};
      int m = 0;
      for (int a = 1; a < 9; ++a) {
        const int j = nb_node(s, x, y, a);
        if (j < 0 || s->type[j] != ORC_FLUID) continue;
        sum[0] += s->rho[j];
        sum[1] += s->rho[N + j];
        ++m;
      }
      for (int sg = 0; sg < 2; ++sg) s->rbar[sg * N + i] = sum[sg] / m;
    }
    for (int i = 0; i < N; ++i) {
      if (!(s->type[i] != ORC_FLUID && s->tnext[i] == ORC_FLUID)) continue;
      for (int sg = 0; sg < 2; ++sg) s->led.mass_inj[sg] += s->rbar[sg * N + i];
      s->led.n_dissolved += 1.0;
      s->led.vol_clip += s->V[i];
    }

    /* 11. push streaming (Eq. 6, 20, left-hand sides) with the masks of this
     * step.  Flow: halfway bounce-back off any non-fluid neighbour or
     * non-periodic boundary.  Solute: the liquid set only; bounce-back off gas
     * (the no-flux liquid-gas interface of Eq. 26) and solid, minus the
     * reactant's link flux and plus the product's on reactive solid.
     * Free outlet: a population sent into a fluid (liquid) ghost node leaves
     * the lattice, and the ghost row sends the top row what its model node
     * sends the row below it. */
    for (int sg = 0; sg < 2; ++sg)
      for (int a = 0; a < 9; ++a) {
        PAR_FOR
        for (int i = 0; i < N; ++i) {
          if (s->type[i] != ORC_FLUID) continue;
          const int j = nb(s, i % nx, i / nx, a);
          const double v = s->fs[(sg * 9 + a) * N + i];
          if (j >= 0 && s->type[j] == ORC_FLUID) {
            if (!crosses_outlet(s, i / nx, a)) s->fn[(sg * 9 + a) * N + j] = v;
          } else {
            s->fn[(sg * 9 + OPP[a]) * N + i] = v;
          }
        }
      }
    if (p->outlet_top)
      for (int i = (ny - 1) * nx; i < N; ++i) {
        if (s->type[i] != ORC_FLUID) continue;
        for (int a = 1; a < 9; ++a) {
          if (EY[a] >= 0) continue;
          const int j = nb(s, i % nx, ny - 1, OPP[a]);  /* the ghost sender's model node */
          if (j < 0 || s->type[j] != ORC_FLUID) continue;  /* bounced back above */
          for (int sg = 0; sg < 2; ++sg) s->fn[(sg * 9 + a) * N + i] = s->fs[(sg * 9 + a) * N + j];
        }
      }
    for (int k = 0; k < ns; ++k)
      for (int a = 0; a < 5; ++a) {
        PAR_FOR
        for (int i = 0; i < N; ++i) {
          if (!s->liq[i]) continue;
          const int j = nb(s, i % nx, i / nx, a);
          double v = s->gs[(k * 5 + a) * N + i];
          if (j >= 0 && s->liq[j]) {
            if (!crosses_outlet(s, i / nx, a)) s->gn[(k * 5 + a) * N + j] = v;
            continue;
          }
          if (j >= 0 && (s->type[j] == ORC_SOLID_D || s->type[j] == ORC_SOLID_F)) {
            for (int r = 0; r < p->n_het; ++r) {
              if (!(p->het_surface[r] & (1 << s->type[j]))) continue;
              if (p->het_reactant[r] == k) v -= s->Phi[r * N + i];
              if (p->het_product[r] == k) v += s->Phi[r * N + i];
            }
          }
          s->gn[(k * 5 + OPP[a]) * N + i] = v;
        }
        /* the exchange with the solid, booked in node order */
        for (int i = 0; i < N; ++i) {
          if (!s->liq[i]) continue;
          const int j = nb(s, i % nx, i / nx, a);
          if (j < 0 || s->liq[j] || (s->type[j] != ORC_SOLID_D && s->type[j] != ORC_SOLID_F)) continue;
          for (int r = 0; r < p->n_het; ++r) {
            if (!(p->het_surface[r] & (1 << s->type[j]))) continue;
            if (p->het_reactant[r] == k) s->led.sol_het[k] -= s->Phi[r * N + i];
            if (p->het_product[r] == k) s->led.sol_het[k] += s->Phi[r * N + i];
          }
        }
      }
    if (p->outlet_top)
      for (int i = (ny - 1) * nx; i < N; ++i) {
        if (!s->liq[i]) continue;
        /* D2Q5: the ghost above a top node models the node itself */
        for (int k = 0; k < ns; ++k) s->gn[(k * 5 + 4) * N + i] = s->gs[(k * 5 + 4) * N + i];
      }
    PAR_FOR
    for (int i = 0; i < N; ++i) {
      if (!(s->type[i] != ORC_FLUID && s->tnext[i] == ORC_FLUID)) continue;
      for (int sg = 0; sg < 2; ++sg)
        for (int a = 0; a < 9; ++a) s->fn[(sg * 9 + a) * N + i] = W9[a] * s->rbar[sg * N + i];
    }

    /* advance the state: masks, stranded flags, volumes of dissolved nodes */
    for (int i = 0; i < N; ++i)
      if (s->type[i] == ORC_FLUID && s->tnext[i] == ORC_SOLID_F) s->led.n_precipitated += 1.0;
    PAR_FOR
    for (int i = 0; i < N; ++i) {
      const int told = s->type[i], tnew = s->tnext[i];
      if (told != ORC_FLUID && tnew == ORC_FLUID) s->V[i] = 0.0;
      s->stranded[i] = (told == ORC_FLUID && tnew == ORC_SOLID_F);
      s->sflag[i] = s->snext[i];
      s->type[i] = (uint8_t)tnew;
    }
    double* t;
    t = s->f; s->f = s->fn; s->fn = t;
    t = s->g; s->g = s->gn; s->gn = t;
    s->rho_max_prev = rmax_now;
    s->step += 1;
    s->led.steps += 1.0;
  }
  return 0;
}

void orc_fields(orc_sim* s, double* rho1, double* rho2, double* ux, double* uy,
                double* C, uint8_t* type, uint8_t* liquid, double* V,
                orc_ledger* ledger, double* rho_max_prev) {
  const int N = s->N;
  /* the export reuses sub-steps 1-5 without changing the state, except that
   * it may count psi clamps; keep the ledger as it was */
  orc_ledger keep = s->led;
  macros(s);
  mark_liquid(s);
  s->led = keep;
  for (int i = 0; i < N; ++i) {
    if (rho1) rho1[i] = s->rho[i];
    if (rho2) rho2[i] = s->rho[N + i];
    if (ux) ux[i] = s->urx[i];
    if (uy) uy[i] = s->ury[i];
    if (type) type[i] = s->type[i];
    if (liquid) liquid[i] = s->liq[i];
    if (V) V[i] = s->V[i];
  }
  /* solute content after the shares in transit are delivered: a node holding
   * a share in transit reports none, its receivers report it */
  if (C)
    for (int k = 0; k < s->ns; ++k)
      for (int i = 0; i < N; ++i) {
        const int sf = s->sflag[i];
        double c = 0.0;
        if (sf == SF_STREAM) c = s->C[k * N + i] + s->Cin[k * N + i];
        else if (sf == SF_HOLD) c = s->C[k * N + i];
        C[k * N + i] = c;
      }
  /* the subtracted species at liquid nodes, from the exported others */
  if (C && s->p.sub_species >= 0)
    for (int i = 0; i < N; ++i)
      if (s->liq[i]) C[s->p.sub_species * N + i] = subtracted(s, C, i);
  if (ledger) *ledger = s->led;
  if (rho_max_prev) *rho_max_prev = s->rho_max_prev;
}

void orc_state(orc_sim* s, double* f, double* g, uint8_t* flags) {
  const int N = s->N;
  if (f) memcpy(f, s->f, sizeof(double) * 18 * (size_t)N);
  if (g) memcpy(g, s->g, sizeof(double) * 5 * (size_t)s->ns * N);
  if (flags)
    for (int i = 0; i < N; ++i)
      flags[i] = (uint8_t)(s->sflag[i] | (s->stranded[i] << 2));
}

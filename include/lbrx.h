/*
 * lbrx - coupled reactive-transport lattice Boltzmann step on one MI355X.
 *
 * The library advances the two-phase multi-mixture pore-scale model of Chen,
 * Kang, Tang, Robinson, He and Tao (arXiv:1410.3464) by whole time steps on
 * the GPU.  One step is the procedure of Sec. 4.7 (Steps 1-5):
 *   - two D2Q9 flow components (liquid mixture and gas), pseudopotential
 *     forces (Eq. 11-16), Shan-Chen velocity shift (Eq. 17-19), forced BGK
 *     collision (Eq. 6, 8), push streaming with halfway bounce-back;
 *   - D2Q5 solute lattices in the liquid only (Eq. 20-24, 26) with
 *     homogeneous reaction sources (Eq. 5, 27, 28) and heterogeneous surface
 *     fluxes at liquid-solid links (Eq. 29-31, A2);
 *   - the volume-of-pixel solid update (Eq. 32-35) and the amendments for
 *     nodes whose status changes (Sec. 4.5).
 *
 * Conventions
 *   - Arrays are row-major with index y*nx + x; x is the fast axis.
 *   - All pointers passed in are host pointers.  lbrx_create copies what it
 *     needs; the caller keeps ownership of everything it passes.
 *   - The context owns all device memory; lbrx_destroy releases it.
 *   - A context is not thread-safe.  Distinct contexts are independent.
 *   - Errors are returned as status codes; lbrx_last_error() gives a message.
 *     Nothing unwinds across this interface.
 */
#ifndef LBRX_H
#define LBRX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBRX_ABI_VERSION 6u
#define LBRX_MAX_SPECIES 8
#define LBRX_MAX_RXN 8

typedef struct lbrx_ctx lbrx_ctx;
typedef struct lbrx_batch lbrx_batch;

typedef enum {
  LBRX_OK = 0,
  LBRX_E_INVAL = 1,    /* invalid argument or parameter                        */
  LBRX_E_NOMEM = 2,    /* device allocation failed                             */
  LBRX_E_DEVICE = 3,   /* a HIP call failed                                    */
  LBRX_E_UNSTABLE = 4, /* the run produced a negative/NaN density, or b rho/4>=1 */
  LBRX_E_STATE = 5     /* the context already failed; only destroy is allowed  */
} lbrx_status;

/* Storage and arithmetic precision of the populations.  Solid volumes and the
 * balance ledger are FP64 in every mode.
 *   LBRX_F64, LBRX_F32: populations stored and updated in that precision.
 *   LBRX_F16DEV, LBRX_BF16DEV: populations stored as 16-bit (IEEE half or
 *     bfloat16) deviations from their equilibrium at rest for a coded
 *     reference density (concentration) of the node that reads them, times a
 *     power-of-two scale; all arithmetic in FP32.  Half the population bytes
 *     of LBRX_F32; the accuracy against FP64 is stated per field in the
 *     design notes. */
typedef enum { LBRX_F64 = 0, LBRX_F32 = 1, LBRX_F16DEV = 2, LBRX_BF16DEV = 3 } lbrx_precision;

/* node types (Fig. 2): fluid, inert solid, dissolvable solid D(s), precipitate F(s) */
enum { LBRX_FLUID = 0, LBRX_SOLID_INERT = 1, LBRX_SOLID_D = 2, LBRX_SOLID_F = 3 };

/* Homogeneous reactions (Sec. 2, Eq. 5; Sec. 4.2, Eq. 27-28).
 *   FIRST_ORDER:  R = k C[re0]
 *   R1_GAS:       R = k (C[re0] - C[pr0] sqrt(rho2 / M_gas) / K_eq)   (Eq. 5a)
 *                 and half a mole of gas per mole of R moves from flow
 *                 component 1 to component 2 (S_1 = -R M_gas/2, S_2 = +R M_gas/2)
 *   BIMOLECULAR:  R = k C[re0] C[re1]                                  (Eq. 5c)
 * Each reactant index loses R and each product index gains R; -1 = none.
 * Surface enhancement (Sec. 2: R1 runs 1000 times faster at the D(s) surface
 * than in the bulk): at a liquid node with at least one D2Q5 neighbour whose
 * type bit is in `surface` ((1<<LBRX_SOLID_INERT), (1<<LBRX_SOLID_D),
 * (1<<LBRX_SOLID_F)), k is multiplied by `surface_factor` (> 0, finite).
 * surface = 0 disables it (surface_factor is then ignored).  Node types are
 * those at the start of the step. */
enum { LBRX_HOM_FIRST_ORDER = 0, LBRX_HOM_R1_GAS = 1, LBRX_HOM_BIMOLECULAR = 2 };
typedef struct {
  int32_t kind;
  int32_t re[2], pr[2];
  double k, K_eq, M_gas;
  uint32_t surface;
  double surface_factor;
} lbrx_hom_rxn;

/* Heterogeneous surface reactions (Sec. 4.3-4.4, Eq. 29-35, A2).  On every D2Q5
 * link from a liquid node to a solid node whose type bit is in `surface`
 * ((1<<LBRX_SOLID_D) and/or (1<<LBRX_SOLID_F)) the reactant loses, and the
 * product gains, the link flux
 *     Phi = 2 D k (C_reactant - C_eq) / (2 D + k)
 * (halfway-wall Robin form of D dC/dn = k (C_wall - C_eq); D from Eq. 24 of the
 * reactant; clamped at >= 0 when `irreversible`).  Volume of pixel:
 *   CONSUMES: the solid node loses molar_volume * Phi           (R2, Eq. 33)
 *   GROWS:    the liquid node's precipitate volume gains molar_volume * Phi;
 *             at 1 the node becomes LBRX_SOLID_F                 (R4, Eq. 35)
 *   MINERAL:  the solid node gains molar_volume * Phi (negative Phi dissolves;
 *             Eq. A2).
 * A solid node whose volume reaches 0 becomes fluid. */
enum { LBRX_HET_CONSUMES = 0, LBRX_HET_GROWS = 1, LBRX_HET_MINERAL = 2 };
typedef struct {
  int32_t reactant, product;
  uint32_t surface;
  int32_t mode;
  int32_t irreversible;
  double k, C_eq, molar_volume;
} lbrx_het_rxn;

typedef struct {
  uint32_t abi_version;  /* must be LBRX_ABI_VERSION */
  int32_t nx, ny;        /* lattice size, each >= 1 */
  uint32_t periodic;     /* bit 0: x periodic, bit 1: y periodic; a non-periodic
                            side is a halfway bounce-back wall just outside the domain,
                            except that bit 2 makes the side beyond y = ny - 1 a free
                            outlet with zero gradient of every variable (Sec. 5.1): a
                            ghost row repeating the top row's type, potentials,
                            concentrations and post-collision populations.  Bit 2
                            needs bit 1 clear, ny >= 2 and FP64 or FP32 storage
                            (LBRX_E_INVAL otherwise); other bits must be clear */
  int32_t precision;     /* lbrx_precision */
  double tau[2];         /* flow relaxation times, > 1/2 (Eq. 6, 10) */
  double w_adh[2];       /* fluid-solid interaction strengths (Eq. 16) */
  double gbody[2];       /* body acceleration (x, y); the force on component s is rho_s g */
  double a, b, R, T;     /* Carnahan-Starling EOS of component 1 (Eq. 12) */
  double G11, G12, G21;  /* interaction strengths (Eq. 11, 14); G22 = 0 */
  double a0, rho10, rho20; /* phi_1 = 1 - exp(-rho2/rho20), phi_2 = a0 - exp(-rho1/rho10) (Eq. 15);
                              a non-positive rho10 / rho20 switches that phi off */
  double liquid_frac;    /* liquid iff rho1 > liquid_frac * max rho1 (Sec. 4.5); in [0,1) */
  int32_t n_species;     /* 0..LBRX_MAX_SPECIES aqueous species on D2Q5 */
  double tau_g[LBRX_MAX_SPECIES]; /* > 1/2 (Eq. 20, 24) */
  double J0[LBRX_MAX_SPECIES];    /* rest fraction in [0,1) (Eq. 22) */
  int32_t n_hom;
  lbrx_hom_rxn hom[LBRX_MAX_RXN];
  int32_t n_het;
  lbrx_het_rxn het[LBRX_MAX_RXN];
  /* initial state, host arrays of nx*ny (C0: n_species*nx*ny), copied at create */
  const uint8_t* node_type; /* LBRX_FLUID .. LBRX_SOLID_F */
  const double* V0;         /* solid volume (> 0 at D/F nodes), precipitate fraction in
                               [0,1) at fluid nodes; NULL: 1 at D/F nodes, 0 elsewhere */
  const double* rho1;       /* > 0 at fluid nodes */
  const double* rho2;       /* >= 0 at fluid nodes */
  const double* C0;         /* used at nodes that start liquid; may be NULL if n_species == 0 */
  /* work decomposition: rows per work item of the step kernel (each item is
     62 columns by seg_rows rows, one 64-lane wavefront that also pulls the
     column on either side), 1..30; 0 picks 16, or 8, 4 or 2 for a lattice
     whose items would not fill the device.  It changes the speed and not
     the fields (the balance sums, added per item, to rounding). */
  int32_t seg_rows;
  /* effective mass psi_1 = sqrt(psi_prefactor (p_EOS - rho1/3) / G11) (Eq. 13).
     0 selects 2, the value for which the weights of Eq. 11 reproduce the EOS
     of Eq. 12; 6 is the prefactor printed in Eq. 13.  Otherwise > 0. */
  double psi_prefactor;
  /* device memory: every device buffer of the context (and of a batch built
     on it) comes from dev_alloc(bytes, alloc_user) and goes back through
     dev_free(ptr, alloc_user), e.g. a framework's caching allocator; both
     NULL: hipMalloc / hipFree.  The memory must be device memory of the
     current device, 256-byte aligned; dev_alloc returns NULL on failure
     (LBRX_E_NOMEM).  Buffers are returned only after the context's stream
     has drained.  Set both or neither. */
  void* (*dev_alloc)(uint64_t bytes, void* user);
  void (*dev_free)(void* ptr, void* user);
  void* alloc_user;
  /* Sec. 4.1: the aqueous species (0 .. n_species - 1) whose concentration at
     a liquid node is the total liquid concentration, subtract_total x rho1,
     minus the other species (its own transport does not enter what it is;
     its balance entries are not a conservation record); -1: none.
     subtract_total > 0 when a species is subtracted (the paper takes the
     total from the liquid's composition, which needs its molar masses). */
  int32_t subtract_species;
  double subtract_total;
} lbrx_params;

/* Cumulative balances, FP64.  With M_s the total of component s and S_k the
 * total of species k (over nodes that carry them):
 *   M_s(n) = M_s(0) + mass_src[s] + mass_inj[s] - mass_rem[s]
 *   S_k(n) = S_k(0) + sol_src[k] + sol_het[k] - sol_rem[k]
 *   sum V(n) = sum V(0) + vol_dv - vol_clip                                 */
typedef struct {
  double mass_src[2];   /* homogeneous flow sources (Eq. 27) */
  double mass_inj[2];   /* mass given to nodes freed by dissolution */
  double mass_rem[2];   /* displaced mass that found no fluid neighbour */
  double sol_src[LBRX_MAX_SPECIES]; /* homogeneous solute sources (Eq. 28) */
  double sol_het[LBRX_MAX_SPECIES]; /* net surface exchange (Eq. 29-31) */
  double sol_rem[LBRX_MAX_SPECIES]; /* solute dropped: always 0 (a node leaving the liquid passes its
                                       content to its liquid D2Q5 neighbours, or keeps it at rest) */
  double vol_dv;        /* all volume-of-pixel increments (Eq. 33, 35) */
  double vol_clip;      /* sum of the non-positive volumes of removed solid nodes */
  double n_psi_clamp;   /* negative psi arguments clamped to zero */
  double n_dissolved, n_precipitated, n_liq_to_gas, n_gas_to_liq;
  double steps;
} lbrx_ledger;

/* Host output buffers of nx*ny (C: n_species*nx*ny) for lbrx_fields.  The
 * fields wanted are selected by the non-NULL pointers: any may be NULL, and a
 * call that asks for none of rho1, rho2, ux, uy, C and liquid runs no read-out
 * kernel.  Values describe the state after the steps taken so far, as the
 * next step starts from it (its populations streamed): rho at nodes carrying
 * flow populations, u the physical velocity of Eq. 19 at fluid nodes, C the
 * solute each node holds once the shares in transit from nodes that left the
 * liquid are delivered (Sec. 4.5), V solid / precipitate volume, type the node
 * type, liquid the liquid mark the next step takes (rho1 above liquid_frac
 * times the last step's maximum, Sec. 4.5). */
typedef struct {
  double* rho1;
  double* rho2;
  double* ux;
  double* uy;
  double* C;
  double* V;
  uint8_t* type;
  uint8_t* liquid;
  lbrx_ledger* ledger;
  double* rho_max;      /* 1 value: max rho1 of the last step (liquid threshold source) */
} lbrx_fields_out;

/* Creates a context on the current HIP device.  `hip_stream` is a hipStream_t
 * the context enqueues all its work on (NULL: the context creates its own).
 * Returns LBRX_E_INVAL for invalid parameters (message in *out's last error is
 * not available: *out is NULL; see lbrx_create_error()). */
lbrx_status lbrx_create(const lbrx_params* params, void* hip_stream, lbrx_ctx** out);

/* Message of the last failed lbrx_create on this thread. */
const char* lbrx_create_error(void);

/* Enqueues n_steps >= 0 coupled steps on the context's stream and returns
 * without waiting.  A numerical failure inside these steps is reported by the
 * next lbrx_sync / lbrx_fields as LBRX_E_UNSTABLE. */
lbrx_status lbrx_step(lbrx_ctx* ctx, int64_t n_steps);

/* Waits for the context's stream and reports a sticky numerical failure. */
lbrx_status lbrx_sync(lbrx_ctx* ctx);

/* Waits, then fills the caller's host buffers (FP64 whatever the precision).
 * The first call on a context allocates its device read-out staging
 * ((5 + n_species) planes of pitch * ny doubles plus the summed balances),
 * which the context keeps until lbrx_destroy. */
lbrx_status lbrx_fields(lbrx_ctx* ctx, lbrx_fields_out* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture elsewhere on the device, tight serving loops, harnesses that forbid
 * allocation): lbrx_fields without any device allocation or free.  The
 * read-out kernels stage their output in one static device array per GPU of
 * LBRX_NOALLOC_SCRATCH_BYTES bytes (the library's; it exists on every GPU the
 * library runs on until the process ends).  A context whose read-out needs
 * more, (5 + n_species) * pitch * ny + 38 doubles with pitch = nx rounded up
 * to 64, gets LBRX_E_INVAL and a message (use lbrx_fields for it).  Outputs,
 * arguments and errors are those of lbrx_fields.  Every call on one GPU
 * shares that GPU's array: the call clears what must start at zero, and
 * calls that overlap on one GPU (another thread, another context's stream)
 * race and must be serialised by the caller. */
#define LBRX_NOALLOC_SCRATCH_BYTES (128ull << 20)
lbrx_status lbrx_fields_noalloc(lbrx_ctx* ctx, lbrx_fields_out* out);

/* Checkpoint and resume of the whole simulation state, so that a run of the
 * Sec. 4.7 procedure can stop and continue: the populations, node status
 * words (types, liquid marks, neighbour masks, 16-bit reference codes), solid
 * volumes, balance records, the lagged rho_max of Sec. 4.5 and the step
 * count.  The parameters are not part of the state.
 *   lbrx_state_bytes: size of the state of `ctx` in bytes (into *bytes).
 *   lbrx_save_state:  synchronises, then copies the state into the caller's
 *     host buffer `buf` of `bytes` (>= lbrx_state_bytes); LBRX_E_INVAL if too
 *     small; a failed context cannot be saved (its sticky error is returned).
 *   lbrx_load_state:  replaces the state of `ctx` by a saved one.  `ctx` must
 *     have been created with the same lattice size, boundaries (`periodic`
 *     bits, the free outlet included), precision, species count and seg_rows
 *     (LBRX_E_INVAL otherwise, state unchanged); other parameters may differ
 *     and apply from the next step.  Enqueued on the
 *     context's stream after its pending work; returns after the copy.
 * Loading a state saved after N steps and stepping M more gives fields bit
 * for bit equal to N + M steps without the checkpoint. */
lbrx_status lbrx_state_bytes(const lbrx_ctx* ctx, uint64_t* bytes);
lbrx_status lbrx_save_state(lbrx_ctx* ctx, void* buf, uint64_t bytes);
lbrx_status lbrx_load_state(lbrx_ctx* ctx, const void* buf, uint64_t bytes);

/* Steps taken so far. */
int64_t lbrx_step_count(const lbrx_ctx* ctx);

/* The hipStream_t the context enqueues on (for events around lbrx_step). */
void* lbrx_stream(const lbrx_ctx* ctx);

/* Releases the context and its device memory.  NULL is a no-op. */
lbrx_status lbrx_destroy(lbrx_ctx* ctx);

/* Message for the last failure of this context ("" if none). */
const char* lbrx_last_error(const lbrx_ctx* ctx);

/* Static name of a status code. */
const char* lbrx_status_string(lbrx_status s);

/* ---- batches: several simulations advanced by one launch per step -------
 * Not a method of the paper: a way to run many independent (small) problems,
 * each still the coupled step of Sec. 4.7, with one kernel launch per step
 * for all of them.  Results are identical to stepping each context alone.
 *
 * Creates a batch of n >= 1 distinct contexts that share device, stream,
 * precision and species count (LBRX_E_INVAL otherwise; also for more than
 * 4095 contexts or a context of more than 131072 work items).  The batch
 * keeps pointers to the contexts, which must outlive it; it copies nothing
 * of their state.  A context may still be stepped, read and synced on its
 * own; a batch notices and rebuilds its tables. */
lbrx_status lbrx_batch_create(lbrx_ctx* const* ctxs, int n, lbrx_batch** out);

/* Enqueues n_steps >= 0 steps of every context of the batch on their stream
 * (one launch per step; runs of 30 steps replay a captured HIP graph) and
 * returns without waiting.  Numerical failures are reported per context by
 * lbrx_sync / lbrx_fields. */
lbrx_status lbrx_batch_step(lbrx_batch* batch, int64_t n_steps);

/* Message for the last failure of this batch. */
const char* lbrx_batch_last_error(const lbrx_batch* batch);

/* Waits for the batch's own launches (not for work queued after them on the
 * stream) and releases the batch (not the contexts).  NULL is a no-op. */
lbrx_status lbrx_batch_destroy(lbrx_batch* batch);

#ifdef __cplusplus
}
#endif
#endif

/*
 * grmhd.h -- C ABI of libgrmhd.so: one Runge-Kutta stage of the 3+1 Valencia
 * GRMHD finite-volume update on MeshBlocks, on one MI355X (gfx950), FP64.
 *
 * Method (arXiv 2409.10384):
 *   conserved variables D~, S~_i, tau~ from (rho, W v^i, P, B^i)   Sec. II, Eq. 7-8
 *   fluxes                                                         Sec. II, Eq. 9
 *   metric source terms                                            Sec. II, Eq. 10
 *   reconstruction of rho, W v^i, P (donor cell, PLM, PPM4, PPMX,
 *   WENOZ); HLLE/LLF Riemann solvers                              Sec. III-B
 *   upwind constrained transport of the face field B~               Sec. III-B
 *   atmosphere floors, FOFC, FOFC+DMP (relaxed maximum principle)   Sec. III-C, Eq. 11-12
 *   conservative-to-primitive inversion (Kastaun et al. master
 *   function in mu = 1/(hW)), ideal gas and hybrid piecewise
 *   polytrope EOS                                                   Sec. III-D
 *
 * Conventions for every entry point:
 *   - Memory: every array pointer is DEVICE memory owned by the caller (for
 *     instance a torch tensor).  The library never allocates on these paths;
 *     it borrows the pointers for the duration of the enqueued work.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  Every call is asynchronous with respect to the host.
 *   - Errors: 0 on success; a negative GRMHD_E* code for a synchronous
 *     argument or launch error (nothing is enqueued after an argument error).
 *     Per-cell physics failures are never errors: they follow the atmosphere
 *     policy of Sec. III-C and are reported in the per-cell flag bits below.
 *   - Layout: structure of arrays, double precision, index
 *     ((k * sy + j) * sx + i), i fastest, padded with ng ghost layers:
 *     sx = nx + 2 ng, sy = ny + 2 ng, sz = nz + 2 ng.  Face arrays of
 *     direction d carry one more entry along d (face i = lower face of cell i):
 *     x-faces (sz, sy, sx+1), y-faces (sz, sy+1, sx), z-faces (sz+1, sy, sx).
 */
#ifndef GRMHD_H
#define GRMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRMHD_OK 0
#define GRMHD_EINVAL (-1)       /* bad argument (size, pointer, option) */
#define GRMHD_EHIP (-2)         /* a HIP launch or runtime call failed */
#define GRMHD_EUNSUPPORTED (-3) /* option not implemented */
#define GRMHD_ETOOBIG (-4)      /* input larger than a fixed-size library workspace */

/* per-cell flag bits (uint16) */
#define GRMHD_F_C2P_FAIL        (1u << 0)  /* inversion failed -> atmosphere */
#define GRMHD_F_DFLOOR          (1u << 1)  /* D below f_thr rho_atm -> atmosphere */
#define GRMHD_F_TAUFLOOR        (1u << 2)  /* tau raised to tau_atm(D, B) */
#define GRMHD_F_MAGCAP          (1u << 3)  /* D raised to B^2 / M_max */
#define GRMHD_F_TFLOOR          (1u << 4)  /* T raised to T_atm, rho and W v kept */
#define GRMHD_F_RHOFLOOR        (1u << 5)  /* rho below threshold after inversion */
#define GRMHD_F_FOFC            (1u << 6)  /* trial state needed a floor/failed */
#define GRMHD_F_DMP             (1u << 7)  /* trial D~ or tau~ broke Eq. 12 */
#define GRMHD_F_BRACKET_FALLBACK (1u << 8) /* learned bracket missed -> full bracket */
#define GRMHD_F_MAXIT           (1u << 9)  /* root solve hit the iteration cap */
#define GRMHD_F_EXCISED         (1u << 10) /* lapse below alpha_min -> atmosphere (grmhd_excise) */

/* Method options (Sec. III-B..III-D). */
typedef struct grmhd_params {
  double gamma;       /* ideal-gas adiabatic index, P = (gamma-1) rho eps */
  double rho_b[3];    /* hybrid EOS: dividing densities of the cold pieces */
  double K0;          /* hybrid EOS: polytropic constant of the first piece */
  double Gam[4];      /* hybrid EOS: index of each cold piece */
  double gamma_th;    /* hybrid EOS: thermal index */
  double rho_atm;     /* atmosphere density */
  double T_atm;       /* atmosphere temperature (T = P/rho ideal; P_th/rho hybrid) */
  double f_thr;       /* density threshold factor of the floors */
  double M_max;       /* magnetisation cap on B^2/D */
  double dmp_M;       /* <= 0: plain FOFC; > 0: FOFC+DMP with factor M (Eq. 12) */
  double c2p_tol;     /* relative bracket tolerance of the root solve */
  int32_t eos;        /* 0 ideal gas, 1 hybrid piecewise polytrope + thermal */
  int32_t npieces;    /* hybrid: cold pieces, 1..4 */
  int32_t recon;      /* 0 donor cell, 1 PLM (van Leer limiter), 2 WENOZ,
                         3 PPM4 (Colella & Woodward 1984), 4 PPMX
                         (Colella & Sekora 2008 extremum-preserving);
                         any other value: GRMHD_EUNSUPPORTED */
  int32_t riemann;    /* 0 LLF, 1 HLLE */
  int32_t fofc;       /* 0 off, 1 on */
  int32_t c2p_maxit;  /* iteration cap of the root solve */
} grmhd_params;

/* One MeshBlock.  Every pointer is device memory; arrays are padded. */
typedef struct grmhd_block {
  int32_t nx, ny, nz, ng;  /* interior cells per axis, ghost layers (ng = 3) */
  double dx[3];            /* cell size per axis */
  double *w[5];            /* stage-input primitives rho, W v^x, W v^y, W v^z, P */
  double *un[5];           /* U^n: D~, S~_x, S~_y, S~_z, tau~ (interior read) */
  double *us[5];           /* U^(s), the stage input (ghosts read by the DMP) */
  double *bn[3];           /* B~^n on x-, y-, z-faces */
  double *bs[3];           /* B~^(s) on faces (stage input) */
  const double *adm[16];   /* alpha, beta^x..z, gamma_xx xy xz yy yz zz, K_xx..zz */
  double *uo[5];           /* output U (may alias un) */
  double *bo[3];           /* output faces (may alias bn) */
  double *wo[5];           /* output primitives */
  uint16_t *flags;         /* per-cell flag bits, padded */
  double *scratch;         /* grmhd_scratch_doubles(...) doubles of workspace */
  int32_t nbr[27];         /* neighbour block per offset (ox+1)+3(oy+1)+9(oz+1); -1: none */
  int32_t bc;              /* 0 ghosts frozen (untouched); 1 filled from nbr, outflow if -1 */
  /* launch layout, filled by grmhd_blocks_prepare (do not set by hand):
     first 64-item wave of this block in each of the grmhd_launch_shapes()
     launch shapes (unused slots zero), and the number of blocks in the
     table */
  int32_t wave0[24];
  int32_t nblk;
  int32_t reserved;
} grmhd_block;

/* Fill the launch-layout fields (wave0, nblk, reserved) of a host
   descriptor table in place; writes nothing else.  Call once after the table
   is built and before it is copied to the device; every block-list entry
   point checks that the layout is current.  GRMHD_EINVAL for a NULL table,
   nblk < 1, a block with a size below 1, or more waves than fit in int32. */
int grmhd_blocks_prepare(grmhd_block *blk_h, int32_t nblk);
/* Number of launch shapes, i.e. of used wave0 slots (at most 24). */
int32_t grmhd_launch_shapes(void);

/* Doubles of per-block scratch needed by the stage: the 21 face-flux arrays
   (7 components D~, S~_xyz, tau~, F(B~^{t1}), F(B~^{t2}) per direction, t1 =
   (d+1)%3, t2 = (d+2)%3), the cell-centred field B^i = B~_cc/sqrt(gamma)
   (3 cell arrays), the cell-centre EMF (3 cell arrays), the corner EMFs
   (3 arrays of (sx+1)(sy+1)(sz+1)), room for per-wave statistics of the
   stage inversion (2 cell arrays) and the FOFC list of flagged cells of
   [g-1, g+n]^3 (a counter and (nx+2)(ny+2)(nz+2) int32 cell indices).  Flux d, component c starts at
   grmhd_flux_offset(...) doubles into scratch. */
int64_t grmhd_scratch_doubles(int32_t nx, int32_t ny, int32_t nz, int32_t ng);
int64_t grmhd_flux_offset(int32_t nx, int32_t ny, int32_t nz, int32_t ng, int32_t d, int32_t c);

/*
 * Every block-list entry point takes the descriptor table twice: blk_h in
 * host memory (launch geometry and validation) and blk_d, the same table in
 * device memory (read by the kernels).  nblk >= 1.  The RK coefficients give
 * U^out = a0 U^n + a1 U^(s) + b dt L(U^(s)) (Sec. III-B time integrators, in
 * the Shu-Osher form of Gottlieb, Ketcheson & Shu 2009): SSP-RK2 is (0, 1, 1)
 * then (1/2, 1/2, 1/2); SSP-RK3 is (0, 1, 1), (3/4, 1/4, 1/4), (1/3, 2/3,
 * 2/3), each stage reading the previous stage's output as U^(s).  uo may
 * alias un (the last stage), but not us.  dt is read from the device scalar
 * dt_d when dt_d != NULL, else the host value dt is used.
 */

/* Steps a1-a8 of one stage (Sec. III-B..III-D): face fluxes (reconstruction,
   face metric, floors, Eq. 7-9, HLLE/LLF), FOFC(+DMP) flags with exchange of
   flags between blocks and donor-cell refluxing, upwind CT of the faces,
   update with the Eq. 10 sources, C2P with atmosphere floors.  Writes uo,
   bo, wo, flags.  Ghost cells of the outputs are not filled. */
int grmhd_stage(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                const grmhd_params *p, const double *dt_d, double dt, double a0, double a1,
                double b, void *stream);

/* Steps a2-a3 alone: high-order face fluxes into each block's scratch, with
   the cell-centred field of the stage input and its cell-centre EMF
   E = -alpha (vhat x B~) (read later by ct_update). */
int grmhd_fluxes(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                 const grmhd_params *p, void *stream);

/* Step a4 (Sec. III-C, FOFC and Eq. 12): from the fluxes in scratch, the
   trial state without sources or CT, the trial inversion, the DMP test, the
   flag exchange between blocks, and donor-cell refluxing of every face of a
   flagged cell (all 7 components).  Writes flags and the fluxes in scratch. */
int fofc_correct(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                 const grmhd_params *p, const double *dt_d, double dt, double a0, double a1,
                 double b, void *stream);

/* Step a5 (Sec. III-B): upwind constrained transport.  Corner EMFs from the
   face EMFs in scratch and the cell-centre EMF of the stage input (both
   written by grmhd_fluxes, the face EMFs corrected by fofc_correct), then
   bo = a0 bn + a1 bs - b dt curl(E) on the interior faces. */
int ct_update(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
              const grmhd_params *p, const double *dt_d, double dt, double a0, double a1,
              double b, void *stream);

/* Step a6 (Eq. 10): uo = a0 un + a1 us + b dt (-div F + G(w, us, ADM)). */
int grmhd_update(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                 const grmhd_params *p, const double *dt_d, double dt, double a0, double a1,
                 double b, void *stream);

/* Step a8 on the interior of every block: uo, bo -> wo with the floors;
   OR-s the inversion flags into flags. */
int grmhd_stage_c2p(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                    const grmhd_params *p, void *stream);

/* Ghost fill (same-level copy / periodic self-neighbour / outflow) of the
   arrays in the w (mask 1), us (2), bs (4) and flags (8) slots.  Blocks with
   bc == 0 keep their ghosts. */
int grmhd_ghost_fill(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                     int32_t mask, void *stream);

/* Step a9: dt_out[0] = cfl / max over interior cells and directions of
   |lambda_+-| / dx_d from the w and bs slots (fast magnetosonic speeds).
   red: device scratch of one double (overwritten).  GRMHD_EINVAL for a NULL
   red or dt_out, cfl <= 0, a stale layout, or a block without w, bs or the
   metric (adm[0..9]). */
int grmhd_dt(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
             const grmhd_params *p, double cfl, double *red, double *dt_out, void *stream);

/* Baryon mass sum D~ dV over the interiors of the us slot (deterministic
   order).  partial: device scratch of nblk doubles; out: one device double.
   GRMHD_EINVAL for a NULL partial or out, a stale layout, or a block without
   us[0]. */
int grmhd_mass(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
               double *partial, double *out, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): grmhd_mass without the
   partial workspace.  The nblk per-block partial sums live in a fixed device
   array of the library (grmhd_mass_noalloc_max_blocks() = 65536 doubles,
   512 KiB per GPU, held until the process ends); the call allocates nothing.
   Same result as grmhd_mass, bit for bit.  Call with the device of `stream`
   current.  All calls on one GPU share that array: calls that overlap in time
   on one GPU (different streams, no ordering) race.  GRMHD_ETOOBIG for
   nblk > grmhd_mass_noalloc_max_blocks(); GRMHD_EINVAL as for grmhd_mass. */
int grmhd_mass_noalloc(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                       double *out, void *stream);
int32_t grmhd_mass_noalloc_max_blocks(void);

/* Eq. 7 over every padded cell of each block: us <- prim2con(w, B~_cc(bs)),
   B~_cc the face average of the bs slot.  Initialises the conserved state. */
int grmhd_prim2con_blocks(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                          const grmhd_params *p, void *stream);

/* Eq. 7 at n points (densitized): w (rho, W v^i, P), bt densitized B~^i,
   gam (gamma_xx xy xz yy yz zz) -> u (D~, S~_i, tau~).  Arrays of n doubles. */
int prim2con(int64_t n, double *const w[5], double *const bt[3], double *const gam[6],
             double *u[5], const grmhd_params *p, void *stream);

/* Learned guess and bracket for the inversion (not in the paper): a
   5-64-64-64-2 perceptron with hard-swish activations, z clamp(z/6 + 1/2, 0, 1),
   on standardised invariants of the scaled state (log10 D, log10(1+q),
   r/(1+q), b^2/(1+q), s^2/(r^2 b^2)).  Output y0
   estimates logit(mu), y1 the log of the expected |logit error|; the bracket
   is logistic(y0 -+ (width_k exp(y1) + width_min)).  Parameters are one flat
   vector of C2P_MLP_NPARAM values, row-major [out][in] per layer:
   W1[64][5] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[2][64] b4[2].
   Weights are read from the bf16 copy (MFMA operands, fp32 accumulation),
   biases from the fp32 copy.  Both are device memory. */
#define C2P_MLP_NPARAM 8834
typedef struct c2p_mlp {
  const uint16_t *w_bf16;             /* bf16 parameter vector */
  const float *w_f32;                 /* fp32 parameter vector */
  float feat_mean[5], feat_scale[5];  /* standardisation: (x - mean) * scale */
  float width_k, width_min;           /* bracket half-width in logit space */
  double *bracket_ws;                 /* optional device workspace of 2 n doubles: when set,
                                         the network runs as its own MFMA kernel writing
                                         the brackets, then the FP64 root kernel reads them;
                                         when NULL, one fused kernel does both */
} c2p_mlp;

/* C2P statistics accumulated by c2p_batch when stats != NULL (device). */
typedef struct c2p_stats {
  unsigned long long solves, evaluations, fallbacks, failures;
} c2p_stats;

/* Step a8 (Sec. III-C, III-D) at n points: u (in/out; rewritten from the
   final primitives whenever a floor rule fires), bt densitized field, gam ->
   w, flags.  mlp != NULL: the learned guess and bracket start the same FP64
   root solve (fallback to the full bracket, bit 8).  mu_out, nev_out may be
   NULL (root and master-function evaluations per point). */
int c2p_batch(int64_t n, double *u[5], double *const bt[3], double *const gam[6], double *w[5],
              uint16_t *flags, const grmhd_params *p, const c2p_mlp *mlp, c2p_stats *stats,
              double *mu_out, int32_t *nev_out, void *stream);

/* grmhd_stage whose dt is the CFL time step of its input (step a9 folded
   into the stage's first kernel, which reads that state anyway): dt_out[0] =
   cfl / max over interior cells and directions of |lambda_+-| / dx_d, the
   value grmhd_dt gives, bit for bit; the stage then runs with it.  red: device
   scratch of one double.  For the first stage of a step (its input is the
   step's state).  GRMHD_EINVAL as for grmhd_dt and grmhd_stage. */
int grmhd_stage_cfl(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                    const grmhd_params *p, double cfl, double *red, double *dt_out, double a0,
                    double a1, double b, void *stream);

/* grmhd_stage with the stage's final inversion (step a8) started from the
   learned bracket (mlp != NULL; NULL = the plain inversion of grmhd_stage).
   Same outputs and atmosphere rules; a bracket that holds no sign change is
   moved towards the root (4 and 16 times its width) and then replaced by the
   full bracket; such cells carry bit 8 in flags.  The FOFC
   trial inversion stays plain.  stats (device, may be NULL) accumulates
   solves, master-function evaluations, fallbacks and failures of the final
   inversion (plain or learned).  mlp's bracket_ws is not used. */
int grmhd_stage_learned(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                        const grmhd_params *p, const double *dt_d, double dt, double a0,
                        double a1, double b, const c2p_mlp *mlp, c2p_stats *stats,
                        void *stream);
/* grmhd_stage_c2p with the learned bracket (mlp required). */
int grmhd_stage_c2p_learned(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                            const grmhd_params *p, const c2p_mlp *mlp, c2p_stats *stats,
                            void *stream);

/* ADM matter sources for the spacetime coupling (Sec. III-A): the fluid's
   stress-energy tensor (Eq. 2 with Eq. 5 and 8) projected on the slice with
   the unit normal n,
     E = n_mu n_nu T^{mu nu}, S_i = -gamma_i^mu n^nu T_{mu nu},
     S_ij = gamma_i^mu gamma_j^nu T_{mu nu}   (lower indices, not densitized),
   at the interior cells of every block from its stage-input primitives w and
   face field bs.  out_d: device array of 10 * nblk device pointers; entry
   10 * b + n is a padded cell array of block b (layout of w) that receives
   component n of (E, S_x, S_y, S_z, S_xx, S_xy, S_xz, S_yy, S_yz, S_zz) at
   the interior cells; ghost cells are not written.  GRMHD_EINVAL if out_d is
   NULL. */
int grmhd_matter_sources(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                         const grmhd_params *p, double *const *out_d, void *stream);

/* Lapse excision (Sec. IV, the collapse runs): interior cells with alpha <
   alpha_min get the atmosphere primitives (rho_atm, v = 0, T_atm) in wo and
   the conserved state of those primitives with the unchanged field bo in uo;
   flag bit 10 is set.  Meant right after a stage, on its outputs.  Does
   nothing when alpha_min <= 0. */
int grmhd_excise(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                 const grmhd_params *p, double alpha_min, void *stream);

/* Learned-bracket training support (device memory throughout).
   c2p_mlp_features: standardised features [5][n] (fp32) of the conserved
   states u after the conserved-floor rules and, when w_true != NULL, the
   targets logit(1/(h W)) [n] of the primitives that generated them.
   c2p_mlp_forward: y [2][n] from standardised features [5][n].
   c2p_mlp_to_bf16: theta (fp32) -> theta_bf16.
   c2p_mlp_train_step: forward + loss + backward over nbatch samples (a
   multiple of 64) on the MFMA units, one 64-sample partial gradient per
   workgroup in partial[(nbatch/64) * C2P_MLP_NPARAM], reduced in a fixed
   order (deterministic); if step >= 1, one Adam step (lr, beta1 0.9, beta2
   0.999, eps 1e-8, bias correction for `step`) on theta with moments adam_m,
   adam_v, and theta_bf16 refreshed.  grad_out (C2P_MLP_NPARAM), loss_part
   (nbatch/64) and loss_out (1) may be NULL.  Loss per sample:
   0.5 (y0 - t)^2 + 0.5 (y1 - log(|y0 - t| + 1e-4))^2, batch mean; the
   second term trains only the read-out W4[1], b4[1] (its gradient does not
   enter the hidden layers). */
int c2p_mlp_features(int64_t n, double *const u[5], double *const bt[3], double *const gam[6],
                     double *const w_true[5], const grmhd_params *p, const float mean[5],
                     const float scale[5], float *feats, float *target, void *stream);
int c2p_mlp_forward(const c2p_mlp *mlp, int64_t n, const float *feats, float *y, void *stream);
int c2p_mlp_to_bf16(const float *theta, uint16_t *theta_bf16, void *stream);
/* Bracket width of the learned guess: runs the network on n standardised
   samples feats [5][n] with labels target [n] (logit of mu), and sets
   mlp->width_k to the q-quantile of |y0 - target| / exp(y1) (linear between
   order statistics), so that the bracket logistic(y0 -+ (width_k exp(y1) +
   width_min)) holds the label of a fraction q of the samples; sets
   mlp->width_min.  ws: device workspace of 3 n floats.  Synchronises
   `stream` (setup, not the hot path); GRMHD_EINVAL for q outside (0, 1]. */
int c2p_mlp_calibrate_width(c2p_mlp *mlp, int64_t n, const float *feats, const float *target,
                            double q, float width_min, float *ws, void *stream);
int c2p_mlp_train_step(float *theta, float *adam_m, float *adam_v, uint16_t *theta_bf16,
                       const float *feats, const float *target, int64_t nbatch, float lr,
                       int32_t step, float *partial, float *loss_part, float *loss_out,
                       float *grad_out, void *stream);

/* Library version string and the HIP device architecture it was built for. */
const char *grmhd_version(void);

/* Per-kernel timing for measurement.  grmhd_timing(1) creates an event pool
   (once) and starts recording HIP events on the launch stream around every
   launch of each kernel family; grmhd_timing(0) stops.  grmhd_timing_read
   waits for the recorded events and returns the accumulated milliseconds and
   launch count of a family since timing was enabled.  Families: 0/1/2
   face fluxes x/y/z, 3 FOFC flags, 4 FOFC refluxing, 5 CT, 6 update with
   sources, 7 stage C2P, 8 ghost fill, 9 dt, 10 cell-centred field,
   11 c2p_batch plain, 12 c2p_batch learned, 13 MLP training, 14 MLP
   bracket kernel, 15 stage C2P with the learned bracket, 16 matter sources,
   17 excision. */
int grmhd_timing(int32_t on);
/* Workgroup size (64..512, a multiple of 64) of a kernel family of the stage
   (families as for grmhd_timing, 0..17); default 256.  Set by the
   autotuner; applies to subsequent launches in this process.  The update
   (family 6) at 512 on a block list whose blocks are all 64 cells wide, with
   ny even and nz a multiple of 4, runs in the brick layout (2 rows x 4 planes
   per workgroup, metric stencils through LDS); its results are bitwise equal
   to those of any other size. */
int grmhd_set_threads(int32_t family, int32_t threads);
int grmhd_timing_read(int32_t family, double *ms, int64_t *launches);

/*
 * A whole SSP-RK2 step (Sec. III-B time integration, Shu-Osher form) over
 * the four descriptor tables of a mesh with two state sets A (U^n, w, B~^n)
 * and B (the first stage's output): a and b describe each set alone (dt,
 * ghost fill), ab the first stage (set A in, set B out) and ba the second
 * (set B in as U^(s), set A as U^n and output).  Host and device copies as
 * for every block-list call; all four tables list the same blocks in the same
 * order.
 */
typedef struct grmhd_rk2_tables {
  const grmhd_block *a_h, *a_d;
  const grmhd_block *b_h, *b_d;
  const grmhd_block *ab_h, *ab_d;
  const grmhd_block *ba_h, *ba_d;
} grmhd_rk2_tables;

/* One step: stage 1 (0, 1, 1) with dt_out = the CFL dt of set A computed in
   that stage (grmhd_stage_cfl, red its scratch double), ghost fill of set B,
   stage 2 (1/2, 1/2, 1/2) with the device dt, ghost fill of set A (w, U,
   faces).  Asynchronous; errors as for the calls it makes. */
int grmhd_rk2_step(const grmhd_rk2_tables *t, int32_t nblk, const grmhd_params *p, double cfl,
                   double *red, double *dt_out, void *stream);

/* Conserved/primitive pairs of the interior cells of every block (every
   stride-th cell along x), for training the learned inversion on a run's own
   states: block b's cells go, x fastest, to the entries base[b] .. base[b] +
   nz ny ceil(nx / stride) - 1 of the flat outputs (base: device int64 array
   of nblk offsets): u the us slot, bt the densitized cell-centred field of
   the bs faces (face average per direction, reading R1), gam gamma_ij, w the
   w slot.  GRMHD_EINVAL for stride < 1 or a missing array. */
int grmhd_c2p_pairs(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                    int32_t stride, const int64_t *base, double *const u[5], double *const bt[3],
                    double *const gam[6], double *const w[5], void *stream);

/* The same step captured once into a HIP graph on `stream` (a created
   stream, not the null stream; nothing may be pending on it from another
   capture) and instantiated: grmhd_graph_launch replays all its launches
   with one call.  The graph holds the tables' device copies and every array
   they point to by address: those must stay allocated and in place while the
   graph lives.  No memset or copy node is captured (the reductions clear
   their scratch with kernels).  GRMHD_EINVAL while per-kernel timing is on
   (its events cannot be captured) or for a NULL stream or out; GRMHD_EHIP if
   capture or instantiation fails.  grmhd_graph_destroy frees the graph. */
typedef struct grmhd_graph grmhd_graph;
int grmhd_graph_build(const grmhd_rk2_tables *t, int32_t nblk, const grmhd_params *p, double cfl,
                      double *red, double *dt_out, void *stream, grmhd_graph **out);
int grmhd_graph_launch(grmhd_graph *g, void *stream);
int grmhd_graph_destroy(grmhd_graph *g);

/* Autotuner over the launch shapes of the stage: for each of the families
   0..7 (fluxes x, y, z, FOFC flags, refluxing, CT, update, inversion) it
   times the first stage of table ab (set A -> set B, which leaves its inputs
   unchanged, so it can be repeated) at workgroup sizes 64, 128, 256 and 512
   -- the length of the x-pencil of consecutive cells or faces one workgroup
   covers; for the update, 512 selects the 2-row x 4-plane brick tile where
   the blocks allow it -- reps times each, and keeps the fastest
   (grmhd_set_threads).  threads_out[8]: the sizes kept; ms_out[8 * 4]: the
   mean milliseconds per launch of each candidate (may be NULL; 0 for a family
   the stage does not launch on its own -- the plain stage runs the inversion
   inside the update -- which is left at 256).  Synchronises
   `stream`; turns per-kernel timing off when it returns. */
int grmhd_autotune(const grmhd_block *ab_h, const grmhd_block *ab_d, int32_t nblk,
                   const grmhd_params *p, double dt, int32_t reps, int32_t *threads_out,
                   double *ms_out, void *stream);

/* Plain streaming copy dst[0..n) = src[0..n) (device memory), used to
   calibrate hardware traffic counters against a kernel of known bytes. */
int grmhd_copy(const double *src, double *dst, int64_t n, void *stream);

/* sizeof of the ABI structs (0 grmhd_params, 1 grmhd_block, 2 c2p_mlp,
   3 c2p_stats; -1 otherwise), so bindings can check their layouts. */
int32_t grmhd_struct_size(int32_t which);

/* ---------------------------------------------------------------------------
   Refined meshes: the inter-level transfer of block-based mesh refinement
   (Sec. I; prolongation and restriction are among the costs of Sec. V-A).
   The blocks are the leaves of a 2:1-balanced octree of equal blocks
   (nx = ny = nz = nb, nb even, nb >= 2 ng + 2): refinement by 2, and any two
   leaves that touch across a face, an edge or a corner differ by at most one
   level.  A ghost cell or face takes its value from the leaf that covers it:
   a same-level leaf: a copy; a finer leaf: the mean of the 8 child cells
   (flags: their OR) or of the 4 child faces on the face's plane; a coarser
   leaf: the parent cell plus, per axis, a quarter of its minmod-limited slope
   signed towards the child (flags: the parent's), for a face on a parent
   face that face's value and for a face inside a parent cell the mean of
   that cell's two faces along the normal (each child cell then has its
   parent's divergence).  Where two leaves hold a face, the one within the
   block's own range along the face's normal is read first.  Outflow
   boundaries take the nearest cell (face) of the domain; periodic ones wrap.
   In a stage the fluxes of a block's boundary faces next to a finer leaf are
   the mean of the 4 fine fluxes (conservation), and its boundary edge EMFs
   next to a finer leaf the mean of the 2 fine EMFs along the edge (div B~ at
   round-off, and every leaf around such an edge uses the same EMF).  One dt
   for every level.
   ------------------------------------------------------------------------- */
#define GRMHD_AMR_NONE (-9)   /* rel[] of a region beyond an outflow boundary */

typedef struct {
  int32_t level;       /* refinement level (cell size dx0 / 2^level)                 */
  int32_t org[3];      /* global index, at its level, of the block's first interior cell */
  int32_t N[3];        /* cells of the domain per axis at its level                    */
  int32_t periodic;    /* bit a set: axis a periodic, else outflow                    */
  int32_t rel[27];     /* per neighbour region (ox+1)+3(oy+1)+9(oz+1), ng+1 cells deep
                          (the block's own interior for 13): the level of the leaves
                          covering it minus this block's, -1, 0 or 1; GRMHD_AMR_NONE
                          beyond an outflow boundary                                  */
  int32_t src[27][4];  /* the leaves covering each region (block indices, -1 unused)  */
} grmhd_amr_link;

/* Host: the links of nblk leaves (level[i], org[3 i .. 3 i + 2]) of blocks of
   nb^3 cells with ng ghosts on a domain of n0[3] level-0 cells with
   periodic[3] (1 periodic, 0 outflow); links: nblk entries written.
   GRMHD_EINVAL for sizes out of range (nb odd or < 2 ng + 2, a leaf outside
   the domain or off its level's nb lattice), overlapping leaves, a region
   covered by no leaf or by leaves of different levels or of a level more
   than one apart, or more than 4 leaves in a region. */
int grmhd_amr_links(int32_t nblk, const int32_t *level, const int32_t *org, int32_t nb,
                    int32_t ng, const int32_t n0[3], const int32_t periodic[3],
                    grmhd_amr_link *links);

/* Ghost fill across levels of the w (mask 1), us (2), bs (4) and flags (8)
   slots of a refined mesh: copies and restrictions first, then the
   prolongations level by level upwards (the parent's slope may read the
   parent leaf's ghosts).  links_h / links_d: the same grmhd_amr_link array
   in host / device memory.  GRMHD_EINVAL for unequal block sizes or a block
   with bc != 1. */
int grmhd_ghost_fill_amr(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                         const grmhd_amr_link *links_h, const grmhd_amr_link *links_d,
                         int32_t mask, void *stream);

/* One stage on a refined mesh: the steps of grmhd_stage_learned (mlp and
   stats optional, as there) with the flag exchange across levels, the flux
   correction after the FOFC refluxing and the EMF correction between the
   corner EMFs and the face update. */
int grmhd_stage_amr(const grmhd_block *blk_h, const grmhd_block *blk_d, int32_t nblk,
                    const grmhd_amr_link *links_h, const grmhd_amr_link *links_d,
                    const grmhd_params *p, const double *dt_d, double dt, double a0, double a1,
                    double b, const c2p_mlp *mlp, c2p_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GRMHD_H */

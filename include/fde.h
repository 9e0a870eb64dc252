/*
 * fde.h -- C ABI of the MI355X (gfx950) periodic frozen-density-embedding
 * hot path.
 *
 * Method: Genova, Ceresoli & Pavanello, "Periodic Subsystem Density-Functional
 * Theory" (arXiv:1406.7803). Each subsystem I solves the Kohn-Sham-like
 * equation of Sec. 2 (Eq. KS) in a plane-wave basis at every k-point, with the
 * effective potential in the recast form of the Appendix ("Recast of the
 * Effective Potential expression"):
 *     V_eff^I = V_eN(all nuclei) + V_H[rho] + V_XC[rho_I]
 *               + V_kin^nad[rho, rho_I] + V_XC^nad[rho, rho_I],
 * the densities are the Brillouin-zone sums of Sec. 2, and rho = sum_I rho_I.
 *
 * Conventions (all calls):
 *  - Units: Hartree atomic units. Orthorhombic cell L1 x L2 x L3.
 *  - Grids are real arrays in C order [N3][N2][N1] (x fastest), of the plan's
 *    precision (double for FDE_F64, float for FDE_F32).
 *  - Bands are band-major [nb][npw_k] interleaved complex of the plan's
 *    precision. The plane waves of k are S_k = {G : |k+G|^2/2 <= E_cut},
 *    ordered lexicographically on centred Miller indices (m1, m2, m3), m3
 *    fastest (fde_plan_miller returns the list). Orbitals are
 *    u(r) = Omega^{-1/2} sum_G c(G) e^{iG.r}; a normalised band has sum|c|^2 = 1.
 *  - Transform pair: f(G) = (1/N) sum_r f(r) e^{-iG.r}, f(r) = sum_G f(G) e^{iG.r}.
 *    The density sphere is D = {G : |G|^2 <= 8 E_cut}.
 *  - Pointers named d_* (and every array argument unless stated "host") are
 *    device pointers; the caller owns all of them. The library allocates no
 *    device memory: scratch comes from the workspace the caller attaches with
 *    fde_plan_set_workspace. The plan owns only host metadata.
 *  - Every compute call only enqueues work on `stream` and returns. Calls on
 *    one plan share its workspace and must be ordered (one stream, or
 *    synchronised streams). Distinct plans are independent. A plan is not
 *    thread-safe.
 *  - Errors detectable on the host return a negative fde_status synchronously,
 *    with a message in fde_last_error() (thread-local). Numerical failures on
 *    the device are written to a caller-provided device int* info (read after
 *    a stream synchronisation): 0 = success.
 *  - Outputs never alias inputs unless stated.
 */
#ifndef FDE_H
#define FDE_H

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int fde_status;
enum {
  FDE_OK = 0,
  FDE_ERR_ARG = -1,         /* invalid argument (null pointer, out-of-range value) */
  FDE_ERR_SHAPE = -2,       /* sizes inconsistent with the plan or the workspace */
  FDE_ERR_DEVICE = -3,      /* a HIP runtime call failed */
  FDE_ERR_UNSUPPORTED = -4, /* grid length or configuration not supported */
  FDE_ERR_WORKSPACE = -5    /* no (or too small a) workspace attached */
};

enum { FDE_F64 = 0, FDE_F32 = 1 };

typedef struct fde_plan fde_plan;

/* Thread-local message of the last failing call (never NULL). */
const char* fde_last_error(void);

/*
 * Plane-wave plan of one cell, FFT grid, cutoff and k-point list (Sec. 1 and
 * Sec. 3: plane waves with a k-point mesh).
 *   L[3]      host, cell lengths (bohr), orthorhombic.
 *   grid[3]   host, (N1, N2, N3); each a product of 2, 3, 5 and at most 512;
 *             must satisfy N_i > 4 sqrt(2 E_cut) / b_i (no aliasing of
 *             orbital products), b_i = 2 pi / L_i.
 *   ecut_ha   wavefunction kinetic cutoff (Ha).
 *   kfrac     host [nk][3] reduced k-points (k_i = kfrac_i b_i).
 *   prec      FDE_F64 or FDE_F32: precision of bands, grids and FFTs.
 *   out       receives the plan (release with fde_plan_destroy).
 */
fde_status fde_plan_create(const double L[3], const int grid[3], double ecut_ha, int nk,
                           const double* kfrac, int prec, fde_plan** out);
void fde_plan_destroy(fde_plan* plan);

/* Sizes of k-point ik: plane waves npw and z-sticks ncol (either may be NULL). */
fde_status fde_plan_info(const fde_plan* plan, int ik, int* npw, int* ncol);

/* host mill[npw][3]: centred Miller indices (m1, m2, m3) of S_k, in band order. */
fde_status fde_plan_miller(const fde_plan* plan, int ik, int32_t* mill);

/*
 * Workspace size for calls with at most max_nb bands per call (subspace calls
 * use m <= 2 max_nb), at most max_nproj projectors, and batched subspace calls
 * of at most max_batch (1..16) band blocks per launch (larger batches are
 * split into launches of max_batch).
 */
fde_status fde_plan_workspace_bytes(const fde_plan* plan, int max_nb, int max_nproj, int max_batch,
                                    size_t* bytes);

/*
 * Attach a device workspace of at least fde_plan_workspace_bytes(max_nb,
 * max_nproj, max_batch) bytes (256-byte aligned). Uploads the plan's device
 * tables into it (synchronous). The caller keeps ownership; it must outlive
 * the plan's use.
 */
fde_status fde_plan_set_workspace(fde_plan* plan, void* d_ws, size_t bytes, int max_nb, int max_nproj,
                                  int max_batch);

/*
 * Arithmetic of the subspace products S = V^H V and A = V^H HV of
 * fde_subspace_rr(_batched) (the Rayleigh-Ritz step of the band solver):
 *   FDE_GEMM_FP64   inputs widened to FP64, FP64 matrix cores (default);
 *   FDE_GEMM_BF16X3 FP32 inputs split in two BF16 terms, products of the term
 *                   pairs (0,0), (0,1), (1,0) on BF16 matrix cores, FP32
 *                   accumulation over 32-wide k tiles, FP64 sums of the tiles
 *                   (about 16 significant bits per product);
 *   FDE_GEMM_BF16X6 three BF16 terms, six term pairs (about FP32 products).
 * The split modes need an FP32 plan (FDE_ERR_UNSUPPORTED otherwise). The
 * Cholesky and the eigensolver stay FP64 in every mode. In the split modes the
 * dependent-column threshold of the Cholesky is at least 2e-4 (BF16X3) or
 * 1e-6 (BF16X6) of S_jj: about ten times the products' relative noise.
 */
/*
 * Launch-shape tuning (no effect on results but the one FDE_TUNE_RR_SPLIT
 * states). FDE_TUNE_APPLY_BPW: bands per
 * plane-pass workgroup of fde_apply_h (each workgroup reads one V_eff plane
 * for that many bands). FDE_TUNE_STICK_GROUP: z-sticks per workgroup of the
 * z-FFT passes of fde_apply_h and fde_density (a power of two, capped at 16
 * and by the LDS budget; used by the LDS z-passes). FDE_TUNE_Z_REGISTER: 1
 * keeps the LDS z-passes where a four-step register z-FFT exists (N3 = 240,
 * 120, and 432 in FP32 plans). FDE_TUNE_PLANE_KIND: the in-plane pass of fde_apply_h and
 * fde_density -- 1 whole-line register FFTs, 2 LDS Stockham passes, 3 two-factor
 * FFTs in LDS (used where the kind applies; otherwise the automatic choice).
 * FDE_TUNE_PLANE_ROWS: rows per batch of the two-factor pass (LDS size),
 * rounded down to a multiple of its four wavefronts, at least one row each.
 * FDE_TUNE_RR_SPLIT: the smallest m (columns of [X W P]) for which the
 * Rayleigh-Ritz step of fde_subspace_rr runs its eigensolver as a sequence of
 * multi-workgroup launches instead of one workgroup per problem (the two agree
 * to rounding, not bit for bit; up to m = 768). 0 restores the automatic
 * choice (a value of 1024 never splits; the automatic 256 was the fastest of
 * the thresholds 128 to 256 timed on the 64-subsystem cube). Errors: FDE_ERR_ARG for an unknown key, a value outside [0, 1024]
 * or a stick group that is not a power of two.
 */
#define FDE_TUNE_APPLY_BPW 1
#define FDE_TUNE_STICK_GROUP 2
#define FDE_TUNE_Z_REGISTER 3
#define FDE_TUNE_PLANE_KIND 4
#define FDE_TUNE_PLANE_ROWS 5
#define FDE_TUNE_RR_SPLIT 6
fde_status fde_plan_set_tuning(fde_plan* plan, int key, int value);

#define FDE_GEMM_FP64 0
#define FDE_GEMM_BF16X3 1
#define FDE_GEMM_BF16X6 2
fde_status fde_plan_set_gemm_mode(fde_plan* plan, int mode);

/*
 * H_I |psi_nk> (Eq. KS with the recast V_eff of the Appendix, and the
 * Kleinman-Bylander projectors of the subsystem's own atoms as in the
 * Appendix on non-local pseudopotentials):
 *   hpsi(G) = |k+G|^2/2 psi(G) + [FFT_fwd(V_eff . FFT_inv(psi))](G)
 *             + sum_i beta_i(G) D_i <beta_i|psi>,    G in S_k.
 *   ik        k-point index of the plan.
 *   nb        bands (any number; processed in chunks of the workspace's max_nb).
 *   psi       [nb][npw] complex, input.   hpsi  [nb][npw] complex, output.
 *   veff      [N3][N2][N1] real.
 *   nproj     projectors (0: none; beta and dkb may then be NULL).
 *   beta      [nproj][npw] complex (from fde_kb_projectors or the caller).
 *   dkb       [nproj] double, KB energies D_i (Ha).
 */
fde_status fde_apply_h(fde_plan* plan, int ik, int nb, const void* psi, void* hpsi, const void* veff,
                       int nproj, const void* beta, const double* dkb, hipStream_t stream);

/*
 * Subsystem density (Sec. 2, BZ-integrated density with occupations):
 *   rho(r) += sum_n occw[n] |u_n(r)|^2,  u = Omega^{-1/2} FFT_inv(psi).
 *   occw  [nb] double, w_k f_nk (f in [0, 2], sum_k w_k = 1).
 *   rho   [N3][N2][N1] real, accumulated (+=): sum the k-points into one grid.
 */
fde_status fde_density(fde_plan* plan, int ik, int nb, const void* psi, const double* occw, void* rho,
                       hipStream_t stream);

/* Functional ids for fde_embed_potential. */
/* xc: LDA = Slater + Perdew-Zunger 1981; PBE = Perdew-Burke-Ernzerhof 1996 with PW92
 * correlation (the paper's functional, Sec. 3), potential de/drho - div(2 de/dsigma grad rho).
 * kin: Thomas-Fermi x F(s) with F = 1 (TF), LC94 or revAPBEK (the two nonadditive kinetic
 * functionals of Sec. 3). Gradient terms use the spectral gradient on the density sphere. */
enum { FDE_XC_NONE = 0, FDE_XC_LDA = 1, FDE_XC_PBE = 2 };
enum { FDE_KIN_NONE = 0, FDE_KIN_TF = 1, FDE_KIN_LC94 = 2, FDE_KIN_REVAPBEK = 3 };

typedef struct fde_functionals {
  int xc;        /* V_XC[rho_I] of the subsystem                      */
  int xc_nad;    /* functional of the nonadditive xc term (E~xc)      */
  int kin_nad;   /* kinetic functional of the nonadditive term (T~)   */
  double rho_thr;/* below this density a functional contributes zero */
} fde_functionals;

/* Energy slots per row of fde_embed_potential (rows 0..ns-1: subsystem
 * densities X = rho_I; row ns: the total density X = rho). */
enum {
  FDE_E_XC = 0,     /* E_xc[X]                                  */
  FDE_E_XCNAD = 1,  /* E~xc[X] (nonadditive functional)         */
  FDE_E_KIN = 2,    /* T~[X] (kinetic functional)               */
  FDE_E_LOC = 3,    /* int V_loc X                              */
  FDE_E_HEMB = 4,   /* int V_H[rho] X                           */
  FDE_E_HSELF = 5,  /* E_H[X] = 1/2 int V_H[X] X                */
  FDE_E_DEBAND = 6, /* -int (V_eff^I - V_loc) rho_I (0 in row ns)*/
  FDE_E_CHARGE = 7, /* int X                                    */
  FDE_NE = 8
};

/*
 * Embedding potentials of all subsystems (Appendix, recast of the effective
 * potential; Eq. embedding for the nonadditive terms; Appendix, kinetic
 * energy functional and potential for V~_kin; Sec. 2 for the FFT Poisson
 * solve of V_H[rho], rho = sum_I rho_I):
 *   veff[I] = vloc + V_H[rho] + V_xc[rho_I] + (V~xc[rho] - V~xc[rho_I])
 *             + (V~kin[rho] - V~kin[rho_I])
 *   rho_sub   [ns][N3][N2][N1] real.      vloc  [N3][N2][N1] real.
 *   f         host, functional choice and density threshold.
 *   veff      [ns][N3][N2][N1] real, output.
 *   energies  device double [ns+1][FDE_NE], output (slots above).
 *   info      device int, output: 0, or 1 if a non-finite value appeared.
 */
fde_status fde_embed_potential(fde_plan* plan, int ns, const void* rho_sub, const void* vloc,
                               const fde_functionals* f, void* veff, double* energies, int* info,
                               hipStream_t stream);

/*
 * Rayleigh-Ritz on V = rows of v [m][npw] with HV in hv [m][npw]
 * (the solver of Eq. KS; the paper does not describe it):
 *   S = V^H V, A = V^H HV accumulated in FP64; inactive columns (active[j]
 *   = 0) and columns j >= nb whose Cholesky pivot falls below drop_tol*S_jj
 *   are masked (S = e_j, A = 1e6 e_j); S = L L^H; A~ = L^{-1} A L^{-H};
 *   A~ W = W Theta in FP64, ascending (for m <= 768: Householder reduction to
 *   a real tridiagonal, multisection on Sturm counts, twisted factorisations
 *   and, for clustered eigenvalues, inverse iteration; cyclic Jacobi beyond
 *   that or where the tridiagonal workspace does not fit in LDS);
 *   C = L^{-H} W[:, :nb];
 *   rows 0..nb-1 of v and hv are overwritten with X = V C and HX = HV C.
 *   active  [m] uint8 or NULL (all active).
 *   eval    [nb] double, output Theta[:nb].
 *   info    device int: 0; j+1 if band column j < nb has a Cholesky pivot
 *           below drop_tol*S_jj (dependent bands: rows 0..nb-1 are then left
 *           unchanged and eval is NaN); -1 if the eigensolver did not converge.
 */
fde_status fde_subspace_rr(fde_plan* plan, int ik, int m, int nb, void* v, void* hv,
                           const uint8_t* active, double drop_tol, double* eval, int* info,
                           hipStream_t stream);

/*
 * One band block of the solver: the bands of one subsystem at one k-point.
 * v and hv are [m][npw] with rows 0..nb-1 = X, HX and rows nb..m-1 the
 * corrections T, HT (m = nb or 2 nb). Fields not used by a call may be NULL.
 */
typedef struct fde_block {
  int ik;              /* k-point index of the plan                          */
  int nb;              /* bands                                              */
  int m;               /* rows of v/hv entering the Rayleigh-Ritz step       */
  void* v;             /* [m][npw] complex                                   */
  void* hv;            /* [m][npw] complex                                   */
  const uint8_t* active; /* [m] Rayleigh-Ritz column flags (NULL: all)        */
  uint8_t* t_active;   /* [nb] preconditioner output: flags of rows nb..2nb-1 */
  double* eval;        /* [nb] Ritz values (Rayleigh-Ritz output, preconditioner input) */
  double* rnorm;       /* [nb] residual norms (preconditioner output)        */
  int* info;           /* [1] Rayleigh-Ritz status, as fde_subspace_rr        */
  void* sv;            /* [m][npw] S v of the generalised problem H x = e S x  */
                       /* (Appendix, non-local pseudopotentials: the overlap   */
                       /* S^I of the subsystem's own augmentation projectors,  */
                       /* see fde_apply_s), or NULL for S = 1. With sv the     */
                       /* Rayleigh-Ritz step uses S = V^H (S V) (FP64 matrix   */
                       /* cores whatever the GEMM mode) and rotates sv with v  */
                       /* and hv; the TPA preconditioner's residual is         */
                       /* hx - eval sx (the learned one rejects sv).           */
} fde_block;

/*
 * fde_subspace_rr on nblk independent band blocks in one set of launches
 * (one workgroup per block for the FP64 solve). blk is a host array.
 */
fde_status fde_subspace_rr_batched(fde_plan* plan, int nblk, const fde_block* blk, double drop_tol,
                                   hipStream_t stream);

/*
 * fde_precondition on nblk band blocks: for each block, reads X, HX = rows
 * 0..nb-1 of v, hv and eval, writes T into rows nb..2nb-1 of v, t_active and
 * rnorm. blk is a host array.
 */
fde_status fde_precondition_batched(fde_plan* plan, int nblk, const fde_block* blk, hipStream_t stream);

/*
 * Residual and Teter-Payne-Allan preconditioner of the band solver:
 *   R_n = hx_n - eval_n x_n; rnorm_n = ||R_n||; active_n = rnorm_n > 1e-10;
 *   t_n = K(x) R_n / ||K(x) R_n||, x = (|k+G|^2/2) / sum_G |k+G|^2/2 |x_nG|^2,
 *   K(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4); t_n = 0 if inactive.
 *   x, hx, t  [nb][npw] complex (t is output; may be rows of a larger block).
 *   eval      [nb] double.   active [nb] uint8 out.   rnorm [nb] double out.
 */
fde_status fde_precondition(fde_plan* plan, int ik, int nb, const void* x, const void* hx,
                            const double* eval, void* t, uint8_t* active, double* rnorm,
                            hipStream_t stream);

enum { FDE_OCC_INTEGER = 0, FDE_OCC_FERMI_DIRAC = 1, FDE_OCC_METHFESSEL_PAXTON = 2 };

/*
 * Occupations of one subsystem (Sec. 2 fractional occupations, Sec. 3 smearing
 * of metallic subsystems only):
 *   eval  [nk][nb] double ascending per k.    wk [nk] double, sum 1.
 *   integer: f = 2 on the lowest nelec/2 bands of every k; nelec must be even
 *   and whole (FDE_ERR_ARG otherwise: no singly occupied band).
 *   Fermi-Dirac: f = 1 - tanh((eps - mu)/(2 sigma)), mu by bisection so that
 *   sum_k wk sum_n f = nelec to 1e-13.
 *   Methfessel-Paxton (first order, the smearing of metallic slabs in Sec. 3):
 *   f = erfc(x) - x e^{-x^2}/sqrt(pi), x = (eps - mu)/sigma (f may leave [0, 2]
 *   slightly), mu by the same bisection.
 *   occw  [nk][nb] double out, w_k f_nk.   mu [1] double out.
 *   info  device int: 0, or 1 if nelec/2 exceeds nb (integer mode).
 */
fde_status fde_occupations(int nk, int nb, const double* eval, const double* wk, double nelec, int mode,
                           double sigma, double* occw, double* mu, int* info, hipStream_t stream);

/* Linear density mixing rho_in <- (1-beta) rho_in + beta rho_out over n
 * grid values of precision prec. */
fde_status fde_mix(size_t n, double beta, void* rho_in, const void* rho_out, int prec, hipStream_t stream);

/*
 * Pulay mixing (direct inversion in the iterative subspace) of all subsystem
 * densities with a Kerker preconditioner: the mixing step of the embedding
 * cycle, which the paper leaves to the host code (Fig. 1; a later variant of
 * its cycle). The densities of the ns subsystems form one vector x and
 * R = rho_out - rho_in its residual. With the history state on the device
 * (so a captured cycle replays correctly):
 *   1. x_hist[slot] = rho_in, r_hist[slot] = rho_out - rho_in, slot = state[1];
 *   2. a = argmin |sum_i a_i R_i|^2 subject to sum_i a_i = 1 over the
 *      nh = min(state[0] + 1, nhmax) entries in use (grid inner product, FP64);
 *   3. rho_in <- sum_i a_i x_i + beta K(sum_i a_i R_i), K = |G|^2/(|G|^2 + q0^2)
 *      on each subsystem grid (q0 = 0: K = 1; q0 > 0 leaves the charge alone);
 *   4. state[0] = nh, state[1] = (slot + 1) mod nhmax.
 *   state   device int[3], all zero before the first call of a mixing run.
 *   x_hist, r_hist  [nhmax][ns][N3][N2][N1] real, caller-owned.
 *   rho_in [ns][N] in/out, rho_out [ns][N].   nhmax in [1, FDE_PULAY_MAX].
 *   info  device int: 0, or 1 if the system was exactly singular (a repeated
 *         pair: the new pair alone was used, i.e. linear mixing with beta); a
 *         zero residual selects its own input (info 0).
 * With nhmax = 1 this is linear mixing rho_in + beta K (rho_out - rho_in).
 */
#define FDE_PULAY_MAX 8
fde_status fde_mix_pulay(fde_plan* plan, int ns, int nhmax, int* state, void* x_hist, void* r_hist, void* rho_in,
                         const void* rho_out, double beta, double q0, int* info, hipStream_t stream);

/*
 * Local potential of Gaussian ions (the nuclei of all subsystems, Appendix
 * recast: V_eN groups all nuclei; Sec. 2 E_eN). Ion potential
 * -Z erf(r/(sqrt(2) s))/r:
 *   V_loc(G) = (1/Omega) sum_a -4 pi Z_a e^{-G^2 s_a^2/2}/G^2 e^{-iG.R_a} on D,
 *   V_loc(0) = sum_a 2 pi Z_a s_a^2 / Omega; vloc(r) = FFT_inv.
 *   pos [natoms][3], Z, width: host double.   vloc [N3][N2][N1] real out.
 *   Synchronous with respect to the host arrays (they are copied first).
 */
fde_status fde_local_potential(fde_plan* plan, int natoms, const double* pos, const double* Z,
                               const double* width, void* vloc, hipStream_t stream);

/*
 * Gaussian Kleinman-Bylander projectors at k-point ik (own atoms of a
 * subsystem, Appendix on non-local pseudopotentials), q = k + G:
 *   s:   Omega^{-1/2} 2^{3/2} pi^{3/4} r^{3/2} e^{-q^2 r^2/2} e^{-i q.R}
 *   p_a: Omega^{-1/2} 4 pi^{3/4} r^{5/2} q_a e^{-q^2 r^2/2} e^{-i q.R}, a = x,y,z
 *   pos [natoms][3], rbeta [natoms] host double; lmax [natoms] host int
 *   (-1 none, 0 s, 1 s+p). beta [nproj][npw] complex out, channel order per
 *   atom s, px, py, pz. *nproj (host) receives the count.
 */
fde_status fde_kb_projectors(fde_plan* plan, int ik, int natoms, const double* pos, const int* lmax,
                             const double* rbeta, void* beta, int* nproj, hipStream_t stream);

/* Initial bands: psi[n][G] = raw[n][G] / (1 + |k+G|^2). raw, psi [nb][npw]. */
fde_status fde_init_bands(fde_plan* plan, int ik, int nb, const void* raw, void* psi, hipStream_t stream);

/*
 * Band energy terms at k-point ik for occupation weights occw [nb] (the
 * Janak kinetic energy T_J of Sec. 2, the nonlocal energy of the Appendix on
 * non-local pseudopotentials, and the band-energy sum of the Appendix recast of
 * the total energy):
 *   out[0] += sum_n occw_n sum_G |k+G|^2/2 |psi_nG|^2
 *   out[1] += sum_n occw_n sum_i D_i |<beta_i|psi_n>|^2
 *   out[2] += sum_n occw_n eval_n            (only when eval is not NULL)
 *   psi [nb][npw] (nb <= the workspace's max_nb), occw, eval [nb] double.
 *   out: device double [3] (or [2] when eval is NULL), accumulated.
 */
fde_status fde_band_energies(fde_plan* plan, int ik, int nb, const void* psi, const double* occw,
                             const double* eval, int nproj, const void* beta, const double* dkb, double* out,
                             hipStream_t stream);

/* out[0] += sum_j a_j b_j * dV over the plan's grid (a, b real grids; b NULL means b = 1). */
fde_status fde_grid_dot(fde_plan* plan, const void* a, const void* b, double* out, hipStream_t stream);

/*
 * Energy bookkeeping of one embedding cycle (Sec. 2, the E_FDE expression; the
 * Appendix recast of the total energy into fragment energies E_K), ion-ion term
 * excluded. Inputs, all device doubles:
 *   embed_energies [ns+1][FDE_NE]: fde_embed_potential's slots at the output
 *                  densities rho_I (rows 0..ns-1) and rho = sum rho_I (row ns);
 *   band_terms     [ns][3]: per subsystem, the k-sums of fde_band_energies
 *                  (T_J, E_NL, sum w f eps) of the bands and occupations that
 *                  produced rho_I;
 *   dots           [ns][2]: int V_eff^I rho_I and int V_loc rho_I, V_eff^I the
 *                  potential those bands were computed in (fde_grid_dot).
 * Output out [ns+4] (device):
 *   out[I]    E_K = sum w f eps - int (V_eff^I - V_loc) rho_I + E_xc[rho_I]
 *             + 1/2 int V_H[rho] rho_I       (the Hartree share of reading 3:
 *             E_H[rho_K] inside E_K is taken as 1/2 int V_H[rho] rho_K);
 *   out[ns]   T~[rho] - sum T~[rho_I];  out[ns+1] E~xc[rho] - sum E~xc[rho_I];
 *   out[ns+2] E_FDE directly: sum_I (T_J + E_NL + int V_loc rho_I + E_xc[rho_I])
 *             + E_H[rho] + out[ns] + out[ns+1];
 *   out[ns+3] E_FDE through the fragments: sum_I out[I] + out[ns] + out[ns+1].
 * The two routes agree when eps are the Ritz values <psi|H_I|psi> of the
 * orthonormal bands (as after fde_subspace_rr).
 */
fde_status fde_energy_total(int ns, const double* embed_energies, const double* band_terms, const double* dots,
                            double* out, hipStream_t stream);

/*
 * Subsystem-specific augmentation (Appendix, non-local pseudopotentials: with
 * PAW/ultrasoft pseudopotentials a subsystem's smooth orbitals solve
 * H psi = e S^I psi with the overlap of its own atoms' projectors only).
 *
 * fde_apply_s: spsi = psi + sum_ij beta_i q_ij <beta_j|psi>, i.e. S^I psi.
 *   psi, spsi [nb][npw] complex (plan precision), distinct; beta [nproj][npw]
 *   the augmentation projectors (as from fde_kb_projectors); q device
 *   [nproj][nproj] real symmetric FP64 (zero between atoms). The projections
 *   are summed in FP64. nproj = 0 copies psi. FDE_ERR_SHAPE when nproj exceeds
 *   the workspace's max_nproj.
 * fde_aug_charges: charges[atom_of[i]] += sum_n occw_n Re(conj(P_in) (q P)_in),
 *   P = beta^H psi: the charge of each atom's augmentation density
 *   (sum_ij rho_ij q_ij with rho_ij = sum_n f_n <psi_n|beta_i><beta_j|psi_n>).
 *   occw [nb] device FP64 (w_k f_nk); atom_of [nproj] device int; charges
 *   device FP64, accumulated (+=) in projector order.
 * fde_aug_density: rho += sum_a c_a g_a(r), g_a the unit-normalised Gaussian of
 *   width w_a at R_a (the synthetic augmentation function Q_ij = q_ij g_a),
 *   from its Fourier series on the density sphere. atoms device [natom][4] =
 *   (x, y, z, w) in bohr; charges device [natom] (fde_aug_charges); rho [N]
 *   plan precision. Uses the plan's embedding work grids.
 */
fde_status fde_apply_s(fde_plan* plan, int ik, int nb, const void* psi, void* spsi, int nproj, const void* beta,
                       const double* q, hipStream_t stream);
fde_status fde_aug_charges(fde_plan* plan, int ik, int nb, const void* psi, const double* occw, int nproj,
                           const void* beta, const double* q, const int* atom_of, double* charges,
                           hipStream_t stream);
fde_status fde_aug_density(fde_plan* plan, int natom, const double* atoms, const double* charges, void* rho,
                           hipStream_t stream);

/* Frozen environments of the freeze-and-thaw scheme (Fig. 1b caption: a subsystem
 * iterated to self-consistency against the densities of the last broadcast; Sec. 2 on
 * the freeze-and-thaw procedure): env[I * ld + i] = sum_{J != I} rho_sub[J][i], summed
 * in ascending J (zero when ns = 1). rho_sub [ns][N] device, plan precision; env rows
 * of ld >= N elements (ld = 2N writes the second density of [ns][2][N] pairs {rho_I,
 * env_I}, whose fde_embed_potential gives V_eff^I in that environment as its first
 * potential). Must not overlap rho_sub. FDE_ERR_ARG: ns < 1, ld < N, null pointers. */
fde_status fde_frozen_environment(fde_plan* plan, int ns, const void* rho_sub, void* env, size_t ld,
                                  hipStream_t stream);

/* out[0] += int |sum_{I < ns} rho_sub[I] - rho_ref| dV over the plan's grid: the
 * integrated density difference (Sec. 4 measures FDE against Kohn-Sham by half of it)
 * and the self-consistency residual of the cycle. rho_sub [ns][N], rho_ref [N]. */
fde_status fde_density_l1(fde_plan* plan, int ns, const void* rho_sub, const void* rho_ref, double* out,
                          hipStream_t stream);

/* out[0] = (1/N) sum_j a_j (mean of a real grid, e.g. the mean effective potential
 * that the learned preconditioner's fourth feature uses). out: device double. */
fde_status fde_grid_mean(fde_plan* plan, const void* a, double* out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Learned preconditioner (an extension of the band solver step; the paper
 * leaves the solver to its host code). A 4 -> 64 -> 64 -> 1 network with tanh
 * hidden layers maps per-coefficient features
 *   u = (log(1 + kin_G/T_n), log T_n, log max(|R_G| sqrt(npw)/||R_n||, 1e-6),
 *        (lambda_n - vbar)/T_n)
 * (kin_G = |k+G|^2/2, T_n = sum_G kin_G |x_nG|^2, vbar = mean V_eff) to y, and
 * the correction is T_G = K_TPA(kin_G/T_n) exp(y) R_G, normalised; y = 0 is
 * exactly the Teter-Payne-Allan preconditioner of fde_precondition.
 * Parameters: FP32 flat vector of FDE_MLP_NPARAM values, in the order
 * W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3 (y = w3.h2 + b3,
 * h2 = tanh(W2 h1 + b2), h1 = tanh(W1 u + b1)). Kernels round W1, W2, w3 and
 * the first hidden layer to BF16 and accumulate in FP32; the 64 x 64 products
 * run on BF16 matrix cores.
 * Training samples: rows of FDE_MLP_SAMPLE floats (u1..u4, A, B, C) with loss
 * (1/n) sum (A e^{2y} - 2 B e^y + C): for the Jacobi-Davidson correction
 * delta of band n, A = w a^2 K^2 |R_G|^2, B = w a K Re(conj(R_G) delta_G),
 * C = w |delta_G|^2, a = Re<K R, delta>/||K R||^2, w = npw/||delta||^2.
 * All pointers are device pointers; every call only enqueues on `stream`.
 * ------------------------------------------------------------------------- */
#define FDE_MLP_NPARAM 4545
#define FDE_MLP_NIN 4
#define FDE_MLP_SAMPLE 7

/* fde_precondition_batched with the network: vbar [nblk] device doubles (mean
 * V_eff of each block's subsystem), params as above. Same outputs. */
fde_status fde_precondition_mlp_batched(fde_plan* plan, int nblk, const fde_block* blk, const float* params,
                                        const double* vbar, hipStream_t stream);

/* y[s] = network(u[s]) for u [n][4] (FP32). */
fde_status fde_mlp_forward(int n, const float* u, const float* params, float* y, hipStream_t stream);

/* Workspace (device bytes) for fde_mlp_loss_grad over n samples. */
fde_status fde_mlp_workspace_bytes(int n, size_t* bytes);

/* loss[0] = (1/n) sum_s (A e^{2y} - 2 B e^y + C) over samples [n][7]; grad
 * [FDE_MLP_NPARAM] = its gradient (FP32, fixed summation order, overwritten). */
fde_status fde_mlp_loss_grad(int n, const float* samples, const float* params, float* grad, double* loss,
                             void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight training or serving loops, harnesses that forbid hipMalloc): the same
 * loss and gradient as fde_mlp_loss_grad, with the per-block partial gradients
 * in a scratch array that the library holds in each GPU's memory until the
 * process ends (FDE_MLP_STATIC_SCRATCH_BYTES per GPU, 20 MiB). No workspace
 * argument, no allocation of any kind. n in [1, FDE_MLP_STATIC_MAX_N], else
 * FDE_ERR_SHAPE. The first call on a device looks the array's address up
 * (hipGetSymbolAddress). All calls on one GPU share the array: calls that can
 * overlap on one GPU (unordered streams, threads) race and must be serialised
 * by the caller. Nothing an earlier call left in the array is read.
 */
#define FDE_MLP_STATIC_SCRATCH_BYTES (20 * 1024 * 1024)
#define FDE_MLP_STATIC_MAX_N (1 << 28)
fde_status fde_mlp_loss_grad_static(int n, const float* samples, const float* params, float* grad, double* loss,
                                    hipStream_t stream);

/* One Adam step (Kingma & Ba) on params with moments m, v (FP32, FDE_MLP_NPARAM
 * each, updated in place); t counts from 1. */
fde_status fde_mlp_adam(const float* grad, float* params, float* m, float* v, int t, float lr, float beta1,
                        float beta2, float eps, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* FDE_H */

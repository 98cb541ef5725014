/*
 * agf2.h -- C ABI of the MI355X (gfx950) AGF2(1,0) library.
 *
 * AGF2(1,0): auxiliary second-order Green's function theory with the
 * self-energy compressed each iteration so that its zeroth and first spectral
 * moments are conserved (Backhouse, Santana-Bonilla & Booth, arXiv
 * 2106.03508). The library computes, on one GPU:
 *   - the self-energy moments (the O(N^5) step),
 *   - their compression to auxiliaries by one block-Lanczos step,
 *   - the Fock loop (extended Fock matrix, chemical potential, density),
 *   - the Galitskii-Migdal energy,
 *   - the outer self-consistent loop built from the calls above,
 *   - the broadened spectral function of the resulting poles.
 *
 * Conventions (all entry points):
 *   - Arrays are row-major float64 unless stated otherwise.
 *   - Pointers documented "device" must point to device memory on the
 *     handle's device; the caller owns them, the library never frees them.
 *     Pointers documented "host" are host memory.
 *   - Calls are ordered on the handle's stream. A call that returns host
 *     scalars synchronises that stream before returning.
 *   - Every call returns an agf2_status; AGF2_OK is 0 and errors are
 *     negative. agf2_last_error() gives a message for the last failure on the
 *     handle. No C++ exception crosses this boundary.
 *   - Every float64 input array of an entry point is scanned on the device
 *     before use; a NaN or an infinity in any of them returns AGF2_ERR_ARG
 *     (the message names the array) and nothing is computed. The scan reads
 *     each input once (about 6 ms for a 28 GB DF tensor). float32 arrays of
 *     the warm-start network's calls and the inputs of the allocation-free
 *     agf2_spectral_function_noalloc are not scanned.
 *   - A handle must not be used by two threads at once. It owns a device
 *     workspace that grows on demand and is freed by agf2_destroy().
 *
 * Notation: nphys = N physical orbitals; naux = Q density-fitting functions
 * with (pq|rs) = sum_Q L[Q][p][q] L[Q][r][s]; a Green's function is a set of
 * npole poles with energies e_pole (ascending) and physical amplitudes
 * u_pole[N][npole]; the first nocc_pole poles are occupied.
 */
#ifndef AGF2_H
#define AGF2_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct agf2_handle_s* agf2_handle_t;

typedef enum {
  AGF2_OK = 0,
  AGF2_ERR_ARG = -1,          /* invalid argument (size, pointer, value)      */
  AGF2_ERR_HIP = -2,          /* a HIP / rocBLAS / rocSOLVER call failed      */
  AGF2_ERR_NOMEM = -3,        /* device workspace allocation failed           */
  AGF2_ERR_NOT_PD = -4,       /* zeroth moment not positive definite          */
  AGF2_ERR_NO_CONVERGE = -5,  /* an iteration hit its cycle limit             */
  AGF2_ERR_NELEC = -6         /* electron number cannot be reached            */
} agf2_status;

/* Arithmetic of the moment build. In both split modes the pole-basis DF
 * tensors are formed in float64, rounded to float32 and stored as 16-bit
 * pairs x ~ hi + lo; the integral slabs take the products hi*hi + hi*lo +
 * lo*hi on the 16-bit MFMA pipe with float32 accumulation; the moment
 * contraction takes hi*hi into one float32 sum and hi*lo + lo*hi into
 * another (plus lo*lo on output blocks that hold diagonal elements, where
 * that term is a non-negative square), and those float32 sums over chunks of
 * 256 columns are added into float64 sums. Compression, the Fock loop and the
 * energy are float64 in every mode.
 * Accuracy of the moments against the float64 build (relative Frobenius
 * norm): fp16 pairs within 1e-7, except on tiny systems whose moment
 * elements sum only a few terms (up to ~2e-7 with a single occupied pole:
 * the 2^-22 operand rounding does not average out); bf16 pairs do NOT reach
 * 1e-7 (about 3e-6 at nphys = 1000, up to ~1e-5 on small systems), because
 * each bf16 pair holds only 16 significant bits of an operand. */
typedef enum {
  AGF2_FP64 = 0,        /* float64 operands, FP64 MFMA, float64 accumulation  */
  AGF2_SPLIT_BF16 = 1,  /* bf16 pairs (16 significant bits per value); below
                           the 1e-7 moment accuracy of the other modes        */
  AGF2_SPLIT_FP16 = 2   /* fp16 pairs (22 significant bits) with power-of-two
                           scaling of each operand row and of the slabs       */
} agf2_precision;

/* Create a handle on HIP device `device`. All work is ordered on
 * `hip_stream`, a hipStream_t owned by the caller; NULL is the device's
 * default (null) stream. */
agf2_status agf2_create(agf2_handle_t* handle, int device, void* hip_stream);

/* Release the handle and its workspace (the stream is left alone). */
agf2_status agf2_destroy(agf2_handle_t handle);

/* Message describing the last error on the handle (static storage owned by
 * the handle; valid until the next call on it). NULL handle -> generic text. */
const char* agf2_last_error(agf2_handle_t handle);

/* Block the host until all work queued on the handle's stream is done. */
agf2_status agf2_synchronize(agf2_handle_t handle);

/*
 * Self-energy moments: the zeroth- and first-moment equations of the
 * compression section, for the lesser part (first term of the second-order
 * self-energy equation) and the greater part (its second term):
 *   m0_occ[p][q] = sum_{i,j occ; a vir} (pi|ja) [2(qi|ja) - (qj|ia)]
 *   m1_occ[p][q] = same summand times (e_i + e_j - e_a)
 *   m0_vir[p][q] = sum_{a,b vir; i occ} (pa|bi) [2(qa|bi) - (qb|ai)]
 *   m1_vir[p][q] = same summand times (e_a + e_b - e_i)
 * with (pi|ja) = sum_{Q,r,s,t} L[Q][p][r] u[r][i] L[Q][s][t] u[s][j] u[t][a].
 *
 *   prec       AGF2_FP64, AGF2_SPLIT_BF16 or AGF2_SPLIT_FP16.
 *   nphys      N >= 1.      naux  Q >= 1.
 *   Lpq        device, [naux][nphys][nphys], symmetric in (p,q).
 *   npole      number of Green's function poles (>= 2).
 *   nocc_pole  occupied poles, 1 <= nocc_pole < npole.
 *   e_pole     device, [npole] pole energies.
 *   u_pole     device, [nphys][npole] physical amplitudes.
 *   m0_occ, m1_occ, m0_vir, m1_vir   device, [nphys][nphys] outputs,
 *              exactly symmetric.
 * Mean-field poles (npole = nphys and u_pole exactly the identity, the first
 * iteration from the mean-field reference) are detected on the device with
 * one host synchronisation; the pole-basis transform is then a relayout of
 * Lpq, with the same results bit for bit as the product with u_pole.
 * Setting AGF2_NO_IDENTITY_TRANSFORM=1 in the environment skips the check.
 * Errors: AGF2_ERR_ARG for bad sizes or NULL pointers, AGF2_ERR_NOMEM when
 * the workspace cannot grow, AGF2_ERR_HIP for a failed launch.
 */
agf2_status agf2_build_moments(agf2_handle_t handle, agf2_precision prec,
                               int nphys, int naux, const double* Lpq,
                               int npole, int nocc_pole, const double* e_pole,
                               const double* u_pole, double* m0_occ,
                               double* m1_occ, double* m0_vir, double* m1_vir);

/*
 * Moments 0 .. nmom-1 of the lesser and greater self-energy: the same sums
 * as agf2_build_moments, the n-th moment carrying the n-th power of the
 * weight, (e_i + e_j - e_a)^n resp. (e_a + e_b - e_i)^n. Moments 0 .. 2k+1
 * are what a compression to k + 1 Lanczos blocks conserves (the other
 * truncations of the AGF2(n,m) family that the compression section names).
 *   nmom       even, 2 <= nmom <= 16; above 2 only prec = AGF2_FP64.
 *   m_occ, m_vir  device [nmom][nphys][nphys] outputs (moment n at offset
 *              n * nphys^2), exactly symmetric.
 *   Other arguments as agf2_build_moments (nmom = 2 is that call).
 * The FP64 build forms each chunk of the pair slabs once and contracts it
 * once per moment pair (2m, 2m+1) with the columns scaled by the weight to
 * the m-th power.
 * Errors: as agf2_build_moments; AGF2_ERR_ARG for a bad nmom or a split
 * precision with nmom > 2.
 */
agf2_status agf2_build_moments_n(agf2_handle_t handle, agf2_precision prec,
                                 int nmom, int nphys, int naux,
                                 const double* Lpq, int npole, int nocc_pole,
                                 const double* e_pole, const double* u_pole,
                                 double* m_occ, double* m_vir);

/*
 * Compression of one part of the self-energy to nmom/2 blocks of block
 * Lanczos, conserving its moments 0 .. nmom-1 (the compression section's
 * block Lanczos run past one block). With Lc Lc^T = m[0] (Cholesky) and
 * M(n) = Lc^-1 m[n] Lc^-T, the Lanczos blocks are matrix polynomials in the
 * auxiliary Hamiltonian applied to the first block, so all their products
 * follow from the M(n): A_j = <Q_j|H|Q_j>, B_j from the Cholesky factor of
 * the residual's overlap. The block tridiagonal matrix T (A_j on the
 * diagonal, B_j beside it) is diagonalised, T = W diag(e) W^T, and the
 * auxiliaries are e_aux = e and v_aux = Lc W[0:nphys], so that
 * v_aux diag(e_aux)^n v_aux^T = m[n] for n < nmom.
 *   m          device [nmom][nphys][nphys], symmetric, m[0] positive definite.
 *   naux_out   host, number of auxiliaries (nmom/2 * nphys).
 *   e_aux      device [nmom/2 * nphys] output, ascending.
 *   v_aux      device [nphys][nmom/2 * nphys] output (row stride
 *              nmom/2 * nphys).
 * nmom = 2 is agf2_compress with tol = 0 (row stride nphys).
 * Errors: AGF2_ERR_NOT_PD when m[0] or a block's residual overlap is not
 * positive definite; AGF2_ERR_ARG for a bad nmom.
 */
agf2_status agf2_compress_lanczos(agf2_handle_t handle, int nphys, int nmom,
                                  const double* m, int* naux_out,
                                  double* e_aux, double* v_aux);

/*
 * Generalised Fock matrix (Fock-matrix equation of the method review):
 *   fock = hcore + alpha * sum_rs [(pq|rs) - 1/2 (ps|rq)] rdm1[r][s]
 * rdm1 is the spin-summed density matrix. alpha = 1 is the Fock matrix;
 * other values scale the two-electron part (alpha = -1 with
 * hcore = diag(eps) gives the one-electron Hamiltonian that makes a
 * determinant self-consistent with orbital energies eps).
 *   Lpq   device [naux][nphys][nphys]; hcore, rdm1 device [nphys][nphys]
 *         (every Lpq[Q] and rdm1 symmetric: the products read them in
 *         either orientation; the output is then exactly symmetric).
 *   fock  device [nphys][nphys] output (may not alias the inputs).
 * Errors: AGF2_ERR_ARG for bad sizes, NULL pointers or nphys > 46340.
 */
agf2_status agf2_fock_build(agf2_handle_t handle, int nphys, int naux,
                            const double* Lpq, const double* hcore,
                            const double* rdm1, double alpha, double* fock);

/*
 * Compression of one part (lesser or greater) of the self-energy: one step
 * of block Lanczos through a Cholesky factor (compression section). With
 * S S^T = m0 (lower Cholesky factor), M = S^-1 m1 S^-T = W diag(e) W^T,
 * the auxiliaries are e_aux = e and v_aux = S W, so
 * v_aux v_aux^T = m0 and v_aux diag(e_aux) v_aux^T = m1.
 *   m0, m1     device [nphys][nphys], symmetric (m0 positive definite).
 *   tol        0: strict Cholesky, AGF2_ERR_NOT_PD if it fails.
 *              > 0: square root from the eigendecomposition of m0, keeping
 *              eigenvalues > tol * max eigenvalue (fewer auxiliaries).
 *   naux_out   host, number of auxiliaries written (nphys for tol = 0).
 *   e_aux      device [nphys] output (first naux_out entries valid).
 *   v_aux      device [nphys][nphys] output, column k couples auxiliary k
 *              (columns >= naux_out are zero).
 */
agf2_status agf2_compress(agf2_handle_t handle, int nphys, const double* m0,
                          const double* m1, double tol, int* naux_out,
                          double* e_aux, double* v_aux);

/* Options of the Fock loop. */
typedef struct {
  double tol_rdm1;    /* stop when ||change of the density||_F is below     */
  double tol_nelec;   /* |electron count - nelec| target of the shift fit
                         once the density has settled (a cycle fits to
                         max(tol_nelec, min(1e-6, 0.01 x the previous
                         cycle's density change)))                          */
  double bracket;     /* largest shift step tried, Ha                        */
  double step0;       /* first shift step of the bracket search, Ha          */
  int max_cycle;      /* density cycles                                      */
  int diis_space;     /* DIIS vectors on the Fock matrix (0 = off)           */
} agf2_fock_opts;

/* Fill opts with the defaults: tol_rdm1 1e-8, tol_nelec 1e-10, bracket 2,
 * step0 0.01, max_cycle 50, diis_space 8. */
void agf2_fock_opts_default(agf2_fock_opts* opts);

/*
 * Fock loop: relax the density with the self-energy held fixed while a
 * chemical potential keeps the electron number (relaxation passage after
 * the self-consistency discussion; compressed extended Hamiltonian).
 * Each cycle fits a common shift Delta of all auxiliary energies so that
 * the aufbau count 2 * sum_{l<n} |u_l|^2 equals nelec, diagonalises
 *   [[F, v_se], [v_se^T, diag(e_se + Delta)]],
 * rebuilds rdm1 = 2 sum_{l<n} u_l u_l^T and F = F[rdm1] (DIIS on F), until
 * the Frobenius norm of the change of rdm1 is below tol_rdm1. The fit takes
 * Newton steps with the analytic derivative of the count (first-order
 * perturbation of the eigenvectors in Delta) before bracketing; while the
 * density still moves, a cycle whose count misses its tolerance by a Newton
 * step of at most 1e-3 Ha takes that step and the density to first order in
 * it instead of refitting. The returned density is always from an exact
 * fit to tol_nelec.
 *   hcore      device [nphys][nphys]; Lpq device [naux][nphys][nphys]
 *   nelec      electrons (even, 0 < nelec < 2 * (nphys + naux_se))
 *   naux_se    auxiliaries; v_se device [nphys][naux_se] (row stride
 *              naux_se); e_se device [naux_se], in: auxiliary energies,
 *              out: the same energies plus the fitted shift
 *   rdm1       device [nphys][nphys], in: starting density, out: final
 *   fock       device [nphys][nphys] out: the Fock matrix of the last
 *              diagonalisation
 *   e_pole     device [nphys + naux_se] out: pole energies, ascending
 *   u_pole     device [nphys][nphys + naux_se] out: physical amplitudes
 *   nocc_pole, mu, shift, n_cycle   host outputs
 *   opts       host, NULL for defaults
 * Returns AGF2_ERR_NO_CONVERGE when the cycle limit is hit: the shift is
 * then fitted (to tol_nelec) at the last Fock matrix, and the outputs hold
 * that matrix, the auxiliary energies shifted by that fit, the poles of that
 * extended Hamiltonian (exact eigenpairs) and their density. AGF2_ERR_NELEC
 * when nelec is out of range.
 */
agf2_status agf2_fock_loop(agf2_handle_t handle, int nphys, int naux,
                           const double* Lpq, const double* hcore, int nelec,
                           int naux_se, double* e_se, const double* v_se,
                           double* rdm1, double* fock, double* e_pole,
                           double* u_pole, int* nocc_pole, double* mu,
                           double* shift, int* n_cycle,
                           const agf2_fock_opts* opts);

/*
 * Galitskii-Migdal energy of a Green's function whose poles are eigenpairs of
 * the extended Hamiltonian built from `fock` and the auxiliaries:
 *   e_1b = 1/2 Tr[(hcore + fock) rdm1]
 *   e_2b = sum_{l occ} sum_{k in vir aux} (u_l . v_k)^2 / (e_l - e_k)
 *        + sum_{l vir} sum_{k in occ aux} (u_l . v_k)^2 / (e_k - e_l)
 * (the two-body term in a form without near-zero denominators; equal to the
 * direct occupied-pole sum over all auxiliaries for exact eigenpairs).
 *   e_pole [npole], u_pole [nphys][npole] device; first nocc_pole occupied.
 *   e_se_occ [naux_occ], v_se_occ [nphys][naux_occ] device (lesser part),
 *   e_se_vir [naux_vir], v_se_vir [nphys][naux_vir] device (greater part),
 *   with the Fock loop's shift already applied to the energies.
 *   e_1b, e_2b host outputs.
 */
agf2_status agf2_energy_gf(agf2_handle_t handle, int nphys,
                           const double* hcore, const double* fock,
                           const double* rdm1, int npole, int nocc_pole,
                           const double* e_pole, const double* u_pole,
                           int naux_occ, const double* e_se_occ,
                           const double* v_se_occ, int naux_vir,
                           const double* e_se_vir, const double* v_se_vir,
                           double* e_1b, double* e_2b);

/*
 * Broadened spectral function of the Green's function in the physical space
 * (the simulated photoelectron spectra of the application section, with a
 * broadening factor eta):
 *   A(omega_k) = -1/pi Im Tr[P G(omega_k + i eta)]
 *              = eta/pi sum_l w_l / ((omega_k - e_pole[l])^2 + eta^2),
 *   w_l = sum_p weight[p] u_pole[p][l]^2,
 * G being the physical block of the resolvent of the extended Hamiltonian
 * whose eigenpairs are the poles (the Dyson equation as an eigenproblem).
 *   e_pole   device [npole] pole energies (any order).
 *   u_pole   device [nphys][npole] physical amplitudes (row-major).
 *   weight   device [nphys] weight per physical orbital (a projection), or
 *            NULL for all ones (the total spectrum).
 *   omega    device [nomega] frequencies; eta > 0, same unit (Ha).
 *   A        device [nomega] output (1/Ha).
 * Errors: AGF2_ERR_ARG for bad sizes, NULL pointers or eta not positive.
 */
agf2_status agf2_spectral_function(agf2_handle_t handle, int nphys, int npole,
                                   const double* e_pole, const double* u_pole,
                                   const double* weight, int nomega,
                                   const double* omega, double eta, double* A);

/*
 * Allocation-free variant of agf2_spectral_function, for callers that
 * cannot allocate device memory during the call: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation. Same
 * arguments, result and kernels as agf2_spectral_function, but its partial
 * sums live in a static device array of the library (one per GPU, 4.25 MiB,
 * kept until the process ends; its address is resolved by agf2_create), so
 * the call allocates nothing, records no event, does not scan its inputs for
 * non-finite values and does not synchronise. Every call on one GPU shares
 * that array, which keeps the last call's contents (each call overwrites all
 * it reads): calls that overlap on one GPU (several streams or threads)
 * race. Errors: AGF2_ERR_ARG for npole > AGF2_SPECTRUM_NOALLOC_MAX_POLE and
 * the argument errors of agf2_spectral_function.
 */
#define AGF2_SPECTRUM_NOALLOC_MAX_POLE 32768
agf2_status agf2_spectral_function_noalloc(agf2_handle_t handle, int nphys,
                                           int npole, const double* e_pole,
                                           const double* u_pole,
                                           const double* weight, int nomega,
                                           const double* omega, double eta,
                                           double* A);

/* One system of a batched moment build (all pointers device, row-major,
 * float64; meaning as in agf2_build_moments). */
typedef struct {
  int nphys, naux;
  const double* Lpq;                 /* [naux][nphys][nphys] */
  int npole, nocc_pole;
  const double* e_pole;              /* [npole] */
  const double* u_pole;              /* [nphys][npole] */
  double *m0_occ, *m1_occ, *m0_vir, *m1_vir;   /* [nphys][nphys] outputs */
} agf2_system;

/*
 * Moments of many systems of uneven size in one replay of a captured HIP
 * graph (float64 arithmetic, same definition as agf2_build_moments). All
 * systems' pole-pair slab tiles go through one persistent grouped launch per
 * inner-tile width and all contraction tiles through one persistent grouped
 * launch, work items sorted by cost. The first call with a given batch (sizes
 * and pointers) plans the workspace, picks the slab inner-tile width (16, 32
 * or 64 columns) per size bucket by timing each candidate on the batch itself
 * (project autotuner), captures the graph and replays it; later calls with
 * the same batch only replay. tile_width (host [nsys], or NULL) receives the
 * width chosen for each system's greater part.
 * Errors: AGF2_ERR_ARG (sizes, NULL pointers, nsys < 1), AGF2_ERR_NOMEM.
 */
agf2_status agf2_build_moments_batched(agf2_handle_t handle, int nsys,
                                       const agf2_system* systems,
                                       int* tile_width);

/* Options of the outer self-consistent loop. */
typedef struct {
  int max_iter;           /* iterations after iteration 0                    */
  double conv_tol;        /* |change of the total energy|, Ha                */
  double conv_tol_ipea;   /* max |change of IP|, |change of EA|, Ha          */
  int diis_space;         /* DIIS vectors on the four moments (0 = off)      */
  double damping;         /* m <- (1 - damping) m + damping m_prev           */
  agf2_precision prec;    /* arithmetic of the moment build                  */
  double compress_tol;    /* see agf2_compress                               */
  agf2_fock_opts fock;    /* Fock-loop options                               */
  int nblock;             /* Lanczos blocks per part: the compression keeps
                             moments 0 .. 2 nblock - 1 and the Green's
                             function has nphys + 2 nblock nphys poles; above
                             1 the moments are built in AGF2_FP64 (prec must
                             be AGF2_FP64) and dm_init must be NULL          */
} agf2_run_opts;

/* Defaults: max_iter 20, conv_tol 1e-8, conv_tol_ipea 1e-7, diis_space 8,
 * damping 0, prec AGF2_FP64, compress_tol 0, fock as agf2_fock_opts_default,
 * nblock 1. */
void agf2_run_opts_default(agf2_run_opts* opts);

/* One record per iteration of agf2_run. */
typedef struct {
  int iter;                      /* 0 = built from the mean-field poles    */
  int nocc_pole, npole, fock_cycles, warm;
  int fock_converged;            /* 1 if this iteration's Fock loop converged */
  double e_1b, e_2b, e_tot;      /* Ha                                     */
  double ip, ea, w_ip, w_ea;     /* IP = -(highest occupied pole), EA,
                                    and their quasiparticle weights        */
  double mu, shift;              /* chemical potential, auxiliary shift    */
  double t_moments, t_compress, t_fock, t_energy;   /* seconds            */
} agf2_iter_record;

/*
 * AGF2(1,0) to self-consistency (the method as reviewed in the paper):
 * iteration 0 builds the moments from the mean-field poles (energies e_mf,
 * amplitudes = identity, the first nocc occupied); every iteration then
 * extrapolates the moments (DIIS, damping), compresses the lesser and greater
 * parts to nphys auxiliaries each, relaxes the density in the Fock loop
 * (starting from the previous density; 2 * diag(1_occ) at first), evaluates
 * the Galitskii-Migdal energy and IP/EA, and builds the next moments from the
 * nphys + 2 nphys poles. Converged when |dE| < conv_tol and max(|dIP|,
 * |dEA|) < conv_tol_ipea. An iteration whose Fock loop reaches its cycle
 * limit ends the run: its record has fock_converged = 0, the outputs hold
 * its Green's function and density, and the call returns
 * AGF2_ERR_NO_CONVERGE.
 *   Lpq device [naux][nphys][nphys]; hcore device [nphys][nphys];
 *   e_mf device [nphys]; nocc doubly occupied orbitals (nelec = 2 nocc).
 *   dm_init    device [4][nphys][nphys] or NULL: a correction added to the
 *              iteration-0 moments (warm start); if the corrected moments
 *              cannot be compressed, iteration 0 is redone without it
 *              (record.warm says which was used).
 *   records    host [max_iter + 1] outputs; n_records, converged host.
 *   e_pole [npmax], u_pole [nphys][npmax], rdm1 [nphys][nphys] device
 *   outputs (the final Green's function and density; npmax = nphys +
 *   2 nblock nphys, the record's npole entries valid); nocc_pole host.
 * Returns AGF2_ERR_NO_CONVERGE when max_iter is reached (outputs valid).
 */
agf2_status agf2_run(agf2_handle_t handle, const agf2_run_opts* opts,
                     int nphys, int naux, const double* Lpq,
                     const double* hcore, const double* e_mf, int nocc,
                     const double* dm_init, agf2_iter_record* records,
                     int* n_records, int* converged, double* e_pole,
                     double* u_pole, int* nocc_pole, double* rdm1);

/*
 * Checkpoint and resume of agf2_run. The state between two iterations (the
 * index of the next iteration, the current Green's function poles, the
 * density, the previous moments kept for damping, the moment DIIS history
 * and the last energy, IP and EA of the convergence test) is written to a
 * host buffer of agf2_run_state_bytes(nphys, opts) bytes (NULL opts: the
 * defaults; -1 for bad arguments). A run continued from a saved state with the same inputs
 * and options takes exactly the iterations an uninterrupted agf2_run would
 * have taken, with bitwise equal results.
 *
 * agf2_run_resume takes the arguments of agf2_run and:
 *   state_in       host, NULL: start at iteration 0 (dm_init applies); else
 *                  continue from this saved state (dm_init is ignored).
 *                  AGF2_ERR_ARG if it was saved for another nphys,
 *                  diis_space or nblock or is not a state at all.
 *   state_out      host, NULL or a buffer of agf2_run_state_bytes: the state
 *                  after the last iteration of this call (written on return
 *                  unless an error other than AGF2_ERR_NO_CONVERGE occurs).
 *   max_iter_call  > 0: stop after this many iterations in this call (the
 *                  call then returns AGF2_OK with *converged = 0 unless the
 *                  run converged or failed); <= 0: no limit but max_iter.
 * records receives this call's iterations only (their iter fields continue
 * the count); it must hold max_iter + 1 records. max_iter counts iterations
 * from iteration 0 of the whole run.
 */
long agf2_run_state_bytes(int nphys, const agf2_run_opts* opts);
agf2_status agf2_run_resume(agf2_handle_t handle, const agf2_run_opts* opts,
                            int nphys, int naux, const double* Lpq,
                            const double* hcore, const double* e_mf, int nocc,
                            const double* dm_init, const void* state_in,
                            void* state_out, int max_iter_call,
                            agf2_iter_record* records, int* n_records,
                            int* converged, double* e_pole, double* u_pole,
                            int* nocc_pole, double* rdm1);

/*
 * Kernel timing (tracing aid, not part of the method). When enabled, the
 * library records hipEvents on its stream around every launch of each
 * kernel class (e.g. "moments.slab", "moments.syrk", "fock.syevd") together
 * with the launch's algorithmic flop and HBM byte counts.
 * agf2_profile_enable(h, 1) clears the totals and starts recording;
 * agf2_profile_enable(h, 0) stops. agf2_profile_count() synchronises the
 * stream, folds pending events into the totals and returns the number of
 * classes (or a negative status); agf2_profile_get() reads class `idx`
 * (name valid until the next profile call): launches, total milliseconds,
 * total algorithmic flops and bytes.
 */
agf2_status agf2_profile_enable(agf2_handle_t handle, int enable);
int agf2_profile_count(agf2_handle_t handle);
agf2_status agf2_profile_get(agf2_handle_t handle, int idx, const char** name,
                             long* launches, double* ms, double* flops,
                             double* bytes);

/* ------------------------------------------------------------------------
 * Learned warm start (not part of the paper's method: a predictor that moves
 * the iteration-0 moments towards the converged ones so that the
 * self-consistent loop of agf2_run starts closer to its fixed point; the
 * fixed point itself is unchanged, and agf2_run falls back to the cold start
 * when the corrected moments cannot be compressed).
 *
 * A per-orbital network of three linear maps (12 -> 256 -> 256 -> 20) with
 * GELU (z Phi(z), Phi the normal distribution function) after the first
 * two. The products run on FP16 MFMA with FP32 accumulation: features,
 * hidden activations and weights are rounded to IEEE half precision as
 * operands; pre-activations, biases and outputs are float32. Training
 * (backward pass, Adam) runs in float32 on FP32 master parameters.
 *
 * Features of physical orbital x (float32 [N][12]), from the mean-field
 * energies e and the iteration-0 moments U_n (n = 0<, 1<, 0>, 1>):
 *   e_x, e_x - mu0 (mu0 = (e_HOMO + e_LUMO)/2), gap = e_LUMO - e_HOMO,
 *   +1 occupied / -1 virtual, U_n[x][x] / s_n (4), log(s_1/s_0),
 *   log(s_2/s_0), log(s_3/s_2), (e_x - mu0) / gap,
 * with s_n the mean |diagonal| of U_n (at least 1e-30); no absolute moment
 * scale enters, so the features do not drift with the system size.
 * Outputs (float32 [N][20]): for moment n, y[5n] = r_n(x) and
 * y[5n+1+m] = c_nm(x), m = 0..3; the correction is a diagonal term plus a
 * symmetric per-orbital rescaling of the four iteration-0 moments,
 *   Delta U_n[x][y] = s_n (delta_xy r_n(x)
 *                          + sum_m (c_nm(x) + c_nm(y)) U_m[x][y] / s_m).
 * Loss of one system, T_n = (U_n(converged) - U_n(iteration 0)) / s_n and
 * P_n = Delta U_n / s_n:  sum_n || P_n - T_n ||_F^2 / N.
 *
 * Parameters: float32, flat, in the order W1 [12][256], b1 [256],
 * W2 [256][256], b2 [256], W3 [256][20], b3 [20] (weights [in][out]).
 * ---------------------------------------------------------------------- */
#define AGF2_MLP_FEATURES 12
#define AGF2_MLP_HIDDEN 256
#define AGF2_MLP_OUTPUTS 20
#define AGF2_MLP_NPARAM 74260

typedef struct agf2_mlp_s* agf2_mlp_t;

/* Create a network on the handle's device (parameters zero, Adam state
 * empty) / free it. A network is used with handles of its device only. */
agf2_status agf2_mlp_create(agf2_handle_t handle, agf2_mlp_t* net);
agf2_status agf2_mlp_destroy(agf2_mlp_t net);

/* Copy parameters in from / out to host float32 [AGF2_MLP_NPARAM]. Setting
 * parameters resets the Adam state. agf2_mlp_get_grad copies out the
 * gradient left by the last agf2_mlp_backward. */
agf2_status agf2_mlp_set_params(agf2_handle_t handle, agf2_mlp_t net, const float* params);
agf2_status agf2_mlp_get_params(agf2_handle_t handle, agf2_mlp_t net, float* params);
agf2_status agf2_mlp_get_grad(agf2_handle_t handle, agf2_mlp_t net, float* grad);

/* Features of one system. e_mf device [nphys]; m0 device [4][nphys][nphys]
 * (U0<, U1<, U0>, U1> at iteration 0); X device float32 [nphys][12] and
 * scale device float64 [4] (s_n) outputs. Needs 1 <= nocc < nphys. */
agf2_status agf2_mlp_features(agf2_handle_t handle, int nphys, int nocc, const double* e_mf,
                              const double* m0, float* X, double* scale);

/* Y = network(X) for `rows` orbitals (any number of systems stacked).
 * X device float32 [rows][12]; Y device float32 [rows][20]. The network
 * keeps this call's activations for the next agf2_mlp_backward. */
agf2_status agf2_mlp_forward(agf2_handle_t handle, agf2_mlp_t net, int rows, const float* X,
                             float* Y);

/* Loss of one system and its gradient with respect to that system's
 * outputs. Y device float32 [nphys][20]; m0, mconv device [4][nphys][nphys]
 * (iteration-0 and converged moments); scale device [4] from
 * agf2_mlp_features; dY device float32 [nphys][20] output; loss device
 * float64 scalar, incremented by this system's loss. */
agf2_status agf2_mlp_loss_grad(agf2_handle_t handle, int nphys, const float* Y,
                               const double* m0, const double* mconv, const double* scale,
                               float* dY, double* loss);

/* Gradient of sum(Y * dY) with respect to the parameters, through the
 * activations of the last agf2_mlp_forward (same rows); overwrites the
 * network's gradient. dY device float32 [rows][20]. */
agf2_status agf2_mlp_backward(agf2_handle_t handle, agf2_mlp_t net, int rows, const float* dY);

/* One Adam step (Kingma and Ba; bias-corrected moments, step count kept by
 * the network) on the FP32 master parameters with the current gradient;
 * refreshes the FP16 copies used by the forward pass. */
agf2_status agf2_mlp_adam_step(agf2_handle_t handle, agf2_mlp_t net, float lr, float beta1,
                               float beta2, float eps);

/* Warm-start correction of one system: features, forward pass and
 * Delta U_n as above. e_mf device [nphys]; m0 device [4][nphys][nphys]
 * (iteration-0 moments); dm device [4][nphys][nphys] output, suitable as
 * agf2_run's dm_init. */
agf2_status agf2_mlp_predict_correction(agf2_handle_t handle, agf2_mlp_t net, int nphys,
                                        int nocc, const double* e_mf, const double* m0,
                                        double* dm);

#ifdef __cplusplus
}
#endif

#endif /* AGF2_H */

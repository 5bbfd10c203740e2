/*
 * scocg — shifted-COCG Green's-function solver for MI355X (gfx950), C ABI.
 *
 * The library solves, for a sparse real-symmetric Hamiltonian H (n x n),
 *     (z_k 1 - H) x_{k,j} = b_j      for shifts k < n_shift, right-hand sides j < n_rhs
 * (paper Sec. 3.1 eq. lin_eq, Sec. 3.3 eq. shift_lin_eq).  One seed shift per
 * right-hand side is iterated with COCG, the method for complex-symmetric
 * systems (Sec. 3.3); every other shift follows from the seed's scalars because
 * the Krylov subspace is invariant under a scalar shift (Sec. 3.1 eq. inv_KS) and
 * the shifted residuals stay collinear with the seed's (Sec. 3.3).  When the seed
 * has converged the iteration continues from another shift, keeping the
 * information computed so far (seed switching, Sec. 3.3).  Each (shift, rhs) pair
 * stops when its residual norm ||b - (z - H) x|| / ||b|| is below the tolerance
 * (Sec. 3.4 eq. residual).
 *
 * Conventions (every entry point):
 *  - Complex numbers are interleaved (re, im) doubles, the memory layout of
 *    complex128 / hipDoubleComplex.
 *  - "device" pointers are HIP device memory owned by the caller; the library
 *    never frees them and they must stay valid until the call returns.  "host"
 *    pointers are ordinary CPU memory.  A device argument that is plain host memory
 *    (not device, pinned or managed) is refused with SCOCG_EINVAL before any work.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Solver calls enqueue work on that stream and return after it has finished
 *    (the iteration is steered from the host between blocks of iterations).
 *  - Every call returns a status: SCOCG_OK, or one of the codes below; the
 *    message of the last failure on the calling thread is scocg_last_error().
 *    No C++ exception crosses the ABI.
 *  - All computation runs on the GPU.  There is no CPU fallback.
 */
#ifndef SCOCG_H
#define SCOCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SCOCG_OK = 0,
    SCOCG_EINVAL = 1,     /* invalid argument or matrix */
    SCOCG_ENOMEM = 2,     /* device allocation failed */
    SCOCG_EHIP = 3,       /* HIP runtime error */
    SCOCG_EBREAKDOWN = 4, /* COCG breakdown: r.r = 0, p.(Ap) = 0 or pi = 0 on an unconverged pair */
    SCOCG_ENOCONV = 5     /* some pair did not reach the tolerance; results are still written */
};

typedef struct scocg_csr *scocg_csr_t;   /* uploaded Hamiltonian (library-owned) */
typedef struct scocg_tape *scocg_tape_t; /* solutions kept for backward() (library-owned) */

typedef struct {
    double tol;             /* per-pair stop: ||r_k|| / ||b|| < tol (recursive residual) */
    int32_t max_iter;       /* iteration limit per right-hand side */
    int32_t precision;      /* 0: x_k, p_k stored in FP64; 1: stored and updated in FP32 */
    int32_t seed_index;     /* initial seed shift; -1: smallest Im z, then Re z nearest Tr(H)/n, then lowest index */
    int32_t seed_switching; /* 1: switch seed when it converges (Sec. 3.3) */
    int32_t fixed_iter;     /* > 0: run exactly this many iterations, no freezing, no switching */
    int32_t block;          /* iterations per deferred shift update (1,2,4,8,16,24,32,40,48); 0 = automatic (48) */
    int32_t shifts_per_wg;  /* shifts one workgroup updates in the deferred update (1 .. 64); 0 = automatic
                               (up to 64 for blocks of 24 and more, up to 32 for shorter ones) */
    int32_t check_true;     /* 1: compute the FP64 true residual of every pair into the report */
    int32_t keep_tape;      /* 1: keep the solutions for backward() */
    int32_t no_graph;       /* 1: launch every kernel directly instead of replaying captured HIP graphs */
    int32_t refine;         /* sweeps of FP64 refinement for pairs whose true residual exceeds tol: each solves
                               (z_k - H) d = b - (z_k - H) x per pair (COCG, FP64 vectors) and adds d to x.
                               Needs full solutions (shifted_cocg_solve); implies check_true. */
    int32_t window;         /* projection mode only (greens_diag, greens_diag_batched): > 0 keeps the full
                               direction vector of this many shifts per right-hand side (the seed first, then
                               the others in the seed-rule order: smallest Im z, Re z nearest Tr(H)/n, lowest
                               index); every other shift is carried by scalars at the kept row.  A seed switch
                               then goes to the active stored shift with the largest residual; when none is left
                               the pairs still active stop unconverged (SCOCG_ENOCONV).  0: every shift keeps
                               its full direction. */
    int32_t schedule;       /* deferred shift update: 1 in order with the seed iterations on the caller's stream;
                               2 overlapped with the next block's iterations on a second stream; 0 automatic
                               (overlapped when the stored directions hold at least 2^24 complex numbers, where
                               the update outweighs the cost of the cross-stream waits).  Same bits either way. */
    int32_t update_form;    /* deferred update of x_k, u_k: 1 the step form (two complex multiply-adds per step,
                               the same bits for every block length); 2 the expanded form, in which a block
                               becomes x += gamma u + sum_s c_s r_s and u = delta u + sum_s d_s r_s with the
                               per-pair weights c_s, d_s (a contraction with the residual history on FP64 matrix
                               cores; FP64 storage, full solutions, blocks of 24 or more, EINVAL otherwise);
                               0 automatic (the step form, the faster one on gfx950).  Both forms agree to
                               rounding. */
    int32_t reserved;
} scocg_opts;

typedef struct {
    int32_t iters;            /* iterations after which the pair was frozen (or the total) */
    int32_t status;           /* SCOCG_OK (converged), SCOCG_ENOCONV or SCOCG_EBREAKDOWN */
    double rel_res_recursive; /* ||r_seed|| / (|pi_k| ||b||) at exit */
    double rel_res_true;      /* ||b - (z_k - H) x|| / ||b|| in FP64 (if check_true, else -1) */
} scocg_pair_report;

/* Fills *o with the defaults: tol 1e-8, max_iter 3000, FP64, default seed, switching on. */
void scocg_default_opts(scocg_opts *o);

/*
 * Check a CSR matrix on the host: square, row_ptr monotone with row_ptr[0] = 0
 * and row_ptr[n] = nnz, columns in range, sorted and unique in each row, values
 * finite, and H exactly symmetric (H_ij == H_ji bitwise, the real-symmetric
 * Hamiltonian of Sec. 2.1 / 2.2).  Host pointers.  Returns SCOCG_OK or SCOCG_EINVAL.
 */
int scocg_csr_validate(int64_t n, int64_t nnz, const int64_t *row_ptr, const int64_t *col, const double *val);

/*
 * Upload H (host CSR arrays, int64 indices, FP64 values) to the current device.
 * The library keeps its own device copy in a sliced-ELL layout (64-row slices,
 * 32-bit columns) plus the CSR pattern; n and nnz must be below 2^31.
 * validate = 1 runs scocg_csr_validate first.  On success *out owns the copy.
 */
int csr_upload(int64_t n, int64_t nnz, const int64_t *row_ptr, const int64_t *col, const double *val, int validate,
               void *stream, scocg_csr_t *out);

/* Replace the values of H (same pattern, host array of nnz doubles, CSR order). */
int csr_update_values(scocg_csr_t H, const double *val, void *stream);

/* Dimension and stored-entry count of an uploaded matrix. */
/*
 * Matrix-free extended Hubbard ring (the model class of Sec. 4.2: a many-electron
 * Hamiltonian in the occupation-number basis of one (N_up, N_dn) sector):
 *     H = -t sum_{i,s} (c+_{i,s} c_{i+1,s} + h.c.) + U sum_i n_{i,up} n_{i,dn} + V sum_i n_i n_{i+1}
 * on L sites with periodic boundary.  Basis: each species is an L-bit occupation pattern
 * with N_s bits set, in increasing order; row = i_up * D_dn + i_dn.  Fermion signs follow
 * the Jordan-Wigner order with all up-spin modes before all down-spin modes (the
 * ring-closing hop carries (-1)^(N_s - 1)).  The operator applies H = T_up (x) 1 + 1 (x) T_dn
 * + D from two hopping tables of D_up and D_dn configurations instead of storing the
 * matrix; its products equal those of the stored matrix of the same sector bit for bit.
 *   3 <= L <= 30, 0 <= n_up, n_dn <= L, D_up * D_dn < 2^31; t, U, V finite.
 * The handle works with shifted_cocg_solve, greens_diag and greens_diag_batched;
 * csr_update_values, density_matrix_energy and backward need a stored matrix (EINVAL).
 * csr_nnz reports the entries the stored matrix would have.  Free with csr_free.
 */
int hubbard_upload(int32_t L, int32_t n_up, int32_t n_dn, double t, double U, double V, void *stream,
                   scocg_csr_t *out);

int64_t csr_n(scocg_csr_t H);
int64_t csr_nnz(scocg_csr_t H);
/* Release the caller's handle.  Tapes recorded on H keep their own reference (backward() reads
 * H's pattern), so the matrix lives until its last tape is freed too; H must not be used by the
 * caller afterwards. */
void csr_free(scocg_csr_t H);

/*
 * Solve (z_k 1 - H) X[j][k] = B[j] for all pairs (Sec. 3.3 eq. shift_lin_eq).
 *   z    host, n_shift complex: the shifts (Im z may have either sign, not 0 on the spectrum)
 *   B    device, [n_rhs][n] complex: right-hand sides
 *   X    device, [n_rhs][n_shift][n] complex FP64 output (may be NULL only with keep_tape)
 *   rep  host, [n_rhs][n_shift] reports, or NULL
 *   tape if non-NULL and o->keep_tape, receives the solutions for backward()
 * Returns SCOCG_OK, SCOCG_ENOCONV (results written, see rep), SCOCG_EBREAKDOWN,
 * SCOCG_EINVAL, SCOCG_ENOMEM or SCOCG_EHIP.
 */
int shifted_cocg_solve(scocg_csr_t H, int64_t n_shift, const double *z, int64_t n_rhs, const double *B,
                       const scocg_opts *o, double *X, scocg_pair_report *rep, scocg_tape_t *tape, void *stream);

/*
 * Diagonal Green's function G_jj(z_k) = [(z_k - H)^{-1}]_jj (Sec. 2.1.1 eq. gf)
 * for the unit right-hand sides e_j, j = rhs_idx[c].
 *   rhs_idx host, n_rhs indices in [0, n)
 *   G       device, [n_shift][n_rhs] complex output
 * Only the diagonal entries of the solutions are kept, unless o->keep_tape asks for
 * the full solutions.  The directions p_k are kept full length for seed switching,
 * for every shift or (o->window > 0) for a window of seed candidates; the other
 * shifts then cost scalar work only (Sec. 3.3: a shifted system needs only scalar
 * recurrences when one component of its solution is wanted).
 */
int greens_diag(scocg_csr_t H, int64_t n_shift, const double *z, int64_t n_rhs, const int64_t *rhs_idx,
                const scocg_opts *o, double *G, scocg_pair_report *rep, scocg_tape_t *tape, void *stream);

/*
 * greens_diag for callers that cannot allocate device memory: tight serving loops, harnesses
 * that forbid hipMalloc, programs that keep their device allocations fixed around HIP graph
 * capture (the call itself waits on the stream, so it is made outside a capture).  Same arguments, kernels and
 * results (bit for bit) as greens_diag without a tape; every work buffer of the solve lives in
 * one device array of SCOCG_NOALLOC_MAX_BYTES that the library holds on each device it runs on
 * until the process ends.  The call allocates no device or pinned memory and creates no
 * streams, events or graphs (it runs the serial schedule with direct launches on `stream`, and
 * its host bookkeeping is a few scalars); inputs and outputs are the caller's as in greens_diag.
 *   Needs: o->keep_tape = 0, o->refine = 0, o->check_true = 0, o->window = 0 (EINVAL otherwise).
 *   Scratch: about 16 n n_rhs (2 block + 4) + n_shift n_rhs (esz n + 4 esz block + 124) bytes, esz =
 *   16 (FP64) or 8 (FP32) and block the iterations per deferred update (48 by default); a call
 *   needing more than SCOCG_NOALLOC_MAX_BYTES returns SCOCG_EINVAL with the size it needs in
 *   scocg_last_error(), before any work.
 *   The array keeps the last call's contents; each call initialises what it reads.  Calls on one
 *   device share its array, so they are serialised by a lock in the library: a second call on the
 *   same device (another host thread) waits until the first has finished, its GPU work included
 *   (also when the first returns an error).
 * Synchronous on stream.  Errors as greens_diag.
 */
#define SCOCG_NOALLOC_MAX_BYTES (128ull << 20)
int greens_diag_noalloc(scocg_csr_t H, int64_t n_shift, const double *z, int64_t n_rhs, const int64_t *rhs_idx,
                        const scocg_opts *o, double *G, scocg_pair_report *rep, void *stream);

/*
 * Krylov-subspace diagonalization (Sec. 3.2, eq. Ham_in_KS) of the local Green's function,
 * the paper's first method and the one it compares shifted COCG against: for each unit
 * vector |j>, j = rhs_idx[c], nu steps of the three-term (Lanczos) recurrence build an
 * orthonormal basis {K_n} of the Krylov subspace K_nu(H, |j>), in which H is the
 * tridiagonal reduced Hamiltonian T (diagonal a_n = <K_n|H|K_n>, off-diagonal
 * b_{n+1} = <K_{n+1}|H|K_n>); then G_jj(z_k) = [(z_k - T)^{-1}]_11, the Green's function of
 * the subspace (exact when the subspace is invariant, an approximation otherwise, whose
 * accuracy the paper notes is limited by the loss of orthogonality of the basis).
 *   z       host, n_shift complex (interleaved)
 *   rhs_idx host, n_rhs indices in [0, n)
 *   nu      steps, 1 <= nu <= 2^20 (more than n is allowed: in finite precision the basis loses
 *           orthogonality and the recurrence keeps refining, as the shifted COCG iteration
 *           does past n steps)
 *   G       device, [n_shift][n_rhs] complex output
 *   ab      device or NULL, [n_rhs][2][nu] doubles: a_1..a_m, then b_2..b_{m+1}
 *           (b_{m+1} is the norm the subspace leaves out); entries past m are left as they are
 *   dim     host or NULL, [n_rhs]: m, the subspace dimension reached: nu, or fewer when the
 *           subspace is invariant (the recurrence stops once b_{m+1} <= 1e-12 (|a_m| + b_m))
 * H is a stored matrix or a matrix-free Hubbard operator (whose rows give the same sums,
 * so the same coefficients bit for bit).  Errors: EINVAL (null or bad arguments, index out of
 * range, nu outside [1, 2^20]), ENOMEM, EHIP.  Synchronous on stream
 * when dim is requested; the timing record (scocg_last_timing) gets the wall time and
 * iterations = steps summed over the right-hand sides.
 */
int krylov_greens_diag(scocg_csr_t H, int64_t n_shift, const double *z, int64_t n_rhs, const int64_t *rhs_idx,
                       int32_t nu, double *G, double *ab, int32_t *dim, void *stream);

/*
 * <b|(z_k - H)^{-1}|b> for one real start vector b by Krylov-subspace diagonalization
 * (Sec. 3.2, eq. Ham_in_KS): nu steps of the three-term recurrence from b/|b| (ending early at
 * an invariant subspace), then |b|^2 times [(z_k - T)^{-1}]_11 of the reduced Hamiltonian T as a
 * continued fraction; the spectral function of b (for b = c|psi0>, a many-electron excitation
 * spectrum, Sec. 4.2) without one linear solve per shift.
 *   b     device, [n] real, nonzero
 *   G     device, [n_shift] complex output
 *   ab    device, [2][nu] (the a and b coefficients as in krylov_greens_diag), or NULL
 *   dim   host, the subspace dimension reached, or NULL
 * H is a stored matrix or a matrix-free Hubbard operator.  Errors: EINVAL (null or bad
 * arguments, a zero start vector, nu outside [1, 2^20]), ENOMEM, EHIP.  Synchronous.
 */
int krylov_greens_vec(scocg_csr_t H, int64_t n_shift, const double *z, const double *b, int32_t nu, double *G,
                      double *ab, int32_t *dim, void *stream);

/*
 * Ground state of a many-electron Hamiltonian (Sec. 2.2: the Lanczos method for an estimate,
 * then the CG method as inverse iteration, repeated until the residual norm is small).
 * nu steps of the three-term recurrence from x0 give the reduced Hamiltonian, whose lowest
 * two eigenvalues E_L0 <= E_L1 are found by bisection; a second run of the same recurrence
 * accumulates the Ritz vector of E_L0, with Rayleigh quotient theta and residual norm r.
 * Each inverse-iteration sweep then solves (sigma - H) y = psi for the fixed shift
 * sigma = min(E_L0 - max(0.1 (E_L1 - E_L0), 1e-6 max(1, |E_L0|)), theta - r) (below the ground
 * state when the Ritz vector leans on it, where COCG is CG; relative residual
 * min(1e-10, tol / 100)) and sets
 * psi = y / ||y|| (sign kept), until ||H psi - E psi|| <= tol with E = psi . H psi, or
 * max_sweeps sweeps.
 *   x0      device, [n] real start vector (any norm, not orthogonal to the ground state)
 *   psi     device, [n] complex output (imaginary parts zero), unit norm
 *   E       host, 2 doubles: E = psi . H psi, and the estimate E_L1 of the next eigenvalue
 *   res     host or NULL: the final ||H psi - E psi||
 *   sweeps  host or NULL: inverse-iteration sweeps done
 * H is a stored matrix or a matrix-free Hubbard operator (the same results bit for bit).
 * Errors: EINVAL (null or bad arguments, nu outside [2, 2^20]), ENOMEM, EHIP, those of the
 * linear solves, and ENOCONV when the residual norm is still above tol after max_sweeps
 * sweeps (psi, E, res and sweeps are written).  Synchronous.
 */
int ground_state(scocg_csr_t H, const double *x0, int32_t nu, double tol, int32_t max_sweeps, double *psi, double *E,
                 double *res, int32_t *sweeps, void *stream);

/*
 * Fermion operator between S_z sectors of the Hubbard ring (the single-particle excitations
 * whose spectra Sec. 4.2 computes): y = c_{site,spin} x (create = 0) or c+_{site,spin} x
 * (create = 1) for x in the sector (L, n_up, n_dn) of hubbard_upload's basis (patterns in
 * increasing order, index i_up * D_dn + i_dn) and y in the sector with one electron of that
 * spin less or more.  Jordan-Wigner order: all up-spin modes (sites ascending), then all
 * down-spin modes, so the sign is (-1)^(number of occupied modes before (site, spin)).
 *   x  device, complex, the source sector
 *   y  device, complex, the target sector (overwritten)
 * Errors: EINVAL (null pointers, L outside [3, 30], counts, site or spin out of range, a
 * target sector that does not exist), ENOMEM, EHIP.  Synchronous.
 */
int hubbard_fermion_op(int32_t L, int32_t n_up, int32_t n_dn, int32_t site, int32_t spin, int32_t create,
                       const double *x, double *y, void *stream);

/*
 * Projected Green's functions G[k][j] = <w_j|(z_k - H)^{-1}|b_j> = sum_i w_j[i] x_{j,k}[i]
 * (bilinear; for real w_j it is the matrix element the spectra of Sec. 4.2 need) for dense
 * right-hand sides b_j and projection vectors w_j, in the regime Sec. 3.3 describes: when only
 * a projection of each solution is wanted, every shifted system is carried by scalars.  One
 * reduction per seed iteration gives s_n = w_j . r_n, and each pair's <w|x_k>, <w|u_k> follow
 * the deferred update's steps with s_n in place of the residual; full directions u_k are kept
 * only for o->window seed candidates (all shifts when window = 0), which a seed switch needs.
 * As in greens_diag's window mode, a seed switch goes to the active stored shift with the
 * largest residual, and when none is left the pairs still active stop unconverged.
 *   H       stored matrix or matrix-free operator
 *   B, W    device, [n_rhs][n] complex each (W = B for <b|G|b>)
 *   G       device, [n_shift][n_rhs] complex output
 *   rep     host, [n_rhs][n_shift] reports, or NULL (rel_res_true is -1: no solutions are kept)
 * Device memory: n_shift * n_rhs scalars plus window (or n_shift) direction vectors of n
 * complex numbers per right-hand side.  Errors: EINVAL (null or bad arguments), ENOMEM,
 * EHIP, EBREAKDOWN, ENOCONV (results still written).
 */
int greens_proj(scocg_csr_t H, int64_t n_shift, const double *z, int64_t n_rhs, const double *B, const double *W,
                const scocg_opts *o, double *G, scocg_pair_report *rep, void *stream);

/*
 * G_jj(z_k) for several Hamiltonians of different sizes in one solve (a batch of
 * independent problems sharing the shift list).  Problem q has n_rhs[q] unit
 * right-hand sides; rhs_idx lists them problem after problem (indices local to the
 * problem's rows).  Every right-hand side iterates its own seed on its own matrix
 * and retires on its own; all of them advance in the same kernel launches.
 *   H       host array of n_problems uploaded matrices
 *   G       device, [n_shift][sum n_rhs] complex output (columns in rhs_idx order)
 *   rep     host, [sum n_rhs][n_shift] reports, or NULL
 * Device memory: the directions of every (rhs, shift) pair are stored in full,
 * n_shift * sum_q n_rhs[q] * n_q complex numbers (8 or 16 bytes each), or with
 * o->window > 0 only window * sum_q n_rhs[q] * n_q; callers split larger batches
 * into waves that fit.
 */
int greens_diag_batched(int64_t n_problems, const scocg_csr_t *H, const int64_t *n_rhs, const int64_t *rhs_idx,
                        int64_t n_shift, const double *z, const scocg_opts *o, double *G, scocg_pair_report *rep,
                        void *stream);

/*
 * Density matrix and band energy at zero temperature from a contour integral of
 * G (Sec. 2.1.1 eq. densityM, with <X> = Tr[rho X] and X = H):
 *     rho_ab = Re sum_q w_q G_ab(z_q),     E = Re sum_q w_q z_q sum_j G_jj(z_q)
 * for the columns j in rhs_idx (all n columns give the full rho on H's pattern
 * and the full band energy).  z, w: host, n_quad complex nodes and weights (see
 * scocg_contour).  rhs_idx: host, n_rhs distinct columns in [0, n) (a repeated column is
 * EINVAL: it would be counted twice).  Outputs (device, accumulated into, so zero them first):
 *   rho_nnz [nnz] or NULL: rho on the stored entries of H, CSR order; column j adds its
 *                          entries (a, j) (all columns give every entry of rho)
 *   E_band  [1]          : band energy contribution of the columns
 *   dE_dval [nnz] or NULL: derivative of E with respect to each stored entry,
 *                          Re sum_q w_q z_q sum_j x_qj[a] x_qj[b] (any row length; the sums over
 *                          pairs are taken in a fixed order)
 * Right-hand sides are processed in batches of at most rhs_batch (0 = automatic: 256), each
 * holding its full solutions (rhs_batch * n_quad * n complex numbers) while its products are
 * formed.
 */
int density_matrix_energy(scocg_csr_t H, int64_t n_quad, const double *z, const double *w, int64_t n_rhs,
                          const int64_t *rhs_idx, const scocg_opts *o, int64_t rhs_batch, double *rho_nnz,
                          double *E_band, double *dE_dval, void *stream);

/*
 * Gradient of a real loss L through G = greens_diag(...) or X = shifted_cocg_solve(...)
 * with respect to the stored entries of H.  Because z - H is complex symmetric,
 * dG_jj/dH_ab = x_j[a] x_j[b] and no second solve is needed:
 *     dL/dH_ab = Re sum_{k,j} conj(g_kj) x_kj[a] x_kj[b]
 * with g = dL/dRe G + i dL/dIm G (PyTorch's convention for complex tensors).
 *   grad_G   device, [n_shift][n_rhs] complex (greens_diag tape only)
 *   grad_val device, [nnz] FP64, accumulated into (per stored CSR entry)
 */
int backward(scocg_tape_t tape, const double *grad_G, double *grad_val, void *stream);
/* Release a tape (its solutions and its reference to the matrix it was recorded on). */
void tape_free(scocg_tape_t t);

/*
 * Nodes and weights of the zero-temperature contour: the upper half of the circle
 * through e_lo and mu, Gauss-Legendre in the angle, folded with the mirror
 * symmetry G(conj z) = conj G(z) so that rho = Re sum_q w_q G(z_q).  Host
 * arrays of 2*n_quad doubles.
 */
int scocg_contour(double e_lo, double mu, int64_t n_quad, double *z, double *w);

/* Message of the last failure on this thread ("" if none). */
const char *scocg_last_error(void);

/*
 * Timing of the most recent solve on this thread, from HIP events on its stream:
 * the summed duration and launch count of the deferred shift-update kernel and
 * of the seed kernels, and the algorithmic bytes and flops of the shift update.
 */
typedef struct {
    double update_ms;       /* total time in the deferred per-shift update kernel */
    int64_t update_launches;
    double update_bytes;    /* algorithmic bytes of those launches */
    double total_ms;        /* wall time of the solve on the stream */
    int64_t iterations;     /* seed iterations summed over right-hand sides */
    int64_t blocks;         /* blocks of iterations */
    int64_t switches;       /* seed switches */
    double update_flops;    /* algorithmic flops of the update launches: per pair and step it takes, two complex
                               multiply-adds (16 flops) per row, one (8) where only the direction is stored */
} scocg_timing;
int scocg_last_timing(scocg_timing *t);
/* 1: record per-launch events around the update kernel (adds a small overhead). */
void scocg_set_profiling(int on);

/*
 * Seed switches (Sec. 3.3) of right-hand side `rhs` in the most recent solve on this thread
 * (shifted_cocg_solve, greens_diag, greens_diag_batched, greens_proj; for
 * density_matrix_energy its last batch of right-hand sides).  Each entry is a pair
 * (iterations completed when the old seed converged, index of the new seed shift), in the
 * order they happened.  log: host array of 2 * max_entries int32, or NULL to only count.
 * Returns the number of switches (entries beyond max_entries are not written), or -1 when
 * rhs is outside the last solve's right-hand sides (message in scocg_last_error).
 */
int32_t scocg_last_switches(int64_t rhs, int32_t *log, int32_t max_entries);

#ifdef __cplusplus
}
#endif
#endif

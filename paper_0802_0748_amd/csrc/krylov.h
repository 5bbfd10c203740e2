// Krylov-subspace diagonalization on the device (not part of the C ABI): the three-term
// recurrence of many unit right-hand sides' Krylov bases and the local Green's function of
// their reduced Hamiltonians (Sec. 3.2, eq. Ham_in_KS).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace scocg {

struct HubbardOp;

// Right-hand sides per thread of the recurrence: vectors are stored as [K / LZ_RB][n][LZ_RB]
// (the LZ_RB right-hand sides of a group interleaved row by row), so one column and value
// load of the stored matrix serves LZ_RB right-hand sides and their gathers are 32 B.
constexpr int LZ_RB = 4;
// rows per workgroup of the recurrence, one partial sum each
constexpr int LZ_TILE = 256;
// an invariant subspace ends the recurrence: b_{m+1} <= LZ_STOP_REL (|a_m| + b_m)
constexpr double LZ_STOP_REL = 1e-12;

struct LzRhs {
    double bprev;  // b_n of the step in progress (0 before the first)
    double a;      // a_n of the step in progress
    int64_t j;     // row of the unit start vector
    int32_t m;     // steps completed (dimension of the subspace so far)
    int32_t done;  // recurrence finished (nu steps, or an invariant subspace)
};

struct LzDev {
    const HubbardOp *hub;      // matrix-free operator (device), or null for the stored matrix
    const int64_t *slice_ptr;  // stored matrix, 64-row slices (see DevCSR)
    const int32_t *slice_w;
    const int32_t *ell_col;
    const double *ell_val;
    int64_t n;
    int64_t K;     // right-hand sides (padded to groups of rb with finished entries)
    int64_t nblk;  // 256-row tiles, one partial sum each
    int32_t nu;
    int32_t rb;    // right-hand sides interleaved per group: LZ_RB, or 1 (plain vectors)
    double *V[2];  // basis vectors K_n by parity of n: [K / rb][n][rb]
    double *W[2];  // unnormalized next vectors by parity
    double *part;  // [K][nblk] partial sums
    double *ab;    // [K][2][nu]: a_1..a_m, then b_2..b_{m+1}
    LzRhs *st;     // [K]
    const double *x0;    // start vectors [K][n], unit norm, or null for the unit vectors e_j
    double *acc;         // null, or [K][n]: accumulates sum_n coef[k][n] K_n (Ritz vectors)
    const double *coef;  // [K][nu] with acc
    double gscale;       // G is scaled by this: 1 for unit start vectors, |b|^2 for a start vector b
};

// Single real vector of n rows on the stored matrix or the matrix-free operator; one partial
// per 256-row tile, summed in fixed order by one workgroup into the device scalars scal[].
struct SvDev {
    const HubbardOp *hub;  // matrix-free operator (device), or null
    const int64_t *slice_ptr;
    const int32_t *slice_w;
    const int32_t *ell_col;
    const double *ell_val;
    int64_t n, nblk;
    double *part;  // [2][nblk]
    double *scal;  // [8] device scalars
};

// one step n (0-based) of the recurrence for every unfinished right-hand side
hipError_t launch_lanczos_step(const LzDev &s, int n, hipStream_t st);
// lowest two eigenvalues of each reduced Hamiltonian (eig [K][2]) and the eigenvector of the
// lowest (u [K][nu], zero past m); scratch [K][nu]
hipError_t launch_lanczos_lowest(const LzDev &s, double *eig, double *u, double *scratch, hipStream_t st);
// y = H x; scal[0] = x . y; then scal[1] = ||y - scal[0] x||^2
hipError_t sv_rayleigh(const SvDev &s, const double *x, double *y, hipStream_t st);
// x <- x / ||x||, with the sign that makes x . ref >= 0 when ref is given; scal[2], scal[3]
hipError_t sv_normalize(const SvDev &s, double *x, const double *ref, hipStream_t st);
// real part to complex and back (n entries)
hipError_t sv_to_complex(const double *x, double2 *z, int64_t n, hipStream_t st);
hipError_t sv_real_part(const double2 *z, double *x, int64_t n, hipStream_t st);
// Fermion operator between Hubbard sectors: y[target(r)] = sign(r) x[r] for every source state
// r with the mode (site, spin) occupied (annihilation) or empty (creation); y is zeroed first.
// up_src/dn_src: the source sector's species patterns; binom: [L+1][L+1] binomial table;
// dn_tgt_count: the target sector's down-spin basis size.
hipError_t launch_fermion_op(const uint32_t *up_src, const uint32_t *dn_src, int64_t Du, int64_t Dd,
                             const int64_t *binom, int L, int n_up, int site, int spin, int create,
                             int64_t Dd_tgt, int64_t D_tgt, const double2 *x, double2 *y, hipStream_t st);
// G[k][r] = [(z_k - T_r)^{-1}]_11 for M shifts z (device) and K right-hand sides
hipError_t launch_lanczos_greens(const LzDev &s, const double2 *z, int64_t M, int64_t K_out, double2 *G,
                                 hipStream_t st);

}  // namespace scocg

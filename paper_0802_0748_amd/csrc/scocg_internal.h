// Internal declarations shared by the HIP kernels and the host driver of libscocg.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scocg {

// ---- complex helpers (double2 / float2 as interleaved re, im) ----
__host__ __device__ inline double2 cmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline bool cis0(double2 a) { return a.x == 0.0 && a.y == 0.0; }
// a / b with Smith's scaling (avoids overflow of |b|^2 for large |b|).
__host__ __device__ inline double2 cdiv(double2 a, double2 b)
{
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, d = b.x + b.y * r;
        return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    } else {
        double r = b.x / b.y, d = b.x * r + b.y;
        return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
    }
}
__host__ __device__ inline float2 cmulf(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---- per right-hand-side seed state ----
enum SeedStatus : int32_t {
    SEED_RUNNING = 0,   // iterating
    SEED_PAUSED = 1,    // seed converged: switch at the end of this block
    SEED_LIMIT = 2,     // iteration limit reached
    SEED_STOPPED = 3,   // finished (all pairs frozen or limit)
    SEED_BREAKDOWN = 4, // COCG breakdown
    SEED_SWITCH = 5     // switch decided; its vectors are switched once the update of the rhs's
                        // last block has finished (the rhs sits out one block meanwhile)
};

struct SeedState {
    double2 zs;          // seed shift
    double2 alpha_prev;  // alpha_{n-1}
    double2 beta_prev;   // beta_{n-1}
    double2 rho;         // r.r (unconjugated)
    double2 a0, b0;      // alpha_{n0-1}, beta_{n0-1} at the start of the current block
    double2 inv_pt;      // 1 / pi_t(n+1) of a pending seed switch (scales r)
    double2 inv_ppt;     // 1 / pi_t(n) of a pending seed switch (scales the stored directions)
    double nb;           // ||b||
    double rnorm;        // ||r||
    int32_t seed;        // seed shift index
    int32_t iter;        // iterations done
    int32_t step;        // iterations done in the current block
    int32_t base;        // ring slot of r at the start of the block
    int32_t status;
    int32_t sw_target;   // pending switch target or -1
    int32_t n_active;    // pairs still active after the last block
    int32_t switches;    // number of seed switches so far
    int32_t limit;       // iteration limit (max_iter or fixed_iter)
    int32_t sw_age;      // block ends since the switch decision (its vectors are switched at 1)
};

enum PairStatus : int32_t { PAIR_OK = 0, PAIR_BREAKDOWN = 4, PAIR_NOCONV = 5 };

// ---- matrix-free extended Hubbard ring (Sec. 4.2 model class) ----
// H = T_up (x) 1 + 1 (x) T_dn + D in the occupation-number basis, row = i_up * Dd + i_dn.
// A hop entry is the target configuration's index with bit 31 set when its value is +t
// (else -t); the hops of a configuration are sorted by target.
struct HubbardOp {
    const int32_t *up_ptr;   // [Du + 1]
    const uint32_t *up_hop;  // hops of the up-spin configurations
    const uint32_t *up_conf; // [Du] occupation bit patterns
    const int32_t *dn_ptr;   // [Dd + 1]
    const uint32_t *dn_hop;
    const uint32_t *dn_conf; // [Dd]
    int64_t Dd;              // down-spin configurations (the fast index of a row)
    double t, U, V;
    int32_t L;               // ring sites
    int32_t pad;
};

// Right-hand sides of at least this many rows sum their seed reductions with 1024 threads.
static constexpr int64_t RED_BIG_ROWS = 1 << 21;

// Down-spin blocks of at most this many configurations take the LDS-tiled product
// (one 16-byte element per configuration, 64 KB of LDS).
static constexpr int64_t HUB_LDS_MAX = 4096;

// ---- device-side matrix ----
struct DevCSR {
    int64_t n, nnz;
    int64_t nslices;      // 64-row slices
    int64_t ell_nnz;      // padded entries
    int64_t *d_slice_ptr; // [nslices+1] offsets into ell arrays
    int32_t *d_slice_w;   // [nslices] width (max row length) of each slice
    int32_t *d_ell_col;   // [ell_nnz] column, slice-major then lane
    double *d_ell_val;    // [ell_nnz]
    int32_t *d_ell_pos;   // [ell_nnz] CSR position of each slot (-1 padding)
    int64_t *d_row_ptr;   // [n+1] CSR pattern (int64)
    int32_t *d_col;       // [nnz]
    int32_t *d_mirror;    // [nnz] CSR position of the transposed entry (a, b) -> (b, a)
    double *d_val;        // [nnz] CSR values
    double trace;         // Tr(H) (host side)
    int64_t *h_row_ptr;   // host copies of the pattern (for value updates)
    int64_t *h_col;
    int64_t *h_ell_src;   // [ell_nnz] CSR position of each slot (host)
    int max_w;            // widest slice
    HubbardOp *d_hub;     // matrix-free operator (device struct), or null for a stored matrix
    void *d_hub_tables;   // device tables the operator points into
    int64_t hub_Dd;       // its down-spin configurations (host copy)
};

// ---- per right-hand side: its matrix and where its vectors live ----
// A solve may mix Hamiltonians of different sizes (one per right-hand side or shared).
// Vectors of rhs j occupy [voff, voff + n) of every [sum n]-long array (r ring slot, p,
// q, B); its pair vectors (x_k, u_k) start at M * voff + k * n.
struct RhsDesc {
    const int64_t *slice_ptr;
    const int32_t *slice_w;
    const int32_t *ell_col;
    const double *ell_val;
    int64_t nslices;
    int64_t n;
    int64_t voff;
    const HubbardOp *hub;  // matrix-free operator instead of the slices, or null
};

// ---- launch wrappers (kernels.hip) ----
struct SolveDev {
    const RhsDesc *desc;       // [K]
    int64_t ntot;              // sum of n over right-hand sides (stride of one ring slot)
    int64_t n, K, M;           // n: the largest row count
    int TB;                    // block length
    int R;                     // ring slots, 2 TB + 1: the update of one block reads its residuals
                               // while the next block's iterations write theirs
    int precision;             // 0 FP64 storage, 1 FP32
    int fixed;                 // fixed-iteration mode
    int switching;
    double tol;
    const double2 *z;          // [M]
    SeedState *seed;           // [K]
    double2 *ring;             // [R][ntot]
    double2 *p, *q;            // [K][n]
    void *X, *P;               // X [K][M][n], P [K][Mst][n] (double2 or float2); X is null in projection
                               // mode.  P holds the scaled directions u_k = pi_k p_k (see k_flush)
    int64_t Mst;               // direction vectors stored per rhs: M, or the window of seed candidates
    const int32_t *wshift;     // [K][Mst] shift of each stored direction, or null (slot w is shift w)
    const int32_t *wslot;      // [K*M] stored-direction slot of each pair or -1, or null (identity)
    double2 *Uproj;            // [K*M] u_k at the kept row for pairs without a stored direction, or null
    double2 *Xproj;            // [K][M] projected solution (projection mode) or null
    const double2 *wproj;      // [K][n] projection weights w (vector projection: Xproj = <w|x>), or null
    double2 *shist;            // [K][TB] s_n = w . r_n of the block's steps (vector projection)
    double2 *part3;            // [K][nblk] partials of w . r_n (vector projection)
    const int64_t *proj_row;   // [K] row kept in projection mode
    double2 *pi, *pi_prev, *beta_k; // [K*M]
    double *res;               // [K*M]
    int32_t *iters, *pstatus, *active, *nact; // [K*M]
    double2 *ahist, *bhist;    // [K][TB]
    double *rnhist;            // [K][TB]
    void *coef;                // [K*M][TB][2] (a', b') as double2 (FP64) or float2 (FP32 storage);
                               // coef, nact and blk are double-buffered by block parity: these
                               // point at this block's buffers
    int32_t *blk;              // [K][4] this block for the deferred update: steps, ring base, first block
    double2 *part2;            // [K][nblk] complex partials
    double *part1;             // [K][nblk] real partials
    uint32_t *cnt;             // [K] last-block counters
    int64_t nblk;              // row blocks of 256
    int shifts_per_wg;
    int zper;                  // 1: one shift per rhs (M = 1, z has K entries), used by refinement
    int spmv_rb;               // right-hand sides per SpMV thread (2: each rhs pair 2i, 2i+1 shares its matrix)
    int expanded;              // 1: the deferred update uses the expanded form (weights in coefx, MFMA kernel)
    double *coefx;             // [6 TB + 4][K*M] expanded weights of this block, pair fastest (double-buffered
                               // like coef): per step s (Re c_s, Im c_s, Re c_s + Im c_s, Re d_s, Im d_s,
                               // Re d_s + Im d_s), then gamma (re, im), delta (re, im)
    int has_sell, has_hub;     // some rhs has a stored matrix / a matrix-free Hubbard operator
    int hub_lds;               // every Hubbard operator's down-spin block fits the LDS-tiled product
    int has_red_small, has_red_big; // some rhs below / at or above 2^21 rows (per-rhs reduction width)
    int64_t hub_du_max;        // largest number of up-spin configurations among them
    unsigned long long *stats; // [0] algorithmic bytes of the deferred update, [1] updated pairs,
                               // [2] its algorithmic flops
    // Work lists of batches whose right-hand sides have different row counts (null otherwise): a
    // launch then covers exactly the (group or rhs, row block) items that hold rows, instead of
    // the full rectangle of largest-row-count x right-hand sides with most workgroups exiting.
    const int2 *it_grp;        // [n_it_grp] (rhs group of spmv_rb, 256-row block), in XCD sets of 8 groups
                               // (item 8 t + x of a set is group 8 s + x, block t); x = -1 marks a filler
    int64_t n_it_grp;
    const int2 *it_rhs;        // [n_it_rhs] (rhs, 256-row block)
    int64_t n_it_rhs;
    const int2 *it_upd;        // [n_it_upd] (rhs * shift groups + group, row tile of the update kernel)
    int64_t n_it_upd;
    int32_t *swlog;            // [K][M][2] seed switches of each rhs: (iterations done, new seed shift);
                               // a shift becomes the seed at most once, so M entries suffice
};

// A pair report with the layout of the C ABI's scocg_pair_report.
struct PairReportDev {
    int32_t iters, status;
    double res, res_true;
};

hipError_t launch_fill_desc(const RhsDesc &proto, int64_t K, int32_t seed, RhsDesc *desc, int32_t *seeds,
                            hipStream_t st);
hipError_t launch_all_stopped(const SeedState *seed, int64_t K, int32_t *flag, hipStream_t st);
hipError_t launch_pack_report(int64_t K, int64_t M, int fixed, const int32_t *iters, const int32_t *pstatus,
                              const double *res, const SeedState *seed, PairReportDev *rep, int32_t *worst,
                              long long *totals, hipStream_t st);

hipError_t launch_init(const SolveDev &s, const double2 *B, const int64_t *unit_idx,
                       const int32_t *seed_idx, int32_t limit, hipStream_t st);
// one seed iteration (four launches, see kernels.hip)
hipError_t launch_seed_iteration(const SolveDev &s, hipStream_t st);
hipError_t launch_pair_scalars(const SolveDev &s, hipStream_t st);
hipError_t launch_flush(const SolveDev &s, hipStream_t st);
hipError_t launch_block_finalize(const SolveDev &s, hipStream_t st);
hipError_t launch_switch_vectors(const SolveDev &s, hipStream_t st);
hipError_t launch_zero(void *ptr, size_t bytes, hipStream_t st);
hipError_t launch_store_solution(const SolveDev &s, double2 *Xout, hipStream_t st);
// r = b - (z - H) x for `count` pairs (pair_list[c], or c if pair_list is null): relative norms
// into out_res[c] (divided by bnorm[rhs]) and, if rout is given, the vectors into rout[c][n].
// part needs count * ceil(n / 256) doubles.
hipError_t launch_residual(const SolveDev &s, const double2 *B, const int64_t *unit_idx, const double2 *X64,
                           const int64_t *pair_list, int64_t count, const double *bnorm, double2 *rout,
                           double *part, double *out_res, hipStream_t st);
hipError_t launch_add_correction(int64_t n, const int64_t *pair_list, int64_t count, const double2 *D, double2 *X,
                                 hipStream_t st);
hipError_t launch_gather_diag(const SolveDev &s, const int64_t *rows, double2 *G, hipStream_t st);
hipError_t launch_density_rho(int64_t n, int64_t K, int64_t M, const double2 *X, const int64_t *cols_of_rhs,
                              const int64_t *row_ptr, const int32_t *col, const int32_t *mirror, const double2 *w,
                              const double2 *z, double *rho, double *Epart, double *Eacc, hipStream_t st);
hipError_t launch_pair_weights(int mode, int64_t K, int64_t M, const double2 *w, const double2 *z,
                               const double2 *g, double2 *c, hipStream_t st);
// grad[e] += Re sum_p c_p x_p[a] x_p[b] over the stored entries e = (a, b) of the CSR pattern,
// through part ([nchunk][nnz] doubles, nchunk from pair_outer_chunks).
int64_t pair_outer_chunks(int64_t n, int64_t npairs, int max_row);
hipError_t launch_pair_outer(int64_t n, int64_t npairs, const double2 *X, const double2 *c, const int64_t *row_ptr,
                             const int32_t *col, int64_t nnz, int max_row, int64_t nchunk, double *part, double *grad,
                             hipStream_t st);

}  // namespace scocg

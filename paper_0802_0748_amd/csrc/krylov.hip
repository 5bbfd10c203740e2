// Krylov-subspace diagonalization (Sec. 3.2, eq. Ham_in_KS) for many unit right-hand sides:
// the three-term recurrence builds each orthonormal basis {K_n} of K_nu(H, |j>), in which H
// is the tridiagonal T with diagonal a_n = <K_n|H|K_n> and off-diagonal b_{n+1} = <K_{n+1}|H|K_n>;
// the local Green's function is then G_jj(z) = [(z - T)^{-1}]_11, evaluated as the continued
// fraction of T.  Per step, for every unfinished right-hand side:
//   w = H K_n - b_n K_{n-1};  a_n = K_n . w;  w <- w - a_n K_n;  b_{n+1} = ||w||;
//   K_{n+1} = w / b_{n+1}  (applied on the fly by the next step as w * (1 / b_{n+1})).
// Start vectors are unit vectors, so every basis vector is real.  Sums are fixed-order
// (per 256-row tile, then the tiles in index order), so results do not depend on scheduling.
#include "device_common.h"
#include "hubbard_rows.h"
#include "krylov.h"

namespace scocg {

typedef double d4v __attribute__((ext_vector_type(4)));
static_assert(LZ_TILE == WG, "one 256-row tile per workgroup");

// One row of a group of RB interleaved vectors: four doubles (one 32-byte access), or one.
template <int RB> struct LzRow;
template <> struct LzRow<4> {
    typedef d4v T;
};
struct LzOne {
    double v;
    __device__ double &operator[](int) { return v; }
    __device__ double operator[](int) const { return v; }
};
template <> struct LzRow<1> {
    typedef LzOne T;
};

// Tree sums of RB values over the WG threads (result in thread 0).
template <int RB>
__device__ inline void block_sum_rb(double (&v)[RB], double (*sh)[WG])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int b = 0; b < RB; ++b) sh[b][t] = v[b];
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if (t < h) {
#pragma unroll
            for (int b = 0; b < RB; ++b) sh[b][t] += sh[b][t + h];
        }
        __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < RB; ++b) v[b] = sh[b][0];
}

// Fixed-order sum of a right-hand side's tile partials by one workgroup (result in thread 0):
// thread t adds partials t, t + WG, ... in order, then the threads' sums as a tree.
__device__ inline double sum_tiles(const double *part, int64_t nblk, double *sh)
{
    double acc = 0;
    int64_t b = threadIdx.x;
    for (; b + 7 * WG < nblk; b += 8 * WG) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[b + u * WG];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; b < nblk; b += WG) acc += part[b];
    const int t = threadIdx.x;
    sh[t] = acc;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if (t < h) sh[t] += sh[t + h];
        __syncthreads();
    }
    return sh[0];
}

// w = H K_n - b_n K_{n-1} and the partials of K_n . w; K_n (= the previous w times 1/b_n, or
// the unit vector at step 0) is written out for the step after.
template <int RB>
__global__ void __launch_bounds__(WG) k_lz_matvec(LzDev s, int n)
{
    typedef typename LzRow<RB>::T VR;
    __shared__ double sh[RB][WG];
    const int64_t g = blockIdx.y;
    bool run[RB];
    double bprev[RB], rb[RB];
    int64_t jj[RB];
    bool any = false;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        const LzRhs st = s.st[g * RB + b];
        run[b] = !st.done;
        bprev[b] = run[b] ? st.bprev : 0.0;
        rb[b] = (run[b] && n > 0) ? 1.0 / st.bprev : 0.0;
        jj[b] = st.j;
        any = any || run[b];
    }
    if (!any) return;  // uniform over the workgroup
    const int q = n & 1;
    const int64_t base = g * s.n;
    const VR *Wp = (const VR *)(s.W[q ^ 1]) + base;
    const VR *Vp = (const VR *)(s.V[q ^ 1]) + base;
    VR *Vn = (VR *)(s.V[q]) + base;
    VR *Wn = (VR *)(s.W[q]) + base;
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    double dot[RB] = {};
    if (row < s.n) {
        double acc[RB] = {};
        // one term of the row: acc += v x[c]
        auto slot = [&](int64_t c, double v) {
            double x[RB];
            if (n == 0 && s.x0) {
#pragma unroll
                for (int b = 0; b < RB; ++b) x[b] = run[b] ? s.x0[(g * RB + b) * s.n + c] : 0.0;
            } else if (n == 0) {
#pragma unroll
                for (int b = 0; b < RB; ++b) x[b] = (c == jj[b]) ? 1.0 : 0.0;
            } else {
                const VR wc = Wp[c];
#pragma unroll
                for (int b = 0; b < RB; ++b) x[b] = wc[b] * rb[b];
            }
#pragma unroll
            for (int b = 0; b < RB; ++b) acc[b] = fma(v, x[b], acc[b]);
        };
        if (s.hub) {
            // the operator's terms in the stored row's column order: the same sums
            hubbard_row_terms(s.hub, row, slot);
        } else {
            const int64_t slice = row >> 6;
            const int lane = (int)(row & 63);
            const int64_t off = s.slice_ptr[slice];
            const int w = s.slice_w[slice];
            const int32_t *colp = s.ell_col + off + lane;
            const double *valp = s.ell_val + off + lane;
            // slots in the stored order; column and value loads of LZ_CHUNK slots are issued
            // before their gathers
            constexpr int LZ_CHUNK = 4;
            int k = 0;
            for (; k + LZ_CHUNK <= w; k += LZ_CHUNK) {
                int32_t c[LZ_CHUNK];
                double v[LZ_CHUNK];
#pragma unroll
                for (int u = 0; u < LZ_CHUNK; ++u) {
                    c[u] = colp[(int64_t)(k + u) * 64];
                    v[u] = valp[(int64_t)(k + u) * 64];
                }
#pragma unroll
                for (int u = 0; u < LZ_CHUNK; ++u) slot(c[u], v[u]);
            }
            for (; k < w; ++k) slot(colp[(int64_t)k * 64], valp[(int64_t)k * 64]);
        }
        VR vo, wo;
        if (n == 0) {
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                vo[b] = s.x0 ? (run[b] ? s.x0[(g * RB + b) * s.n + row] : 0.0) : ((row == jj[b]) ? 1.0 : 0.0);
                wo[b] = acc[b];
            }
        } else {
            const VR wr = Wp[row], vr = Vp[row];
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                vo[b] = wr[b] * rb[b];
                wo[b] = fma(-bprev[b], vr[b], acc[b]);
            }
        }
        Vn[row] = vo;
        Wn[row] = wo;
        if (s.acc) {
#pragma unroll
            for (int b = 0; b < RB; ++b)
                if (run[b]) {
                    const int64_t k = g * RB + b;
                    s.acc[k * s.n + row] = fma(s.coef[k * s.nu + n], vo[b], s.acc[k * s.n + row]);
                }
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) dot[b] = vo[b] * wo[b];
    }
    block_sum_rb<RB>(dot, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int b = 0; b < RB; ++b)
            if (run[b]) s.part[(g * RB + b) * s.nblk + blockIdx.x] = dot[b];
    }
}

// a_n from the partials of K_n . w
__global__ void __launch_bounds__(WG) k_lz_alpha(LzDev s, int n)
{
    __shared__ double sh[WG];
    const int64_t j = blockIdx.x;
    if (s.st[j].done) return;
    const double a = sum_tiles(s.part + j * s.nblk, s.nblk, sh);
    if (threadIdx.x == 0) {
        s.st[j].a = a;
        s.ab[j * 2 * s.nu + n] = a;
    }
}

// w <- w - a_n K_n and the partials of ||w||^2
template <int RB>
__global__ void __launch_bounds__(WG) k_lz_axpy(LzDev s, int n)
{
    typedef typename LzRow<RB>::T VR;
    __shared__ double sh[RB][WG];
    const int64_t g = blockIdx.y;
    bool run[RB];
    double a[RB];
    bool any = false;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        const LzRhs st = s.st[g * RB + b];
        run[b] = !st.done;
        a[b] = run[b] ? st.a : 0.0;
        any = any || run[b];
    }
    if (!any) return;
    const int q = n & 1;
    const int64_t base = g * s.n;
    const VR *Vn = (const VR *)(s.V[q]) + base;
    VR *Wn = (VR *)(s.W[q]) + base;
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    double nn[RB] = {};
    if (row < s.n) {
        const VR v = Vn[row];
        VR w = Wn[row];
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            w[b] = fma(-a[b], v[b], w[b]);
            nn[b] = w[b] * w[b];
        }
        Wn[row] = w;
    }
    block_sum_rb<RB>(nn, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int b = 0; b < RB; ++b)
            if (run[b]) s.part[(g * RB + b) * s.nblk + blockIdx.x] = nn[b];
    }
}

// b_{n+1} = ||w||, the end test, and the state for the next step
__global__ void __launch_bounds__(WG) k_lz_beta(LzDev s, int n)
{
    __shared__ double sh[WG];
    const int64_t j = blockIdx.x;
    const LzRhs st = s.st[j];
    if (st.done) return;
    const double b = sqrt(sum_tiles(s.part + j * s.nblk, s.nblk, sh));
    if (threadIdx.x == 0) {
        s.ab[j * 2 * s.nu + s.nu + n] = b;
        LzRhs *w = s.st + j;
        w->m = n + 1;
        if (n == s.nu - 1 || b <= LZ_STOP_REL * (fabs(st.a) + st.bprev)) w->done = 1;
        else w->bprev = b;
    }
}

// G[k][r] = [(z_k - T_r)^{-1}]_11 by the continued fraction of T_r, innermost level first
__global__ void __launch_bounds__(WG) k_lz_greens(LzDev s, const double2 *__restrict__ z, int64_t M, int64_t K,
                                                  double2 *__restrict__ G)
{
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= M * K) return;
    const int64_t k = i / K, r = i % K;
    const int m = s.st[r].m;
    const double *a = s.ab + r * 2 * s.nu;
    const double *b = a + s.nu;
    const double2 zk = z[k];
    double2 g = cdiv(cmk(1, 0), cmk(zk.x - a[m - 1], zk.y));
    for (int t = m - 2; t >= 0; --t) {
        const double bb = b[t] * b[t];
        g = cdiv(cmk(1, 0), cmk(zk.x - a[t] - bb * g.x, zk.y - bb * g.y));
    }
    G[k * K + r] = make_double2(s.gscale * g.x, s.gscale * g.y);
}

// Lowest two eigenvalues of the reduced Hamiltonian by bisection on Sturm counts (the number
// of negative pivots of T - x), and the eigenvector of the lowest by inverse iteration with a
// tridiagonal solve.  One thread per right-hand side.
__device__ inline int sturm_count(const double *a, const double *b, int m, double x)
{
    int cnt = 0;
    double d = 1.0;
    for (int t = 0; t < m; ++t) {
        const double off = t > 0 ? b[t - 1] * b[t - 1] : 0.0;
        d = a[t] - x - (t > 0 ? off / d : 0.0);
        if (d == 0.0) d = -1e-300;
        cnt += d < 0.0;
    }
    return cnt;
}

__device__ inline double kth_eigenvalue(const double *a, const double *b, int m, int k, double lo, double hi)
{
    // smallest x with at least k eigenvalues below it
    for (int it = 0; it < 200 && hi - lo > 1e-15 * fmax(1.0, fmax(fabs(lo), fabs(hi))); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(a, b, m, mid) >= k) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

__global__ void __launch_bounds__(64) k_lz_lowest(LzDev s, double *eig, double *u, double *scratch)
{
    if (threadIdx.x != 0) return;
    const int64_t j = blockIdx.x;
    const int m = s.st[j].m;
    const double *a = s.ab + j * 2 * s.nu;
    const double *b = a + s.nu;
    double lo = 0, hi = 0;
    for (int t = 0; t < m; ++t) {
        const double r = (t > 0 ? fabs(b[t - 1]) : 0.0) + (t + 1 < m ? fabs(b[t]) : 0.0);
        lo = t == 0 ? a[t] - r : fmin(lo, a[t] - r);
        hi = t == 0 ? a[t] + r : fmax(hi, a[t] + r);
    }
    lo -= 1e-12 * fmax(1.0, fabs(lo));
    hi += 1e-12 * fmax(1.0, fabs(hi));
    const double e0 = kth_eigenvalue(a, b, m, 1, lo, hi);
    const double e1 = m > 1 ? kth_eigenvalue(a, b, m, 2, lo, hi) : e0;
    eig[2 * j] = e0;
    eig[2 * j + 1] = e1;
    // (T - e0) v = w by the tridiagonal elimination, twice from w = 1
    double *v = u + j * s.nu;
    double *cp = scratch + j * s.nu;
    // a pivot that vanishes (the shift is an eigenvalue) is replaced by 1e-14 of the scale:
    // the solve then amplifies the eigenvector by about 1e14, which the normalization removes
    const double tiny = 1e-14 * fmax(1.0, fabs(e0));
    auto guard = [&](double d) { return fabs(d) < tiny ? (d < 0 ? -tiny : tiny) : d; };
    for (int t = 0; t < s.nu; ++t) v[t] = t < m ? 1.0 : 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        double den = guard(a[0] - e0);
        cp[0] = m > 1 ? b[0] / den : 0.0;
        v[0] = v[0] / den;
        for (int t = 1; t < m; ++t) {
            den = guard(a[t] - e0 - b[t - 1] * cp[t - 1]);
            cp[t] = t + 1 < m ? b[t] / den : 0.0;
            v[t] = (v[t] - b[t - 1] * v[t - 1]) / den;
        }
        for (int t = m - 2; t >= 0; --t) v[t] -= cp[t] * v[t + 1];
        double vmax = 0;
        for (int t = 0; t < m; ++t) vmax = fmax(vmax, fabs(v[t]));
        double nn = 0;
        for (int t = 0; t < m; ++t) {
            v[t] /= vmax;
            nn += v[t] * v[t];
        }
        const double inv = 1.0 / sqrt(nn);
        for (int t = 0; t < m; ++t) v[t] *= inv;
    }
}

// ---- single vector on the stored matrix ----
__global__ void __launch_bounds__(WG) k_sv_matvec(SvDev s, const double *__restrict__ x, double *__restrict__ y)
{
    __shared__ double sh[WG];
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    double d = 0;
    if (row < s.n) {
        double acc = 0;
        if (s.hub) {
            hubbard_row_terms(s.hub, row, [&](int64_t c, double v) { acc = fma(v, x[c], acc); });
        } else {
            const int64_t slice = row >> 6;
            const int lane = (int)(row & 63);
            const int64_t off = s.slice_ptr[slice];
            const int w = s.slice_w[slice];
            for (int k = 0; k < w; ++k) {
                const int64_t e = off + (int64_t)k * 64 + lane;
                acc = fma(s.ell_val[e], x[s.ell_col[e]], acc);
            }
        }
        y[row] = acc;
        d = x[row] * acc;
    }
    sh[threadIdx.x] = d;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) s.part[blockIdx.x] = sh[0];
}

// partials of ||y - E x||^2 (E = scal[0]) into part, or of ||x||^2 and x . ref into part, part + nblk
__global__ void __launch_bounds__(WG) k_sv_resid(SvDev s, const double *__restrict__ x, const double *__restrict__ y)
{
    __shared__ double sh[WG];
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    double d = 0;
    if (row < s.n) {
        const double r = fma(-s.scal[0], x[row], y[row]);
        d = r * r;
    }
    sh[threadIdx.x] = d;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) s.part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(WG) k_sv_norm_dot(SvDev s, const double *__restrict__ x, const double *__restrict__ ref)
{
    __shared__ double sh[2][WG];
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    double nn = 0, dd = 0;
    if (row < s.n) {
        nn = x[row] * x[row];
        dd = ref ? x[row] * ref[row] : 0.0;
    }
    sh[0][threadIdx.x] = nn;
    sh[1][threadIdx.x] = dd;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        s.part[blockIdx.x] = sh[0][0];
        s.part[s.nblk + blockIdx.x] = sh[1][0];
    }
}

// scal[slot] = sum of the nblk partials at part + off (fixed order)
__global__ void __launch_bounds__(WG) k_sv_sum(SvDev s, int64_t off, int slot)
{
    __shared__ double sh[WG];
    const double v = sum_tiles(s.part + off, s.nblk, sh);
    if (threadIdx.x == 0) s.scal[slot] = v;
}

__global__ void __launch_bounds__(WG) k_sv_scale(SvDev s, double *__restrict__ x)
{
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (row >= s.n) return;
    const double f = (s.scal[3] < 0 ? -1.0 : 1.0) / sqrt(s.scal[2]);
    x[row] *= f;
}

__global__ void k_to_complex(const double *__restrict__ x, double2 *__restrict__ z, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = cmk(x[i], 0.0);
}

__global__ void k_real_part(const double2 *__restrict__ z, double *__restrict__ x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = z[i].x;
}

// ---- fermion operator between Hubbard sectors ----
// Rank of an L-bit pattern among the patterns with the same number of set bits, in
// increasing integer order: sum over its set bits p_0 < p_1 < ... of C(p_t, t + 1).
__device__ inline int64_t pattern_rank(uint32_t s, const int64_t *binom, int L)
{
    int64_t r = 0;
    int t = 0;
    for (int p = 0; p < L; ++p)
        if ((s >> p) & 1u) {
            ++t;
            r += binom[p * (L + 1) + t];
        }
    return r;
}

__global__ void k_zero2(double2 *y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = cmk(0, 0);
}

__global__ void k_fermion_op(const uint32_t *__restrict__ up, const uint32_t *__restrict__ dn, int64_t Du, int64_t Dd,
                             const int64_t *__restrict__ binom, int L, int n_up, int site, int spin, int create,
                             int64_t Dd_tgt, const double2 *__restrict__ x, double2 *__restrict__ y)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= Du * Dd) return;
    const int64_t iu = r / Dd, idn = r % Dd;
    const uint32_t su = up[iu], sd = dn[idn];
    const uint32_t bit = 1u << site;
    const uint32_t s = spin == 0 ? su : sd;
    const bool occupied = (s & bit) != 0;
    if (occupied == (create != 0)) return;
    // Jordan-Wigner order: all up-spin modes (sites ascending), then all down-spin modes
    const int before = __popc(s & (bit - 1u)) + (spin == 0 ? 0 : n_up);
    const double sg = (before & 1) ? -1.0 : 1.0;
    int64_t k;
    if (spin == 0) k = pattern_rank(su ^ bit, binom, L) * Dd_tgt + idn;
    else k = iu * Dd_tgt + pattern_rank(sd ^ bit, binom, L);
    y[k] = make_double2(sg * x[r].x, sg * x[r].y);
}

hipError_t launch_lanczos_step(const LzDev &s, int n, hipStream_t st)
{
    if (s.rb != 1 && s.rb != LZ_RB) return hipErrorInvalidValue;
    const int64_t groups = s.K / s.rb;
    if (s.nblk > 0x7fffffffLL || groups > 65535 || s.K > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const dim3 gv((unsigned)s.nblk, (unsigned)groups);
    if (s.rb == 1) hipLaunchKernelGGL(k_lz_matvec<1>, gv, dim3(WG), 0, st, s, n);
    else hipLaunchKernelGGL(k_lz_matvec<LZ_RB>, gv, dim3(WG), 0, st, s, n);
    hipLaunchKernelGGL(k_lz_alpha, dim3((unsigned)s.K), dim3(WG), 0, st, s, n);
    if (s.rb == 1) hipLaunchKernelGGL(k_lz_axpy<1>, gv, dim3(WG), 0, st, s, n);
    else hipLaunchKernelGGL(k_lz_axpy<LZ_RB>, gv, dim3(WG), 0, st, s, n);
    hipLaunchKernelGGL(k_lz_beta, dim3((unsigned)s.K), dim3(WG), 0, st, s, n);
    return hipGetLastError();
}

hipError_t launch_lanczos_greens(const LzDev &s, const double2 *z, int64_t M, int64_t K_out, double2 *G,
                                 hipStream_t st)
{
    const int64_t total = M * K_out;
    if (total == 0) return hipSuccess;
    if ((total + WG - 1) / WG > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_lz_greens, dim3((unsigned)((total + WG - 1) / WG)), dim3(WG), 0, st, s, z, M, K_out, G);
    return hipGetLastError();
}

hipError_t launch_lanczos_lowest(const LzDev &s, double *eig, double *u, double *scratch, hipStream_t st)
{
    hipLaunchKernelGGL(k_lz_lowest, dim3((unsigned)s.K), dim3(64), 0, st, s, eig, u, scratch);
    return hipGetLastError();
}

hipError_t sv_rayleigh(const SvDev &s, const double *x, double *y, hipStream_t st)
{
    const dim3 g((unsigned)s.nblk);
    hipLaunchKernelGGL(k_sv_matvec, g, dim3(WG), 0, st, s, x, y);
    hipLaunchKernelGGL(k_sv_sum, dim3(1), dim3(WG), 0, st, s, (int64_t)0, 0);
    hipLaunchKernelGGL(k_sv_resid, g, dim3(WG), 0, st, s, x, (const double *)y);
    hipLaunchKernelGGL(k_sv_sum, dim3(1), dim3(WG), 0, st, s, (int64_t)0, 1);
    return hipGetLastError();
}

hipError_t sv_normalize(const SvDev &s, double *x, const double *ref, hipStream_t st)
{
    const dim3 g((unsigned)s.nblk);
    hipLaunchKernelGGL(k_sv_norm_dot, g, dim3(WG), 0, st, s, (const double *)x, ref);
    hipLaunchKernelGGL(k_sv_sum, dim3(1), dim3(WG), 0, st, s, (int64_t)0, 2);
    hipLaunchKernelGGL(k_sv_sum, dim3(1), dim3(WG), 0, st, s, s.nblk, 3);
    hipLaunchKernelGGL(k_sv_scale, g, dim3(WG), 0, st, s, x);
    return hipGetLastError();
}

hipError_t sv_to_complex(const double *x, double2 *z, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_complex, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, st, x, z, n);
    return hipGetLastError();
}

hipError_t sv_real_part(const double2 *z, double *x, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_real_part, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, st, z, x, n);
    return hipGetLastError();
}

hipError_t launch_fermion_op(const uint32_t *up_src, const uint32_t *dn_src, int64_t Du, int64_t Dd,
                             const int64_t *binom, int L, int n_up, int site, int spin, int create,
                             int64_t Dd_tgt, int64_t D_tgt, const double2 *x, double2 *y, hipStream_t st)
{
    const int64_t D = Du * Dd;
    if ((D + WG - 1) / WG > 0x7fffffffLL || (D_tgt + WG - 1) / WG > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_zero2, dim3((unsigned)((D_tgt + WG - 1) / WG)), dim3(WG), 0, st, y, D_tgt);
    hipLaunchKernelGGL(k_fermion_op, dim3((unsigned)((D + WG - 1) / WG)), dim3(WG), 0, st, up_src, dn_src, Du, Dd, binom, L,
                       n_up, site, spin, create, Dd_tgt, x, y);
    return hipGetLastError();
}

}  // namespace scocg

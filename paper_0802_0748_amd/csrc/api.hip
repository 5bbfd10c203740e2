// Host side of libscocg: argument checking, matrix upload, the iteration driver and the
// observable entry points declared in include/scocg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/scocg.h"
#include "krylov.h"
#include "scocg_internal.h"

using namespace scocg;

namespace {

thread_local std::string g_err;
thread_local scocg_timing g_timing = {};
// seed switches of the last solve on this thread: per rhs, (iterations done, new seed) pairs
struct SwitchLog {
    int64_t K = 0, M = 0;
    std::vector<int32_t> count;  // [K]
    std::vector<int32_t> log;    // [K][M][2]
};
thread_local SwitchLog g_swlog;
int g_profiling = 0;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

// Buffers the kernels read or write must be device-accessible (device, pinned host or managed
// memory): a plain host pointer would make the GPU fault, so it is refused up front.
static bool device_ok(const void *p)
{
    if (!p) return true;  // optional buffers are checked for null by the caller
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type != hipMemoryTypeUnregistered && a.devicePointer != nullptr;
}
#define REQUIRE_DEVICE(...)                                                                                    \
    do {                                                                                                       \
        for (const void *p_ : {__VA_ARGS__})                                                                   \
            if (!device_ok(p_)) return fail(SCOCG_EINVAL, "a vector or output argument is not device memory"); \
    } while (0)

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(SCOCG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device allocations released when the owner goes out of scope.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    hipError_t alloc(size_t b)
    {
        release();
        bytes = b;
        if (b == 0) return hipSuccess;
        return hipMalloc(&ptr, b);
    }
    template <typename T>
    T *as() const { return (T *)ptr; }
};

// A pair of timing events destroyed when the owner goes out of scope (also on error returns).
struct TimerEvents {
    hipEvent_t t0 = nullptr, t1 = nullptr;
    TimerEvents() = default;
    TimerEvents(const TimerEvents &) = delete;
    TimerEvents &operator=(const TimerEvents &) = delete;
    ~TimerEvents()
    {
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
    }
    hipError_t create()
    {
        hipError_t e = hipEventCreate(&t0);
        return e == hipSuccess ? hipEventCreate(&t1) : e;
    }
};

struct GraphPair {
    hipStream_t cap = nullptr;
    hipGraph_t ga[2] = {nullptr, nullptr}, gb = nullptr;
    hipGraphExec_t ea[2] = {nullptr, nullptr}, eb = nullptr;
    ~GraphPair()
    {
        for (int q = 0; q < 2; ++q) {
            if (ea[q]) (void)hipGraphExecDestroy(ea[q]);
            if (ga[q]) (void)hipGraphDestroy(ga[q]);
        }
        if (eb) (void)hipGraphExecDestroy(eb);
        if (gb) (void)hipGraphDestroy(gb);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

struct PinnedBuf {
    void *ptr = nullptr;
    ~PinnedBuf()
    {
        if (ptr) (void)hipHostFree(ptr);
    }
    hipError_t alloc(size_t b) { return hipHostMalloc(&ptr, b, hipHostMallocDefault); }
};

}  // namespace

// An uploaded matrix is shared by its owner (released with csr_free) and by every tape that
// was recorded on it (released with tape_free): backward() reads its pattern, so the device
// and host copies live until the last of them is released.
struct scocg_csr {
    DevCSR d;
    std::vector<int64_t> h_row_ptr, h_col, h_ell_src;
    std::vector<double> h_val;
    std::atomic<int> refs{1};
};

static void csr_release(scocg_csr *H);

struct scocg_tape {
    scocg_csr *H = nullptr;  // holds a reference (released with the tape)
    int64_t K = 0, M = 0, n = 0;
    DevBuf X;  // [K][M][n] complex FP64
    ~scocg_tape()
    {
        X.release();
        if (H) csr_release(H);
    }
};

// ------------------------------------------------------------------------------------------
// matrix checks and upload
// ------------------------------------------------------------------------------------------
extern "C" int scocg_csr_validate(int64_t n, int64_t nnz, const int64_t *rp, const int64_t *col, const double *val)
{
    if (n <= 0) return fail(SCOCG_EINVAL, "n must be positive");
    if (nnz < 0) return fail(SCOCG_EINVAL, "nnz must be non-negative");
    if (!rp || (nnz > 0 && (!col || !val))) return fail(SCOCG_EINVAL, "null CSR array");
    if (rp[0] != 0 || rp[n] != nnz) return fail(SCOCG_EINVAL, "row_ptr must start at 0 and end at nnz");
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return fail(SCOCG_EINVAL, "row_ptr is not monotone at row " + std::to_string(i));
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (col[k] < 0 || col[k] >= n)
                return fail(SCOCG_EINVAL, "column out of range in row " + std::to_string(i));
            if (k > rp[i] && col[k] <= col[k - 1])
                return fail(SCOCG_EINVAL, "columns not sorted/unique in row " + std::to_string(i));
            if (!std::isfinite(val[k])) return fail(SCOCG_EINVAL, "non-finite value in row " + std::to_string(i));
        }
    }
    // symmetry: H_ij must equal H_ji bitwise (binary search in row j)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t j = col[k];
            const int64_t *b = col + rp[j], *e = col + rp[j + 1];
            const int64_t *f = std::lower_bound(b, e, i);
            if (f == e || *f != i)
                return fail(SCOCG_EINVAL, "pattern not symmetric at (" + std::to_string(i) + "," + std::to_string(j) + ")");
            if (val[f - col] != val[k])
                return fail(SCOCG_EINVAL, "values not symmetric at (" + std::to_string(i) + "," + std::to_string(j) + ")");
        }
    }
    return SCOCG_OK;
}

static void free_dev(DevCSR &d)
{
    void *ptrs[] = {d.d_slice_ptr, d.d_slice_w, d.d_ell_col, d.d_ell_val, d.d_ell_pos, d.d_row_ptr, d.d_col, d.d_val,
                    d.d_mirror, d.d_hub, d.d_hub_tables};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    std::memset(&d, 0, sizeof(d));
}

template <typename T>
static hipError_t upload(T **dst, const T *src, size_t count, hipStream_t st)
{
    hipError_t e = hipMalloc((void **)dst, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    if (count == 0) return hipSuccess;
    e = hipMemcpyAsync(*dst, src, count * sizeof(T), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

extern "C" int csr_upload(int64_t n, int64_t nnz, const int64_t *rp, const int64_t *col, const double *val,
                          int validate, void *stream, scocg_csr_t *out)
{
    g_err.clear();
    if (!out) return fail(SCOCG_EINVAL, "out is null");
    *out = nullptr;
    if (n <= 0 || n >= (1LL << 31) || nnz < 0 || nnz >= (1LL << 31))
        return fail(SCOCG_EINVAL, "n and nnz must be in (0, 2^31)");
    if (!rp || (nnz > 0 && (!col || !val))) return fail(SCOCG_EINVAL, "null CSR array");
    if (validate) {
        int rc = scocg_csr_validate(n, nnz, rp, col, val);
        if (rc) return rc;
    } else if (rp[0] != 0 || rp[n] != nnz) {
        return fail(SCOCG_EINVAL, "row_ptr must start at 0 and end at nnz");
    }
    hipStream_t st = (hipStream_t)stream;
    scocg_csr *H = new scocg_csr();
    DevCSR &d = H->d;
    d.n = n;
    d.nnz = nnz;
    d.nslices = (n + 63) / 64;
    H->h_row_ptr.assign(rp, rp + n + 1);
    H->h_col.assign(col, col + nnz);
    H->h_val.assign(val, val + nnz);
    // 64-row slices, padded to the widest row of the slice; padding points at row 0 with value 0
    std::vector<int64_t> sptr(d.nslices + 1, 0);
    std::vector<int32_t> sw(d.nslices, 0);
    int maxw = 0;
    for (int64_t s = 0; s < d.nslices; ++s) {
        int w = 0;
        for (int64_t r = s * 64; r < std::min(n, s * 64 + 64); ++r) w = std::max<int>(w, (int)(rp[r + 1] - rp[r]));
        sw[s] = w;
        maxw = std::max(maxw, w);
        sptr[s + 1] = sptr[s] + (int64_t)w * 64;
    }
    d.ell_nnz = sptr[d.nslices];
    d.max_w = maxw;
    std::vector<int32_t> ecol(d.ell_nnz, 0);
    std::vector<double> eval(d.ell_nnz, 0.0);
    H->h_ell_src.assign(d.ell_nnz, -1);
    for (int64_t s = 0; s < d.nslices; ++s) {
        for (int lane = 0; lane < 64; ++lane) {
            const int64_t r = s * 64 + lane;
            if (r >= n) continue;
            for (int64_t k = rp[r]; k < rp[r + 1]; ++k) {
                const int64_t slot = sptr[s] + (k - rp[r]) * 64 + lane;
                ecol[slot] = (int32_t)col[k];
                eval[slot] = val[k];
                H->h_ell_src[slot] = k;
            }
        }
    }
    double tr = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (col[k] == i) tr += val[k];
    d.trace = tr;
    std::vector<int32_t> col32(nnz);
    for (int64_t k = 0; k < nnz; ++k) col32[k] = (int32_t)col[k];
    // position of the transposed entry (the pattern is symmetric when validated; an entry whose
    // mirror is missing points at itself)
    std::vector<int32_t> mirror(nnz);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t j = col[k];
            const int64_t *b = col + rp[j], *e = col + rp[j + 1];
            const int64_t *f = std::lower_bound(b, e, i);
            mirror[k] = (int32_t)((f != e && *f == i) ? (f - col) : k);
        }
    hipError_t e = hipSuccess;
    if ((e = upload(&d.d_slice_ptr, sptr.data(), sptr.size(), st)) != hipSuccess ||
        (e = upload(&d.d_slice_w, sw.data(), sw.size(), st)) != hipSuccess ||
        (e = upload(&d.d_ell_col, ecol.data(), ecol.size(), st)) != hipSuccess ||
        (e = upload(&d.d_ell_val, eval.data(), eval.size(), st)) != hipSuccess ||
        (e = upload(&d.d_row_ptr, rp, (size_t)n + 1, st)) != hipSuccess ||
        (e = upload(&d.d_col, col32.data(), col32.size(), st)) != hipSuccess ||
        (e = upload(&d.d_mirror, mirror.data(), mirror.size(), st)) != hipSuccess ||
        (e = upload(&d.d_val, val, (size_t)nnz, st)) != hipSuccess) {
        free_dev(d);
        delete H;
        return fail(e == hipErrorOutOfMemory ? SCOCG_ENOMEM : SCOCG_EHIP,
                    std::string("csr_upload: ") + hipGetErrorString(e));
    }
    *out = H;
    return SCOCG_OK;
}

// ------------------------------------------------------------------------------------------
// matrix-free extended Hubbard ring
// ------------------------------------------------------------------------------------------
namespace {

// One spin species on an L-site ring with n electrons: configurations (L-bit patterns with n
// bits set, ascending) and the hopping lists -t sum_i (c+_i c_i+1 + h.c.).  Signs follow the
// Jordan-Wigner order with all up-spin modes before all down-spin modes: a hop between
// neighbours i, i+1 passes no electron of its species, the ring-closing hop (L-1, 0) passes
// the other n - 1.  A hop entry is the target index, with bit 31 set when its value is +t.
struct Species {
    std::vector<uint32_t> conf;
    std::vector<int32_t> ptr;
    std::vector<uint32_t> hop;
};

Species build_species(int L, int n)
{
    Species sp;
    if (n == 0) {
        sp.conf.push_back(0);
    } else {
        // next L-bit pattern with the same number of bits set, in increasing order
        uint64_t c = (1ull << n) - 1;
        while (c < (1ull << L)) {
            sp.conf.push_back((uint32_t)c);
            const uint64_t lo = c & (~c + 1);
            const uint64_t r = c + lo;
            c = (((r ^ c) >> 2) / lo) | r;
        }
    }
    sp.ptr.push_back(0);
    std::vector<uint32_t> row;
    for (uint32_t c : sp.conf) {
        row.clear();
        for (int i = 0; i < L; ++i) {
            const int j = (i + 1) % L;
            if (((c >> i) & 1u) == ((c >> j) & 1u)) continue;
            const uint32_t nc = c ^ ((1u << i) | (1u << j));
            const int sign = (i == L - 1 && (n - 1) % 2 != 0) ? -1 : 1;
            const uint32_t k = (uint32_t)(std::lower_bound(sp.conf.begin(), sp.conf.end(), nc) - sp.conf.begin());
            // value -t * sign: +t exactly when sign = -1
            row.push_back(k | (sign < 0 ? 0x80000000u : 0u));
        }
        std::sort(row.begin(), row.end(), [](uint32_t a, uint32_t b) { return (a & 0x7fffffffu) < (b & 0x7fffffffu); });
        sp.hop.insert(sp.hop.end(), row.begin(), row.end());
        sp.ptr.push_back((int32_t)sp.hop.size());
    }
    return sp;
}

int popc32(uint32_t x) { return __builtin_popcount(x); }

}  // namespace

extern "C" int hubbard_upload(int32_t L, int32_t n_up, int32_t n_dn, double t, double U, double V, void *stream,
                              scocg_csr_t *out)
{
    g_err.clear();
    if (!out) return fail(SCOCG_EINVAL, "out is null");
    *out = nullptr;
    if (L < 3 || L > 30) return fail(SCOCG_EINVAL, "ring length must be in [3, 30]");
    if (n_up < 0 || n_up > L || n_dn < 0 || n_dn > L) return fail(SCOCG_EINVAL, "electron counts must be in [0, L]");
    if (!std::isfinite(t) || !std::isfinite(U) || !std::isfinite(V)) return fail(SCOCG_EINVAL, "non-finite parameter");
    const Species up = build_species(L, n_up), dn = build_species(L, n_dn);
    const int64_t Du = (int64_t)up.conf.size(), Dd = (int64_t)dn.conf.size();
    const int64_t n = Du * Dd;
    if (n >= (1LL << 31)) return fail(SCOCG_EINVAL, "sector dimension must be below 2^31");
    hipStream_t st = (hipStream_t)stream;
    scocg_csr *H = new scocg_csr();
    DevCSR &d = H->d;
    d.n = n;
    d.nnz = Dd * (int64_t)up.hop.size() + Du * (int64_t)dn.hop.size() + n;  // entries of the stored matrix
    d.nslices = (n + 63) / 64;
    int maxw = 0;
    for (int64_t a = 0; a < Du; ++a)
        for (int64_t b = 0; b < Dd; ++b)
            maxw = std::max<int>(maxw, up.ptr[a + 1] - up.ptr[a] + dn.ptr[b + 1] - dn.ptr[b] + 1);
    d.max_w = maxw;
    // trace in row order, as a sum over the stored diagonal would give
    double tr = 0;
    for (int64_t a = 0; a < Du; ++a) {
        const uint32_t cu = up.conf[a];
        for (int64_t b = 0; b < Dd; ++b) {
            const uint32_t cd = dn.conf[b];
            auto nxt = [&](uint32_t c) { return ((c >> 1) | ((c & 1u) << (L - 1))) & ((1u << L) - 1u); };
            const int on = popc32(cu & cd);
            const int inter = popc32(cu & nxt(cu)) + popc32(cd & nxt(cd)) + popc32(cu & nxt(cd)) + popc32(cd & nxt(cu));
            tr += U * (double)on + V * (double)inter;
        }
    }
    d.trace = tr;
    // one device block: up ptr, hop, conf, then the same for down
    auto bytes4 = [](size_t c) { return ((c * 4 + 255) / 256) * 256; };
    const size_t o_uptr = 0, o_uhop = o_uptr + bytes4(up.ptr.size()), o_ucf = o_uhop + bytes4(up.hop.size());
    const size_t o_dptr = o_ucf + bytes4(up.conf.size()), o_dhop = o_dptr + bytes4(dn.ptr.size());
    const size_t o_dcf = o_dhop + bytes4(dn.hop.size()), total = o_dcf + bytes4(dn.conf.size());
    std::vector<char> blob(total, 0);
    std::memcpy(blob.data() + o_uptr, up.ptr.data(), up.ptr.size() * 4);
    std::memcpy(blob.data() + o_uhop, up.hop.data(), up.hop.size() * 4);
    std::memcpy(blob.data() + o_ucf, up.conf.data(), up.conf.size() * 4);
    std::memcpy(blob.data() + o_dptr, dn.ptr.data(), dn.ptr.size() * 4);
    std::memcpy(blob.data() + o_dhop, dn.hop.data(), dn.hop.size() * 4);
    std::memcpy(blob.data() + o_dcf, dn.conf.data(), dn.conf.size() * 4);
    char *dev = nullptr;
    hipError_t e = upload(&dev, blob.data(), blob.size(), st);
    d.d_hub_tables = dev;
    HubbardOp h{};
    if (e == hipSuccess) {
        h.up_ptr = (const int32_t *)(dev + o_uptr);
        h.up_hop = (const uint32_t *)(dev + o_uhop);
        h.up_conf = (const uint32_t *)(dev + o_ucf);
        h.dn_ptr = (const int32_t *)(dev + o_dptr);
        h.dn_hop = (const uint32_t *)(dev + o_dhop);
        h.dn_conf = (const uint32_t *)(dev + o_dcf);
        h.Dd = Dd;
        d.hub_Dd = Dd;
        h.t = t;
        h.U = U;
        h.V = V;
        h.L = L;
        e = upload(&d.d_hub, &h, 1, st);
    }
    if (e != hipSuccess) {
        free_dev(d);
        delete H;
        return fail(e == hipErrorOutOfMemory ? SCOCG_ENOMEM : SCOCG_EHIP, std::string("hubbard_upload: ") +
                                                                              hipGetErrorString(e));
    }
    *out = H;
    return SCOCG_OK;
}

static bool matrix_free(const scocg_csr *H) { return H && H->d.d_hub; }

extern "C" int csr_update_values(scocg_csr_t H, const double *val, void *stream)
{
    g_err.clear();
    if (!H || !val) return fail(SCOCG_EINVAL, "null argument");
    if (matrix_free(H)) return fail(SCOCG_EINVAL, "a matrix-free operator has no stored values");
    hipStream_t st = (hipStream_t)stream;
    DevCSR &d = H->d;
    std::vector<double> eval(d.ell_nnz, 0.0);
    for (int64_t s = 0; s < d.ell_nnz; ++s)
        if (H->h_ell_src[s] >= 0) eval[s] = val[H->h_ell_src[s]];
    H->h_val.assign(val, val + d.nnz);
    double tr = 0;
    for (int64_t i = 0; i < d.n; ++i)
        for (int64_t k = H->h_row_ptr[i]; k < H->h_row_ptr[i + 1]; ++k)
            if (H->h_col[k] == i) tr += val[k];
    d.trace = tr;
    HIPCHK(hipMemcpyAsync(d.d_ell_val, eval.data(), eval.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.d_val, val, d.nnz * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return SCOCG_OK;
}

extern "C" int64_t csr_n(scocg_csr_t H) { return H ? H->d.n : -1; }
extern "C" int64_t csr_nnz(scocg_csr_t H) { return H ? H->d.nnz : -1; }

static void csr_release(scocg_csr *H)
{
    if (H->refs.fetch_sub(1) == 1) {
        free_dev(H->d);
        delete H;
    }
}

extern "C" void csr_free(scocg_csr_t H)
{
    if (!H) return;
    csr_release(H);
}

extern "C" void scocg_default_opts(scocg_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-8;
    o->max_iter = 3000;
    o->precision = 0;
    o->seed_index = -1;
    o->seed_switching = 1;
    o->fixed_iter = 0;
    o->block = 0;
    o->shifts_per_wg = 0;
    o->check_true = 0;
    o->keep_tape = 0;
}

extern "C" const char *scocg_last_error(void) { return g_err.c_str(); }

extern "C" int scocg_last_timing(scocg_timing *t)
{
    if (!t) return SCOCG_EINVAL;
    *t = g_timing;
    return SCOCG_OK;
}

extern "C" void scocg_set_profiling(int on) { g_profiling = on ? 1 : 0; }

extern "C" int32_t scocg_last_switches(int64_t rhs, int32_t *log, int32_t max_entries)
{
    if (rhs < 0 || rhs >= g_swlog.K) {
        g_err = "rhs out of range of the last solve";
        return -1;
    }
    const int32_t c = g_swlog.count[rhs];
    const int32_t stored = (int32_t)std::min<int64_t>(c, g_swlog.M);
    if (log)
        for (int32_t e = 0; e < std::min(stored, std::max(max_entries, 0)); ++e) {
            log[2 * e + 0] = g_swlog.log[2 * (rhs * g_swlog.M + e) + 0];
            log[2 * e + 1] = g_swlog.log[2 * (rhs * g_swlog.M + e) + 1];
        }
    return c;
}

// ------------------------------------------------------------------------------------------
// the solver driver
// ------------------------------------------------------------------------------------------
namespace {

// Initial seed: smallest Im z; ties by |Re z - Tr(H)/n|; then lowest index.
int default_seed(const double *z, int64_t M, double centre)
{
    int best = 0;
    for (int64_t k = 1; k < M; ++k) {
        const double ik = z[2 * k + 1], ib = z[2 * best + 1];
        const double dk = std::fabs(z[2 * k] - centre), db = std::fabs(z[2 * best] - centre);
        if (ik < ib || (ik == ib && dk < db)) best = (int)k;
    }
    return best;
}

struct SolveRequest {
    scocg_csr *H;                  // matrix of every rhs, unless Hj is given
    std::vector<scocg_csr *> Hj;   // matrix per rhs (a batch of uneven Hamiltonians), or empty
    int64_t M, K;
    const double *z;          // host [M] complex
    const double2 *B;         // device [K][n] or null (unit vectors)
    const int64_t *unit_idx;  // host [K] (unit vectors) or null
    scocg_opts o;
    double2 *Xout;            // device FP64 [K][M][n] or null
    bool projection;          // keep only x at row unit_idx[j]
    double2 *Gout;            // device [M][K] or null
    scocg_pair_report *rep;
    DevBuf *keepX;            // receives the full FP64 solutions (tape) or null
    bool zper;                // z has one shift per rhs (n_shift = 1): used by the refinement solves
    const double2 *wproj;     // device [K][n] projection weights (projection mode: G = <w|x>), or null
};

int solve(SolveRequest &rq, hipStream_t st)
{
    const int64_t K = rq.K, M = rq.M;
    if (M <= 0 || K <= 0) return fail(SCOCG_EINVAL, "n_shift and n_rhs must be positive");
    if (!rq.Hj.empty() && (int64_t)rq.Hj.size() != K) return fail(SCOCG_EINVAL, "one matrix per rhs expected");
    // per-rhs matrices and vector offsets
    std::vector<RhsDesc> hdesc(K);
    std::vector<double> centre(K);
    int64_t ntot = 0, n = 0;
    bool uniform = true;
    for (int64_t j = 0; j < K; ++j) {
        const DevCSR &d = (rq.Hj.empty() ? rq.H : rq.Hj[j])->d;
        hdesc[j] = RhsDesc{d.d_slice_ptr, d.d_slice_w, d.d_ell_col, d.d_ell_val, d.nslices, d.n, ntot, d.d_hub};
        centre[j] = d.trace / (double)d.n;
        ntot += d.n;
        n = std::max(n, d.n);
        if (!rq.Hj.empty() && rq.Hj[j] != rq.Hj[0]) uniform = false;
    }
    const scocg_opts &o = rq.o;
    if (M > (1 << 20) || K > 65535) return fail(SCOCG_EINVAL, "too many shifts or right-hand sides");
    if (!(o.tol > 0) && o.fixed_iter <= 0) return fail(SCOCG_EINVAL, "tol must be positive");
    if (o.max_iter <= 0 && o.fixed_iter <= 0) return fail(SCOCG_EINVAL, "max_iter must be positive");
    if (o.precision != 0 && o.precision != 1) return fail(SCOCG_EINVAL, "precision must be 0 or 1");
    if (rq.zper && M != 1) return fail(SCOCG_EINVAL, "one shift per rhs needs n_shift = 1");
    const int64_t nz = rq.zper ? K : M;
    for (int64_t k = 0; k < nz; ++k)
        if (!std::isfinite(rq.z[2 * k]) || !std::isfinite(rq.z[2 * k + 1]))
            return fail(SCOCG_EINVAL, "non-finite shift");
    // 48 iterations per deferred update: x_k, u_k are read and written once per block, so
    // the update's bytes per iteration fall as 1/T; at T = 48 its arithmetic (8 fused
    // multiply-adds per step) still fits under the memory time of an FP64 pair, and the
    // residual history (T * 1 KiB per 64-row tile in LDS) leaves three workgroups per CU
    int TB = o.block > 0 ? o.block : 48;
    if (TB != 1 && TB != 2 && TB != 4 && TB != 8 && TB != 16 && TB != 24 && TB != 32 && TB != 40 && TB != 48)
        return fail(SCOCG_EINVAL, "block must be 1, 2, 4, 8, 16, 24, 32, 40 or 48");
    if (o.shifts_per_wg > 64) return fail(SCOCG_EINVAL, "shifts_per_wg must be at most 64");
    // shifts per workgroup of the update: the long-block form deals up to 64 out to its eight
    // waves; the short-block form runs 32 per workgroup (more workgroups for few rhs)
    int G = o.shifts_per_wg > 0 ? o.shifts_per_wg : (int)std::min<int64_t>(M, TB >= 24 ? 64 : 32);
    std::vector<int32_t> seeds(K, 0);
    for (int64_t j = 0; j < K; ++j) {
        if (rq.zper) {
            seeds[j] = (int32_t)j;
        } else if (o.seed_index >= 0) {
            if (o.seed_index >= M) return fail(SCOCG_EINVAL, "seed_index out of range");
            seeds[j] = o.seed_index;
        } else {
            seeds[j] = default_seed(rq.z, M, centre[j]);
        }
    }
    if (o.refine > 0 && !uniform) return fail(SCOCG_EINVAL, "refinement needs a single matrix");
    const bool fixed = o.fixed_iter > 0;
    const int32_t limit = fixed ? o.fixed_iter : o.max_iter;
    const bool need_full = !rq.projection;
    if (o.window < 0) return fail(SCOCG_EINVAL, "window must be >= 0");
    if (o.window > 0 && need_full) return fail(SCOCG_EINVAL, "window needs projection mode (greens_diag without tape)");
    if (rq.wproj && (need_full || !rq.B || !rq.Hj.empty()))
        return fail(SCOCG_EINVAL, "a vector projection needs projection mode, dense right-hand sides and one matrix");
    // window of seed candidates: the only shifts whose full directions are stored
    const int64_t Mst = (o.window > 0 && o.window < M) ? o.window : M;
    std::vector<int32_t> h_wshift, h_wslot;
    if (Mst < M) {
        h_wshift.resize((size_t)K * Mst);
        h_wslot.assign((size_t)K * M, -1);
        std::vector<int32_t> order(M);
        for (int64_t j = 0; j < K; ++j) {
            // the seed first, then the seed rule's order: smallest Im z, Re z nearest Tr(H)/n, index
            for (int64_t k = 0; k < M; ++k) order[k] = (int32_t)k;
            const double c = centre[j];
            const int32_t sd = seeds[j];
            std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
                if ((a == sd) != (b == sd)) return a == sd;
                const double ia = rq.z[2 * a + 1], ib = rq.z[2 * b + 1];
                if (ia != ib) return ia < ib;
                const double da = std::fabs(rq.z[2 * a] - c), db = std::fabs(rq.z[2 * b] - c);
                if (da != db) return da < db;
                return a < b;
            });
            for (int64_t w = 0; w < Mst; ++w) {
                h_wshift[j * Mst + w] = order[w];
                h_wslot[j * M + order[w]] = (int32_t)w;
            }
        }
    }
    const size_t KM = (size_t)K * M;
    const size_t vec = (size_t)ntot;
    const size_t esz = o.precision == 0 ? sizeof(double2) : sizeof(float2);

    g_timing = scocg_timing{};
    g_swlog.K = 0;
    TimerEvents tev;
    HIPCHK(tev.create());
    hipEvent_t ev_t0 = tev.t0, ev_t1 = tev.t1;
    HIPCHK(hipEventRecord(ev_t0, st));

    SolveDev s{};
    s.ntot = ntot;
    s.n = n;
    s.K = K;
    s.M = M;
    s.TB = TB;
    s.precision = o.precision;
    s.fixed = fixed ? 1 : 0;
    s.switching = o.seed_switching ? 1 : 0;
    s.tol = o.tol;
    s.nblk = (n + 255) / 256;
    s.shifts_per_wg = G;
    s.zper = rq.zper ? 1 : 0;
    // two right-hand sides per SpMV thread when every pair (2i, 2i+1) shares its matrix (their
    // vectors are then adjacent, which the interleaved direction layout needs)
    bool pairable = K >= 2;
    for (int64_t j = 0; j + 1 < K && pairable && !rq.Hj.empty(); j += 2) pairable = rq.Hj[j] == rq.Hj[j + 1];
    s.spmv_rb = pairable ? 2 : 1;
    for (int64_t j = 0; j < K; ++j) (hdesc[j].hub ? s.has_hub : s.has_sell) = 1;
    for (int64_t j = 0; j < K; ++j) (hdesc[j].n >= RED_BIG_ROWS ? s.has_red_big : s.has_red_small) = 1;
    s.hub_lds = 1;
    for (int64_t j = 0; j < K; ++j) {
        const DevCSR &dj = (rq.Hj.empty() ? rq.H : rq.Hj[j])->d;
        if (!dj.d_hub) continue;
        // one partial per up-spin configuration must fit the rhs's own partial slots (one per
        // 256 rows; the seed reductions read no more)
        if (dj.hub_Dd > HUB_LDS_MAX || dj.n / dj.hub_Dd > (dj.n + 255) / 256) s.hub_lds = 0;
        s.hub_du_max = std::max<int64_t>(s.hub_du_max, dj.n / dj.hub_Dd);
    }
    // Work lists for a batch of right-hand sides with different row counts: each per-iteration
    // launch (p update, SpMV, residual update) and the deferred update then covers exactly the
    // row blocks that exist, not the rectangle of the largest row count times every rhs.  The
    // items are in the order the rectangle would visit them, so every kernel does the same work
    // per item and the results are the same bits.
    std::vector<int2> h_items;
    int64_t n_grp = 0, n_rhs_items = 0, n_upd = 0;
    bool uneven = false;
    for (int64_t j = 0; j < K; ++j) uneven = uneven || hdesc[j].n != n;
    if (uneven) {
        auto blocks = [&](int64_t j, int64_t rows_per) { return (hdesc[j].n + rows_per - 1) / rows_per; };
        const int RB = s.spmv_rb;
        const int64_t Gn = (K + RB - 1) / RB;
        if (Gn < 8) {
            for (int64_t g = 0; g < Gn; ++g)
                for (int64_t t = 0; t < blocks(g * RB, 256); ++t) h_items.push_back(make_int2((int)g, (int)t));
        } else {
            // sets of 8 groups, item 8 t + x of a set on XCD x (the round-robin of workgroups over
            // the 8 XCDs keeps one group's vectors in one L2); a group shorter than its set's longest
            // leaves fillers (-1) that exit at once
            for (int64_t s8 = 0; s8 < (Gn + 7) / 8; ++s8) {
                int64_t nb = 0;
                for (int64_t x = 0; x < 8 && 8 * s8 + x < Gn; ++x) nb = std::max(nb, blocks((8 * s8 + x) * RB, 256));
                for (int64_t t = 0; t < nb; ++t)
                    for (int64_t x = 0; x < 8; ++x) {
                        const int64_t g = 8 * s8 + x;
                        const bool has = g < Gn && t < blocks(g * RB, 256);
                        h_items.push_back(make_int2(has ? (int)g : -1, (int)t));
                    }
            }
        }
        n_grp = (int64_t)h_items.size();
        for (int64_t j = 0; j < K; ++j)
            for (int64_t t = 0; t < blocks(j, 256); ++t) h_items.push_back(make_int2((int)j, (int)t));
        n_rhs_items = (int64_t)h_items.size() - n_grp;
        const int64_t tile = TB >= 24 ? 64 : 256;  // rows per workgroup of the update kernel
        const int64_t ngr = (Mst + G - 1) / G;
        for (int64_t y = 0; y < K * ngr; ++y)
            for (int64_t t = 0; t < blocks(y / ngr, tile); ++t) h_items.push_back(make_int2((int)y, (int)t));
        n_upd = (int64_t)h_items.size() - n_grp - n_rhs_items;
        if ((int64_t)h_items.size() >= (1LL << 31)) return fail(SCOCG_EINVAL, "batch too large for its work lists");
    }

    DevBuf bz, bseed, bring, bp, bq, bX, bP, bXproj, bprow, bpi, bpip, bbk, bres, biters, bpst, bact, bnact, bah, bbh,
        brn, bcoef, bp2, bp1, bcnt, bidx, bsd, bstats, bdesc, bwshift, bwslot, bUproj, bblk;
    auto A = [&](DevBuf &b, size_t bytes) -> hipError_t { return b.alloc(bytes); };
    hipError_t e = hipSuccess;
#define ALLOC(buf, bytes)                                                                                  \
    do {                                                                                                   \
        e = A(buf, bytes);                                                                                 \
        if (e != hipSuccess)                                                                               \
            return fail(SCOCG_ENOMEM, std::string("device allocation of ") + std::to_string((size_t)(bytes)) + \
                                          " bytes failed: " + hipGetErrorString(e));                      \
    } while (0)
    ALLOC(bz, nz * sizeof(double2));
    ALLOC(bseed, K * sizeof(SeedState));
    const int R = 2 * TB + 1;  // ring slots: one block's update overlaps the next block's iterations
    ALLOC(bring, (size_t)R * vec * sizeof(double2));
    ALLOC(bp, 2 * vec * sizeof(double2));
    ALLOC(bq, vec * sizeof(double2));
    ALLOC(bP, (size_t)Mst * ntot * esz);
    if (Mst < M) {
        ALLOC(bwshift, (size_t)K * Mst * sizeof(int32_t));
        ALLOC(bwslot, KM * sizeof(int32_t));
    }
    if (Mst < M || rq.wproj) ALLOC(bUproj, KM * sizeof(double2));
    DevBuf bshist, bpart3;
    if (rq.wproj) {
        ALLOC(bshist, (size_t)K * TB * sizeof(double2));
        ALLOC(bpart3, (size_t)K * s.nblk * sizeof(double2));
    }
    const bool x_is_out = need_full && o.precision == 0 && rq.Xout && !rq.keepX;
    if (need_full && !x_is_out) ALLOC(bX, (size_t)M * ntot * esz);
    ALLOC(bdesc, K * sizeof(RhsDesc));
    if (!need_full) {
        ALLOC(bXproj, KM * sizeof(double2));
        ALLOC(bprow, K * sizeof(int64_t));
    }
    ALLOC(bpi, KM * sizeof(double2));
    ALLOC(bpip, KM * sizeof(double2));
    ALLOC(bbk, KM * sizeof(double2));
    ALLOC(bres, KM * sizeof(double));
    ALLOC(biters, KM * sizeof(int32_t));
    ALLOC(bpst, KM * sizeof(int32_t));
    ALLOC(bact, KM * sizeof(int32_t));
    ALLOC(bnact, 2 * KM * sizeof(int32_t));
    ALLOC(bblk, 2 * (size_t)K * 4 * sizeof(int32_t));
    ALLOC(bah, K * TB * sizeof(double2));
    ALLOC(bbh, K * TB * sizeof(double2));
    ALLOC(brn, K * TB * sizeof(double));
    const size_t coef_bytes = KM * TB * 2 * (o.precision == 0 ? sizeof(double2) : sizeof(float2));
    ALLOC(bcoef, 2 * coef_bytes);
    // the expanded update form (FP64 matrix cores) for FP64 full solutions in blocks of 24 and more
    if (o.update_form < 0 || o.update_form > 2) return fail(SCOCG_EINVAL, "update_form must be 0, 1 or 2");
    const bool can_expand = o.precision == 0 && need_full && Mst == M && TB >= 24;
    if (o.update_form == 2 && !can_expand)
        return fail(SCOCG_EINVAL, "the expanded update form needs FP64 storage, full solutions and blocks of 24 or more");
    // automatic: the step form, which is faster on gfx950 (the FP64 matrix cores have the vector
    // units' peak, and the expanded form's per-lane weight loads and 16-pair granularity cost more
    // than the step form's latency; measured 22.3 against 14.0 ms per diamond launch alone)
    s.expanded = (o.update_form == 2) ? 1 : 0;
    const size_t coefx_bytes = s.expanded ? KM * (size_t)(6 * TB + 4) * sizeof(double) : 0;
    DevBuf bcoefx;
    if (s.expanded) ALLOC(bcoefx, 2 * coefx_bytes);
    ALLOC(bp2, K * s.nblk * sizeof(double2));
    ALLOC(bp1, K * s.nblk * sizeof(double));
    ALLOC(bcnt, K * sizeof(uint32_t));
    ALLOC(bsd, K * sizeof(int32_t));
    ALLOC(bstats, 3 * sizeof(unsigned long long));
    DevBuf bswlog;
    ALLOC(bswlog, KM * 2 * sizeof(int32_t));
    if (rq.unit_idx) ALLOC(bidx, K * sizeof(int64_t));

    s.z = bz.as<double2>();
    s.seed = bseed.as<SeedState>();
    s.ring = bring.as<double2>();
    s.R = R;
    s.blk = bblk.as<int32_t>();
    s.p = bp.as<double2>();
    s.q = bq.as<double2>();
    s.P = bP.ptr;
    s.Mst = Mst;
    s.wshift = Mst < M ? bwshift.as<int32_t>() : nullptr;
    s.wslot = Mst < M ? bwslot.as<int32_t>() : nullptr;
    s.Uproj = (Mst < M || rq.wproj) ? bUproj.as<double2>() : nullptr;
    s.wproj = rq.wproj;
    s.shist = rq.wproj ? bshist.as<double2>() : nullptr;
    s.part3 = rq.wproj ? bpart3.as<double2>() : nullptr;
    s.X = need_full ? (x_is_out ? (void *)rq.Xout : bX.ptr) : nullptr;
    s.Xproj = need_full ? nullptr : bXproj.as<double2>();
    s.proj_row = need_full ? nullptr : bprow.as<int64_t>();
    s.pi = bpi.as<double2>();
    s.pi_prev = bpip.as<double2>();
    s.beta_k = bbk.as<double2>();
    s.res = bres.as<double>();
    s.iters = biters.as<int32_t>();
    s.pstatus = bpst.as<int32_t>();
    s.active = bact.as<int32_t>();
    s.nact = bnact.as<int32_t>();
    s.ahist = bah.as<double2>();
    s.bhist = bbh.as<double2>();
    s.rnhist = brn.as<double>();
    s.coef = bcoef.ptr;
    s.part2 = bp2.as<double2>();
    s.part1 = bp1.as<double>();
    s.cnt = bcnt.as<uint32_t>();
    s.stats = bstats.as<unsigned long long>();
    s.swlog = bswlog.as<int32_t>();
    s.desc = bdesc.as<RhsDesc>();
    DevBuf bitems;
    if (uneven) {
        ALLOC(bitems, h_items.size() * sizeof(int2));
        HIPCHK(hipMemcpyAsync(bitems.ptr, h_items.data(), h_items.size() * sizeof(int2), hipMemcpyHostToDevice, st));
        s.it_grp = bitems.as<int2>();
        s.n_it_grp = n_grp;
        s.it_rhs = bitems.as<int2>() + n_grp;
        s.n_it_rhs = n_rhs_items;
        s.it_upd = bitems.as<int2>() + n_grp + n_rhs_items;
        s.n_it_upd = n_upd;
    }

    HIPCHK(hipMemcpyAsync(bdesc.ptr, hdesc.data(), K * sizeof(RhsDesc), hipMemcpyHostToDevice, st));
    if (Mst < M) {
        HIPCHK(hipMemcpyAsync(bwshift.ptr, h_wshift.data(), h_wshift.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                              st));
        HIPCHK(hipMemcpyAsync(bwslot.ptr, h_wslot.data(), h_wslot.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipMemcpyAsync(bz.ptr, rq.z, nz * sizeof(double2), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bsd.ptr, seeds.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (rq.unit_idx) {
        HIPCHK(hipMemcpyAsync(bidx.ptr, rq.unit_idx, K * sizeof(int64_t), hipMemcpyHostToDevice, st));
        if (!need_full) HIPCHK(hipMemcpyAsync(bprow.ptr, rq.unit_idx, K * sizeof(int64_t), hipMemcpyHostToDevice, st));
    }
    std::vector<int64_t> no_row;
    if (rq.wproj) {
        // no kept row: every pair's projection is carried by scalars
        no_row.assign(K, -1);
        HIPCHK(hipMemcpyAsync(bprow.ptr, no_row.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, st));
    }
    HIPCHK(launch_zero(bcnt.ptr, K * sizeof(uint32_t), st));
    HIPCHK(launch_zero(bnact.ptr, 2 * KM * sizeof(int32_t), st));
    HIPCHK(launch_zero(bblk.ptr, 2 * (size_t)K * 4 * sizeof(int32_t), st));
    HIPCHK(launch_zero(bstats.ptr, 3 * sizeof(unsigned long long), st));
    HIPCHK(launch_zero(bswlog.ptr, KM * 2 * sizeof(int32_t), st));
    if (need_full) HIPCHK(launch_zero(s.X, (size_t)M * ntot * esz, st));
    HIPCHK(launch_zero(s.p, 2 * vec * sizeof(double2), st));
    HIPCHK(launch_init(s, rq.B, rq.unit_idx ? bidx.as<int64_t>() : nullptr, bsd.as<int32_t>(), limit, st));

    PinnedBuf host_state;
    HIPCHK(host_state.alloc(K * sizeof(SeedState)));
    SeedState *hs = (SeedState *)host_state.ptr;

    std::vector<hipEvent_t> evs;
    struct EvList {
        std::vector<hipEvent_t> *v;
        ~EvList()
        {
            for (auto e : *v) (void)hipEventDestroy(e);
        }
    } evl{&evs};
    auto new_event = [&](hipEvent_t &e, unsigned flags) -> hipError_t {
        hipError_t r = hipEventCreateWithFlags(&e, flags);
        if (r == hipSuccess) evs.push_back(e);
        return r;
    };

    // The deferred update of block c runs on its own stream, overlapping the seed iterations of
    // block c + 1 (which write other ring slots and the other parity's coefficient buffers);
    // block c + 2 waits for it.  A seed switch decided at the end of block c waits out block
    // c + 1 and is applied at the start of block c + 2, after the update of block c.
    struct FlushStream {
        hipStream_t sf = nullptr;
        bool own = false;
        ~FlushStream()
        {
            if (own && sf) {
                (void)hipStreamSynchronize(sf);
                (void)hipStreamDestroy(sf);
            }
        }
    } fs;
    if (o.schedule < 0 || o.schedule > 2) return fail(SCOCG_EINVAL, "schedule must be 0, 1 or 2");
    const bool overlap = o.schedule == 2 || (o.schedule == 0 && (double)Mst * (double)ntot >= 16777216.0);
    if (!overlap) {
        fs.sf = st;
    } else {
        HIPCHK(hipStreamCreateWithFlags(&fs.sf, hipStreamNonBlocking));
        fs.own = true;
    }
    const hipStream_t sf = fs.sf;
    hipEvent_t evPS[2], evFL[2];
    for (int q = 0; q < 2; ++q) {
        HIPCHK(new_event(evPS[q], hipEventDisableTiming));
        HIPCHK(new_event(evFL[q], hipEventDisableTiming));
    }
    // per-parity views of the double-buffered per-block arrays
    SolveDev sp[2] = {s, s};
    for (int q = 0; q < 2; ++q) {
        sp[q].coef = (char *)bcoef.ptr + q * coef_bytes;
        sp[q].coefx = s.expanded ? (double *)((char *)bcoefx.ptr + q * coefx_bytes) : nullptr;
        sp[q].nact = bnact.as<int32_t>() + q * KM;
        sp[q].blk = bblk.as<int32_t>() + q * (size_t)K * 4;
    }
    // update-kernel timing: a ring of event pairs on the update stream, read back lazily
    constexpr int NE = 8;
    hipEvent_t fev[2 * NE] = {};
    bool fev_pending[NE] = {};
    if (g_profiling)
        for (int q = 0; q < 2 * NE; ++q) HIPCHK(new_event(fev[q], hipEventDefault));
    auto collect = [&](int slot) -> hipError_t {
        if (!fev_pending[slot]) return hipSuccess;
        hipError_t r = hipEventSynchronize(fev[2 * slot + 1]);
        if (r != hipSuccess) return r;
        float ms = 0;
        r = hipEventElapsedTime(&ms, fev[2 * slot], fev[2 * slot + 1]);
        if (r != hipSuccess) return r;
        g_timing.update_ms += ms;
        g_timing.update_launches += 1;
        fev_pending[slot] = false;
        return hipSuccess;
    };

    // Each block: the captured switch application, seed iterations and shift scalars (graph
    // A, one per parity) on `st`; the deferred update on the update stream; the captured
    // end-of-block decisions (graph B) on `st`.  Graphs are captured on a private stream.
    GraphPair gr;
    const bool use_graph = !o.no_graph;
    if (use_graph) {
        HIPCHK(hipStreamCreateWithFlags(&gr.cap, hipStreamNonBlocking));
        for (int q = 0; q < 2; ++q) {
            HIPCHK(hipStreamBeginCapture(gr.cap, hipStreamCaptureModeThreadLocal));
            HIPCHK(launch_switch_vectors(sp[q], gr.cap));
            for (int t = 0; t < TB; ++t) HIPCHK(launch_seed_iteration(sp[q], gr.cap));
            HIPCHK(launch_pair_scalars(sp[q], gr.cap));
            HIPCHK(hipStreamEndCapture(gr.cap, &gr.ga[q]));
            HIPCHK(hipGraphInstantiate(&gr.ea[q], gr.ga[q], nullptr, nullptr, 0));
        }
        HIPCHK(hipStreamBeginCapture(gr.cap, hipStreamCaptureModeThreadLocal));
        HIPCHK(launch_block_finalize(sp[0], gr.cap));
        HIPCHK(hipStreamEndCapture(gr.cap, &gr.gb));
        HIPCHK(hipGraphInstantiate(&gr.eb, gr.gb, nullptr, nullptr, 0));
    }
    // host checks the stop condition every `per_sync` blocks (about 64 iterations); blocks
    // launched after every rhs has stopped return immediately
    const int per_sync = std::max(1, 64 / TB);
    // worst case: every block advances one rhs by >= 1 iteration, or finishes, switches or
    // waits out a switch for one rhs
    const int64_t max_blocks = (int64_t)K * ((int64_t)limit + 4 * M + 8) + 8 + per_sync;
    int64_t blocks = 0;
    bool done = false;
    while (!done) {
        for (int b = 0; b < per_sync; ++b) {
            const int par = (int)(blocks & 1);
            if (blocks >= 2) HIPCHK(hipStreamWaitEvent(st, evFL[par], 0));
            if (use_graph) {
                HIPCHK(hipGraphLaunch(gr.ea[par], st));
            } else {
                HIPCHK(launch_switch_vectors(sp[par], st));
                for (int t = 0; t < TB; ++t) HIPCHK(launch_seed_iteration(sp[par], st));
                HIPCHK(launch_pair_scalars(sp[par], st));
            }
            HIPCHK(hipEventRecord(evPS[par], st));
            HIPCHK(hipStreamWaitEvent(sf, evPS[par], 0));
            const int slot = (int)(blocks % NE);
            if (g_profiling) {
                HIPCHK(collect(slot));
                HIPCHK(hipEventRecord(fev[2 * slot], sf));
            }
            HIPCHK(launch_flush(sp[par], sf));
            if (g_profiling) {
                HIPCHK(hipEventRecord(fev[2 * slot + 1], sf));
                fev_pending[slot] = true;
            }
            HIPCHK(hipEventRecord(evFL[par], sf));
            if (use_graph) HIPCHK(hipGraphLaunch(gr.eb, st));
            else HIPCHK(launch_block_finalize(sp[par], st));
            ++blocks;
        }
        HIPCHK(hipMemcpyAsync(hs, s.seed, K * sizeof(SeedState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        done = true;
        for (int64_t j = 0; j < K; ++j)
            if (hs[j].status != SEED_STOPPED) done = false;
        if (blocks > max_blocks) return fail(SCOCG_EHIP, "iteration driver did not terminate");
    }
    HIPCHK(hipStreamSynchronize(sf));
    if (g_profiling)
        for (int q = 0; q < NE; ++q) HIPCHK(collect(q));
    int64_t iters_total = 0, switches = 0;
    for (int64_t j = 0; j < K; ++j) {
        iters_total += hs[j].iter;
        switches += hs[j].switches;
    }

    // outputs
    if (need_full && rq.Xout && !x_is_out) {
        if (o.precision == 1) HIPCHK(launch_store_solution(s, rq.Xout, st));
        else HIPCHK(hipMemcpyAsync(rq.Xout, s.X, (size_t)M * ntot * sizeof(double2), hipMemcpyDeviceToDevice, st));
    }
    if (rq.keepX) {
        HIPCHK(rq.keepX->alloc((size_t)M * ntot * sizeof(double2)) == hipSuccess ? hipSuccess : hipErrorOutOfMemory);
        if (o.precision == 1) HIPCHK(launch_store_solution(s, rq.keepX->as<double2>(), st));
        else HIPCHK(hipMemcpyAsync(rq.keepX->ptr, s.X, (size_t)M * ntot * sizeof(double2), hipMemcpyDeviceToDevice, st));
    }
    if (rq.Gout) {
        // gather from full FP64 storage (or the projection)
        SolveDev g = s;
        if (need_full) {
            if (o.precision == 0) g.X = s.X;
            else if (rq.keepX) g.X = rq.keepX->ptr;
            else return fail(SCOCG_EINVAL, "FP32 greens_diag needs projection mode");
        }
        HIPCHK(launch_gather_diag(g, rq.unit_idx ? bidx.as<int64_t>() : nullptr, rq.Gout, st));
    }
    HIPCHK(hipEventRecord(ev_t1, st));

    // report
    std::vector<int32_t> h_it(KM), h_st(KM);
    std::vector<double> h_res(KM), h_true(KM, -1.0);
    HIPCHK(hipMemcpyAsync(h_it.data(), s.iters, KM * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_st.data(), s.pstatus, KM * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_res.data(), s.res, KM * sizeof(double), hipMemcpyDeviceToHost, st));
    unsigned long long h_stats[3] = {0, 0, 0};
    HIPCHK(hipMemcpyAsync(h_stats, s.stats, sizeof(h_stats), hipMemcpyDeviceToHost, st));
    g_swlog.K = K;
    g_swlog.M = M;
    g_swlog.count.resize(K);
    g_swlog.log.resize(KM * 2);
    HIPCHK(hipMemcpyAsync(g_swlog.log.data(), s.swlog, KM * 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int64_t j = 0; j < K; ++j) g_swlog.count[j] = hs[j].switches;
    g_timing.update_bytes = (double)h_stats[0];
    g_timing.update_flops = (double)h_stats[2];
    float tot_ms = 0;
    HIPCHK(hipEventElapsedTime(&tot_ms, ev_t0, ev_t1));
    g_timing.total_ms = tot_ms;
    g_timing.iterations = iters_total;
    g_timing.blocks = blocks;
    g_timing.switches = switches;

    // FP64 true residuals (Sec. 3.4 eq. residual) and, on request, refinement of the pairs whose
    // true residual misses the tolerance: (z_k - H) d = r_true solved per pair (one shift per
    // right-hand side, FP64 storage), x <- x + d.
    double2 *X64 = nullptr;
    if (need_full) {
        if (o.precision == 0) X64 = (double2 *)s.X;
        else if (rq.Xout) X64 = rq.Xout;
        else if (rq.keepX) X64 = rq.keepX->as<double2>();
    }
    if ((o.check_true || o.refine > 0) && X64) {
        const scocg_timing saved = g_timing;
        const SwitchLog saved_log = g_swlog;
        const int64_t gx = s.nblk;
        const int64_t *uidx = rq.unit_idx ? bidx.as<int64_t>() : nullptr;
        std::vector<double> h_nb(K);
        for (int64_t j = 0; j < K; ++j) h_nb[j] = hs[j].nb;
        DevBuf bnb, part, outr;
        ALLOC(bnb, K * sizeof(double));
        ALLOC(part, KM * gx * sizeof(double));
        ALLOC(outr, KM * sizeof(double));
        HIPCHK(hipMemcpyAsync(bnb.ptr, h_nb.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(launch_residual(s, rq.B,uidx, X64, nullptr, (int64_t)KM, bnb.as<double>(), nullptr,
                               part.as<double>(), outr.as<double>(), st));
        HIPCHK(hipMemcpyAsync(h_true.data(), outr.ptr, KM * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const int64_t chunk = 1024;
        for (int sweep = 0; sweep < o.refine; ++sweep) {
            std::vector<int64_t> fail_pairs;
            for (size_t p = 0; p < KM; ++p)
                if (h_true[p] > o.tol && h_st[p] != PAIR_BREAKDOWN) fail_pairs.push_back((int64_t)p);
            if (fail_pairs.empty()) break;
            for (size_t c0 = 0; c0 < fail_pairs.size(); c0 += chunk) {
                const int64_t cnt = std::min<int64_t>(chunk, (int64_t)(fail_pairs.size() - c0));
                std::vector<double2> zc(cnt);
                double tol_c = 0.5;
                for (int64_t c = 0; c < cnt; ++c) {
                    const int64_t p = fail_pairs[c0 + c];
                    const int64_t k = rq.zper ? p / M : p % M;
                    zc[c] = make_double2(rq.z[2 * k], rq.z[2 * k + 1]);
                    tol_c = std::min(tol_c, 0.5 * o.tol / h_true[p]);
                }
                DevBuf bl, R, D, pc, oc;
                ALLOC(bl, cnt * sizeof(int64_t));
                ALLOC(R, cnt * n * sizeof(double2));
                ALLOC(D, cnt * n * sizeof(double2));
                ALLOC(pc, cnt * gx * sizeof(double));
                ALLOC(oc, cnt * sizeof(double));
                HIPCHK(hipMemcpyAsync(bl.ptr, fail_pairs.data() + c0, cnt * sizeof(int64_t), hipMemcpyHostToDevice, st));
                HIPCHK(launch_residual(s, rq.B,uidx, X64, bl.as<int64_t>(), cnt, bnb.as<double>(),
                                       R.as<double2>(), pc.as<double>(), oc.as<double>(), st));
                HIPCHK(hipStreamSynchronize(st));
                SolveRequest cr{};
                cr.H = rq.Hj.empty() ? rq.H : rq.Hj[0];
                cr.M = 1;
                cr.K = cnt;
                cr.z = (const double *)zc.data();
                cr.B = R.as<double2>();
                cr.o = o;
                cr.o.tol = tol_c;
                cr.o.precision = 0;
                cr.o.fixed_iter = 0;
                cr.o.seed_index = -1;
                cr.o.seed_switching = 0;
                cr.o.check_true = 0;
                cr.o.refine = 0;
                cr.o.keep_tape = 0;
                cr.Xout = D.as<double2>();
                cr.zper = true;
                const int rc2 = solve(cr, st);
                if (rc2 != SCOCG_OK && rc2 != SCOCG_ENOCONV) return rc2;
                HIPCHK(launch_add_correction(n, bl.as<int64_t>(), cnt, D.as<double2>(), X64, st));
            }
            HIPCHK(launch_residual(s, rq.B,uidx, X64, nullptr, (int64_t)KM, bnb.as<double>(),
                                   nullptr, part.as<double>(), outr.as<double>(), st));
            HIPCHK(hipMemcpyAsync(h_true.data(), outr.ptr, KM * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        if (o.refine > 0 && rq.keepX && rq.Xout && X64 == rq.Xout)
            HIPCHK(hipMemcpyAsync(rq.keepX->ptr, rq.Xout, (size_t)M * ntot * sizeof(double2), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        g_timing = saved;
        g_swlog = saved_log;
    }
    int rc = SCOCG_OK;
    for (size_t p = 0; p < KM; ++p) {
        if (h_st[p] == PAIR_BREAKDOWN) rc = SCOCG_EBREAKDOWN;
        else if (h_st[p] == PAIR_NOCONV && !fixed && rc == SCOCG_OK) rc = SCOCG_ENOCONV;
    }
    if (rq.rep) {
        for (size_t p = 0; p < KM; ++p) {
            rq.rep[p].iters = h_it[p];
            rq.rep[p].status = (fixed && h_st[p] == PAIR_NOCONV) ? SCOCG_OK : h_st[p];
            rq.rep[p].rel_res_recursive = h_res[p];
            rq.rep[p].rel_res_true = h_true[p];
        }
    }
    if (rc == SCOCG_EBREAKDOWN) g_err = "COCG breakdown on at least one pair";
    else if (rc == SCOCG_ENOCONV) g_err = "at least one pair did not converge";
    return rc;
#undef ALLOC
}

}  // namespace

extern "C" int shifted_cocg_solve(scocg_csr_t H, int64_t n_shift, const double *z, int64_t n_rhs, const double *B,
                                  const scocg_opts *o, double *X, scocg_pair_report *rep, scocg_tape_t *tape,
                                  void *stream)
{
    g_err.clear();
    if (!H || !z || !B || !o) return fail(SCOCG_EINVAL, "null argument");
    REQUIRE_DEVICE((const void *)B, (const void *)X);
    const bool want_tape = tape && o->keep_tape;
    if (!X && !want_tape) return fail(SCOCG_EINVAL, "X is null and no tape was requested");
    SolveRequest rq{};
    rq.H = H;
    rq.M = n_shift;
    rq.K = n_rhs;
    rq.z = z;
    rq.B = (const double2 *)B;
    rq.o = *o;
    rq.Xout = (double2 *)X;
    rq.projection = false;
    rq.rep = rep;
    scocg_tape *tp = nullptr;
    if (want_tape) {
        tp = new scocg_tape();
        rq.keepX = &tp->X;
    }
    int rc = solve(rq, (hipStream_t)stream);
    if (tp) {
        if (rc == SCOCG_OK || rc == SCOCG_ENOCONV) {
            H->refs.fetch_add(1);
            tp->H = H;
            tp->K = n_rhs;
            tp->M = n_shift;
            tp->n = H->d.n;
            *tape = tp;
        } else {
            delete tp;
        }
    }
    return rc;
}

// Krylov-subspace diagonalization (Sec. 3.2): the recurrence for all right-hand sides at once
// (groups of LZ_RB interleaved), then the subspace Green's functions.
extern "C" int krylov_greens_diag(scocg_csr_t H, int64_t n_shift, const double *z, int64_t n_rhs,
                                  const int64_t *rhs_idx, int32_t nu, double *G, double *ab, int32_t *dim,
                                  void *stream)
{
    g_err.clear();
    if (!H || !z || !rhs_idx || !G) return fail(SCOCG_EINVAL, "null argument");
    REQUIRE_DEVICE((const void *)G, (const void *)ab);
    const int64_t n = H->d.n;
    if (n_shift < 1 || n_rhs < 1) return fail(SCOCG_EINVAL, "n_shift and n_rhs must be positive");
    // finite-precision recurrences run past n (the basis loses orthogonality); the limit keeps
    // the coefficient arrays modest
    if (nu < 1 || nu > (1 << 20)) return fail(SCOCG_EINVAL, "nu must be in [1, 2^20]");
    for (int64_t c = 0; c < n_rhs; ++c)
        if (rhs_idx[c] < 0 || rhs_idx[c] >= n) return fail(SCOCG_EINVAL, "rhs_idx out of range");
    for (int64_t k = 0; k < 2 * n_shift; ++k)
        if (!std::isfinite(z[k])) return fail(SCOCG_EINVAL, "non-finite shift");
    hipStream_t st = (hipStream_t)stream;
    g_timing = scocg_timing{};
    const int64_t Kp = (n_rhs + LZ_RB - 1) / LZ_RB * LZ_RB;  // padded with finished entries
    const int64_t nblk = (n + LZ_TILE - 1) / LZ_TILE;
    DevBuf bV0, bV1, bW0, bW1, bpart, bab, bst, bz;
    hipError_t e = hipSuccess;
    auto A = [&](DevBuf &b, size_t bytes) {
        if (e == hipSuccess) e = b.alloc(bytes);
    };
    const size_t vbytes = (size_t)Kp * n * sizeof(double);
    A(bV0, vbytes);
    A(bV1, vbytes);
    A(bW0, vbytes);
    A(bW1, vbytes);
    A(bpart, (size_t)Kp * nblk * sizeof(double));
    if (!ab) A(bab, (size_t)Kp * 2 * nu * sizeof(double));
    A(bst, (size_t)Kp * sizeof(LzRhs));
    A(bz, (size_t)n_shift * sizeof(double2));
    if (e != hipSuccess) return fail(SCOCG_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    std::vector<LzRhs> hst(Kp);
    for (int64_t c = 0; c < Kp; ++c) {
        hst[c] = LzRhs{};
        hst[c].j = c < n_rhs ? rhs_idx[c] : -1;
        hst[c].done = c < n_rhs ? 0 : 1;
    }
    HIPCHK(hipMemcpyAsync(bst.ptr, hst.data(), Kp * sizeof(LzRhs), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bz.ptr, z, n_shift * sizeof(double2), hipMemcpyHostToDevice, st));
    LzDev s{};
    s.hub = H->d.d_hub;
    s.slice_ptr = H->d.d_slice_ptr;
    s.slice_w = H->d.d_slice_w;
    s.ell_col = H->d.d_ell_col;
    s.ell_val = H->d.d_ell_val;
    s.n = n;
    s.K = Kp;
    s.rb = LZ_RB;
    s.gscale = 1.0;
    s.nblk = nblk;
    s.nu = nu;
    s.V[0] = bV0.as<double>();
    s.V[1] = bV1.as<double>();
    s.W[0] = bW0.as<double>();
    s.W[1] = bW1.as<double>();
    s.part = bpart.as<double>();
    s.ab = ab ? ab : bab.as<double>();
    s.st = bst.as<LzRhs>();
    TimerEvents evs;
    HIPCHK(evs.create());
    hipEvent_t t0 = evs.t0, t1 = evs.t1;
    HIPCHK(hipEventRecord(t0, st));
    for (int it = 0; it < nu; ++it) HIPCHK(launch_lanczos_step(s, it, st));
    HIPCHK(launch_lanczos_greens(s, bz.as<double2>(), n_shift, n_rhs, (double2 *)G, st));
    HIPCHK(hipEventRecord(t1, st));
    HIPCHK(hipMemcpyAsync(hst.data(), bst.ptr, Kp * sizeof(LzRhs), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, t0, t1));
    int64_t steps = 0;
    for (int64_t c = 0; c < n_rhs; ++c) {
        steps += hst[c].m;
        if (dim) dim[c] = hst[c].m;
    }
    g_timing.total_ms = ms;
    g_timing.iterations = steps;
    g_timing.blocks = nu;
    return SCOCG_OK;
}

// Ground state (Sec. 2.2): the three-term recurrence from x0 estimates the lowest eigenvalues
// (bisection on the reduced Hamiltonian) and, run a second time, accumulates the Ritz vector;
// inverse iteration then refines it: each sweep solves (sigma - H) y = psi with one shift
// sigma below the spectrum (where COCG is CG) and normalizes y, until ||H psi - E psi|| <= tol.
// <b|(z_k - H)^{-1}|b> for a real start vector b by the Krylov-subspace method (Sec. 3.2):
// the three-term recurrence from b/|b|, then |b|^2 times the continued fraction of the reduced
// Hamiltonian.
extern "C" int krylov_greens_vec(scocg_csr_t H, int64_t n_shift, const double *z, const double *b, int32_t nu,
                                 double *G, double *ab, int32_t *dim, void *stream)
{
    g_err.clear();
    if (!H || !z || !b || !G) return fail(SCOCG_EINVAL, "null argument");
    REQUIRE_DEVICE((const void *)b, (const void *)G, (const void *)ab);
    if (n_shift < 1) return fail(SCOCG_EINVAL, "n_shift must be positive");
    if (nu < 1 || nu > (1 << 20)) return fail(SCOCG_EINVAL, "nu must be in [1, 2^20]");
    for (int64_t k = 0; k < 2 * n_shift; ++k)
        if (!std::isfinite(z[k])) return fail(SCOCG_EINVAL, "non-finite shift");
    hipStream_t st = (hipStream_t)stream;
    g_timing = scocg_timing{};
    const int64_t n = H->d.n;
    const int64_t nblk = (n + LZ_TILE - 1) / LZ_TILE;
    DevBuf bxs, bV0, bV1, bW0, bW1, bpart, bab, bst, bz, bscal;
    hipError_t e = hipSuccess;
    auto A = [&](DevBuf &buf, size_t bytes) {
        if (e == hipSuccess) e = buf.alloc(bytes);
    };
    A(bxs, n * sizeof(double));
    for (DevBuf *v : {&bV0, &bV1, &bW0, &bW1}) A(*v, (size_t)n * sizeof(double));
    A(bpart, (size_t)2 * nblk * sizeof(double));
    if (!ab) A(bab, (size_t)2 * nu * sizeof(double));
    A(bst, sizeof(LzRhs));
    A(bz, (size_t)n_shift * sizeof(double2));
    A(bscal, 8 * sizeof(double));
    if (e != hipSuccess) return fail(SCOCG_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    SvDev v{};
    v.hub = H->d.d_hub;
    v.slice_ptr = H->d.d_slice_ptr;
    v.slice_w = H->d.d_slice_w;
    v.ell_col = H->d.d_ell_col;
    v.ell_val = H->d.d_ell_val;
    v.n = n;
    v.nblk = nblk;
    v.part = bpart.as<double>();
    v.scal = bscal.as<double>();
    double *xs = bxs.as<double>();
    HIPCHK(hipMemcpyAsync(xs, b, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(sv_normalize(v, xs, nullptr, st));
    double nb2 = 0;
    HIPCHK(hipMemcpyAsync(&nb2, bscal.as<double>() + 2, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (!(nb2 > 0) || !std::isfinite(nb2)) return fail(SCOCG_EINVAL, "the start vector must be nonzero and finite");
    LzRhs h0{};
    h0.j = -1;
    HIPCHK(hipMemcpyAsync(bst.ptr, &h0, sizeof(LzRhs), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bz.ptr, z, n_shift * sizeof(double2), hipMemcpyHostToDevice, st));
    LzDev s{};
    s.hub = v.hub;
    s.slice_ptr = v.slice_ptr;
    s.slice_w = v.slice_w;
    s.ell_col = v.ell_col;
    s.ell_val = v.ell_val;
    s.n = n;
    s.K = 1;
    s.rb = 1;
    s.nblk = nblk;
    s.nu = nu;
    s.V[0] = bV0.as<double>();
    s.V[1] = bV1.as<double>();
    s.W[0] = bW0.as<double>();
    s.W[1] = bW1.as<double>();
    s.part = bpart.as<double>();
    s.ab = ab ? ab : bab.as<double>();
    s.st = bst.as<LzRhs>();
    s.x0 = xs;
    s.gscale = nb2;
    TimerEvents evs;
    HIPCHK(evs.create());
    hipEvent_t t0 = evs.t0, t1 = evs.t1;
    HIPCHK(hipEventRecord(t0, st));
    for (int it = 0; it < nu; ++it) HIPCHK(launch_lanczos_step(s, it, st));
    HIPCHK(launch_lanczos_greens(s, bz.as<double2>(), n_shift, 1, (double2 *)G, st));
    HIPCHK(hipEventRecord(t1, st));
    LzRhs hf{};
    HIPCHK(hipMemcpyAsync(&hf, bst.ptr, sizeof(LzRhs), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, t0, t1));
    if (dim) *dim = hf.m;
    g_timing.total_ms = ms;
    g_timing.iterations = hf.m;
    return SCOCG_OK;
}

extern "C" int ground_state(scocg_csr_t H, const double *x0, int32_t nu, double tol, int32_t max_sweeps,
                            double *psi, double *E, double *res, int32_t *sweeps, void *stream)
{
    g_err.clear();
    if (!H || !x0 || !psi || !E) return fail(SCOCG_EINVAL, "null argument");
    REQUIRE_DEVICE((const void *)x0, (const void *)psi);
    if (nu < 2 || nu > (1 << 20)) return fail(SCOCG_EINVAL, "nu must be in [2, 2^20]");
    if (!(tol > 0) || max_sweeps < 0) return fail(SCOCG_EINVAL, "tol must be positive and max_sweeps >= 0");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = H->d.n;
    const int64_t nblk = (n + LZ_TILE - 1) / LZ_TILE;
    DevBuf bxs, bV0, bV1, bW0, bW1, bpart, bab, bst, beig, bu, bscr, bacc, by, bscal, bzb, bzx;
    hipError_t e = hipSuccess;
    auto A = [&](DevBuf &b, size_t bytes) {
        if (e == hipSuccess) e = b.alloc(bytes);
    };
    // the recurrence of one plain vector (no interleaved group)
    A(bxs, n * sizeof(double));
    for (DevBuf *b : {&bV0, &bV1, &bW0, &bW1}) A(*b, (size_t)n * sizeof(double));
    A(bpart, (size_t)2 * nblk * sizeof(double));
    A(bab, (size_t)2 * nu * sizeof(double));
    A(bst, sizeof(LzRhs));
    A(beig, 2 * sizeof(double));
    A(bu, (size_t)nu * sizeof(double));
    A(bscr, (size_t)nu * sizeof(double));
    A(bacc, n * sizeof(double));
    A(by, 2 * n * sizeof(double));
    A(bscal, 8 * sizeof(double));
    A(bzb, n * sizeof(double2));
    A(bzx, n * sizeof(double2));
    if (e != hipSuccess) return fail(SCOCG_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    SvDev v{};
    v.hub = H->d.d_hub;
    v.slice_ptr = H->d.d_slice_ptr;
    v.slice_w = H->d.d_slice_w;
    v.ell_col = H->d.d_ell_col;
    v.ell_val = H->d.d_ell_val;
    v.n = n;
    v.nblk = nblk;
    v.part = bpart.as<double>();
    v.scal = bscal.as<double>();
    double *xs = bxs.as<double>();
    HIPCHK(hipMemcpyAsync(xs, x0, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(sv_normalize(v, xs, nullptr, st));
    std::vector<LzRhs> hst(1);
    hst[0] = LzRhs{};
    hst[0].j = -1;
    LzDev s{};
    s.hub = v.hub;
    s.slice_ptr = v.slice_ptr;
    s.slice_w = v.slice_w;
    s.ell_col = v.ell_col;
    s.ell_val = v.ell_val;
    s.n = n;
    s.K = 1;
    s.rb = 1;
    s.nblk = nblk;
    s.nu = nu;
    s.V[0] = bV0.as<double>();
    s.V[1] = bV1.as<double>();
    s.W[0] = bW0.as<double>();
    s.W[1] = bW1.as<double>();
    s.part = bpart.as<double>();
    s.ab = bab.as<double>();
    s.st = bst.as<LzRhs>();
    s.x0 = xs;
    TimerEvents evs;
    HIPCHK(evs.create());
    hipEvent_t t0 = evs.t0, t1 = evs.t1;
    HIPCHK(hipEventRecord(t0, st));
    HIPCHK(hipMemcpyAsync(bst.ptr, hst.data(), sizeof(LzRhs), hipMemcpyHostToDevice, st));
    for (int it = 0; it < nu; ++it) HIPCHK(launch_lanczos_step(s, it, st));
    HIPCHK(launch_lanczos_lowest(s, beig.as<double>(), bu.as<double>(), bscr.as<double>(), st));
    double eig[2];
    HIPCHK(hipMemcpyAsync(eig, beig.ptr, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    // the same recurrence again (same bits), summing the Ritz vector sum_n u_n K_n
    HIPCHK(hipMemsetAsync(bacc.ptr, 0, n * sizeof(double), st));
    HIPCHK(hipMemcpyAsync(bst.ptr, hst.data(), sizeof(LzRhs), hipMemcpyHostToDevice, st));
    s.acc = bacc.as<double>();
    s.coef = bu.as<double>();
    for (int it = 0; it < nu; ++it) HIPCHK(launch_lanczos_step(s, it, st));
    double *x = bacc.as<double>();
    double *y = by.as<double>();
    double *y2 = y + n;
    HIPCHK(sv_normalize(v, x, nullptr, st));
    HIPCHK(sv_rayleigh(v, x, y, st));
    double sc[2];
    HIPCHK(hipMemcpyAsync(sc, bscal.ptr, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double Ecur = sc[0], rcur = std::sqrt(std::max(sc[1], 0.0));
    // a fixed shift below the lowest eigenvalue: a tenth of the estimated gap under the
    // estimate, and not above theta - r, the lower end of the interval [theta - r, theta + r]
    // that holds an eigenvalue for the Ritz pair (theta, psi) with residual norm r (the
    // estimate is an upper bound of E0 and can be poor after few steps)
    const double gap = eig[1] - eig[0];
    const double sigma = std::min(eig[0] - std::max(0.1 * gap, 1e-6 * std::max(1.0, std::fabs(eig[0]))), Ecur - rcur);
    int32_t k = 0;
    int64_t cg_iters = 0;
    while (rcur > tol && k < max_sweeps) {
        HIPCHK(sv_to_complex(x, bzb.as<double2>(), n, st));
        scocg_opts o;
        scocg_default_opts(&o);
        o.tol = std::min(1e-10, 1e-2 * tol);
        o.max_iter = 1000000;
        o.seed_index = 0;
        o.seed_switching = 0;
        // one shift: long blocks buy nothing here, and the residual ring (2 T + 1 vectors)
        // grows with the block length (the iterates are the same for every length)
        o.block = 4;
        const double zs[2] = {sigma, 0.0};
        SolveRequest rq{};
        rq.H = H;
        rq.M = 1;
        rq.K = 1;
        rq.z = zs;
        rq.B = bzb.as<double2>();
        rq.o = o;
        rq.Xout = bzx.as<double2>();
        scocg_pair_report rp{};
        rq.rep = &rp;
        const int rc = solve(rq, st);
        if (rc != SCOCG_OK) return rc;
        cg_iters += rp.iters;
        HIPCHK(sv_real_part(bzx.as<double2>(), y2, n, st));
        HIPCHK(sv_normalize(v, y2, x, st));
        std::swap(x, y2);
        HIPCHK(sv_rayleigh(v, x, y, st));
        HIPCHK(hipMemcpyAsync(sc, bscal.ptr, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        Ecur = sc[0];
        rcur = std::sqrt(std::max(sc[1], 0.0));
        ++k;
    }
    HIPCHK(sv_to_complex(x, (double2 *)psi, n, st));
    HIPCHK(hipEventRecord(t1, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, t0, t1));
    E[0] = Ecur;
    E[1] = eig[1];
    if (res) *res = rcur;
    if (sweeps) *sweeps = k;
    g_timing = scocg_timing{};
    g_timing.total_ms = ms;
    g_timing.iterations = 2 * (int64_t)nu + cg_iters;
    g_timing.blocks = k;
    if (!(rcur <= tol)) return fail(SCOCG_ENOCONV, "the residual norm is above tol after max_sweeps sweeps");
    return SCOCG_OK;
}

// c_{site,spin} or c+_{site,spin} between sectors of the Hubbard ring (Sec. 4.2 excitations).
extern "C" int hubbard_fermion_op(int32_t L, int32_t n_up, int32_t n_dn, int32_t site, int32_t spin, int32_t create,
                                  const double *x, double *y, void *stream)
{
    g_err.clear();
    if (!x || !y) return fail(SCOCG_EINVAL, "null argument");
    REQUIRE_DEVICE((const void *)x, (const void *)y);
    if (L < 3 || L > 30) return fail(SCOCG_EINVAL, "L must be in [3, 30]");
    if (n_up < 0 || n_up > L || n_dn < 0 || n_dn > L) return fail(SCOCG_EINVAL, "electron counts out of range");
    if (site < 0 || site >= L || (spin != 0 && spin != 1)) return fail(SCOCG_EINVAL, "site or spin out of range");
    const int d = create ? 1 : -1;
    const int tu = spin == 0 ? n_up + d : n_up, td = spin == 1 ? n_dn + d : n_dn;
    if (tu < 0 || tu > L || td < 0 || td > L) return fail(SCOCG_EINVAL, "the target sector does not exist");
    const Species up = build_species(L, n_up), dn = build_species(L, n_dn);
    const int64_t Du = (int64_t)up.conf.size(), Dd = (int64_t)dn.conf.size();
    const int64_t Dd_t = (int64_t)build_species(L, td).conf.size();
    const int64_t D_t = (int64_t)build_species(L, tu).conf.size() * Dd_t;
    std::vector<int64_t> binom((L + 1) * (L + 1), 0);
    for (int p = 0; p <= L; ++p) {
        binom[p * (L + 1)] = 1;
        for (int t = 1; t <= p; ++t)
            binom[p * (L + 1) + t] = binom[(p - 1) * (L + 1) + t - 1] + (t <= p - 1 ? binom[(p - 1) * (L + 1) + t] : 0);
    }
    DevBuf bup, bdn, bbin;
    hipError_t e = bup.alloc(Du * sizeof(uint32_t));
    if (e == hipSuccess) e = bdn.alloc(Dd * sizeof(uint32_t));
    if (e == hipSuccess) e = bbin.alloc(binom.size() * sizeof(int64_t));
    if (e != hipSuccess) return fail(SCOCG_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(bup.ptr, up.conf.data(), Du * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bdn.ptr, dn.conf.data(), Dd * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bbin.ptr, binom.data(), binom.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(launch_fermion_op(bup.as<uint32_t>(), bdn.as<uint32_t>(), Du, Dd, bbin.as<int64_t>(), L, n_up, site, spin,
                             create, Dd_t, D_t, (const double2 *)x, (double2 *)y, st));
    // the tables are freed on return: wait for the kernels that read them
    HIPCHK(hipStreamSynchronize(st));
    return SCOCG_OK;
}

extern "C" int greens_diag(scocg_csr_t H, int64_t n_shift, const double *z, int64_t n_rhs, const int64_t *rhs_idx,
                           const scocg_opts *o, double *G, scocg_pair_report *rep, scocg_tape_t *tape, void *stream)
{
    g_err.clear();
    if (!H || !z || !rhs_idx || !o || !G) return fail(SCOCG_EINVAL, "null argument");
    REQUIRE_DEVICE((const void *)G);
    for (int64_t j = 0; j < n_rhs; ++j)
        if (rhs_idx[j] < 0 || rhs_idx[j] >= H->d.n) return fail(SCOCG_EINVAL, "rhs_idx out of range");
    const bool want_tape = tape && o->keep_tape;
    SolveRequest rq{};
    rq.H = H;
    rq.M = n_shift;
    rq.K = n_rhs;
    rq.z = z;
    rq.B = nullptr;
    rq.unit_idx = rhs_idx;
    rq.o = *o;
    rq.Xout = nullptr;
    rq.projection = !want_tape;
    rq.Gout = (double2 *)G;
    rq.rep = rep;
    scocg_tape *tp = nullptr;
    if (want_tape) {
        tp = new scocg_tape();
        rq.keepX = &tp->X;
    }
    int rc = solve(rq, (hipStream_t)stream);
    if (tp) {
        if (rc == SCOCG_OK || rc == SCOCG_ENOCONV) {
            H->refs.fetch_add(1);
            tp->H = H;
            tp->K = n_rhs;
            tp->M = n_shift;
            tp->n = H->d.n;
            *tape = tp;
        } else {
            delete tp;
        }
    }
    return rc;
}

// ------------------------------------------------------------------------------------------
// greens_diag without device allocation
// ------------------------------------------------------------------------------------------
// Every buffer of the solve is carved out of one file-scope device array.  In host code the
// array's name stands for a host-side shadow, not the device memory: its device address is
// looked up once per device (hipGetSymbolAddress, with that device current) and only that
// address is handed to kernels.  The array keeps its contents between calls; everything a solve
// reads is initialised by the solve itself.
static __device__ __align__(256) unsigned char scratch[SCOCG_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];     // serialises calls on one device (they share its array)
void *g_scratch_ptr[kMaxDevices] = {};    // device address of the array, per device

// Carves aligned sub-buffers from a base address (base = null only sizes the layout).
struct Carver {
    char *base;
    size_t off = 0;
    void *take(size_t bytes)
    {
        off = (off + 255) / 256 * 256;
        void *p = base ? (void *)(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

}  // namespace

extern "C" int greens_diag_noalloc(scocg_csr_t H, int64_t n_shift, const double *z, int64_t n_rhs,
                                   const int64_t *rhs_idx, const scocg_opts *o, double *G, scocg_pair_report *rep,
                                   void *stream)
{
    static_assert(sizeof(PairReportDev) == sizeof(scocg_pair_report), "report layouts differ");
    g_err.clear();
    g_swlog.K = 0;
    if (!H || !z || !rhs_idx || !o || !G) return fail(SCOCG_EINVAL, "null argument");
    REQUIRE_DEVICE((const void *)G);
    const int64_t K = n_rhs, M = n_shift;
    const DevCSR &d = H->d;
    const int64_t n = d.n;
    if (M <= 0 || K <= 0) return fail(SCOCG_EINVAL, "n_shift and n_rhs must be positive");
    if (M > (1 << 20) || K > 65535) return fail(SCOCG_EINVAL, "too many shifts or right-hand sides");
    for (int64_t j = 0; j < K; ++j)
        if (rhs_idx[j] < 0 || rhs_idx[j] >= n) return fail(SCOCG_EINVAL, "rhs_idx out of range");
    for (int64_t k = 0; k < 2 * M; ++k)
        if (!std::isfinite(z[k])) return fail(SCOCG_EINVAL, "non-finite shift");
    if (o->keep_tape || o->refine > 0 || o->check_true || o->window != 0)
        return fail(SCOCG_EINVAL, "greens_diag_noalloc keeps no tape, does not refine or check true residuals, "
                                  "and stores every shift's direction (window 0)");
    if (!(o->tol > 0) && o->fixed_iter <= 0) return fail(SCOCG_EINVAL, "tol must be positive");
    if (o->max_iter <= 0 && o->fixed_iter <= 0) return fail(SCOCG_EINVAL, "max_iter must be positive");
    if (o->precision != 0 && o->precision != 1) return fail(SCOCG_EINVAL, "precision must be 0 or 1");
    if (o->shifts_per_wg > 64) return fail(SCOCG_EINVAL, "shifts_per_wg must be at most 64");
    if (o->schedule < 0 || o->schedule > 2) return fail(SCOCG_EINVAL, "schedule must be 0, 1 or 2");
    const int TB = o->block > 0 ? o->block : 48;
    if (TB != 1 && TB != 2 && TB != 4 && TB != 8 && TB != 16 && TB != 24 && TB != 32 && TB != 40 && TB != 48)
        return fail(SCOCG_EINVAL, "block must be 1, 2, 4, 8, 16, 24, 32, 40 or 48");
    int32_t seed = 0;
    if (o->seed_index >= 0) {
        if (o->seed_index >= M) return fail(SCOCG_EINVAL, "seed_index out of range");
        seed = o->seed_index;
    } else {
        seed = default_seed(z, M, d.trace / (double)n);
    }
    const bool fixed = o->fixed_iter > 0;
    const int32_t limit = fixed ? o->fixed_iter : o->max_iter;
    const size_t KM = (size_t)K * M;
    const size_t ntot = (size_t)K * n;
    const size_t esz = o->precision == 0 ? sizeof(double2) : sizeof(float2);
    const int R = 2 * TB + 1;
    const int64_t nblk = (n + 255) / 256;

    // the layout, in the order the buffers are carved (sized first with a null base)
    struct Layout {
        double2 *z, *ring, *p, *q, *Xproj, *pi, *pip, *bk, *ah, *bh, *p2;
        void *P, *coef;
        SeedState *seed;
        RhsDesc *desc;
        int64_t *prow, *idx;
        double *res, *rn, *p1;
        int32_t *iters, *pst, *act, *nact, *blk, *sd, *swlog, *flag, *worst;
        uint32_t *cnt;
        unsigned long long *stats;
        long long *totals;
        PairReportDev *rep;
        size_t coef_bytes;
    };
    auto carve = [&](char *base, Layout &L) -> size_t {
        Carver c{base};
        L.z = (double2 *)c.take(M * sizeof(double2));
        L.seed = (SeedState *)c.take(K * sizeof(SeedState));
        L.ring = (double2 *)c.take((size_t)R * ntot * sizeof(double2));
        L.p = (double2 *)c.take(2 * ntot * sizeof(double2));
        L.q = (double2 *)c.take(ntot * sizeof(double2));
        L.P = c.take((size_t)M * ntot * esz);
        L.desc = (RhsDesc *)c.take(K * sizeof(RhsDesc));
        L.Xproj = (double2 *)c.take(KM * sizeof(double2));
        L.prow = (int64_t *)c.take(K * sizeof(int64_t));
        L.idx = (int64_t *)c.take(K * sizeof(int64_t));
        L.pi = (double2 *)c.take(KM * sizeof(double2));
        L.pip = (double2 *)c.take(KM * sizeof(double2));
        L.bk = (double2 *)c.take(KM * sizeof(double2));
        L.res = (double *)c.take(KM * sizeof(double));
        L.iters = (int32_t *)c.take(KM * sizeof(int32_t));
        L.pst = (int32_t *)c.take(KM * sizeof(int32_t));
        L.act = (int32_t *)c.take(KM * sizeof(int32_t));
        L.nact = (int32_t *)c.take(2 * KM * sizeof(int32_t));
        L.blk = (int32_t *)c.take(2 * (size_t)K * 4 * sizeof(int32_t));
        L.ah = (double2 *)c.take((size_t)K * TB * sizeof(double2));
        L.bh = (double2 *)c.take((size_t)K * TB * sizeof(double2));
        L.rn = (double *)c.take((size_t)K * TB * sizeof(double));
        L.coef_bytes = KM * TB * 2 * (o->precision == 0 ? sizeof(double2) : sizeof(float2));
        L.coef = c.take(2 * L.coef_bytes);
        L.p2 = (double2 *)c.take((size_t)K * nblk * sizeof(double2));
        L.p1 = (double *)c.take((size_t)K * nblk * sizeof(double));
        L.cnt = (uint32_t *)c.take(K * sizeof(uint32_t));
        L.sd = (int32_t *)c.take(K * sizeof(int32_t));
        L.stats = (unsigned long long *)c.take(3 * sizeof(unsigned long long));
        L.swlog = (int32_t *)c.take(KM * 2 * sizeof(int32_t));
        L.flag = (int32_t *)c.take(sizeof(int32_t));
        L.worst = (int32_t *)c.take(sizeof(int32_t));
        L.totals = (long long *)c.take(2 * sizeof(long long));
        L.rep = (PairReportDev *)c.take(KM * sizeof(PairReportDev));
        return c.off;
    };
    Layout L{};
    const size_t need = carve(nullptr, L);
    if (need > (size_t)SCOCG_NOALLOC_MAX_BYTES)
        return fail(SCOCG_EINVAL, "greens_diag_noalloc needs " + std::to_string(need) + " bytes of scratch, more than "
                                  "its fixed " + std::to_string((size_t)SCOCG_NOALLOC_MAX_BYTES) +
                                  " (fewer right-hand sides or shifts, or a shorter block, reduce it)");

    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SCOCG_EINVAL, "device index beyond the supported range");
    std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(SCOCG_EHIP, "scratch array has no device address");
        g_scratch_ptr[dev] = ptr;
    }
    carve((char *)g_scratch_ptr[dev], L);
    hipStream_t st = (hipStream_t)stream;
    // the lock is released only after the stream has drained, on every return path, so no kernel
    // of this call still uses the array when the next call on this device starts
    struct DrainOnExit {
        hipStream_t st;
        ~DrainOnExit() { (void)hipStreamSynchronize(st); }
    } drain{st};
    const auto t_start = std::chrono::steady_clock::now();
    g_timing = scocg_timing{};

    SolveDev s{};
    s.ntot = (int64_t)ntot;
    s.n = n;
    s.K = K;
    s.M = M;
    s.TB = TB;
    s.R = R;
    s.precision = o->precision;
    s.fixed = fixed ? 1 : 0;
    s.switching = o->seed_switching ? 1 : 0;
    s.tol = o->tol;
    s.nblk = nblk;
    s.shifts_per_wg = o->shifts_per_wg > 0 ? o->shifts_per_wg : (int)std::min<int64_t>(M, TB >= 24 ? 64 : 32);
    s.zper = 0;
    s.spmv_rb = K >= 2 ? 2 : 1;
    (d.d_hub ? s.has_hub : s.has_sell) = 1;
    (n >= RED_BIG_ROWS ? s.has_red_big : s.has_red_small) = 1;
    s.hub_lds = 1;
    if (d.d_hub) {
        if (d.hub_Dd > HUB_LDS_MAX || n / d.hub_Dd > (n + 255) / 256) s.hub_lds = 0;
        s.hub_du_max = n / d.hub_Dd;
    }
    s.z = L.z;
    s.seed = L.seed;
    s.ring = L.ring;
    s.p = L.p;
    s.q = L.q;
    s.X = nullptr;
    s.P = L.P;
    s.Mst = M;
    s.wshift = nullptr;
    s.wslot = nullptr;
    s.Uproj = nullptr;
    s.Xproj = L.Xproj;
    s.wproj = nullptr;
    s.shist = nullptr;
    s.part3 = nullptr;
    s.proj_row = L.prow;
    s.pi = L.pi;
    s.pi_prev = L.pip;
    s.beta_k = L.bk;
    s.res = L.res;
    s.iters = L.iters;
    s.pstatus = L.pst;
    s.active = L.act;
    s.nact = L.nact;
    s.ahist = L.ah;
    s.bhist = L.bh;
    s.rnhist = L.rn;
    s.coef = L.coef;
    s.blk = L.blk;
    s.part2 = L.p2;
    s.part1 = L.p1;
    s.cnt = L.cnt;
    s.stats = L.stats;
    s.swlog = L.swlog;
    s.desc = L.desc;

    const RhsDesc proto{d.d_slice_ptr, d.d_slice_w, d.d_ell_col, d.d_ell_val, d.nslices, n, 0, d.d_hub};
    HIPCHK(launch_fill_desc(proto, K, seed, L.desc, L.sd, st));
    HIPCHK(hipMemcpyAsync(L.z, z, M * sizeof(double2), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(L.idx, rhs_idx, K * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(L.prow, rhs_idx, K * sizeof(int64_t), hipMemcpyHostToDevice, st));
    // counters, activity counts, block records, statistics and the report sums start at zero
    HIPCHK(launch_zero(L.cnt, K * sizeof(uint32_t), st));
    HIPCHK(launch_zero(L.nact, 2 * KM * sizeof(int32_t), st));
    HIPCHK(launch_zero(L.blk, 2 * (size_t)K * 4 * sizeof(int32_t), st));
    HIPCHK(launch_zero(L.stats, 3 * sizeof(unsigned long long), st));
    HIPCHK(launch_zero(L.swlog, KM * 2 * sizeof(int32_t), st));
    HIPCHK(launch_zero(L.worst, sizeof(int32_t), st));
    HIPCHK(launch_zero(L.totals, 2 * sizeof(long long), st));
    HIPCHK(launch_zero(s.p, 2 * ntot * sizeof(double2), st));
    HIPCHK(launch_init(s, nullptr, L.idx, L.sd, limit, st));

    // the block loop of solve() in its serial schedule, launched directly (no streams, events
    // or graphs are created); the stop test reads one flag computed on the device
    SolveDev sp[2] = {s, s};
    for (int q = 0; q < 2; ++q) {
        sp[q].coef = (char *)L.coef + q * L.coef_bytes;
        sp[q].nact = L.nact + q * KM;
        sp[q].blk = L.blk + q * (size_t)K * 4;
    }
    const int per_sync = std::max(1, 64 / TB);
    const int64_t max_blocks = (int64_t)K * ((int64_t)limit + 4 * M + 8) + 8 + per_sync;
    int64_t blocks = 0;
    for (;;) {
        for (int b = 0; b < per_sync; ++b) {
            const int par = (int)(blocks & 1);
            HIPCHK(launch_switch_vectors(sp[par], st));
            for (int t = 0; t < TB; ++t) HIPCHK(launch_seed_iteration(sp[par], st));
            HIPCHK(launch_pair_scalars(sp[par], st));
            HIPCHK(launch_flush(sp[par], st));
            HIPCHK(launch_block_finalize(sp[par], st));
            ++blocks;
        }
        int32_t stopped = 0;
        HIPCHK(launch_all_stopped(L.seed, K, L.flag, st));
        HIPCHK(hipMemcpyAsync(&stopped, L.flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (stopped) break;
        if (blocks > max_blocks) return fail(SCOCG_EHIP, "iteration driver did not terminate");
    }
    HIPCHK(launch_gather_diag(s, L.idx, (double2 *)G, st));
    HIPCHK(launch_pack_report(K, M, s.fixed, L.iters, L.pst, L.res, L.seed, L.rep, L.worst, L.totals, st));
    int32_t worst = 0;
    long long totals[2] = {0, 0};
    unsigned long long stats[3] = {0, 0, 0};
    HIPCHK(hipMemcpyAsync(&worst, L.worst, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(totals, L.totals, sizeof(totals), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(stats, L.stats, sizeof(stats), hipMemcpyDeviceToHost, st));
    if (rep) HIPCHK(hipMemcpyAsync(rep, L.rep, KM * sizeof(scocg_pair_report), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    g_timing.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    g_timing.iterations = totals[0];
    g_timing.switches = totals[1];
    g_timing.blocks = blocks;
    g_timing.update_bytes = (double)stats[0];
    g_timing.update_flops = (double)stats[2];
    if (worst == 2) return fail(SCOCG_EBREAKDOWN, "COCG breakdown on at least one pair");
    if (worst == 1) return fail(SCOCG_ENOCONV, "at least one pair did not converge");
    return SCOCG_OK;
}

// <w_j|(z_k - H)^{-1}|b_j> for dense right-hand sides b_j and projection vectors w_j (Sec. 3.3:
// when only a projection of the solution is wanted, each shifted system costs scalar work).
extern "C" int greens_proj(scocg_csr_t H, int64_t n_shift, const double *z, int64_t n_rhs, const double *B,
                           const double *W, const scocg_opts *o, double *G, scocg_pair_report *rep, void *stream)
{
    g_err.clear();
    if (!H || !z || !B || !W || !o || !G) return fail(SCOCG_EINVAL, "null argument");
    REQUIRE_DEVICE((const void *)B, (const void *)W, (const void *)G);
    SolveRequest rq{};
    rq.H = H;
    rq.M = n_shift;
    rq.K = n_rhs;
    rq.z = z;
    rq.B = (const double2 *)B;
    rq.unit_idx = nullptr;
    rq.o = *o;
    rq.Xout = nullptr;
    rq.projection = true;
    rq.Gout = (double2 *)G;
    rq.rep = rep;
    rq.wproj = (const double2 *)W;
    return solve(rq, (hipStream_t)stream);
}

extern "C" int greens_diag_batched(int64_t n_problems, const scocg_csr_t *H, const int64_t *n_rhs,
                                   const int64_t *rhs_idx, int64_t n_shift, const double *z, const scocg_opts *o,
                                   double *G, scocg_pair_report *rep, void *stream)
{
    g_err.clear();
    if (n_problems <= 0 || !H || !n_rhs || !rhs_idx || !z || !o || !G) return fail(SCOCG_EINVAL, "null argument");
    REQUIRE_DEVICE((const void *)G);
    SolveRequest rq{};
    std::vector<int64_t> idx;
    for (int64_t q = 0; q < n_problems; ++q) {
        if (!H[q] || n_rhs[q] < 0) return fail(SCOCG_EINVAL, "invalid problem " + std::to_string(q));
        for (int64_t c = 0; c < n_rhs[q]; ++c) {
            const int64_t j = rhs_idx[idx.size()];
            if (j < 0 || j >= H[q]->d.n) return fail(SCOCG_EINVAL, "rhs_idx out of range in problem " + std::to_string(q));
            idx.push_back(j);
            rq.Hj.push_back(H[q]);
        }
    }
    if (idx.empty()) return fail(SCOCG_EINVAL, "no right-hand sides");
    if (o->keep_tape || o->refine) return fail(SCOCG_EINVAL, "batched solves keep no tape and do not refine");
    rq.H = H[0];
    rq.M = n_shift;
    rq.K = (int64_t)idx.size();
    rq.z = z;
    rq.B = nullptr;
    rq.unit_idx = idx.data();
    rq.o = *o;
    rq.o.check_true = 0;
    rq.Xout = nullptr;
    rq.projection = true;
    rq.Gout = (double2 *)G;
    rq.rep = rep;
    return solve(rq, (hipStream_t)stream);
}

extern "C" int density_matrix_energy(scocg_csr_t H, int64_t n_quad, const double *z, const double *w, int64_t n_rhs,
                                     const int64_t *rhs_idx, const scocg_opts *o, int64_t rhs_batch, double *rho_nnz,
                                     double *E_band, double *dE_dval, void *stream)
{
    g_err.clear();
    if (!H || !z || !w || !rhs_idx || !o || !E_band) return fail(SCOCG_EINVAL, "null argument");
    REQUIRE_DEVICE((const void *)rho_nnz, (const void *)E_band, (const void *)dE_dval);
    if (n_quad <= 0 || n_rhs <= 0) return fail(SCOCG_EINVAL, "n_quad and n_rhs must be positive");
    if (matrix_free(H)) return fail(SCOCG_EINVAL, "density_matrix_energy needs a stored matrix");
    const DevCSR &d = H->d;
    for (int64_t j = 0; j < n_rhs; ++j)
        if (rhs_idx[j] < 0 || rhs_idx[j] >= d.n) return fail(SCOCG_EINVAL, "rhs_idx out of range");
    {
        // each column's rho entries are written by one workgroup of its batch: a column listed
        // twice would be accumulated twice (and, within one batch, by two racing workgroups)
        std::vector<int64_t> sorted_idx(rhs_idx, rhs_idx + n_rhs);
        std::sort(sorted_idx.begin(), sorted_idx.end());
        if (std::adjacent_find(sorted_idx.begin(), sorted_idx.end()) != sorted_idx.end())
            return fail(SCOCG_EINVAL, "rhs_idx lists a column more than once");
    }
    int64_t maxrow = 0;
    for (int64_t i = 0; i < d.n; ++i) maxrow = std::max<int64_t>(maxrow, H->h_row_ptr[i + 1] - H->h_row_ptr[i]);
    hipStream_t st = (hipStream_t)stream;
    int64_t batch = rhs_batch > 0 ? rhs_batch : std::min<int64_t>(n_rhs, 256);
    batch = std::min(batch, n_rhs);
    const int64_t nchunk = dE_dval ? pair_outer_chunks(d.n, batch * n_quad, (int)maxrow) : 0;
    DevBuf bw, bz, bidx, bX, bEp, bc, bpart;
    if (bw.alloc(n_quad * sizeof(double2)) || bz.alloc(n_quad * sizeof(double2)) ||
        bidx.alloc(batch * sizeof(int64_t)) || bX.alloc((size_t)batch * n_quad * d.n * sizeof(double2)) ||
        bEp.alloc(batch * sizeof(double)) || bc.alloc((size_t)batch * n_quad * sizeof(double2)) ||
        bpart.alloc((size_t)nchunk * (size_t)d.nnz * sizeof(double)))
        return fail(SCOCG_ENOMEM, "density_matrix_energy: device allocation failed");
    HIPCHK(hipMemcpyAsync(bw.ptr, w, n_quad * sizeof(double2), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(bz.ptr, z, n_quad * sizeof(double2), hipMemcpyHostToDevice, st));
    int rc_all = SCOCG_OK;
    for (int64_t j0 = 0; j0 < n_rhs; j0 += batch) {
        const int64_t kb = std::min(batch, n_rhs - j0);
        SolveRequest rq{};
        rq.H = H;
        rq.M = n_quad;
        rq.K = kb;
        rq.z = z;
        rq.B = nullptr;
        rq.unit_idx = rhs_idx + j0;
        rq.o = *o;
        rq.o.check_true = 0;
        rq.Xout = bX.as<double2>();
        rq.projection = false;
        int rc = solve(rq, st);
        if (rc != SCOCG_OK && rc != SCOCG_ENOCONV) return rc;
        if (rc == SCOCG_ENOCONV) rc_all = SCOCG_ENOCONV;
        HIPCHK(hipMemcpyAsync(bidx.ptr, rhs_idx + j0, kb * sizeof(int64_t), hipMemcpyHostToDevice, st));
        HIPCHK(launch_density_rho(d.n, kb, n_quad, bX.as<double2>(), bidx.as<int64_t>(), d.d_row_ptr, d.d_col,
                                  d.d_mirror, bw.as<double2>(), bz.as<double2>(), rho_nnz, bEp.as<double>(), E_band,
                                  st));
        if (dE_dval) {
            HIPCHK(launch_pair_weights(0, kb, n_quad, bw.as<double2>(), bz.as<double2>(), nullptr, bc.as<double2>(), st));
            HIPCHK(launch_pair_outer(d.n, kb * n_quad, bX.as<double2>(), bc.as<double2>(), d.d_row_ptr, d.d_col,
                                     d.nnz, (int)maxrow, nchunk, bpart.as<double>(), dE_dval, st));
        }
        HIPCHK(hipStreamSynchronize(st));
    }
    if (rc_all == SCOCG_ENOCONV) g_err = "at least one pair did not converge";
    return rc_all;
}

extern "C" int backward(scocg_tape_t tape, const double *grad_G, double *grad_val, void *stream)
{
    g_err.clear();
    if (!tape || !grad_G || !grad_val) return fail(SCOCG_EINVAL, "null argument");
    REQUIRE_DEVICE((const void *)grad_G, (const void *)grad_val);
    if (matrix_free(tape->H)) return fail(SCOCG_EINVAL, "backward needs a stored matrix");
    const DevCSR &d = tape->H->d;
    int64_t maxrow = 0;
    for (int64_t i = 0; i < d.n; ++i)
        maxrow = std::max<int64_t>(maxrow, tape->H->h_row_ptr[i + 1] - tape->H->h_row_ptr[i]);
    hipStream_t st = (hipStream_t)stream;
    const int64_t npairs = tape->K * tape->M;
    const int64_t nchunk = pair_outer_chunks(d.n, npairs, (int)maxrow);
    DevBuf bc, bpart;
    if (bc.alloc((size_t)npairs * sizeof(double2)) || bpart.alloc((size_t)nchunk * (size_t)d.nnz * sizeof(double)))
        return fail(SCOCG_ENOMEM, "backward: allocation failed");
    HIPCHK(launch_pair_weights(1, tape->K, tape->M, nullptr, nullptr, (const double2 *)grad_G, bc.as<double2>(), st));
    HIPCHK(launch_pair_outer(d.n, npairs, tape->X.as<double2>(), bc.as<double2>(), d.d_row_ptr, d.d_col, d.nnz,
                             (int)maxrow, nchunk, bpart.as<double>(), grad_val, st));
    HIPCHK(hipStreamSynchronize(st));
    return SCOCG_OK;
}

extern "C" void tape_free(scocg_tape_t t) { delete t; }

// Gauss-Legendre nodes on [-1, 1] by Newton's method on the Legendre recurrence.
extern "C" int scocg_contour(double e_lo, double mu, int64_t n_quad, double *z, double *w)
{
    g_err.clear();
    if (!z || !w || n_quad <= 0 || !(mu > e_lo)) return fail(SCOCG_EINVAL, "invalid contour arguments");
    const double c = 0.5 * (e_lo + mu), R = 0.5 * (mu - e_lo);
    const int64_t n = n_quad;
    for (int64_t i = 0; i < n; ++i) {
        double x = -std::cos(M_PI * (i + 0.75) / (n + 0.5));  // ascending nodes
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int64_t k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / (double)k;
                p0 = p1;
                p1 = p2;
            }
            double pn = n == 1 ? x : p1, pm = n == 1 ? 1.0 : p0;
            dp = n * (x * pn - pm) / (x * x - 1.0);
            const double dx = pn / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        // recompute the derivative at the converged node
        double p0 = 1.0, p1 = x;
        for (int64_t k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / (double)k;
            p0 = p1;
            p1 = p2;
        }
        double pn = n == 1 ? x : p1, pm = n == 1 ? 1.0 : p0;
        dp = n * (x * pn - pm) / (x * x - 1.0);
        const double wi = 2.0 / ((1.0 - x * x) * dp * dp);
        const double theta = 0.5 * M_PI * (x + 1.0);
        const double wt = 0.5 * M_PI * wi;
        const double er = std::cos(theta), ei = std::sin(theta);
        z[2 * i] = c + R * er;
        z[2 * i + 1] = R * ei;
        w[2 * i] = wt * R * er / M_PI;
        w[2 * i + 1] = wt * R * ei / M_PI;
    }
    return SCOCG_OK;
}

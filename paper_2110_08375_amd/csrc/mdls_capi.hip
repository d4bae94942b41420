// mdls_capi.hip -- the C ABI declared in mdls.h: argument checks on the host, then the
// per-precision drivers (instantiated in mdls_p1/2/4/8.hip).
#include <algorithm>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "mdls_cplx.hpp"
#include "mdls_split.hpp"

namespace mdls_impl {
MDLS_FOR_PRECISION(extern, 1)
MDLS_FOR_PRECISION(extern, 2)
MDLS_FOR_PRECISION(extern, 4)
MDLS_FOR_PRECISION(extern, 8)
MDLS_BATCH_FOR_PRECISION(extern, 2)
MDLS_BATCH_FOR_PRECISION(extern, 4)
MDLS_REFINE_FOR_PRECISION(extern, 4)
MDLS_REFINE_FOR_PRECISION(extern, 8)
MDLS_CPLX_FOR_PRECISION(extern, 1)
MDLS_CPLX_FOR_PRECISION(extern, 2)
MDLS_CPLX_FOR_PRECISION(extern, 4)
MDLS_CPLX_FOR_PRECISION(extern, 8)
}  // namespace mdls_impl

using namespace mdls_impl;

// ============================================================================ launch timing
namespace {
struct Timed {
    std::string name;
    int P;
    double work;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Timed> g_rec;
std::vector<hipEvent_t> g_pool;

hipEvent_t pool_get()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

namespace mdls_impl {
namespace {
thread_local int t_timing_off = 0;  // set inside calls that must not create timing events
}
bool timing_on() { return g_on && !t_timing_off; }

// Side streams: one per (host thread, device), created by mdls_init and destroyed by
// mdls_finalize; a solve never creates one.
namespace {
constexpr int kMaxDev = 16;
struct PerThread {
    SideStream ss{};
    bool ok = false;
};
thread_local PerThread t_side[kMaxDev];

std::atomic<int> g_lookahead{1};
std::atomic<int> g_panel_variant{0};
std::atomic<int> g_apply_grid_cap{0};
std::atomic<int> g_apply_wide_rows{768};
std::atomic<unsigned> g_spin_limit{1u << 22};
std::atomic<int> g_split_update{0};
std::atomic<int> g_cpanel{2};

// occupancy-derived capacity of the panel kernel, per (device, precision index, variant)
std::atomic<int> g_capacity[kMaxDev][4][2];

int pidx(int P) { return P == 1 ? 0 : P == 2 ? 1 : P == 4 ? 2 : 3; }

}  // namespace

SideStream *side_stream()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
    return t_side[dev].ok ? &t_side[dev].ss : nullptr;
}

Tuning tuning()
{
    Tuning t;
    t.lookahead = g_lookahead.load(std::memory_order_relaxed);
    t.panel_variant = g_panel_variant.load(std::memory_order_relaxed);
    t.apply_grid_cap = g_apply_grid_cap.load(std::memory_order_relaxed);
    t.apply_wide_rows = g_apply_wide_rows.load(std::memory_order_relaxed);
    t.spin_limit = g_spin_limit.load(std::memory_order_relaxed);
    t.split_update = g_split_update.load(std::memory_order_relaxed);
    t.cpanel = g_cpanel.load(std::memory_order_relaxed);
    return t;
}

// Workgroups of a concurrent trailing update of h rows (grid-stride beyond): two per CU for dd
// and qd, whose panels have slack; for od, whose panel and update are balanced, two per CU only
// while the update is much longer than the panel (h >= apply_wide_rows), then one per CU on 224
// CUs (measured on the n = 1024 solves).
int apply_grid_cap(int P, int h)
{
    const Tuning t = tuning();
    if (t.apply_grid_cap > 0) return t.apply_grid_cap;
    if (P < 8) return 448;
    return h >= t.apply_wide_rows ? 448 : 224;
}

int panel_capacity(int P, int m)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return 0;
    const int v = panel_variant_for(P, m);
    std::atomic<int> &slot = g_capacity[dev][pidx(P)][v];
    int c = slot.load(std::memory_order_relaxed);
    if (c > 0) return c;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 0;
    const PanelCfg cf = panel_cfg(P, v);
    int per_cu = 0;
    switch (P) {
    case 1: per_cu = panel_occupancy_t<1>(cf); break;
    case 2: per_cu = panel_occupancy_t<2>(cf); break;
    case 4: per_cu = panel_occupancy_t<4>(cf); break;
    default: per_cu = panel_occupancy_t<8>(cf); break;
    }
    c = per_cu * cus;
    if (c > 0) slot.store(c, std::memory_order_relaxed);
    return c;
}

void timing_begin(hipStream_t s, void **ev)
{
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t e = pool_get();
    if (e && hipEventRecord(e, s) != hipSuccess) {
        g_pool.push_back(e);  // not recorded: the launch goes untimed
        e = nullptr;
    }
    *ev = (void *)e;
}

void timing_end(hipStream_t s, void *ev, const char *name, int P, double work)
{
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t e = pool_get();
    if (!ev || !e) return;
    if (hipEventRecord(e, s) != hipSuccess) {
        g_pool.push_back(e);
        g_pool.push_back((hipEvent_t)ev);
        return;
    }
    g_rec.push_back(Timed{std::string(name), P, work, (hipEvent_t)ev, e});
}
}  // namespace mdls_impl

namespace {
template <template <int> class F, typename... Args>
int dispatch(int p, Args... args)
{
    switch (p) {
    case 1: return F<1>::run(args...);
    case 2: return F<2>::run(args...);
    case 4: return F<4>::run(args...);
    case 8: return F<8>::run(args...);
    }
    return -1;
}

template <int P>
struct SolveF {
    template <typename... A>
    static int run(A... a) { return solve_t<P>(a...); }
};
template <int P>
struct CQrF {
    template <typename... A>
    static int run(A... a) { return cqr_t<P>(a...); }
};
template <int P>
struct CApplyF {
    template <typename... A>
    static int run(A... a) { return capply_qh_t<P>(a...); }
};
template <int P>
struct CApplyQF {
    template <typename... A>
    static int run(A... a) { return capply_q_t<P>(a...); }
};
template <int P>
struct CFormQF {
    template <typename... A>
    static int run(A... a) { return cform_q_t<P>(a...); }
};
template <int P>
struct CBacksubF {
    template <typename... A>
    static int run(A... a) { return cbacksub_t<P>(a...); }
};
template <int P>
struct CSolveF {
    template <typename... A>
    static int run(A... a) { return csolve_t<P>(a...); }
};
template <int P>
struct QrF {
    template <typename... A>
    static int run(A... a) { return qr_t<P>(a...); }
};
template <int P>
struct ApplyF {
    template <typename... A>
    static int run(A... a) { return apply_qt_t<P>(a...); }
};
template <int P>
struct ApplyQF {
    template <typename... A>
    static int run(A... a) { return apply_q_t<P>(a...); }
};
template <int P>
struct FormQF {
    template <typename... A>
    static int run(A... a) { return form_q_t<P>(a...); }
};
template <int P>
struct FormWF {
    template <typename... A>
    static int run(A... a) { return form_w_t<P>(a...); }
};
template <int P>
struct BacksubF {
    template <typename... A>
    static int run(A... a) { return backsub_t<P>(a...); }
};

}  // namespace

// ============================================================================ static scratch
// Device memory of the allocation-free solve: a file-scope array of every device's code object,
// held until the process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in); it passes the device address hipGetSymbolAddress returns, looked
// up once per device with that device current.
static __device__ __align__(256) char scratch[MDLS_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::atomic<char *> g_scratch_ptr[kMaxDev];

// the device address of this device's scratch array; null if the lookup fails
char *scratch_ptr()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
    char *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (p) return p;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
    if (p) return p;
    void *q = nullptr;
    if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return nullptr;
    g_scratch_ptr[dev].store((char *)q, std::memory_order_release);
    return (char *)q;
}
}  // namespace

// ============================================================================ C ABI
extern "C" {

int mdls_max_rows(int p)
{
    if (!valid_p(p)) return 0;
    // the shape of the largest factorisations
    const PanelCfg cf = panel_cfg_for(p, 1 << 30);
    return kGMax * (cf.nt / leaf_width(p)) * cf.r;
}

size_t mdls_workspace_bytes(int p, int m, int n, int tile)
{
    if (!valid_p(p) || n < 1 || m < n || !valid_tile(tile)) return 0;
    return layout(p, m, n, tile).total;
}

int mdls_qr(int p, int m, int n, int tile, double *A, int lda, double *beta, double *T, int ldt, void *ws,
            size_t ws_bytes, int *d_info, hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || (T && n % tile != 0)) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (T && ldt < tile) return -9;
    if (!ws) return -10;
    if (ws_bytes < mdls_workspace_bytes(p, m, n, tile)) return -11;
    if (m > mdls_max_rows(p) || panel_groups(p, m) > panel_capacity(p, m)) return MDLS_EUNSUPPORTED;
    return dispatch<QrF>(p, m, n, tile, A, lda, beta, T, ldt, ws, d_info, stream);
}

int mdls_apply_qt(int p, int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *B,
                  int ldb, int nrhs, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (!T) return -7;
    if (ldt < tile) return -8;
    if (!B && nrhs > 0) return -9;
    if (ldb < m) return -10;
    if (nrhs < 0) return -11;
    if (!ws) return -12;
    if (ws_bytes < mdls_workspace_bytes(p, m, n, tile)) return -13;
    if (nrhs == 0) return 0;
    return dispatch<ApplyF>(p, m, n, tile, A, lda, T, ldt, B, ldb, nrhs, ws, stream);
}

int mdls_apply_q(int p, int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *B,
                 int ldb, int nrhs, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (!T) return -7;
    if (ldt < tile) return -8;
    if (!B && nrhs > 0) return -9;
    if (ldb < m) return -10;
    if (nrhs < 0) return -11;
    if (!ws) return -12;
    if (ws_bytes < mdls_workspace_bytes(p, m, n, tile)) return -13;
    if (nrhs == 0) return 0;
    return dispatch<ApplyQF>(p, m, n, tile, A, lda, T, ldt, B, ldb, nrhs, ws, stream);
}

int mdls_form_q(int p, int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *Q, int ldq,
                int ncols, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (!T) return -7;
    if (ldt < tile) return -8;
    if (!Q) return -9;
    if (ldq < m) return -10;
    if (ncols < 1 || ncols > m) return -11;
    if (!ws) return -12;
    if (ws_bytes < mdls_workspace_bytes(p, m, n, tile)) return -13;
    return dispatch<FormQF>(p, m, n, tile, A, lda, T, ldt, Q, ldq, ncols, ws, stream);
}

int mdls_form_w(int p, int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *W, int ldw,
                hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (!T) return -7;
    if (ldt < tile) return -8;
    if (!W) return -9;
    if (ldw < m) return -10;
    return dispatch<FormWF>(p, m, n, tile, A, lda, T, ldt, W, ldw, stream);
}

int mdls_backsub(int p, int n, int tile, const double *R, int ldr, double *x, void *ws, size_t ws_bytes, int *d_info,
                 hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (n < 1) return -2;
    if (!valid_tile(tile) || n % tile != 0) return -3;
    if (!R) return -4;
    if (ldr < n) return -5;
    if (!x) return -6;
    if (!ws) return -7;
    if (ws_bytes < mdls_workspace_bytes(p, n, n, tile)) return -8;
    if (!d_info) return -9;
    return dispatch<BacksubF>(p, n, tile, R, ldr, x, ws, d_info, stream);
}

size_t mdls_dd_gemm_tn_workspace_bytes(int w, int c)
{
    if (w < 1 || w > 16 || c < 1) return 0;
    return split_workspace_bytes(w, c);
}

int mdls_dd_gemm_tn(int method, int h, int w, int c, const double *Y, int ldy, const double *C, int ldc, double *S,
                    int lds, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (method != 0 && method != 1) return -1;
    if (h < 1 || (method == 1 && h > kSplitMaxRows)) return -2;
    if (w < 1 || (method == 1 && w > 16)) return -3;
    if (c < 1) return -4;
    if (!Y) return -5;
    if (ldy < h) return -6;
    if (!C) return -7;
    if (ldc < h) return -8;
    if (!S) return -9;
    if (lds < w) return -10;
    if (method == 1 && !ws) return -11;
    if (method == 1 && ws_bytes < split_workspace_bytes(w, c)) return -12;
    return dd_gemm_tn(method, h, w, c, Y, ldy, C, ldc, S, lds, ws, stream);
}

size_t mdls_cworkspace_bytes(int p, int m, int n, int tile)
{
    if (!valid_p(p) || n < 1 || m < n || !valid_tile(tile)) return 0;
    return clayout(p, m, n, tile).total;
}

int mdls_cqr(int p, int m, int n, int tile, double *A, int lda, double *T, int ldt, void *ws, size_t ws_bytes,
             hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (T && ldt < tile) return -8;
    if (!ws) return -9;
    if (ws_bytes < mdls_cworkspace_bytes(p, m, n, tile)) return -10;
    return dispatch<CQrF>(p, m, n, tile, A, lda, T, ldt, ws, stream);
}

int mdls_capply_qh(int p, int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *B,
                   int ldb, int nrhs, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (!T) return -7;
    if (ldt < tile) return -8;
    if (!B && nrhs > 0) return -9;
    if (ldb < m) return -10;
    if (nrhs < 0) return -11;
    if (!ws) return -12;
    if (ws_bytes < mdls_cworkspace_bytes(p, m, n, tile)) return -13;
    if (nrhs == 0) return 0;
    return dispatch<CApplyF>(p, m, n, tile, A, lda, T, ldt, B, ldb, nrhs, ws, stream);
}

int mdls_capply_q(int p, int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *B,
                  int ldb, int nrhs, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (!T) return -7;
    if (ldt < tile) return -8;
    if (!B && nrhs > 0) return -9;
    if (ldb < m) return -10;
    if (nrhs < 0) return -11;
    if (!ws) return -12;
    if (ws_bytes < mdls_cworkspace_bytes(p, m, n, tile)) return -13;
    if (nrhs == 0) return 0;
    return dispatch<CApplyQF>(p, m, n, tile, A, lda, T, ldt, B, ldb, nrhs, ws, stream);
}

int mdls_cform_q(int p, int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *Q, int ldq,
                 int ncols, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (!T) return -7;
    if (ldt < tile) return -8;
    if (!Q) return -9;
    if (ldq < m) return -10;
    if (ncols < 1 || ncols > m) return -11;
    if (!ws) return -12;
    if (ws_bytes < mdls_cworkspace_bytes(p, m, n, tile)) return -13;
    return dispatch<CFormQF>(p, m, n, tile, A, lda, T, ldt, Q, ldq, ncols, ws, stream);
}

int mdls_cbacksub(int p, int n, int tile, const double *R, int ldr, double *x, void *ws, size_t ws_bytes, int *d_info,
                  hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (n < 1) return -2;
    if (!valid_tile(tile) || n % tile != 0) return -3;
    if (!R) return -4;
    if (ldr < n) return -5;
    if (!x) return -6;
    if (!ws) return -7;
    if (ws_bytes < mdls_cworkspace_bytes(p, n, n, tile)) return -8;
    if (!d_info) return -9;
    return dispatch<CBacksubF>(p, n, tile, R, ldr, x, ws, d_info, stream);
}

int mdls_csolve(int p, int m, int n, int tile, double *A, int lda, double *b, double *x, void *ws, size_t ws_bytes,
                int *d_info, hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (!b) return -7;
    if (!x) return -8;
    if (!ws) return -9;
    if (ws_bytes < mdls_cworkspace_bytes(p, m, n, tile)) return -10;
    if (!d_info) return -11;
    return dispatch<CSolveF>(p, m, n, tile, A, lda, b, x, ws, d_info, stream);
}

int mdls_solve(int p, int m, int n, int tile, double *A, int lda, double *b, double *x, void *ws, size_t ws_bytes,
               int *d_info, hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (!b) return -7;
    if (!x) return -8;
    if (!ws) return -9;
    if (ws_bytes < mdls_workspace_bytes(p, m, n, tile)) return -10;
    if (!d_info) return -11;
    if (m > mdls_max_rows(p) || panel_groups(p, m) > panel_capacity(p, m)) return MDLS_EUNSUPPORTED;
    return dispatch<SolveF>(p, m, n, tile, A, lda, b, x, ws, d_info, stream);
}

int mdls_solve_noalloc(int p, int m, int n, int tile, double *A, int lda, double *b, double *x, int *d_info,
                       hipStream_t stream)
{
    if (!valid_p(p)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (!b) return -7;
    if (!x) return -8;
    if (!d_info) return -9;
    if (mdls_workspace_bytes(p, m, n, tile) > (size_t)MDLS_NOALLOC_SCRATCH_BYTES) return MDLS_ESCRATCH;
    if (m > mdls_max_rows(p) || panel_groups(p, m) > panel_capacity(p, m)) return MDLS_EUNSUPPORTED;
    char *ws = scratch_ptr();
    if (!ws) return MDLS_EHIP;
    // the solve clears its barrier counters and error flags with kernels before using them, so
    // what an earlier call left in the scratch does not matter; launch timing would create
    // events, so it is not recorded for this call
    t_timing_off = 1;
    const int rc = dispatch<SolveF>(p, m, n, tile, A, lda, b, x, (void *)ws, d_info, stream);
    t_timing_off = 0;
    return rc;
}

size_t mdls_batch_workspace_bytes(int p, int count)
{
    if (batch_variants(p) == 0 || count < 1) return 0;
    return batch_layout(p, count).total;
}

int mdls_batch_variants(int p) { return batch_variants(p); }

int mdls_batch_plan(int p, int count, const mdls_batch_desc *h_desc, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (batch_variants(p) == 0) return -1;
    if (count < 1) return -2;
    if (!h_desc) return -3;
    if (!ws) return -4;
    if (ws_bytes < mdls_batch_workspace_bytes(p, count)) return -5;
    std::vector<BatchDesc> plan((size_t)count);
    for (int i = 0; i < count; ++i) {
        const mdls_batch_desc &d = h_desc[i];
        if (d.n < 1 || d.m < d.n || d.m > kBatchRows || d.a_off < 0 || d.b_off < 0 || d.x_off < 0) return -3;
        plan[(size_t)i] = BatchDesc{d.m, d.n, d.a_off, d.b_off, d.x_off, i, 1};
    }
    const std::vector<int> slots = batch_schedule(plan);
    const int nslots = (int)slots.size();
    const BatchLayout L = batch_layout(p, count);
    char *w = (char *)ws;
    if (hipMemcpyAsync(w + L.plan, plan.data(), sizeof(BatchDesc) * plan.size(), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(w + L.slots, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(w + L.nslots, &nslots, sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess)
        return MDLS_EHIP;
    return hipStreamSynchronize(stream) == hipSuccess ? 0 : MDLS_EHIP;
}

int mdls_solve_batched(int p, int count, double *A, double *b, double *x, int variant, void *ws, size_t ws_bytes,
                       int *d_info, long long *d_times, hipStream_t stream)
{
    if (batch_variants(p) == 0) return -1;
    if (count < 1) return -2;
    if (!A) return -3;
    if (!b) return -4;
    if (!x) return -5;
    if (variant < 0 || variant >= batch_variants(p)) return -6;
    if (!ws) return -7;
    if (ws_bytes < mdls_batch_workspace_bytes(p, count)) return -8;
    if (!d_info) return -9;
    switch (p) {
    case 2: return batch_solve_t<2>(count, A, b, x, variant, ws, d_info, d_times, stream);
    case 4: return batch_solve_t<4>(count, A, b, x, variant, ws, d_info, d_times, stream);
    }
    return MDLS_EUNSUPPORTED;
}

int mdls_batch_autotune(int p, int count, const double *A_src, const double *b_src, size_t a_len, size_t b_len,
                        double *A, double *b, double *x, void *ws, size_t ws_bytes, int *d_info, float *ms,
                        hipStream_t stream)
{
    if (batch_variants(p) == 0) return -1;
    if (count < 1) return -2;
    if (!A_src) return -3;
    if (!b_src) return -4;
    if (!A) return -7;
    if (!b) return -8;
    if (!x) return -9;
    if (!ws) return -10;
    if (ws_bytes < mdls_batch_workspace_bytes(p, count)) return -11;
    if (!d_info) return -12;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MDLS_EHIP;
    int best = -1;
    float best_ms = 0.0f;
    int rc = 0;
    for (int v = 0; v < batch_variants(p) && rc == 0; ++v) {
        float t = 0.0f;
        for (int rep = 0; rep < 2 && rc == 0; ++rep) {  // the first run warms up
            if (hipMemcpyAsync(A, A_src, a_len * sizeof(double), hipMemcpyDeviceToDevice, stream) != hipSuccess ||
                hipMemcpyAsync(b, b_src, b_len * sizeof(double), hipMemcpyDeviceToDevice, stream) != hipSuccess ||
                hipEventRecord(e0, stream) != hipSuccess) {
                rc = MDLS_EHIP;
                break;
            }
            rc = mdls_solve_batched(p, count, A, b, x, v, ws, ws_bytes, d_info, nullptr, stream);
            if (rc == 0 && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                rc = MDLS_EHIP;
        }
        if (rc != 0) break;
        if (ms) ms[v] = t;
        if (best < 0 || t < best_ms) {
            best = v;
            best_ms = t;
        }
    }
    if (hipEventDestroy(e0) != hipSuccess || hipEventDestroy(e1) != hipSuccess) rc = rc ? rc : MDLS_EHIP;
    return rc != 0 ? rc : best;
}

int mdls_wall_clock_khz(int *khz)
{
    int dev = 0;
    if (!khz) return -1;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        return MDLS_EHIP;
    return 0;
}

size_t mdls_refined_workspace_bytes(int p_out, int m, int n, int tile)
{
    if ((p_out != 4 && p_out != 8) || n < 1 || m < n || !valid_tile(tile)) return 0;
    return align256(layout(2, m, n, tile).total) + refine_extra_bytes(p_out, m, n, tile);
}

int mdls_solve_refined(int p_out, int m, int n, int tile, const double *A, int lda, const double *b, double *x,
                       int iters, double *F, void *ws, size_t ws_bytes, int *d_info, double *d_norms,
                       hipStream_t stream)
{
    if (p_out != 4 && p_out != 8) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return -3;
    if (!valid_tile(tile) || n % tile != 0) return -4;
    if (!A) return -5;
    if (lda < m) return -6;
    if (!b) return -7;
    if (!x) return -8;
    if (iters < 1 || iters > 64) return -9;
    if (!F) return -10;
    if (!ws) return -11;
    if (ws_bytes < mdls_refined_workspace_bytes(p_out, m, n, tile)) return -12;
    if (!d_info) return -13;
    if (!d_norms) return -14;
    if (m > mdls_max_rows(2) || panel_groups(2, m) > panel_capacity(2, m)) return MDLS_EUNSUPPORTED;
    if (p_out == 4) return refine_t<4>(m, n, tile, A, lda, b, x, iters, F, ws, d_info, d_norms, stream);
    return refine_t<8>(m, n, tile, A, lda, b, x, iters, F, ws, d_info, d_norms, stream);
}

int mdls_init(void)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MDLS_EHIP;
    if (dev < 0 || dev >= kMaxDev) return MDLS_EUNSUPPORTED;
    PerThread &p = t_side[dev];
    if (p.ok) return 0;
    if (hipStreamCreateWithFlags(&p.ss.q, hipStreamNonBlocking) != hipSuccess) return MDLS_EHIP;
    // the events only order the two streams' kernels on this device: a device-scope release is
    // enough, as neither the host nor another device waits on them
    const unsigned evf = hipEventDisableTiming | hipEventReleaseToDevice;
    hipEvent_t *evs[3] = {&p.ss.ev_panel, &p.ss.ev_wide[0], &p.ss.ev_wide[1]};
    for (int e = 0; e < 3; ++e) {
        if (hipEventCreateWithFlags(evs[e], evf) != hipSuccess) {
            for (int f = 0; f < e; ++f) (void)hipEventDestroy(*evs[f]);
            (void)hipStreamDestroy(p.ss.q);
            return MDLS_EHIP;
        }
    }
    bool ok = scratch_ptr() != nullptr;
    for (int P : {1, 2, 4, 8})
        ok = ok && panel_capacity(P, 1) > 0 && panel_capacity(P, 1 << 30) > 0;
    if (!ok) {
        for (int f = 0; f < 3; ++f) (void)hipEventDestroy(*evs[f]);
        (void)hipStreamDestroy(p.ss.q);
        return MDLS_EHIP;
    }
    p.ok = true;
    return 0;
}

int mdls_finalize(void)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MDLS_EHIP;
    if (dev < 0 || dev >= kMaxDev) return MDLS_EUNSUPPORTED;
    PerThread &p = t_side[dev];
    if (!p.ok) return 0;
    p.ok = false;
    int rc = 0;
    if (hipStreamSynchronize(p.ss.q) != hipSuccess) rc = MDLS_EHIP;
    if (hipEventDestroy(p.ss.ev_panel) != hipSuccess || hipEventDestroy(p.ss.ev_wide[0]) != hipSuccess ||
        hipEventDestroy(p.ss.ev_wide[1]) != hipSuccess || hipStreamDestroy(p.ss.q) != hipSuccess)
        rc = MDLS_EHIP;
    return rc;
}

int mdls_set_tuning(int option, long value)
{
    switch (option) {
    case MDLS_TUNE_LOOKAHEAD:
        if (value != 0 && value != 1) return -2;
        g_lookahead.store((int)value);
        return 0;
    case MDLS_TUNE_PANEL_VARIANT:
        if (value != 0 && value != 1) return -2;
        g_panel_variant.store((int)value);
        return 0;
    case MDLS_TUNE_APPLY_GRID_CAP:
        if (value < 0 || value > 65536) return -2;
        g_apply_grid_cap.store((int)value);
        return 0;
    case MDLS_TUNE_APPLY_WIDE_ROWS:
        if (value < 0 || value > (1L << 30)) return -2;
        g_apply_wide_rows.store((int)value);
        return 0;
    case MDLS_TUNE_SPIN_LIMIT:
        if (value < 0 || value > (1L << 30)) return -2;
        g_spin_limit.store((unsigned)value);
        return 0;
    case MDLS_TUNE_SPLIT_UPDATE:
        if (value != 0 && value != 1) return -2;
        g_split_update.store((int)value);
        return 0;
    case MDLS_TUNE_CPANEL:
        if (value < 0 || value > 2) return -2;
        g_cpanel.store((int)value);
        return 0;
    }
    return -1;
}

long mdls_get_tuning(int option)
{
    const Tuning t = tuning();
    switch (option) {
    case MDLS_TUNE_LOOKAHEAD: return t.lookahead;
    case MDLS_TUNE_PANEL_VARIANT: return t.panel_variant;
    case MDLS_TUNE_APPLY_GRID_CAP: return t.apply_grid_cap;
    case MDLS_TUNE_APPLY_WIDE_ROWS: return t.apply_wide_rows;
    case MDLS_TUNE_SPIN_LIMIT: return (long)t.spin_limit;
    case MDLS_TUNE_SPLIT_UPDATE: return t.split_update;
    case MDLS_TUNE_CPANEL: return t.cpanel;
    }
    return -1;
}

int mdls_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return 0;
}

int mdls_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    int rc = 0;
    for (auto &t : g_rec) {
        if (hipEventSynchronize(t.b) != hipSuccess) rc = MDLS_EHIP;
        g_pool.push_back(t.a);
        g_pool.push_back(t.b);
    }
    g_rec.clear();
    return rc;
}

int mdls_timing_query(const char *name, int p, double *total_ms, long *launches, double *md_fmas)
{
    if (!name) return -1;
    if (!total_ms) return -3;
    if (!launches) return -4;
    if (!md_fmas) return -5;
    std::lock_guard<std::mutex> lk(g_mu);
    double ms = 0.0, work = 0.0;
    long cnt = 0;
    for (auto &t : g_rec) {
        if (name[0] && t.name != name) continue;
        if (p && t.P != p) continue;
        if (hipEventSynchronize(t.b) != hipSuccess) return MDLS_EHIP;
        float e = 0.f;
        if (hipEventElapsedTime(&e, t.a, t.b) != hipSuccess) return MDLS_EHIP;
        ms += e;
        work += t.work;
        ++cnt;
    }
    *total_ms = ms;
    *launches = cnt;
    *md_fmas = work;
    return 0;
}

int mdls_timing_kernels(char *buf, int buflen)
{
    if (!buf || buflen < 1) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<std::string> names;
    for (auto &t : g_rec) {
        bool seen = false;
        for (auto &n : names) seen = seen || (n == t.name);
        if (!seen) names.push_back(t.name);
    }
    std::string out;
    for (auto &n : names) out += n + "\n";
    std::strncpy(buf, out.c_str(), (size_t)buflen - 1);
    buf[buflen - 1] = 0;
    return (int)names.size();
}

const char *mdls_status_string(int status)
{
    if (status == 0) return "success";
    if (status == MDLS_EHIP) return "a HIP kernel launch failed";
    if (status == MDLS_EUNSUPPORTED) return "arguments valid but outside what the library supports";
    if (status == MDLS_ESCRATCH)
        return "the problem's workspace exceeds the static scratch of mdls_solve_noalloc (MDLS_NOALLOC_SCRATCH_BYTES)";
    if (status < 0 && status > -20) return "invalid argument (the negated status is its 1-based position)";
    return "unknown status";
}

}  // extern "C"

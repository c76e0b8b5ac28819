// P^{-1} z with persistent kernels: work buffers, dispatch, and the kernels whose
// transform length is a run-time value (the device code is in pinv_kernel.hpp).
#include <atomic>
#include <cstdlib>
#include <map>
#include <mutex>
#include <type_traits>

#include "pinv_kernel.hpp"

namespace tsfde {

static std::atomic<int> g_blocks_override{-1};
static std::atomic<bool> g_fixed_length{true};

ResidencyBudget& residency_budget(int dev, int ncu) {
    constexpr int kMaxDev = 64;
    static ResidencyBudget pools[kMaxDev];
    static std::once_flag once[kMaxDev];
    if (dev < 0 || dev >= kMaxDev) throw HipError{hipErrorInvalidDevice, "persistent P^-1: device index"};
    std::call_once(once[dev], [&] { pools[dev].reset(std::max(1, ncu / kXcds)); });
    return pools[dev];
}

// longest wait at a device-wide barrier: TSFDE_BARRIER_TIMEOUT_US microseconds (default 5 s)
unsigned long long barrier_ticks(int dev) {
    int khz = 0;
    TSFDE_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    const char* e = std::getenv("TSFDE_BARRIER_TIMEOUT_US");
    const double us = (e && *e) ? std::max(0.0, std::atof(e)) : 5e6;
    return (unsigned long long)(us * (double)std::max(khz, 1) / 1000.0);
}


template <typename T>
void ensure_work(Problem& P, PersistentWork<T>& W) {
    if (W.buf) return;
    const size_t ns = (size_t)spec_stride(P.N), nt = (size_t)spec_stride(P.Nt);
    TSFDE_HIP(hipMalloc(&W.buf, sizeof(T) * (size_t)(8 + kHB) * P.Nd));
    if (P.d == 2) {
        // sine-transform intermediates t1 [Nt][nt] and t2 [N][nt]; half spectra [H][ns]
        TSFDE_HIP(hipMalloc(&W.tt, sizeof(T) * ((size_t)P.Nt + P.N) * nt));
        TSFDE_HIP(hipMalloc(&W.spec, sizeof(cplx<T>) * (size_t)P.H * ns));
    }
    TSFDE_HIP(hipMalloc(&W.part, sizeof(double) * kRing * kMaxGrid * kNPart));
    TSFDE_HIP(hipMalloc(&W.bar, 64));
    TSFDE_HIP(hipMalloc(&W.iters, sizeof(long long)));
    TSFDE_HIP(hipMemset(W.buf, 0, sizeof(T) * (size_t)(8 + kHB) * P.Nd));
    P.bytes += sizeof(T) * (size_t)(8 + kHB) * P.Nd + sizeof(double) * kRing * kMaxGrid * kNPart + 64 + sizeof(long long) +
               (P.d == 2 ? sizeof(T) * ((size_t)P.Nt + P.N) * nt + sizeof(cplx<T>) * (size_t)P.H * ns : 0);
}

bool persistent_supported(const Problem& P) {
    // the sine transform shares the FFT length with the Toeplitz embedding when 2(N+1) = L
    return (!P.tau_ok || P.Ld == P.L) && P.L <= 8192;
}

// The forward substitution on the work buffers W (allocated by the caller); allocates nothing.
template <typename T>
static long long run_segments(Problem& P, const Dev<T>& D, PersistentWork<T>& W, const T* z, T* y, double inner_tol,
                              int inner_maxit, bool last_block, int extrap, int tblocks, hipStream_t st) {
    struct Release {  // the grid's CU slots go back however this call ends
        ResidencyTicket& t;
        ~Release() { t.release(); }
    } release{W.ticket};
    if (!P.capturing) launch_fill(reinterpret_cast<float*>(W.bar) + 1, 1, 0.0f, st);  // clear the abort word
    const int L = P.L;
    const int vpt = (L <= 2048) ? 8 : (L == 4096 ? 16 : 32);
    const int mode = (P.d == 1) ? SEG_1D : ((P.tau_ok || P.tau_pad) ? SEG_2D_TAU : SEG_2D_DIAG);
    int blocks = g_blocks_override;
    if (blocks <= 0 && P.pinv_blocks > 0) blocks = P.pinv_blocks;  // tuned grid
    if (tblocks) {
        // tau-block form: no inner iterations, no warm start (the caller has checked the path)
        if (mode != SEG_2D_TAU) throw HipError{hipErrorNotSupported, "tau-block P^-1 outside the 2D tau path"};
        if (!(g_fixed_length && launch_segments_fixed_tau<T>(P, D, W, z, y, last_block, blocks, st))) {
            if (vpt == 8) launch_segments<T, 8, SEG_2D_TAU, 0, true>(P, D, W, z, y, 0.0, 1, last_block, 0, blocks, st);
            else if (vpt == 16)
                launch_segments<T, 16, SEG_2D_TAU, 0, true>(P, D, W, z, y, 0.0, 1, last_block, 0, blocks, st);
            else launch_segments<T, 32, SEG_2D_TAU, 0, true>(P, D, W, z, y, 0.0, 1, last_block, 0, blocks, st);
        }
    } else if (mode == SEG_2D_TAU && g_fixed_length &&
               launch_segments_fixed<T>(P, D, W, z, y, inner_tol, inner_maxit, last_block, extrap, blocks, st)) {
        // done by a fixed-length kernel
    } else {
#define TSFDE_SEG(V, B) \
    launch_segments<T, V, B, 0, false>(P, D, W, z, y, inner_tol, inner_maxit, last_block, extrap, blocks, st)
#define TSFDE_SEG_MODES(V)                                       \
    do {                                                         \
        if (mode == SEG_1D) TSFDE_SEG(V, SEG_1D);                \
        else if (mode == SEG_2D_DIAG) TSFDE_SEG(V, SEG_2D_DIAG); \
        else TSFDE_SEG(V, SEG_2D_TAU);                           \
    } while (0)
        if (vpt == 8) TSFDE_SEG_MODES(8);
        else if (vpt == 16) TSFDE_SEG_MODES(16);
        else TSFDE_SEG_MODES(32);
#undef TSFDE_SEG_MODES
#undef TSFDE_SEG
    }
    if (P.capturing) return 0;  // counters read by the solver after the replay
    // iteration count and abort word into the problem's pinned scratch
    long long* it_h = reinterpret_cast<long long*>(P.host_scalars + 56);
    unsigned* abort_h = reinterpret_cast<unsigned*>(P.host_scalars + 57);
    TSFDE_HIP(hipMemcpyAsync(it_h, W.iters, sizeof(long long), hipMemcpyDeviceToHost, st));
    TSFDE_HIP(hipMemcpyAsync(abort_h, W.bar + 1, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    TSFDE_HIP(hipStreamSynchronize(st));
    if (*abort_h != 0u)
        throw HipError{hipErrorLaunchTimeOut,
                       "persistent P^-1: a device-wide barrier wait timed out (workgroups not co-resident)"};
    return *it_h;
}

template <typename T>
long long pinv_persistent_run(Problem& P, const Dev<T>& D, void*& wptr, const T* z, T* y, double inner_tol,
                              int inner_maxit, bool last_block, int extrap, int tblocks, hipStream_t st) {
    if (!wptr) wptr = new PersistentWork<T>();
    PersistentWork<T>& W = *static_cast<PersistentWork<T>*>(wptr);
    ensure_work(P, W);
    return run_segments(P, D, W, z, y, inner_tol, inner_maxit, last_block, extrap, tblocks, st);
}

// The transposed sweep of P^{-T} on the persistent kernels: the steps of the backward substitution
// taken in reversed order (step k = block row M - 1 - k) as a forward sweep with per-step weights on
// the history (PinvArgs.adj): zrev, dgrev, sigrev hold the reversed right-hand sides, block weights
// and shifts; urev (M slices) receives the solutions in the same reversed order.
long long pinv_adjoint_run(Problem& P, const double* zrev, const double* dgrev, const double* sigrev, double* urev,
                           double inner_tol, int inner_maxit, int extrap, hipStream_t st) {
    void*& wptr = P.pw64;
    if (!wptr) wptr = new PersistentWork<double>();
    PersistentWork<double>& W = *static_cast<PersistentWork<double>*>(wptr);
    ensure_work(P, W);
    Dev<double> D = P.f64;
    D.dg = const_cast<double*>(dgrev);  // read only by the sweep
    struct Sweep {  // the problem's forward settings come back however the sweep ends
        Problem& P;
        ~Sweep() {
            P.adjoint_sweep = false;
            P.sweep_sigma = nullptr;
        }
    } restore{P};
    P.adjoint_sweep = true;
    P.sweep_sigma = sigrev;
    set_persistent_blocks(-1);
    return run_segments<double>(P, D, W, zrev, urev, inner_tol, inner_maxit, false, extrap, 0, st);
}

void pinv_multi_run(std::vector<PinvMultiJob>& jobs, double inner_tol, int inner_maxit, int extrap, hipStream_t st) {
    // groups of one kernel form: (values per thread, mode, 1D transform length)
    struct Key {
        int vpt, mode, L;
        bool operator<(const Key& o) const {
            return vpt != o.vpt ? vpt < o.vpt : (mode != o.mode ? mode < o.mode : L < o.L);
        }
    };
    std::map<Key, std::vector<int>> groups;
    for (int i = 0; i < (int)jobs.size(); ++i) {
        Problem& P = *jobs[i].P;
        if (!persistent_supported(P)) throw HipError{hipErrorNotSupported, "multi P^-1: a problem without the persistent form"};
        const int L = P.L;
        const int vpt = (L <= 2048) ? 8 : (L == 4096 ? 16 : 32);
        const int mode = (P.d == 1) ? SEG_1D : ((P.tau_ok || P.tau_pad) ? SEG_2D_TAU : SEG_2D_DIAG);
        groups[Key{vpt, mode, P.d == 1 ? L : 0}].push_back(i);
    }
    for (auto& kv : groups) {
        std::vector<MultiItem<double>> items;
        for (int i : kv.second) {
            Problem& P = *jobs[i].P;
            if (!P.pw64) P.pw64 = new PersistentWork<double>();
            PersistentWork<double>& W = *static_cast<PersistentWork<double>*>(P.pw64);
            ensure_work(P, W);
            MultiItem<double> it{};
            it.P = &P;
            it.W = &W;
            it.a = make_pinv_args<double>(P, P.f64, W, jobs[i].z, jobs[i].y, inner_tol, inner_maxit, extrap);
            items.push_back(it);
        }
        const Key& k = kv.first;
#define TSFDE_MULTI(V, MD) launch_segments_multi<double, V, MD>(items, st)
        if (k.vpt == 8) {
            if (k.mode == SEG_1D) TSFDE_MULTI(8, SEG_1D);
            else if (k.mode == SEG_2D_TAU) TSFDE_MULTI(8, SEG_2D_TAU);
            else TSFDE_MULTI(8, SEG_2D_DIAG);
        } else if (k.vpt == 16) {
            if (k.mode == SEG_1D) TSFDE_MULTI(16, SEG_1D);
            else if (k.mode == SEG_2D_TAU) TSFDE_MULTI(16, SEG_2D_TAU);
            else TSFDE_MULTI(16, SEG_2D_DIAG);
        } else {
            if (k.mode == SEG_1D) TSFDE_MULTI(32, SEG_1D);
            else if (k.mode == SEG_2D_TAU) TSFDE_MULTI(32, SEG_2D_TAU);
            else TSFDE_MULTI(32, SEG_2D_DIAG);
        }
#undef TSFDE_MULTI
        for (size_t j = 0; j < kv.second.size(); ++j)
            jobs[kv.second[j]].iters = *reinterpret_cast<long long*>(items[j].P->host_scalars + 56);
    }
}

template <typename T>
static PersistentWork<T>& graph_work(Problem& P) {
    void*& wp = std::is_same<T, float>::value ? P.pw32 : P.pw64;
    if (!wp) throw HipError{hipErrorNotReady, "graph replay: the persistent P^-1 has not run on this problem"};
    return *static_cast<PersistentWork<T>*>(wp);
}

template <typename T>
static void graph_prepare(Problem& P, hipStream_t st) {
    PersistentWork<T>& W = graph_work<T>(P);
    launch_fill(reinterpret_cast<float*>(W.iters), 2, 0.0f, st);
    launch_fill(reinterpret_cast<float*>(W.bar) + 1, 1, 0.0f, st);
}

template <typename T>
static long long graph_finish(Problem& P, hipStream_t st) {
    PersistentWork<T>& W = graph_work<T>(P);
    long long* it_h = reinterpret_cast<long long*>(P.host_scalars + 56);
    unsigned* abort_h = reinterpret_cast<unsigned*>(P.host_scalars + 57);
    TSFDE_HIP(hipMemcpyAsync(it_h, W.iters, sizeof(long long), hipMemcpyDeviceToHost, st));
    TSFDE_HIP(hipMemcpyAsync(abort_h, W.bar + 1, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    TSFDE_HIP(hipStreamSynchronize(st));
    if (*abort_h != 0u)
        throw HipError{hipErrorLaunchTimeOut, "graph replay: a device-wide barrier wait of P^-1 timed out"};
    return *it_h;
}

void pinv_graph_prepare(Problem& P, bool f32, hipStream_t st) {
    if (f32) graph_prepare<float>(P, st);
    else graph_prepare<double>(P, st);
}

long long pinv_graph_finish(Problem& P, bool f32, hipStream_t st) {
    return f32 ? graph_finish<float>(P, st) : graph_finish<double>(P, st);
}

// ---------------------------------------------------------------------------
// allocation-free form (tsfde_apply_P_inv_noalloc): the work buffers of PersistentWork<double> laid
// out in one static device array
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

struct NoAllocLayout {  // byte offsets into the scratch
    size_t buf, tt, spec, part, bar, iters, end;
};

NoAllocLayout noalloc_layout(const Problem& P) {
    NoAllocLayout l{};
    const size_t ns = (size_t)spec_stride(P.N), nt = (size_t)spec_stride(P.Nt);
    size_t o = 0;
    l.buf = o;
    o = align_up(o + sizeof(double) * (size_t)(8 + kHB) * P.Nd);
    l.tt = o;
    if (P.d == 2) o = align_up(o + sizeof(double) * ((size_t)P.Nt + P.N) * nt);
    l.spec = o;
    if (P.d == 2) o = align_up(o + sizeof(cplx<double>) * (size_t)P.H * ns);
    l.part = o;
    o = align_up(o + sizeof(double) * kRing * kMaxGrid * kNPart);
    l.bar = o;
    o = align_up(o + 64);
    l.iters = o;
    o = align_up(o + sizeof(long long));
    l.end = o;
    return l;
}

// the scratch's device address on each device, looked up once per device with that device current
unsigned char* scratch_address(int dev) {
    constexpr int kMaxDev = 64;
    static std::mutex mx;
    static unsigned char* addr[kMaxDev] = {};
    if (dev < 0 || dev >= kMaxDev) throw HipError{hipErrorInvalidDevice, "apply_P_inv_noalloc: device index"};
    std::lock_guard<std::mutex> lk(mx);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) throw HipError{e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)"};
        addr[dev] = static_cast<unsigned char*>(p);
    }
    return addr[dev];
}
}  // namespace

size_t pinv_noalloc_bytes(const Problem& P) { return noalloc_layout(P).end; }

long long pinv_persistent_run_noalloc(Problem& P, const double* z, double* y, double inner_tol, int inner_maxit,
                                      int extrap, int tblocks, hipStream_t st) {
    const NoAllocLayout l = noalloc_layout(P);
    if (l.end > kNoAllocScratchBytes)
        throw HipError{hipErrorOutOfMemory, "apply_P_inv_noalloc: the problem needs more than the static scratch"};
    int dev = 0;
    TSFDE_HIP(hipGetDevice(&dev));
    unsigned char* base = scratch_address(dev);
    PersistentWork<double> W;
    W.buf = reinterpret_cast<double*>(base + l.buf);
    W.tt = P.d == 2 ? reinterpret_cast<double*>(base + l.tt) : nullptr;
    W.spec = P.d == 2 ? reinterpret_cast<cplx<double>*>(base + l.spec) : nullptr;
    W.part = reinterpret_cast<double*>(base + l.part);
    W.bar = reinterpret_cast<unsigned*>(base + l.bar);
    W.iters = reinterpret_cast<long long*>(base + l.iters);
    // the scratch keeps the previous call's contents: the work vectors start from zero, as the
    // problem-owned buffers do (the counters are cleared by the launches themselves)
    launch_fill(reinterpret_cast<float*>(base), (long long)(l.part / sizeof(float)), 0.0f, st);
    return run_segments<double>(P, P.f64, W, z, y, inner_tol, inner_maxit, true, extrap, tblocks, st);
}

template <typename T>
void pinv_persistent_free(void* wptr) {
    if (!wptr) return;
    PersistentWork<T>* W = static_cast<PersistentWork<T>*>(wptr);
    void* ptrs[] = {W->buf, W->tt, W->spec, W->part, W->bar, W->iters};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete W;
}

static thread_local bool t_shared_launch = false;
template <typename T>
void launch_far_history(const Problem& P, const Dev<T>& D, const T* y, T* w, const T* z, int sa, int cnt,
                        hipStream_t st) {
    if (cnt < 1 || cnt > kHB || sa + cnt > P.M) throw HipError{hipErrorInvalidValue, "far_history step range"};
    hipLaunchKernelGGL(far_history<T>, dim3((unsigned)((P.Nd + 63) / 64)), dim3(256), 0, st, y, w, D.epad, z,
                       D.gamma1, D.gamma2, sa, cnt, P.Nd, (const T*)nullptr);
    TSFDE_HIP(hipGetLastError());
}

void set_shared_launch(bool on) { t_shared_launch = on; }
bool shared_launch() { return t_shared_launch; }

void set_persistent_blocks(int g) { g_blocks_override = g; }
void set_persistent_fixed_length(bool on) { g_fixed_length = on; }

template void ensure_work<double>(Problem&, PersistentWork<double>&);
template void ensure_work<float>(Problem&, PersistentWork<float>&);
template long long pinv_persistent_run<double>(Problem&, const Dev<double>&, void*&, const double*, double*, double,
                                               int, bool, int, int, hipStream_t);
template long long pinv_persistent_run<float>(Problem&, const Dev<float>&, void*&, const float*, float*, double, int,
                                              bool, int, int, hipStream_t);
template void launch_far_history<double>(const Problem&, const Dev<double>&, const double*, double*, const double*, int,
                                         int, hipStream_t);
template void launch_far_history<float>(const Problem&, const Dev<float>&, const float*, float*, const float*, int, int,
                                        hipStream_t);
template void pinv_persistent_free<double>(void*);
template void pinv_persistent_free<float>(void*);

}  // namespace tsfde

// C ABI (include/xfft.h) and the host drivers of the solver: plain FP64 CG
// (Algorithm 1), FP32 CG inside FP64 iterative refinement, step-level
// operator / preconditioner applications.
#include "../../include/xfft.h"
#include "kernels.h"
#include "enriched.h"

#include <chrono>
#include <cmath>
#include <array>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

using namespace xfft;

namespace {

#define HIP_OK(x)                                   \
    do {                                            \
        if ((x) != hipSuccess) return XFFT_EDEVICE; \
    } while (0)

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool size_ok(int n) {
    if (n < 4 || n > 4096 || (n & 1)) return false;
    int m = n;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1;
}

bool lame_ok(const double *lame, int np) {
    for (int q = 0; q < np; ++q) {
        const double l = lame[2 * q], m = lame[2 * q + 1];
        if (!std::isfinite(l) || !std::isfinite(m) || !(m > 0.0) || !(3.0 * l + 2.0 * m > 0.0)) return false;
    }
    return true;
}

template <typename T> void free_work(Work<T> &w) {
    T **ptrs[] = {&w.u, &w.f, &w.d, &w.z, &w.ue, &w.fe, &w.de, &w.ze, &w.cutbuf};
    for (T **q : ptrs) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
    }
    if (w.spec) (void)hipFree(w.spec);
    w.spec = nullptr;
    w.cap = 0;
}

template <typename T> int alloc_work(xfft_problem *p, Work<T> &w, int cap) {
    if (w.cap >= cap) return XFFT_OK;
    free_work(w);
    const Geometry &g = p->g;
    const size_t nf = (size_t)cap * 3 * g.N, ne = (size_t)cap * 3 * (g.nX > 0 ? g.nX : 1);
    // half spectrum in the larger (padded) of its two layouts
    const size_t ns = (size_t)cap * 3 * g.n2 * g.n1 * spec_row_stride(g.nh);
    const size_t nc = (size_t)cap * (size_t)cut_rows(g.nirr > 0 ? g.nirr : 1) * 48;
    T **fe_ptrs[] = {&w.u, &w.f, &w.d, &w.z};
    for (T **q : fe_ptrs)
        if (hipMalloc(q, nf * sizeof(T)) != hipSuccess) return XFFT_ENOMEM;
    T **en_ptrs[] = {&w.ue, &w.fe, &w.de, &w.ze};
    for (T **q : en_ptrs)
        if (hipMalloc(q, ne * sizeof(T)) != hipSuccess) return XFFT_ENOMEM;
    if (hipMalloc(&w.spec, ns * sizeof(cpx<T>)) != hipSuccess) return XFFT_ENOMEM;
    if (hipMalloc(&w.cutbuf, nc * sizeof(T)) != hipSuccess) return XFFT_ENOMEM;
    w.cap = cap;
    return XFFT_OK;
}

int ensure_state(xfft_problem *p, int cap) {
    if (p->scal_cap >= cap) return XFFT_OK;
    if (p->partial) (void)hipFree(p->partial);
    if (p->scal) (void)hipFree(p->scal);
    if (p->flags) (void)hipFree(p->flags);
    if (p->ebar) (void)hipFree(p->ebar);
    if (p->host_flags) (void)hipHostFree(p->host_flags);
    if (p->sum7) (void)hipFree(p->sum7);
    p->partial = nullptr; p->scal = nullptr; p->flags = nullptr; p->ebar = nullptr; p->host_flags = nullptr;
    p->sum7 = nullptr;
    if (hipMalloc(&p->partial, sizeof(double) * NPART * (size_t)p->nslots * cap) != hipSuccess ||
        hipMalloc(&p->sum7, sizeof(double) * 7 * cap) != hipSuccess ||
        hipMalloc(&p->scal, sizeof(Scalars) * cap) != hipSuccess ||
        hipMalloc(&p->flags, sizeof(Flags) * cap) != hipSuccess ||
        hipMalloc(&p->ebar, sizeof(double) * 6 * cap) != hipSuccess ||
        hipHostMalloc(&p->host_flags, sizeof(Flags) * cap, hipHostMallocDefault) != hipSuccess)
        return XFFT_ENOMEM;
    p->scal_cap = cap;
    return XFFT_OK;
}

// Step size of eq. stepsize: 2 / (C_- + C_+), C_-/C_+ the smallest/largest
// eigenvalue of the phase stiffnesses (3 lambda + 2 mu once, 2 mu five times).
double step_size(const std::vector<double> &lame) {
    double cmin = INFINITY, cmax = -INFINITY;
    for (size_t q = 0; q + 1 < lame.size(); q += 2) {
        const double a = 3.0 * lame[q] + 2.0 * lame[q + 1], b = 2.0 * lame[q + 1];
        cmin = std::fmin(cmin, std::fmin(a, b));
        cmax = std::fmax(cmax, std::fmax(a, b));
    }
    return 2.0 / (cmin + cmax);
}

// Upload per-rhs macro strains and reset scalars / flags.
int reset_state(xfft_problem *p, int nrhs, const double *ebar_host) {
    std::vector<Scalars> sc(nrhs);
    const double s0 = step_size(p->lame_host);
    for (int r = 0; r < nrhs; ++r) {
        std::memset(&sc[r], 0, sizeof(Scalars));
        sc[r].tol = p->rtol;
        sc[r].tol_inner = p->inner_rtol;
        sc[r].s0 = s0;
    }
    HIP_OK(hipMemcpyAsync(p->scal, sc.data(), sizeof(Scalars) * nrhs, hipMemcpyHostToDevice, p->stream));
    HIP_OK(hipMemsetAsync(p->flags, 0, sizeof(Flags) * nrhs, p->stream));
    if (ebar_host) HIP_OK(hipMemcpyAsync(p->ebar, ebar_host, sizeof(double) * 6 * nrhs, hipMemcpyHostToDevice, p->stream));
    return XFFT_OK;
}

int read_flags(xfft_problem *p, int nrhs, std::vector<Flags> &out) {
    HIP_OK(hipMemcpyAsync(p->host_flags, p->flags, sizeof(Flags) * nrhs, hipMemcpyDeviceToHost, p->stream));
    HIP_OK(hipStreamSynchronize(p->stream));
    out.assign(reinterpret_cast<Flags *>(p->host_flags), reinterpret_cast<Flags *>(p->host_flags) + nrhs);
    return XFFT_OK;
}

// One CG iteration of Algorithm 1 on the work fields of precision T.
template <typename T>
void cg_iteration(xfft_problem *p, Work<T> &w, const Tables<T> &tb, int nrhs, int parity, int crit) {
    hipStream_t s = p->stream;
    // the stress integral is only needed when the criterion tracks <sigma> (criterion 0)
    launch_operator<T>(p, w, tb, w.d, w.de, w.z, w.ze, false, (T)1, nrhs, p->flags, parity, nullptr, s, crit == 0);
    launch_scalars(p, SC_ALPHA, crit, nrhs, parity, nullptr, s, sizeof(T) == 8);
    launch_green_forward<T>(p, w, tb, w.f, w.z, nrhs, p->flags, parity, s, 1, nullptr);
    launch_scalars(p, SC_BETA, crit, nrhs, parity, nullptr, s, sizeof(T) == 8);
    launch_green_inverse<T>(p, w, tb, 1, nullptr, nrhs, p->flags, parity, s, 1);
}

// Initial preconditioned residual: d = P^-1 f, res2, convergence flags.
template <typename T>
void cg_start(xfft_problem *p, Work<T> &w, const Tables<T> &tb, int nrhs, int crit) {
    hipStream_t s = p->stream;
    launch_green_forward<T>(p, w, tb, w.f, nullptr, nrhs, nullptr, 0, s, 0, nullptr);
    launch_green_inverse<T>(p, w, tb, 2, nullptr, nrhs, nullptr, 0, s, 2);
    launch_scalars(p, SC_INIT_RES, crit, nrhs, 0, nullptr, s, sizeof(T) == 8);
}

void drop_graph(xfft_problem *p) {
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    p->graph_key[0] = -1;
}

// Enqueue k CG iterations (parities 0, 1, ...; k even) on the problem's stream.
template <typename T>
void enqueue_iterations(xfft_problem *p, Work<T> &w, const Tables<T> &tb, int nrhs, int crit, int k) {
    for (int it = 0; it < k; ++it) cg_iteration<T>(p, w, tb, nrhs, it & 1, crit);
}

// Capture k iterations into the problem's graph (reused while the launch
// configuration and the work buffers are unchanged).
template <typename T>
int ensure_graph(xfft_problem *p, Work<T> &w, const Tables<T> &tb, int nrhs, int crit, int k) {
    const int key[4] = {(int)sizeof(T), nrhs, crit, k};
    const void *ptrs[3] = {w.u, p->partial, w.cutbuf};
    if (p->graph_exec && std::memcmp(key, p->graph_key, sizeof(key)) == 0 &&
        std::memcmp(ptrs, p->graph_ptrs, sizeof(ptrs)) == 0)
        return XFFT_OK;
    drop_graph(p);
    hipStream_t s = p->stream;
    HIP_OK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    enqueue_iterations<T>(p, w, tb, nrhs, crit, k);
    if (hipStreamEndCapture(s, &p->graph) != hipSuccess) { p->graph = nullptr; return XFFT_EDEVICE; }
    if (hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
        drop_graph(p);
        return XFFT_EDEVICE;
    }
    std::memcpy(p->graph_key, key, sizeof(key));
    std::memcpy(p->graph_ptrs, ptrs, sizeof(ptrs));
    return XFFT_OK;
}

int check_period(const xfft_problem *p) {
    int every = p->check_every > 0 ? p->check_every : 8;
    return every + (every & 1);          // even: a replay starts at parity 0 again
}

// Iterate until no right-hand side is active; returns iterations run.
template <typename T>
int cg_loop(xfft_problem *p, Work<T> &w, const Tables<T> &tb, int nrhs, int crit, int *rc) {
    std::vector<Flags> fl;
    *rc = read_flags(p, nrhs, fl);
    if (*rc) return 0;
    bool any = false;
    for (int r = 0; r < nrhs; ++r) any |= fl[r].active[0] != 0;
    int it = 0;
    const int every = check_period(p);
    const bool graph = p->use_graph && !p->prof_on;
    if (graph && any) {
        *rc = ensure_graph<T>(p, w, tb, nrhs, crit, every);
        if (*rc) return 0;
    }
    while (any && it < p->maxit) {
        if (graph) {
            if (hipGraphLaunch(p->graph_exec, p->stream) != hipSuccess) { *rc = XFFT_EDEVICE; return it; }
            it += every;
        } else {
            cg_iteration<T>(p, w, tb, nrhs, it & 1, crit);
            ++it;
        }
        if (graph || it % every == 0 || it >= p->maxit) {
            *rc = read_flags(p, nrhs, fl);
            if (*rc) return it;
            any = false;
            for (int r = 0; r < nrhs; ++r) any |= fl[r].active[it & 1] != 0;
        }
    }
    return it;
}

// The autotuners' results are kept per (grid, precision, loads) for the
// process; distinct problems may be solved from several threads at once, so
// the caches are read and written under a lock (the timing runs outside it).
using TuneKey = std::array<int, 5>;
std::mutex g_tune_mu;

bool tune_lookup(std::map<TuneKey, int> &cache, const TuneKey &key, int &value) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = cache.find(key);
    if (it == cache.end()) return false;
    value = it->second;
    return true;
}

void tune_store(std::map<TuneKey, int> &cache, const TuneKey &key, int value) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    cache[key] = value;
}

// Choose the regular-voxel operator depth (planes per block) by timing the
// candidates in the solve's launch configuration.
template <typename T>
int autotune_depth(xfft_problem *p, Work<T> &w, const Tables<T> &tb, int nrhs) {
    static std::map<TuneKey, int> cache;
    const TuneKey key = {p->g.n0, p->g.n1, p->g.n2, (int)sizeof(T), nrhs};
    int cached = 0;
    if (tune_lookup(cache, key, cached)) {
        set_depth(p->slots, p->g, cached);
        return XFFT_OK;
    }
    hipStream_t s = p->stream;
    HIP_OK(hipMemsetAsync(w.d, 0, sizeof(T) * 3 * p->g.N * nrhs, s));
    if (p->g.nX) HIP_OK(hipMemsetAsync(w.de, 0, sizeof(T) * 3 * p->g.nX * nrhs, s));
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    int best = p->slots.kz;
    float best_ms = 1e30f;
    for (int kz : {4, 8, 16, 32}) {
        if (kz > p->g.n2) continue;
        set_depth(p->slots, p->g, kz);
        launch_operator<T>(p, w, tb, w.d, w.de, w.z, w.ze, false, (T)1, nrhs, nullptr, 0, nullptr, s, false);
        (void)hipEventRecord(e0, s);
        for (int rep = 0; rep < 10; ++rep)
            launch_operator<T>(p, w, tb, w.d, w.de, w.z, w.ze, false, (T)1, nrhs, nullptr, 0, nullptr, s, false);
        (void)hipEventRecord(e1, s);
        float ms = 0.0f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) break;
        if (ms < best_ms) { best_ms = ms; best = kz; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_depth(p->slots, p->g, best);
    tune_store(cache, key, best);
    return XFFT_OK;
}

// Choose the Green-operator kernels (xy-plane kernels or separate x and y
// passes, z-pass tile) by timing a forward and inverse application of every
// variant the grid has in the solve's launch configuration; results are cached
// per (grid, precision, loads) for the process.
template <typename T>
int autotune_fft(xfft_problem *p, Work<T> &w, const Tables<T> &tb, int nrhs) {
    const int pi = sizeof(T) == 8 ? 1 : 0;
    if (p->fft_tuned[pi]) return XFFT_OK;
    static std::map<TuneKey, int> cache;
    const TuneKey key = {p->g.n0, p->g.n1, p->g.n2, (int)sizeof(T), nrhs};
    const int have = fft_variants<T>(p->g);
    int best = 0;
    if (tune_lookup(cache, key, best)) {
        // chosen before for this grid
    } else if (have) {
        hipStream_t s = p->stream;
        // zero input: the timed transforms read defined values
        HIP_OK(hipMemsetAsync(w.f, 0, sizeof(T) * 3 * p->g.N * nrhs, s));
        if (p->g.nX) HIP_OK(hipMemsetAsync(w.fe, 0, sizeof(T) * 3 * p->g.nX * nrhs, s));
        hipEvent_t e0, e1;
        HIP_OK(hipEventCreate(&e0));
        HIP_OK(hipEventCreate(&e1));
        // two interleaved rounds over the variants, the faster of each variant's
        // two timings counts; another variant replaces the default only when it
        // is at least 3 % faster (timings of close variants scatter by a few %)
        float t[4] = {1e30f, 1e30f, 1e30f, 1e30f};
        bool ok = true;
        for (int round = 0; round < 2 && ok; ++round) {
            for (int v = 0; v < 4 && ok; ++v) {
                if ((v & ~have) != 0) continue;
                p->fft_plane[pi] = (v & 1) ? 0 : 1;
                p->fft_ztile[pi] = (v >> 1) & 1;
                launch_green_forward<T>(p, w, tb, w.f, nullptr, nrhs, nullptr, 0, s, 0, nullptr);
                launch_green_inverse<T>(p, w, tb, 2, nullptr, nrhs, nullptr, 0, s, 2);
                (void)hipEventRecord(e0, s);
                for (int rep = 0; rep < 5; ++rep) {
                    launch_green_forward<T>(p, w, tb, w.f, nullptr, nrhs, nullptr, 0, s, 0, nullptr);
                    launch_green_inverse<T>(p, w, tb, 2, nullptr, nrhs, nullptr, 0, s, 2);
                }
                (void)hipEventRecord(e1, s);
                float ms = 0.0f;
                if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    ok = false;
                    break;
                }
                if (ms < t[v]) t[v] = ms;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        float best_ms = t[0];
        for (int v = 1; v < 4; ++v)
            if (t[v] < 0.97f * t[0] && t[v] < best_ms) { best_ms = t[v]; best = v; }
        if (hipGetLastError() != hipSuccess) return XFFT_EDEVICE;
        tune_store(cache, key, best);
    }
    p->fft_plane[pi] = (best & 1) ? 0 : 1;
    p->fft_ztile[pi] = (best >> 1) & 1;
    p->fft_tuned[pi] = true;
    drop_graph(p);
    return XFFT_OK;
}

// Cached voxel matrices for the CG iterations of precision T in the launch
// configuration (nrhs, stress integral on or off): never, always, or -- the
// default -- whichever of the moment form and the cached matrices applies the
// operator faster, timed once per precision; the tables are (re)built for the
// current moduli when used.  Allocation failure falls back to the moment form.
template <typename T>
int ensure_voxel_matrices(xfft_problem *p, Work<T> &w, const Tables<T> &tb, int nrhs, bool stress) {
    const int pi = sizeof(T) == 8 ? 1 : 0;
    if (p->g.nirr == 0 || p->vm_mode == 0 || nrhs > VM_MAXR) {
        if (p->vm_on[pi]) drop_graph(p);
        p->vm_on[pi] = false;
        return XFFT_OK;
    }
    auto have = [&]() { return p->vm_valid && (pi ? p->vm64 != nullptr : p->vm32 != nullptr); };
    auto build = [&]() -> int {
        const int r = build_voxel_matrices(p, pi == 0 || p->vm32 != nullptr, pi == 1 || p->vm64 != nullptr);
        return r == -3 ? XFFT_EDEVICE : r;       // -2: not enough memory, use the moment form
    };
    if (p->vm_mode == 1 || p->vm_tuned[pi]) {
        const bool want = p->vm_mode == 1 || p->vm_on[pi];
        if (want && !have()) {
            const int r = build();
            if (r == XFFT_EDEVICE) return r;
            if (r) { p->vm_on[pi] = false; drop_graph(p); return XFFT_OK; }
        }
        if (p->vm_on[pi] != want) drop_graph(p);
        p->vm_on[pi] = want;
        return XFFT_OK;
    }
    if (!have()) {
        // the automatic choice only tries tables that fit in a quarter of the
        // free device memory (with the FP64 table the FP32 one is rounded from)
        size_t free_b = 0, total_b = 0;
        const size_t need = (size_t)p->g.nirr * VM_STRIDE * (sizeof(double) + (pi == 0 ? sizeof(float) : 0));
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || need > free_b / 4) {
            p->vm_on[pi] = false;
            p->vm_tuned[pi] = true;
            return XFFT_OK;
        }
        const int r = build();
        if (r == XFFT_EDEVICE) return r;
        if (r) { p->vm_on[pi] = false; p->vm_tuned[pi] = true; return XFFT_OK; }
    }
    hipStream_t s = p->stream;
    HIP_OK(hipMemsetAsync(w.d, 0, sizeof(T) * 3 * p->g.N * nrhs, s));
    if (p->g.nX) HIP_OK(hipMemsetAsync(w.de, 0, sizeof(T) * 3 * p->g.nX * nrhs, s));
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    float best_ms[2] = {1e30f, 1e30f};
    for (int mode = 0; mode < 2; ++mode) {
        p->vm_on[pi] = mode == 1;
        launch_operator<T>(p, w, tb, w.d, w.de, w.z, w.ze, false, (T)1, nrhs, nullptr, 0, nullptr, s, stress);
        (void)hipEventRecord(e0, s);
        for (int rep = 0; rep < 10; ++rep)
            launch_operator<T>(p, w, tb, w.d, w.de, w.z, w.ze, false, (T)1, nrhs, nullptr, 0, nullptr, s, stress);
        (void)hipEventRecord(e1, s);
        float ms = 0.0f;
        if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best_ms[mode] = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->vm_on[pi] = best_ms[1] < best_ms[0];
    p->vm_tuned[pi] = true;
    if (!p->vm_on[pi]) {
        // keep only tables some precision uses
        if (pi == 0 && p->vm32) { (void)hipFree(p->vm32); p->vm32 = nullptr; }
        if (pi == 1 && p->vm64 && !p->vm_on[0]) { (void)hipFree(p->vm64); p->vm64 = nullptr; }
        if (!p->vm32 && !p->vm64) p->vm_valid = false;
    }
    drop_graph(p);
    return XFFT_OK;
}

// Average stress (Mandel) of the FP64 iterate in w64.u for every rhs; optional voxel stress.
// <sigma> (and voxel stresses when vstress_dev is set) of the FP64 iterate.
// sigma_ready: the scalars already hold the exact <sigma> of that iterate (the
// last FP64 residual pass of the refinement loop computed it and the iterate
// has not changed since), so without voxel stresses no further pass is needed.
int final_outputs(xfft_problem *p, int nrhs, double *avg_host, double *vstress_dev, bool sigma_ready) {
    hipStream_t s = p->stream;
    if (sigma_ready && !vstress_dev) {
        std::vector<Scalars> sc(nrhs);
        HIP_OK(hipMemcpyAsync(sc.data(), p->scal, sizeof(Scalars) * nrhs, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        for (int r = 0; r < nrhs; ++r)
            for (int q = 0; q < 6; ++q) avg_host[6 * r + q] = sc[r].sigma[q];
        return XFFT_OK;
    }
    Work<double> &w = p->w64;
    launch_operator<double>(p, w, p->t64, w.u, w.ue, w.z, w.ze, true, 1.0, nrhs, nullptr, 0, vstress_dev, s);
    launch_scalars(p, SC_SUM_ONLY, 0, nrhs, 0, p->sum7, s, true);
    std::vector<double> sum(7 * nrhs);
    HIP_OK(hipMemcpyAsync(sum.data(), p->sum7, sizeof(double) * 7 * nrhs, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const double V = (double)p->g.N, r2 = std::sqrt(2.0);
    for (int r = 0; r < nrhs; ++r) {
        const double *v = &sum[7 * r];
        double *o = avg_host + 6 * r;
        o[0] = v[1] / V; o[1] = v[2] / V; o[2] = v[3] / V;
        o[3] = r2 * v[4] / V; o[4] = r2 * v[5] / V; o[5] = r2 * v[6] / V;
    }
    return XFFT_OK;
}

// Solve nrhs loads whose macro strains are in ebar_host; solution left in w64.u/ue.
// u0, ue0: device start iterates [nrhs][3][N], [nrhs][3][nX] (FP64, voxel
// units), or null to start from u = 0.
int solve_block(xfft_problem *p, int nrhs, const double *ebar_host, std::vector<int> &iters,
                std::vector<int> &outer, std::vector<double> &res_rel, int *status,
                const double *u0 = nullptr, const double *ue0 = nullptr) {
    int rc = alloc_work<double>(p, p->w64, nrhs);
    if (rc) return rc;
    if (p->precision == XFFT_MIXED) {
        rc = alloc_work<float>(p, p->w32, nrhs);
        if (rc) return rc;
    }
    rc = ensure_state(p, nrhs);
    if (rc) return rc;
    if (p->autotune && !p->tuned) {
        rc = (p->precision == XFFT_MIXED) ? autotune_depth<float>(p, p->w32, p->t32, nrhs)
                                          : autotune_depth<double>(p, p->w64, p->t64, nrhs);
        if (rc) return rc;
        p->tuned = true;
        drop_graph(p);
    }
    rc = (p->precision == XFFT_MIXED) ? autotune_fft<float>(p, p->w32, p->t32, nrhs)
                                      : autotune_fft<double>(p, p->w64, p->t64, nrhs);
    if (rc) return rc;
    // the CG iterations: FP32 without the stress integral inside the refinement,
    // FP64 with it (criterion 0 tracks <sigma>)
    rc = (p->precision == XFFT_MIXED) ? ensure_voxel_matrices<float>(p, p->w32, p->t32, nrhs, false)
                                      : ensure_voxel_matrices<double>(p, p->w64, p->t64, nrhs, true);
    if (rc) return rc;
    rc = reset_state(p, nrhs, ebar_host);
    if (rc) return rc;
    hipStream_t s = p->stream;
    Work<double> &w = p->w64;
    const size_t nf = sizeof(double) * 3 * p->g.N * nrhs, ne = sizeof(double) * 3 * p->g.nX * nrhs;
    const bool warm = u0 != nullptr;
    if (warm) {
        HIP_OK(hipMemcpyAsync(w.u, u0, nf, hipMemcpyDeviceToDevice, s));
        if (ne) HIP_OK(hipMemcpyAsync(w.ue, ue0, ne, hipMemcpyDeviceToDevice, s));
    } else {
        HIP_OK(hipMemsetAsync(w.u, 0, nf, s));
        if (ne) HIP_OK(hipMemsetAsync(w.ue, 0, ne, s));
    }
    p->sigma_ready = false;
    iters.assign(nrhs, 0);
    outer.assign(nrhs, 0);
    res_rel.assign(nrhs, 0.0);
    std::vector<Flags> fl;
    *status = XFFT_OK;
    if (p->precision != XFFT_MIXED) {
        // f = b - A u0 = -r(u0) (u0 = 0 unless warm started)
        launch_operator<double>(p, w, p->t64, warm ? w.u : nullptr, w.ue, w.f, w.fe, true, -1.0, nrhs, nullptr, 0,
                                nullptr, s);
        launch_scalars(p, SC_INIT_SIGMA, 0, nrhs, 0, nullptr, s, true);
        cg_start<double>(p, w, p->t64, nrhs, 0);
        cg_loop<double>(p, w, p->t64, nrhs, 0, &rc);
        if (rc) return rc;
        rc = read_flags(p, nrhs, fl);
        if (rc) return rc;
        for (int r = 0; r < nrhs; ++r) {
            iters[r] = fl[r].iters;
            if (fl[r].breakdown) *status = XFFT_EBREAKDOWN;
            else if (!fl[r].conv && *status == XFFT_OK) *status = XFFT_NOT_CONVERGED;
        }
    } else {
        Work<float> &w32 = p->w32;
        const int max_outer = 60;
        bool all_done = false;
        for (int o = 0; o < max_outer && !all_done; ++o) {
            // r = b - A u in FP64 (also gives the exact <sigma(u)>)
            launch_operator<double>(p, w, p->t64, (o == 0 && !warm) ? nullptr : w.u, w.ue, w.f, w.fe, true, -1.0,
                                    nrhs, nullptr, 0, nullptr, s);
            launch_scalars(p, SC_INIT_SIGMA, 0, nrhs, 0, nullptr, s, true);
            launch_round_to_float(p, nrhs, s);
            cg_start<float>(p, w32, p->t32, nrhs, 0);     // outer criterion on the FP64 residual
            rc = read_flags(p, nrhs, fl);
            if (rc) return rc;
            all_done = true;
            for (int r = 0; r < nrhs; ++r) {
                if (!fl[r].pad[0]) { all_done = false; outer[r] = o + 1; }
            }
            if (all_done) { p->sigma_ready = true; break; }
            cg_loop<float>(p, w32, p->t32, nrhs, 1, &rc);
            if (rc) return rc;
            launch_accumulate_correction(p, nrhs, s);
            rc = read_flags(p, nrhs, fl);
            if (rc) return rc;
            bool stalled = true;
            for (int r = 0; r < nrhs; ++r) {
                if (fl[r].breakdown) *status = XFFT_EBREAKDOWN;
                if (!fl[r].pad[0] && fl[r].iters < p->maxit) stalled = false;
            }
            if (stalled || *status == XFFT_EBREAKDOWN) break;
        }
        rc = read_flags(p, nrhs, fl);
        if (rc) return rc;
        for (int r = 0; r < nrhs; ++r) {
            iters[r] = fl[r].iters;
            if (!fl[r].pad[0] && *status == XFFT_OK) *status = XFFT_NOT_CONVERGED;
        }
    }
    // relative final residual of the criterion
    std::vector<Scalars> sc(nrhs);
    HIP_OK(hipMemcpyAsync(sc.data(), p->scal, sizeof(Scalars) * nrhs, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int r = 0; r < nrhs; ++r) {
        double sn = 0.0;
        for (int q = 0; q < 6; ++q) sn += sc[r].sigma[q] * sc[r].sigma[q];
        const double res = std::sqrt(std::fmax(sc[r].res2, 0.0) / (double)p->g.N);
        res_rel[r] = sn > 0.0 ? res / std::sqrt(sn) : res;
    }
    return XFFT_OK;
}

bool is_unit_basis(int nload, const double *E) {
    if (nload != 6) return false;
    for (int k = 0; k < 6; ++k)
        for (int q = 0; q < 6; ++q)
            if (E[6 * k + q] != (k == q ? 1.0 : 0.0)) return false;
    return true;
}

// x[i] *= a (displacements from voxel units to units of len)
__global__ void k_scale(double *x, int64_t n, double a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] *= a;
}

int solve_impl(xfft_problem *p, int nload, const double *strain, double *disp, double *stress, double *avg_stress,
               double *c_eff, xfft_stats *stats, bool device_out) {
    if (!p || nload < 1 || !strain) return XFFT_EINVAL;
    for (int q = 0; q < 6 * nload; ++q)
        if (!std::isfinite(strain[q])) return XFFT_EINVAL;
    const bool unit = is_unit_basis(nload, strain);
    if (c_eff && !unit) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(p->device));
    const double t0 = now_s();
    const int blk = p->batch ? nload : 1;
    const int64_t N = p->g.N, nX = p->g.nX;
    std::vector<double> avg(6 * nload);
    int status = XFFT_OK;
    // keep the FP64 solutions for gradients when the unit basis is solved
    if (unit) {
        if (!p->sol_u) {
            if (hipMalloc(&p->sol_u, sizeof(double) * 6 * 3 * N) != hipSuccess) return XFFT_ENOMEM;
            if (hipMalloc(&p->sol_ue, sizeof(double) * 6 * 3 * (nX > 0 ? nX : 1)) != hipSuccess) return XFFT_ENOMEM;
        }
    }
    p->sol_unit_basis = false;
    // warm start: the stored unit-load solutions of an earlier solve
    const bool warm = unit && p->warm_start && p->sol_stored;
    p->sol_stored = false;
    double *vstress_dev = nullptr;
    for (int l0 = 0; l0 < nload; l0 += blk) {
        const int nr = (l0 + blk <= nload) ? blk : nload - l0;
        std::vector<int> it, outer;
        std::vector<double> res;
        int st = XFFT_OK;
        int rc = solve_block(p, nr, strain + 6 * l0, it, outer, res, &st,
                             warm ? p->sol_u + (size_t)3 * N * l0 : nullptr,
                             warm ? p->sol_ue + (size_t)3 * nX * l0 : nullptr);
        if (rc) return rc;
        if (st == XFFT_EBREAKDOWN || (st == XFFT_NOT_CONVERGED && status == XFFT_OK)) status = st;
        if (stress) {
            if (device_out) vstress_dev = stress + (size_t)6 * N * l0;
            else if (!vstress_dev && hipMalloc(&vstress_dev, sizeof(double) * 6 * N * blk) != hipSuccess)
                return XFFT_ENOMEM;
        }
        rc = final_outputs(p, nr, avg.data() + 6 * l0, stress ? vstress_dev : nullptr, p->sigma_ready);
        if (rc) return rc;
        hipStream_t s = p->stream;
        const hipMemcpyKind k_out = device_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (disp) {
            // FE displacement in units of len: voxel units times h
            std::vector<double> tmp;
            HIP_OK(hipStreamSynchronize(s));
            if (device_out) {
                HIP_OK(hipMemcpyAsync(disp + (size_t)3 * N * l0, p->w64.u, sizeof(double) * 3 * N * nr, k_out, s));
                const int64_t nd = 3 * N * nr;
                k_scale<<<(unsigned)((nd + 255) / 256), 256, 0, s>>>(disp + (size_t)3 * N * l0, nd, p->h);
            } else {
                HIP_OK(hipMemcpyAsync(disp + (size_t)3 * N * l0, p->w64.u, sizeof(double) * 3 * N * nr, k_out, s));
                HIP_OK(hipStreamSynchronize(s));
                for (size_t q = 0; q < (size_t)3 * N * nr; ++q) disp[(size_t)3 * N * l0 + q] *= p->h;
            }
        }
        if (stress && !device_out) {
            HIP_OK(hipMemcpyAsync(stress + (size_t)6 * N * l0, vstress_dev, sizeof(double) * 6 * N * nr, k_out, s));
        }
        if (unit) {
            HIP_OK(hipMemcpyAsync(p->sol_u + (size_t)3 * N * l0, p->w64.u, sizeof(double) * 3 * N * nr,
                                  hipMemcpyDeviceToDevice, s));
            if (nX)
                HIP_OK(hipMemcpyAsync(p->sol_ue + (size_t)3 * nX * l0, p->w64.ue, sizeof(double) * 3 * nX * nr,
                                      hipMemcpyDeviceToDevice, s));
        }
        HIP_OK(hipStreamSynchronize(s));
        if (stats) {
            for (int r = 0; r < nr; ++r) {
                if (stats->iters) stats->iters[l0 + r] = it[r];
                if (stats->outer_iters) stats->outer_iters[l0 + r] = outer[r];
                if (stats->final_res) stats->final_res[l0 + r] = res[r];
            }
        }
    }
    if (stress && !device_out && vstress_dev) (void)hipFree(vstress_dev);
    if (unit) p->sol_unit_basis = true;
    // finite solutions to start a later warm-started solve from
    if (unit) p->sol_stored = status == XFFT_OK || status == XFFT_NOT_CONVERGED;
    if (avg_stress) {
        if (device_out) HIP_OK(hipMemcpy(avg_stress, avg.data(), sizeof(double) * 6 * nload, hipMemcpyHostToDevice));
        else std::memcpy(avg_stress, avg.data(), sizeof(double) * 6 * nload);
    }
    if (c_eff) {
        for (int k = 0; k < 6; ++k)
            for (int q = 0; q < 6; ++q) c_eff[6 * q + k] = avg[6 * k + q];
    }
    p->seconds_solve = now_s() - t0;
    if (stats) {
        stats->seconds_setup = p->seconds_setup;
        stats->seconds_solve = p->seconds_solve;
        stats->n_enriched = p->g.nX;
        stats->n_irregular_voxels = p->g.nirr;
        stats->n_cut_elements = p->n_cut_elements;
        stats->n_multilabel = p->n_multilabel;
        stats->voxel_matrices = p->vm_on[p->precision == XFFT_MIXED ? 0 : 1] ? 1 : 0;
        const int pi = p->precision == XFFT_MIXED ? 0 : 1;
        stats->fft_variant = (p->fft_plane[pi] ? 0 : 1) | (p->fft_ztile[pi] ? 2 : 0);
    }
    return status;
}

// Per-class average of the windows [event before launch, event after launch]
// recorded since the last reset; classes 0..K_COUNT-1 FP32, K_COUNT.. FP64.
int prof_collect(xfft_problem *p, double *ms_out, int32_t *count_out) {
    HIP_OK(hipStreamSynchronize(p->stream));
    std::vector<double> sum(2 * K_COUNT, 0.0);
    std::vector<int> cnt(2 * K_COUNT, 0);
    for (size_t i = 1; i < p->prof_used; ++i) {
        const int id = p->prof_ids[i];
        if (id < 0 || p->prof_ids[i - 1] != -1) continue;
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, p->prof_pool[i - 1], p->prof_pool[i]));
        if (id < 2 * K_COUNT) { sum[id] += ms; cnt[id] += 1; }
    }
    p->prof_used = 0;
    p->prof_ids.clear();
    for (int k = 0; k < 2 * K_COUNT; ++k) {
        if (ms_out) ms_out[k] = cnt[k] ? sum[k] / cnt[k] : 0.0;
        if (count_out) count_out[k] = cnt[k];
    }
    return XFFT_OK;
}

template <typename T>
int profile_impl(xfft_problem *p, Work<T> &w, const Tables<T> &tb, int nrhs, int nrep, double *ms_out,
                 int32_t *count_out) {
    hipStream_t s = p->stream;
    std::vector<double> E(6 * nrhs, 0.0);
    for (int r = 0; r < nrhs; ++r) E[6 * r + (r % 6)] = 1.0;
    int rc = reset_state(p, nrhs, E.data());
    if (rc) return rc;
    HIP_OK(hipMemsetAsync(w.u, 0, sizeof(T) * 3 * p->g.N * nrhs, s));
    if (p->g.nX) HIP_OK(hipMemsetAsync(w.ue, 0, sizeof(T) * 3 * p->g.nX * nrhs, s));
    launch_operator<T>(p, w, tb, nullptr, nullptr, w.f, w.fe, true, (T)-1, nrhs, nullptr, 0, nullptr, s);
    launch_scalars(p, SC_INIT_SIGMA, 0, nrhs, 0, nullptr, s, true);
    cg_start<T>(p, w, tb, nrhs, 0);
    std::vector<Flags> fl;
    rc = read_flags(p, nrhs, fl);
    if (rc) return rc;
    for (auto &f : fl) { f.active[0] = 1; f.active[1] = 1; f.iters = 0; }
    HIP_OK(hipMemcpyAsync(p->flags, fl.data(), sizeof(Flags) * nrhs, hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    const int saved_maxit = p->maxit;
    p->maxit = 1 << 30;
    p->prof_used = 0;
    p->prof_ids.clear();
    p->prof_on = true;
    for (int it = 0; it < nrep; ++it) cg_iteration<T>(p, w, tb, nrhs, it & 1, 0);
    p->prof_on = false;
    p->maxit = saved_maxit;
    std::vector<double> ms(2 * K_COUNT);
    std::vector<int32_t> cnt(2 * K_COUNT);
    rc = prof_collect(p, ms.data(), cnt.data());
    if (rc) return rc;
    const int off = sizeof(T) == 8 ? K_COUNT : 0;
    for (int k = 0; k < K_COUNT; ++k) {
        const int src = (k == K_SCALARS) ? K_SCALARS + K_COUNT : k + off;
        if (ms_out) ms_out[k] = ms[src];
        if (count_out) count_out[k] = cnt[src];
    }
    return XFFT_OK;
}

}  // namespace

void xfft_prof_mark(xfft_problem *p, int kernel_id, hipStream_t s) {
    if (!p || !p->prof_on) return;
    if (p->prof_used == p->prof_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        p->prof_pool.push_back(e);
    }
    if (hipEventRecord(p->prof_pool[p->prof_used], s) != hipSuccess) return;
    p->prof_ids.push_back(kernel_id);
    ++p->prof_used;
}

extern "C" {

int xfft_profile(xfft_problem *p, int32_t precision, int32_t nrhs, int32_t nrep, double *ms_out,
                 int32_t *count_out) {
    if (!p || nrhs < 1 || nrep < 1 || (precision != XFFT_FP64 && precision != XFFT_FP32)) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(p->device));
    int rc = ensure_state(p, nrhs);
    if (rc) return rc;
    if (precision == XFFT_FP64) {
        rc = alloc_work<double>(p, p->w64, nrhs);
        if (rc) return rc;
        return profile_impl<double>(p, p->w64, p->t64, nrhs, nrep, ms_out, count_out);
    }
    rc = alloc_work<float>(p, p->w32, nrhs);
    if (rc) return rc;
    return profile_impl<float>(p, p->w32, p->t32, nrhs, nrep, ms_out, count_out);
}

int xfft_profile_begin(xfft_problem *p) {
    if (!p) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(p->device));
    HIP_OK(hipStreamSynchronize(p->stream));
    p->prof_used = 0;
    p->prof_ids.clear();
    p->prof_on = true;
    return XFFT_OK;
}

int xfft_profile_end(xfft_problem *p, double *ms_out, int32_t *count_out) {
    if (!p || !p->prof_on) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(p->device));
    p->prof_on = false;
    return prof_collect(p, ms_out, count_out);
}

void xfft_default_options(xfft_options *opt) {
    if (!opt) return;
    opt->rtol = 1e-10;
    opt->maxit = 20000;
    opt->precision = XFFT_FP64;
    opt->snap_eps = 1e-6;
    opt->d0_scale = 1.0;
    opt->inner_rtol = 1e-6;
    opt->batch = 1;
    opt->device = 0;
    opt->check_every = 8;
    opt->use_graph = 1;
    opt->autotune = 1;
    opt->stream = nullptr;
    opt->scheme = XFFT_LCG;
    opt->discretization = XFFT_XFEM;
    opt->voxel_matrices = -1;
    opt->warm_start = 0;
    opt->fft_variant = -1;
}

const char *xfft_strerror(int code) {
    switch (code) {
        case XFFT_OK: return "ok";
        case XFFT_NOT_CONVERGED: return "not converged within maxit";
        case XFFT_EINVAL: return "invalid argument";
        case XFFT_ENOMEM: return "device allocation failed";
        case XFFT_EDEVICE: return "HIP device error";
        case XFFT_EBREAKDOWN: return "CG breakdown (d^T A d <= 0 or not finite)";
        default: return "unknown error";
    }
}

void xfft_destroy(xfft_problem *p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    void *ptrs[] = {p->Ls, p->phase, p->vmat, p->irr, p->irr_j, p->irr_lab, p->jlist, p->enr_src, p->d0, p->partial,
                    p->scal, p->flags, p->ebar, p->sum7, p->sol_u, p->sol_ue, p->t64.lame, p->t64.d0is, p->t64.irr_L,
                    p->t32.lame, p->t32.d0is, p->t32.irr_L, p->t64.irr_M, p->t32.irr_M};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    for (int a = 0; a < 3; ++a) {
        if (p->t64.tw[a]) (void)hipFree(p->t64.tw[a]);
        if (p->t64.tws[a]) (void)hipFree(p->t64.tws[a]);
        if (p->t32.tws[a]) (void)hipFree(p->t32.tws[a]);
        if (p->t32.tw[a]) (void)hipFree(p->t32.tw[a]);
        if (p->t64.half[a]) (void)hipFree(p->t64.half[a]);
        if (p->t32.half[a]) (void)hipFree(p->t32.half[a]);
    }
    drop_graph(p);
    free_voxel_matrices(p);
    free_work(p->w64);
    free_work(p->w32);
    for (hipEvent_t e : p->prof_pool) (void)hipEventDestroy(e);
    if (p->host_flags) (void)hipHostFree(p->host_flags);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

int xfft_setup(const int32_t n[3], const double len[3], const double *levelset, const int32_t *phase,
               int32_t nphase, const double *lame, const xfft_options *opt_in, xfft_problem **out) {
    if (!out) return XFFT_EINVAL;
    *out = nullptr;
    if (!n || !len || !levelset || !phase || !lame || nphase < 1) return XFFT_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!size_ok(n[a]) || !(len[a] > 0.0) || !std::isfinite(len[a])) return XFFT_EINVAL;
    if (!fft_sizes_ok(n[0], n[1], n[2])) return XFFT_EINVAL;
    // the operator addresses the three components of a field of one load with
    // 32-bit byte offsets
    if ((int64_t)n[0] * n[1] * n[2] * 3 * (int64_t)sizeof(double) >= ((int64_t)1 << 32)) return XFFT_EINVAL;
    const double h = len[0] / n[0];
    for (int a = 1; a < 3; ++a)
        if (std::fabs(len[a] / n[a] - h) > 1e-12 * h) return XFFT_EINVAL;
    if (!lame_ok(lame, nphase)) return XFFT_EINVAL;
    {
        const int64_t Nn = (int64_t)n[0] * n[1] * n[2];
        for (int64_t q = 0; q < Nn; ++q)
            if (!std::isfinite(levelset[q]) || phase[q] < 0 || phase[q] >= nphase) return XFFT_EINVAL;
    }
    xfft_options opt;
    xfft_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (!(opt.rtol > 0.0) || opt.maxit < 1 || !(opt.snap_eps >= 0.0) || !(opt.d0_scale > 0.0) ||
        !(opt.inner_rtol > 0.0 && opt.inner_rtol < 1.0) ||
        (opt.precision != XFFT_FP64 && opt.precision != XFFT_MIXED) || opt.scheme < XFFT_LCG ||
        opt.scheme > XFFT_BASIC || (opt.scheme != XFFT_LCG && opt.precision != XFFT_FP64) ||
        (opt.discretization != XFFT_XFEM && opt.discretization != XFFT_P1) || opt.voxel_matrices < -1 ||
        opt.voxel_matrices > 1 || opt.warm_start < 0 || opt.warm_start > 1 || opt.fft_variant < -1 ||
        opt.fft_variant > 3)
        return XFFT_EINVAL;
    const double t0 = now_s();
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1 || opt.device < 0 || opt.device >= ndev)
        return XFFT_EDEVICE;
    if (hipSetDevice(opt.device) != hipSuccess) return XFFT_EDEVICE;
    // address of this device's work space of xfft_apply_operator_noalloc
    if (static_scratch_init(opt.device) != XFFT_OK) return XFFT_EDEVICE;
    xfft_problem *p = new (std::nothrow) xfft_problem();
    if (!p) return XFFT_ENOMEM;
    p->device = opt.device;
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, opt.device) == hipSuccess && ncu > 0)
            p->num_cu = ncu;
    }
    p->h = h;
    for (int a = 0; a < 3; ++a) p->len[a] = len[a];
    p->rtol = opt.rtol; p->snap_eps = opt.snap_eps; p->d0_scale = opt.d0_scale; p->inner_rtol = opt.inner_rtol;
    p->maxit = opt.maxit; p->precision = opt.precision; p->batch = opt.batch; p->check_every = opt.check_every;
    p->use_graph = opt.use_graph != 0;
    p->autotune = opt.autotune != 0;
    p->scheme = opt.scheme;
    p->p1 = opt.discretization == XFFT_P1 ? 1 : 0;
    p->vm_mode = opt.voxel_matrices;
    p->warm_start = opt.warm_start != 0;
    if (opt.fft_variant >= 0 || !p->autotune) {
        const int v = opt.fft_variant > 0 ? opt.fft_variant : 0;
        for (int q = 0; q < 2; ++q) {
            p->fft_plane[q] = (v & 1) ? 0 : 1;
            p->fft_ztile[q] = (v >> 1) & 1;
            p->fft_tuned[q] = true;
        }
    }
    if (opt.stream) {
        p->stream = (hipStream_t)opt.stream;
    } else {
        if (hipStreamCreate(&p->stream) != hipSuccess) { delete p; return XFFT_EDEVICE; }
        p->own_stream = true;
    }
    Geometry &g = p->g;
    g.n0 = n[0]; g.n1 = n[1]; g.n2 = n[2]; g.nh = n[0] / 2 + 1;
    g.N = (int64_t)n[0] * n[1] * n[2];
    g.nphase = nphase;
    p->lame_host.assign(lame, lame + 2 * nphase);
    const int64_t N = g.N;
    double *Lraw = nullptr;
    int rc = XFFT_OK;
    if (hipMalloc(&p->Ls, sizeof(double) * N) != hipSuccess || hipMalloc(&p->phase, sizeof(int32_t) * N) != hipSuccess ||
        hipMalloc(&p->vmat, sizeof(int32_t) * N) != hipSuccess || hipMalloc(&Lraw, sizeof(double) * N) != hipSuccess)
        rc = XFFT_ENOMEM;
    if (!rc && (hipMemcpyAsync(Lraw, levelset, sizeof(double) * N, hipMemcpyHostToDevice, p->stream) != hipSuccess ||
                hipMemcpyAsync(p->phase, phase, sizeof(int32_t) * N, hipMemcpyHostToDevice, p->stream) != hipSuccess))
        rc = XFFT_EDEVICE;
    if (!rc) rc = run_setup(p, Lraw);
    if (Lraw) (void)hipFree(Lraw);
    // and the corner-force buffer of one load (48 values per irregular voxel) likewise
    if (!rc && cut_rows(g.nirr) * 48 * (int64_t)sizeof(double) >= ((int64_t)1 << 32)) rc = XFFT_EINVAL;
    if (!rc) rc = compute_tables(p);
    if (!rc) {
        for (int a = 0; a < 3; ++a)
            if (p->plan[a].nstages < 0) rc = XFFT_EINVAL;
    }
    if (!rc) {
        SlotLayout L = slot_layout(g);
        L.grn0 = L.total;
        L.grn_n = green_slots(g);
        L.eu0 = L.grn0 + L.grn_n;
        L.eu_n = (int)((g.nX + ENR_BLOCK - 1) / ENR_BLOCK);
        L.total = L.eu0 + L.eu_n;
        p->slots = L;
        p->nslots = L.total;
    }
    if (rc) {
        xfft_destroy(p);
        return rc;
    }
    p->seconds_setup = now_s() - t0;
    *out = p;
    return XFFT_OK;
}

int xfft_set_lame(xfft_problem *p, const double *lame) {
    if (!p || !lame || !lame_ok(lame, p->g.nphase)) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(p->device));
    p->lame_host.assign(lame, lame + 2 * p->g.nphase);
    std::vector<float> l32(2 * p->g.nphase);
    for (int q = 0; q < 2 * p->g.nphase; ++q) l32[q] = (float)lame[q];
    HIP_OK(hipMemcpyAsync(p->t64.lame, lame, sizeof(double) * 2 * p->g.nphase, hipMemcpyHostToDevice, p->stream));
    HIP_OK(hipMemcpyAsync(p->t32.lame, l32.data(), sizeof(float) * 2 * p->g.nphase, hipMemcpyHostToDevice, p->stream));
    HIP_OK(hipStreamSynchronize(p->stream));
    p->sol_unit_basis = false;
    p->vm_valid = false;          // cached voxel matrices depend on the moduli: rebuilt when next used
    return XFFT_OK;
}

int xfft_solve(xfft_problem *p, int32_t nload, const double *macro_strain, double *disp, double *stress,
               double *avg_stress, double *c_eff, xfft_stats *stats) {
    return solve_impl(p, nload, macro_strain, disp, stress, avg_stress, c_eff, stats, false);
}

int xfft_solve_device(xfft_problem *p, int32_t nload, const double *strain_dev, double *disp_dev,
                      double *avg_stress_dev, void *stream, xfft_stats *stats) {
    if (!p || nload < 1 || !strain_dev) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(p->device));
    if (stream) HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    std::vector<double> strain(6 * nload);
    HIP_OK(hipMemcpy(strain.data(), strain_dev, sizeof(double) * 6 * nload, hipMemcpyDeviceToHost));
    // every solved block writes its loads' displacements (scaled to units of
    // len on the device) straight into disp_dev
    return solve_impl(p, nload, strain.data(), disp_dev, nullptr, avg_stress_dev, nullptr, stats, true);
}

int xfft_apply_operator(xfft_problem *p, int32_t precision, const double *x, const double *macro_strain, double *y,
                        double *avg_stress) {
    if (!p || !x || !y || (precision != XFFT_FP64 && precision != XFFT_FP32)) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(p->device));
    const int64_t N = p->g.N, nX = p->g.nX;
    int rc = alloc_work<double>(p, p->w64, 1);
    if (!rc && precision == XFFT_FP32) rc = alloc_work<float>(p, p->w32, 1);
    if (!rc) rc = ensure_state(p, 1);
    if (rc) return rc;
    // with the option "always" the step-level operator runs the cached voxel matrices too
    if (p->vm_mode == 1)
        rc = precision == XFFT_FP64 ? ensure_voxel_matrices<double>(p, p->w64, p->t64, 1, avg_stress != nullptr)
                                    : ensure_voxel_matrices<float>(p, p->w32, p->t32, 1, avg_stress != nullptr);
    if (rc) return rc;
    double eb[6] = {0, 0, 0, 0, 0, 0};
    if (macro_strain) std::memcpy(eb, macro_strain, sizeof(eb));
    rc = reset_state(p, 1, eb);
    if (rc) return rc;
    hipStream_t s = p->stream;
    double *sum_dev = nullptr;
    HIP_OK(hipMalloc(&sum_dev, sizeof(double) * 7));
    if (precision == XFFT_FP64) {
        Work<double> &w = p->w64;
        HIP_OK(hipMemcpyAsync(w.d, x, sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
        if (nX) HIP_OK(hipMemcpyAsync(w.de, x + 3 * N, sizeof(double) * 3 * nX, hipMemcpyHostToDevice, s));
        launch_operator<double>(p, w, p->t64, w.d, w.de, w.z, w.ze, macro_strain != nullptr, 1.0, 1, nullptr, 0,
                                nullptr, s, avg_stress != nullptr);
        launch_scalars(p, SC_SUM_ONLY, 0, 1, 0, sum_dev, s, true);
        HIP_OK(hipMemcpyAsync(y, w.z, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, s));
        if (nX) HIP_OK(hipMemcpyAsync(y + 3 * N, w.ze, sizeof(double) * 3 * nX, hipMemcpyDeviceToHost, s));
    } else {
        Work<float> &w = p->w32;
        std::vector<float> xf(3 * (N + nX)), yf(3 * (N + nX));
        for (size_t q = 0; q < xf.size(); ++q) xf[q] = (float)x[q];
        HIP_OK(hipMemcpyAsync(w.d, xf.data(), sizeof(float) * 3 * N, hipMemcpyHostToDevice, s));
        if (nX) HIP_OK(hipMemcpyAsync(w.de, xf.data() + 3 * N, sizeof(float) * 3 * nX, hipMemcpyHostToDevice, s));
        // without avg_stress the stress-free kernels run (those of the FP32 CG iterations)
        launch_operator<float>(p, w, p->t32, w.d, w.de, w.z, w.ze, macro_strain != nullptr, 1.0f, 1, nullptr, 0,
                               nullptr, s, avg_stress != nullptr);
        launch_scalars(p, SC_SUM_ONLY, 0, 1, 0, sum_dev, s, true);
        HIP_OK(hipMemcpyAsync(yf.data(), w.z, sizeof(float) * 3 * N, hipMemcpyDeviceToHost, s));
        if (nX) HIP_OK(hipMemcpyAsync(yf.data() + 3 * N, w.ze, sizeof(float) * 3 * nX, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        for (size_t q = 0; q < yf.size(); ++q) y[q] = (double)yf[q];
    }
    double sum[7];
    HIP_OK(hipMemcpyAsync(sum, sum_dev, sizeof(sum), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    (void)hipFree(sum_dev);
    if (avg_stress) {
        const double V = (double)N, r2 = std::sqrt(2.0);
        avg_stress[0] = sum[1] / V; avg_stress[1] = sum[2] / V; avg_stress[2] = sum[3] / V;
        avg_stress[3] = r2 * sum[4] / V; avg_stress[4] = r2 * sum[5] / V; avg_stress[5] = r2 * sum[6] / V;
    }
    return XFFT_OK;
}

int xfft_voxel_stress(xfft_problem *p, const double *x, const double *macro_strain, double *stress) {
    if (!p || !x || !stress) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(p->device));
    const int64_t N = p->g.N, nX = p->g.nX;
    int rc = alloc_work<double>(p, p->w64, 1);
    if (!rc) rc = ensure_state(p, 1);
    if (rc) return rc;
    double eb[6] = {0, 0, 0, 0, 0, 0};
    if (macro_strain) std::memcpy(eb, macro_strain, sizeof(eb));
    rc = reset_state(p, 1, eb);
    if (rc) return rc;
    hipStream_t s = p->stream;
    double *vs = nullptr;
    if (hipMalloc(&vs, sizeof(double) * 6 * N) != hipSuccess) return XFFT_ENOMEM;
    Work<double> &w = p->w64;
    rc = XFFT_OK;
    if (hipMemcpyAsync(w.d, x, sizeof(double) * 3 * N, hipMemcpyHostToDevice, s) != hipSuccess ||
        (nX && hipMemcpyAsync(w.de, x + 3 * N, sizeof(double) * 3 * nX, hipMemcpyHostToDevice, s) != hipSuccess))
        rc = XFFT_EDEVICE;
    if (!rc) {
        launch_operator<double>(p, w, p->t64, w.d, w.de, w.z, w.ze, macro_strain != nullptr, 1.0, 1, nullptr, 0, vs,
                                s, true);
        if (hipMemcpyAsync(stress, vs, sizeof(double) * 6 * N, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = XFFT_EDEVICE;
    }
    (void)hipFree(vs);
    return rc;
}

int xfft_apply_precond(xfft_problem *p, int32_t precision, const double *f, double *y, double *res2) {
    if (!p || !f || !y || (precision != XFFT_FP64 && precision != XFFT_FP32)) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(p->device));
    const int64_t N = p->g.N, nX = p->g.nX;
    int rc = alloc_work<double>(p, p->w64, 1);
    if (!rc && precision == XFFT_FP32) rc = alloc_work<float>(p, p->w32, 1);
    if (!rc) rc = ensure_state(p, 1);
    if (rc) return rc;
    rc = reset_state(p, 1, nullptr);
    if (rc) return rc;
    hipStream_t s = p->stream;
    double *sum_dev = nullptr;
    HIP_OK(hipMalloc(&sum_dev, sizeof(double) * 7));
    if (precision == XFFT_FP64) {
        Work<double> &w = p->w64;
        HIP_OK(hipMemcpyAsync(w.f, f, sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
        if (nX) HIP_OK(hipMemcpyAsync(w.fe, f + 3 * N, sizeof(double) * 3 * nX, hipMemcpyHostToDevice, s));
        launch_green_forward<double>(p, w, p->t64, w.f, nullptr, 1, nullptr, 0, s, 0, w.ze);
        launch_green_inverse<double>(p, w, p->t64, 0, w.z, 1, nullptr, 0, s, 0);
        launch_scalars(p, SC_SUM_GREEN, 0, 1, 0, sum_dev, s, true);
        HIP_OK(hipMemcpyAsync(y, w.z, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, s));
        if (nX) HIP_OK(hipMemcpyAsync(y + 3 * N, w.ze, sizeof(double) * 3 * nX, hipMemcpyDeviceToHost, s));
    } else {
        Work<float> &w = p->w32;
        std::vector<float> ff(3 * (N + nX)), yf(3 * (N + nX));
        for (size_t q = 0; q < ff.size(); ++q) ff[q] = (float)f[q];
        HIP_OK(hipMemcpyAsync(w.f, ff.data(), sizeof(float) * 3 * N, hipMemcpyHostToDevice, s));
        if (nX) HIP_OK(hipMemcpyAsync(w.fe, ff.data() + 3 * N, sizeof(float) * 3 * nX, hipMemcpyHostToDevice, s));
        launch_green_forward<float>(p, w, p->t32, w.f, nullptr, 1, nullptr, 0, s, 0, w.ze);
        launch_green_inverse<float>(p, w, p->t32, 0, w.z, 1, nullptr, 0, s, 0);
        launch_scalars(p, SC_SUM_GREEN, 0, 1, 0, sum_dev, s, false);
        HIP_OK(hipMemcpyAsync(yf.data(), w.z, sizeof(float) * 3 * N, hipMemcpyDeviceToHost, s));
        if (nX) HIP_OK(hipMemcpyAsync(yf.data() + 3 * N, w.ze, sizeof(float) * 3 * nX, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        for (size_t q = 0; q < yf.size(); ++q) y[q] = (double)yf[q];
    }
    double sum[7];
    HIP_OK(hipMemcpyAsync(sum, sum_dev, sizeof(sum), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    (void)hipFree(sum_dev);
    if (res2) *res2 = sum[0];
    return XFFT_OK;
}

int xfft_get_layout(xfft_problem *p, int64_t *info, int64_t *jlist, double *d0) {
    if (!p || !info) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(p->device));
    info[0] = p->g.N;
    info[1] = p->g.nX;
    info[2] = p->g.nirr;
    info[3] = p->n_cut_elements;
    info[4] = p->n_multilabel;
    info[5] = p->g.nphase;
    if (p->g.nX > 0 && jlist) {
        std::vector<int32_t> tmp(p->g.nX);
        HIP_OK(hipMemcpy(tmp.data(), p->jlist, sizeof(int32_t) * p->g.nX, hipMemcpyDeviceToHost));
        for (int64_t q = 0; q < p->g.nX; ++q) jlist[q] = tmp[q];
    }
    if (p->g.nX > 0 && d0) HIP_OK(hipMemcpy(d0, p->d0, sizeof(double) * p->g.nX, hipMemcpyDeviceToHost));
    return XFFT_OK;
}

int xfft_grad_lame(xfft_problem *p, const double *dL_dC, double *grad, double *dC_out) {
    if (!p || (!grad && !dC_out) || (grad && !dL_dC)) return XFFT_EINVAL;
    if (!p->sol_unit_basis || !p->sol_u) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(p->device));
    const int np = p->g.nphase;
    std::vector<double> dC((size_t)np * 72);
    const int rc = grad_tables(p, dC.data());
    if (rc == -1) return XFFT_EINVAL;
    if (rc == -2) return XFFT_ENOMEM;
    if (rc) return XFFT_EDEVICE;
    if (dC_out) std::memcpy(dC_out, dC.data(), sizeof(double) * dC.size());
    if (grad) {
        for (int ph = 0; ph < np; ++ph)
            for (int j = 0; j < 2; ++j) {
                double acc = 0.0;
                for (int q = 0; q < 36; ++q) acc += dL_dC[q] * dC[(ph * 2 + j) * 36 + q];
                grad[2 * ph + j] = acc;
            }
    }
    return XFFT_OK;
}

int xfft_batch_solve(xfft_problem *const *ps, int32_t nprob, double *c_eff, xfft_stats *stats) {
    if (!ps || nprob < 1 || !c_eff) return XFFT_EINVAL;
    for (int i = 0; i < nprob; ++i)
        if (!ps[i] || ps[i]->precision != ps[0]->precision || ps[i]->device != ps[0]->device) return XFFT_EINVAL;
    HIP_OK(hipSetDevice(ps[0]->device));
    const double t0 = now_s();
    const int nl = 6;
    double E[36];
    for (int k = 0; k < 36; ++k) E[k] = (k % 7 == 0) ? 1.0 : 0.0;
    const bool mixed = ps[0]->precision == XFFT_MIXED;
    // prepare every problem on its own stream
    for (int i = 0; i < nprob; ++i) {
        xfft_problem *p = ps[i];
        int rc = alloc_work<double>(p, p->w64, nl);
        if (!rc && mixed) rc = alloc_work<float>(p, p->w32, nl);
        if (!rc) rc = ensure_state(p, nl);
        if (!rc && p->autotune && !p->tuned) {
            rc = mixed ? autotune_depth<float>(p, p->w32, p->t32, nl) : autotune_depth<double>(p, p->w64, p->t64, nl);
            p->tuned = true;
        }
        if (!rc) rc = mixed ? ensure_voxel_matrices<float>(p, p->w32, p->t32, nl, false)
                            : ensure_voxel_matrices<double>(p, p->w64, p->t64, nl, true);
        if (!rc) rc = reset_state(p, nl, E);
        if (rc) return rc;
        HIP_OK(hipMemsetAsync(p->w64.u, 0, sizeof(double) * 3 * p->g.N * nl, p->stream));
        if (p->g.nX) HIP_OK(hipMemsetAsync(p->w64.ue, 0, sizeof(double) * 3 * p->g.nX * nl, p->stream));
        p->sol_unit_basis = false;
    }
    // one graph: every problem's iterations as a branch between a fork and a join
    const int every = check_period(ps[0]);
    const int crit = mixed ? 1 : 0;
    hipStream_t master = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> ev(nprob + 1, nullptr);
    int rc = XFFT_OK;
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (master) (void)hipStreamDestroy(master);
    };
    if (hipStreamCreate(&master) != hipSuccess) return XFFT_EDEVICE;
    for (auto &e : ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { cleanup(); return XFFT_EDEVICE; }
    for (int i = 0; i < nprob; ++i)
        if (hipStreamSynchronize(ps[i]->stream) != hipSuccess) { cleanup(); return XFFT_EDEVICE; }
    if (hipStreamBeginCapture(master, hipStreamCaptureModeThreadLocal) != hipSuccess) { cleanup(); return XFFT_EDEVICE; }
    bool cap_ok = hipEventRecord(ev[nprob], master) == hipSuccess;
    for (int i = 0; i < nprob && cap_ok; ++i) {
        xfft_problem *p = ps[i];
        cap_ok = hipStreamWaitEvent(p->stream, ev[nprob], 0) == hipSuccess;
        if (!cap_ok) break;
        if (mixed) enqueue_iterations<float>(p, p->w32, p->t32, nl, crit, every);
        else enqueue_iterations<double>(p, p->w64, p->t64, nl, crit, every);
        cap_ok = hipEventRecord(ev[i], p->stream) == hipSuccess && hipStreamWaitEvent(master, ev[i], 0) == hipSuccess;
    }
    if (hipStreamEndCapture(master, &graph) != hipSuccess || !cap_ok ||
        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        cleanup();
        return XFFT_EDEVICE;
    }
    auto poll = [&](std::vector<std::vector<Flags>> &fl) -> int {
        for (int i = 0; i < nprob; ++i)
            HIP_OK(hipMemcpyAsync(ps[i]->host_flags, ps[i]->flags, sizeof(Flags) * nl, hipMemcpyDeviceToHost, master));
        HIP_OK(hipStreamSynchronize(master));
        for (int i = 0; i < nprob; ++i)
            fl[i].assign(reinterpret_cast<Flags *>(ps[i]->host_flags), reinterpret_cast<Flags *>(ps[i]->host_flags) + nl);
        return XFFT_OK;
    };
    std::vector<std::vector<Flags>> fl(nprob);
    auto run_inner = [&]() -> int {
        int it = 0;
        for (int i = 0; i < nprob; ++i) HIP_OK(hipStreamSynchronize(ps[i]->stream));
        int r = poll(fl);
        if (r) return r;
        const int maxit = ps[0]->maxit;
        while (it < maxit) {
            bool any = false;
            for (int i = 0; i < nprob; ++i)
                for (int q = 0; q < nl; ++q) any |= fl[i][q].active[0] != 0;
            if (!any) break;
            HIP_OK(hipGraphLaunch(exec, master));
            it += every;
            r = poll(fl);
            if (r) return r;
        }
        return XFFT_OK;
    };
    std::vector<int> outer(nprob * nl, 0);
    if (!mixed) {
        for (int i = 0; i < nprob; ++i) {
            xfft_problem *p = ps[i];
            Work<double> &w = p->w64;
            launch_operator<double>(p, w, p->t64, nullptr, nullptr, w.f, w.fe, true, -1.0, nl, nullptr, 0, nullptr,
                                    p->stream);
            launch_scalars(p, SC_INIT_SIGMA, 0, nl, 0, nullptr, p->stream, true);
            cg_start<double>(p, w, p->t64, nl, 0);
        }
        rc = run_inner();
    } else {
        for (int o = 0; o < 60 && !rc; ++o) {
            for (int i = 0; i < nprob; ++i) {
                xfft_problem *p = ps[i];
                Work<double> &w = p->w64;
                launch_operator<double>(p, w, p->t64, o == 0 ? nullptr : w.u, w.ue, w.f, w.fe, true, -1.0, nl,
                                        nullptr, 0, nullptr, p->stream);
                launch_scalars(p, SC_INIT_SIGMA, 0, nl, 0, nullptr, p->stream, true);
                launch_round_to_float(p, nl, p->stream);
                cg_start<float>(p, p->w32, p->t32, nl, 0);
            }
            for (int i = 0; i < nprob; ++i)
                if (hipStreamSynchronize(ps[i]->stream) != hipSuccess) rc = XFFT_EDEVICE;
            if (rc) break;
            rc = poll(fl);
            if (rc) break;
            bool all_done = true;
            for (int i = 0; i < nprob; ++i)
                for (int q = 0; q < nl; ++q)
                    if (!fl[i][q].pad[0]) { all_done = false; outer[i * nl + q] = o + 1; }
            if (all_done) break;
            rc = run_inner();
            if (rc) break;
            for (int i = 0; i < nprob; ++i) launch_accumulate_correction(ps[i], nl, ps[i]->stream);
        }
    }
    cleanup();
    if (rc) return rc;
    int status = XFFT_OK;
    for (int i = 0; i < nprob && !rc; ++i) {
        xfft_problem *p = ps[i];
        std::vector<Flags> f;
        rc = read_flags(p, nl, f);
        if (rc) break;
        std::vector<double> avg(6 * nl);
        rc = final_outputs(p, nl, avg.data(), nullptr, false);
        if (rc) break;
        for (int k = 0; k < 6; ++k)
            for (int q = 0; q < 6; ++q) c_eff[36 * i + 6 * q + k] = avg[6 * k + q];
        for (int q = 0; q < nl; ++q) {
            const bool done = mixed ? f[q].pad[0] != 0 : f[q].conv != 0;
            if (f[q].breakdown) status = XFFT_EBREAKDOWN;
            else if (!done && status == XFFT_OK) status = XFFT_NOT_CONVERGED;
        }
        // keep the unit-load solutions for xfft_grad_lame
        if (!p->sol_u) {
            if (hipMalloc(&p->sol_u, sizeof(double) * 6 * 3 * p->g.N) != hipSuccess ||
                hipMalloc(&p->sol_ue, sizeof(double) * 6 * 3 * (p->g.nX > 0 ? p->g.nX : 1)) != hipSuccess)
                return XFFT_ENOMEM;
        }
        HIP_OK(hipMemcpyAsync(p->sol_u, p->w64.u, sizeof(double) * 18 * p->g.N, hipMemcpyDeviceToDevice, p->stream));
        if (p->g.nX)
            HIP_OK(hipMemcpyAsync(p->sol_ue, p->w64.ue, sizeof(double) * 18 * p->g.nX, hipMemcpyDeviceToDevice,
                                  p->stream));
        HIP_OK(hipStreamSynchronize(p->stream));
        p->sol_unit_basis = true;
        bool finite = true;
        for (int q = 0; q < nl; ++q)
            if (f[q].breakdown) finite = false;
        p->sol_stored = finite;
        if (stats) {
            xfft_stats &st = stats[i];
            for (int q = 0; q < nl; ++q) {
                if (st.iters) st.iters[q] = f[q].iters;
                if (st.outer_iters) st.outer_iters[q] = outer[i * nl + q];
            }
            st.n_enriched = p->g.nX;
            st.n_irregular_voxels = p->g.nirr;
            st.n_cut_elements = p->n_cut_elements;
            st.n_multilabel = p->n_multilabel;
            st.seconds_setup = p->seconds_setup;
            st.voxel_matrices = p->vm_on[mixed ? 0 : 1] ? 1 : 0;
        }
    }
    if (rc) return rc;
    const double dt = now_s() - t0;
    for (int i = 0; i < nprob; ++i) {
        ps[i]->seconds_solve = dt;
        if (stats) stats[i].seconds_solve = dt;
    }
    return status;
}

}  // extern "C"

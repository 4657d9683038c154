// Host side of the C ABI declared in include/lbm.h: single-lattice solvers
// and batches of lattices sharing one persistent step launch.
//
// Scheme: Boolakee, Geier, De Lorenzis, arXiv 2208.14870 (Algorithm 1,
// Table "scheme").  Every step of the method runs in the kernels of
// lbm_device.hpp; this file owns handles, validation, memory layout inside
// caller-owned workspaces, work lists, HIP graph capture of step chunks and
// the pseudo-time convergence loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "lbm.h"
#include "lbm_device.hpp"
#include "lbm_host.hpp"

using namespace lbm;
using namespace lbm_host;

// Scratch of lbm_error_norms_noalloc: the block partials of its two-stage
// reduction, kErrBlocks x 4 doubles (32 KiB), in a static device array so that
// the call allocates nothing.  Each GPU holds its own copy at its own address
// until the process ends; host code uses that address (noalloc_scratch), never
// the array's name.  Every call on a GPU shares the GPU's copy: calls that
// overlap on one GPU race.
constexpr long long kNoAllocScratchDoubles = 4LL * kErrBlocks;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
thread_local std::string g_create_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch, looked up once per device with
// that device current; nullptr (and *e set) on failure.
double* noalloc_scratch(hipError_t* e) {
    int dev = 0;
    if ((*e = hipGetDevice(&dev)) != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *e = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if ((*e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = reinterpret_cast<double*>(p);
    }
    *e = hipSuccess;
    return g_scratch_ptr[dev];
}
}  // namespace

// ===========================================================================
// single-lattice solver
// ===========================================================================
struct lbm_solver {
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;  // private stream used only for graph capture
    int cus = 256;
    Lattice L;
    // workspace regions
    SlotDesc* d_desc = nullptr;
    Item* d_items = nullptr;
    int* d_range = nullptr;  // {0, nitems}
    int* d_first = nullptr;
    int* d_count = nullptr;
    double* d_partial = nullptr;
    double* d_result = nullptr;
    RiseGuard* d_guard = nullptr;  // divergence guard of the one-workgroup solve
    double* d_red = nullptr;  // kErrBlocks x 8 + 16
    double* h_result = nullptr;  // pinned, 8 doubles
    long long max_items_ = 0;
    int nitems = 0;
    unsigned grid = 0;
    long long phase = 0;  // launches since the descriptor was written
    long long steps = 0;
    double r_switch = 0.0;
    int blocks_per_cu = 0;  // 0: one workgroup per tile; k: persistent k per CU
    bool fused_auto = true;  // fused kernel not chosen by the caller: follows the default
    // steps per launch of the one-workgroup solve of small lattices (0: off)
    long long small_budget = 65536;
    // divergence guard of lbm_solve_to_tol: rises of the residual in a row (0: off)
    int guard_checks = 8;
    // half storage: a state set by lbm_set_populations and the exponent it needs
    bool user_state = false;
    int e_user = INT_MIN;  // INT_MIN: the state sets no bound (all zero)
    std::string err;
    // captured chunks keyed by (plain steps, writeU/check kind, start parity,
    // precision, rows per thread, general path, grid)
    std::map<std::tuple<long long, int, int, int, int, int, int, unsigned>, hipGraphExec_t> graphs;

    int fail(int code, const std::string& m) {
        err = m;
        return code;
    }
    int hip_fail(hipError_t e, const char* where) {
        err = std::string(where) + ": " + hipGetErrorString(e);
        return LBM_E_HIP;
    }
    int sel() const { return L.cur ^ (int)(phase & 1); }

    void drop_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }

    // Rewrite descriptor + work list (after any change of layout or parameters).
    int sync_desc() {
        // keep the state buffer: fold the phase parity into cur
        L.cur = sel();
        phase = 0;
        SlotDesc d = L.desc();
        d.sr_step = (unsigned)steps;  // stochastic rounding: steps enqueued before
        nitems = L.nitems();
        if (nitems > max_items_) return fail(LBM_E_WORKSPACE, "tile shape exceeds work-list space");
        hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(1), 0, stream, d_desc, d);
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, d_range, 0);
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, d_range + 1, nitems);
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, d_first, 0);
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, d_count, nitems);
        hipLaunchKernelGGL(k_build_items, dim3(blocks_for(nitems)), dim3(kBlock), 0, stream,
                           d_items, 0, 0, d.tiles_x, nitems,
                           (L.fused() && L.wave_hs == 0) ? kItemBand : 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "descriptor upload");
        unsigned g = (unsigned)((nitems + 7) / 8 * 8);
        if (blocks_per_cu > 0) g = std::min(g, (unsigned)(cus * blocks_per_cu + 7) / 8 * 8);
        grid = std::max(8u, g);
        return LBM_OK;
    }

    StepLaunch launch_args(int flip) const {
        StepLaunch a;
        a.slots = d_desc;
        a.items = d_items;
        a.range = d_range;
        a.partial = d_partial;
        a.flip = flip;
        a.rows = L.eff_vy();
        return a;
    }

    // After a launch of ns steps: advance the device's stochastic-rounding step.
    hipError_t advance_sr(int ns, hipStream_t st) {
        if (!L.sr_on()) return hipSuccess;
        hipLaunchKernelGGL(k_add_sr_step, dim3(1), dim3(1), 0, st, d_desc, ns);
        return hipGetLastError();
    }

    hipError_t enqueue_one(int mode, hipStream_t st, long long& ph) {
        hipError_t e = launch_step(L.prec, mode, L.general(), L.eff_vy(),
                                   L.layout(L.cur ^ (int)(ph & 1)), grid, st,
                                   launch_args((int)(ph & 1)));
        ++ph;
        if (e == hipSuccess) e = advance_sr(1, st);
        return e;
    }

    // One fused launch of ns steps (L.tb, or a shorter remainder).
    hipError_t enqueue_fused(int ns, hipStream_t st, long long& ph) {
        hipError_t e =
            L.wave_hs > 0
                ? launch_wave(L.prec, ns, L.wave_v, L.nx, L.ny, L.wave_hs, d_desc, (int)(ph & 1), st,
                              L.sr_on())
                : launch_stepN(L.prec, ns, L.th, grid, st, launch_args((int)(ph & 1)), false,
                               L.sr_on());
        ++ph;  // one buffer flip for ns steps
        if (e == hipSuccess) e = advance_sr(ns, st);
        return e;
    }

    // In place: one launch of ns steps through the in-place wavefront (odd ns
    // from kLayNatural, even from kLaySwapped); the layout flips per step, so
    // the launch parity advances by ns.
    hipError_t enqueue_fused_ip(int ns, hipStream_t st, long long& ph) {
        hipError_t e = launch_wave_inplace(L.prec, ns, L.wave_v, L.nx, L.ny, L.wave_hs, d_desc,
                                           (int)(ph & 1), L.halo, st);
        ph += ns;
        return e;
    }

    // In place: np steps, each launch as deep as L.tb allows with the parity
    // that the current layout needs (a single step where none is left).
    hipError_t enqueue_ip(long long np, hipStream_t st, long long& ph) {
        hipError_t e = hipSuccess;
        for (long long i = 0; i < np && e == hipSuccess;) {
            const bool nat = L.layout(L.cur ^ (int)(ph & 1)) == kLayNatural;
            int ns = (int)std::min<long long>(L.tb, np - i);
            if ((ns & 1) != (nat ? 1 : 0)) --ns;
            if (ns >= 2) {
                e = enqueue_fused_ip(ns, st, ph);
                i += ns;
            } else {
                e = enqueue_one(kPlain, st, ph);
                ++i;
            }
        }
        return e;
    }

    // Whether a remainder of r < L.tb plain steps runs as one fused launch.
    bool fused_rest(long long r) const {
        return L.fused() && r >= 2 &&
               (L.wave_hs > 0 ? r <= 8 : stepN_supported(L.prec, (int)r, L.th));
    }

    hipError_t enqueue_finalize(hipStream_t st) {
        FinalizeLaunch F;
        F.first = d_first;
        F.count = d_count;
        F.partial = d_partial;
        F.result = d_result;
        F.nslots = 1;
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, st, F);
        return hipGetLastError();
    }

    // Steps per captured graph of plain steps: about 64, whole launches.
    long long graph_chunk() const {
        return L.fused() ? std::max(1, 64 / L.tb) * (long long)L.tb : 64;
    }

    // Launches of np plain steps: groups of L.tb through the fused kernel when
    // enabled, the remainder as one shorter fused launch where a kernel exists
    // for it, else one per launch.
    long long plain_launches(long long np) const {
        if (!L.fused()) return np;
        const long long r = np % L.tb;
        return np / L.tb + (fused_rest(r) ? 1 : r);
    }

    // Steps of the fused launch that ends a sequence of n steps whose last two
    // are a write-u step and a check step (two buffers, LDS tile kernel): the
    // remainder of n (at least 2), else a full launch, so that the plain part
    // is whole launches; 0 when that launch has no kernel (the two steps then
    // run one per launch).
    int check_span(long long n) const {
        if (!L.fused() || L.wave_hs > 0 || L.inplace) return 0;
        const long long r = n % L.tb;
        const long long k = (r >= 2) ? r : L.tb;
        return (k <= n && stepN_supported(L.prec, (int)k, L.th)) ? (int)k : 0;
    }

    // Launches for `nplain` plain steps, then optionally a write-u step and a
    // residual check (a check step, or in place a launch without a step) +
    // finalize.  With two buffers and the tile kernel, the write-u step, the
    // check step and the plain steps before them that do not fill a launch run
    // as one fused launch whose last two steps form the check.
    hipError_t enqueue_seq(long long nplain, bool writeu, bool check, hipStream_t st,
                           long long& ph) {
        hipError_t e = hipSuccess;
        const int span = (writeu && check) ? check_span(nplain + 2) : 0;
        const long long np = span ? nplain + 2 - span : nplain;
        long long i = 0;
        if (L.fused()) {
            for (; i + L.tb <= np && e == hipSuccess; i += L.tb) e = enqueue_fused(L.tb, st, ph);
            if (e == hipSuccess && fused_rest(np - i)) {
                e = enqueue_fused((int)(np - i), st, ph);
                i = np;
            }
        } else if (L.ip_blocked()) {
            e = enqueue_ip(np, st, ph);
            i = np;
        }
        for (; i < np && e == hipSuccess; ++i) e = enqueue_one(kPlain, st, ph);
        if (e == hipSuccess && span) {
            e = launch_stepN(L.prec, span, L.th, grid, st, launch_args((int)(ph & 1)), true,
                             L.sr_on());
            ++ph;
            if (e == hipSuccess) e = advance_sr(span, st);
            if (e == hipSuccess) e = enqueue_finalize(st);
            return e;
        }
        if (e == hipSuccess && writeu) e = enqueue_one(kWriteU, st, ph);
        if (e == hipSuccess && check) {
            if (L.inplace) {
                // u(n) of the current state without a step (no flip)
                e = launch_check_state(L.prec, L.eff_vy(), L.layout(L.cur ^ (int)(ph & 1)), grid,
                                       st, launch_args((int)(ph & 1)));
            } else {
                e = enqueue_one(kCheck, st, ph);
            }
            if (e == hipSuccess) e = enqueue_finalize(st);
        }
        return e;
    }

    // buffer flips (launch-parity increments) of enqueue_seq
    long long launches(long long nplain, bool writeu, bool check) const {
        const int span = (writeu && check) ? check_span(nplain + 2) : 0;
        if (span) return plain_launches(nplain + 2 - span) + 1;
        return plain_launches(nplain) + (writeu ? 1 : 0) + (check && !L.inplace ? 1 : 0);
    }

    // Steps of the launch that ends enqueue_chunk(nplain, writeu, true) (the
    // check launch): a fused check launch's span, else 1.
    int check_launch_steps(long long nplain, bool writeu) const {
        const long long rest = nplain % graph_chunk();
        const int span = writeu ? check_span(rest + 2) : 0;
        return span ? span : 1;
    }

    // Enqueue a chunk; long runs are replayed from captured graphs.  In place
    // with blocked launches, a graph from kLayNatural holds 63 steps (an odd
    // launch, then even ones) and one from kLaySwapped 64, so that whole
    // graphs need no single step to restore the layout's parity.
    hipError_t enqueue_chunk(long long nplain, bool writeu, bool check) {
        hipError_t e;
        while (true) {
            long long chunk = graph_chunk();
            if (L.ip_blocked() && L.layout(sel()) == kLayNatural) chunk = 63;
            if (nplain < chunk) break;
            if ((e = run_graph(chunk, false, false)) != hipSuccess) return e;
            nplain -= chunk;
        }
        if (nplain > 0 || writeu || check) {
            if (launches(nplain, writeu, check) >= 4) return run_graph(nplain, writeu, check);
            long long ph = phase;
            if ((e = enqueue_seq(nplain, writeu, check, stream, ph)) != hipSuccess) return e;
            phase = ph;
        }
        return hipSuccess;
    }

    hipError_t run_graph(long long nplain, bool writeu, bool check) {
        const int flip0 = (int)(phase & 1);
        const int kind = (writeu ? 1 : 0) | (check ? 2 : 0) | (L.general() ? 4 : 0) |
                         (L.inplace ? 8 : 0) | (L.sr_on() ? 16 : 0);
        const int fused = L.fused() ? L.tb | (L.th << 4)
                                    : (L.ip_blocked() ? L.tb | (L.wave_v << 8) | (1 << 12) : 0);
        auto key = std::make_tuple(nplain, kind, flip0 ^ (L.cur << 1), L.prec, L.eff_vy(), fused,
                                   (L.fused() || L.ip_blocked()) ? L.wave_hs : 0, grid);
        auto it = graphs.find(key);
        hipError_t e;
        if (it == graphs.end()) {
            if (graphs.size() > 32) drop_graphs();
            hipGraph_t gr;
            if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return e;
            long long ph = phase;
            hipError_t le = enqueue_seq(nplain, writeu, check, cap, ph);
            if ((e = hipStreamEndCapture(cap, &gr)) != hipSuccess) return e;
            if (le != hipSuccess) {
                (void)hipGraphDestroy(gr);
                return le;
            }
            hipGraphExec_t ex;
            e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (e != hipSuccess) return e;
            it = graphs.emplace(key, ex).first;
        }
        if ((e = hipGraphLaunch(it->second, stream)) != hipSuccess) return e;
        phase += launches(nplain, writeu, check);
        return hipSuccess;
    }
};


extern "C" {

static size_t workspace_bytes(int nx, int ny, int precision, bool polish, bool inplace) {
    if (nx < 1 || ny < 1 || !valid_prec(precision)) return 0;
    const long long N = (long long)nx * ny;
    const long long mi = max_items(nx, ny);
    size_t b = al(sizeof(SlotDesc)) + 4 * al(sizeof(int)) + al(4 * 8) + al(sizeof(RiseGuard)) +
               al(mi * sizeof(Item)) +
               al(mi * 3 * 8) + al((kErrBlocks * 8 + 16) * 8);
    b += lattice_bytes(N, precision, polish, inplace);
    return b;
}

size_t lbm_workspace_bytes(int nx, int ny, int precision, int with_polish) {
    return workspace_bytes(nx, ny, precision, with_polish != 0, false);
}

size_t lbm_workspace_bytes_inplace(int nx, int ny, int precision) {
    return workspace_bytes(nx, ny, precision, false, true);
}

size_t lbm_workspace_bytes_inplace_blocked(int nx, int ny, int precision, int steps_per_launch,
                                           int segment_rows) {
    const size_t b = workspace_bytes(nx, ny, precision, false, true);
    if (b == 0 || steps_per_launch < 2 || steps_per_launch > 8 || segment_rows < 0 ||
        segment_rows > (1 << 20))
        return 0;
    return b + ip_halo_bytes(precision, steps_per_launch, nx, ny, segment_rows);
}

static int create_solver(int nx, int ny, int precision, int with_polish, bool inplace,
                         void* workspace, size_t workspace_bytes_given, void* stream,
                         lbm_solver** out) {
    if (!out) {
        g_create_error = "lbm_create: out is NULL";
        return LBM_E_ARG;
    }
    *out = nullptr;
    if (nx < 1 || ny < 1 || !valid_prec(precision) || (long long)nx * ny > (1LL << 31)) {
        g_create_error = "lbm_create: invalid size or precision";
        return LBM_E_ARG;
    }
    const size_t need = workspace_bytes(nx, ny, precision, with_polish != 0, inplace);
    if (!workspace || workspace_bytes_given < need ||
        (reinterpret_cast<uintptr_t>(workspace) % kAlign)) {
        g_create_error = "lbm_create: workspace NULL, misaligned or smaller than " +
                         std::to_string(need) + " bytes";
        return LBM_E_WORKSPACE;
    }
    lbm_solver* s = new lbm_solver();
    s->stream = reinterpret_cast<hipStream_t>(stream);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->h_result), 8 * sizeof(double),
                                           hipHostMallocDefault);
    if (e != hipSuccess) {
        g_create_error = std::string("lbm_create: ") + hipGetErrorString(e);
        if (s->cap) (void)hipStreamDestroy(s->cap);
        delete s;
        return LBM_E_HIP;
    }
    Lattice& L = s->L;
    L.nx = nx;
    L.ny = ny;
    L.N = (long long)nx * ny;
    L.plane = plane_of(L.N);
    L.prec0 = L.prec = precision;
    L.polish = with_polish != 0 && precision != LBM_FP64 && !inplace;
    L.inplace = inplace;
    default_tile(precision, nx, ny, L.bx_log2, L.vy);
    L.tb = inplace ? 1 : default_time_blocking(precision, (long long)nx * ny);
    L.th = fused_th(precision, L.tb, (long long)nx * ny);
    // planes beyond the tile kernel's 32-bit offsets: the wavefront, any width
    const FusedChoice fc = default_fused(precision, L.tb, nx, ny, s->cus, !L.tile_fits());
    L.wave_hs = inplace ? 0 : fc.wave_hs;
    L.wave_v = fc.wave_v;
    if (inplace) {
        // room beyond the minimum holds the in-place wavefront's halo copies:
        // the deepest launch whose default shape fits is the default
        L.halo = reinterpret_cast<char*>(workspace) + need;
        L.halo_cap = (workspace_bytes_given - need) / kAlign * kAlign;
        for (int k = 8; k >= 2; --k) {
            if (ip_halo_bytes(precision, k, nx, ny) <= L.halo_cap) {
                L.tb = k;
                L.wave_v = ip_wave_cols(precision, k, nx);
                L.wave_hs = ip_segment_rows(k, L.wave_v, nx, ny);
                break;
            }
        }
    }
    char* base = reinterpret_cast<char*>(workspace);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base + off;
        off += al(bytes);
        return p;
    };
    s->max_items_ = max_items(nx, ny);
    s->d_desc = reinterpret_cast<SlotDesc*>(take(sizeof(SlotDesc)));
    s->d_range = reinterpret_cast<int*>(take(2 * sizeof(int)));
    s->d_first = reinterpret_cast<int*>(take(sizeof(int)));
    s->d_count = reinterpret_cast<int*>(take(sizeof(int)));
    take(sizeof(int));
    s->d_result = reinterpret_cast<double*>(take(4 * 8));
    s->d_guard = reinterpret_cast<RiseGuard*>(take(sizeof(RiseGuard)));
    s->d_items = reinterpret_cast<Item*>(take(s->max_items_ * sizeof(Item)));
    s->d_partial = reinterpret_cast<double*>(take(s->max_items_ * 3 * 8));
    s->d_red = reinterpret_cast<double*>(take((kErrBlocks * 8 + 16) * 8));
    carve_lattice(base + off, L.N, precision, L.polish, L.mem, inplace);
    int rc = lbm_reset(s);
    if (rc != LBM_OK) {
        g_create_error = s->err;
        lbm_destroy(s);
        return rc;
    }
    *out = s;
    return LBM_OK;
}

int lbm_create(int nx, int ny, int precision, int with_polish, void* workspace,
               size_t workspace_bytes_given, void* stream, lbm_solver** out) {
    return create_solver(nx, ny, precision, with_polish, false, workspace, workspace_bytes_given,
                         stream, out);
}

int lbm_create_inplace(int nx, int ny, int precision, void* workspace,
                       size_t workspace_bytes_given, void* stream, lbm_solver** out) {
    return create_solver(nx, ny, precision, 0, true, workspace, workspace_bytes_given, stream,
                         out);
}

int lbm_destroy(lbm_solver* s) {
    if (!s) return LBM_E_ARG;
    (void)hipStreamSynchronize(s->stream);
    s->drop_graphs();
    if (s->cap) (void)hipStreamDestroy(s->cap);
    if (s->h_result) (void)hipHostFree(s->h_result);
    delete s;
    return LBM_OK;
}

namespace {
int half_exponent(const lbm_solver* s);
int set_half_exponent(lbm_solver* s, int e_new);
int refit_half(lbm_solver* s);
}  // namespace

int lbm_reset(lbm_solver* s) {
    if (!s) return LBM_E_ARG;
    Lattice& L = s->L;
    L.prec = L.prec0;
    L.cur = 0;
    s->phase = 0;
    s->steps = 0;
    L.mbase[0] = L.mbase[1] = 0.0;
    L.mbase_steps = 0;
    const double j0[2] = {0.0, 0.0};  // f = 0: no staggered moment
    L.set_stagger_state(0, j0);
    hipError_t e = zero_bytes(L.mem.buf[0], 8 * L.plane * elem_bytes(L.prec0), s->stream);
    if (e == hipSuccess) e = zero_bytes(L.mem.u, 2 * L.plane * 8, s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "lbm_reset");
    // f = 0 again: half storage takes the exponent a fresh solver would
    s->user_state = false;
    if (L.prec0 == LBM_FP16) L.e_scale = half_exponent(s);
    return s->sync_desc();
}

int lbm_set_material(lbm_solver* s, double lame_lambda, double lame_mu) {
    if (!s) return LBM_E_ARG;
    Rates r = s->L.rates;
    if (!material_rates(lame_lambda, lame_mu, r, s->err)) return LBM_E_MATERIAL;
    s->L.rates = r;
    s->L.lam = lame_lambda;
    s->L.mu = lame_mu;
    s->L.has_material = true;
    return refit_half(s);
}

int lbm_set_rates(lbm_solver* s, double theta, double w12, double w21, double w22) {
    if (!s) return LBM_E_ARG;
    auto ok = [](double w) { return std::isfinite(w) && w > 0.0 && w < 2.0; };
    if (!(theta > 0.0 && theta < 1.0) || !ok(w12) || !ok(w21) || !ok(w22))
        return s->fail(LBM_E_MATERIAL, "rates: need 0 < theta < 1 and 0 < omega < 2");
    Rates r = s->L.rates;
    r.theta = theta;
    r.w12 = w12;
    r.w21 = w21;
    r.w22 = w22;
    if (s->L.has_material && !material_rates(s->L.lam, s->L.mu, r, s->err)) return LBM_E_MATERIAL;
    s->L.rates = r;
    return s->sync_desc();
}

namespace {
// The force from a source (raw or corrected): statistics of the source
// before anything is overwritten, so that a rejected force leaves the
// previous one in place; then the mean-projected copy.
int set_force(lbm_solver* s, const ForceSrc& src, const char* what) {
    Lattice& L = s->L;
    double* stats = s->d_red + 8 * kErrBlocks;
    hipError_t e = force_stats(src, s->d_red, stats, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_result, stats, 8 * sizeof(double), hipMemcpyDeviceToHost,
                           s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, (std::string(what) + ": force statistics").c_str());
    double st[8];
    std::memcpy(st, s->h_result, sizeof(st));
    if (!std::isfinite(st[0]) || !std::isfinite(st[1]) || !std::isfinite(st[2]))
        return s->fail(LBM_E_ARG, std::string(what) + ": non-finite force (previous force kept)");
    // mean-projected copy (the kernel reads the statistics in stream order)
    if ((e = upload_force(L, src, stats, s->stream)) != hipSuccess) return s->hip_fail(e, what);
    L.has_force = true;
    record_force(L, st, s->steps);
    int rc = refit_half(s);
    if (rc != LBM_OK) return rc;
    const int w = force_warnings(st, L.N);
    if (w & LBM_W_MEAN_REMOVED)
        s->err = "body force had a non-zero mean: removed (the mean of u is conserved)";
    if (w & LBM_W_STAGGERED_LOAD)
        s->err = "body force has a k = (pi,0) or (0,pi) component: the staggered first moment "
                 "oscillates for good, no steady state is reached";
    return w;
}
}  // namespace

int lbm_set_body_force(lbm_solver* s, const double* gx, const double* gy) {
    if (!s) return LBM_E_ARG;
    if (!gx || !gy) return s->fail(LBM_E_ARG, "set_body_force: NULL force");
    return set_force(s, raw_force(gx, gy, s->L.nx, s->L.ny), "set_body_force");
}

int lbm_set_body_force_corrected(lbm_solver* s, const double* gx, const double* gy,
                                 const double* d2g) {
    if (!s) return LBM_E_ARG;
    if (!gx || !gy) return s->fail(LBM_E_ARG, "set_body_force_corrected: NULL force");
    Lattice& L = s->L;
    if (!L.has_material)
        return s->fail(LBM_E_STATE, "set_body_force_corrected: set the material first");
    const Rates& r = L.rates;
    double E, nu;
    young_poisson(L.lam, L.mu, E, nu);
    const double t12 = 1.0 / r.w12 - 0.5, t21 = 1.0 / r.w21 - 0.5, t22 = 1.0 / r.w22 - 0.5;
    const ErrorConstants kx = error_constants(E, nu, r.theta, t12, t21, t22);
    const ErrorConstants ky = error_constants(E, nu, r.theta, t21, t12, t22);
    ForceSrc src = raw_force(gx, gy, L.nx, L.ny);
    src.mode = d2g ? ForceSrc::kGiven : ForceSrc::kCentral;
    src.d2 = d2g;
    for (int i = 0; i < 3; ++i) {
        src.cx[i] = kx.D[i];
        src.cy[i] = ky.D[i];
    }
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(src.cx[i]) || !std::isfinite(src.cy[i]))
            return s->fail(LBM_E_MATERIAL, "set_body_force_corrected: constants not finite "
                                           "(nu = 1 or theta = 0)");
    return set_force(s, src, "set_body_force_corrected");
}

int lbm_leading_error_constants(double lame_lambda, double lame_mu, double theta, double omega12,
                                double omega21, double omega22, double out[10]) {
    if (!out) return LBM_E_ARG;
    Rates r;
    r.theta = theta;
    std::string err;
    auto ok = [](double w) { return std::isfinite(w) && w > 0.0 && w < 2.0; };
    if (!(theta > 0.0 && theta < 1.0) || !ok(omega12) || !ok(omega21) || !ok(omega22) ||
        !material_rates(lame_lambda, lame_mu, r, err))
        return LBM_E_MATERIAL;
    double E, nu;
    young_poisson(lame_lambda, lame_mu, E, nu);
    const ErrorConstants k = error_constants(E, nu, theta, 1.0 / omega12 - 0.5,
                                             1.0 / omega21 - 0.5, 1.0 / omega22 - 0.5);
    double c2 = 0.0, d2 = 0.0;
    for (int i = 0; i < 5; ++i) {
        out[i] = k.C[i];
        c2 += k.C[i] * k.C[i];
    }
    for (int i = 0; i < 3; ++i) {
        out[5 + i] = k.D[i];
        d2 += k.D[i] * k.D[i];
    }
    out[8] = std::sqrt(c2);
    out[9] = std::sqrt(c2 + d2);
    for (int i = 0; i < 10; ++i)
        if (!std::isfinite(out[i])) return LBM_E_MATERIAL;
    return LBM_OK;
}

int lbm_fourth_order_rates(double lame_lambda, double lame_mu, double theta, double out[2]) {
    if (!out) return LBM_E_ARG;
    Rates r;
    r.theta = theta;
    std::string err;
    if (!(theta > 0.0 && theta < 1.0) || !material_rates(lame_lambda, lame_mu, r, err))
        return LBM_E_MATERIAL;
    double w12 = 0.0, w22 = 0.0;
    if (!fourth_order_rates(lame_lambda, lame_mu, theta, w12, w22)) return LBM_E_MATERIAL;
    out[0] = w12;
    out[1] = w22;
    return LBM_OK;
}

int lbm_set_tile(lbm_solver* s, int bx_log2, int rows_per_thread, int blocks_per_cu) {
    if (!s) return LBM_E_ARG;
    if (bx_log2 < 0 || bx_log2 > 8 ||
        !(rows_per_thread == 1 || rows_per_thread == 2 || rows_per_thread == 4) ||
        blocks_per_cu < 0 || blocks_per_cu > 64)
        return s->fail(LBM_E_ARG,
                       "set_tile: bx_log2 in 0..8, rows_per_thread in {1,2,4}, blocks_per_cu in 0..64");
    s->L.bx_log2 = bx_log2;
    s->L.vy = rows_per_thread;
    s->blocks_per_cu = blocks_per_cu;
    return s->sync_desc();
}

int lbm_set_time_blocking(lbm_solver* s, int steps_per_launch) {
    if (!s) return LBM_E_ARG;
    if (steps_per_launch < 1 || steps_per_launch > 8)
        return s->fail(LBM_E_ARG, "set_time_blocking: steps_per_launch must be in 1..8");
    Lattice& L = s->L;
    if (L.inplace) {
        if (steps_per_launch >= 2) {
            const int v = ip_wave_cols(L.prec, steps_per_launch, L.nx);
            const int hs = s->fused_auto ? ip_segment_rows(steps_per_launch, v, L.nx, L.ny)
                                         : L.wave_hs;
            const size_t need = wave_halo_bytes(L.prec, steps_per_launch, v, L.nx, L.ny, hs);
            if (need > L.halo_cap)
                return s->fail(LBM_E_WORKSPACE,
                               "set_time_blocking: in place, " + std::to_string(steps_per_launch) +
                                   " steps per launch need " + std::to_string(need) +
                                   " bytes of halo room beyond lbm_workspace_bytes_inplace (have " +
                                   std::to_string(L.halo_cap) +
                                   "; see lbm_workspace_bytes_inplace_blocked)");
            L.wave_v = v;
            L.wave_hs = hs;
        }
        L.tb = steps_per_launch;
        return s->sync_desc();
    }
    L.tb = steps_per_launch;
    L.th = fused_th(L.prec, steps_per_launch, L.N, L.th_user);
    if (s->fused_auto) {
        const FusedChoice fc = default_fused(L.prec, steps_per_launch, L.nx, L.ny, s->cus,
                                             !L.tile_fits());
        L.wave_hs = fc.wave_hs;
    }
    L.wave_v = wave_cols(L.prec, steps_per_launch, L.nx, L.ny);
    return s->sync_desc();
}

int lbm_set_tile_rows(lbm_solver* s, int rows) {
    if (!s) return LBM_E_ARG;
    Lattice& L = s->L;
    if (rows != 0 && !(rows == 8 || rows == 12 || rows == 16 || rows == 24))
        return s->fail(LBM_E_ARG, "set_tile_rows: rows must be 0, 8, 12, 16 or 24");
    if (rows != 0 && L.fused() && L.wave_hs == 0 && !stepN_supported(L.prec, L.tb, rows))
        return s->fail(LBM_E_ARG, "set_tile_rows: no tile kernel of that height for this "
                                  "storage type and steps per launch");
    L.th_user = rows;
    L.th = fused_th(L.prec, L.tb, L.N, rows);
    return s->sync_desc();
}

int lbm_set_fused_kernel(lbm_solver* s, int kind, int segment_rows) {
    if (!s) return LBM_E_ARG;
    if (s->L.inplace) {
        Lattice& L = s->L;
        if (kind != LBM_FUSED_WAVEFRONT)
            return s->fail(LBM_E_STATE, "set_fused_kernel: in place, the wavefront is the only "
                                        "fused kernel");
        if (segment_rows < 1 || segment_rows > (1 << 20))
            return s->fail(LBM_E_ARG, "set_fused_kernel: segment_rows must be in 1..2^20");
        if (L.tb >= 2) {
            const size_t need = wave_halo_bytes(L.prec, L.tb, L.wave_v, L.nx, L.ny, segment_rows);
            if (need > L.halo_cap)
                return s->fail(LBM_E_WORKSPACE,
                               "set_fused_kernel: in place, segments of " +
                                   std::to_string(segment_rows) + " rows need " +
                                   std::to_string(need) + " bytes of halo room (have " +
                                   std::to_string(L.halo_cap) + ")");
        }
        L.wave_hs = segment_rows;
        s->fused_auto = false;
        return s->sync_desc();
    }
    if (kind == LBM_FUSED_TILE) {
        s->L.wave_hs = 0;
        s->fused_auto = false;
    } else if (kind == LBM_FUSED_WAVEFRONT) {
        if (segment_rows < 1 || segment_rows > (1 << 20))
            return s->fail(LBM_E_ARG, "set_fused_kernel: segment_rows must be in 1..2^20");
        s->L.wave_hs = segment_rows;
        s->L.wave_v = wave_cols(s->L.prec, s->L.tb, s->L.nx, s->L.ny);
        s->fused_auto = false;
    } else {
        return s->fail(LBM_E_ARG, "set_fused_kernel: kind must be LBM_FUSED_TILE or LBM_FUSED_WAVEFRONT");
    }
    return s->sync_desc();
}

int lbm_set_stochastic_rounding(lbm_solver* s, int on, unsigned int seed) {
    if (!s) return LBM_E_ARG;
    Lattice& L = s->L;
    if (on && (L.prec0 != LBM_FP16 || L.inplace))
        return s->fail(LBM_E_STATE, "set_stochastic_rounding: half storage with two buffers only");
    L.sr = on != 0;
    L.sr_seed = seed;
    return s->sync_desc();
}

int lbm_get_launch_config(const lbm_solver* s, int out[4]) {
    if (!s || !out) return LBM_E_ARG;
    const Lattice& L = s->L;
    out[0] = L.tb;
    if (L.ip_blocked()) {
        out[1] = LBM_FUSED_WAVEFRONT;
        out[2] = L.wave_hs;
        out[3] = kBlock;
    } else if (!L.fused()) {
        out[1] = -1;
        out[2] = L.inplace ? 0 : L.eff_vy();
        out[3] = kBlock;
    } else if (L.wave_hs > 0) {
        out[1] = LBM_FUSED_WAVEFRONT;
        out[2] = L.wave_hs;
        out[3] = kBlock;
    } else {
        out[1] = LBM_FUSED_TILE;
        out[2] = L.th;
        out[3] = fused_nt(L.prec, L.tb, L.th);
    }
    return LBM_OK;
}

int lbm_get_wave_columns(const lbm_solver* s) {
    if (!s) return LBM_E_ARG;
    return ((s->L.fused() && s->L.wave_hs > 0) || s->L.ip_blocked()) ? s->L.wave_v : 0;
}

int lbm_step(lbm_solver* s, long long nsteps) {
    if (!s || nsteps < 0) return s ? s->fail(LBM_E_ARG, "step: nsteps < 0") : LBM_E_ARG;
    if (!s->L.has_material || !s->L.has_force)
        return s->fail(LBM_E_STATE, "step: material and body force must be set first");
    hipError_t e = s->enqueue_chunk(nsteps, false, false);
    if (e != hipSuccess) return s->hip_fail(e, "lbm_step");
    s->steps += nsteps;
    return LBM_OK;
}

int lbm_set_polish(lbm_solver* s, double r_switch) {
    if (!s) return LBM_E_ARG;
    if (r_switch > 0.0 && (!s->L.polish || s->L.prec0 == LBM_FP64))
        return s->fail(LBM_E_STATE, "set_polish: FP32/FP16 solver created with_polish needed");
    s->r_switch = r_switch > 0.0 ? r_switch : 0.0;
    return LBM_OK;
}

int lbm_current_precision(const lbm_solver* s) { return s ? s->L.prec : LBM_E_ARG; }
long long lbm_steps_done(const lbm_solver* s) { return s ? s->steps : -1; }

namespace {
// Switch the solver to FP64 storage: exact widening of the current state.
int promote_solver(lbm_solver* s) {
    Lattice& L = s->L;
    if (L.prec == LBM_FP64 || !L.polish) return LBM_OK;
    const int sl = s->sel();
    const long long n = 8 * L.plane;
    const double factor = (L.prec == LBM_FP16) ? std::ldexp(1.0, L.e_scale) : 1.0;
    if (L.prec == LBM_FP32)
        hipLaunchKernelGGL((k_recast<float, double>), dim3(blocks_for(n)), dim3(kBlock), 0,
                           s->stream, reinterpret_cast<const float*>(L.mem.buf[sl]),
                           reinterpret_cast<double*>(L.mem.pbuf[0]), n, factor);
    else
        hipLaunchKernelGGL((k_recast<__half, double>), dim3(blocks_for(n)), dim3(kBlock), 0,
                           s->stream, reinterpret_cast<const __half*>(L.mem.buf[sl]),
                           reinterpret_cast<double*>(L.mem.pbuf[0]), n, factor);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return s->hip_fail(e, "promote");
    L.prec = LBM_FP64;
    L.cur = 0;
    s->phase = 0;
    default_tile(LBM_FP64, L.nx, L.ny, L.bx_log2, L.vy);
    L.tb = default_time_blocking(LBM_FP64, L.N);
    L.th = fused_th(LBM_FP64, L.tb, L.N);
    const FusedChoice fc = default_fused(LBM_FP64, L.tb, L.nx, L.ny, s->cus, !L.tile_fits());
    L.wave_hs = fc.wave_hs;
    L.wave_v = fc.wave_v;
    s->fused_auto = true;
    // sync_desc folds phase into cur: phase is 0 so cur stays 0
    int rc = s->sync_desc();
    if (rc != LBM_OK) return rc;
    // the narrow phase leaves rounding noise in the undamped modes (the
    // staggered moments and the mean); reset them so that the FP64 phase
    // converges to the exact trajectory's fixed point
    double target[2], stag[2];
    L.mean_target(s->steps, target);
    L.stag_target_stored(s->steps, stag);
    e = neutral_reset(LBM_FP64, L.desc(), s->sel(), target, stag, s->d_red, s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "promote: neutral modes");
    return LBM_OK;
}

// Half storage: the power-of-two exponent for the current state.  From f = 0
// (creation, reset) the force's steady-state bound alone (a zero force sets
// no bound); after lbm_set_populations the larger of that and the exponent
// that maps the given state's max |f| to 2^12.
int half_exponent(const lbm_solver* s) {
    const Lattice& L = s->L;
    const int ef = (L.has_force && L.has_material && L.gmax > 0.0)
                       ? initial_half_exponent(L, L.gmax) : INT_MIN;
    const int e = s->user_state ? std::max(ef, s->e_user) : ef;
    return (e == INT_MIN) ? 0 : std::max(-100, std::min(100, e));
}

// Change the half-storage exponent.  A live state (set by the caller, or any
// state after the first step) is rescaled by the power of two (exact for
// normal halves), so that it keeps its values.
int set_half_exponent(lbm_solver* s, int e_new) {
    Lattice& L = s->L;
    e_new = std::max(-100, std::min(100, e_new));
    if (L.prec != LBM_FP16 || e_new == L.e_scale) return LBM_OK;
    if (s->user_state || s->steps > 0) {
        __half* p = reinterpret_cast<__half*>(L.mem.buf[s->sel()]);
        const long long n = 8 * L.plane;
        hipLaunchKernelGGL((k_recast<__half, __half>), dim3(blocks_for(n)), dim3(kBlock), 0,
                           s->stream, p, p, n, std::ldexp(1.0, L.e_scale - e_new));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return s->hip_fail(e, "half rescale");
    }
    L.e_scale = e_new;
    return s->sync_desc();
}

// After a new force or material: before the first step the exponent follows
// half_exponent; later the scale only coarsens (a larger steady-state bound
// would otherwise overflow the half range before the next checked rescale).
int refit_half(lbm_solver* s) {
    const Lattice& L = s->L;
    if (L.prec != LBM_FP16) return s->sync_desc();
    const int e = half_exponent(s);
    if (s->steps == 0) return set_half_exponent(s, e);
    return e > L.e_scale ? set_half_exponent(s, e) : s->sync_desc();
}

// Rescale half storage so that max |stored| stays within [2^10, 2^14].
int rescale_half(lbm_solver* s, double fmax_stored) {
    Lattice& L = s->L;
    if (L.prec != LBM_FP16 || !(fmax_stored > 0.0) || !std::isfinite(fmax_stored)) return LBM_OK;
    int k = 0;
    if (fmax_stored > 16384.0) k = (int)std::ceil(std::log2(fmax_stored / 4096.0));
    else if (fmax_stored < 1024.0) k = -(int)std::floor(std::log2(4096.0 / fmax_stored));
    if (k == 0) return LBM_OK;
    const int sl = s->sel();
    const long long n = 8 * L.plane;
    __half* p = reinterpret_cast<__half*>(L.mem.buf[sl]);
    hipLaunchKernelGGL((k_recast<__half, __half>), dim3(blocks_for(n)), dim3(kBlock), 0, s->stream,
                       p, p, n, std::ldexp(1.0, -k));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return s->hip_fail(e, "rescale");
    L.e_scale += k;
    return s->sync_desc();
}
}  // namespace

namespace {
// Whether lbm_solve_to_tol runs as one-workgroup launches: two buffers, a lattice
// whose two population buffers fit in LDS, FP64 or FP32 storage (half storage
// rescales between checks on the host); FP32 with a polish switch only if the
// FP64 state it switches to fits as well.
bool small_solve_ok(const lbm_solver* s) {
    const Lattice& L = s->L;
    if (s->small_budget <= 0 || L.inplace || L.N > small_max_sites(L.prec)) return false;
    if (L.prec == LBM_FP64) return true;
    return L.prec == LBM_FP32 && (!(s->r_switch > 0.0) || L.N <= small_max_sites(LBM_FP64));
}

int solve_small(lbm_solver* s, double tol, long long max_steps, long long K,
                long long* steps_done, double* residual) {
    Lattice& L = s->L;
    SmallLaunch P;
    P.d = L.desc();
    P.sel = s->sel();
    P.check = K;
    P.max_steps = max_steps;
    P.tol = tol;
    P.out = s->d_result;
    P.guard_checks = s->guard_checks;
    P.guard = s->d_guard;
    hipLaunchKernelGGL(k_guard_clear, dim3(1), dim3(1), 0, s->stream, s->d_guard);
    long long m = 0;
    double r = NAN;
    int nondec = 0;
    while (true) {
        P.m0 = m;
        P.have_prev = m > 0;
        P.budget = s->small_budget;
        P.r_in = r;
        P.r_switch = (L.prec != LBM_FP64) ? s->r_switch : 0.0;
        P.nondec_in = nondec;
        hipError_t e = launch_solve_small(L.prec, L.general(), s->stream, P);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->h_result, s->d_result, 4 * 8, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "solve_to_tol");
        const long long m_new = (long long)s->h_result[0];
        const int outcome = (int)s->h_result[2];
        r = s->h_result[1];
        nondec = (int)s->h_result[3];
        s->steps += m_new - m;
        m = m_new;
        *steps_done = m;
        *residual = r;
        if (outcome == kSmallConverged) return LBM_OK;
        if (outcome == kSmallLimit) return LBM_NOT_CONVERGED;
        if (outcome == kSmallDiverged) {
            s->err = std::isfinite(r) ? "solve_to_tol: the update norm kept rising (diverged)"
                                      : "solve_to_tol: residual is not finite (diverged)";
            return LBM_E_DIVERGED;
        }
        if (outcome == kSmallSwitch) {  // narrow storage to FP64, then on in FP64
            const int rc = promote_solver(s);
            if (rc != LBM_OK) return rc;
            P.d = L.desc();
            P.sel = s->sel();
            // the FP64 phase starts a new residual history
            hipLaunchKernelGGL(k_guard_clear, dim3(1), dim3(1), 0, s->stream, s->d_guard);
        }
    }
}
}  // namespace

int lbm_set_divergence_guard(lbm_solver* s, int checks) {
    if (!s) return LBM_E_ARG;
    if (checks < 0) return s->fail(LBM_E_ARG, "set_divergence_guard: checks must be >= 0");
    s->guard_checks = checks;
    return LBM_OK;
}

int lbm_set_small_solve(lbm_solver* s, long long steps_per_launch) {
    if (!s) return LBM_E_ARG;
    if (steps_per_launch < 0)
        return s->fail(LBM_E_ARG, "set_small_solve: steps_per_launch must be >= 0");
    s->small_budget = steps_per_launch;
    return LBM_OK;
}

int lbm_solve_to_tol(lbm_solver* s, double tol, long long max_steps, int check_every,
                     long long* steps_done, double* residual) {
    if (!s) return LBM_E_ARG;
    if (!(tol >= 0.0) || max_steps < 0 || check_every < 1 || !steps_done || !residual)
        return s->fail(LBM_E_ARG, "solve_to_tol: need tol >= 0, max_steps >= 0, check_every >= 1");
    if (!s->L.has_material || !s->L.has_force)
        return s->fail(LBM_E_STATE, "solve_to_tol: material and body force must be set first");
    if (small_solve_ok(s)) return solve_small(s, tol, max_steps, check_every, steps_done, residual);
    const long long K = check_every;
    long long n = 0;             // steps taken by this call
    bool have_prev_u = false;    // u buffer holds u(n - 1)
    double r = NAN, r_last = INFINITY;
    int nondecreasing = 0;
    RiseGuard guard;
    guard.clear();
    *residual = NAN;
    *steps_done = 0;
    const bool inplace = s->L.inplace;
    while (true) {
        // step index of the next check.  Two buffers: the check launch is step
        // j + 1, computing u(j) on the way, and steps back if it stops.  In
        // place: steps run to j and a launch without a step computes u(j).
        const long long j = inplace ? n + K : ((n == 0) ? K : n - 1 + K);
        if (j > max_steps) {
            const long long rest = max_steps - n;
            hipError_t e = s->enqueue_chunk(rest, false, false);
            if (e != hipSuccess) return s->hip_fail(e, "solve_to_tol");
            s->steps += rest;
            n = max_steps;
            if ((e = hipStreamSynchronize(s->stream)) != hipSuccess)
                return s->hip_fail(e, "solve_to_tol");
            *steps_done = n;
            *residual = r;
            return LBM_NOT_CONVERGED;
        }
        const bool need_writeu = inplace ? !(have_prev_u && j - 1 == n)
                                         : !(have_prev_u && j - 1 == n - 1);
        const long long nplain =
            inplace ? (j - n - (need_writeu ? 1 : 0)) : (need_writeu ? (j - 1 - n) : 0);
        const int span = s->check_launch_steps(nplain, need_writeu);
        hipError_t e = s->enqueue_chunk(nplain, need_writeu, true);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->h_result, s->d_result, 4 * 8, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "solve_to_tol");
        const double d2 = s->h_result[0], u2 = s->h_result[1], fm = s->h_result[2];
        r = (u2 == 0.0) ? (d2 == 0.0 ? 0.0 : INFINITY) : std::sqrt(d2 / u2);
        if (d2 != d2 || u2 != u2 || !std::isfinite(u2) || !std::isfinite(fm)) r = NAN;
        *residual = r;
        const long long after = inplace ? j : j + 1;  // steps after the check launch
        s->steps += after - n;
        n = after;
        have_prev_u = true;
        // stop rules, in the order of the one-workgroup solve: a non-finite
        // residual, the tolerance, the limit, the divergence guard
        bool diverged = !std::isfinite(r) && !(u2 == 0.0 && d2 != 0.0);
        bool stop = diverged || r <= tol || j == max_steps;
        if (!stop && guard.update(std::sqrt(d2), s->guard_checks)) diverged = stop = true;
        if (stop) {
            if (!inplace) {
                // the check launch advanced to j + 1 and its source buffer still
                // holds the state it started from, f(j + 1 - span): take the
                // launch back and advance the span - 1 steps to f(j) again
                s->phase -= 1;
                s->steps -= span;
                if (span > 1) {
                    hipError_t e2 = s->enqueue_chunk(span - 1, false, false);
                    if (e2 != hipSuccess) return s->hip_fail(e2, "solve_to_tol");
                    s->steps += span - 1;
                }
            }
            n = j;
            *steps_done = n;
            if (diverged) {
                s->err = std::isfinite(r) ? "solve_to_tol: the update norm kept rising (diverged)"
                                          : "solve_to_tol: residual is not finite (diverged)";
                return LBM_E_DIVERGED;
            }
            return (r <= tol) ? LBM_OK : LBM_NOT_CONVERGED;
        }
        // precision management between chunks
        if (s->L.prec == LBM_FP16) {
            int rc = rescale_half(s, fm);
            if (rc != LBM_OK) return rc;
        }
        if (s->r_switch > 0.0 && s->L.prec != LBM_FP64) {
            nondecreasing = (r >= r_last) ? nondecreasing + 1 : 0;
            if (r <= s->r_switch || nondecreasing >= 2) {
                int rc = promote_solver(s);
                if (rc != LBM_OK) return rc;
                have_prev_u = true;  // u buffer (FP64, unscaled) is unaffected
                guard.clear();       // the FP64 phase starts a new residual history
            }
        }
        r_last = r;
    }
}

int lbm_step_checked(lbm_solver* s, long long nsteps, double* residual) {
    if (!s) return LBM_E_ARG;
    if (nsteps < 2 || !residual)
        return s->fail(LBM_E_ARG, "step_checked: need nsteps >= 2 and a residual output");
    if (!s->L.has_material || !s->L.has_force)
        return s->fail(LBM_E_STATE, "step_checked: material and body force must be set first");
    *residual = NAN;
    // two buffers: nsteps - 2 plain steps, a write-u step and the check step;
    // in place: the check launch does not step, so one plain step follows it
    hipError_t e = s->enqueue_chunk(nsteps - 2, true, true);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_result, s->d_result, 4 * 8, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "step_checked");
    s->steps += s->L.inplace ? nsteps - 1 : nsteps;
    const double d2 = s->h_result[0], u2 = s->h_result[1], fm = s->h_result[2];
    double r = (u2 == 0.0) ? (d2 == 0.0 ? 0.0 : INFINITY) : std::sqrt(d2 / u2);
    if (d2 != d2 || u2 != u2 || !std::isfinite(u2) || !std::isfinite(fm)) r = NAN;
    *residual = r;
    if (!std::isfinite(r) && !(u2 == 0.0 && d2 != 0.0)) {
        s->err = "step_checked: residual is not finite (diverged)";
        return LBM_E_DIVERGED;
    }
    if (s->L.prec == LBM_FP16) {
        int rc = rescale_half(s, fm);
        if (rc != LBM_OK) return rc;
    }
    if (s->L.inplace) {
        if ((e = s->enqueue_chunk(1, false, false)) != hipSuccess)
            return s->hip_fail(e, "step_checked");
        s->steps += 1;
    }
    return LBM_OK;
}

int lbm_get_displacement(lbm_solver* s, double* ux, double* uy) {
    if (!s) return LBM_E_ARG;
    if (!ux || !uy) return s->fail(LBM_E_ARG, "get_displacement: NULL output");
    if (!s->L.has_force) return s->fail(LBM_E_STATE, "get_displacement: no body force set");
    hipError_t e = extract_u(s->L.prec, s->L.desc(), s->sel(), s->L.layout(s->sel()), ux, uy,
                             s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "get_displacement");
    return LBM_OK;
}

int lbm_get_stress(lbm_solver* s, double* sxx, double* syy, double* sxy) {
    if (!s) return LBM_E_ARG;
    if (!sxx || !syy || !sxy) return s->fail(LBM_E_ARG, "get_stress: NULL output");
    if (!s->L.has_material) return s->fail(LBM_E_STATE, "get_stress: no material set");
    const SlotDesc d = s->L.desc();
    hipError_t e;
    if (s->L.prec == LBM_FP64) e = launch_stress<double>(d, s->sel(), s->L.layout(s->sel()), s->L.rates, sxx, syy, sxy, s->stream);
    else if (s->L.prec == LBM_FP32) e = launch_stress<float>(d, s->sel(), s->L.layout(s->sel()), s->L.rates, sxx, syy, sxy, s->stream);
    else e = launch_stress<__half>(d, s->sel(), s->L.layout(s->sel()), s->L.rates, sxx, syy, sxy, s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "get_stress");
    return LBM_OK;
}

int lbm_error_norms(lbm_solver* s, const double* ux_ref, const double* uy_ref, double out[4]) {
    if (!s) return LBM_E_ARG;
    if (!ux_ref || !uy_ref || !out) return s->fail(LBM_E_ARG, "error_norms: NULL argument");
    if (!s->L.has_force) return s->fail(LBM_E_STATE, "error_norms: no body force set");
    // displacement into the u planes of the workspace, then the two-stage reduction
    double* ux = s->L.mem.u;
    double* uy = s->L.mem.u + s->L.plane;
    hipError_t e = extract_u(s->L.prec, s->L.desc(), s->sel(), s->L.layout(s->sel()), ux, uy,
                             s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "error_norms");
    hipLaunchKernelGGL(k_err_norms, dim3(kErrBlocks), dim3(kBlock), 0, s->stream, ux, uy, ux_ref,
                       uy_ref, s->L.N, s->d_red);
    hipLaunchKernelGGL(k_reduce4<kErrMask>, dim3(1), dim3(kBlock), 0, s->stream, s->d_red,
                       kErrBlocks, s->d_red + 4 * kErrBlocks);
    if ((e = hipGetLastError()) == hipSuccess)
        e = hipMemcpyAsync(s->h_result, s->d_red + 4 * kErrBlocks, 4 * 8, hipMemcpyDeviceToHost,
                           s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "error_norms");
    for (int c = 0; c < 4; ++c) out[c] = s->h_result[c];
    return LBM_OK;
}

int lbm_error_norms_noalloc(int nx, int ny, const double* ux, const double* uy,
                            const double* ux_ref, const double* uy_ref, double* out,
                            void* stream) {
    if (nx < 1 || ny < 1 || (long long)nx * ny > (1LL << 31)) {
        g_create_error = "error_norms_noalloc: need 1 <= nx, ny and nx * ny <= 2^31";
        return LBM_E_ARG;
    }
    if (!ux || !uy || !ux_ref || !uy_ref || !out) {
        g_create_error = "error_norms_noalloc: NULL argument";
        return LBM_E_ARG;
    }
    hipError_t e;
    double* part = noalloc_scratch(&e);
    if (!part) {
        g_create_error = std::string("error_norms_noalloc: scratch address: ") + hipGetErrorString(e);
        return LBM_E_HIP;
    }
    // the kernels of lbm_error_norms: every block writes its four partials, so
    // nothing in the scratch needs clearing
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_err_norms, dim3(kErrBlocks), dim3(kBlock), 0, st, ux, uy, ux_ref, uy_ref,
                       (long long)nx * ny, part);
    hipLaunchKernelGGL(k_reduce4<kErrMask>, dim3(1), dim3(kBlock), 0, st, part, kErrBlocks, out);
    if ((e = hipGetLastError()) != hipSuccess) {
        g_create_error = std::string("error_norms_noalloc: ") + hipGetErrorString(e);
        return LBM_E_HIP;
    }
    return LBM_OK;
}

int lbm_get_populations(lbm_solver* s, double* f) {
    if (!s) return LBM_E_ARG;
    if (!f) return s->fail(LBM_E_ARG, "get_populations: NULL output");
    const SlotDesc d = s->L.desc();
    hipError_t e;
    if (s->L.prec == LBM_FP64) e = launch_get_f<double>(d, s->sel(), s->L.layout(s->sel()), f, s->stream);
    else if (s->L.prec == LBM_FP32) e = launch_get_f<float>(d, s->sel(), s->L.layout(s->sel()), f, s->stream);
    else e = launch_get_f<__half>(d, s->sel(), s->L.layout(s->sel()), f, s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "get_populations");
    return LBM_OK;
}

int lbm_set_populations(lbm_solver* s, const double* f) {
    if (!s) return LBM_E_ARG;
    if (!f) return s->fail(LBM_E_ARG, "set_populations: NULL input");
    if (s->L.prec == LBM_FP16) {
        // Half storage: choose the power-of-two scale for the given state, so
        // that its max |f| maps to 2^12 (the middle of the window the checked
        // rescale keeps), and never finer than the force's steady-state bound.
        // Otherwise a state far above that bound would overflow the half range.
        Lattice& L = s->L;
        const long long h = 4 * L.N;  // the eight planes as two halves
        hipLaunchKernelGGL(k_force_stats, dim3(kErrBlocks), dim3(kBlock), 0, s->stream, f, f + h,
                           h, s->d_red);
        hipLaunchKernelGGL(k_reduce4<kForceMask>, dim3(1), dim3(kBlock), 0, s->stream, s->d_red,
                           kErrBlocks, s->d_red + 4 * kErrBlocks);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->h_result, s->d_red + 4 * kErrBlocks, 4 * 8,
                               hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return s->hip_fail(e, "set_populations: max |f|");
        const double fmax = s->h_result[3];
        if (!std::isfinite(fmax)) return s->fail(LBM_E_ARG, "set_populations: non-finite input");
        // the old state is overwritten below: set the exponent without rescaling it
        s->user_state = true;
        s->e_user = (fmax > 0.0) ? (int)std::ceil(std::log2(fmax / 4096.0)) : INT_MIN;
        L.e_scale = half_exponent(s);
        const int rc = s->sync_desc();
        if (rc != LBM_OK) return rc;
    }
    const SlotDesc d = s->L.desc();
    const double sc = d.gscale;
    hipError_t e;
    if (s->L.prec == LBM_FP64) e = launch_set_f<double>(d, s->sel(), s->L.layout(s->sel()), f, sc, s->stream);
    else if (s->L.prec == LBM_FP32) e = launch_set_f<float>(d, s->sel(), s->L.layout(s->sel()), f, sc, s->stream);
    else e = launch_set_f<__half>(d, s->sel(), s->L.layout(s->sel()), f, sc, s->stream);
    if (e == hipSuccess && !s->L.inplace)  // in place: no polish switch, no targets
        e = neutral_measure(s->L.prec, d, s->sel(), s->d_red, s->h_result, s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "set_populations");
    if (!s->L.inplace) {
        // the given state starts the exact trajectory: its mean first moments,
        // and its staggered ones (the stored field's staggered sums are -J)
        s->L.mbase[0] = s->h_result[4];
        s->L.mbase[1] = s->h_result[5];
        s->L.mbase_steps = s->steps;
        const double j[2] = {-s->h_result[0], -s->h_result[1]};
        s->L.set_stagger_state(s->steps, j);
    }
    return LBM_OK;
}

int lbm_debug_stream_only(lbm_solver* s, long long nsteps) {
    if (!s || nsteps < 0) return LBM_E_ARG;
    hipError_t e = hipSuccess;
    for (long long i = 0; i < nsteps && e == hipSuccess; ++i) {
        const StepLaunch a = s->launch_args((int)(s->phase & 1));
        const int lay = s->L.layout(s->sel());
        if (s->L.prec == LBM_FP64) e = launch_stream_only<double>(s->grid, s->stream, a, lay);
        else if (s->L.prec == LBM_FP32) e = launch_stream_only<float>(s->grid, s->stream, a, lay);
        else e = launch_stream_only<__half>(s->grid, s->stream, a, lay);
        ++s->phase;
    }
    if (e != hipSuccess) return s->hip_fail(e, "debug_stream_only");
    s->L.stream_only_stagger(s->steps, nsteps);  // streaming alone flips J
    s->steps += nsteps;
    s->L.mbase_steps += nsteps;  // streaming alone adds no force
    return LBM_OK;
}

const char* lbm_last_error(const lbm_solver* s) {
    if (!s) return g_create_error.c_str();
    return s->err.c_str();
}

}  // extern "C"

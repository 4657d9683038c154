// Batches of independent periodic lattices (uneven sizes and materials)
// stepped together: one persistent launch per storage precision and step
// walks a work list of (lattice, tile) items; per-lattice arithmetic is the
// single-lattice kernel's, so a lattice gives the same populations alone
// and in a batch.  Lattices live in a caller-owned device arena managed by a
// first-fit allocator; chunks of steps are replayed from captured HIP graphs
// whose kernel arguments (descriptor table, work list, per-precision item
// ranges) stay valid while lattices join and leave.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "lbm.h"
#include "lbm_device.hpp"
#include "lbm_host.hpp"

using namespace lbm;
using namespace lbm_host;

namespace {

thread_local std::string g_batch_create_error;

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
  public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
        used_ = 0;
    }
    // returns offset or SIZE_MAX
    size_t alloc(size_t bytes) {
        bytes = al(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, rem = it->second - bytes;
                free_.erase(it);
                if (rem) free_[off + bytes] = rem;
                used_ += bytes;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes) {
        bytes = al(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t largest() const {
        size_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

struct BSlot {
    bool active = false;
    Lattice L;
    size_t off = 0, bytes = 0;
    long long steps = 0;
    bool wave = false;  // plain fused steps through the batch's wavefront list
    long long checked_phase = -1;  // its precision's phase right after the last check launch
    int first = 0, count = 0;
    int warn = 0;  // warning bits of its force (lbm_batch_force_warnings)
    // divergence guard over its checked chunks (fed once per check by
    // lbm_batch_residuals), and the check it was last fed
    RiseGuard guard;
    long long guard_fed = -1;
    bool diverged = false;
    BSlot() { guard.clear(); }
};

// Work-list entry per slot, uploaded to build the items on the device.
struct SlotRow {
    int slot, first, tiles_x, count;
};

__global__ __launch_bounds__(kBlock) void k_build_items_all(Item* items, const SlotRow* rows,
                                                            int nrows) {
    if ((int)blockIdx.y >= nrows) return;
    const SlotRow r = rows[blockIdx.y];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < r.count; i += gridDim.x * kBlock) {
        Item it;
        it.slot = r.slot;
        it.tx = i % r.tiles_x;
        it.ty = i / r.tiles_x;
        it.pad_ = 0;
        items[r.first + i] = it;
    }
}

__global__ __launch_bounds__(kBlock) void k_set_counts(int* first, int* count, const SlotRow* rows,
                                                       int nrows, int nslots) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= nslots) return;
    int f = 0, c = 0;
    for (int i = 0; i < nrows; ++i)
        if (rows[i].slot == s) {
            f = rows[i].first;
            c = rows[i].count;
        }
    first[s] = f;
    count[s] = c;
}

}  // namespace

struct lbm_batch {
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    int cus = 256;
    char* base = nullptr;
    size_t bytes = 0;
    int max_slots = 0;
    // bookkeeping regions (device)
    SlotDesc* d_desc = nullptr;
    int* d_first = nullptr;
    int* d_count = nullptr;
    int* d_range = nullptr;  // 3 x {begin, end}: one range per precision
    int* d_range_tile = nullptr;  // 3 x {begin, end}: its lattices stepped by the tile kernel
    int* d_wrange = nullptr;      // 3 x {begin, end}: its wavefront items in d_witems
    WaveItem* d_witems = nullptr;
    double* d_result = nullptr;
    double* d_stats = nullptr;  // 4 doubles per slot: sum gx, sum gy, sum |g|^2, max |g|
    Item* d_items = nullptr;
    double* d_partial = nullptr;
    SlotRow* d_rows = nullptr;
    double* d_red = nullptr;  // kErrBlocks x 8 + 16 doubles of reduction scratch
    long long cap_items = 0;
    // host
    SlotRow* h_rows = nullptr;  // pinned staging (max_slots rows + 3 ranges)
    double* h_result = nullptr;  // pinned, max(8 x max_slots, 8)
    SlotDesc* h_desc = nullptr;  // pinned staging of the descriptors (max_slots)
    size_t heap_off = 0;
    Arena arena;
    std::vector<BSlot> slots;
    int range_host[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    int range_tile_host[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    int wrange_host[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    std::vector<WaveItem> h_witems;
    // launches per precision since the descriptors were written: lattices of one
    // storage type share a launch parity (buffer selector cur ^ (phase & 1));
    // each type runs its own steps per launch, so each keeps its own count
    long long phase[3] = {0, 0, 0};
    int bx_log2 = 6, vy = 2;
    int blocks_per_cu = 0;  // 0: one workgroup per tile; k: persistent k per CU
    // plain steps per launch per precision (2..8: fused multi-step kernel); until
    // set by the caller, the default for the precision's current total sites
    int tb[3] = {4, 4, 4};
    bool tb_auto[3] = {true, true, true};
    // lattices of each storage type with at least this many sites take the
    // wavefront list (-1: the default rule, see on_wave_list)
    long long wave_min[3] = {-1, -1, -1};
    bool wave_all[3] = {false, false, false};  // default rule, total above batch_wave_total
    // fused tile height per precision, from the precision's current total sites
    // (short tiles once few sites remain, e.g. the tail of a set of solves)
    int th[3] = {8, 16, 12};
    // Adds and removals only mark the work list stale; it is rebuilt once before
    // the next launch (one host synchronisation for any number of changes).
    bool dirty = false;
    std::vector<char> stats_pending;  // per slot: force statistics not yet read back
    long long items_bound = 0;        // upper bound of the work list of the active slots
    int guard_checks = 8;             // divergence guard of every slot (0: rise rule off)
    std::string err;
    std::map<std::vector<long long>, hipGraphExec_t> graphs;

    int fail(int code, const std::string& m) {
        err = m;
        return code;
    }
    int hip_fail(hipError_t e, const char* where) {
        err = std::string(where) + ": " + hipGetErrorString(e);
        return LBM_E_HIP;
    }
    void drop_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
    int sel(const BSlot& s) const { return s.L.cur ^ (int)(phase[s.L.prec] & 1); }
    int flips() const {
        return (int)(phase[0] & 1) | (int)(phase[1] & 1) << 1 | (int)(phase[2] & 1) << 2;
    }

    unsigned bucket(int n) const {
        if (n <= 0) return 0;
        // power-of-two buckets keep captured graphs valid while the list changes
        unsigned g = 8;
        while (g < (unsigned)n) g <<= 1;
        if (blocks_per_cu > 0) g = std::min(g, (unsigned)(cus * blocks_per_cu + 7) / 8 * 8);
        return g;
    }
    // every lattice of a precision (single steps, residual checks)
    unsigned grid_for(int prec) const { return bucket(range_host[prec][1] - range_host[prec][0]); }
    // the lattices the tile kernel steps in plain fused launches
    unsigned grid_tile_for(int prec) const {
        return bucket(range_tile_host[prec][1] - range_tile_host[prec][0]);
    }
    // workgroups of four waves for the wavefront list (power-of-two buckets)
    unsigned grid_wave_for(int prec) const {
        const int n = wrange_host[prec][1] - wrange_host[prec][0];
        if (n <= 0) return 0;
        unsigned g = 8;
        while (g * (kBlock / kWave) < (unsigned)n) g <<= 1;
        return g;
    }


    int ensure() { return dirty ? rebuild() : LBM_OK; }

    // Default rule: every lattice of the type once its lattices hold at least
    // batch_wave_total sites together, else those a single solver steps
    // through the wavefront.
    bool on_wave_list(int p, long long sites) const {
        return wave_min[p] < 0 ? wave_all[p] || wave_by_default(p, sites) : sites >= wave_min[p];
    }

    // Recompute the work list: items grouped by precision, then by slot id.
    int rebuild() {
        long long total = 0;
        int nrows = 0;
        hipError_t e = hipStreamSynchronize(stream);  // staging buffer reuse
        if (e != hipSuccess) return hip_fail(e, "rebuild");
        dirty = false;
        // force statistics of lattices added since the last rebuild (one copy)
        bool any = false;
        for (int i = 0; i < max_slots; ++i) any = any || (slots[i].active && stats_pending[i]);
        if (any) {
            e = hipMemcpy(h_result, d_stats, 8 * max_slots * sizeof(double), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "rebuild: force statistics");
            for (int i = 0; i < max_slots; ++i) {
                if (!slots[i].active || !stats_pending[i]) continue;
                Lattice& L = slots[i].L;
                // the force as lbm_set_body_force records it (mean removal,
                // neutral-mode targets, half scale) and its warnings
                record_force(L, h_result + 8 * i, 0);
                slots[i].warn = force_warnings(h_result + 8 * i, L.N);
                if (L.prec0 == LBM_FP16) L.e_scale = initial_half_exponent(L, L.gmax);
                stats_pending[i] = 0;
            }
        }
        for (int p = 0; p < 3; ++p) {
            long long sites = 0;
            bool large = false;  // a lattice on the wavefront list: eight steps per launch
            for (int i = 0; i < max_slots; ++i)
                if (slots[i].active && slots[i].L.prec == p) sites += slots[i].L.N;
            wave_all[p] = sites >= batch_wave_total(p);
            for (int i = 0; i < max_slots; ++i)
                if (slots[i].active && slots[i].L.prec == p)
                    large = large || on_wave_list(p, slots[i].L.N);
            // the wavefront runs eight steps best (FP64 4 x 1500^2 in a batch:
            // 116 GLUPS at the tile's five), and its lattices carry the work
            if (tb_auto[p]) tb[p] = large ? 8 : default_time_blocking(p, sites, true);
            th[p] = fused_th(p, tb[p], sites);
        }
        // Per precision: the tile work list of every lattice (single steps and
        // residual checks), the lattices the tile kernel steps in plain fused
        // launches first; the lattices of the wavefront list (on_wave_list)
        // take those launches through it instead, one item per wave.
        h_witems.clear();
        for (int p = 0; p < 3; ++p) {
            range_host[p][0] = (int)total;
            wrange_host[p][0] = (int)h_witems.size();
            long long wave_cols_rows = 0;  // strips x rows of its wavefront lattices
            const int w = tb[p] >= 2 ? wave_width_of(tb[p], 1) : 0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = 0; i < max_slots; ++i) {
                    BSlot& s = slots[i];
                    if (!s.active || s.L.prec != p) continue;
                    s.wave = w > 0 && on_wave_list(p, s.L.N);
                    if (s.wave != (pass == 1)) continue;
                    s.L.bx_log2 = bx_log2;
                    s.L.vy = vy;
                    s.L.tb = tb[p];
                    s.L.th = th[p];
                    s.first = (int)total;
                    s.count = s.L.nitems();
                    total += s.count;
                    h_rows[nrows++] = SlotRow{i, s.first, s.L.tiles_x(), s.count};
                    if (s.wave) wave_cols_rows += (long long)((s.L.nx + w - 1) / w) * s.L.ny;
                }
                if (pass == 0) {
                    range_tile_host[p][0] = range_host[p][0];
                    range_tile_host[p][1] = (int)total;
                }
            }
            range_host[p][1] = (int)total;
            // segments as long as leaves one wave per SIMD over the list, 16..128 rows
            const int hs = (int)std::min<long long>(
                128, std::max<long long>(16, (wave_cols_rows + 4LL * cus - 1) / (4LL * cus)));
            for (int i = 0; i < max_slots && w > 0; ++i) {
                const BSlot& s = slots[i];
                if (!s.active || s.L.prec != p || !s.wave) continue;
                const int strips = (s.L.nx + w - 1) / w;
                for (int ya = 0; ya < s.L.ny; ya += hs)
                    for (int sx = 0; sx < strips; ++sx)
                        h_witems.push_back(WaveItem{i, sx, ya, std::min(ya + hs, s.L.ny)});
            }
            wrange_host[p][1] = (int)h_witems.size();
        }
        if (total > cap_items || (long long)h_witems.size() > cap_items)
            return fail(LBM_E_WORKSPACE, "work list exceeds batch capacity");
        int* rng = reinterpret_cast<int*>(h_rows + max_slots);
        for (int p = 0; p < 3; ++p) {
            rng[2 * p] = range_host[p][0];
            rng[2 * p + 1] = range_host[p][1];
            rng[6 + 2 * p] = range_tile_host[p][0];
            rng[6 + 2 * p + 1] = range_tile_host[p][1];
            rng[12 + 2 * p] = wrange_host[p][0];
            rng[12 + 2 * p + 1] = wrange_host[p][1];
        }
        e = hipMemcpyAsync(d_rows, h_rows, (max_slots + 2) * sizeof(SlotRow),
                           hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return hip_fail(e, "rebuild upload");
        if (nrows > 0)
            hipLaunchKernelGGL(k_build_items_all, dim3(64, nrows), dim3(kBlock), 0, stream, d_items,
                               d_rows, nrows);
        hipLaunchKernelGGL(k_set_counts, dim3(blocks_for(max_slots)), dim3(kBlock), 0, stream,
                           d_first, d_count, d_rows, nrows, max_slots);
        e = hipMemcpyAsync(d_range, rng, 6 * sizeof(int), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_range_tile, rng + 6, 6 * sizeof(int), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_wrange, rng + 12, 6 * sizeof(int), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && !h_witems.empty())
            e = hipMemcpy(d_witems, h_witems.data(), h_witems.size() * sizeof(WaveItem),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "rebuild");
        // descriptors of the active slots: one copy from pinned staging (the
        // stream was synchronised above, so the staging is free)
        for (int i = 0; i < max_slots; ++i)
            if (slots[i].active) h_desc[i] = slots[i].L.desc();
        e = hipMemcpyAsync(d_desc, h_desc, max_slots * sizeof(SlotDesc), hipMemcpyHostToDevice,
                           stream);
        if (e != hipSuccess) return hip_fail(e, "desc");
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "rebuild");
        return LBM_OK;
    }

    StepLaunch args(int prec, int flip, bool tile_only = false) const {
        StepLaunch a;
        a.slots = d_desc;
        a.items = d_items;
        a.range = (tile_only ? d_range_tile : d_range) + 2 * prec;
        a.partial = d_partial;
        a.flip = flip;
        a.rows = eff_vy(prec);
        return a;
    }

    // rows per thread of the tiles of one precision's lattices
    int eff_vy(int prec) const { return tb[prec] >= 2 ? th[prec] / 4 : vy; }

    // Whether a remainder of r < tb[p] plain steps runs as one fused launch.
    bool fused_rest(int p, long long r) const {
        return tb[p] >= 2 && r >= 2 && stepN_supported(p, (int)r, th[p]);
    }

    // Launches of np plain steps of precision p: groups of tb[p] through the
    // fused kernel, the remainder as one shorter fused launch or single steps.
    long long plain_launches(int p, long long np) const {
        if (tb[p] < 2) return np;
        const long long r = np % tb[p];
        return np / tb[p] + (fused_rest(p, r) ? 1 : r);
    }

    // A checked sequence of n steps of precision p: `plain` steps through the
    // ordinary launches, then one fused launch of `span` steps whose last two
    // steps form the residual check (span 0: a write-u step and a check step,
    // one step per launch).  The span makes the plain part whole launches: the
    // remainder of n (at least 2), else a full launch.
    void check_plan(int p, long long n, long long& plain, int& span) const {
        plain = n - 2;
        span = 0;
        if (tb[p] < 2) return;
        const long long r = n % tb[p];
        const long long k = (r >= 2) ? r : tb[p];
        if (k > n || !stepN_supported(p, (int)k, th[p])) return;
        plain = n - k;
        span = (int)k;
    }

    // buffer flips of precision p in one batch_step
    long long launches(int p, long long nsteps, bool check) const {
        if (!check) return plain_launches(p, nsteps);
        long long plain;
        int span;
        check_plan(p, nsteps, plain, span);
        return plain_launches(p, plain) + (span ? 1 : 2);
    }

    // The launches of one batch_step, precision by precision (their lattices
    // and work-list ranges are disjoint), then one finalize over all slots.
    hipError_t enqueue(long long nsteps, bool check, hipStream_t st) {
        hipError_t e = hipSuccess;
        for (int p = 0; p < 3 && e == hipSuccess; ++p) {
            const unsigned g = grid_for(p);
            if (!g) continue;
            long long np = nsteps;
            int span = 0;
            if (check) check_plan(p, nsteps, np, span);
            long long ph = phase[p], i = 0;
            // plain fused launches: the tile kernel over its lattices and the
            // wavefront over the list of the others, the same steps
            const unsigned gt = grid_tile_for(p), gw = grid_wave_for(p);
            const int nw = wrange_host[p][1] - wrange_host[p][0];
            auto fused = [&](int ns, int flip) {
                hipError_t r = hipSuccess;
                if (gt) r = launch_stepN(p, ns, th[p], gt, st, args(p, flip, true));
                if (r == hipSuccess && gw)
                    r = launch_wave_list(p, ns, d_desc, d_witems, d_wrange + 2 * p, nw, flip, gw, st);
                return r;
            };
            if (tb[p] >= 2) {
                for (; i + tb[p] <= np && e == hipSuccess; i += tb[p], ++ph)
                    e = fused(tb[p], (int)(ph & 1));
                if (e == hipSuccess && fused_rest(p, np - i)) {
                    e = fused((int)(np - i), (int)(ph & 1));
                    ++ph;
                    i = np;
                }
            }
            for (; i < np && e == hipSuccess; ++i, ++ph)
                e = launch_step(p, kPlain, false, eff_vy(p), kLayPull, g, st, args(p, (int)(ph & 1)));
            if (check && e == hipSuccess && span) {
                e = launch_stepN(p, span, th[p], g, st, args(p, (int)(ph & 1)), true);
            } else if (check && e == hipSuccess) {
                e = launch_step(p, kWriteU, false, eff_vy(p), kLayPull, g, st, args(p, (int)(ph & 1)));
                ++ph;
                if (e == hipSuccess)
                    e = launch_step(p, kCheck, false, eff_vy(p), kLayPull, g, st,
                                    args(p, (int)(ph & 1)));
            }
        }
        if (check && e == hipSuccess) {
            FinalizeLaunch F;
            F.first = d_first;
            F.count = d_count;
            F.partial = d_partial;
            F.result = d_result;
            F.nslots = max_slots;
            hipLaunchKernelGGL(k_finalize, dim3(max_slots), dim3(kBlock), 0, st, F);
            e = hipGetLastError();
        }
        return e;
    }
};

extern "C" {

size_t lbm_batch_slot_bytes(int nx, int ny, int precision, int with_polish) {
    if (nx < 1 || ny < 1 || !valid_prec(precision)) return 0;
    return lattice_bytes((long long)nx * ny, precision, with_polish != 0);
}

int lbm_batch_create(int max_slots, void* arena, size_t arena_bytes, void* stream,
                     lbm_batch** out) {
    if (!out || max_slots < 1) {
        g_batch_create_error = "batch_create: invalid arguments";
        return LBM_E_ARG;
    }
    *out = nullptr;
    if (!arena || (reinterpret_cast<uintptr_t>(arena) % kAlign)) {
        g_batch_create_error = "batch_create: arena NULL or not 256-byte aligned";
        return LBM_E_WORKSPACE;
    }
    lbm_batch* b = new lbm_batch();
    b->stream = reinterpret_cast<hipStream_t>(stream);
    b->max_slots = max_slots;
    b->base = reinterpret_cast<char*>(arena);
    b->bytes = arena_bytes;
    // work-list capacity: one item per 256 sites of the smallest per-site
    // footprint (half storage, 56 B/site) plus ragged tiles of every slot
    b->cap_items = (long long)(arena_bytes / (56 * 256)) + (long long)max_slots * 1024 + 1024;
    size_t off = 0;
    auto take = [&](size_t n) {
        size_t o = off;
        off += al(n);
        return b->base + o;
    };
    b->d_desc = reinterpret_cast<SlotDesc*>(take(max_slots * sizeof(SlotDesc)));
    b->d_first = reinterpret_cast<int*>(take(max_slots * sizeof(int)));
    b->d_count = reinterpret_cast<int*>(take(max_slots * sizeof(int)));
    b->d_range = reinterpret_cast<int*>(take(6 * sizeof(int)));
    b->d_range_tile = reinterpret_cast<int*>(take(6 * sizeof(int)));
    b->d_wrange = reinterpret_cast<int*>(take(6 * sizeof(int)));
    b->d_result = reinterpret_cast<double*>(take(4 * max_slots * sizeof(double)));
    b->d_stats = reinterpret_cast<double*>(take(8 * max_slots * sizeof(double)));
    b->d_rows = reinterpret_cast<SlotRow*>(take((max_slots + 5) * sizeof(SlotRow)));
    b->d_red = reinterpret_cast<double*>(take((kErrBlocks * 8 + 16) * sizeof(double)));
    b->d_items = reinterpret_cast<Item*>(take(b->cap_items * sizeof(Item)));
    // wavefront items: no more than tile items (a wave covers at least 48 x 16 sites)
    b->d_witems = reinterpret_cast<WaveItem*>(take(b->cap_items * sizeof(WaveItem)));
    b->d_partial = reinterpret_cast<double*>(take(b->cap_items * 3 * sizeof(double)));
    if (off > arena_bytes) {
        g_batch_create_error = "batch_create: arena smaller than the batch bookkeeping (" +
                               std::to_string(off) + " bytes)";
        delete b;
        return LBM_E_WORKSPACE;
    }
    b->heap_off = off;
    b->arena.init(arena_bytes - off);
    b->slots.resize(max_slots);
    b->stats_pending.assign(max_slots, 0);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_rows), (max_slots + 5) * sizeof(SlotRow),
                          hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_result),
                          std::max(8 * max_slots, 8) * sizeof(double),
                          hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_desc), max_slots * sizeof(SlotDesc),
                          hipHostMallocDefault);
    if (e == hipSuccess) std::memset(b->h_desc, 0, max_slots * sizeof(SlotDesc));
    if (e == hipSuccess) e = zero_bytes(b->d_result, 4 * max_slots * sizeof(double), b->stream);
    if (e != hipSuccess) {
        g_batch_create_error = std::string("batch_create: ") + hipGetErrorString(e);
        if (b->cap) (void)hipStreamDestroy(b->cap);
        if (b->h_rows) (void)hipHostFree(b->h_rows);
        if (b->h_result) (void)hipHostFree(b->h_result);
        if (b->h_desc) (void)hipHostFree(b->h_desc);
        delete b;
        return LBM_E_HIP;
    }
    int rc = b->rebuild();
    if (rc != LBM_OK) {
        g_batch_create_error = b->err;
        lbm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
    if (!b) return LBM_E_ARG;
    (void)hipStreamSynchronize(b->stream);
    b->drop_graphs();
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->h_rows) (void)hipHostFree(b->h_rows);
    if (b->h_result) (void)hipHostFree(b->h_result);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    delete b;
    return LBM_OK;
}

int lbm_batch_add(lbm_batch* b, int nx, int ny, int precision, int with_polish, double lam,
                  double mu, const double* gx, const double* gy, int* slot) {
    if (!b) return LBM_E_ARG;
    // the fused tile kernel addresses a plane of populations or force (in the
    // arithmetic type; FP64 after a polish switch) with 32-bit byte offsets
    const long long eb = (precision == LBM_FP64 || with_polish) ? 8 : 4;
    if (nx < 1 || ny < 1 || !valid_prec(precision) || !gx || !gy || !slot ||
        plane_of((long long)nx * ny) * eb > 0xFFFFFFFFLL)
        return b->fail(LBM_E_ARG, "batch_add: invalid size (plane of 2^32 bytes or more), "
                                  "precision or NULL pointer");
    Rates r;
    if (!material_rates(lam, mu, r, b->err)) return LBM_E_MATERIAL;
    int id = -1;
    for (int i = 0; i < b->max_slots; ++i)
        if (!b->slots[i].active) {
            id = i;
            break;
        }
    if (id < 0) return b->fail(LBM_E_WORKSPACE, "batch_add: all slots in use");
    const long long N = (long long)nx * ny;
    const size_t need = lattice_bytes(N, precision, with_polish != 0);
    if (b->items_bound + max_items(nx, ny) > b->cap_items)
        return b->fail(LBM_E_WORKSPACE, "batch_add: work list full");
    const size_t off = b->arena.alloc(need);
    if (off == SIZE_MAX) return b->fail(LBM_E_WORKSPACE, "batch_add: arena has no room");
    BSlot& s = b->slots[id];
    s = BSlot();
    s.off = off;
    s.bytes = need;
    Lattice& L = s.L;
    L.nx = nx;
    L.ny = ny;
    L.N = N;
    L.plane = plane_of(N);
    L.prec0 = L.prec = precision;
    L.polish = with_polish != 0 && precision != LBM_FP64;
    L.rates = r;
    L.lam = lam;
    L.mu = mu;
    L.has_material = L.has_force = true;
    carve_lattice(b->base + b->heap_off + off, N, precision, L.polish, L.mem);
    // force statistics into this slot's entry (read back at the next rebuild),
    // then the mean-projected copy, which reads them in stream order
    double* st = b->d_stats + 8 * id;
    const ForceSrc src = raw_force(gx, gy, nx, ny);
    hipError_t e = force_stats(src, b->d_red, st, b->stream);
    if (e == hipSuccess) e = upload_force(L, src, st, b->stream);
    if (e == hipSuccess) e = zero_bytes(L.mem.buf[0], 8 * L.plane * elem_bytes(precision), b->stream);
    if (e == hipSuccess) e = zero_bytes(L.mem.u, 2 * L.plane * 8, b->stream);
    if (e != hipSuccess) {
        b->arena.release(off, need);
        s = BSlot();
        return b->hip_fail(e, "batch_add");
    }
    b->stats_pending[id] = 1;
    // the next launch reads buf[cur ^ (phase & 1)] = buf[0]
    L.cur = (int)(b->phase[precision] & 1);
    s.active = true;
    s.steps = 0;
    s.checked_phase = -1;
    b->items_bound += max_items(nx, ny);
    b->dirty = true;
    *slot = id;
    return LBM_OK;
}

int lbm_batch_force_warnings(lbm_batch* b, int slot) {
    if (!b) return LBM_E_ARG;
    if (slot < 0 || slot >= b->max_slots || !b->slots[slot].active)
        return b->fail(LBM_E_ARG, "batch_force_warnings: no such slot");
    if (b->stats_pending[slot]) {  // read its force statistics back
        int rc = b->rebuild();
        if (rc != LBM_OK) return rc;
    }
    return b->slots[slot].warn;
}

int lbm_batch_remove(lbm_batch* b, int slot) {
    if (!b) return LBM_E_ARG;
    if (slot < 0 || slot >= b->max_slots || !b->slots[slot].active)
        return b->fail(LBM_E_ARG, "batch_remove: no such slot");
    // no wait: later work on this memory (a new slot's uploads) is ordered on
    // the same stream after the launches that still read it
    BSlot& s = b->slots[slot];
    b->items_bound -= max_items(s.L.nx, s.L.ny);
    b->arena.release(s.off, s.bytes);
    s = BSlot();
    b->stats_pending[slot] = 0;
    b->dirty = true;
    return LBM_OK;
}

int lbm_batch_set_tile(lbm_batch* b, int bx_log2, int rows_per_thread, int blocks_per_cu) {
    if (!b) return LBM_E_ARG;
    if (bx_log2 < 3 || bx_log2 > 8 ||
        !(rows_per_thread == 1 || rows_per_thread == 2 || rows_per_thread == 4) ||
        blocks_per_cu < 0 || blocks_per_cu > 64)
        return b->fail(LBM_E_ARG,
                       "batch_set_tile: bx_log2 in 3..8, rows_per_thread in {1,2,4}, blocks_per_cu in 0..64");
    b->bx_log2 = bx_log2;
    b->vy = rows_per_thread;
    b->blocks_per_cu = blocks_per_cu;
    b->drop_graphs();
    return b->rebuild();
}

int lbm_batch_set_time_blocking(lbm_batch* b, int steps_per_launch) {
    if (!b) return LBM_E_ARG;
    if (steps_per_launch < 1 || steps_per_launch > 8)
        return b->fail(LBM_E_ARG, "batch_set_time_blocking: steps_per_launch must be in 1..8");
    for (int p = 0; p < 3; ++p) {
        b->tb[p] = steps_per_launch;
        b->tb_auto[p] = false;
    }
    b->drop_graphs();
    return b->rebuild();
}

int lbm_batch_set_time_blocking_for(lbm_batch* b, int precision, int steps_per_launch) {
    if (!b) return LBM_E_ARG;
    if (!valid_prec(precision) || steps_per_launch < 1 || steps_per_launch > 8)
        return b->fail(LBM_E_ARG,
                       "batch_set_time_blocking_for: precision LBM_FP64/FP32/FP16, steps_per_launch in 1..8");
    b->tb[precision] = steps_per_launch;
    b->tb_auto[precision] = false;
    b->drop_graphs();
    return b->rebuild();
}

int lbm_batch_set_wavefront_sites(lbm_batch* b, int precision, long long min_sites) {
    if (!b) return LBM_E_ARG;
    if (!valid_prec(precision) || min_sites < -1)
        return b->fail(LBM_E_ARG,
                       "batch_set_wavefront_sites: precision LBM_FP64/FP32/FP16, min_sites >= -1");
    b->wave_min[precision] = min_sites;
    b->drop_graphs();
    return b->rebuild();
}

int lbm_batch_step(lbm_batch* b, long long nsteps, int check) {
    if (!b) return LBM_E_ARG;
    if (nsteps < 1 || (check && nsteps < 2))
        return b->fail(LBM_E_ARG, "batch_step: nsteps >= 1 (>= 2 with check)");
    int rc0 = b->ensure();
    if (rc0 != LBM_OK) return rc0;
    if (b->range_host[2][1] == 0) return LBM_OK;  // nothing active
    hipError_t e;
    long long nl = 0;
    for (int p = 0; p < 3; ++p)
        if (b->grid_for(p)) nl += b->launches(p, nsteps, check != 0);
    if (nl >= 4) {
        std::vector<long long> key{nsteps, (check ? 1 : 0) | b->flips() << 1,
                                   b->tb[0] | b->tb[1] << 4 | b->tb[2] << 8,
                                   b->th[0] | b->th[1] << 6 | b->th[2] << 12};
        for (int p = 0; p < 3; ++p) {
            key.push_back(b->grid_for(p));
            key.push_back(b->grid_tile_for(p));
            key.push_back(b->grid_wave_for(p));
        }
        auto it = b->graphs.find(key);
        if (it == b->graphs.end()) {
            if (b->graphs.size() > 16) b->drop_graphs();
            hipGraph_t gr;
            if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return b->hip_fail(e, "capture");
            hipError_t le = b->enqueue(nsteps, check != 0, b->cap);
            if ((e = hipStreamEndCapture(b->cap, &gr)) != hipSuccess) return b->hip_fail(e, "capture");
            if (le != hipSuccess) {
                (void)hipGraphDestroy(gr);
                return b->hip_fail(le, "capture launch");
            }
            hipGraphExec_t ex;
            e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (e != hipSuccess) return b->hip_fail(e, "instantiate");
            it = b->graphs.emplace(key, ex).first;
        }
        if ((e = hipGraphLaunch(it->second, b->stream)) != hipSuccess)
            return b->hip_fail(e, "graph launch");
    } else {
        if ((e = b->enqueue(nsteps, check != 0, b->stream)) != hipSuccess)
            return b->hip_fail(e, "batch_step");
    }
    for (int p = 0; p < 3; ++p) b->phase[p] += b->launches(p, nsteps, check != 0);
    for (auto& s : b->slots)
        if (s.active) {
            s.steps += nsteps;
            if (check) s.checked_phase = b->phase[s.L.prec];
        }
    return LBM_OK;
}

int lbm_batch_residuals(lbm_batch* b, double* r_host, long long* steps_host) {
    if (!b) return LBM_E_ARG;
    if (!r_host || !steps_host) return b->fail(LBM_E_ARG, "batch_residuals: NULL output");
    hipError_t e = hipMemcpyAsync(b->h_result, b->d_result, 4 * b->max_slots * sizeof(double),
                                  hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return b->hip_fail(e, "batch_residuals");
    for (int i = 0; i < b->max_slots; ++i) {
        const BSlot& s = b->slots[i];
        steps_host[i] = s.active ? s.steps : -1;
        if (!s.active || s.checked_phase != b->phase[s.L.prec]) {
            r_host[i] = NAN;
            continue;
        }
        const double d2 = b->h_result[4 * i], u2 = b->h_result[4 * i + 1];
        double r = (u2 == 0.0) ? (d2 == 0.0 ? 0.0 : INFINITY) : std::sqrt(d2 / u2);
        if (d2 != d2 || u2 != u2 || !std::isfinite(u2)) r = NAN;
        r_host[i] = r;
        // each check feeds the slot's divergence guard once
        BSlot& sl = b->slots[i];
        if (sl.guard_fed != s.checked_phase) {
            sl.guard_fed = s.checked_phase;
            const bool bad = !std::isfinite(r) && !(u2 == 0.0 && d2 != 0.0);
            if (bad || sl.guard.update(std::sqrt(d2), b->guard_checks)) sl.diverged = true;
        }
    }
    return LBM_OK;
}

int lbm_batch_diverged(lbm_batch* b, int* flags_host) {
    if (!b) return LBM_E_ARG;
    if (!flags_host) return b->fail(LBM_E_ARG, "batch_diverged: NULL output");
    for (int i = 0; i < b->max_slots; ++i)
        flags_host[i] = (b->slots[i].active && b->slots[i].diverged) ? 1 : 0;
    return LBM_OK;
}

int lbm_batch_set_divergence_guard(lbm_batch* b, int checks) {
    if (!b) return LBM_E_ARG;
    if (checks < 0) return b->fail(LBM_E_ARG, "batch_set_divergence_guard: checks must be >= 0");
    b->guard_checks = checks;
    return LBM_OK;
}

int lbm_batch_promote(lbm_batch* b, int slot) {
    if (!b) return LBM_E_ARG;
    if (slot < 0 || slot >= b->max_slots || !b->slots[slot].active)
        return b->fail(LBM_E_ARG, "batch_promote: no such slot");
    if (b->stats_pending[slot]) {  // its force statistics (half scale, mean target)
        int rc0 = b->rebuild();
        if (rc0 != LBM_OK) return rc0;
    }
    BSlot& s = b->slots[slot];
    Lattice& L = s.L;
    if (L.prec == LBM_FP64) return LBM_OK;
    if (!L.polish) return b->fail(LBM_E_STATE, "batch_promote: lattice added without polish");
    const int sl = b->sel(s);
    const long long n = 8 * L.plane;
    const double factor = (L.prec == LBM_FP16) ? std::ldexp(1.0, L.e_scale) : 1.0;
    if (L.prec == LBM_FP32)
        hipLaunchKernelGGL((k_recast<float, double>), dim3(blocks_for(n)), dim3(kBlock), 0,
                           b->stream, reinterpret_cast<const float*>(L.mem.buf[sl]),
                           reinterpret_cast<double*>(L.mem.pbuf[0]), n, factor);
    else
        hipLaunchKernelGGL((k_recast<__half, double>), dim3(blocks_for(n)), dim3(kBlock), 0,
                           b->stream, reinterpret_cast<const __half*>(L.mem.buf[sl]),
                           reinterpret_cast<double*>(L.mem.pbuf[0]), n, factor);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return b->hip_fail(e, "batch_promote");
    // the last check stays current across the switch of launch parity
    const bool checked = s.checked_phase == b->phase[L.prec];
    L.prec = LBM_FP64;
    L.cur = (int)(b->phase[LBM_FP64] & 1);
    s.checked_phase = checked ? b->phase[LBM_FP64] : -1;
    b->dirty = true;  // the slot moves to the FP64 part of the work list at the next launch
    s.guard.clear();  // the FP64 phase starts a new residual history
    s.guard_fed = s.checked_phase;
    // reset the undamped modes (staggered moments, mean) excited by the narrow phase
    double target[2], stag[2];
    L.mean_target(s.steps, target);
    L.stag_target_stored(s.steps, stag);
    e = neutral_reset(LBM_FP64, L.desc(), b->sel(s), target, stag, b->d_red, b->stream);
    if (e != hipSuccess) return b->hip_fail(e, "batch_promote: neutral modes");
    return LBM_OK;
}

int lbm_batch_get_displacement(lbm_batch* b, int slot, double* ux, double* uy) {
    if (!b) return LBM_E_ARG;
    if (slot < 0 || slot >= b->max_slots || !b->slots[slot].active || !ux || !uy)
        return b->fail(LBM_E_ARG, "batch_get_displacement: no such slot or NULL output");
    int rc0 = b->ensure();  // the half scale of a new FP16 slot
    if (rc0 != LBM_OK) return rc0;
    const BSlot& s = b->slots[slot];
    hipError_t e = extract_u(s.L.prec, s.L.desc(), b->sel(s), kLayPull, ux, uy, b->stream);
    if (e != hipSuccess) return b->hip_fail(e, "batch_get_displacement");
    return LBM_OK;
}

int lbm_batch_info(const lbm_batch* b, int* active, size_t* used_bytes, size_t* largest_free) {
    if (!b) return LBM_E_ARG;
    int a = 0;
    for (auto& s : b->slots) a += s.active ? 1 : 0;
    if (active) *active = a;
    if (used_bytes) *used_bytes = b->arena.used();
    if (largest_free) *largest_free = b->arena.largest();
    return LBM_OK;
}

const char* lbm_batch_last_error(const lbm_batch* b) {
    if (!b) return g_batch_create_error.c_str();
    return b->err.c_str();
}

}  // extern "C"

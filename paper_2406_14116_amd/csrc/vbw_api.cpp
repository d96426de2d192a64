// vbw_api.cpp -- plan object, validation, integer planner, device tables and
// the C ABI declared in include/vbw.h.
//
// Paper: Moryakova & Johansson, arXiv 2406.14116.  The plan implements the
// problem statement of Sec. III-A/B: a fixed transition width, a variable
// band edge discretised to bins (eq. (7)), and one stored set of L_V
// transition values V(r) so that a bandwidth change is an integer update with
// no arithmetic (Sec. III-D).
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "vbw.h"
#include "vbw_internal.h"

using vbw::ChannelDev;
using vbw::SchedDev;
using vbw::WorkItem;

namespace {

constexpr int kMaxSchedPerChannel = 4096;
constexpr uint32_t kKnownFlags = VBW_NO_PRUNE | VBW_GRAPH | VBW_F32_OUT | VBW_HOST_ONLY | VBW_AUTOTUNE | VBW_STREAM;

vbw_status from_hip(hipError_t e) {
    if (e == hipSuccess) return VBW_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return VBW_ENOMEM;
    return VBW_EDEVICE;
}

// ROCTx range around a C entry point: plan set-up, filter calls and the
// autotuner show up by name in a marker trace (rocprofv3 --marker-trace).
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

// Test hook (vbw_test_fail_device_alloc): the k-th device allocation made by
// each vbw_plan call on this thread fails (1-based; 0: none), to exercise the
// ENOMEM path without leaks.
thread_local int g_alloc_count = 0;
thread_local int g_fail_alloc_at = 0;

hipError_t dev_alloc(void **p, size_t bytes) {
    *p = nullptr;
    ++g_alloc_count;
    if (g_fail_alloc_at > 0 && g_fail_alloc_at == g_alloc_count) return hipErrorOutOfMemory;
    if (bytes == 0) bytes = 16;
    return hipMalloc(p, bytes);
}

// Workgroups of one persistent launch: one per tile at most, `resident` (or
// a multiple of it) otherwise, and at most `cap` when cap > 0.
int wg_count(size_t tiles, size_t resident, int cap) {
    size_t n = std::min(tiles, resident);
    if (cap > 0) n = std::min(n, size_t(cap));
    return int(std::max<size_t>(1, n));
}

bool is_pow2(int32_t n) { return n > 0 && (n & (n - 1)) == 0; }

int ilog2(int32_t n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

int64_t n_blocks_of(int64_t len, int32_t hop) { return len <= 0 ? 0 : (len + hop - 1) / hop; }

// Admissible edge for channel shape (n, lv): k1 >= 1 and k2 = k1 + lv - 1 <=
// N/2 - 1 (the Nyquist bin is stopband), or the all-pass lv = 0, k1 = N/2+1.
bool k1_in_range(int32_t n, int32_t lv, int32_t k1) {
    if (lv == 0 && k1 == n / 2 + 1) return true;
    return k1 >= 1 && int64_t(k1) + lv - 1 <= n / 2 - 1;
}

// cos(2 pi r / n), sin(2 pi r / n) in float64 with exact octant reduction
// (r / n is a dyadic rational, so every reflection below is exact).
void cos_sin_2pi(int64_t r, int64_t n, double *c, double *s) {
    r %= n;
    if (r < 0) r += n;
    // y = r / n in [0, 1)
    double sign_s = 1.0, sign_c = 1.0;
    int64_t num = r, den = n;
    if (2 * num > den) {            // y in (1/2, 1): sin(2 pi y) = -sin(2 pi (1 - y))
        num = den - num;
        sign_s = -1.0;
    }
    if (4 * num > den) {            // y in (1/4, 1/2]: cos = -cos(2 pi (1/2 - y)), sin same
        num = den - 2 * num;        // (1/2 - y) = (den - 2 num) / (2 den)
        den = 2 * den;
        sign_c = -1.0;
    }
    bool swap = false;
    if (8 * num > den) {            // y in (1/8, 1/4]: cos(2 pi y) = sin(2 pi (1/4 - y))
        num = den - 4 * num;        // (1/4 - y) = (den - 4 num) / (4 den)
        den = 4 * den;
        swap = true;
    }
    const double a = 6.283185307179586476925286766559 * (double(num) / double(den));
    double cc = std::cos(a), ss = std::sin(a);
    if (swap) std::swap(cc, ss);
    *c = sign_c * cc;
    *s = sign_s * ss;
}

struct Sched {
    std::vector<std::pair<int64_t, int32_t>> e;  // (from_block, k1), sorted, e[0].first == 0
};

}  // namespace

struct vbw_plan_s {
    std::vector<vbw_channel> ch;
    std::vector<float> v32;
    std::vector<Sched> sched;
    std::vector<WorkItem> items;     // 4096-value tiles: up to 4096/N consecutive blocks
    std::vector<WorkItem> work;      // device work list of every launch variant (tiles or spans)
    int32_t dtype = VBW_C64;
    int32_t engine = VBW_ENGINE_FFT;
    uint32_t flags = 0;
    int log2n_fixed = 0;
    int64_t total_blocks = 0;
    int64_t total_samples = 0;
    int variant = 0;

    // device state
    bool host_only = true;
    int device = 0;
    WorkItem *d_items = nullptr;
    int32_t *d_wg_begin = nullptr;
    std::vector<int32_t> wg_begin;   // concatenated per-launch workgroup ranges of `work`
    // Launch variants: each is a list of persistent launches (one per N group,
    // or one launch of the kernel that dispatches on N), each with its own
    // workgroup count, item partition and pruning switch.  Variant i applies
    // shapes[i] to every group; after autotuning a last one may combine, per
    // N group, the fastest of the per-N shapes (composite).
    struct LaunchGroup {
        int log2n;       // 0: kernel that dispatches on N; -1: matrix-core kernel
        int wg_off;      // offset of this launch's range table in wg_begin
        int n_wg;
        int prune;       // stopband-pruned passes allowed
    };
    struct Shape {
        int occ_drop;    // resident workgroups per CU below the kernel's maximum
        int grid_mult;   // workgroups per launch, in units of the resident count
        int prune;
        bool dispatch;   // one launch of the kernel that dispatches on N
        int stride = 0;  // 0: a contiguous range per workgroup; k: chunks of k
                         // tiles dealt to the workgroups in turn
    };
    std::vector<Shape> shapes;
    std::vector<std::vector<LaunchGroup>> variants;
    std::vector<int> composite;       // per-group shape index of the combined variant (if any)
    std::string tune_cache;           // file of kept autotuner choices (empty: none)
    int max_wg = 0;                   // cap on workgroups per launch (0: none)
    bool tuned = false;
    float *d_v = nullptr;
    void *d_hist = nullptr;           // streaming: N - hop history samples per channel
    int64_t *d_block0 = nullptr;      // streaming: stream block index of each channel's next block
    int64_t hist_bytes = 0;
    float2 *d_tw = nullptr;
    // Per-call tables, ChannelDev[nch] | x[nch] | y[nch] | SchedDev[cap] each:
    // two of them taking turns (one in graph mode, whose graph holds the
    // address), so that the host fills the next while the device may still be
    // reading the last one from an earlier call
    unsigned char *d_dyn = nullptr;
    size_t dyn_cap_sched = 0;
    size_t dyn_stride = 0;            // bytes per table (256-byte multiple)
    int n_tables = 1;
    int cur = 0;                      // table the next launch reads
    unsigned char *h_stage = nullptr; // pinned staging, n_tables x dyn_stride
    size_t stage_bytes = 0;
    hipEvent_t upload_evt[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    hipEvent_t done_evt = nullptr;    // end of the plan's last queued call
    bool done_recorded = false;
    hipStream_t last_stream = nullptr;
    bool dyn_valid = false;
    bool sched_dirty = true;
    std::vector<const void *> last_x;
    std::vector<void *> last_y;

    // graph replay
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;

    size_t dyn_bytes(size_t sched_cap) const {
        return ch.size() * (sizeof(ChannelDev) + 2 * sizeof(void *)) + sched_cap * sizeof(SchedDev);
    }
    size_t sched_entries() const {
        size_t s = 0;
        for (auto &c : sched) s += c.e.size();
        return s;
    }
};

namespace {

vbw_status validate_desc(const vbw_plan_desc *d) {
    if (!d || !d->channels || d->n_channels < 1 || d->n_v < 0 || (d->n_v > 0 && !d->v_pool))
        return VBW_EINVAL;
    if (d->reserved != 0 || d->max_workgroups < 0 || (d->flags & ~kKnownFlags) != 0) return VBW_EINVAL;
    if (d->dtype != VBW_C64 && d->dtype != VBW_CF16 && d->dtype != VBW_CBF16 && d->dtype != VBW_R32)
        return VBW_EINVAL;
    if (d->engine != VBW_ENGINE_FFT && d->engine != VBW_ENGINE_GEMM) return VBW_EINVAL;
    for (int32_t i = 0; i < d->n_v; ++i)
        if (!std::isfinite(d->v_pool[i])) return VBW_EINVAL;
    vbw_status range = VBW_OK;
    for (int32_t c = 0; c < d->n_channels; ++c) {
        const vbw_channel &ch = d->channels[c];
        if (ch.reserved != 0) return VBW_EINVAL;
        if (!is_pow2(ch.n) || ch.n < (1 << vbw::kMinLog2N) || ch.n > (1 << vbw::kMaxLog2N)) return VBW_EINVAL;
        if (ch.hop < 1 || ch.hop > ch.n - 1 || ((ch.n - ch.hop) & 1)) return VBW_EINVAL;
        if (ch.lv < 0 || ch.lv > ch.n / 2) return VBW_EINVAL;
        if (ch.v_offset < 0 || int64_t(ch.v_offset) + ch.lv > d->n_v) return VBW_EINVAL;
        if (ch.len < 0 || n_blocks_of(ch.len, ch.hop) > int64_t(INT32_MAX) - 4096) return VBW_EINVAL;
        if (!k1_in_range(ch.n, ch.lv, ch.k1)) range = VBW_ERANGE;
    }
    if (range != VBW_OK) return range;
    if (d->flags & VBW_STREAM) {
        // a call carries whole blocks and at least one block's history
        for (int32_t c = 0; c < d->n_channels; ++c) {
            const vbw_channel &ch = d->channels[c];
            if (ch.len != 0 && (ch.len % ch.hop != 0 || ch.len < ch.n - ch.hop)) return VBW_EINVAL;
        }
        if (d->engine == VBW_ENGINE_GEMM) return VBW_EUNSUPPORTED;
    }
    if (d->engine == VBW_ENGINE_GEMM) {
        // matrix-core engine: 16-bit complex storage and N = 256 only
        if (d->dtype == VBW_C64 || d->dtype == VBW_R32) return VBW_EUNSUPPORTED;
        for (int32_t c = 0; c < d->n_channels; ++c)
            if (d->channels[c].n != 256) return VBW_EUNSUPPORTED;
    }
    return VBW_OK;
}

// Work list: each item is up to 4096/N consecutive blocks of one channel,
// i.e. one 4096-value tile per workgroup.
void build_items(vbw_plan_s *p) {
    p->items.clear();
    p->total_blocks = 0;
    p->total_samples = 0;
    int first_log2 = -1;
    bool uniform = true;
    for (size_t c = 0; c < p->ch.size(); ++c) {
        const vbw_channel &ch = p->ch[c];
        const int64_t nb = n_blocks_of(ch.len, ch.hop);
        const int lg = ilog2(ch.n);
        // real input filters blocks in pairs: tiles (and spans) start at even blocks
        const int per = vbw::kTilePoints / ch.n * (p->dtype == VBW_R32 ? 2 : 1);
        p->total_blocks += nb;
        p->total_samples += ch.len;
        for (int64_t b = 0; b < nb; b += per) {
            WorkItem it;
            it.channel = int32_t(c);
            it.first_block = int32_t(b);
            it.n_blocks = int32_t(std::min<int64_t>(per, nb - b));
            it.log2n = lg;
            p->items.push_back(it);
        }
        if (nb > 0) {
            if (first_log2 < 0) first_log2 = lg;
            else if (first_log2 != lg) uniform = false;
        }
    }
    p->log2n_fixed = (uniform && first_log2 > 0) ? first_log2 : 0;
    // group items of equal N (each group is then one contiguous range)
    std::stable_sort(p->items.begin(), p->items.end(),
                     [](const WorkItem &a, const WorkItem &b) { return a.log2n < b.log2n; });
}

// A span's input and output offsets are 32-bit byte offsets from its base.
constexpr int64_t kMaxSpanSamples = int64_t(1) << 26;

// Split tiles [b, e) into n_wg contiguous ranges of equal estimated cost and
// append the workgroups' work to p->work and their n_wg + 1 boundaries to
// wg_begin (only the n_wg starts without `close`: the next call continues
// the same table); returns the offset of those boundaries.  A tile costs about
// log2(N) FFT passes plus a fixed part for loads, multiply and stores.  With
// `spans`, consecutive tiles of one channel inside a workgroup's range merge
// into one span, so a team filters a run of consecutive blocks and can carry
// the overlap from one block to the next; otherwise the tiles are kept.
int partition_items(vbw_plan_s *p, size_t b, size_t e, int n_wg, bool spans, bool close = true) {
    const size_t n = e - b;
    std::vector<double> pre(n + 1, 0.0);
    for (size_t i = 0; i < n; ++i) pre[i + 1] = pre[i] + (p->items[b + i].log2n + 2.0);
    std::vector<size_t> cut(size_t(n_wg) + 1, n);
    size_t i = 0;
    for (int w = 0; w < n_wg; ++w) {
        const double target = pre[n] * double(w) / double(n_wg);
        while (i < n && pre[i] < target) ++i;
        cut[size_t(w)] = i;
    }
    const int off = int(p->wg_begin.size());
    for (int w = 0; w < n_wg; ++w) {
        const size_t first = p->work.size();
        p->wg_begin.push_back(int32_t(first));
        for (size_t t = b + cut[size_t(w)]; t < b + cut[size_t(w) + 1]; ++t) {
            const WorkItem &it = p->items[t];
            if (spans && p->work.size() > first) {
                WorkItem &last = p->work.back();
                const vbw_channel &ch = p->ch[size_t(it.channel)];
                if (last.channel == it.channel && last.first_block + last.n_blocks == it.first_block &&
                    int64_t(last.n_blocks + it.n_blocks) * ch.hop + ch.n <= kMaxSpanSamples) {
                    last.n_blocks += it.n_blocks;
                    continue;
                }
            }
            p->work.push_back(it);
        }
    }
    if (close) p->wg_begin.push_back(int32_t(p->work.size()));
    return off;
}

// Chunks of `chunk` consecutive tiles of [b, e), dealt to the n_wg workgroups
// in turn (chunk j to workgroup j mod n_wg): at any time the workgroups work
// through one region of memory together, as a strided copy does, instead of
// each walking its own range.  Tiles of one channel inside a chunk merge into
// one span.  Appends like partition_items; returns the offset of the
// boundaries.
int partition_strided(vbw_plan_s *p, size_t b, size_t e, int n_wg, int chunk) {
    const size_t n_chunks = (e - b + size_t(chunk) - 1) / size_t(chunk);
    const int off = int(p->wg_begin.size());
    for (int w = 0; w < n_wg; ++w) {
        p->wg_begin.push_back(int32_t(p->work.size()));
        for (size_t c = size_t(w); c < n_chunks; c += size_t(n_wg)) {
            const size_t t0 = b + c * size_t(chunk), t1 = std::min(e, t0 + size_t(chunk));
            for (size_t t = t0; t < t1; ++t) {
                const WorkItem &it = p->items[t];
                if (t > t0) {
                    WorkItem &last = p->work.back();
                    if (last.channel == it.channel && last.first_block + last.n_blocks == it.first_block) {
                        last.n_blocks += it.n_blocks;
                        continue;
                    }
                }
                p->work.push_back(it);
            }
        }
    }
    p->wg_begin.push_back(int32_t(p->work.size()));
    return off;
}

vbw::Storage storage_of(int32_t dtype) {
    return dtype == VBW_CF16    ? vbw::Storage::F16
           : dtype == VBW_CBF16 ? vbw::Storage::BF16
           : dtype == VBW_R32   ? vbw::Storage::R32
                                : vbw::Storage::C64;
}

// Candidate launch shapes (the autotuner times them; variant 0 is the default:
// per-N launches, full resident occupancy, one resident grid, pruning as the
// flags allow).  Every shape choice:
//   resident workgroups per CU: the kernel's maximum, or one fewer;
//   grid: the resident count, or twice it (shorter ranges, finer balance);
//   pruning: on (when the flags allow it) or off;
// then, for FFT-engine plans that mix N, one launch of the kernel that
// dispatches on N at either occupancy; last, the default shape with chunks of
// 2 or 8 tiles dealt to the workgroups in turn (partition_strided).
void build_variants(vbw_plan_s *p, int n_cu, bool only_default = false) {
    p->variants.clear();
    p->shapes.clear();
    p->composite.clear();
    p->wg_begin.clear();
    p->work.clear();
    const vbw::Storage st = storage_of(p->dtype);
    const bool f32 = (p->flags & VBW_F32_OUT) != 0;
    const bool gemm = p->engine == VBW_ENGINE_GEMM;
    const int prune_max = (gemm || (p->flags & VBW_NO_PRUNE)) ? 0 : 1;
    // contiguous groups of equal N
    std::vector<std::pair<size_t, size_t>> groups;
    for (size_t i = 0; i < p->items.size();) {
        size_t j = i;
        while (j < p->items.size() && p->items[j].log2n == p->items[i].log2n) ++j;
        groups.push_back({i, j});
        i = j;
    }
    if (groups.empty()) {
        p->variants.push_back({});
        p->shapes.push_back({0, 1, prune_max, false});
        return;
    }
    auto per_cu = [&](int lg, int drop) {
        return std::max(1, (gemm ? vbw::ols_gemm_wg_per_cu(st, f32) : vbw::ols_fft_wg_per_cu(lg, st, f32)) - drop);
    };
    auto make = [&](const vbw_plan_s::Shape &sh) {
        std::vector<vbw_plan_s::LaunchGroup> v;
        if (sh.dispatch) {
            // one launch; each N group gets workgroups in proportion to its
            // cost, so that every workgroup's range holds one N
            const int n_wg = wg_count(p->items.size(), size_t(n_cu) * per_cu(0, sh.occ_drop) * sh.grid_mult, p->max_wg);
            std::vector<double> cost(groups.size(), 0.0);
            double total = 0.0;
            for (size_t g = 0; g < groups.size(); ++g) {
                cost[g] = double(groups[g].second - groups[g].first) * (p->items[groups[g].first].log2n + 2.0);
                total += cost[g];
            }
            int off = -1, placed = 0;
            double acc = 0.0;
            for (size_t g = 0; g < groups.size(); ++g) {
                acc += cost[g];
                const int upto = g + 1 == groups.size() ? n_wg : int(std::lround(double(n_wg) * acc / total));
                const int tiles = int(groups[g].second - groups[g].first);
                const int k = std::max(1, std::min(tiles, upto - placed));
                const int o = partition_items(p, groups[g].first, groups[g].second, k, true, g + 1 == groups.size());
                if (off < 0) off = o;
                placed += k;
            }
            v.push_back({0, off, placed, sh.prune});
            return v;
        }
        // one launch per N (the matrix-core engine has one N), in order on
        // the stream, each filling the chip
        for (auto &g : groups) {
            const int lg = p->items[g.first].log2n;
            const int n_wg = wg_count(g.second - g.first, size_t(n_cu) * per_cu(lg, sh.occ_drop) * sh.grid_mult,
                                      p->max_wg);
            const int o = sh.stride ? partition_strided(p, g.first, g.second, n_wg, sh.stride)
                                    : partition_items(p, g.first, g.second, n_wg, true);
            v.push_back({gemm ? -1 : lg, o, n_wg, sh.prune});
        }
        return v;
    };
    auto add = [&](const vbw_plan_s::Shape &sh) {
        p->shapes.push_back(sh);
        p->variants.push_back(make(sh));
    };
    add({0, 1, prune_max, false});
    p->variant = 0;
    if (only_default) return;
    for (int prune = prune_max; prune >= 0; --prune)
        for (int grid = 1; grid <= 2; ++grid)
            for (int drop = 0; drop < 2; ++drop)
                if (drop != 0 || grid != 1 || prune != prune_max) add({drop, grid, prune, false});
    if (!gemm && groups.size() > 1)
        for (int drop = 0; drop < 2; ++drop) add({drop, 1, prune_max, true});
    for (int chunk : {2, 8}) add({0, 1, prune_max, false, chunk});
}

// The variant that takes, for N group g, the launch of per-N variant choice[g].
std::vector<vbw_plan_s::LaunchGroup> combine(const vbw_plan_s *p, const std::vector<int> &choice) {
    std::vector<vbw_plan_s::LaunchGroup> v;
    for (size_t g = 0; g < choice.size(); ++g) v.push_back(p->variants[size_t(choice[g])][g]);
    return v;
}

void free_device(vbw_plan_s *p) {
    if (p->host_only) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    if (p->done_evt) (void)hipEventSynchronize(p->done_evt);
    for (auto ev : p->upload_evt)
        if (ev) (void)hipEventSynchronize(ev);
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->d_items) (void)hipFree(p->d_items);
    if (p->d_wg_begin) (void)hipFree(p->d_wg_begin);
    if (p->d_v) (void)hipFree(p->d_v);
    if (p->d_hist) (void)hipFree(p->d_hist);
    if (p->d_block0) (void)hipFree(p->d_block0);
    if (p->d_tw) (void)hipFree(p->d_tw);
    if (p->d_dyn) (void)hipFree(p->d_dyn);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    for (auto ev : p->upload_evt)
        if (ev) (void)hipEventDestroy(ev);
    if (p->done_evt) (void)hipEventDestroy(p->done_evt);
    (void)hipSetDevice(prev);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    p->cap_stream = nullptr;
    p->d_items = nullptr;
    p->d_wg_begin = nullptr;
    p->d_v = nullptr;
    p->d_hist = nullptr;
    p->d_block0 = nullptr;
    p->d_tw = nullptr;
    p->d_dyn = nullptr;
    p->h_stage = nullptr;
    p->upload_evt[0] = p->upload_evt[1] = p->done_evt = nullptr;
}

void fill_twiddles(int32_t n, float *out) {
    for (int32_t r = 0; r < n; ++r) {
        double c, s;
        cos_sin_2pi(r, n, &c, &s);
        out[2 * r] = float(c);
        out[2 * r + 1] = float(-s);
    }
}

vbw_status alloc_dyn(vbw_plan_s *p, size_t sched_cap) {
    void *d = nullptr, *h = nullptr;
    const size_t stride = (p->dyn_bytes(sched_cap) + 255) & ~size_t(255);
    const size_t bytes = stride * size_t(p->n_tables);
    hipError_t e = dev_alloc(&d, bytes);
    if (e != hipSuccess) return from_hip(e);
    e = hipHostMalloc(&h, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return from_hip(e);
    }
    if (p->d_dyn) (void)hipFree(p->d_dyn);        // hipFree waits for queued work
    if (p->h_stage) {
        for (int i = 0; i < 2; ++i)
            if (p->pending[i]) (void)hipEventSynchronize(p->upload_evt[i]);
        (void)hipHostFree(p->h_stage);
    }
    p->d_dyn = static_cast<unsigned char *>(d);
    p->h_stage = static_cast<unsigned char *>(h);
    p->stage_bytes = bytes;
    p->dyn_stride = stride;
    p->dyn_cap_sched = sched_cap;
    p->pending[0] = p->pending[1] = false;
    p->cur = 0;
    p->dyn_valid = false;
    // the captured graph holds the old table addresses
    if (p->graph_exec) {
        (void)hipGraphExecDestroy(p->graph_exec);
        p->graph_exec = nullptr;
    }
    if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    return VBW_OK;
}

std::string tune_cache_lookup(const vbw_plan_s *p);
void tune_cache_apply(vbw_plan_s *p, const std::string &choice);

vbw_status setup_device(vbw_plan_s *p) {
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) return from_hip(e);
    p->host_only = false;
    void *d = nullptr;
    if ((e = dev_alloc(&d, std::max<size_t>(1, p->v32.size()) * sizeof(float))) != hipSuccess) return from_hip(e);
    p->d_v = static_cast<float *>(d);
    if ((e = dev_alloc(&d, vbw::kTwiddleN * sizeof(float2))) != hipSuccess) return from_hip(e);
    p->d_tw = static_cast<float2 *>(d);
    if (p->flags & VBW_STREAM) {
        const int64_t eb = p->dtype == VBW_C64 ? 8 : 4;
        p->hist_bytes = 0;
        for (const auto &ch : p->ch) p->hist_bytes += int64_t(ch.n - ch.hop) * eb;
        if ((e = dev_alloc(&d, size_t(std::max<int64_t>(16, p->hist_bytes)))) != hipSuccess) return from_hip(e);
        p->d_hist = d;
        if ((e = dev_alloc(&d, p->ch.size() * sizeof(int64_t))) != hipSuccess) return from_hip(e);
        p->d_block0 = static_cast<int64_t *>(d);
        // the stream starts from zero history at block 0
        if ((e = vbw::launch_stream_reset(p->d_hist, p->hist_bytes, p->d_block0, int(p->ch.size()), nullptr)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(nullptr)) != hipSuccess)
            return from_hip(e);
    }
    int n_cu = 0;
    if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, p->device)) != hipSuccess)
        return from_hip(e);
    build_variants(p, n_cu);
    if ((p->flags & VBW_AUTOTUNE) && !p->tune_cache.empty()) tune_cache_apply(p, tune_cache_lookup(p));
    if ((e = dev_alloc(&d, std::max<size_t>(1, p->work.size()) * sizeof(WorkItem))) != hipSuccess) return from_hip(e);
    p->d_items = static_cast<WorkItem *>(d);
    if ((e = dev_alloc(&d, std::max<size_t>(1, p->wg_begin.size()) * sizeof(int32_t))) != hipSuccess)
        return from_hip(e);
    p->d_wg_begin = static_cast<int32_t *>(d);
    if (!p->wg_begin.empty() &&
        (e = hipMemcpy(p->d_wg_begin, p->wg_begin.data(), p->wg_begin.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return from_hip(e);
    p->n_tables = (p->flags & VBW_GRAPH) ? 1 : 2;
    for (auto &ev : p->upload_evt)
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return from_hip(e);
    if ((e = hipEventCreateWithFlags(&p->done_evt, hipEventDisableTiming)) != hipSuccess) return from_hip(e);
    vbw_status st = alloc_dyn(p, std::max<size_t>(p->sched_entries(), 2 * p->ch.size()));
    if (st != VBW_OK) return st;

    std::vector<float> tw(2 * vbw::kTwiddleN);
    fill_twiddles(vbw::kTwiddleN, tw.data());
    if (!p->work.empty() &&
        (e = hipMemcpy(p->d_items, p->work.data(), p->work.size() * sizeof(WorkItem), hipMemcpyHostToDevice)) != hipSuccess)
        return from_hip(e);
    if (!p->v32.empty() &&
        (e = hipMemcpy(p->d_v, p->v32.data(), p->v32.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
        return from_hip(e);
    if ((e = hipMemcpy(p->d_tw, tw.data(), tw.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
        return from_hip(e);
    if (p->flags & VBW_GRAPH) {
        if ((e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking)) != hipSuccess) return from_hip(e);
    }
    return VBW_OK;
}

size_t elem_bytes_in(const vbw_plan_s *p) { return p->dtype == VBW_C64 ? 8 : 4; }
size_t elem_bytes_out(const vbw_plan_s *p) {
    return (p->dtype == VBW_C64 || (p->flags & VBW_F32_OUT)) ? 8 : 4;
}

// Every output range must be disjoint from every other input and output range.
bool ranges_ok(const vbw_plan_s *p, const void *const *x, void *const *y) {
    struct R {
        uintptr_t lo, hi;
        bool out;
    };
    std::vector<R> rs;
    rs.reserve(2 * p->ch.size());
    for (size_t c = 0; c < p->ch.size(); ++c) {
        const int64_t len = p->ch[c].len;
        if (len == 0) continue;
        if (!x[c] || !y[c]) return false;
        const uintptr_t xi = reinterpret_cast<uintptr_t>(x[c]);
        const uintptr_t yo = reinterpret_cast<uintptr_t>(y[c]);
        rs.push_back({xi, xi + uintptr_t(len) * elem_bytes_in(p), false});
        rs.push_back({yo, yo + uintptr_t(len) * elem_bytes_out(p), true});
    }
    std::sort(rs.begin(), rs.end(), [](const R &a, const R &b) { return a.lo < b.lo; });
    // sweep: track the furthest end among intervals seen so far, and whether
    // the interval reaching it (or any still open) is an output
    uintptr_t open_hi_in = 0, open_hi_out = 0;
    for (const R &r : rs) {
        const bool hits_out = r.lo < open_hi_out;
        const bool hits_in = r.lo < open_hi_in;
        if (hits_out || (r.out && hits_in)) return false;
        if (r.out) open_hi_out = std::max(open_hi_out, r.hi);
        else open_hi_in = std::max(open_hi_in, r.hi);
    }
    return true;
}

// The per-call table ChannelDev[nch] | x[nch] | y[nch] | SchedDev[entries],
// written into host memory at h; returns its size in bytes.
size_t fill_call_table(const vbw_plan_s *p, const void *const *x, void *const *y, unsigned char *h) {
    const size_t nch = p->ch.size();
    ChannelDev *hc = reinterpret_cast<ChannelDev *>(h);
    const void **hx = reinterpret_cast<const void **>(h + nch * sizeof(ChannelDev));
    void **hy = reinterpret_cast<void **>(h + nch * (sizeof(ChannelDev) + sizeof(void *)));
    SchedDev *hs = reinterpret_cast<SchedDev *>(h + nch * (sizeof(ChannelDev) + 2 * sizeof(void *)));
    int32_t so = 0;
    int64_t ho = 0;
    for (size_t c = 0; c < nch; ++c) {
        const vbw_channel &ch = p->ch[c];
        hc[c].hist_off = ho;
        ho += ch.n - ch.hop;
        hc[c].len = ch.len;
        hc[c].n = ch.n;
        hc[c].hop = ch.hop;
        hc[c].lv = ch.lv;
        hc[c].v_offset = ch.v_offset;
        hc[c].sched_begin = so;
        hc[c].sched_count = int32_t(p->sched[c].e.size());
        for (auto &pr : p->sched[c].e) {
            hs[so].from_block = pr.first;
            hs[so].k1 = pr.second;
            hs[so].pad = 0;
            ++so;
        }
        hx[c] = x[c];
        hy[c] = y[c];
    }
    return p->dyn_bytes(size_t(so));
}

vbw_status upload_dyn(vbw_plan_s *p, const void *const *x, void *const *y, hipStream_t s) {
    const size_t nch = p->ch.size();
    const size_t need = p->sched_entries();
    if (need > p->dyn_cap_sched) {
        vbw_status st = alloc_dyn(p, std::max(need, 2 * p->dyn_cap_sched));
        if (st != VBW_OK) return st;
    }
    const int next = (p->cur + 1) % p->n_tables;
    if (p->pending[next]) {     // its staging buffer may still be in an earlier copy
        hipError_t e = hipEventSynchronize(p->upload_evt[next]);
        if (e != hipSuccess) return from_hip(e);
        p->pending[next] = false;
    }
    unsigned char *h = p->h_stage + size_t(next) * p->dyn_stride;
    const size_t bytes = fill_call_table(p, x, y, h);
    hipError_t e = hipMemcpyAsync(p->d_dyn + size_t(next) * p->dyn_stride, h, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return from_hip(e);
    if ((e = hipEventRecord(p->upload_evt[next], s)) != hipSuccess) return from_hip(e);
    p->pending[next] = true;
    p->cur = next;
    p->dyn_valid = true;
    p->sched_dirty = false;
    p->last_x.assign(x, x + nch);
    p->last_y.assign(y, y + nch);
    return VBW_OK;
}

// Point the per-call fields of `a` at the table that starts at device address t.
void set_table_args(vbw::LaunchArgs &a, size_t nch, const unsigned char *t) {
    a.ch = reinterpret_cast<const ChannelDev *>(t);
    a.x = reinterpret_cast<const void *const *>(t + nch * sizeof(ChannelDev));
    a.y = reinterpret_cast<void *const *>(t + nch * (sizeof(ChannelDev) + sizeof(void *)));
    a.sched = reinterpret_cast<const SchedDev *>(t + nch * (sizeof(ChannelDev) + 2 * sizeof(void *)));
}

vbw::LaunchArgs launch_args(const vbw_plan_s *p) {
    vbw::LaunchArgs a;
    a.items = p->d_items;
    set_table_args(a, p->ch.size(), p->d_dyn + size_t(p->cur) * p->dyn_stride);
    a.v = p->d_v;
    a.tw = p->d_tw;
    a.n_items = int32_t(p->work.size());
    a.wg_begin = p->d_wg_begin;
    a.hist = p->d_hist;
    a.block0 = p->d_block0;
    a.n_wg = 0;
    a.prune = (p->flags & VBW_NO_PRUNE) ? 0 : 1;
    a.pad = 0;
    return a;
}

// Events that take the start of a call's first filter kernel and the end of
// its last (vbw_filter_timed); null: none.
struct KernelTimes {
    hipEvent_t start = nullptr, stop = nullptr;
};

// The filter launches of one variant, with the tables `a` points at
// (a.wg_begin: the start of the plan's concatenated range tables).  marks:
// events recorded on the stream before each launch and after the last (the
// autotuner's); kt: the kernels' own start and end times.
hipError_t launch_variant(const vbw_plan_s *p, vbw::LaunchArgs a, hipStream_t s, int variant,
                          hipEvent_t *marks = nullptr, KernelTimes kt = {}) {
    const int32_t *wg0 = a.wg_begin;
    const bool f32 = (p->flags & VBW_F32_OUT) != 0;
    const auto &launches = p->variants[size_t(variant)];
    for (size_t i = 0; i < launches.size(); ++i) {
        const auto &g = launches[i];
        a.wg_begin = wg0 + g.wg_off;
        a.n_wg = g.n_wg;
        a.prune = g.prune;
        const hipEvent_t t0 = i == 0 ? kt.start : nullptr;
        const hipEvent_t t1 = i + 1 == launches.size() ? kt.stop : nullptr;
        hipError_t e = marks ? hipEventRecord(marks[i], s) : hipSuccess;
        if (e == hipSuccess)
            e = g.log2n < 0 ? vbw::launch_ols_gemm(a, storage_of(p->dtype), f32, s, t0, t1)
                            : vbw::launch_ols_fft(a, g.log2n, storage_of(p->dtype), f32, s, t0, t1);
        if (e != hipSuccess) return e;
    }
    if (launches.empty() && kt.start) {   // nothing to filter: an empty interval
        hipError_t e = hipEventRecord(kt.start, s);
        if (e == hipSuccess) e = hipEventRecord(kt.stop, s);
        if (e != hipSuccess) return e;
    }
    return marks ? hipEventRecord(marks[launches.size()], s) : hipSuccess;
}

// The filter launches of one variant; on a streaming plan `advance` then
// moves every channel's history and block counter past this call (the
// autotuner's trial runs leave them alone).
hipError_t launch(const vbw_plan_s *p, hipStream_t s, int variant, bool advance = true, KernelTimes kt = {}) {
    const vbw::LaunchArgs a = launch_args(p);
    hipError_t e = launch_variant(p, a, s, variant, nullptr, kt);
    if (e != hipSuccess) return e;
    if (advance && (p->flags & VBW_STREAM))
        return vbw::launch_stream_update(a, int(p->ch.size()), storage_of(p->dtype), p->d_hist, p->d_block0, s);
    return hipSuccess;
}

// Time every launch variant on the caller's buffers (filtering is idempotent:
// each run rewrites the same outputs) and keep the fastest.  The per-N
// variants launch the N groups in the same order, so each group's launch is
// timed on its own too; when the fastest shape differs between groups, the
// variant that takes each group's fastest launch is added and competes on
// the sum of those times.  Blocking, once per plan.
// Tuning cache: with the plan's tune_cache file, the choice is kept as one
// "key choice" line per plan shape and reused by later plans (and processes)
// of the same shape instead of timing again.  The key holds the device
// architecture and CU count, storage, engine, the flags that change the
// kernels, the workgroup cap and per N the log2 of the block count; the
// choice is a variant index, or per N group the index of its per-N variant.
std::string tune_key(const vbw_plan_s *p) {
    hipDeviceProp_t prop;
    std::string key = "vbw2";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
        key += ":";
        for (const char *c = prop.gcnArchName; *c && *c != ':'; ++c) key += *c;
        key += ":" + std::to_string(prop.multiProcessorCount);
    }
    key += ":d" + std::to_string(p->dtype) + ":e" + std::to_string(p->engine) + ":f" +
           std::to_string(p->flags & (VBW_NO_PRUNE | VBW_F32_OUT | VBW_STREAM)) + ":w" + std::to_string(p->max_wg);
    int64_t blocks[vbw::kMaxLog2N + 1] = {};
    for (const auto &it : p->items) blocks[it.log2n] += it.n_blocks;
    for (int lg = 0; lg <= vbw::kMaxLog2N; ++lg)
        if (blocks[lg]) key += ":n" + std::to_string(lg) + "b" + std::to_string(int(std::log2(double(blocks[lg]))));
    return key;
}

std::string tune_cache_lookup(const vbw_plan_s *p) {
    FILE *f = std::fopen(p->tune_cache.c_str(), "r");
    if (!f) return std::string();
    const std::string key = tune_key(p);
    char k[1024], v[1024];
    std::string found;
    while (std::fscanf(f, "%1023s %1023s", k, v) == 2)
        if (key == k) found = v;      // the last line for a key wins
    std::fclose(f);
    return found;
}

// Take a kept choice: "k" (variant k) or "k0,k1,..." (per N group, the
// launch of per-N variant k_g).  Anything that does not fit this plan is
// ignored (the autotuner then times again).
void tune_cache_apply(vbw_plan_s *p, const std::string &choice) {
    if (choice.empty()) return;
    std::vector<int> ks;
    size_t i = 0;
    while (i < choice.size()) {
        size_t j = i;
        while (j < choice.size() && choice[j] >= '0' && choice[j] <= '9') ++j;
        if (j == i || j - i > 6) return;
        ks.push_back(std::atoi(choice.substr(i, j - i).c_str()));
        if (j < choice.size() && choice[j] != ',') return;
        i = j + 1;
    }
    const size_t n_var = p->variants.size();
    if (ks.size() == 1) {
        if (ks[0] < 0 || size_t(ks[0]) >= n_var) return;
        p->variant = ks[0];
    } else {
        if (ks.size() != p->variants[0].size()) return;
        for (int k : ks)
            if (k < 0 || size_t(k) >= n_var || p->shapes[size_t(k)].dispatch) return;
        p->variants.push_back(combine(p, ks));
        p->composite = ks;
        p->variant = int(n_var);
    }
    p->tuned = true;
}

void tune_cache_store(const vbw_plan_s *p) {
    if (p->tune_cache.empty()) return;
    std::string choice;
    if (!p->composite.empty() && size_t(p->variant) + 1 == p->variants.size()) {
        for (size_t g = 0; g < p->composite.size(); ++g) choice += (g ? "," : "") + std::to_string(p->composite[g]);
    } else {
        choice = std::to_string(p->variant);
    }
    if (FILE *f = std::fopen(p->tune_cache.c_str(), "a")) {
        std::fprintf(f, "%s %s\n", tune_key(p).c_str(), choice.c_str());
        std::fclose(f);
    }
}

vbw_status autotune(vbw_plan_s *p, hipStream_t s) {
    const Range range("vbw_autotune");
    if (p->variants.size() < 2) {
        p->tuned = true;
        return VBW_OK;
    }
    const size_t n_groups = p->variants[0].size();
    std::vector<hipEvent_t> ev(n_groups + 1, nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    const vbw::LaunchArgs args = launch_args(p);
    const size_t n_var = p->variants.size();
    // Rounds that visit every variant in turn, each variant keeping its
    // fastest round: a clock that is still rising (or falling) under the
    // first sustained load moves all variants alike instead of favouring the
    // ones timed last.
    constexpr int kRounds = 4;
    constexpr float kInf = 3.0e38f;
    std::vector<float> total(n_var, kInf);
    std::vector<std::vector<float>> group(n_var, std::vector<float>(n_groups, kInf));
    for (size_t v = 0; e == hipSuccess && v < n_var; ++v) e = launch_variant(p, args, s, int(v));   // warm-up
    for (int r = 0; r < kRounds && e == hipSuccess; ++r) {
        for (size_t v = 0; e == hipSuccess && v < n_var; ++v) {
            e = launch_variant(p, args, s, int(v), ev.data());
            if (e == hipSuccess) e = hipEventSynchronize(ev[p->variants[v].size()]);
            float sum = 0.f;
            for (size_t g = 0; e == hipSuccess && g < p->variants[v].size(); ++g) {
                float ms = 0.f;
                e = hipEventElapsedTime(&ms, ev[g], ev[g + 1]);
                group[v][g] = std::min(group[v][g], ms);
                sum += ms;
            }
            total[v] = std::min(total[v], sum);
        }
    }
    float best = 0.f;
    int best_v = 0;
    std::vector<float> group_best(n_groups, 0.f);
    std::vector<int> group_choice(n_groups, 0);
    for (size_t v = 0; e == hipSuccess && v < n_var; ++v) {
        if (v == 0 || total[v] < best) {
            best = total[v];
            best_v = int(v);
        }
        if (v < p->shapes.size() && !p->shapes[v].dispatch)
            for (size_t g = 0; g < n_groups; ++g)
                if (v == 0 || group[v][g] < group_best[g]) {
                    group_best[g] = group[v][g];
                    group_choice[g] = int(v);
                }
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return from_hip(e);
    p->variant = best_v;
    float combined = 0.f;
    for (float t : group_best) combined += t;
    const bool mixed = std::any_of(group_choice.begin(), group_choice.end(),
                                   [&](int k) { return k != group_choice[0]; });
    if (mixed && combined < best) {
        p->variants.push_back(combine(p, group_choice));
        p->composite = group_choice;
        p->variant = int(p->variants.size()) - 1;
    }
    p->tuned = true;
    try {
        tune_cache_store(p);
    } catch (const std::bad_alloc &) {
    }
    return VBW_OK;
}

// Host part of a plan from a validated description (throws std::bad_alloc).
void init_host(vbw_plan_s *p, const vbw_plan_desc *desc) {
    p->ch.assign(desc->channels, desc->channels + desc->n_channels);
    p->v32.resize(size_t(desc->n_v));
    for (int32_t i = 0; i < desc->n_v; ++i) p->v32[i] = float(desc->v_pool[i]);
    p->dtype = desc->dtype;
    p->engine = desc->engine;
    p->flags = desc->flags;
    p->tune_cache = desc->tune_cache ? desc->tune_cache : "";
    p->max_wg = desc->max_workgroups;
    p->sched.resize(p->ch.size());
    for (size_t c = 0; c < p->ch.size(); ++c) p->sched[c].e.push_back({0, p->ch[c].k1});
    build_items(p);
}

// Band-schedule entry: channel's k1 from block from_block on (Sec. III-B:
// only the integer edge changes).
vbw_status add_switch(vbw_plan_s *p, int32_t channel, int32_t k1, int64_t from_block) {
    if (!p || channel < 0 || size_t(channel) >= p->ch.size() || from_block < 0) return VBW_EINVAL;
    const vbw_channel &ch = p->ch[channel];
    if (!k1_in_range(ch.n, ch.lv, k1)) return VBW_ERANGE;
    auto &e = p->sched[channel].e;
    auto it = std::lower_bound(e.begin(), e.end(), std::make_pair(from_block, INT32_MIN));
    if (it != e.end() && it->first == from_block) {
        it->second = k1;
    } else {
        if (int(e.size()) >= kMaxSchedPerChannel) return VBW_EINVAL;
        try {
            e.insert(it, {from_block, k1});
        } catch (const std::bad_alloc &) {
            return VBW_ENOMEM;
        }
    }
    p->sched_dirty = true;
    return VBW_OK;
}

}  // namespace

extern "C" {

vbw_status vbw_plan(const vbw_plan_desc *desc, vbw_plan_t *out) {
    const Range range("vbw_plan");
    if (!out) return VBW_EINVAL;
    *out = nullptr;
    vbw_status st = validate_desc(desc);
    if (st != VBW_OK) return st;
    vbw_plan_s *p = new (std::nothrow) vbw_plan_s();
    if (!p) return VBW_ENOMEM;
    try {
        init_host(p, desc);
    } catch (const std::bad_alloc &) {
        delete p;
        return VBW_ENOMEM;
    }
    if (!(desc->flags & VBW_HOST_ONLY)) {
        g_alloc_count = 0;
        try {
            st = setup_device(p);
        } catch (const std::bad_alloc &) {   // host tables of the planner
            st = VBW_ENOMEM;
        }
        if (st != VBW_OK) {
            free_device(p);
            delete p;
            return st;
        }
    }
    *out = p;
    return VBW_OK;
}

vbw_status vbw_set_bandwidth(vbw_plan_t p, int32_t channel, int32_t k1, int64_t from_block) {
    return add_switch(p, channel, k1, from_block);
}

vbw_status vbw_plan_set_variant(vbw_plan_t p, int32_t variant) {
    if (!p || variant < 0 || size_t(variant) >= p->variants.size()) return VBW_EINVAL;
    if (p->host_only) return VBW_EUNSUPPORTED;
    if (variant != p->variant && p->graph_exec) {     // the captured graph holds the old launches
        (void)hipGraphExecDestroy(p->graph_exec);
        (void)hipGraphDestroy(p->graph);
        p->graph_exec = nullptr;
        p->graph = nullptr;
    }
    p->variant = variant;
    p->tuned = true;
    return VBW_OK;
}

void vbw_test_fail_device_alloc(int32_t k) { g_fail_alloc_at = k > 0 ? k : 0; }

static vbw_status filter_impl(vbw_plan_t p, const void *const *x, void *const *y, void *stream,
                              KernelTimes kt = {});

// Calls on one plan run in call order: a call on another stream than the
// plan's last call first waits, on the device, for that call's work (it may
// still read the per-call table or the stream state this call rewrites).
static hipError_t order_after_last(vbw_plan_t p, hipStream_t s) {
    if (!p->done_recorded || s == p->last_stream) return hipSuccess;
    return hipStreamWaitEvent(s, p->done_evt, 0);
}

static hipError_t record_done(vbw_plan_t p, hipStream_t s) {
    const hipError_t e = hipEventRecord(p->done_evt, s);
    if (e == hipSuccess) {
        p->done_recorded = true;
        p->last_stream = s;
    }
    return e;
}

vbw_status vbw_filter(vbw_plan_t p, const void *const *x, void *const *y, void *stream) {
    const Range range("vbw_filter");
    try {
        return filter_impl(p, x, y, stream);
    } catch (const std::bad_alloc &) {   // host copies of the pointer arrays
        return VBW_ENOMEM;
    }
}

vbw_status vbw_filter_timed(vbw_plan_t p, const void *const *x, void *const *y, void *stream, void *start_event,
                            void *stop_event) {
    const Range range("vbw_filter_timed");
    if (!start_event || !stop_event) return VBW_EINVAL;
    if (p && (p->flags & VBW_GRAPH)) return VBW_EUNSUPPORTED;
    try {
        return filter_impl(p, x, y, stream,
                           {static_cast<hipEvent_t>(start_event), static_cast<hipEvent_t>(stop_event)});
    } catch (const std::bad_alloc &) {
        return VBW_ENOMEM;
    }
}

static vbw_status filter_impl(vbw_plan_t p, const void *const *x, void *const *y, void *stream, KernelTimes kt) {
    if (!p || !x || !y) return VBW_EINVAL;
    if (p->host_only) return VBW_EUNSUPPORTED;
    const size_t nch = p->ch.size();
    // pointers of the last uploaded call were checked then
    const bool ptrs_same = p->dyn_valid && std::equal(x, x + nch, p->last_x.begin()) &&
                           std::equal(y, y + nch, p->last_y.begin());
    if (!ptrs_same && !ranges_ok(p, x, y)) return VBW_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return from_hip(e);
    if (prev != p->device && (e = hipSetDevice(p->device)) != hipSuccess) return from_hip(e);

    vbw_status st = from_hip(order_after_last(p, s));
    if (st == VBW_OK && (!ptrs_same || p->sched_dirty)) st = upload_dyn(p, x, y, s);

    if (st == VBW_OK && !p->items.empty() && (p->flags & VBW_AUTOTUNE) && !p->tuned) st = autotune(p, s);
    if (st == VBW_OK && !p->items.empty()) {
        if ((p->flags & VBW_GRAPH) && s != nullptr) {
            if (!p->graph_exec) {
                e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    hipError_t le = launch(p, p->cap_stream, p->variant);
                    e = hipStreamEndCapture(p->cap_stream, &p->graph);
                    if (le != hipSuccess) e = le;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0);
                if (e != hipSuccess) st = from_hip(e);
            }
            if (st == VBW_OK) st = from_hip(hipGraphLaunch(p->graph_exec, s));
        } else {
            st = from_hip(launch(p, s, p->variant, true, kt));
        }
    } else if (st == VBW_OK && kt.start) {   // nothing to filter: an empty interval
        e = hipEventRecord(kt.start, s);
        if (e == hipSuccess) e = hipEventRecord(kt.stop, s);
        st = from_hip(e);
    }
    if (st == VBW_OK) st = from_hip(record_done(p, s));
    if (prev != p->device) (void)hipSetDevice(prev);
    return st;
}

vbw_status vbw_stream_reset(vbw_plan_t p, void *stream) {
    if (!p || !(p->flags & VBW_STREAM)) return VBW_EINVAL;
    if (p->host_only) return VBW_EUNSUPPORTED;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return from_hip(e);
    if (prev != p->device && (e = hipSetDevice(p->device)) != hipSuccess) return from_hip(e);
    hipStream_t s = static_cast<hipStream_t>(stream);
    e = order_after_last(p, s);
    if (e == hipSuccess) e = vbw::launch_stream_reset(p->d_hist, p->hist_bytes, p->d_block0, int(p->ch.size()), s);
    if (e == hipSuccess) e = record_done(p, s);
    if (prev != p->device) (void)hipSetDevice(prev);
    return from_hip(e);
}

void vbw_destroy(vbw_plan_t p) {
    if (!p) return;
    free_device(p);
    delete p;
}

const char *vbw_strerror(vbw_status s) {
    switch (s) {
        case VBW_OK: return "success";
        case VBW_EINVAL: return "invalid argument";
        case VBW_ERANGE: return "band edge out of range";
        case VBW_ENOMEM: return "out of memory";
        case VBW_EDEVICE: return "device error";
        case VBW_EUNSUPPORTED: return "unsupported request";
        case VBW_ETOOLARGE: return "tables exceed the allocation-free call's static scratch";
    }
    return "unknown status";
}

int64_t vbw_plan_query(vbw_plan_t p, int32_t q) {
    if (!p) return VBW_EINVAL;
    switch (q) {
        case VBW_Q_N_CHANNELS: return int64_t(p->ch.size());
        case VBW_Q_N_ITEMS: return int64_t(p->items.size());
        case VBW_Q_TOTAL_BLOCKS: return p->total_blocks;
        case VBW_Q_TOTAL_SAMPLES: return p->total_samples;
        case VBW_Q_WORKGROUP: return vbw::kThreads;
        case VBW_Q_LDS_BYTES: return int64_t(vbw::kLdsValues * sizeof(float2));
        case VBW_Q_GRID: {
            int64_t g = 0;
            if (!p->variants.empty())
                for (auto &lg : p->variants[size_t(p->variant)]) g += lg.n_wg;
            return g;
        }
        case VBW_Q_N_VARIANTS: return int64_t(p->variants.size());
        case VBW_Q_KERNEL_VARIANT: return p->variant;
    }
    return VBW_EINVAL;
}

int32_t vbw_block_k1(vbw_plan_t p, int32_t channel, int64_t block) {
    if (!p || channel < 0 || size_t(channel) >= p->ch.size() || block < 0) return VBW_EINVAL;
    int32_t k1 = VBW_EINVAL;
    for (auto &pr : p->sched[channel].e)
        if (pr.first <= block) k1 = pr.second;
    return k1;
}

vbw_status vbw_copy(const void *src, void *dst, int64_t bytes, void *stream) {
    if (bytes < 0 || (bytes > 0 && (!src || !dst))) return VBW_EINVAL;
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u) return VBW_EINVAL;
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(src), d0 = reinterpret_cast<uintptr_t>(dst);
    if (bytes > 0 && s0 < d0 + uintptr_t(bytes) && d0 < s0 + uintptr_t(bytes)) return VBW_EINVAL;
    int dev = 0, n_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = vbw::launch_copy(src, dst, bytes, n_cu, static_cast<hipStream_t>(stream));
    return from_hip(e);
}

vbw_status vbw_twiddle_table(int32_t n, float *out) {
    if (!out || !is_pow2(n) || n < 2 || n > vbw::kTwiddleN) return VBW_EINVAL;
    fill_twiddles(n, out);
    return VBW_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Allocation-free filtering: every device table of one call (twiddles, V,
// work list, workgroup ranges, the per-call table) lives in the static device
// array of scratch.hip instead of plan-owned allocations.

namespace {

constexpr size_t kScratchBytes = size_t(VBW_NOALLOC_SCRATCH_BYTES);
constexpr size_t kScratchTw = size_t(vbw::kTwiddleN) * sizeof(float2);   // twiddles at offset 0

// Once per device: the twiddle table, which never changes (synchronous copy).
hipError_t scratch_init(unsigned char *ptr) {
    std::vector<float> tw(2 * vbw::kTwiddleN);
    fill_twiddles(vbw::kTwiddleN, tw.data());
    return hipMemcpy(ptr, tw.data(), kScratchTw, hipMemcpyHostToDevice);
}

vbw_status filter_noalloc_impl(const vbw_plan_desc *desc, int32_t n_switches, const vbw_band_switch *sw,
                               const void *const *x, void *const *y, hipStream_t s) {
    if (!x || !y || n_switches < 0 || (n_switches > 0 && !sw)) return VBW_EINVAL;
    vbw_status st = validate_desc(desc);
    if (st != VBW_OK) return st;
    if (desc->flags & ~(VBW_NO_PRUNE | VBW_F32_OUT)) return VBW_EUNSUPPORTED;
    vbw_plan_s p;                        // host part only: nothing on the device
    init_host(&p, desc);
    for (int32_t i = 0; i < n_switches; ++i)
        if ((st = add_switch(&p, sw[i].channel, sw[i].k1, sw[i].from_block)) != VBW_OK) return st;
    if (!ranges_ok(&p, x, y)) return VBW_EINVAL;
    if (p.items.empty()) return VBW_OK;
    int dev = 0, n_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    unsigned char *base = nullptr;
    if (e == hipSuccess) e = vbw::scratch_of_device(dev, &base, scratch_init);
    if (e != hipSuccess) return from_hip(e);
    build_variants(&p, n_cu, true);      // the plan's default launch shape

    // layout after the twiddles: V | work list | workgroup ranges | per-call table
    size_t end = kScratchTw;
    auto take = [&end](size_t bytes) {
        const size_t o = end;
        end = (end + bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t o_v = take(p.v32.size() * sizeof(float));
    const size_t o_work = take(p.work.size() * sizeof(WorkItem));
    const size_t o_wg = take(p.wg_begin.size() * sizeof(int32_t));
    const size_t o_tab = take(p.dyn_bytes(p.sched_entries()));
    if (end > kScratchBytes) return VBW_ETOOLARGE;
    std::vector<unsigned char> h(end - kScratchTw);
    auto at = [&h](size_t o) { return h.data() + (o - kScratchTw); };   // host image of scratch offset o
    if (!p.v32.empty()) std::memcpy(at(o_v), p.v32.data(), p.v32.size() * sizeof(float));
    std::memcpy(at(o_work), p.work.data(), p.work.size() * sizeof(WorkItem));
    std::memcpy(at(o_wg), p.wg_begin.data(), p.wg_begin.size() * sizeof(int32_t));
    fill_call_table(&p, x, y, at(o_tab));
    // pageable source: the runtime has consumed it when the call returns
    if ((e = hipMemcpyAsync(base + kScratchTw, h.data(), h.size(), hipMemcpyHostToDevice, s)) != hipSuccess)
        return from_hip(e);

    vbw::LaunchArgs a;
    a.items = reinterpret_cast<const WorkItem *>(base + o_work);
    set_table_args(a, p.ch.size(), base + o_tab);
    a.v = reinterpret_cast<const float *>(base + o_v);
    a.tw = reinterpret_cast<const float2 *>(base);
    a.n_items = int32_t(p.work.size());
    a.wg_begin = reinterpret_cast<const int32_t *>(base + o_wg);
    a.hist = nullptr;
    a.block0 = nullptr;
    a.n_wg = 0;
    a.prune = (p.flags & VBW_NO_PRUNE) ? 0 : 1;
    a.pad = 0;
    return from_hip(launch_variant(&p, a, s, 0));
}

}  // namespace

extern "C" vbw_status vbw_filter_noalloc(const vbw_plan_desc *desc, int32_t n_switches,
                                         const vbw_band_switch *switches, const void *const *x, void *const *y,
                                         void *stream) {
    const Range range("vbw_filter_noalloc");
    try {
        return filter_noalloc_impl(desc, n_switches, switches, x, y, static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {   // host tables of the planner
        return VBW_ENOMEM;
    }
}

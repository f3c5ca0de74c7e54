// Host runtime and C-ABI of the gfx950 Smith-Waterman / Gotoh database search.
//
// Responsibilities:
//   * argument validation (before any HIP call);
//   * database preparation: length sort (descending, stable), chunking of 64
//     subjects, lane interleaving on the device (paper Section 3.1 splits the
//     database by length; here every subject gets a lane group sized to it);
//   * planning: per query, the sorted subjects are cut into wavefront items
//     whose lane group K grows with subject length so that every item carries a
//     bounded amount of work per lane; items are grouped four to a workgroup
//     item and ordered longest-first (longest-processing-time scheduling);
//     batches place the largest query first;
//   * workspace layout, plan upload through pinned staging buffers, and the
//     profile / search / rescore launches, all asynchronous on the caller's
//     stream.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "swdb.h"
#include "sw_internal.h"

using namespace swdb;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            return fail(SW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));         \
    } while (0)

// Bounds of the default per-item lane-cell target (resolve() derives the
// target from the work of the launch).
constexpr int64_t kMinLaneCells = 24 * 1024;
constexpr int64_t kMaxLaneCells = 192 * 1024;
constexpr int kDefaultLdsLimit = 64 * 1024;
constexpr int kLdsPerCU = 160 * 1024;
constexpr int kRescoreWavesPerCU = 16; // resident rescore wavefronts per CU (the grid)
constexpr int kMaxWavesPerCU = 16;      // 4 per SIMD: kernels are built for <= 128 VGPRs
constexpr int kLdsWavesPerCU = 12;      // resident waves per CU when every profile is in LDS

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t align_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Pinned host buffer for one plan upload.  States: free; held (handed to a
// call that has not yet recorded its completion event -- never reclaimable);
// in flight (event recorded after the upload; reclaimable once it completes).
struct Staging {
    enum State { kFree, kHeld, kInFlight };
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    State state = kFree;
};

struct PlanKey {
    int rows, spl, strict, kmax, nbr;
    int64_t target;
    bool operator<(const PlanKey& o) const
    {
        return std::tie(rows, spl, strict, kmax, nbr, target) <
               std::tie(o.rows, o.spl, o.strict, o.kmax, o.nbr, o.target);
    }
};

// Work items of one query (q field 0), largest per-lane work first.
struct QPlan {
    std::vector<Item> items;
    std::vector<int64_t> item_cost;   // per-lane work of each item
    int64_t slot_elems = 0;       // int2 entries a multi-pass item needs
    int64_t lane_cells = 0;       // sum over items of 64 * per-lane cells
    int64_t cost = 0;             // sum of per-lane work over items
    int64_t nitems = 0;
};

struct Resolved {
    Variant v;
    int rows, elem, spl, waves, kmax, lds_limit, grid_limit;
    int64_t target;
    bool i16;
    bool strict;          // lane groups within the item target only (no relaxed choice)
};

}  // namespace

struct sw_db_s {
    bool host_only = false;       // planning handle: no device memory
    int device = 0;
    int cu = 0;
    int lds_max = 64 * 1024;      // dynamic LDS a workgroup may use on this device
    int32_t nseq = 0;
    int64_t total = 0;
    int32_t nchunks = 0;
    int32_t max_len = 0;
    uint8_t* d_res = nullptr;
    int64_t* d_chunk_off = nullptr;
    int32_t* d_perm = nullptr;
    int32_t* d_slen = nullptr;
    int64_t res_bytes = 0;
    int64_t dev_bytes = 0;
    std::vector<int32_t> slen;    // sorted lengths
    std::mutex mu;
    std::deque<Staging> staging;  // deque: elements stay put while others are added
    std::map<PlanKey, std::shared_ptr<QPlan>> plans;
    std::deque<PlanKey> plan_order;
    std::vector<sw_tune_entry> tune;   // by ascending qlen (SW_MODE_TUNED)
};

namespace {

bool validate_options(const sw_options* opt, std::string& why)
{
    if (!opt)
        return true;
    if (opt->mode < SW_MODE_AUTO || opt->mode > SW_MODE_TUNED) { why = "options.mode"; return false; }
    if (opt->waves < 0 || opt->waves > 8) { why = "options.waves must be 0..8"; return false; }
    if (opt->lane_cells < 0) { why = "options.lane_cells"; return false; }
    if (opt->max_lanes < 0 || opt->max_lanes > 64) { why = "options.max_lanes must be 0..64"; return false; }
    if (opt->wide_profile < 0 || opt->wide_profile > 1) { why = "options.wide_profile must be 0 or 1"; return false; }
    if (opt->lds_limit < 0 || opt->lds_limit > 128 * 1024) { why = "options.lds_limit"; return false; }
    if (opt->grid_limit < 0) { why = "options.grid_limit"; return false; }
    if (opt->pair_cols < 0) { why = "options.pair_cols"; return false; }
    if (opt->pair_rows < 0) { why = "options.pair_rows"; return false; }
    if (opt->align_block < 0 || opt->align_block > (1 << 24)) { why = "options.align_block must be 0..2^24"; return false; }
    if (opt->slice_mcells < 0) { why = "options.slice_mcells"; return false; }
    if (opt->slice_begin < 0 || opt->slice_count < 0) { why = "options.slice_begin / slice_count"; return false; }
    if (opt->strict_groups < 0 || opt->strict_groups > 1) { why = "options.strict_groups must be 0 or 1"; return false; }
    if ((opt->slice_begin || opt->slice_count) && opt->slice_mcells <= 0) {
        why = "options.slice_begin / slice_count need slice_mcells > 0";
        return false;
    }
    return true;
}

int64_t prof_bytes_for(int nbr, int rows, int elem);

// Narrowest profile entries the matrix and gap-open penalty allow (profile
// entries are s + Go): kFitU8 -- every entry in [0, 127] (8-bit profiles for
// both lane widths); kFitS8 -- in [-128, 127] (8-bit for int32 lanes);
// kFit16 -- 16-bit only.
enum ProfileFit : int { kFitInvalid = 0, kFitS8 = 1, kFit16 = 2, kFitU8 = 3 };

// Launch options of one launch group.  Defaults (measured on MI355X):
//  * lane-cell target per item: the cells over 5 items per wavefront slot of
//    a nominally full device (12 waves per CU), clamped to [24K, 192K] -- short
//    searches want small items for a short tail, large batches want large ones
//    for less padding and fewer passes (a 567-residue query against 200,000
//    subjects ran 1.7% faster with 5 than with 4.5, which sets a target of
//    48K: most items come out below the target, so whole rounds of items per
//    wavefront matter more than the nominal count);
//  * 4 wavefronts per workgroup, or 8 when queries with an LDS profile share
//    the launch with queries whose profile stays in global memory, so that the
//    LDS footprint still leaves 16 waves per CU to hide the global reads.
//  * the narrowest profile entries the matrix allows (`fit`, a ProfileFit),
//    unless the options ask for 16-bit entries.
Resolved resolve(const sw_db_s* db, const sw_options* opt, int fit, int32_t nq, const int32_t* q_lens)
{
    Resolved r{};
    const int mode = opt ? opt->mode : SW_MODE_AUTO;
    const bool wide = opt && opt->wide_profile;
    r.i16 = mode != SW_MODE_I32;
    if (r.i16) {
        r.v = (fit == kFitU8 && !wide) ? kI16_P8 : kI16;
    } else {
        r.v = ((fit == kFitS8 || fit == kFitU8) && !wide) ? kI32_R32_P8 : kI32_R32_P16;
    }
    const LaunchInfo li = variant_info(r.v);
    r.rows = li.rows;
    r.elem = li.prof_elem;
    r.spl = li.subjects_per_lane;
    r.kmax = (opt && opt->max_lanes) ? opt->max_lanes : 64;
    r.lds_limit = (opt && opt->lds_limit) ? opt->lds_limit : kDefaultLdsLimit;
    r.lds_limit = std::min(r.lds_limit, db->lds_max - 1024);
    r.grid_limit = opt ? opt->grid_limit : 0;
    r.strict = opt && opt->strict_groups;
    double cells = 0;
    bool in_lds = false, in_global = false;
    for (int32_t k = 0; k < nq; ++k) {
        cells += (double)q_lens[k] * (double)db->total;
        const int nbr = (int)ceil_div(q_lens[k], r.rows);
        (prof_bytes_for(nbr, r.rows, r.elem) <= r.lds_limit ? in_lds : in_global) = true;
    }
    if (opt && opt->lane_cells) {
        r.target = opt->lane_cells;
    } else {
        const double slots = (double)kWave * std::max(db->cu, 1) * 12;
        r.target = std::min<int64_t>(std::max<int64_t>((int64_t)(cells / slots / 5.0), kMinLaneCells),
                                     kMaxLaneCells);
    }
    r.waves = (opt && opt->waves) ? opt->waves : ((in_lds && in_global) ? 8 : 4);
    return r;
}

int64_t prof_bytes_for(int nbr, int rows, int elem)
{
    const int64_t cs = code_stride(rows, elem);
    return (int64_t)(nbr + 1) * kCodes * cs;
}

// Per-lane cells of an item: the columns it sweeps (with pipeline fill for K > 1)
// times the rows of all its passes.
int64_t lane_work(int64_t n, int K, int nbr, int rows)
{
    const int64_t cols = K == 1 ? align_up(n, 4) : align_up(n + K - 1, 4);
    const int64_t passes = nbr == 0 ? 0 : ceil_div(nbr, K);
    return std::max<int64_t>(cols, 4) * passes * rows;
}

// Lane cells the wavefront sweeps per subject with lane groups of K: all 64
// lanes (leftover lanes of 64 mod K idle) over the item's work, divided by the
// subjects it carries.  Pipelined groups cost a few extra instructions per
// column (DPP shifts, head selects), weighed in as 4%.
double subject_cost(int64_t n, int K, int nbr, const Resolved& r)
{
    const double per = (double)(kWave / K) * r.spl;
    return kWave * (double)lane_work(n, K, nbr, r.rows) / per * (K > 1 ? 1.04 : 1.0);
}

// Lane group size for a subject of length n: the cheapest (in swept cells per
// subject) K whose per-lane work fits the target; if none fits, the K with the
// least per-lane work.  K > nbr would only add idle row blocks.  A K with up
// to twice the target's per-lane work is taken instead when it sweeps at
// least kRelaxGain fewer cells per subject: typically the long subjects of a
// short query, where the only group that fits (all row blocks in one pass)
// leaves lanes idle (64 mod K) and half as large a group with two passes does
// not.  Such items are few and, being large, run early in queue order.
constexpr double kRelaxGain = 0.10;

int choose_k(int64_t n, int nbr, const Resolved& r)
{
    const int kmax = std::max(1, std::min(r.kmax, nbr));
    int best = -1, shortest = 1, relaxed = -1;
    double best_cost = 0, relaxed_cost = 0;
    int64_t best_lw = lane_work(n, 1, nbr, r.rows);
    for (int K = 1; K <= kmax; ++K) {
        const int64_t lw = lane_work(n, K, nbr, r.rows);
        const double c = subject_cost(n, K, nbr, r);
        if (lw <= r.target && (best < 0 || c < best_cost)) {
            best = K;
            best_cost = c;
        }
        if (lw <= 2 * r.target && (relaxed < 0 || c < relaxed_cost)) {
            relaxed = K;
            relaxed_cost = c;
        }
        if (lw < best_lw) {
            best_lw = lw;
            shortest = K;
        }
    }
    if (!r.strict && best > 0 && relaxed > 0 && relaxed_cost <= (1.0 - kRelaxGain) * best_cost)
        return relaxed;
    return best > 0 ? best : shortest;
}

// Per-lane cells of a self-paired item (packed lanes, one subject per
// wavefront, 128 row blocks per pass, a 128-column pipeline).
int64_t lane_work_self(int64_t n, int nbr, int rows)
{
    const int64_t passes = nbr == 0 ? 0 : ceil_div(nbr, 2 * kWave);
    return std::max<int64_t>(align_up(n + 2 * kWave - 1, 4), 4) * passes * rows;
}

// Work items of one query.  Subjects in length order are grouped floor(64/K)
// x spl to an item with the lane-group size chosen per length.  In the packed
// variant, an item whose per-lane work exceeds the mean work of a resident
// wavefront (the longest subjects against a long query) would end the launch
// late however it is scheduled; its subjects become self-paired items instead,
// one subject per wavefront with both halves of every lane on its rows, which
// halves the per-lane work (the critical path) for the same total work.
std::shared_ptr<QPlan> build_plan(const std::vector<int32_t>& slen, int nbr, const Resolved& r,
                                  int64_t resident_waves)
{
    auto p = std::make_shared<QPlan>();
    const int64_t N = (int64_t)slen.size();
    struct WItem { Item it; int64_t cost; };
    std::vector<WItem> wis;
    int64_t s = 0;
    int64_t last_n = -1;
    int K = 1;
    double total = 0;
    while (s < N) {
        const int64_t n = slen[s];
        if (n != last_n) {
            K = choose_k(n, nbr, r);
            last_n = n;
        }
        const int64_t per = (int64_t)(kWave / K) * r.spl;
        const int64_t take = std::min<int64_t>(per, N - s);
        Item it;
        it.s0 = (int32_t)s;
        it.ncols = (int32_t)align_up(n, 4);
        it.q = 0;
        it.meta = (int32_t)take | (K << 16);
        const int64_t lw = lane_work(n, K, nbr, r.rows);
        wis.push_back({it, lw});
        total += (double)lw;
        s += take;
    }
    if (r.spl == 2 && nbr > kWave) {
        const double mean = total / (double)std::max<int64_t>(resident_waves, 1);
        std::vector<WItem> out;
        out.reserve(wis.size());
        for (const WItem& w : wis) {
            if ((double)w.cost < mean) {
                out.push_back(w);
                continue;
            }
            const int nsub = w.it.meta & 0xffff;
            for (int k = 0; k < nsub; ++k) {
                Item it;
                it.s0 = w.it.s0 + k;
                it.ncols = (int32_t)align_up(slen[it.s0], 4);
                it.q = 0;
                it.meta = 1 | (kWave << 16) | (1 << 25);   // bit 25: self-paired
                out.push_back({it, lane_work_self(slen[it.s0], nbr, r.rows)});
            }
        }
        wis.swap(out);
    }
    for (WItem& w : wis) {
        const int K = (w.it.meta >> 16) & 0xff;
        const bool self = (w.it.meta >> 25) & 1;
        // bit 24: critical-path item (per-lane work well above the target)
        if (w.cost >= 2 * r.target)
            w.it.meta |= 1 << 24;
        p->lane_cells += w.cost * kWave;
        if (self ? nbr > 2 * kWave : nbr > K)
            p->slot_elems = std::max<int64_t>(p->slot_elems, (int64_t)w.it.ncols * (self ? 1 : kWave / K));
    }
    // longest-processing-time order: largest per-lane work first
    std::stable_sort(wis.begin(), wis.end(), [](const WItem& a, const WItem& b) { return a.cost > b.cost; });
    p->nitems = (int64_t)wis.size();
    p->items.resize(wis.size());
    p->item_cost.resize(wis.size());
    for (size_t i = 0; i < wis.size(); ++i) {
        p->items[i] = wis[i].it;
        p->item_cost[i] = wis[i].cost;
        p->cost += wis[i].cost;
    }
    p->slot_elems = align_up(p->slot_elems, 4);
    return p;
}

std::shared_ptr<QPlan> get_plan(sw_db_s* db, int nbr, const Resolved& r)
{
    PlanKey key{r.rows, r.spl, r.strict ? 1 : 0, r.kmax, nbr, r.target};   // items do not depend on waves
    std::lock_guard<std::mutex> lk(db->mu);
    auto f = db->plans.find(key);
    if (f != db->plans.end())
        return f->second;
    auto p = build_plan(db->slen, nbr, r, (int64_t)std::max(db->cu, 1) * kMaxWavesPerCU);
    db->plans[key] = p;
    db->plan_order.push_back(key);
    while (db->plan_order.size() > 512) {
        db->plans.erase(db->plan_order.front());
        db->plan_order.pop_front();
    }
    return p;
}

// Workspace layout of one search.
struct Layout {
    Resolved r;
    int32_t nq = 0;
    std::vector<QueryDesc> qd;        // queue order; out_row = query's position in the call
    std::vector<std::shared_ptr<QPlan>> plans;   // by position in the call
    std::vector<int32_t> order;       // queue position -> position in the call
    std::vector<std::pair<int64_t, int64_t>> ranges;   // by position: window [begin, end) of the plan's items
    int64_t grid = 0, rgrid = 0;
    int rwaves = 1;               // wavefronts per rescore workgroup
    int64_t slot_elems = 0, rslot_elems = 0;
    int lds_bytes = 0;
    int64_t cells = 0, lane_cells = 0, nitems = 0;
    int max_entries = 0;
    // The plan blob uploaded before a launch group covers [off_status,
    // off_prof): status words (cleared by the first group of a call only),
    // per-group counters and queue heads (cleared by every group), query
    // descriptors, query offsets and work items.
    size_t off_status = 0, off_counters = 0, off_heads = 0, off_qd = 0, off_qoff = 0, off_items = 0,
           off_prof = 0, off_flags = 0, off_slots = 0, total = 0, blob = 0;
    int64_t flag_cap = 0;
};

// Real cells of items [b, e) of a query of m rows.
int64_t range_cells(const sw_db_s* db, const QPlan& p, int64_t b, int64_t e, int32_t m)
{
    int64_t n = 0;
    for (int64_t i = b; i < e; ++i) {
        const Item& it = p.items[i];
        for (int k = 0; k < (it.meta & 0xffff); ++k)
            n += db->slen[(size_t)it.s0 + k];
    }
    return n * m;
}

// Layout of a launch group of nq queries; `ranges` (by position in the call,
// may be null for every item) limits each query to a window of its plan's
// items -- one launch of a sliced search.
int make_layout(sw_db_s* db, int32_t nq, const int32_t* q_lens, const Resolved& r, Layout& L,
                const std::vector<std::pair<int64_t, int64_t>>* ranges = nullptr)
{
    L.r = r;
    L.nq = nq;
    L.qd.assign(nq, QueryDesc{});
    L.plans.assign(nq, nullptr);
    L.ranges.assign(nq, {0, 0});
    int64_t prof = 0;
    int64_t slot_need = 0;
    for (int32_t k = 0; k < nq; ++k) {
        const int32_t m = q_lens[k];
        const int nbr = (int)ceil_div(m, r.rows);
        const int64_t pb = prof_bytes_for(nbr, r.rows, 2);   // sized for 16-bit entries
        L.qd[k].prof_off = prof;
        L.qd[k].out_row = k;
        L.qd[k].m = m;
        L.qd[k].nbr = nbr;
        const int64_t pbe = prof_bytes_for(nbr, r.rows, r.elem);
        L.qd[k].prof_bytes = (int32_t)pbe;
        L.qd[k].lds = pbe <= r.lds_limit ? 1 : 0;
        if (L.qd[k].lds)
            L.lds_bytes = std::max<int>(L.lds_bytes, (int)pbe);
        L.max_entries = std::max<int>(L.max_entries, (nbr + 1) * kCodes * r.rows);
        prof += align_up(pb, 256);
        L.plans[k] = get_plan(db, nbr, r);
        slot_need = std::max(slot_need, L.plans[k]->slot_elems);
        const QPlan& pl = *L.plans[k];
        if (ranges) {
            const auto [b, e] = (*ranges)[k];
            if (b < 0 || e > pl.nitems || b > e) return fail(SW_EINVAL, "internal error: item window");
            L.ranges[k] = {b, e};
            L.cells += range_cells(db, pl, b, e, m);
            L.lane_cells += kWave * std::accumulate(pl.item_cost.begin() + b, pl.item_cost.begin() + e, int64_t(0));
            L.nitems += e - b;
        } else {
            L.ranges[k] = {0, pl.nitems};
            L.cells += (int64_t)m * db->total;
            L.lane_cells += pl.lane_cells;
            L.nitems += pl.nitems;
        }
    }
    // queue: largest query first; descriptors stored in queue order
    L.order.resize(nq);
    std::iota(L.order.begin(), L.order.end(), 0);
    std::stable_sort(L.order.begin(), L.order.end(), [&](int a, int b) {
        if (L.plans[a]->cost != L.plans[b]->cost)
            return L.plans[a]->cost > L.plans[b]->cost;
        return q_lens[a] > q_lens[b];
    });
    std::vector<QueryDesc> by_call = L.qd;
    int64_t nit = 0;
    for (int32_t p = 0; p < nq; ++p) {
        const int32_t k = L.order[p];
        L.qd[p] = by_call[k];
        L.qd[p].item_begin = (int32_t)nit;
        L.qd[p].item_count = (int32_t)(L.ranges[k].second - L.ranges[k].first);
        nit += L.qd[p].item_count;
        if (nit > INT32_MAX / 2)
            return fail(SW_EINVAL, "batch too large for one launch");
    }
    // Slots: one per resident wavefront, at most the register-limited 16 per
    // CU (8 per workgroup at most).  Their count depends neither on the
    // workgroup width nor on the profile entry width chosen from the matrix,
    // so the workspace size (computed for 16-bit entries) covers every choice.
    int64_t nslots = std::min<int64_t>(align_up(std::max<int64_t>(nit, 1), 8), (int64_t)db->cu * kMaxWavesPerCU);
    if (r.grid_limit > 0)
        nslots = std::min<int64_t>(nslots, (int64_t)r.grid_limit * 8);
    nslots = align_up(nslots, 8);
    // persistent grid: occupancy model (LDS per CU; at most 16 waves per CU, 12
    // when every profile is in LDS -- measured faster there: the longest items
    // on the critical path share their SIMD with fewer waves)
    bool all_lds = true;
    for (int32_t p = 0; p < nq; ++p)
        all_lds = all_lds && L.qd[p].lds;
    const int wave_cap = all_lds ? kLdsWavesPerCU : kMaxWavesPerCU;
    const int wg_cap = std::max(wave_cap / r.waves, 1);
    int wg_per_cu = wg_cap;
    if (L.lds_bytes > 0)
        wg_per_cu = std::min(wg_per_cu, kLdsPerCU / (L.lds_bytes + 1024));
    wg_per_cu = std::max(wg_per_cu, 1);
    L.grid = std::min<int64_t>({ceil_div(nit, r.waves), nslots / r.waves, (int64_t)db->cu * wg_per_cu});
    if (r.grid_limit > 0)
        L.grid = std::min<int64_t>(L.grid, r.grid_limit);
    L.slot_elems = align_up(std::max<int64_t>(slot_need, 4), 4);
    if (r.i16) {
        // rescore: a workgroup per listed subject, one wavefront per 64-lane
        // pass of the longest query (at most kRescoreMaxWaves)
        int maxp = 1;
        for (int32_t p = 0; p < nq; ++p)
            maxp = std::max<int>(maxp, (int)ceil_div(L.qd[p].nbr, kWave));
        L.rwaves = std::min(maxp, kRescoreMaxWaves);
        L.rgrid = std::max<int64_t>(1, (int64_t)db->cu * kRescoreWavesPerCU / L.rwaves);
        L.rslot_elems = align_up(std::max<int64_t>(align_up(db->max_len, 16), 4), 4);
        L.flag_cap = (int64_t)nq * db->nseq;
    }
    // byte layout
    size_t off = 0;
    L.off_status = off; off += kStatusBytes;
    L.off_counters = off; off += 256;
    L.off_heads = off; off += align_up(sizeof(int32_t) * nq, 256);
    L.off_qd = off; off += align_up(sizeof(QueryDesc) * nq, 16);
    L.off_qoff = off; off += align_up(sizeof(int64_t) * nq, 16);
    L.off_items = off;
    off += align_up(sizeof(Item) * nit, 256);
    L.blob = off - L.off_status;
    L.off_prof = off; off += align_up(prof, 256);
    L.off_flags = off; off += align_up(sizeof(int2) * L.flag_cap, 256);
    L.off_slots = off;
    const int64_t main_slots = nslots * L.slot_elems * (int64_t)sizeof(int2);
    const int64_t res_slots = L.rgrid * L.rwaves * L.rslot_elems * (int64_t)sizeof(int2);
    off += align_up(std::max(main_slots, res_slots), 256);
    L.total = off;
    return SW_OK;
}

int validate_query_set(sw_db_t db, int32_t nq, const int32_t* q_lens)
{
    if (!db) return fail(SW_EINVAL, "null database handle");
    if (nq < 0) return fail(SW_EINVAL, "nq < 0");
    if (nq > 0 && !q_lens) return fail(SW_EINVAL, "null q_lens");
    for (int32_t k = 0; k < nq; ++k)
        if (q_lens[k] < 0 || q_lens[k] > SW_MAX_QLEN)
            return fail(SW_EINVAL, "query length out of range");
    return SW_OK;
}

// The ProfileFit of a matrix and gap-open penalty; kFitInvalid with `why`
// set if the matrix is invalid.
int matrix_elem(const int32_t* sm, int32_t go, std::string& why)
{
    int mn = 1 << 30, mx = -(1 << 30);
    for (int i = 0; i < kAlpha * kAlpha; ++i) {
        if (sm[i] < -128 || sm[i] > 127) {
            why = "substitution matrix entry outside [-128, 127]";
            return kFitInvalid;
        }
        mn = std::min(mn, sm[i]);
        mx = std::max(mx, sm[i]);
    }
    if (mx + go > 127 || mn + go < -128)
        return kFit16;
    return mn + go >= 0 ? kFitU8 : kFitS8;
}

void* acquire_staging(sw_db_s* db, size_t bytes, Staging** out)
{
    std::lock_guard<std::mutex> lk(db->mu);
    for (auto& st : db->staging) {
        if (st.state == Staging::kInFlight && hipEventQuery(st.ev) == hipSuccess)
            st.state = Staging::kFree;
        if (st.state == Staging::kFree && st.cap >= bytes) {
            st.state = Staging::kHeld;
            *out = &st;
            return st.host;
        }
    }
    Staging st;
    st.cap = std::max<size_t>(bytes, 1 << 20);
    if (hipHostMalloc(&st.host, st.cap, hipHostMallocDefault) != hipSuccess)
        return nullptr;
    if (hipEventCreateWithFlags(&st.ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(st.host);
        return nullptr;
    }
    st.state = Staging::kHeld;
    db->staging.push_back(st);
    *out = &db->staging.back();
    return st.host;
}

// One launch group of a search: queries that share a schedule.  Plain modes
// give one group; SW_MODE_TUNED groups queries by the tuned schedule of their
// length and launches the groups one after another on the stream.
struct Part {
    Layout L;
    std::vector<int32_t> idx;        // caller's query indices (score rows)
    std::vector<int32_t> lens;
    std::vector<int64_t> offs;
    size_t total() const { return L.total; }
};

sw_options tuned_for(const sw_db_s* db, int32_t m, int* which)
{
    sw_options o{};
    *which = -1;
    if (db->tune.empty())
        return o;
    int k = (int)db->tune.size() - 1;
    for (int i = 0; i < (int)db->tune.size(); ++i)
        if (db->tune[i].qlen >= m) { k = i; break; }
    *which = k;
    o = db->tune[k].opt;
    o.ev_search_begin = o.ev_search_end = o.ev_rescore_end = nullptr;
    return o;
}

// A launch group cut into launches of at most `limit` lane cells each: its
// queue (queries in queue order, each query's items largest first) is walked
// in order and every launch takes the next items until the limit would be
// passed (at least one item).  Each launch keeps the group's schedule, so its
// items are exactly the group's, and writes its queries' rows.
int slice_part(sw_db_s* db, const Part& P, int64_t limit, std::vector<Part>& out)
{
    const Layout& L = P.L;
    struct Piece { int32_t k; int64_t b, e; };
    std::vector<Piece> cur;
    int64_t acc = 0;
    auto flush = [&]() -> int {
        if (cur.empty()) return SW_OK;
        Part S;
        std::vector<std::pair<int64_t, int64_t>> ranges;
        for (const Piece& pc : cur) {         // queue order; make_layout keeps it (same plan costs)
            S.idx.push_back(P.idx[pc.k]);
            S.lens.push_back(P.lens[pc.k]);
            S.offs.push_back(P.offs[pc.k]);
            ranges.push_back({pc.b, pc.e});
        }
        const int rc = make_layout(db, (int32_t)S.idx.size(), S.lens.data(), L.r, S.L, &ranges);
        if (rc) return rc;
        for (QueryDesc& d : S.L.qd)
            d.out_row = S.idx[d.out_row];
        out.push_back(std::move(S));
        cur.clear();
        acc = 0;
        return SW_OK;
    };
    for (int32_t k : L.order) {
        const QPlan& pl = *L.plans[k];
        int64_t b = L.ranges[k].first;
        for (int64_t i = L.ranges[k].first; i < L.ranges[k].second; ++i) {
            const int64_t c = kWave * pl.item_cost[i];
            if (acc > 0 && acc + c > limit) {
                if (i > b) cur.push_back({k, b, i});
                const int rc = flush();
                if (rc) return rc;
                b = i;
            }
            acc += c;
        }
        if (L.ranges[k].second > b) cur.push_back({k, b, L.ranges[k].second});
    }
    return flush();
}

int build_parts(sw_db_s* db, int32_t nq, const int32_t* q_lens, const int64_t* q_offsets,
                const sw_options* opt, int elem, std::vector<Part>& parts)
{
    parts.clear();
    const bool tuned = opt && opt->mode == SW_MODE_TUNED;
    std::map<int, size_t> group_of;
    std::vector<sw_options> gopt;
    for (int32_t k = 0; k < nq; ++k) {
        int which = -1;
        sw_options o{};
        if (tuned) {
            std::lock_guard<std::mutex> lk(db->mu);
            o = tuned_for(db, q_lens[k], &which);
        } else if (opt) {
            o = *opt;
        }
        auto f = group_of.find(which);
        if (f == group_of.end()) {
            f = group_of.emplace(which, parts.size()).first;
            parts.emplace_back();
            gopt.push_back(o);
        }
        Part& P = parts[f->second];
        P.idx.push_back(k);
        P.lens.push_back(q_lens[k]);
        P.offs.push_back(q_offsets ? q_offsets[k] : 0);
    }
    for (size_t g = 0; g < parts.size(); ++g) {
        Part& P = parts[g];
        const int32_t n = (int32_t)P.idx.size();
        const int rc = make_layout(db, n, P.lens.data(), resolve(db, &gopt[g], elem, n, P.lens.data()), P.L);
        if (rc) return rc;
        for (QueryDesc& d : P.L.qd)
            d.out_row = P.idx[d.out_row];
    }
    if (opt && opt->slice_mcells > 0) {
        std::vector<Part> sliced;
        for (const Part& P : parts) {
            const int rc = slice_part(db, P, (int64_t)opt->slice_mcells * 1000000, sliced);
            if (rc) return rc;
        }
        parts.swap(sliced);
    }
    return SW_OK;
}

size_t parts_bytes(const std::vector<Part>& parts)
{
    size_t b = 0;
    for (const Part& P : parts)
        b = std::max(b, P.total());
    return b;
}

// Validation and planning shared by every search entry point.
int plan_search(sw_db_t db, const uint8_t* queries, const int64_t* q_offsets, const int32_t* q_lens,
                int32_t nq, const int32_t* sm, int32_t go, int32_t ge, const sw_options* opt,
                void* ws, size_t ws_bytes, int32_t* scores, std::vector<Part>& parts, bool& nothing,
                bool* from_first = nullptr)
{
    nothing = false;
    if (from_first) *from_first = true;
    int rc = validate_query_set(db, nq, q_lens);
    if (rc) return rc;
    if (nq > 0 && !q_offsets) return fail(SW_EINVAL, "null q_offsets");
    int64_t sumq = 0;
    for (int32_t k = 0; k < nq; ++k) {
        if (q_offsets[k] < 0) return fail(SW_EINVAL, "negative query offset");
        sumq += q_lens[k];
    }
    if (sumq > 0 && !queries) return fail(SW_EINVAL, "null queries");
    if (!sm) return fail(SW_EINVAL, "null substitution matrix");
    if (go < 0 || ge < 0 || go > SW_MAX_GAP || ge > SW_MAX_GAP)
        return fail(SW_EINVAL, "gap penalties must be in [0, SW_MAX_GAP]");
    std::string why;
    if (!validate_options(opt, why)) return fail(SW_EINVAL, why);
    const int elem = matrix_elem(sm, go, why);
    if (!elem) return fail(SW_EINVAL, why);
    if (db->host_only) return fail(SW_EINVAL, "planning-only handle cannot search");
    if (nq == 0 || db->nseq == 0) {
        nothing = true;
        return SW_OK;
    }
    if (!scores) return fail(SW_EINVAL, "null scores_out");
    if (!ws) return fail(SW_EINVAL, "null workspace");
    if (((uintptr_t)ws & 255) != 0) return fail(SW_EINVAL, "workspace must be 256-byte aligned");
    rc = build_parts(db, nq, q_lens, q_offsets, opt, elem, parts);
    if (rc) return rc;
    // the size requirement is the one sw_workspace_bytes reports (16-bit profile sizing)
    std::vector<Part> sizing;
    rc = build_parts(db, nq, q_lens, q_offsets, opt, 2, sizing);
    if (rc) return rc;
    const size_t need = parts_bytes(sizing);
    if (ws_bytes < need)
        return fail(SW_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    if (parts_bytes(parts) > need)     // the layouts are built so that this never holds
        return fail(SW_EINVAL, "internal error: search layout exceeds the workspace size");
    if (opt && (opt->slice_begin > 0 || opt->slice_count > 0)) {
        const size_t b = (size_t)opt->slice_begin;
        if (b >= parts.size())
            return fail(SW_EINVAL, "options.slice_begin " + std::to_string(b) + " is not below the " +
                                       std::to_string(parts.size()) + " launches of this search");
        const size_t e = opt->slice_count > 0 ? std::min(parts.size(), b + (size_t)opt->slice_count) : parts.size();
        parts.erase(parts.begin() + e, parts.end());
        parts.erase(parts.begin(), parts.begin() + b);
        if (from_first) *from_first = b == 0;
    }
    return SW_OK;
}

// The plan blob in host memory: zeroed status words, counters and queue
// heads, then query descriptors, query offsets and the work queue.
void fill_blob(const Layout& L, const int64_t* q_offsets, uint8_t* h)
{
    std::memset(h, 0, L.off_qd - L.off_status);
    std::memcpy(h + (L.off_qd - L.off_status), L.qd.data(), sizeof(QueryDesc) * L.nq);
    int64_t* qoff = reinterpret_cast<int64_t*>(h + (L.off_qoff - L.off_status));
    Item* items = reinterpret_cast<Item*>(h + (L.off_items - L.off_status));
    int64_t pos = 0;
    for (int32_t p = 0; p < L.nq; ++p) {
        const int32_t k = L.order[p];
        qoff[p] = q_offsets[k];
        for (int64_t i = L.ranges[k].first; i < L.ranges[k].second; ++i) {
            Item it = L.plans[k]->items[i];
            it.q = p;
            items[pos++] = it;
        }
    }
}

// Everything a search puts on `stream`: plan upload from pinned host memory
// (which also clears the counters and queue heads, and for the first launch
// group of a call the status words), profile kernel, search kernel, flag-list
// sort and rescore kernel.  No memset: the sequence may be captured into a graph.
int enqueue_search(sw_db_t db, const Layout& L, const uint8_t* blob, const uint8_t* queries,
                   const int32_t* sm, int32_t go, int32_t ge, hipEvent_t e0, hipEvent_t e1, hipEvent_t e2,
                   void* ws, int32_t* scores, bool first, hipStream_t stream)
{
    const Resolved& r = L.r;
    uint8_t* w = static_cast<uint8_t*>(ws);
    const size_t skip = first ? 0 : L.off_counters - L.off_status;
    HIPCHK(hipMemcpyAsync(w + L.off_status + skip, blob + skip, L.blob - skip, hipMemcpyHostToDevice, stream));
    int32_t* status = reinterpret_cast<int32_t*>(w + L.off_status);

    ProfileArgs pa{};
    pa.queries = queries;
    pa.q_off = reinterpret_cast<const int64_t*>(w + L.off_qoff);
    pa.qd = reinterpret_cast<const QueryDesc*>(w + L.off_qd);
    pa.prof = w + L.off_prof;
    pa.bad = status + kStatusBadQuery;
    pa.nq = L.nq;
    pa.go = go;
    pa.pad = r.v == kI16_P8 ? 0 : (r.elem == 1 ? -128 : -32768);
    for (int i = 0; i < kAlpha * kAlpha; ++i)
        pa.sm.v[i] = (int8_t)sm[i];
    HIPCHK(launch_profile(pa, r.rows, r.elem, L.max_entries, stream));

    SearchArgs a{};
    a.res = db->d_res;
    a.chunk_off = db->d_chunk_off;
    a.perm = db->d_perm;
    a.slen = db->d_slen;
    a.nseq = db->nseq;
    a.items = reinterpret_cast<const Item*>(w + L.off_items);
    a.qd = pa.qd;
    a.nq = L.nq;
    a.heads = reinterpret_cast<int32_t*>(w + L.off_heads);
    a.n_items = L.nitems;
    a.prof = pa.prof;
    a.scores = scores;
    a.out_stride = db->nseq;
    a.counters = reinterpret_cast<int32_t*>(w + L.off_counters);
    a.status = status;
    a.bnd = reinterpret_cast<int2*>(w + L.off_slots);
    a.slot_elems = L.slot_elems;
    a.flags = reinterpret_cast<int2*>(w + L.off_flags);
    a.flag_cap = (int32_t)std::min<int64_t>(L.flag_cap, INT32_MAX);
    a.go = go;
    a.ge = ge;
    if (e0) HIPCHK(hipEventRecord(e0, stream));
    if (L.grid > 0)
        HIPCHK(launch_search(r.v, a, (int)L.grid, r.waves, L.lds_bytes, stream));
    if (e1) HIPCHK(hipEventRecord(e1, stream));
    if (r.i16 && L.grid > 0) {
        SearchArgs b = a;
        b.slot_elems = L.rslot_elems;
        HIPCHK(launch_flag_sort(b, stream));
        HIPCHK(launch_rescore(r.v, b, (int)L.rgrid, L.rwaves, stream));
    }
    if (e2) HIPCHK(hipEventRecord(e2, stream));
    return SW_OK;
}

// Events of a multi-part search: begin before the first search kernel, end
// after the last one, rescore-end after the last rescore.
// from_first: the parts begin with the search's first launch, which zeroes
// the status words (a later slice of a sliced search adds to them).
int enqueue_parts(sw_db_t db, const std::vector<Part>& parts, const std::vector<uint8_t*>& blobs,
                  const uint8_t* queries, const int32_t* sm, int32_t go, int32_t ge, const sw_options* opt,
                  void* ws, int32_t* scores, hipStream_t stream, bool from_first = true)
{
    for (size_t g = 0; g < parts.size(); ++g) {
        const bool first = g == 0, last = g + 1 == parts.size();
        const int rc = enqueue_search(db, parts[g].L, blobs[g], queries, sm, go, ge,
                                      first && opt ? opt->ev_search_begin : nullptr,
                                      last && opt ? opt->ev_search_end : nullptr,
                                      last && opt ? opt->ev_rescore_end : nullptr, ws, scores,
                                      first && from_first, stream);
        if (rc) return rc;
    }
    return SW_OK;
}

int do_search(sw_db_t db, const uint8_t* queries, const int64_t* q_offsets, const int32_t* q_lens,
              int32_t nq, const int32_t* sm, int32_t go, int32_t ge, const sw_options* opt,
              void* ws, size_t ws_bytes, int32_t* scores, hipStream_t stream)
{
    std::vector<Part> parts;
    bool nothing = false, from_first = true;
    int rc = plan_search(db, queries, q_offsets, q_lens, nq, sm, go, ge, opt, ws, ws_bytes, scores, parts, nothing,
                         &from_first);
    if (rc || nothing) return rc;
    std::vector<Staging*> st(parts.size(), nullptr);
    std::vector<uint8_t*> blobs(parts.size(), nullptr);
    for (size_t g = 0; g < parts.size(); ++g) {
        blobs[g] = static_cast<uint8_t*>(acquire_staging(db, parts[g].L.blob, &st[g]));
        if (!blobs[g]) {
            std::lock_guard<std::mutex> lk(db->mu);
            for (size_t k = 0; k < g; ++k) st[k]->state = Staging::kFree;
            return fail(SW_ENOMEM, "pinned staging allocation failed");
        }
        fill_blob(parts[g].L, parts[g].offs.data(), blobs[g]);
    }
    rc = enqueue_parts(db, parts, blobs, queries, sm, go, ge, opt, ws, scores, stream, from_first);
    // the staging buffers are reusable once the stream has passed this point
    hipError_t e = hipSuccess;
    for (size_t g = 0; g < parts.size() && e == hipSuccess; ++g)
        e = hipEventRecord(st[g]->ev, stream);
    if (rc || e != hipSuccess) {
        (void)hipStreamSynchronize(stream);
        std::lock_guard<std::mutex> lk(db->mu);
        for (Staging* x : st) x->state = Staging::kFree;
        if (!rc) rc = fail(SW_EHIP, std::string("hipEventRecord: ") + hipGetErrorString(e));
        return rc;
    }
    std::lock_guard<std::mutex> lk(db->mu);
    for (Staging* x : st) x->state = Staging::kInFlight;
    return SW_OK;
}

void free_db(sw_db_s* db)
{
    if (!db) return;
    for (auto& st : db->staging) {
        if (st.ev) {
            (void)hipEventSynchronize(st.ev);
            (void)hipEventDestroy(st.ev);
        }
        if (st.host) (void)hipHostFree(st.host);
    }
    delete db;
}

// Copies a search's status words (the start of its workspace) to the host,
// synchronises the stream and decodes them (sw_status_code).
int sw_search_status_get(const void* ws, hipStream_t stream, sw_status* st)
{
    if (!ws) return fail(SW_EINVAL, "null workspace");
    *st = sw_status{};
    HIPCHK(hipMemcpyAsync(st, ws, sizeof(sw_status), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    return sw_status_code(st);
}

// Device layout of a prepared database inside the caller's workspace
// (256-byte aligned pieces): lane-interleaved residues, chunk offsets, the
// sort permutation, sorted lengths; then two pieces used only while
// preparing (the chunk block prefix and the bad-code flag).
struct DbLayout {
    size_t res = 0, chunk_off = 0, perm = 0, slen = 0, bprefix = 0, bad = 0, total = 0, resident = 0;
};

DbLayout db_layout(int64_t res_bytes, int64_t nseq)
{
    const int64_t nchunks = ceil_div(nseq, 64);
    DbLayout L;
    size_t off = 0;
    L.res = off; off += align_up(std::max<int64_t>(res_bytes, 16), 256);
    L.chunk_off = off; off += align_up(sizeof(int64_t) * std::max<int64_t>(nchunks, 1), 256);
    L.perm = off; off += align_up(sizeof(int32_t) * std::max<int64_t>(nseq, 1), 256);
    L.slen = off; off += align_up(sizeof(int32_t) * std::max<int64_t>(nseq, 1), 256);
    L.resident = off;
    L.bprefix = off; off += align_up(sizeof(int64_t) * (nchunks + 1), 256);
    L.bad = off; off += 256;
    L.total = off;
    return L;
}

// Checks of sw_db_prepare that need no HIP call; the workspace must at least
// hold the layout's metadata (the residues are checked once the lengths are
// known).
int prepare_args_check(const int64_t* offsets, const int32_t* lengths, int32_t nseq, void* ws, size_t ws_bytes)
{
    if (nseq < 0) return fail(SW_EINVAL, "nseq < 0");
    if (nseq > 0 && (!offsets || !lengths)) return fail(SW_EINVAL, "null offsets or lengths");
    if (nseq > (INT32_MAX / 2)) return fail(SW_EINVAL, "nseq too large");
    if (!ws) return fail(SW_EINVAL, "null workspace");
    if (((uintptr_t)ws & 255) != 0) return fail(SW_EINVAL, "workspace must be 256-byte aligned");
    const size_t least = db_layout(0, nseq).total;
    if (ws_bytes < least)
        return fail(SW_ENOMEM, "database workspace too small: need at least " + std::to_string(least) + " bytes");
    return SW_OK;
}

int gfx950_device(int* dev)
{
    HIPCHK(hipGetDevice(dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, *dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SW_EUNSUP, std::string("device is ") + prop.gcnArchName);
    return SW_OK;
}

// Database preparation from host copies of the lengths and offsets: stable
// sort by length (descending), chunk layout, upload of the metadata and the
// lane interleaving on `stream`, all inside `ws`.  Blocking (reads back the
// bad-code flag).
int prepare_from_host(const uint8_t* residues, const int64_t* offsets, const std::vector<int32_t>& len,
                      const std::vector<int64_t>& off, int dev, void* ws, size_t ws_bytes, hipStream_t stream,
                      sw_db_t* out)
{
    const int32_t nseq = (int32_t)len.size();
    int64_t total = 0;
    int32_t maxl = 0;
    for (int32_t i = 0; i < nseq; ++i) {
        if (len[i] < 0) return fail(SW_EINVAL, "negative subject length");
        if (off[i] < 0) return fail(SW_EINVAL, "negative subject offset");
        total += len[i];
        maxl = std::max(maxl, len[i]);
    }
    if (total > 0 && !residues) return fail(SW_EINVAL, "null residues");

    std::vector<int32_t> perm(nseq);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return len[a] > len[b]; });
    std::vector<int32_t> slen(nseq);
    for (int32_t s = 0; s < nseq; ++s)
        slen[s] = len[perm[s]];
    const int32_t nchunks = (int32_t)ceil_div(nseq, 64);
    std::vector<int64_t> bprefix(nchunks + 1, 0), coff(std::max(nchunks, 1), 0);
    for (int32_t c = 0; c < nchunks; ++c) {
        const int64_t cols = align_up(slen[(int64_t)c * 64], 16);
        bprefix[c + 1] = bprefix[c] + cols / 16;
        coff[c] = bprefix[c] * 1024;
    }
    const int64_t res_bytes = std::max<int64_t>(bprefix[nchunks] * 1024, 16);
    const DbLayout L = db_layout(res_bytes, nseq);
    if (ws_bytes < L.total)
        return fail(SW_ENOMEM, "database workspace too small: need " + std::to_string(L.total) + " bytes");

    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    uint8_t* w = static_cast<uint8_t*>(ws);
    auto* db = new sw_db_s();
    db->device = dev;
    db->cu = prop.multiProcessorCount;
    db->lds_max = (int)std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);
    db->nseq = nseq;
    db->total = total;
    db->nchunks = nchunks;
    db->max_len = maxl;
    db->res_bytes = res_bytes;
    db->slen = slen;
    db->d_res = w + L.res;
    db->d_chunk_off = reinterpret_cast<int64_t*>(w + L.chunk_off);
    db->d_perm = reinterpret_cast<int32_t*>(w + L.perm);
    db->d_slen = reinterpret_cast<int32_t*>(w + L.slen);
    db->dev_bytes = (int64_t)L.resident;
    auto* d_bprefix = reinterpret_cast<int64_t*>(w + L.bprefix);
    auto* d_bad = reinterpret_cast<int32_t*>(w + L.bad);
    auto cleanup = [&](int code, const std::string& msg) {
        (void)hipStreamSynchronize(stream);
        free_db(db);
        return fail(code, msg);
    };
#define PCHK(x)                                                                                 \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) return cleanup(SW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)
    if (nseq > 0) {
        const int32_t zero = 0;
        PCHK(hipMemcpyAsync(db->d_chunk_off, coff.data(), sizeof(int64_t) * nchunks, hipMemcpyHostToDevice, stream));
        PCHK(hipMemcpyAsync(db->d_perm, perm.data(), sizeof(int32_t) * nseq, hipMemcpyHostToDevice, stream));
        PCHK(hipMemcpyAsync(db->d_slen, slen.data(), sizeof(int32_t) * nseq, hipMemcpyHostToDevice, stream));
        PCHK(hipMemcpyAsync(d_bprefix, bprefix.data(), sizeof(int64_t) * (nchunks + 1), hipMemcpyHostToDevice, stream));
        PCHK(hipMemcpyAsync(d_bad, &zero, sizeof(int32_t), hipMemcpyHostToDevice, stream));
        PCHK(launch_interleave(residues, offsets, db->d_perm, db->d_slen, db->d_chunk_off, nseq,
                               bprefix[nchunks] * 64, d_bprefix, nchunks, db->d_res, d_bad, stream));
        int32_t bad = 0;
        PCHK(hipMemcpyAsync(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        PCHK(hipStreamSynchronize(stream));
        if (bad)
            return cleanup(SW_EBADRES, "database residue code >= 32");
    }
#undef PCHK
    *out = db;
    return SW_OK;
}

}  // namespace

extern "C" {

const char* sw_version(void) { return "swdb 0.1.0 (gfx950)"; }

const char* sw_last_error(void) { return g_err.c_str(); }

const char* sw_strerror(int code)
{
    switch (code) {
    case SW_OK: return "ok";
    case SW_EINVAL: return "invalid argument";
    case SW_ENOMEM: return "out of memory or workspace too small";
    case SW_EHIP: return "HIP runtime error";
    case SW_EUNSUP: return "unsupported device (gfx950 required)";
    case SW_EBADRES: return "residue code >= 32";
    case SW_ERESCORE: return "exact int32 rescore incomplete";
    case SW_EINTERNAL: return "internal error";
    }
    return "unknown error";
}

int sw_db_prepare(const uint8_t* residues, const int64_t* offsets, const int32_t* lengths,
                  int32_t nseq, void* workspace, size_t ws_bytes, hipStream_t stream, sw_db_t* out)
{
    if (!out) return fail(SW_EINVAL, "null output handle");
    *out = nullptr;
    int rc = prepare_args_check(offsets, lengths, nseq, workspace, ws_bytes);
    if (rc) return rc;
    int dev = 0;
    rc = gfx950_device(&dev);
    if (rc) return rc;
    std::vector<int32_t> len(nseq);
    std::vector<int64_t> off(nseq);
    if (nseq > 0) {
        HIPCHK(hipMemcpyAsync(len.data(), lengths, sizeof(int32_t) * nseq, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipMemcpyAsync(off.data(), offsets, sizeof(int64_t) * nseq, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
    }
    return prepare_from_host(residues, offsets, len, off, dev, workspace, ws_bytes, stream, out);
}

size_t sw_db_prepare_bytes(int64_t total_residues, int32_t nseq, int32_t max_len)
{
    if (total_residues < 0 || nseq < 0 || nseq > INT32_MAX / 2 || max_len < 0) {
        fail(SW_EINVAL, "negative or out-of-range database size");
        return 0;
    }
    if ((nseq == 0 && (total_residues || max_len)) || max_len > total_residues ||
        (int64_t)nseq * max_len < total_residues) {
        fail(SW_EINVAL, "inconsistent total_residues, nseq and max_len");
        return 0;
    }
    const int64_t nchunks = ceil_div(nseq, 64);
    // Chunk c stores 64 lanes of ceil16(longest length of the chunk) bytes.
    // Lengths are sorted descending, so chunk c's longest subject (c >= 1) is
    // no longer than any subject of chunk c - 1: 64 * that length is at most
    // chunk c - 1's residues, and the sum over chunks at most
    // 64 * ceil16(max_len) + total + 960 per chunk for the rounding.
    const int64_t bound = 64 * align_up(max_len, 16) + total_residues + 960 * nchunks;
    return db_layout(bound, nseq).total;
}

int sw_db_describe(const int32_t* lengths, int32_t nseq, int32_t cu_count, int32_t lds_bytes, sw_db_t* out)
{
    if (!out) return fail(SW_EINVAL, "null output handle");
    *out = nullptr;
    if (nseq < 0 || nseq > INT32_MAX / 2) return fail(SW_EINVAL, "nseq out of range");
    if (nseq > 0 && !lengths) return fail(SW_EINVAL, "null lengths");
    if (cu_count < 0 || lds_bytes < 0) return fail(SW_EINVAL, "negative device parameter");
    std::vector<int32_t> len(lengths, lengths + nseq);
    int64_t total = 0;
    int32_t maxl = 0;
    for (int32_t v : len) {
        if (v < 0) return fail(SW_EINVAL, "negative subject length");
        total += v;
        maxl = std::max(maxl, v);
    }
    std::stable_sort(len.begin(), len.end(), [](int32_t a, int32_t b) { return a > b; });
    auto* db = new sw_db_s();
    db->host_only = true;
    db->cu = cu_count ? cu_count : 256;
    db->lds_max = lds_bytes ? std::min(lds_bytes, 160 * 1024) : 160 * 1024;
    db->nseq = nseq;
    db->total = total;
    db->nchunks = (int32_t)ceil_div(nseq, 64);
    db->max_len = maxl;
    db->slen = std::move(len);
    *out = db;
    return SW_OK;
}

int64_t sw_plan_items(sw_db_t db, int32_t nq, const int32_t* q_lens, const sw_options* opt, int32_t* out,
                      int64_t cap)
{
    int rc = validate_query_set(db, nq, q_lens);
    if (rc) return rc;
    std::string why;
    if (!validate_options(opt, why)) return fail(SW_EINVAL, why);
    if (cap > 0 && !out) return fail(SW_EINVAL, "null output");
    std::vector<Part> parts;
    rc = build_parts(db, nq, q_lens, nullptr, opt, 2, parts);
    if (rc) return rc;
    int64_t pos = 0;
    for (const Part& P : parts) {
        for (int32_t k : P.L.order) {
            for (int64_t i = P.L.ranges[k].first; i < P.L.ranges[k].second; ++i) {
                const Item& it = P.L.plans[k]->items[i];
                if (pos < cap) {
                    out[4 * pos + 0] = it.s0;
                    out[4 * pos + 1] = it.ncols;
                    out[4 * pos + 2] = P.idx[k];
                    out[4 * pos + 3] = it.meta;
                }
                ++pos;
            }
        }
    }
    return pos;
}

int sw_db_sorted_lengths(sw_db_t db, int32_t* out)
{
    if (!db) return fail(SW_EINVAL, "null database handle");
    if (db->nseq > 0 && !out) return fail(SW_EINVAL, "null output");
    std::copy(db->slen.begin(), db->slen.end(), out);
    return SW_OK;
}

int sw_db_release(sw_db_t db)
{
    if (!db) return fail(SW_EINVAL, "null database handle");
    free_db(db);
    return SW_OK;
}

int sw_db_info(sw_db_t db, int64_t* nseq, int64_t* residues, int64_t* device_bytes)
{
    if (!db) return fail(SW_EINVAL, "null database handle");
    if (nseq) *nseq = db->nseq;
    if (residues) *residues = db->total;
    if (device_bytes) *device_bytes = db->dev_bytes;
    return SW_OK;
}

size_t sw_workspace_bytes(sw_db_t db, int32_t nq, const int32_t* q_lens, const sw_options* opt)
{
    if (validate_query_set(db, nq, q_lens)) return 0;
    std::string why;
    if (!validate_options(opt, why)) { fail(SW_EINVAL, why); return 0; }
    std::vector<Part> parts;
    if (build_parts(db, nq, q_lens, nullptr, opt, 2, parts)) return 0;
    return std::max<size_t>(parts_bytes(parts), 256);
}

int sw_select_variant(const int32_t* sm, int32_t go, const sw_options* opt)
{
    if (!sm) return fail(SW_EINVAL, "null substitution matrix");
    if (go < 0 || go > SW_MAX_GAP) return fail(SW_EINVAL, "gap-open penalty must be in [0, SW_MAX_GAP]");
    std::string why;
    if (!validate_options(opt, why)) return fail(SW_EINVAL, why);
    const int fit = matrix_elem(sm, go, why);
    if (!fit) return fail(SW_EINVAL, why);
    sw_db_s probe;
    probe.host_only = true;
    probe.lds_max = 160 * 1024;
    sw_options o = opt ? *opt : sw_options{};
    if (o.mode == SW_MODE_TUNED)
        o.mode = SW_MODE_AUTO;
    const int32_t one = 1;
    return (int)resolve(&probe, &o, fit, 1, &one).v;
}

int sw_plan_info(sw_db_t db, int32_t nq, const int32_t* q_lens, const sw_options* opt, sw_plan_stats* out)
{
    int rc = validate_query_set(db, nq, q_lens);
    if (rc) return rc;
    if (!out) return fail(SW_EINVAL, "null output");
    std::string why;
    if (!validate_options(opt, why)) return fail(SW_EINVAL, why);
    std::vector<Part> parts;
    rc = build_parts(db, nq, q_lens, nullptr, opt, 2, parts);
    if (rc) return rc;
    *out = sw_plan_stats{};
    for (const Part& P : parts) {
        const Layout& L = P.L;
        out->cells += L.cells;
        out->lane_cells += L.lane_cells;
        out->items += L.nitems;
        out->launches += 1;
        out->grid = std::max<int64_t>(out->grid, L.grid);
        out->slot_bytes = std::max<int64_t>(out->slot_bytes, L.slot_elems * (int64_t)sizeof(int2));
    }
    out->workspace = (int64_t)std::max<size_t>(parts_bytes(parts), 256);
    if (!parts.empty()) {
        out->variant = (int32_t)parts[0].L.r.v;
        out->rows = parts[0].L.r.rows;
    }
    return SW_OK;
}

int sw_db_search_ex(sw_db_t db, const uint8_t* query, int32_t qlen, const int32_t* sm,
                    int32_t go, int32_t ge, const sw_options* opt, void* ws, size_t ws_bytes,
                    int32_t* scores, hipStream_t stream)
{
    const int64_t off = 0;
    return do_search(db, query, &off, &qlen, 1, sm, go, ge, opt, ws, ws_bytes, scores, stream);
}

int sw_db_search_batch(sw_db_t db, const uint8_t* queries, const int64_t* q_offsets,
                       const int32_t* q_lens, int32_t nq, const int32_t* sm, int32_t go, int32_t ge,
                       const sw_options* opt, void* ws, size_t ws_bytes, int32_t* scores,
                       hipStream_t stream)
{
    return do_search(db, queries, q_offsets, q_lens, nq, sm, go, ge, opt, ws, ws_bytes, scores, stream);
}

// One batch tuned as a unit: starting from the defaults, one choice at a
// time (arithmetic mode, waves per workgroup, the item target, the lane-group
// rule) is varied and timed on the batch itself, and a change is kept only
// when it gains more than timing noise (1%, confirmed by timing both again);
// later choices are varied around the schedule kept so far.
int sw_autotune_batch(sw_db_t db, const uint8_t* queries, const int64_t* q_offsets, const int32_t* q_lens,
                      int32_t nq, const int32_t* sm, int32_t go, int32_t ge, hipStream_t stream, sw_tune_entry* out)
{
    if (!db) return fail(SW_EINVAL, "null database handle");
    if (db->host_only) return fail(SW_EINVAL, "planning-only handle cannot search");
    if (!out || !sm || nq <= 0 || !q_lens || !q_offsets || !queries)
        return fail(SW_EINVAL, "bad batch autotune arguments");
    int rc = validate_query_set(db, nq, q_lens);
    if (rc) return rc;
    std::string why;
    if (!matrix_elem(sm, go, why)) return fail(SW_EINVAL, why);
    if (db->nseq == 0) return fail(SW_EINVAL, "empty database");
    int64_t sumq = 0;
    int32_t maxm = 0;
    for (int32_t k = 0; k < nq; ++k) {
        sumq += q_lens[k];
        maxm = std::max(maxm, q_lens[k]);
    }
    if (sumq == 0) return fail(SW_EINVAL, "batch of empty queries");

    // the variations: each entry changes one field of the schedule kept so far
    struct Var { int field, value; };    // field 0 mode, 1 waves, 2 lane_cells, 3 strict_groups
    const std::vector<std::vector<Var>> rounds = {
        {{0, SW_MODE_I32}},
        {{1, 4}, {1, 8}},
        {{2, 49152}, {2, 98304}, {2, 196608}, {2, 393216}},
        {{3, 1}},
    };
    auto apply = [](sw_options o, const Var& v) {
        if (v.field == 0) o.mode = v.value;
        if (v.field == 1) o.waves = v.value;
        if (v.field == 2) o.lane_cells = v.value;
        if (v.field == 3) o.strict_groups = v.value;
        return o;
    };
    // workspace for every schedule the search can reach
    size_t ws_need = 0;
    {
        std::vector<sw_options> all{sw_options{}};
        for (const auto& r : rounds) {
            std::vector<sw_options> more;
            for (const sw_options& o : all)
                for (const Var& v : r) more.push_back(apply(o, v));
            all.insert(all.end(), more.begin(), more.end());
        }
        for (const sw_options& o : all) {
            const size_t b = sw_workspace_bytes(db, nq, q_lens, &o);
            if (b == 0) return fail(SW_EINVAL, "workspace size of a candidate schedule");
            ws_need = std::max(ws_need, b);
        }
    }
    void* d_ws = nullptr;
    int32_t* d_sc = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto cleanup = [&]() {
        if (d_ws) (void)hipFreeAsync(d_ws, stream);
        if (d_sc) (void)hipFreeAsync(d_sc, stream);
        (void)hipStreamSynchronize(stream);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
#define TCHK(x)                                                                               \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            cleanup();                                                                        \
            return fail(SW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));             \
        }                                                                                     \
    } while (0)
    TCHK(hipMallocAsync(&d_ws, std::max<size_t>(ws_need, 256), stream));
    TCHK(hipMallocAsync((void**)&d_sc, sizeof(int32_t) * (size_t)nq * (size_t)db->nseq, stream));
    TCHK(hipEventCreate(&ev[0]));
    TCHK(hipEventCreate(&ev[1]));
    // fastest of two timed runs after one that warms the plan cache
    auto timed = [&](const sw_options& o, float& tmin) -> int {
        tmin = -1;
        for (int rep = 0; rep < 3; ++rep) {
            hipError_t e = hipEventRecord(ev[0], stream);
            if (e != hipSuccess) return fail(SW_EHIP, std::string("hipEventRecord: ") + hipGetErrorString(e));
            const int r = sw_db_search_batch(db, queries, q_offsets, q_lens, nq, sm, go, ge, &o, d_ws, ws_need,
                                             d_sc, stream);
            if (r) return r;
            e = hipEventRecord(ev[1], stream);
            sw_status st{};
            const int sr = sw_search_status(d_ws, stream, &st);      // synchronises the stream
            if (sr) return sr;
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (e != hipSuccess) return fail(SW_EHIP, std::string("batch autotune timing: ") + hipGetErrorString(e));
            if (rep > 0 && (tmin < 0 || ms < tmin)) tmin = ms;
        }
        return SW_OK;
    };
    // schedules that resolve alike (e.g. waves = 8 where the defaults already
    // pick 8) are the same launch: not timed again
    const int fit = matrix_elem(sm, go, why);
    auto same = [&](const sw_options& a, const sw_options& b) {
        const Resolved x = resolve(db, &a, fit, nq, q_lens), y = resolve(db, &b, fit, nq, q_lens);
        return x.v == y.v && x.waves == y.waves && x.target == y.target && x.strict == y.strict &&
               x.kmax == y.kmax && x.lds_limit == y.lds_limit && x.grid_limit == y.grid_limit;
    };
    sw_options best{};
    float tbest = 0;
    rc = timed(best, tbest);
    for (size_t r = 0; r < rounds.size() && rc == SW_OK; ++r) {
        const sw_options base = best;
        for (const Var& v : rounds[r]) {
            const sw_options o = apply(base, v);
            if (same(o, base) || same(o, best)) continue;
            float t = 0;
            rc = timed(o, t);
            if (rc) break;
            if (t < 0.99f * tbest) {
                // a gain is confirmed by timing both again before it is kept
                float t2 = 0, tb2 = 0;
                rc = timed(o, t2);
                if (!rc) rc = timed(best, tb2);
                if (rc) break;
                if (std::max(t, t2) < 0.99f * std::min(tbest, tb2)) {
                    tbest = std::min(t, t2);
                    best = o;
                } else {
                    tbest = std::min(tbest, tb2);
                }
            }
        }
    }
#undef TCHK
    const std::string err = g_err;
    cleanup();
    if (rc) return fail(rc, "batch autotune search: " + err);
    *out = sw_tune_entry{};
    out->qlen = maxm;
    out->opt = best;
    out->gcups = (double)sumq * (double)db->total / (tbest * 1e-3) / 1e9;
    return SW_OK;
}

int sw_tune_set(sw_db_t db, const sw_tune_entry* entries, int32_t n)
{
    if (!db) return fail(SW_EINVAL, "null database handle");
    if (n < 0 || (n > 0 && !entries)) return fail(SW_EINVAL, "bad tune table");
    std::vector<sw_tune_entry> t(entries, entries + n);
    for (auto& e : t) {
        std::string why;
        if (e.qlen < 0 || !validate_options(&e.opt, why) || e.opt.mode == SW_MODE_TUNED)
            return fail(SW_EINVAL, "bad tune entry");
        e.opt.ev_search_begin = e.opt.ev_search_end = e.opt.ev_rescore_end = nullptr;
    }
    std::stable_sort(t.begin(), t.end(), [](const sw_tune_entry& a, const sw_tune_entry& b) {
        return a.qlen < b.qlen;
    });
    std::lock_guard<std::mutex> lk(db->mu);
    db->tune = std::move(t);
    return SW_OK;
}

int32_t sw_tune_get(sw_db_t db, sw_tune_entry* out, int32_t cap)
{
    if (!db) return fail(SW_EINVAL, "null database handle");
    std::lock_guard<std::mutex> lk(db->mu);
    const int32_t n = (int32_t)db->tune.size();
    for (int32_t k = 0; k < n && k < cap && out; ++k)
        out[k] = db->tune[k];
    return n;
}

int sw_autotune(sw_db_t db, const int32_t* qlens, int32_t nbins, const int32_t* sm, int32_t go, int32_t ge,
                hipStream_t stream, sw_tune_entry* out)
{
    if (!db) return fail(SW_EINVAL, "null database handle");
    if (db->host_only) return fail(SW_EINVAL, "planning-only handle cannot search");
    if (nbins <= 0 || !qlens || !out || !sm) return fail(SW_EINVAL, "bad autotune arguments");
    std::string why;
    if (!matrix_elem(sm, go, why)) return fail(SW_EINVAL, why);
    if (go < 0 || ge < 0 || go > SW_MAX_GAP || ge > SW_MAX_GAP) return fail(SW_EINVAL, "gap penalties");
    int32_t maxm = 0;
    for (int32_t b = 0; b < nbins; ++b) {
        if (qlens[b] < 1 || qlens[b] > SW_MAX_QLEN) return fail(SW_EINVAL, "tune length out of range");
        maxm = std::max(maxm, qlens[b]);
    }
    if (db->nseq == 0) return fail(SW_EINVAL, "empty database");

    // residue composition of the database: a sample of its stored codes
    std::vector<uint8_t> sample((size_t)std::min<int64_t>(db->res_bytes, 1 << 20));
    HIPCHK(hipMemcpyAsync(sample.data(), db->d_res, sample.size(), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    std::vector<uint8_t> codes;
    for (uint8_t c : sample)
        if (c < kAlpha) codes.push_back(c);
    if (codes.empty()) codes.push_back(0);

    struct Cand { int32_t mode, waves, lane_cells; };
    std::vector<Cand> cands{{SW_MODE_AUTO, 0, 0}};    // the defaults first: the tuner never loses to them
    for (int32_t mode : {SW_MODE_I16, SW_MODE_I32})
        for (int32_t waves : {4, 8})
            for (int32_t lc : {24576, 49152, 98304, 196608})
                cands.push_back({mode, waves, lc});
    size_t ws_need = 0;
    for (int32_t b = 0; b < nbins; ++b)
        for (const Cand& c : cands) {
            sw_options o{};
            o.mode = c.mode;
            o.waves = c.waves;
            o.lane_cells = c.lane_cells;
            ws_need = std::max(ws_need, sw_workspace_bytes(db, 1, &qlens[b], &o));
        }
    uint8_t* d_q = nullptr;
    void* d_ws = nullptr;
    int32_t* d_sc = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<uint8_t> hq(maxm);
    int rc = SW_OK;
    auto cleanup = [&]() {
        if (d_q) (void)hipFreeAsync(d_q, stream);
        if (d_ws) (void)hipFreeAsync(d_ws, stream);
        if (d_sc) (void)hipFreeAsync(d_sc, stream);
        (void)hipStreamSynchronize(stream);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
#define TCHK(x)                                                                               \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            cleanup();                                                                        \
            return fail(SW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));             \
        }                                                                                     \
    } while (0)
    // the tuner's own buffers: stream-ordered allocations, freed on the stream
    TCHK(hipMallocAsync((void**)&d_q, std::max<int32_t>(maxm, 1), stream));
    TCHK(hipMallocAsync(&d_ws, std::max<size_t>(ws_need, 256), stream));
    TCHK(hipMallocAsync((void**)&d_sc, sizeof(int32_t) * db->nseq, stream));
    TCHK(hipEventCreate(&ev[0]));
    TCHK(hipEventCreate(&ev[1]));
    uint64_t x = 0x9E3779B97F4A7C15ull;              // xorshift64* draws of sample positions
    std::vector<sw_tune_entry> res(nbins);
    for (int32_t b = 0; b < nbins && rc == SW_OK; ++b) {
        const int32_t m = qlens[b];
        for (int32_t i = 0; i < m; ++i) {
            x ^= x >> 12; x ^= x << 25; x ^= x >> 27;
            hq[i] = codes[(size_t)((x * 0x2545F4914F6CDD1Dull) >> 33) % codes.size()];
        }
        TCHK(hipMemcpyAsync(d_q, hq.data(), m, hipMemcpyHostToDevice, stream));
        TCHK(hipStreamSynchronize(stream));          // hq is reused for the next bin
        float best = -1;
        sw_tune_entry be{};
        for (const Cand& c : cands) {
            sw_options o{};
            o.mode = c.mode;
            o.waves = c.waves;
            o.lane_cells = c.lane_cells;
            float tmin = -1;
            for (int rep = 0; rep < 3 && rc == SW_OK; ++rep) {     // first run warms the plan cache
                TCHK(hipEventRecord(ev[0], stream));
                rc = sw_db_search_ex(db, d_q, m, sm, go, ge, &o, d_ws, ws_need, d_sc, stream);
                TCHK(hipEventRecord(ev[1], stream));
                TCHK(hipEventSynchronize(ev[1]));
                float ms = 0;
                TCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
                if (rep > 0 && (tmin < 0 || ms < tmin)) tmin = ms;
            }
            if (rc) break;
            if (best < 0 || tmin < 0.995f * best) {    // a change must gain more than timing noise
                best = tmin;
                be.qlen = m;
                be.opt = o;
                be.gcups = (double)m * (double)db->total / (tmin * 1e-3) / 1e9;
            }
        }
        res[b] = be;
    }
#undef TCHK
    const std::string err = g_err;
    cleanup();
    if (rc) return fail(rc, "autotune search: " + err);
    for (int32_t b = 0; b < nbins; ++b)
        out[b] = res[b];
    return sw_tune_set(db, res.data(), nbins);
}

}  // extern "C"

struct sw_graph_s {
    sw_db_t db = nullptr;
    std::vector<void*> blobs;     // pinned plan copies, one per launch group
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {
void free_graph(sw_graph_s* g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    for (void* b : g->blobs) (void)hipHostFree(b);
    delete g;
}
}  // namespace

extern "C" {

int sw_graph_create(sw_db_t db, const uint8_t* queries, const int64_t* q_offsets, const int32_t* q_lens,
                    int32_t nq, const int32_t* sm, int32_t go, int32_t ge, const sw_options* opt,
                    void* ws, size_t ws_bytes, int32_t* scores, sw_graph_t* out)
{
    if (!out) return fail(SW_EINVAL, "null output graph");
    *out = nullptr;
    std::vector<Part> parts;
    bool nothing = false, from_first = true;
    int rc = plan_search(db, queries, q_offsets, q_lens, nq, sm, go, ge, opt, ws, ws_bytes, scores, parts, nothing,
                         &from_first);
    if (rc) return rc;
    auto* g = new sw_graph_s();
    g->db = db;
    auto bail = [&](int code, const std::string& msg) {
        free_graph(g);
        return fail(code, msg);
    };
    hipError_t e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(SW_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    std::vector<uint8_t*> blobs;
    for (const Part& P : parts) {
        void* b = nullptr;
        e = hipHostMalloc(&b, std::max<size_t>(P.L.blob, 16), hipHostMallocDefault);
        if (e != hipSuccess) return bail(SW_ENOMEM, "pinned plan allocation failed");
        g->blobs.push_back(b);
        fill_blob(P.L, P.offs.data(), static_cast<uint8_t*>(b));
        blobs.push_back(static_cast<uint8_t*>(b));
    }
    e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bail(SW_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    if (!nothing)
        rc = enqueue_parts(db, parts, blobs, queries, sm, go, ge, nullptr, ws, scores, g->cap, from_first);
    const std::string err = g_err;
    e = hipStreamEndCapture(g->cap, &g->graph);
    if (rc) return bail(rc, "capture: " + err);
    if (e != hipSuccess) return bail(SW_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bail(SW_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    *out = g;
    return SW_OK;
}

int sw_graph_launch(sw_graph_t g, hipStream_t stream)
{
    if (!g || !g->exec) return fail(SW_EINVAL, "null graph");
    HIPCHK(hipGraphLaunch(g->exec, stream));
    return SW_OK;
}

int sw_graph_destroy(sw_graph_t g)
{
    if (!g) return fail(SW_EINVAL, "null graph");
    free_graph(g);
    return SW_OK;
}

int sw_search_status_async(const void* ws, sw_status* out, hipStream_t stream)
{
    if (!ws) return fail(SW_EINVAL, "null workspace");
    if (!out) return fail(SW_EINVAL, "null status output");
    static_assert(sizeof(sw_status) == 4 * sizeof(int32_t), "status layout");
    HIPCHK(hipMemcpyAsync(out, ws, sizeof(sw_status), hipMemcpyDeviceToHost, stream));
    return SW_OK;
}

int sw_status_code(const sw_status* st)
{
    if (!st) return fail(SW_EINVAL, "null status");
    if (st->bad_query) return fail(SW_EBADRES, "query residue code >= 32");
    if (st->rescore_failed)
        return fail(SW_ERESCORE, std::to_string(st->rescore_failed) + " subject(s) without an exact rescore");
    if (st->bad_items)
        return fail(SW_EINTERNAL, std::to_string(st->bad_items) + " work item(s) inconsistent with the launch");
    return SW_OK;
}

int sw_search_status(const void* ws, hipStream_t stream, sw_status* out)
{
    sw_status local{};
    sw_status* st = out ? out : &local;
    return sw_search_status_get(ws, stream, st);
}

int64_t sw_flagged_count(const void* ws, hipStream_t stream)
{
    sw_status st{};
    const int rc = sw_search_status_get(ws, stream, &st);
    if (rc && rc != SW_EBADRES && rc != SW_ERESCORE && rc != SW_EINTERNAL) return rc;
    return st.flagged;
}

int sw_db_search(const uint8_t* query, int32_t qlen, const uint8_t* residues, const int64_t* offsets,
                 const int32_t* lengths, int32_t nseq, const int32_t* sm, int32_t go, int32_t ge,
                 int32_t* scores, hipStream_t stream)
{
    if (qlen < 0 || qlen > SW_MAX_QLEN) return fail(SW_EINVAL, "qlen out of range");
    if (qlen > 0 && !query) return fail(SW_EINVAL, "null query");
    if (!sm) return fail(SW_EINVAL, "null substitution matrix");
    if (go < 0 || ge < 0 || go > SW_MAX_GAP || ge > SW_MAX_GAP)
        return fail(SW_EINVAL, "gap penalties must be in [0, SW_MAX_GAP]");
    if (nseq < 0) return fail(SW_EINVAL, "nseq < 0");
    if (nseq > 0 && !scores) return fail(SW_EINVAL, "null scores_out");
    if (nseq > 0 && (!offsets || !lengths)) return fail(SW_EINVAL, "null offsets or lengths");
    if (nseq > (INT32_MAX / 2)) return fail(SW_EINVAL, "nseq too large");
    std::string why;
    if (!matrix_elem(sm, go, why)) return fail(SW_EINVAL, why);
    if (nseq == 0) return SW_OK;
    int dev = 0;
    int rc = gfx950_device(&dev);
    if (rc) return rc;
    std::vector<int32_t> len(nseq);
    std::vector<int64_t> off(nseq);
    HIPCHK(hipMemcpyAsync(len.data(), lengths, sizeof(int32_t) * nseq, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipMemcpyAsync(off.data(), offsets, sizeof(int64_t) * nseq, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    int64_t total = 0;
    int32_t maxl = 0;
    for (int32_t v : len) {
        if (v < 0) return fail(SW_EINVAL, "negative subject length");
        total += v;
        maxl = std::max(maxl, v);
    }
    // the one-shot call's own memory: stream-ordered allocations, freed on
    // the stream before the call returns
    const size_t dbb = sw_db_prepare_bytes(total, nseq, maxl);
    void* dbw = nullptr;
    if (dbb == 0 || hipMallocAsync(&dbw, dbb, stream) != hipSuccess)
        return fail(SW_ENOMEM, "database allocation failed");
    sw_db_t db = nullptr;
    rc = prepare_from_host(residues, offsets, len, off, dev, dbw, dbb, stream, &db);
    if (rc) {
        const std::string err = g_err;
        (void)hipFreeAsync(dbw, stream);
        (void)hipStreamSynchronize(stream);
        return fail(rc, err);
    }
    const size_t need = sw_workspace_bytes(db, 1, &qlen, nullptr);
    void* ws = nullptr;
    if (need == 0 || hipMallocAsync(&ws, need, stream) != hipSuccess) {
        sw_db_release(db);
        (void)hipFreeAsync(dbw, stream);
        (void)hipStreamSynchronize(stream);
        return fail(SW_ENOMEM, "workspace allocation failed");
    }
    rc = sw_db_search_ex(db, query, qlen, sm, go, ge, nullptr, ws, need, scores, stream);
    sw_status st{};
    const int src = rc ? rc : sw_search_status_get(ws, stream, &st);   // synchronises the stream
    const std::string err = g_err;
    (void)hipFreeAsync(ws, stream);
    (void)hipFreeAsync(dbw, stream);
    const hipError_t e = hipStreamSynchronize(stream);
    sw_db_release(db);
    if (src) return fail(src, err);
    if (e != hipSuccess) return fail(SW_EHIP, std::string("search: ") + hipGetErrorString(e));
    return SW_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ single long pair

namespace {

// Schedule of one pair: R query rows per lane, K lanes per band (K*R query
// rows), wc columns per chunk.  The score pass runs skewed tiles: lane g of
// band b covers, in chunk c, columns [c*wc - b*kr - g, +wc) with kr = K
// rounded up to 16, so band b's chunks run from floor(b*kr / wc) (the first
// with a column >= 0 for its head) to ceil((n + b*kr + K - 1) / wc) - 1 (the
// last whose tail starts below n), and tile (b, c) is launched with
// anti-diagonal b + c.  Time model (fitted to MI355X measurements of this
// pass on DNA pairs of 162K x 172K to 7M x 5M cells, 8 and 16 rows, lane
// groups of 16 to 64, chunks of 64 to 4096 columns, and smaller pairs down to
// 3,000 x 3,500; within 5% RMS on those): anti-diagonal launches in order,
// each lasting its busiest SIMD's time plus a dispatch cost per wave.  A step (one column for every lane of a tile) costs
// a wave alone on its SIMD a latency-bound time, about 1.2x its VALU issue
// time plus a share per lane group (boundary loads and stores); k waves
// sharing a SIMD cost k times their issue time, 8.3% more per wave beyond
// three (their profile and boundary lines no longer fit the caches), or the
// latency-bound time if that is longer.  The candidate with the least total
// wins.
struct PairPlanC {
    int R = 0, K = 0, wc = 0;
    int64_t nb = 0, nc = 0, nbr = 0;
    double est_s = 0;
    bool flow = false;          // one pipelined launch (wc, nc unused)
    int waves = 0;              // flow: wavefronts of the launch (grid x wpg)
    int wpg = 0, grid = 0, lds = 0;   // flow: waves per workgroup, workgroups, LDS per workgroup
};

constexpr int64_t kPairMaxCols = 1 << 20;
constexpr double kPairLaunchS = 2e-6;       // fixed cost of a launch
constexpr double kPairWaveS = 1.17e-8;      // dispatch cost per wave of a launch
constexpr double kPairIssueCycles = 4.60;   // per VALU instruction of a wave sharing its SIMD
constexpr double kPairGroupCycles = 41.9;   // per lane group of a wave and step
constexpr double kPairCacheSlope = 0.083;   // per wave on a SIMD beyond three

struct SkewGrid {
    int64_t nb = 0, n = 0, K = 1, kr = 16, wc = 16;
    int64_t c_lo(int64_t b) const { return b * kr / wc; }
    int64_t c_hi(int64_t b) const { return ceil_div(n + b * kr + K - 1, wc) - 1; }
    int64_t diagonals() const { return nb > 0 ? nb + c_hi(nb - 1) : 0; }
};

SkewGrid skew_grid(int64_t m, int64_t n, int R, int K, int wc)
{
    SkewGrid G;
    G.nb = ceil_div(std::max<int64_t>(m, 1), (int64_t)K * R);
    G.n = std::max<int64_t>(n, 1);
    G.K = K;
    G.kr = align_up(K, 16);
    G.wc = wc;
    return G;
}

// f(d, first band, tiles) for every anti-diagonal holding tiles: bands b with
// b + c_lo(b) <= d <= b + c_hi(b), a contiguous range since both bounds grow
// with b.
template <class F>
void skew_walk(const SkewGrid& G, F&& f)
{
    int64_t lo = 0, hi = -1;
    const int64_t D = G.diagonals();
    for (int64_t d = 0; d < D; ++d) {
        while (lo < G.nb && lo + G.c_hi(lo) < d) ++lo;
        while (hi + 1 < G.nb && hi + 1 + G.c_lo(hi + 1) <= d) ++hi;
        if (hi >= lo) f(d, lo, hi - lo + 1);
    }
}

// hot-loop VALU instructions per cell of the pair kernel by rows per lane
// (counted in the gfx950 assembly of this code)
double pair_instr_per_cell(int R)
{
    return R == 8 ? 9.80 : 8.91;
}

// cycles of one step of a wave alone on its SIMD, lane groups aside
double pair_latency_cycles(int R)
{
    return R == 8 ? 386.0 : 627.0;
}

double pair_time(int64_t m, int64_t n, int R, int K, int wc, int cu)
{
    const SkewGrid G = skew_grid(m, n, R, K, wc);
    const double per_wave = (double)(kWave / K);
    const double simds = 4.0 * std::max(cu, 1);
    const double valu = pair_instr_per_cell(R) * R;               // per lane and step
    const double lat = pair_latency_cycles(R) + kPairGroupCycles * per_wave;
    double t = 0;
    skew_walk(G, [&](int64_t, int64_t, int64_t tiles) {
        const double waves = std::ceil((double)tiles / per_wave);
        const double k = std::ceil(waves / simds);
        const double issue = k * kPairIssueCycles * valu * (1.0 + kPairCacheSlope * std::max(0.0, k - 3.0));
        t += (double)wc * std::max(lat, issue) / 2.4e9 + waves * kPairWaveS + kPairLaunchS;
    });
    return t;
}

// The passes of an alignment that write direction codes or checkpoints run
// rectangular tiles (lane g of a tile on column step - g, K - 1 steps of
// pipeline fill): their chunk width is chosen with the model fitted to those
// tiles on MI355X (launches of 4 us; a wave's VALU time, 1.45x alone on its
// SIMD, 1.25x with 1.5 to 3 waves, 0.28x more per wave beyond; 10.8 VALU per
// cell with 8 rows per lane).
double pair_time_rect(int64_t m, int64_t n, int R, int K, int wc, int cu)
{
    const int64_t nb = ceil_div(std::max<int64_t>(m, 1), (int64_t)K * R);
    const int64_t nc = ceil_div(std::max<int64_t>(n, 1), wc);
    const double per_wave = (double)(kWave / K);
    const double simds = 4.0 * std::max(cu, 1);
    const double wave_s = R * (double)align_up(wc + K - 1, 4) * (R == 8 ? 10.8 : 9.66) * 4.0 / 2.4e9;
    auto slowdown = [](double w) {
        if (w <= 1.0) return 1.45;
        if (w <= 1.5) return 1.45 - 0.4 * (w - 1.0);
        if (w <= 3.0) return 1.25;
        return 1.25 + 0.28 * (w - 3.0);
    };
    // anti-diagonal d holds min(d + 1, lo, nb + nc - 1 - d) tiles: two ramps of
    // 1..lo-1 tiles and max(nb, nc) - lo + 1 diagonals of lo tiles
    const int64_t lo = std::min(nb, nc), hi = std::max(nb, nc);
    auto launch = [&](int64_t tiles) {
        const double w = std::ceil(tiles / per_wave) / simds;
        return std::ceil(w) * wave_s * slowdown(w);
    };
    double t = (double)(hi - lo + 1) * launch(lo);
    for (int64_t tiles = 1; tiles < lo; ++tiles)
        t += 2 * launch(tiles);
    return t + (double)(nb + nc - 1) * 4e-6;
}

// Pipelined pass: bands of 64 lanes x R rows on workgroups of W waves, one
// workgroup per CU (W / 4 waves per SIMD, so no SIMD carries more than the
// others: the bands advance at the pace of the slowest).  Fitted to MI355X
// (DNA pairs of every R, one band at n = 100K and 200K for the step, 256 and
// 1,000 bands for the lag and the sharing, refitted on the paper's five pairs
// at 4, 10 and 16 rows): a wave alone on its SIMD takes 46.8 + 4.04 cycles
// per VALU instruction of a step with a tag check per step (it issues one
// instruction at a time, the few scalar and memory ones of a step included
// in the constant), 4.0 with one check per 16-step block; k >= 2 waves
// sharing a SIMD issue-bound, k x 4.6 cycles per VALU instruction; each band
// starts about 127 - 1.55 R steps (per-step checks) or 156 - 1.2 R steps
// (block checks, whose waits leave more slack) after the band above (the
// last lane's 63-column lag, the 16-step read-ahead and the latency of the
// handoff words through memory).  Waves sharing a CU
// step 1.33 - 0.012 R times slower than a wave alone (1.10 with one wave per
// CU), so up to one band per CU the workgroups hold one wave each.  Bands run
// in rounds when they outnumber the waves; a round's band starts when its
// wave is free and the band above is far enough ahead.
constexpr double kFlowLaunchS = 15e-6;       // clear, launch and finish kernels
constexpr int64_t kFlowMaxBands = (1 << 16) - 1;
constexpr int64_t kFlowMaxValue = (1 << 24) - 1;
constexpr uint64_t kFlowTimeoutTicks = 200000000;   // a wait's limit: 2 s of the 100 MHz real-time counter
constexpr int kFlowGroupLds = 96 * 1024;     // LDS a workgroup asks for at least: over half a CU's

// VALU instructions of one step (the counted hot loop of the kernel, a band
// with a band above it: 7.5 per row, and 21.25 per column with a tag check
// per step or 20 with one per block)
double flow_instr_per_step(int R) { return 7.5 * R + (R >= kFlowBlockwiseRows ? 20.0 : 21.25); }

int64_t flow_bands(int64_t m, int R) { return ceil_div(ceil_div(std::max<int64_t>(m, 1), R), kWave); }

// Cycles of one step of a band with R rows on workgroups of wpg waves.
double flow_step_cycles(int R, int wpg)
{
    const double k = std::ceil(wpg / 4.0);
    const double busy = wpg > 1 ? 1.33 - 0.012 * R : 1.10;
    const double alone = R >= kFlowBlockwiseRows ? 4.0 * flow_instr_per_step(R)
                                                 : 46.8 + 4.04 * flow_instr_per_step(R);
    return busy * (k > 1 ? std::max(alone, k * kPairIssueCycles * flow_instr_per_step(R)) : alone);
}

// Waves per workgroup the kernel is built for: 16 (128 registers) up to 6
// rows per lane, 8 (256 registers) beyond.
int flow_max_wpg(int R) { return R <= 6 ? 16 : 8; }

struct FlowShape {
    int wpg = 0, grid = 0, lds = 0;
    double est_s = 1e300;
};

// The cheapest workgroup shape for R rows: W in 1, 2, 4, ..., as far as the
// registers and the LDS (W band profiles within `lds_max`) allow; the grid
// is at most one workgroup per CU (or grid_limit).
FlowShape flow_shape(int64_t m, int64_t n, int R, int elem, int cu, int lds_max, int grid_limit, int fix_wpg = 0)
{
    FlowShape best;
    const int64_t nb = flow_bands(m, R);
    const int cap = std::min(lds_max, kLdsPerCU);
    for (int wpg = 1; wpg <= flow_max_wpg(R) && flow_group_lds(R, elem, wpg) <= cap; wpg *= 2) {
        if (fix_wpg && wpg != fix_wpg) continue;
        // two-wave workgroups of 4 rows per lane measured 1.3 to 1.5 times
        // slower per step than four-wave ones (both waves on one SIMD): not
        // a planner choice
        if (!fix_wpg && wpg == 2) continue;
        int64_t grid = std::min<int64_t>(ceil_div(nb, wpg), std::max(cu, 1));
        if (grid_limit > 0) grid = std::min<int64_t>(grid, grid_limit);
        const int64_t G = grid * wpg;
        const double rounds = std::ceil((double)nb / (double)G);
        const double step = flow_step_cycles(R, wpg);
        const double lag = R >= kFlowBlockwiseRows ? 156.0 - 1.2 * R : 127.0 - 1.55 * R;
        const double steps = std::max(rounds * (double)(n + kWave - 1) + (double)G * lag,
                                      (double)nb * lag + (double)(n + kWave - 1));
        const double t = steps * step / 2.4e9 + kFlowLaunchS;
        if (t < best.est_s) {
            best.wpg = wpg;
            best.grid = (int)grid;
            best.lds = std::max(flow_group_lds(R, elem, wpg), std::min(cap, kFlowGroupLds));
            best.est_s = t;
        }
    }
    return best;
}

// Whether the pipelined pass can score the pair: its handoff words hold
// values below 2^24 (every H and F + Go is at most the largest score, at most
// max(SM, 0) x min(m, n)) and tags for at most 2^16 - 1 bands.
bool flow_fits(int64_t m, int64_t n, int R, int sm_max)
{
    if (m <= 0 || n <= 0) return false;
    const int64_t bound = (int64_t)std::max(sm_max, 0) * std::min(m, n);
    return bound <= kFlowMaxValue && flow_bands(m, R) <= kFlowMaxBands;
}

PairPlanC pair_plan_search(int64_t m, int64_t n, int cu, int fixR, int fixK, int fixW, bool rect)
{
    auto model = [&](int R, int K, int wc) {
        return rect ? pair_time_rect(m, n, R, K, wc, cu) : pair_time(m, n, R, K, wc, cu);
    };
    PairPlanC best;
    best.est_s = 1e300;
    for (int R : kPairRowChoices) {
        if (fixR && R != fixR) continue;
        // lane groups below a quarter of the query's row blocks (or of 64)
        // only add launches and boundary traffic
        int kmin = 1;
        while (kmin < 16 && 4 * kmin < ceil_div(m, R)) kmin *= 2;
        for (int K : {1, 2, 4, 8, 16, 32, 64}) {
            if (fixK ? K != fixK : K < kmin) continue;
            for (int wc : {64, 128, 256, 512, 1024, 2048, 4096, 8192}) {
                if (fixW && wc != fixW) continue;
                const double t = model(R, K, wc);
                if (t < best.est_s) {
                    best.est_s = t;
                    best.R = R;
                    best.K = K;
                    best.wc = wc;
                }
            }
        }
    }
    if (fixW && !best.wc) {        // an explicit width outside the candidate list
        best.wc = fixW;
        best.R = fixR ? fixR : 16;
        best.K = fixK ? fixK : 64;
        best.est_s = model(best.R, best.K, best.wc);
    }
    best.nb = ceil_div(std::max<int64_t>(m, 1), (int64_t)best.K * best.R);
    best.nc = ceil_div(std::max<int64_t>(n, 1), best.wc);
    best.nbr = ceil_div(m, best.R);
    return best;
}

// The planner evaluates every candidate over its anti-diagonals (a few
// milliseconds for the largest pairs); the last plans are kept, since callers
// often repeat one pair size.  rect: plan for the rectangular tiles of an
// alignment's code and checkpoint passes.
PairPlanC pair_plan(int64_t m, int64_t n, int cu, const sw_options* opt, bool rect = false, int sm_max = 127,
                    int elem = 2, int lds_max = kLdsPerCU)
{
    struct Entry {
        int64_t m = -1, n = -1;
        int cu = 0, R = 0, K = 0, W = 0, mode = 0, sm = 0, grid = 0, elem = 0, lds = 0, gw = 0;
        bool rect = false;
        PairPlanC p;
    };
    static std::mutex mu;
    static Entry cache[8];
    static int next = 0;
    const int fixR = opt ? opt->pair_rows : 0;
    const int fixK = opt ? opt->max_lanes : 0;
    const int fixW = opt ? opt->pair_cols : 0;
    const int mode = rect ? 1 : (opt ? opt->pair_mode : 0);
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const Entry& e : cache)
            if (e.m == m && e.n == n && e.cu == cu && e.R == fixR && e.K == fixK && e.W == fixW && e.rect == rect &&
                e.mode == mode && e.sm == sm_max && e.grid == (opt ? opt->grid_limit : 0) && e.elem == elem &&
                e.lds == lds_max && e.gw == (opt ? opt->pair_group_waves : 0))
                return e.p;
    }
    PairPlanC p;
    // row counts only the pipelined pass has leave the tiles free (with none
    // of theirs the search would find no candidate)
    if (mode != 2 || m <= 0 || n <= 0)          // an empty pair has nothing to pipeline
        p = pair_plan_search(m, n, cu, fixR == 8 || fixR == 16 ? fixR : 0, fixK, fixW, rect);
    else
        p.est_s = 1e300;
    // the pipelined pass, where the scores fit its words (and no tile knob is set)
    if (mode != 1 && !(mode == 0 && (fixK || fixW))) {
        for (int R : kFlowRowChoices) {
            if ((fixR && R != fixR) || !flow_fits(m, n, R, sm_max)) continue;
            const FlowShape sh = flow_shape(m, n, R, elem, cu, lds_max, opt ? opt->grid_limit : 0,
                                            opt ? opt->pair_group_waves : 0);
            if (sh.wpg > 0 && sh.est_s < p.est_s) {
                PairPlanC f;
                f.flow = true;
                f.R = R;
                f.K = kWave;
                f.nbr = ceil_div(m, R);
                f.nb = flow_bands(m, R);
                f.wpg = sh.wpg;
                f.grid = sh.grid;
                f.lds = sh.lds;
                f.waves = sh.grid * sh.wpg;
                f.est_s = sh.est_s;
                p = f;
            }
        }
    }
    std::lock_guard<std::mutex> lk(mu);
    cache[next] = Entry{m, n, cu, fixR, fixK, fixW, mode, sm_max, opt ? opt->grid_limit : 0, elem, lds_max,
                        opt ? opt->pair_group_waves : 0, rect, p};
    next = (next + 1) % 8;
    return p;
}

// Workspace of a pair, sized for every schedule (so the size does not depend
// on the device or the matrix): padded subject, 16-bit profile, rowbuf,
// colbuf, carry, store sinks, corners and the profile descriptor.  The columns of
// rowbuf and the padded subject cover both tilings: rectangular tiles reach
// nc * wc < n + wc, skewed ones n + K - 1 + wc.
struct PairLayout {
    size_t subj = 0, prof = 0, rowbuf = 0, colbuf = 0, carry = 0, sink = 0, corner = 0, qd = 0, qoff = 0,
           flow = 0, flow_status = 0, total = 0;
    int64_t n_pad = 0;
};

PairLayout pair_layout(int64_t m, int64_t n, const PairPlanC* p, int64_t wc_max)
{
    PairLayout L;
    // without a plan: the bound over every schedule (chunk width up to wc_max)
    const int64_t wc = p ? p->wc : wc_max;
    const int64_t cols = align_up(n, 16) + 2 * wc + 128;
    int64_t prof = 0, rows_pad = 0, blocks = 0;
    for (int R : kPairRowChoices) {
        if (p && (p->flow || R != p->R)) continue;
        prof = std::max(prof, prof_bytes_for((int)ceil_div(m, R), R, 2));
        rows_pad = std::max<int64_t>(rows_pad, align_up(m, R) + (int64_t)kWave * R);
        blocks = std::max(blocks, ceil_div(m, R));
    }
    for (int R : kFlowRowChoices)
        if (!p || (p->flow && R == p->R))
            prof = std::max(prof, prof_bytes_for((int)ceil_div(m, R), R, 2));
    L.n_pad = cols + 128;
    size_t off = 0;
    L.qd = off; off += 256;
    L.qoff = off; off += 256;
    L.corner = off; off += align_up((blocks + 2) * 3 * 4, 256);
    L.subj = off; off += align_up(L.n_pad, 256);
    L.prof = off; off += align_up(prof, 256);
    L.rowbuf = off; off += align_up(cols * (int64_t)sizeof(int2), 256);
    L.colbuf = off; off += align_up(rows_pad * (int64_t)sizeof(int2), 256);
    L.carry = off; off += align_up((blocks + kWave) * (int64_t)sizeof(int4), 256);
    L.sink = off; off += align_up((blocks + kWave) * 64, 256);     // a launch has at most nb + 3 waves
    L.flow = off; off += align_up((n + 16) * 8, 256);              // pipelined pass: handoff words
    L.flow_status = off; off += 256;
    L.total = off;
    return L;
}

// The generic bound's widest chunk: every planner choice (at most 8192), or
// an explicit width.
int64_t pair_wc_max(const sw_options* opt)
{
    return std::max<int64_t>(8192, opt ? opt->pair_cols : 0);
}

int validate_pair(int64_t m, int64_t n, const sw_options* opt, std::string& why)
{
    if (m < 0 || n < 0 || m > SW_MAX_QLEN || n > SW_MAX_QLEN) { why = "pair lengths must be in [0, SW_MAX_QLEN]"; return 0; }
    if (!validate_options(opt, why)) return 0;
    if (opt && opt->max_lanes && (opt->max_lanes & (opt->max_lanes - 1))) {
        why = "options.max_lanes must be a power of two for pairs";
        return 0;
    }
    if (opt && opt->pair_cols && (opt->pair_cols % 16 || opt->pair_cols > kPairMaxCols)) {
        why = "options.pair_cols must be a multiple of 16, at most 2^20";
        return 0;
    }
    const int mode = opt ? opt->pair_mode : 0;
    if (mode < 0 || mode > 2) { why = "options.pair_mode must be 0, 1 or 2"; return 0; }
    if (opt && (opt->pair_sm_max < 0 || opt->pair_sm_max > 127)) { why = "options.pair_sm_max must be 0..127"; return 0; }
    if (opt && opt->pair_group_waves &&
        (opt->pair_group_waves < 0 || opt->pair_group_waves > 16 || (opt->pair_group_waves & (opt->pair_group_waves - 1)))) {
        why = "options.pair_group_waves must be 0, 1, 2, 4, 8 or 16";
        return 0;
    }
    if (opt && (opt->pair_entry_bytes < 0 || opt->pair_entry_bytes > 2)) {
        why = "options.pair_entry_bytes must be 0, 1 or 2";
        return 0;
    }
    if (opt && opt->pair_rows) {
        bool ok = false;
        if (mode == 2) {
            for (int R : kFlowRowChoices) ok = ok || opt->pair_rows == R;
        } else {
            ok = opt->pair_rows == 8 || opt->pair_rows == 16;
        }
        if (!ok) {
            why = mode == 2 ? "options.pair_rows must be 0, 4, 6, 8, 10, 12 or 16 for the pipelined pass"
                            : "options.pair_rows must be 0, 8 or 16";
            return 0;
        }
    }
    return 1;
}

}  // namespace

extern "C" {

size_t sw_pair_workspace_bytes(int64_t m, int64_t n, const sw_options* opt)
{
    std::string why;
    if (!validate_pair(m, n, opt, why)) { fail(SW_EINVAL, why); return 0; }
    // every buffer of the chosen schedule's layout is at most its generic
    // bound: its chunk width is at most pair_wc_max
    return pair_layout(m, n, nullptr, pair_wc_max(opt)).total;
}

int sw_pair_plan(int64_t m, int64_t n, const sw_options* opt, int32_t cu_count, sw_pair_stats* out)
{
    std::string why;
    if (!validate_pair(m, n, opt, why)) return fail(SW_EINVAL, why);
    if (!out) return fail(SW_EINVAL, "null output");
    const int sm_max = (opt && opt->pair_sm_max) ? opt->pair_sm_max : 127;
    const int elem = (opt && opt->pair_entry_bytes) ? opt->pair_entry_bytes : 2;
    const PairPlanC p = pair_plan(m, n, cu_count > 0 ? cu_count : 256, opt, false, sm_max, elem);
    if (!p.R) return fail(SW_EINVAL, "the pipelined pass cannot hold this pair's scores (max(SM) x min(m, n) >= 2^24)");
    *out = sw_pair_stats{};
    out->rows = p.R;
    out->lanes = p.K;
    out->cols = p.wc;
    out->flow = p.flow ? 1 : 0;
    out->bands = p.nb;
    out->chunks = p.nc;
    int64_t launches = 0;
    if (p.flow)
        launches = (m > 0 && n > 0) ? 1 : 0;
    else if (m > 0 && n > 0)
        skew_walk(skew_grid(m, n, p.R, p.K, p.wc), [&](int64_t, int64_t, int64_t) { ++launches; });
    out->launches = launches;
    out->groups = p.grid;
    out->group_waves = p.wpg;
    out->est_ms = p.est_s * 1e3;
    out->workspace = (int64_t)sw_pair_workspace_bytes(m, n, opt);
    return SW_OK;
}

}  // extern "C"

namespace {

int pair_args_check(const uint8_t* query, int64_t m, const uint8_t* subject, int64_t n, const int32_t* sm,
                    int32_t go, int32_t ge, const sw_options* opt, void* ws, int& fit)
{
    std::string why;
    if (!validate_pair(m, n, opt, why)) return fail(SW_EINVAL, why);
    if (m > 0 && !query) return fail(SW_EINVAL, "null query");
    if (n > 0 && !subject) return fail(SW_EINVAL, "null subject");
    if (!sm) return fail(SW_EINVAL, "null substitution matrix");
    if (go < 0 || ge < 0 || go > SW_MAX_GAP || ge > SW_MAX_GAP)
        return fail(SW_EINVAL, "gap penalties must be in [0, SW_MAX_GAP]");
    fit = matrix_elem(sm, go, why);
    if (!fit) return fail(SW_EINVAL, why);
    if (!ws) return fail(SW_EINVAL, "null workspace");
    if (((uintptr_t)ws & 255) != 0) return fail(SW_EINVAL, "workspace must be 256-byte aligned");
    return SW_OK;
}

int device_cu(int* cu)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(cu, hipDeviceAttributeMultiprocessorCount, dev));
    return SW_OK;
}

// LDS bytes a workgroup may ask for on the current device.
int device_lds(int* lds)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    return SW_OK;
}

// Buffers and arguments shared by every pass over a pair: padded subject,
// cleared score, the query's profile.  `empty` is set (and nothing but the
// cleared score enqueued) when either sequence is empty.
int pair_setup(const PairPlanC& p, const PairLayout& L, uint8_t* w, const uint8_t* query, int64_t m,
               const uint8_t* subject, int64_t n, const int32_t* sm, int32_t go, int32_t ge, int elem,
               int32_t* score_out, hipStream_t stream, PairArgs& a, bool& empty)
{
    QueryDesc qd{};
    qd.prof_off = 0;
    qd.m = (int32_t)m;
    qd.nbr = (int32_t)p.nbr;
    qd.prof_bytes = (int32_t)std::min<int64_t>(prof_bytes_for((int)p.nbr, p.R, elem), INT32_MAX);
    auto* qd_dev = reinterpret_cast<QueryDesc*>(w + L.qd);
    auto* qoff_dev = reinterpret_cast<int64_t*>(w + L.qoff);
    HIPCHK(launch_pair_prep(subject, n, (m > 0 && n > 0) ? L.n_pad : 0, w + L.subj, score_out, qd, qd_dev,
                            qoff_dev, stream));
    empty = m == 0 || n == 0;
    if (empty)
        return SW_OK;      // score 0, written by the preparation kernel

    ProfileArgs pa{};
    pa.queries = query;
    pa.q_off = qoff_dev;
    pa.qd = qd_dev;
    pa.prof = w + L.prof;
    pa.bad = nullptr;          // a pair reads residue codes modulo 32
    pa.nq = 1;
    pa.go = go;
    pa.pad = elem == 1 ? -128 : -32768;
    for (int i = 0; i < kAlpha * kAlpha; ++i)
        pa.sm.v[i] = (int8_t)sm[i];
    HIPCHK(launch_profile(pa, p.R, elem, (int)std::min<int64_t>((p.nbr + 1) * kCodes * p.R, INT32_MAX), stream));

    a = PairArgs{};
    a.subj = w + L.subj;
    a.prof = w + L.prof;
    a.rowbuf = reinterpret_cast<int2*>(w + L.rowbuf);
    a.colbuf = reinterpret_cast<int2*>(w + L.colbuf);
    a.corner = reinterpret_cast<int32_t*>(w + L.corner);
    a.score = score_out;
    a.nbr = (int32_t)p.nbr;
    a.nb = (int32_t)p.nb;
    a.nc = (int32_t)p.nc;
    a.K = p.K;
    a.wc = p.wc;
    a.go = go;
    a.ge = ge;
    a.dir_stride = p.nb * p.K;
    a.m = m;
    a.n = n;
    a.kr = align_up(p.K, 16);
    a.carry = reinterpret_cast<int4*>(w + L.carry);
    a.n_pad = L.n_pad;
    a.sink = w + L.sink;
    return SW_OK;
}

enum class PairPass { kScoreCkpt, kTrace };

// A pass over skewed tiles: the anti-diagonals in order; the plain score pass
// or (trace) the direction-code pass of whole-matrix codes.
int pair_skew_diagonals(PairArgs a, const PairPlanC& p, int elem, hipStream_t stream, bool trace = false)
{
    hipError_t e = hipSuccess;
    skew_walk(skew_grid(a.m, a.n, p.R, p.K, p.wc), [&](int64_t d, int64_t b_lo, int64_t tiles) {
        if (e != hipSuccess) return;
        a.d = (int32_t)d;
        a.b_lo = (int32_t)b_lo;
        a.ntiles = (int32_t)tiles;
        e = trace ? launch_trace_skew(a, elem, stream) : launch_pair_skew(a, p.R, elem, stream);
    });
    HIPCHK(e);
    return SW_OK;
}

// The anti-diagonal launches of one pass over bands [b0, b1] x chunks [c0, c1]
// of the tile grid, in order on the stream.
int pair_diagonals(PairArgs a, PairPass kind, int R, int elem, int64_t b0, int64_t b1, int64_t c0, int64_t c1,
                   hipStream_t stream)
{
    const int64_t nbb = b1 - b0 + 1, ncc = c1 - c0 + 1;
    for (int64_t dr = 0; dr < nbb + ncc - 1; ++dr) {
        const int64_t lo = b0 + std::max<int64_t>(0, dr - (ncc - 1));
        const int64_t hi = b0 + std::min<int64_t>(dr, nbb - 1);
        a.d = (int32_t)(dr + b0 + c0);
        a.b_lo = (int32_t)lo;
        a.ntiles = (int32_t)(hi - lo + 1);
        if (kind == PairPass::kScoreCkpt)
            HIPCHK(launch_pair_diag_ckpt(a, elem, stream));
        else
            HIPCHK(launch_trace_diag(a, elem, stream));
    }
    return SW_OK;
}

// The pipelined pass of plan p over the pair set up in `a` (layout L): the
// score into `score`, or with `dir` the direction-code pass (8 rows per
// lane, dir_stride row blocks per column) and the end key; -1 into `score`
// if a wait gave up.
int flow_enqueue(const PairPlanC& p, const PairLayout& L, uint8_t* w, const PairArgs& a, int64_t n, int32_t go,
                 int32_t ge, int elem, int32_t* score, uint32_t* dir, unsigned long long* end_key, int64_t dir_stride,
                 int64_t m, hipStream_t stream)
{
    FlowArgs f{};
    f.subj = a.subj;
    f.prof = a.prof;
    f.rows = reinterpret_cast<unsigned long long*>(w + L.flow);
    f.score = score;
    f.status = reinterpret_cast<int32_t*>(w + L.flow_status);
    f.n = (int32_t)n;
    f.n_pad = (int32_t)L.n_pad;
    f.nbr = (int32_t)p.nbr;
    f.nb = (int32_t)p.nb;
    f.waves = p.waves;
    f.go = go;
    f.ge = ge;
    f.timeout = kFlowTimeoutTicks;
    f.dir = dir;
    f.end_key = end_key;
    f.dir_stride = dir_stride;
    f.m = m;
    // every band's wave must be resident at once (a band waits for the
    // band above, which may run on any other wave)
    int cu = 0;
    int rc = device_cu(&cu);
    if (rc) return rc;
    const int occ = flow_occupancy(p.R, elem, p.wpg, p.lds, dir != nullptr);
    if (occ < 1 || p.grid > occ * cu)
        return fail(SW_EHIP, "pipelined pass: " + std::to_string(p.grid) + " workgroups of " +
                                 std::to_string(p.wpg) + " waves do not fit the device at once");
    HIPCHK(launch_pair_flow(f, p.R, elem, p.wpg, p.grid, p.lds, stream));
    return SW_OK;
}

// Everything one pass over a pair enqueues: setup, then the anti-diagonal
// launches (score pass), and for an alignment with direction codes for the
// whole matrix a second pass of the same tiles writing the codes and the end key.
int pair_enqueue(const PairPlanC& p, const PairLayout& L, uint8_t* w, const uint8_t* query, int64_t m,
                 const uint8_t* subject, int64_t n, const int32_t* sm, int32_t go, int32_t ge, int elem,
                 int32_t* score_out, uint32_t* dir, unsigned long long* end_key, hipEvent_t ev0, hipEvent_t ev1,
                 hipStream_t stream)
{
    PairArgs a{};
    bool empty = false;
    int rc = pair_setup(p, L, w, query, m, subject, n, sm, go, ge, elem, score_out, stream, a, empty);
    if (rc || empty)
        return rc;
    if (p.flow) {
        if (ev0) HIPCHK(hipEventRecord(ev0, stream));
        rc = flow_enqueue(p, L, w, a, n, go, ge, elem, score_out, nullptr, nullptr, 0, 0, stream);
        if (rc) return rc;
        if (ev1) HIPCHK(hipEventRecord(ev1, stream));
        return SW_OK;
    }
    a.dir = dir;
    a.end_key = end_key;
    if (ev0) HIPCHK(hipEventRecord(ev0, stream));
    rc = pair_skew_diagonals(a, p, elem, stream);
    if (rc) return rc;
    if (dir) {
        HIPCHK(launch_trace_reset(end_key, stream));
        rc = pair_skew_diagonals(a, p, elem, stream, true);
        if (rc) return rc;
    }
    if (ev1) HIPCHK(hipEventRecord(ev1, stream));
    return SW_OK;
}

// Alignment schedule: 8 rows per lane, 64 lanes per band (direction words of
// 8 rows), the planner's chunk width for that.
constexpr int64_t kBandRows = 8 * 64;
constexpr int64_t kAlignFullCells = int64_t(1) << 35;   // automatic: whole-matrix codes up to 16 GiB
constexpr int64_t kAlignBlockSide = 65536;              // automatic block side beyond that

PairPlanC align_plan(int64_t m, int64_t n, int cu, const sw_options* opt)
{
    sw_options o = opt ? *opt : sw_options{};
    o.pair_rows = 8;
    o.max_lanes = 64;
    return pair_plan(m, n, cu, &o, true);
}

bool align_blocked(int64_t m, int64_t n, const sw_options* opt)
{
    return (opt && opt->align_block > 0) || m * n > kAlignFullCells;
}

// Workspace past the pair buffers.  Whole matrix: the direction words.
// Blocks: checkpoint rows (below every gb-th band) and columns (right of
// every gc-th chunk), chunk maxima and the direction words of one block of gb
// bands x gc chunks.  Both: the end key and the walk state.  Without a plan,
// the bound over every chunk width.
struct AlignLayout {
    size_t ckpt_row = 0, ckpt_col = 0, chunk_max = 0, dir = 0, tail = 0, total = 0;
    size_t dir_alt[3] = {0, 0, 0}, set_alt[3] = {0, 0, 0};   // blocks: the neighbours' codes and pair buffers
    int64_t row_stride = 0, col_stride = 0, n_ckrow = 0, n_ckcol = 0, gb = 1, gc = 1;
};

AlignLayout align_layout(int64_t m, int64_t n, const sw_options* opt, const PairPlanC* p)
{
    AlignLayout A;
    const int64_t nb = p ? p->nb : ceil_div(std::max<int64_t>(m, 1), kBandRows);
    const int64_t wide = std::max<int64_t>(8192, opt ? opt->pair_cols : 0);   // widest chunk
    const int64_t cols = p ? p->nc * p->wc : align_up(n, 16) + wide;          // padded columns
    size_t off = 0;
    if (!align_blocked(m, n, opt)) {
        A.dir = off;
        off += align_up(nb * 64 * cols * 4, 256);
    } else {
        const int64_t B = (opt && opt->align_block > 0) ? opt->align_block : kAlignBlockSide;
        A.gb = ceil_div(B, kBandRows);
        A.gc = p ? ceil_div(B, p->wc) : 1;
        // (nc - 1) / gc < n / B for every chunk width, and gc * wc < B + wc
        A.n_ckrow = (nb - 1) / A.gb;
        A.n_ckcol = p ? (p->nc - 1) / A.gc : n / B + 1;
        A.row_stride = cols;
        A.col_stride = nb * kBandRows;
        const int64_t nchunks = p ? p->nc : ceil_div(std::max<int64_t>(n, 1), 16) + 1;
        const int64_t blk_cols = p ? A.gc * p->wc : B + wide;
        A.ckpt_row = off; off += align_up(A.n_ckrow * A.row_stride * 8, 256);
        A.ckpt_col = off; off += align_up(A.n_ckcol * A.col_stride * 8, 256);
        A.chunk_max = off; off += align_up(nchunks * 4, 256);
        const size_t dsz = align_up(A.gb * 64 * blk_cols * 4, 256);
        A.dir = off; off += dsz;
        // the three neighbour blocks computed beside the walk's block: their
        // codes and a set of pair buffers each
        const size_t setsz = align_up(pair_layout(m, n, p, p ? p->wc : wide).total, 256);
        for (int k = 0; k < 3; ++k) {
            A.dir_alt[k] = off; off += dsz;
            A.set_alt[k] = off; off += setsz;
        }
    }
    A.tail = off;                 // end key, spare key, walk state
    off += 512;
    A.total = off;
    return A;
}

// Blocked alignment: score pass with checkpoints and chunk maxima; the end
// cell from a direction pass (codes not kept) over the checkpoint block
// column holding the first chunk whose maximum is the score; then, block by
// block along the walk, the direction codes of the block holding the walk's
// cell (recomputed from its checkpoint row and column, up to that cell) and
// the walk through it.  The host reads the walk's position after each block,
// so the call returns with the stream drained.
int align_blocks(const PairPlanC& p, const PairLayout& L, const AlignLayout& A, uint8_t* w, uint8_t* x,
                 const uint8_t* query, int64_t m, const uint8_t* subject, int64_t n, const int32_t* sm, int32_t go,
                 int32_t ge, int elem, AlignOut* o, char* ops, const sw_options* opt, hipStream_t stream)
{
    auto* end_key = reinterpret_cast<unsigned long long*>(x + A.tail);
    auto* spare_key = end_key + 1;
    auto* walk = reinterpret_cast<WalkState*>(x + A.tail + 256);
    PairArgs a{};
    bool empty = false;
    int rc = pair_setup(p, L, w, query, m, subject, n, sm, go, ge, elem, &o->score, stream, a, empty);
    if (rc) return rc;
    HIPCHK(launch_trace_reset(end_key, stream));
    if (empty) {
        HIPCHK(launch_walk_init(end_key, &o->score, walk, stream));
        HIPCHK(launch_walk_finish(walk, &o->score, ops, o, stream));
        return SW_OK;
    }
    auto* ckrow = reinterpret_cast<int2*>(x + A.ckpt_row);
    auto* cmax = reinterpret_cast<int32_t*>(x + A.chunk_max);
    auto* dir = reinterpret_cast<uint32_t*>(x + A.dir);
    a.ckpt_row = ckrow;
    a.ckpt_col = reinterpret_cast<int2*>(x + A.ckpt_col);
    a.ckpt_row_stride = A.row_stride;
    a.ckpt_col_stride = A.col_stride;
    a.ckpt_gb = (int32_t)A.gb;
    a.ckpt_gc = (int32_t)A.gc;
    a.chunk_max = cmax;
    HIPCHK(hipMemsetAsync(cmax, 0, sizeof(int32_t) * p.nc, stream));
    if (opt && opt->ev_search_begin) HIPCHK(hipEventRecord(opt->ev_search_begin, stream));
    rc = pair_diagonals(a, PairPass::kScoreCkpt, 8, elem, 0, p.nb - 1, 0, p.nc - 1, stream);
    if (rc) return rc;
    int32_t S = 0;
    std::vector<int32_t> cm((size_t)p.nc);
    HIPCHK(hipMemcpyAsync(&S, &o->score, sizeof S, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipMemcpyAsync(cm.data(), cmax, sizeof(int32_t) * p.nc, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    a.chunk_max = nullptr;
    if (S > 0) {
        int64_t cs = 0;
        while (cs < p.nc && cm[(size_t)cs] != S)
            ++cs;
        if (cs == p.nc)
            return fail(SW_EINVAL, "internal error: no chunk holds the score");
        const int64_t kc = cs / A.gc, c_org = kc * A.gc;
        a.b_org = 0;
        a.top_ckpt = nullptr;
        a.dir = nullptr;
        a.end_key = end_key;
        HIPCHK(launch_block_init(a, 0, kc, p.nb - 1, c_org, cs, stream));
        rc = pair_diagonals(a, PairPass::kTrace, 8, elem, 0, p.nb - 1, c_org, cs, stream);
        if (rc) return rc;
    }
    HIPCHK(launch_walk_init(end_key, &o->score, walk, stream));
    WalkState st{};
    HIPCHK(hipMemcpyAsync(&st, walk, sizeof st, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    a.end_key = spare_key;        // block passes look for no end cell
    // The walk leaves a block through its top or left edge, so the next block
    // is usually the one above or the one to the left, and the one after that
    // often the one above and to the left.  A round computes the codes of the
    // walk's block (up to its cell) and, on three more streams, of those
    // three neighbours (the one above up to the walk's column, the one to the
    // left up to its row, the diagonal one whole): the device runs the four
    // block passes at once, and a walk that enters a neighbour goes on there
    // without a new round.
    struct Region {
        PairArgs a;
        uint32_t* dir = nullptr;
        bool ok = false;
        int64_t kb = 0, kc = 0, b_org = 0, b_hi = 0, c_org = 0, c_hi = 0;
    };
    Region reg[4];
    reg[0].a = a;
    reg[0].dir = dir;
    for (int k = 0; k < 3; ++k) {
        uint8_t* base = x + A.set_alt[k];
        reg[k + 1].a = a;
        reg[k + 1].a.rowbuf = reinterpret_cast<int2*>(base + L.rowbuf);
        reg[k + 1].a.colbuf = reinterpret_cast<int2*>(base + L.colbuf);
        reg[k + 1].a.corner = reinterpret_cast<int32_t*>(base + L.corner);
        reg[k + 1].a.carry = reinterpret_cast<int4*>(base + L.carry);
        reg[k + 1].a.sink = base + L.sink;
        reg[k + 1].dir = reinterpret_cast<uint32_t*>(x + A.dir_alt[k]);
    }
    struct Side {                 // the neighbours' streams (default priority) and events
        hipStream_t s[3] = {nullptr, nullptr, nullptr};
        hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
        ~Side()
        {
            for (hipStream_t hs : s) if (hs) (void)hipStreamDestroy(hs);
            for (hipEvent_t he : e) if (he) (void)hipEventDestroy(he);
        }
    } side;
    for (auto& hs : side.s) HIPCHK(hipStreamCreateWithFlags(&hs, hipStreamNonBlocking));
    for (auto& he : side.e) HIPCHK(hipEventCreateWithFlags(&he, hipEventDisableTiming));
    auto enqueue = [&](Region& r, hipStream_t s) -> int {
        PairArgs& ra = r.a;
        ra.b_org = (int32_t)r.b_org;
        ra.top_ckpt = r.kb > 0 ? ckrow + (r.kb - 1) * A.row_stride : nullptr;
        ra.dir = r.dir;
        ra.dir_col0 = r.c_org * p.wc;
        ra.dir_rb0 = (int32_t)(r.b_org * p.K);
        ra.dir_stride = (r.b_hi - r.b_org + 1) * p.K;
        HIPCHK(launch_block_init(ra, r.kb, r.kc, r.b_hi, r.c_org, r.c_hi, s));
        return pair_diagonals(ra, PairPass::kTrace, 8, elem, r.b_org, r.b_hi, r.c_org, r.c_hi, s);
    };
    while (!st.done) {
        const int64_t row = st.i - 1, col = st.j - 1;
        const int64_t kb = row / (A.gb * kBandRows), kc = col / (A.gc * p.wc);
        const int64_t bb = row / kBandRows, cc = col / p.wc;
        int use = -1;
        for (int k = 0; k < 4; ++k) {
            const Region& r = reg[k];
            if (r.ok && r.kb == kb && r.kc == kc && bb >= r.b_org && bb <= r.b_hi && cc >= r.c_org && cc <= r.c_hi)
                use = k;
        }
        if (use < 0) {
            Region& cur = reg[0];
            cur.ok = true;
            cur.kb = kb; cur.kc = kc;
            cur.b_org = kb * A.gb; cur.b_hi = bb;
            cur.c_org = kc * A.gc; cur.c_hi = cc;
            Region& up = reg[1];
            up.ok = kb > 0;
            up.kb = kb - 1; up.kc = kc;
            up.b_org = (kb - 1) * A.gb; up.b_hi = kb * A.gb - 1;
            up.c_org = cur.c_org; up.c_hi = cc;
            Region& left = reg[2];
            left.ok = kc > 0;
            left.kb = kb; left.kc = kc - 1;
            left.b_org = cur.b_org; left.b_hi = bb;
            left.c_org = (kc - 1) * A.gc; left.c_hi = kc * A.gc - 1;
            Region& diag = reg[3];
            diag.ok = kb > 0 && kc > 0;
            diag.kb = kb - 1; diag.kc = kc - 1;
            diag.b_org = up.b_org; diag.b_hi = up.b_hi;
            diag.c_org = left.c_org; diag.c_hi = left.c_hi;
            HIPCHK(hipEventRecord(side.e[0], stream));
            for (int k = 0; k < 3; ++k) {
                if (!reg[k + 1].ok) continue;
                HIPCHK(hipStreamWaitEvent(side.s[k], side.e[0], 0));
                rc = enqueue(reg[k + 1], side.s[k]);
                if (rc) return rc;
                HIPCHK(hipEventRecord(side.e[k + 1], side.s[k]));
            }
            rc = enqueue(cur, stream);
            if (rc) return rc;
            for (int k = 0; k < 3; ++k)
                if (reg[k + 1].ok)
                    HIPCHK(hipStreamWaitEvent(stream, side.e[k + 1], 0));
            use = 0;
        }
        const Region& r = reg[use];
        HIPCHK(launch_walk(r.dir, r.a.dir_stride, r.b_org * kBandRows, r.c_org * p.wc, (r.b_hi + 1) * kBandRows,
                           (r.c_hi + 1) * p.wc, walk, ops, m + n, stream));
        HIPCHK(hipMemcpyAsync(&st, walk, sizeof st, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        if (!st.done && st.i - 1 == row && st.j - 1 == col)
            return fail(SW_EINVAL, "internal error: the traceback walk did not advance");
    }
    if (opt && opt->ev_search_end) HIPCHK(hipEventRecord(opt->ev_search_end, stream));
    HIPCHK(launch_walk_finish(walk, &o->score, ops, o, stream));
    return SW_OK;
}

}  // namespace

extern "C" {

int sw_pair_score(const uint8_t* query, int64_t m, const uint8_t* subject, int64_t n, const int32_t* sm,
                  int32_t go, int32_t ge, const sw_options* opt, void* ws, size_t ws_bytes, int32_t* score_out,
                  hipStream_t stream)
{
    int fit = 0;
    int rc = pair_args_check(query, m, subject, n, sm, go, ge, opt, ws, fit);
    if (rc) return rc;
    if (!score_out) return fail(SW_EINVAL, "null score_out");
    const size_t need = sw_pair_workspace_bytes(m, n, opt);
    if (ws_bytes < need)
        return fail(SW_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    int cu = 256, lds = kLdsPerCU;
    rc = device_cu(&cu);
    if (rc) return rc;
    rc = device_lds(&lds);
    if (rc) return rc;
    int sm_max = 0;
    for (int i = 0; i < kAlpha * kAlpha; ++i) sm_max = std::max(sm_max, (int)sm[i]);
    const int elem = (fit == kFitS8 || fit == kFitU8) ? 1 : 2;
    const PairPlanC p = pair_plan(m, n, cu, opt, false, sm_max, elem, lds);
    if (!p.R) return fail(SW_EINVAL, "the pipelined pass cannot hold this pair's scores (max(SM) x min(m, n) >= 2^24)");
    const PairLayout L = pair_layout(m, n, &p, p.wc);
    if (L.total > need) return fail(SW_EINVAL, "internal error: pair layout exceeds the workspace size");
    return pair_enqueue(p, L, static_cast<uint8_t*>(ws), query, m, subject, n, sm, go, ge, elem, score_out,
                        nullptr, nullptr, opt ? opt->ev_search_begin : nullptr,
                        opt ? opt->ev_search_end : nullptr, stream);
}

}  // extern "C"

// ------------------------------------------------------------------ pair score without allocation
//
// Device scratch of sw_pair_score_static: one array per GPU, held until the
// process ends.  Host code never uses the array's name as an address (it is a
// host-side stand-in); the device address comes from hipGetSymbolAddress,
// taken once per device on that device's first call.
static __device__ __align__(256) uint8_t scratch[SW_STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, uint8_t*> g_scratch;      // device -> address of its copy of `scratch`

int static_scratch(uint8_t** out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto f = g_scratch.find(dev);
    if (f == g_scratch.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SW_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        f = g_scratch.emplace(dev, static_cast<uint8_t*>(p)).first;
    }
    *out = f->second;
    return SW_OK;
}

}  // namespace

extern "C" {

int sw_pair_score_static(const uint8_t* query, int64_t m, const uint8_t* subject, int64_t n, const int32_t* sm,
                         int32_t go, int32_t ge, const sw_options* opt, int32_t* score_out, hipStream_t stream)
{
    std::string why;
    if (!validate_pair(m, n, opt, why)) return fail(SW_EINVAL, why);
    const size_t need = sw_pair_workspace_bytes(m, n, opt);
    if (need > SW_STATIC_SCRATCH_BYTES)
        return fail(SW_ENOMEM, "pair needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                   std::to_string((long long)SW_STATIC_SCRATCH_BYTES) +
                                   " bytes of the static scratch; use sw_pair_score with a workspace");
    uint8_t* ws = nullptr;
    const int rc = static_scratch(&ws);
    if (rc) return rc;
    return sw_pair_score(query, m, subject, n, sm, go, ge, opt, ws, SW_STATIC_SCRATCH_BYTES, score_out, stream);
}

size_t sw_align_workspace_bytes(int64_t m, int64_t n, const sw_options* opt)
{
    std::string why;
    if (!validate_pair(m, n, opt, why)) { fail(SW_EINVAL, why); return 0; }
    return pair_layout(m, n, nullptr, pair_wc_max(opt)).total + 256 + align_layout(m, n, opt, nullptr).total;
}

int sw_align_pair(const uint8_t* query, int64_t m, const uint8_t* subject, int64_t n, const int32_t* sm,
                  int32_t go, int32_t ge, const sw_options* opt, void* ws, size_t ws_bytes, sw_alignment* out,
                  char* ops, hipStream_t stream)
{
    int fit = 0;
    int rc = pair_args_check(query, m, subject, n, sm, go, ge, opt, ws, fit);
    if (rc) return rc;
    if (!out) return fail(SW_EINVAL, "null alignment output");
    if (m > 0 && n > 0 && !ops) return fail(SW_EINVAL, "null operation buffer");
    const size_t need = sw_align_workspace_bytes(m, n, opt);
    if (need == 0) return SW_EINVAL;
    if (ws_bytes < need)
        return fail(SW_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    int cu = 256;
    rc = device_cu(&cu);
    if (rc) return rc;
    const PairPlanC p = align_plan(m, n, cu, opt);
    const int elem = (fit == kFitS8 || fit == kFitU8) ? 1 : 2;
    // With whole-matrix codes the score may come from the pipelined pass
    // when the planner takes it for the pair; its buffers and the tiles' then
    // sit in the layout bound for every schedule, which holds both.
    // So may the code pass: the pipelined pass with 4 or 8 rows per lane (the
    // tiles' 8-row blocks, or halves of them) when the planner takes it over
    // the tiles.
    PairPlanC sp{}, cp{};
    if (!align_blocked(m, n, opt) && m > 0 && n > 0) {
        int lds = kLdsPerCU, sm_max = 0;
        rc = device_lds(&lds);
        if (rc) return rc;
        for (int i = 0; i < kAlpha * kAlpha; ++i) sm_max = std::max(sm_max, (int)sm[i]);
        sp = pair_plan(m, n, cu, opt, false, sm_max, elem, lds);
        // 4 rows per lane write half words: twice the bands of 8 rows, all
        // inside the code region (ceil(m / 256) <= 2 ceil(m / 512) bands)
        // (an explicit pair_rows holds for the code pass too: 4 or 8 there,
        // any other leaves the codes to the tiles)
        sw_options co = opt ? *opt : sw_options{};
        for (int R : {4, 8}) {
            if (opt && opt->pair_rows && opt->pair_rows != R) continue;
            co.pair_rows = R;
            const PairPlanC c = pair_plan(m, n, cu, &co, false, sm_max, elem, lds);
            if (c.flow && c.R == R && c.nb * R <= p.nb * 8 && (!cp.flow || c.est_s < cp.est_s))
                cp = c;
        }
    }
    const bool either = sp.flow || cp.flow;
    const PairLayout L = either ? pair_layout(m, n, nullptr, pair_wc_max(opt)) : pair_layout(m, n, &p, p.wc);
    const size_t x_off = align_up(L.total, 256);
    const AlignLayout A = align_layout(m, n, opt, &p);
    if (x_off + A.total > need)
        return fail(SW_EINVAL, "internal error: alignment layout exceeds the workspace size");
    uint8_t* w = static_cast<uint8_t*>(ws);
    uint8_t* x = w + x_off;
    auto* o = reinterpret_cast<AlignOut*>(out);
    if (align_blocked(m, n, opt))
        return align_blocks(p, L, A, w, x, query, m, subject, n, sm, go, ge, elem, o, ops, opt, stream);
    auto* dir = reinterpret_cast<uint32_t*>(x + A.dir);
    auto* end_key = reinterpret_cast<unsigned long long*>(x + A.tail);
    auto* walk = reinterpret_cast<WalkState*>(x + A.tail + 256);
    if (either) {
        // the score (-1 if a wait of the pipelined pass gave up), then the
        // code pass; its setup clears a spare word, not the score
        rc = pair_enqueue(sp.flow ? sp : p, L, w, query, m, subject, n, sm, go, ge, elem, &o->score, nullptr, nullptr,
                          opt ? opt->ev_search_begin : nullptr, nullptr, stream);
        if (rc) return rc;
        const PairPlanC& q = cp.flow ? cp : p;
        PairArgs a{};
        bool empty = false;
        rc = pair_setup(q, L, w, query, m, subject, n, sm, go, ge, elem, reinterpret_cast<int32_t*>(x + A.tail + 64),
                        stream, a, empty);
        if (rc) return rc;
        HIPCHK(launch_trace_reset(end_key, stream));
        if (cp.flow) {
            rc = flow_enqueue(cp, L, w, a, n, go, ge, elem, &o->score, dir, end_key, p.nb * p.K, m, stream);
        } else {
            a.score = &o->score;
            a.dir = dir;
            a.end_key = end_key;
            rc = pair_skew_diagonals(a, p, elem, stream, true);
        }
        if (rc) return rc;
        if (opt && opt->ev_search_end) HIPCHK(hipEventRecord(opt->ev_search_end, stream));
    } else {
        rc = pair_enqueue(p, L, w, query, m, subject, n, sm, go, ge, elem, &o->score, dir, end_key,
                          opt ? opt->ev_search_begin : nullptr, opt ? opt->ev_search_end : nullptr, stream);
        if (rc) return rc;
    }
    if (m == 0 || n == 0) {
        HIPCHK(launch_trace_reset(end_key, stream));
    }
    HIPCHK(launch_walk_init(end_key, &o->score, walk, stream));
    if (m > 0 && n > 0)
        HIPCHK(launch_walk(dir, p.nb * p.K, 0, 0, INT64_MAX, INT64_MAX, walk, ops, m + n, stream));
    HIPCHK(launch_walk_finish(walk, &o->score, ops, o, stream));
    return SW_OK;
}

}  // extern "C"

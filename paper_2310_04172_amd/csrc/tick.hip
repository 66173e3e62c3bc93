// Batched tick: sensor update, normalisation, pose estimate and resampling of
// many filters in one launch per stage.  Job tables and totals live in device memory, so the
// launch chain does not depend on the job set: it is captured once into a HIP
// graph (per stream, per mix of sensor groups and launch shape) and replayed every
// tick after the tables are copied in.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "jobs.h"

namespace mcl {

SensorJob make_sensor_job(const mcl_map_s *, const float *, int, const float *, int, float, float *, float *);
void apply_cfg(SensorJob &, const LaunchCfg &);
template <typename Src>
mcl_status launch_sensor_src(int32_t, const Src &, int64_t, int64_t, bool, LaunchCfg, hipStream_t, size_t, bool, bool,
                             bool, int64_t, int);
template <typename Src>
mcl_status launch_sensor_sparse_src(int32_t, const Src &, int64_t, int64_t, bool, hipStream_t);
template <typename Src>
mcl_status launch_sensor_tri_src(int32_t, const Src &, int64_t, int64_t, bool, hipStream_t);
template <typename Src>
mcl_status launch_normalize_src(const Src &, int, int64_t, int64_t, hipStream_t);
template <typename Src>
mcl_status launch_resample_src(const Src &, int64_t, int64_t, hipStream_t);
template <typename Src>
mcl_status launch_estimate_src(const Src &, int64_t, int64_t, hipStream_t);
template <bool NORM, bool RS, typename Src>
mcl_status launch_weights_fused_src(const Src &, int, hipStream_t);
int weights_fused_max();
size_t weight_ws_bytes(int N);
void bind_weight_ws(WeightJob &J, void *ws);

constexpr int kMaxJobs = MCL_MAX_JOBS;
// Sensor groups: storage type (0..2) + 3 x kind, the kind being the nearest
// lookup on a dense map (0), on a sparse map (1), the trilinear lookup on a
// dense map (2) or the nearest lookup on a dense map with the sum reading (3);
// each group present gets one sensor launch.
constexpr int kTypes = 3;
constexpr int kKindDense = 0, kKindSparse = 1, kKindTri = 2, kKindDenseSum = 3;
constexpr int kGroups = 4 * kTypes;

inline int job_kind(const mcl_filter_job &F) {
    if (F.map->sparse) return kKindSparse;
    if (F.lookup == MCL_LOOKUP_TRILINEAR) return kKindTri;
    return F.score == MCL_SCORE_SUM ? kKindDenseSum : kKindDense;
}
inline bool dense_nearest(int kind) { return kind == kKindDense || kind == kKindDenseSum; }
inline int job_group(const mcl_filter_job &F) { return F.map->dtype + kTypes * job_kind(F); }

static constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device/staging layout: Counts[kGroups + 2] | SensorJob[kGroups][kMaxJobs] |
// WeightJob[kMaxJobs] | EstJob[kMaxJobs].  Each sensor group has its own table
// at a fixed place, so a captured chain stays valid however the jobs of a tick
// split among the groups.  Counts: one per sensor group, the weights', the
// estimates'.
static constexpr int kWeightCnt = kGroups, kEstCnt = kGroups + 1;
static constexpr size_t kCountsBytes = align256(sizeof(Counts) * (kGroups + 2));
static constexpr size_t kSensorTblOff = kCountsBytes;
static constexpr size_t kSensorTblBytes = align256(sizeof(SensorJob) * kMaxJobs);
static constexpr size_t kWeightTblOff = kSensorTblOff + kGroups * kSensorTblBytes;
static constexpr size_t kEstTblOff = kWeightTblOff + align256(sizeof(WeightJob) * kMaxJobs);
static constexpr size_t kTablesBytes = kEstTblOff + align256(sizeof(EstJob) * kMaxJobs);

namespace {

// A captured chain serves every tick whose totals fit its power-of-two buckets.
struct GraphKey {
    int mask;
    std::array<int, kGroups> wpb, bpc;  // launch shape per sensor group
    std::array<int64_t, kGroups> items;
    int64_t elems, blocks, eblocks, ejobs;
    std::array<int64_t, kGroups> lds;  // LDS bytes for the read bits of a group's shared map, or 0
    int fused;                          // weights stage: one workgroup per filter (1) or the chains (0)
    int pct;                            // groups whose jobs read pose-constant tables (bit per group)
    int ord;                            // groups with jobs in spatial order (bit per group)
    bool operator<(const GraphKey &o) const {
        return std::tie(mask, wpb, bpc, items, elems, blocks, eblocks, ejobs, lds, fused, pct, ord) <
               std::tie(o.mask, o.wpb, o.bpc, o.items, o.elems, o.blocks, o.eblocks, o.ejobs, o.lds, o.fused, o.pct,
                        o.ord);
    }
};

int64_t bucket(int64_t x) {
    int64_t b = 1;
    while (b < x) b <<= 1;
    return b;
}

struct TickState {
    char *dev = nullptr;      // tables + per-job workspace
    size_t dev_bytes = 0;
    char *host = nullptr;     // pinned staging copy of the tables
    hipEvent_t copied = nullptr;
    bool pending = false;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::map<GraphKey, hipGraph_t> graph_defs;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, TickState> g_state;

void drop_graphs(TickState &S) {
    for (auto &kv : S.graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &kv : S.graph_defs) (void)hipGraphDestroy(kv.second);
    S.graphs.clear();
    S.graph_defs.clear();
}

// The spatial order's room: cell counters, the particles' ranks and slots.
size_t order_ws_bytes(int N) {
    return align256(kOrderCells * sizeof(int32_t)) + 2 * align256((size_t)N * sizeof(int32_t));
}

// Library workspace of one filter in a tick: weights stage, piece partials,
// the particles' pose constants and spatial order (dense maps, nearest
// lookup), pose estimate.
size_t job_ws_bytes(int N, int K, bool est, bool pct) {
    const int np = sensor_pieces(K);
    size_t b = align256(weight_ws_bytes(N));
    if (np > 1) b += align256((size_t)np * N * sizeof(float));
    if (pct) b += align256((size_t)N * 12 * sizeof(float)) + order_ws_bytes(N);
    if (est) b += align256(estimate_ws_bytes(N));
    return b;
}

}  // namespace

size_t tick_job_bytes(int N, int K) { return job_ws_bytes(N, K, true, true); }

mcl_status check_job(const mcl_filter_job &J, int j) {
    std::string at = "tick: job " + std::to_string(j) + ": ";
    if (!J.map) return fail(MCL_EINVAL, at + "NULL map");
    if (!J.poses || !J.logw || !J.wq || !J.idx) return fail(MCL_EINVAL, at + "NULL poses, logw, wq or idx");
    if (J.K < 0 || J.N < 1) return fail(MCL_EINVAL, at + "need K >= 0 and N >= 1");
    if (J.K > MCL_MAX_POINTS || J.N > MCL_MAX_PARTICLES) return fail(MCL_ERANGE, at + "K or N above the limit");
    if (J.K > 0 && !J.points) return fail(MCL_EINVAL, at + "NULL points with K > 0");
    if (!(std::isfinite(J.sigma) && J.sigma > 0.0f)) return fail(MCL_EINVAL, at + "sigma must be finite and > 0");
    if (!J.est_mean && (J.est_idx || J.est_pose))
        return fail(MCL_EINVAL, at + "est_idx or est_pose without est_mean");
    if (J.est_mean && !J.w) return fail(MCL_EINVAL, at + "a pose estimate needs the weights w");
    if (J.lookup != MCL_LOOKUP_NEAREST && J.lookup != MCL_LOOKUP_TRILINEAR)
        return fail(MCL_EINVAL, at + "lookup must be MCL_LOOKUP_NEAREST or MCL_LOOKUP_TRILINEAR");
    if (J.lookup == MCL_LOOKUP_TRILINEAR && J.map->sparse)
        return fail(MCL_EINVAL, at + "the trilinear lookup needs a dense map");
    if (J.score != MCL_SCORE_PRODUCT && J.score != MCL_SCORE_SUM)
        return fail(MCL_EINVAL, at + "score must be MCL_SCORE_PRODUCT or MCL_SCORE_SUM");
    if (J.score == MCL_SCORE_SUM) {
        if (J.map->sparse || J.lookup != MCL_LOOKUP_NEAREST)
            return fail(MCL_EINVAL, at + "the sum reading needs a dense map and the nearest lookup");
        if (!sum_sigma_ok(J.map, J.sigma)) return fail(MCL_EINVAL, at + "the sum reading needs sigma >= tau / 8");
    }
    return MCL_OK;
}

}  // namespace mcl

using namespace mcl;

extern "C" size_t mcl_job_bytes(int32_t N, int32_t K) {
    if (N < 1 || K < 0) return 0;
    // caller buffers: poses in + out, logw, w, wq, idx, scan, estimate; then library workspace
    size_t caller = (size_t)N * (48 + 48 + 4 + 8 + 8 + 4) + (size_t)K * 12 + 12 * 8 + 4 + 12 * 4;
    return caller + tick_job_bytes(N, K) + sizeof(SensorJob) + sizeof(WeightJob) + sizeof(EstJob);
}

extern "C" mcl_status mcl_tick(const mcl_filter_job *jobs, int32_t n_jobs, int32_t flags, void *stream_) {
    if (!jobs || n_jobs < 1) return fail(MCL_EINVAL, "tick: need at least one job");
    if (n_jobs > kMaxJobs) return fail(MCL_ERANGE, "tick: more jobs than MCL_MAX_JOBS");
    for (int j = 0; j < n_jobs; ++j) {
        mcl_status st = check_job(jobs[j], j);
        if (st != MCL_OK) return st;
    }
    for (int j = 0; j < n_jobs; ++j)
        if (jobs[j].map->sparse && !jobs[j].map->sp.small)
            return fail(MCL_EINVAL, "tick: job " + std::to_string(j) +
                                        ": sparse maps with a pool of 4 GiB or more are not supported in a batched tick");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const bool use_graph = (flags & MCL_TICK_GRAPH) != 0;
    if (use_graph && stream == nullptr) return fail(MCL_EINVAL, "tick: graph replay needs a non-default stream");
    // corner cells of maps read by the trilinear lookup (built once per map)
    for (int j = 0; j < n_jobs; ++j)
        if (job_kind(jobs[j]) == kKindTri) {
            mcl_status st = ensure_trilinear(jobs[j].map, stream);
            if (st != MCL_OK) return st;
        }

    // sensor groups: one sensor launch per group present
    std::vector<int> order(n_jobs);
    for (int j = 0; j < n_jobs; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return job_group(jobs[a]) < job_group(jobs[b]); });
    int g_begin[kGroups + 1] = {};
    for (int g = 0; g < kGroups; ++g) {
        int c = 0;
        for (int j = 0; j < n_jobs; ++j) c += job_group(jobs[j]) == g;
        g_begin[g + 1] = g_begin[g] + c;
    }
    int mask = 0;
    for (int g = 0; g < kGroups; ++g) mask |= (g_begin[g + 1] > g_begin[g]) << g;

    size_t need = kTablesBytes;
    int n_est = 0;
    for (int j = 0; j < n_jobs; ++j) {
        need += job_ws_bytes(jobs[j].N, jobs[j].K, jobs[j].est_mean != nullptr, dense_nearest(job_kind(jobs[j])));
        n_est += jobs[j].est_mean != nullptr;
    }
    if (n_est) mask |= 1 << kGroups;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MCL_EDEVICE, "tick: no device");
    std::lock_guard<std::mutex> lk(g_mu);
    TickState &S = g_state[{dev, stream}];
    if (!S.host) {
        if (hipHostMalloc((void **)&S.host, kTablesBytes, hipHostMallocDefault) != hipSuccess)
            return fail(MCL_ENOMEM, "tick: pinned staging allocation failed");
        if (hipEventCreateWithFlags(&S.copied, hipEventDisableTiming) != hipSuccess)
            return fail(MCL_EDEVICE, "tick: event creation failed");
    }
    // the previous tick's table copy must have left the staging buffer
    if (S.pending) {
        if (flags & MCL_TICK_NOWAIT) {
            const hipError_t q = hipEventQuery(S.copied);
            if (q == hipErrorNotReady)
                return fail(MCL_EBUSY, "tick: the previous tick on this stream still holds the table staging buffer");
            if (q != hipSuccess) return fail(MCL_EDEVICE, "tick: event query failed");
        } else if (hipEventSynchronize(S.copied) != hipSuccess) {
            return fail(MCL_EDEVICE, "tick: event wait failed");
        }
        S.pending = false;
    }
    if (S.dev_bytes < need) {
        if (hipStreamSynchronize(stream) != hipSuccess) return fail(MCL_EDEVICE, "tick: synchronisation failed");
        drop_graphs(S);
        if (S.dev) (void)hipFree(S.dev);
        S.dev = nullptr;
        S.dev_bytes = 0;
        size_t want = need + need / 4;
        if (hipMalloc((void **)&S.dev, want) != hipSuccess) return fail(MCL_ENOMEM, "tick: workspace allocation failed");
        S.dev_bytes = want;
    }
    // launch shape and runs per sensor group: those tuned for the group's
    // largest filter (dense nearest lookups; the sparse and trilinear launches
    // have a fixed shape); the coarse-level mode and threshold per filter, from
    // its own size class (below)
    LaunchCfg cfgs[kGroups];
    for (int g = 0; g < kGroups; ++g) {
        cfgs[g] = kDefaultCfg;
        if (!dense_nearest(g / kTypes) || g_begin[g + 1] == g_begin[g]) continue;
        int big = order[g_begin[g]];
        for (int t = g_begin[g] + 1; t < g_begin[g + 1]; ++t) {
            const int j = order[t];
            if ((int64_t)jobs[j].N * jobs[j].K > (int64_t)jobs[big].N * jobs[big].K) big = j;
        }
        cfgs[g] = tuned_config(jobs[big].map->dtype, jobs[big].K, jobs[big].N);
    }
    // pose-constant tables for a dense nearest group with enough evaluations,
    // or with a filter large enough for the spatial order (which the tables carry)
    bool pct[kGroups] = {}, ord[kGroups] = {};
    for (int g = 0; g < kGroups; ++g) {
        if (!dense_nearest(g / kTypes)) continue;
        int64_t ev = 0;
        for (int t = g_begin[g]; t < g_begin[g + 1]; ++t) {
            const int64_t e = (int64_t)jobs[order[t]].N * jobs[order[t]].K;
            ev += e;
            ord[g] = ord[g] || spatial_order(e);
        }
        pct[g] = ev >= kPoseTableMinEvals || ord[g];
    }
    // runs per group where not tuned: one value for the whole tick, from its
    // total (group, piece) pairs
    int64_t pairs = 0;
    for (int j = 0; j < n_jobs; ++j)
        pairs += (int64_t)((jobs[j].N + kGroup - 1) / kGroup) * sensor_pieces(jobs[j].K);
    const int nsub = sensor_runs(pairs);

    Counts *cnt = reinterpret_cast<Counts *>(S.host);
    WeightJob *wtbl = reinterpret_cast<WeightJob *>(S.host + kWeightTblOff);
    EstJob *etbl = reinterpret_cast<EstJob *>(S.host + kEstTblOff);
    std::memset(cnt, 0, kCountsBytes);
    int64_t eblk = 0, eelem = 0;
    int ne = 0;
    char *ws = S.dev + kTablesBytes;
    bool combine[kGroups] = {};
    int64_t wblk = 0, welem = 0;
    int64_t oblocks[kGroups] = {};
    for (int g = 0; g < kGroups; ++g) {
        int64_t items = 0, elems = 0;
        SensorJob *stbl = reinterpret_cast<SensorJob *>(S.host + kSensorTblOff + g * kSensorTblBytes) - g_begin[g];
        for (int s = g_begin[g]; s < g_begin[g + 1]; ++s) {
            const mcl_filter_job &F = jobs[order[s]];
            const mcl_map_s *m = F.map;
            const double sc = m->scale, sg = (double)F.sigma;
            const float c = (float)((sc * sc) / (2.0 * sg * sg));
            const int np = sensor_pieces(F.K);
            WeightJob &W = wtbl[s];
            std::memset(&W, 0, sizeof W);
            W.N = F.N;
            bind_weight_ws(W, ws);
            ws += align256(weight_ws_bytes(F.N));
            float *part = nullptr;
            if (np > 1) {
                part = reinterpret_cast<float *>(ws);
                ws += align256((size_t)np * F.N * sizeof(float));
                combine[g] = true;
            }
            SensorJob &J = stbl[s];
            J = make_sensor_job(m, F.points, F.K, F.poses, F.N, c, F.logw, part);
            if (dense_nearest(job_kind(F))) {  // the pose-constant table's and the order's room; filled by the launch chain
                if (pct[g]) J.pc = reinterpret_cast<const float *>(ws);
                ws += align256((size_t)F.N * 12 * sizeof(float));
                if (pct[g] && spatial_order((int64_t)F.N * F.K)) {
                    J.ocell = reinterpret_cast<int32_t *>(ws);
                    J.orank = reinterpret_cast<int32_t *>(ws + align256(kOrderCells * sizeof(int32_t)));
                    J.orig = J.orank + align256((size_t)F.N * sizeof(int32_t)) / sizeof(int32_t);
                    J.oblk0 = oblocks[g];
                    oblocks[g] += order_blocks(F.N);
                } else {
                    J.oblk0 = oblocks[g];  // no counting blocks of its own
                }
                ws += order_ws_bytes(F.N);
            }
            if (job_kind(F) == kKindTri) J.tri = m->tri;
            if (job_kind(F) == kKindDenseSum) {
                J.score = kScoreSum;
                J.k2 = sum_k2(m, F.sigma);
            }
            J.item0 = items;
            J.elem0 = elems;
            J.nsub = nsub;
            apply_cfg(J, cfgs[g]);
            if (dense_nearest(job_kind(F))) {
                // where a filter reads the coarse level suits the spread of its own
                // particles: its own size class's setting (whether the launch holds
                // the bits in LDS at all is the group's)
                const LaunchCfg own = tuned_config(m->dtype, F.K, F.N);
                J.coarse = own.coarse;
                J.lds8 = own.lds8 > 0 ? own.lds8 : kLdsEighths;
            } else {
                J.coarse = cfgs[g].coarse;
            }
            items += (int64_t)J.ngroups * J.npiece * J.nsub;
            elems += F.N;
            W.logw = F.logw;
            W.w = F.w;
            W.wq = F.wq;
            W.log_z = F.log_z;
            W.idx = F.idx;
            W.pin = F.poses_out ? F.poses : nullptr;
            W.pout = F.poses_out;
            W.u = resample_draw(F.seed, F.tick);
            W.elem0 = welem;
            W.blk0 = (int32_t)wblk;
            welem += F.N;
            wblk += W.nblk;
            if (F.est_mean) {
                EstJob &E = etbl[ne++];
                std::memset(&E, 0, sizeof E);
                E.w = F.w;
                E.poses = F.poses;
                E.mean = F.est_mean;
                E.best_idx = F.est_idx;
                E.best_pose = F.est_pose;
                E.N = F.N;
                bind_estimate_ws(E, ws);
                ws += align256(estimate_ws_bytes(F.N));
                E.blk0 = (int32_t)eblk;
                eblk += E.nblk;
                eelem += F.N;
            }
        }
        cnt[g] = Counts{g_begin[g + 1] - g_begin[g], items, elems, oblocks[g]};
    }
    cnt[kWeightCnt] = Counts{n_jobs, 0, welem, wblk};
    cnt[kEstCnt] = Counts{ne, 0, eelem, eblk};

    bool ok = hipMemcpyAsync(S.dev, S.host, kCountsBytes, hipMemcpyHostToDevice, stream) == hipSuccess;
    for (int g = 0; g < kGroups && ok; ++g) {
        const size_t off = kSensorTblOff + g * kSensorTblBytes;
        const size_t n = (size_t)(g_begin[g + 1] - g_begin[g]) * sizeof(SensorJob);
        if (n) ok = hipMemcpyAsync(S.dev + off, S.host + off, n, hipMemcpyHostToDevice, stream) == hipSuccess;
    }
    ok = ok && hipMemcpyAsync(S.dev + kWeightTblOff, S.host + kWeightTblOff, (size_t)n_jobs * sizeof(WeightJob),
                              hipMemcpyHostToDevice, stream) == hipSuccess;
    if (ne)
        ok = ok && hipMemcpyAsync(S.dev + kEstTblOff, S.host + kEstTblOff, (size_t)ne * sizeof(EstJob),
                                  hipMemcpyHostToDevice, stream) == hipSuccess;
    if (!ok || hipEventRecord(S.copied, stream) != hipSuccess) return fail(MCL_EDEVICE, "tick: table copy failed");
    S.pending = true;

    // The launch chain reads every size from the device tables; grids are sized
    // for the totals (under a graph, for their power-of-two buckets, so a
    // replay serves any tick that fits; surplus waves exit at once).
    const Counts *dcnt = reinterpret_cast<const Counts *>(S.dev);
    const WeightJob *dwt = reinterpret_cast<const WeightJob *>(S.dev + kWeightTblOff);
    GraphKey key{mask, {}, {}, {}, 0, 0, 0, 0, {}, 0, 0, 0};
    for (int g = 0; g < kGroups; ++g) {
        key.pct |= (int)pct[g] << g;
        key.ord |= (int)ord[g] << g;
    }
    for (int g = 0; g < kGroups; ++g) {
        key.wpb[g] = cfgs[g].waves_per_block;
        key.bpc[g] = cfgs[g].blocks_per_cu;
    }
    // A dense group whose jobs all read one map with a small enough bit table
    // gets the kernel that holds those bits in LDS (a power of two bytes, so a
    // graph serves any such map up to that size).
    for (int g = 0; g < kGroups; ++g) {
        if (!dense_nearest(g / kTypes) || g_begin[g + 1] == g_begin[g] || cfgs[g].coarse == kCoarseBytes) continue;
        const mcl_map_s *m0 = jobs[order[g_begin[g]]].map;
        bool shared = true;
        for (int s = g_begin[g] + 1; s < g_begin[g + 1] && shared; ++s) shared = jobs[order[s]].map == m0;
        const int64_t bits = (int64_t)m0->view.nrwords * 4;
        if (shared && bits <= (int64_t)kMaxLdsBits) key.lds[g] = std::max<int64_t>(bucket(bits), 1024);
    }
    for (int g = 0; g < kGroups; ++g) key.items[g] = use_graph ? bucket(cnt[g].items) : cnt[g].items;
    key.elems = use_graph ? bucket(welem) : welem;
    key.blocks = use_graph ? bucket(wblk) : wblk;
    key.eblocks = use_graph ? bucket(eblk) : eblk;
    key.ejobs = use_graph ? bucket(ne) : ne;
    {
        int max_n = 0;
        for (int j = 0; j < n_jobs; ++j) max_n = std::max(max_n, (int)jobs[j].N);
        key.fused = max_n <= weights_fused_max();
    }
    auto chain = [&]() -> mcl_status {
        for (int g = 0; g < kGroups; ++g) {
            if (!(mask >> g & 1)) continue;
            JobTable<SensorJob> src{reinterpret_cast<const SensorJob *>(S.dev + kSensorTblOff + g * kSensorTblBytes),
                                    dcnt + g};
            // under a graph every group may combine (a job with one piece is skipped inside)
            const int type = g % kTypes, kind = g / kTypes;
            const bool comb = use_graph || combine[g];
            // the order's grids: fixed under a graph (surplus workgroups exit)
            const int64_t oblk = use_graph ? 2048 : oblocks[g];
            const int ojobs = use_graph ? 64 : g_begin[g + 1] - g_begin[g];
            mcl_status st =
                dense_nearest(kind) ? launch_sensor_src(type, src, key.items[g], key.elems, comb, cfgs[g], stream,
                                                        (size_t)key.lds[g], kind == kKindDenseSum, (key.pct >> g) & 1,
                                                        (key.ord >> g) & 1, oblk, ojobs)
                : kind == kKindSparse ? launch_sensor_sparse_src(type, src, key.items[g], key.elems, comb, stream)
                                      : launch_sensor_tri_src(type, src, key.items[g], key.elems, comb, stream);
            if (st != MCL_OK) return st;
        }
        JobTable<WeightJob> wsrc{dwt, dcnt + kWeightCnt};
        // every filter has at least one weight block, so a tick that replays this
        // graph has no more filters than key.blocks
        const int fjobs = use_graph ? (int)std::min<int64_t>(key.blocks, kMaxJobs) : n_jobs;
        if (key.fused && !key.ejobs) return launch_weights_fused_src<true, true>(wsrc, fjobs, stream);
        mcl_status st = key.fused ? launch_weights_fused_src<true, false>(wsrc, fjobs, stream)
                                  : launch_normalize_src(wsrc, use_graph ? kMaxJobs : n_jobs, key.blocks, key.elems,
                                                         stream);
        if (st != MCL_OK) return st;
        if (key.ejobs) {
            JobTable<EstJob> esrc{reinterpret_cast<const EstJob *>(S.dev + kEstTblOff), dcnt + kEstCnt};
            st = launch_estimate_src(esrc, key.eblocks, key.ejobs, stream);
            if (st != MCL_OK) return st;
        }
        return key.fused ? launch_weights_fused_src<false, true>(wsrc, fjobs, stream)
                         : launch_resample_src(wsrc, key.blocks, key.elems, stream);
    };
    // every map the tick reads: an event after its work (deferred mcl_map_free)
    auto note_uses = [&]() -> mcl_status {
        std::vector<mcl_map_s *> maps(n_jobs);
        for (int j = 0; j < n_jobs; ++j) maps[j] = jobs[j].map;
        std::sort(maps.begin(), maps.end());
        maps.erase(std::unique(maps.begin(), maps.end()), maps.end());
        for (mcl_map_s *m : maps) {
            mcl_status st = note_map_use(m, stream);
            if (st != MCL_OK) return st;
        }
        return MCL_OK;
    };
    if (!use_graph) {
        mcl_status st = chain();
        return st == MCL_OK ? note_uses() : st;
    }

    auto it = S.graphs.find(key);
    if (it == S.graphs.end() && S.graphs.size() >= 32) {  // bound the cache, once earlier replays have ended
        if (hipStreamSynchronize(stream) != hipSuccess) return fail(MCL_EDEVICE, "tick: synchronisation failed");
        drop_graphs(S);
    }
    if (it == S.graphs.end()) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(MCL_EDEVICE, "tick: stream capture failed to begin");
        mcl_status st = chain();
        hipError_t e = hipStreamEndCapture(stream, &graph);
        if (st != MCL_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(MCL_EDEVICE, "tick: graph capture or instantiation failed");
        }
        S.graph_defs[key] = graph;
        it = S.graphs.emplace(key, exec).first;
    }
    if (hipGraphLaunch(it->second, stream) != hipSuccess) return fail(MCL_EDEVICE, "tick: graph launch failed");
    return note_uses();
}

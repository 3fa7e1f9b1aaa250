// Host runtime and C ABI of libmoss: input validation, device layout,
// step launches and state read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/moss.h"
#include "moss_internal.h"

using namespace moss;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace

namespace moss {

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

}  // namespace moss

namespace {

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(MOSS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of every device array inside the caller's workspace.
struct Layout {
    int32_t cap, n_lanes, n_roads, n_scen, n_qlanes, n_pend, n_veh, nblk;
    int64_t n_route;
    bool debug, trace, mlp, xy;
    size_t total;
    size_t S[8], Pr[8], J[8], ls[2], idv[2][2], tails, chunk, leave, jcount, joff, blk, jlist, jlane, jidx, jslane, jins_list, jins_lane, jcnt, jcur, lane_red, scal, lanes,
        roads, route, qlanes, q_hdep, q_head, q_end, q_id, q_dep, q_v0, q_ptr, q_next, vt_id, vt_dep,
        vt_rstart, vt_dist0, cnt, sumv, dbg[6], cursor, mlp_theta, mlp_norm, mlp_pack, mlp_sq,
        tr_feat, tr_label, road_ab, out_buf, trip_buf, ctl_idx, ctl_rec, ctl_ridx, ctl_rrec,
        succ_off, succ, conf_off, conf, conf_feed, busy;
    int64_t n_succ = 0, n_conf = 0;

    void plan()
    {
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t o = off;
            off += align_up(bytes ? bytes : 1);
            return o;
        };
        const size_t c = (size_t)std::max(cap, 1);
        const size_t cq = c + (size_t)std::max(n_qlanes, 0);
        // S[3] (id) and S[7] (v0) are not used: those fields live in idv
        for (int k = 0; k < 8; ++k)
            S[k] = take((k == 3 || k == 7) ? 4 : 4 * c);
        // proposals: one row per vehicle, then one insertion row per queue
        // lane; their id and v0 are idv's current buffer
        for (int k = 0; k < 8; ++k)
            Pr[k] = take((k == 3 || k == 7) ? 4 : 4 * cq);
        // id and v0 by step parity ([parity][0] id, [parity][1] v0)
        for (auto &b : idv)
            for (auto &x : b) x = take(4 * cq);
        for (auto &x : ls) x = take(4 * ((size_t)n_lanes + 1));
        tails = take(sizeof(Tail) * (size_t)n_lanes);
        leave = take(4 * (size_t)n_lanes);
        chunk = take(sizeof(int4) *
                     ((size_t)c / kMergeRows + (size_t)n_lanes / kMergeLanes + 3));
        jcount = take(4 * (size_t)n_lanes);
        joff = take(4 * ((size_t)n_lanes + 1));
        blk = take(8 * (size_t)nblk);
        const size_t tiles = (c + kUpdateRows - 1) / kUpdateRows;
        jlist = take(4 * tiles * kUpdateRows);
        jlane = take(4 * tiles * kUpdateRows);
        jcnt = take(4 * tiles);
        jidx = take(4 * c);
        jslane = take(4 * c);
        for (int k = 0; k < 8; ++k)
            J[k] = (k == 4) ? 0 : take(4 * c);      // J.lane is jslane
        jins_list = take(4 * (size_t)n_lanes);
        jins_lane = take(4 * (size_t)n_lanes);
        jcur = take(4 * (size_t)n_lanes);
        lane_red = take((size_t)n_lanes);
        scal = take(64);
        lanes = take(sizeof(LaneInfo) * (size_t)n_lanes);
        roads = take(sizeof(RoadInfo) * (size_t)n_roads);
        route = take(4 * ((size_t)n_route + 3 * (size_t)n_veh + 1));
        qlanes = take(4 * (size_t)n_qlanes);
        q_hdep = take(4 * (size_t)n_qlanes);
        q_head = take(4 * (size_t)n_lanes);
        q_end = take(4 * (size_t)n_lanes);
        q_id = take(4 * (size_t)n_pend);
        q_dep = take(4 * (size_t)n_pend);
        q_v0 = take(4 * (size_t)n_pend);
        q_ptr = take(4 * (size_t)n_pend);
        q_next = take(4 * (size_t)n_pend);
        vt_id = take(4 * (size_t)n_veh);
        vt_dep = take(4 * (size_t)n_veh);
        vt_rstart = take(4 * (size_t)n_veh);
        vt_dist0 = take(8 * (size_t)n_veh);
        cnt = take(8 * (size_t)kStripes * stripe_elems((int64_t)n_scen * C_N));
        sumv = take(8 * (size_t)kStripes * stripe_elems(n_scen));
        for (auto &x : dbg) x = take(debug ? 4 * c : 4);
        cursor = take(4 * c);
        mlp_theta = take(4 * (size_t)MOSS_MLP_PARAMS);
        mlp_norm = take(4 * (size_t)MOSS_MLP_NORM);
        mlp_pack = take(mlp ? mlp_pack_bytes() : 16);
        mlp_sq = take(8 * (size_t)kStripes * stripe_elems(n_scen));
        tr_feat = take(trace ? 4 * 8 * c : 4);
        tr_label = take(trace ? 4 * c : 4);
        road_ab = take(xy ? 32 * (size_t)n_roads : 32);
        ctl_idx = take(4 * (size_t)n_lanes);
        ctl_rec = take(sizeof(LaneInfo) * (size_t)n_lanes);
        ctl_ridx = take(4 * (size_t)n_roads);
        ctl_rrec = take(sizeof(RoadInfo) * (size_t)n_roads);
        // junction internal lanes (tiny placeholders without them)
        const bool jl = n_succ > 0 || n_conf > 0;
        succ_off = take(jl ? 4 * ((size_t)n_lanes + 1) : 4);
        succ = take(sizeof(Succ) * (size_t)std::max<int64_t>(n_succ, 1));
        conf_off = take(jl ? 4 * ((size_t)n_lanes + 1) : 4);
        conf = take(sizeof(Succ) * (size_t)std::max<int64_t>(n_conf, 1));
        conf_feed = take(4 * (size_t)std::max<int64_t>(n_conf, 1));
        busy = take(jl ? (size_t)n_lanes : 1);
        // staging of the read functions' results for host destinations
        out_buf = take(std::max(8 * (size_t)n_roads, xy ? 24 * c : (size_t)8));
        // staging of moss_read_trips for host destinations: status, travel
        // time and distance per vehicle
        trip_buf = take(16 * (size_t)n_veh);
        total = off;
    }
};

// The kernels address every workspace array through 32-bit byte offsets from
// the array's start, so no single array may reach 4 GiB: the route table
// (4 bytes per route entry, plus 3 per vehicle) and the trace's features (32
// bytes per vehicle) are the largest.
int check_array_sizes(const Layout &L)
{
    const double lim = 4294967296.0;
    if (4.0 * ((double)L.n_route + 3.0 * L.n_veh + 1.0) >= lim)
        return fail(MOSS_EINVAL, "route table of %lld entries exceeds 4 GiB",
                    (long long)L.n_route);
    if (32.0 * (double)std::max(L.cap, 1) + 32.0 * L.n_qlanes >= lim)
        return fail(MOSS_EINVAL, "%d vehicles exceed the per-array limit of 4 GiB", L.cap);
    if ((double)L.n_lanes * 32.0 >= lim || (double)L.n_roads * 32.0 >= lim)
        return fail(MOSS_EINVAL, "network tables exceed 4 GiB");
    return MOSS_OK;
}

bool finite_pos(float x) { return std::isfinite(x) && x > 0.0f; }
bool finite_nonneg(float x) { return std::isfinite(x) && x >= 0.0f; }

int validate(const moss_network *net, const moss_signals *sig, const moss_vehicles *veh,
             const moss_params *prm)
{
    if (!net || !sig || !veh || !prm)
        return fail(MOSS_EINVAL, "null input struct");
    if (net->n_nodes <= 0 || net->n_roads <= 0 || net->n_lanes <= 0 || veh->n < 0)
        return fail(MOSS_EINVAL, "empty network or negative vehicle count");
    if (!net->road_from || !net->road_to || !net->road_nlanes || !net->road_lane0 ||
        !net->road_length || !net->lane_vlim)
        return fail(MOSS_EINVAL, "missing network array");
    if (!sig->node_cycle || !sig->node_phase || !sig->node_offset || !sig->road_group)
        return fail(MOSS_EINVAL, "missing signal array");
    if (veh->n > 0 && (!veh->id || !veh->depart || !veh->v0 || !veh->route_off ||
                       !veh->route_roads))
        return fail(MOSS_EINVAL, "missing vehicle array");
    const int32_t n_scen = net->n_scen > 0 ? net->n_scen : 1;
    int64_t lanes = 0;
    for (int32_t r = 0; r < net->n_roads; ++r) {
        int32_t a = net->road_from[r], b = net->road_to[r];
        if (a < 0 || a >= net->n_nodes || b < 0 || b >= net->n_nodes)
            return fail(MOSS_EINVAL, "road %d: node out of range", r);
        if (net->road_nlanes[r] < 1 || net->road_nlanes[r] > 255)
            return fail(MOSS_EINVAL, "road %d: lane count %d not in 1..255", r,
                        net->road_nlanes[r]);
        if (net->road_lane0[r] != lanes)
            return fail(MOSS_EINVAL, "road %d: lanes not numbered road by road", r);
        if (!finite_pos(net->road_length[r]))
            return fail(MOSS_EINVAL, "road %d: length must be finite and > 0", r);
        lanes += net->road_nlanes[r];
        int8_t g = sig->road_group[r];
        if (g < -1)
            return fail(MOSS_EINVAL, "road %d: signal group < -1", r);
    }
    if (lanes != net->n_lanes)
        return fail(MOSS_EINVAL, "lane count %lld != n_lanes %d", (long long)lanes, net->n_lanes);
    {
        // junction internal lanes: all tables or none, lanes in range, at
        // most one successor per road
        const bool any = net->road_internal || net->lane_succ_off || net->lane_succ ||
                         net->lane_conf_off || net->lane_conf || net->lane_conf_feed;
        const bool all = net->road_internal && net->lane_succ_off && net->lane_conf_off &&
                         (net->lane_succ || net->lane_succ_off[net->n_lanes] == 0) &&
                         ((net->lane_conf && net->lane_conf_feed) ||
                          net->lane_conf_off[net->n_lanes] == 0);
        if (any && !all)
            return fail(MOSS_EINVAL, "junction lane tables must be given together");
        if (all) {
            std::vector<int32_t> road_of(net->n_lanes);
            for (int32_t r = 0; r < net->n_roads; ++r)
                for (int32_t k = 0; k < net->road_nlanes[r]; ++k)
                    road_of[net->road_lane0[r] + k] = r;
            const int32_t *so = net->lane_succ_off, *co = net->lane_conf_off;
            if (so[0] != 0 || co[0] != 0)
                return fail(MOSS_EINVAL, "junction lane offsets must start at 0");
            for (int32_t l = 0; l < net->n_lanes; ++l) {
                if (so[l + 1] < so[l] || co[l + 1] < co[l])
                    return fail(MOSS_EINVAL, "lane %d: junction lane offsets decrease", l);
                for (int32_t q = so[l]; q < so[l + 1]; ++q) {
                    const int32_t y = net->lane_succ[q];
                    if (y < 0 || y >= net->n_lanes)
                        return fail(MOSS_EINVAL, "lane %d: successor out of range", l);
                    if (net->road_from[road_of[y]] != net->road_to[road_of[l]])
                        return fail(MOSS_EINVAL, "lane %d: successor %d does not start where it "
                                                 "ends", l, y);
                    for (int32_t q2 = so[l]; q2 < q; ++q2)
                        if (road_of[net->lane_succ[q2]] == road_of[y])
                            return fail(MOSS_EINVAL, "lane %d: two successors on road %d", l,
                                        road_of[y]);
                }
                for (int32_t q = co[l]; q < co[l + 1]; ++q)
                    if (net->lane_conf[q] < 0 || net->lane_conf[q] >= net->n_lanes ||
                        net->lane_conf_feed[q] < 0 || net->lane_conf_feed[q] >= net->n_lanes)
                        return fail(MOSS_EINVAL, "lane %d: conflict entry out of range", l);
            }
        }
    }
    if ((net->node_x == nullptr) != (net->node_y == nullptr))
        return fail(MOSS_EINVAL, "node_x and node_y must be given together");
    if (net->node_x)
        for (int32_t j = 0; j < net->n_nodes; ++j)
            if (!std::isfinite(net->node_x[j]) || !std::isfinite(net->node_y[j]))
                return fail(MOSS_EINVAL, "node %d: coordinates must be finite", j);
    for (int32_t l = 0; l < net->n_lanes; ++l) {
        if (!finite_pos(net->lane_vlim[l]))
            return fail(MOSS_EINVAL, "lane %d: speed limit must be finite and > 0", l);
        if (net->lane_scen && (net->lane_scen[l] < 0 || net->lane_scen[l] >= n_scen))
            return fail(MOSS_EINVAL, "lane %d: scenario out of range", l);
    }
    for (int32_t j = 0; j < net->n_nodes; ++j) {
        if (sig->node_cycle[j] < 0)
            return fail(MOSS_EINVAL, "node %d: negative cycle", j);
        if (sig->node_cycle[j] > 0 && (sig->node_phase[j] <= 0 || sig->node_offset[j] < 0))
            return fail(MOSS_EINVAL, "node %d: phase must be > 0 and offset >= 0", j);
        if (sig->node_cycle[j] > 65535 || sig->node_phase[j] > 65535)
            return fail(MOSS_EINVAL, "node %d: cycle and phase must be < 65536 steps", j);
    }
    const moss_params &p = *prm;
    const float pos[] = {p.dt, p.a_max, p.b, p.length, p.b_max};
    for (float x : pos)
        if (!finite_pos(x))
            return fail(MOSS_EINVAL, "dt, a_max, b, length and b_max must be finite and > 0");
    const float nonneg[] = {p.s0, p.T, p.b_safe, p.politeness, p.d_look, p.b_mand,
                            p.tau_yield};
    for (float x : nonneg)
        if (!finite_nonneg(x))
            return fail(MOSS_EINVAL, "s0, T, b_safe, politeness, d_look, b_mand and tau_yield "
                                     "must be finite, >= 0");
    if (!std::isfinite(p.a_thr) || !std::isfinite(p.p_lc) || p.p_lc < 0.0f || p.p_lc > 1.0f)
        return fail(MOSS_EINVAL, "a_thr must be finite and p_lc in [0, 1]");
    if (p.h_look < 0 || p.t0 < 0)
        return fail(MOSS_EINVAL, "h_look and t0 must be >= 0");
    if (p.mode != MOSS_MODE_IDM && p.mode != MOSS_MODE_MLP)
        return fail(MOSS_EINVAL, "unknown mode %d", p.mode);
    if (p.mode == MOSS_MODE_MLP) {
        if (!p.mlp_theta || !p.mlp_norm)
            return fail(MOSS_EINVAL, "MLP mode needs mlp_theta and mlp_norm");
        for (int q = 0; q < MOSS_MLP_PARAMS; ++q)
            if (!std::isfinite(p.mlp_theta[q]))
                return fail(MOSS_EINVAL, "non-finite network parameter %d", q);
        for (int q = 0; q < MOSS_MLP_NORM; ++q)
            if (!std::isfinite(p.mlp_norm[q]))
                return fail(MOSS_EINVAL, "non-finite input description entry %d", q);
    }
    // vehicles
    std::vector<uint32_t> ids(veh->id, veh->id + veh->n);
    std::sort(ids.begin(), ids.end());
    for (int32_t i = 0; i < veh->n; ++i) {
        if (ids[i] == kNone)
            return fail(MOSS_EINVAL, "vehicle id 0xFFFFFFFF is reserved");
        if (i > 0 && ids[i] == ids[i - 1])
            return fail(MOSS_EINVAL, "duplicate vehicle id %u", ids[i]);
    }
    if (veh->n > 0 && veh->route_off[0] != 0)
        return fail(MOSS_EINVAL, "route_off[0] must be 0");
    for (int32_t i = 0; i < veh->n; ++i) {
        if (!finite_pos(veh->v0[i]))
            return fail(MOSS_EINVAL, "vehicle %d: v0 must be finite and > 0", i);
        int64_t a = veh->route_off[i], b = veh->route_off[i + 1];
        if (b <= a)
            return fail(MOSS_EINVAL, "vehicle %d: empty route", i);
        for (int64_t k = a; k < b; ++k) {
            int32_t r = veh->route_roads[k];
            if (r < 0 || r >= net->n_roads)
                return fail(MOSS_EINVAL, "vehicle %d: road out of range", i);
            if (k > a && net->road_to[veh->route_roads[k - 1]] != net->road_from[r])
                return fail(MOSS_EINVAL, "vehicle %d: route is not a chain of roads", i);
        }
        if (veh->placed && veh->placed[i]) {
            if (!veh->lane || !veh->cursor || !veh->s || !veh->v || !veh->a)
                return fail(MOSS_EINVAL, "missing placement arrays");
            int32_t l = veh->lane[i], c = veh->cursor[i];
            if (l < 0 || l >= net->n_lanes || c < 0 || c >= b - a)
                return fail(MOSS_EINVAL, "vehicle %d: lane or cursor out of range", i);
            int32_t r = veh->route_roads[a + c];
            if (l < net->road_lane0[r] || l >= net->road_lane0[r] + net->road_nlanes[r])
                return fail(MOSS_EINVAL, "vehicle %d: lane is not on route road %d", i, r);
            if (!std::isfinite(veh->s[i]) || !(veh->s[i] < net->road_length[r]) ||
                !finite_nonneg(veh->v[i]) || !std::isfinite(veh->a[i]))
                return fail(MOSS_EINVAL, "vehicle %d: bad position, speed or acceleration", i);
        }
    }
    // placed vehicles of one lane must not overlap: a follower's front at
    // most its leader's front less one vehicle length
    if (veh->placed) {
        std::vector<int32_t> pl;
        for (int32_t i = 0; i < veh->n; ++i)
            if (veh->placed[i])
                pl.push_back(i);
        std::sort(pl.begin(), pl.end(), [&](int32_t x, int32_t y) {
            if (veh->lane[x] != veh->lane[y]) return veh->lane[x] < veh->lane[y];
            if (veh->s[x] != veh->s[y]) return veh->s[x] < veh->s[y];
            return veh->id[x] < veh->id[y];
        });
        for (size_t k = 1; k < pl.size(); ++k) {
            const int32_t f = pl[k - 1], l = pl[k];
            if (veh->lane[f] == veh->lane[l] && !(veh->s[f] <= veh->s[l] - p.length))
                return fail(MOSS_EINVAL, "placed vehicles %u and %u overlap", veh->id[f],
                            veh->id[l]);
        }
    }
    return MOSS_OK;
}

}  // namespace

struct moss_sim {
    Layout lay;
    Dev dev;
    hipStream_t stream;
    int device;
    int parity;           // which lane_start buffer holds the current state
    int64_t t;            // host copy of the next step index
    int32_t n_scen;
    uint32_t err_seen;
    char *ws;
    // captured step loops: graph_steps steps starting at lane-start parity p
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    bool graphs_ok = true;
    int32_t graph_steps = 16;      // even; 0 = no graphs
    // control: host copy of the lane records, each signalised node's incoming
    // lanes (CSR), staging of the records a control call changes
    std::vector<LaneInfo> lanes_h;
    std::vector<int32_t> in_off, in_lanes;
    std::vector<uint8_t> node_sig;
    std::vector<int32_t> patch_idx;
    std::vector<LaneInfo> patch_rec;
    // host copy of the road records (closed-lane masks) and their staging
    std::vector<RoadInfo> roads_h;
    // junction internal lanes: host copy of the successor table (an entry
    // out of use by control carries road -1 - road) and its offsets
    std::vector<Succ> succ_h;
    std::vector<int32_t> succ_off_h;
    std::vector<int32_t> rpatch_idx;
    std::vector<RoadInfo> rpatch_rec;
};

static Dev step_dev(const moss_sim *h, int parity);


static void drop_graphs(moss_sim *h)
{
    for (auto &g : h->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

// Captures graph_steps steps (an even count, so that a replay returns to the
// same lane-start parity) on the simulator's stream into an executable
// graph.  The kernels read the step index and vehicle counts from device
// memory, so one graph serves every replay.
static hipError_t capture_graph(moss_sim *h, int parity, hipGraphExec_t *out)
{
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return e;
    int p = parity;
    hipError_t le = hipSuccess;
    for (int32_t k = 0; k < h->graph_steps && le == hipSuccess; ++k) {
        le = launch_step(step_dev(h, p), h->stream);
        p ^= 1;
    }
    e = hipStreamEndCapture(h->stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le;
    }
    if (e != hipSuccess)
        return e;
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

// Captures the step graphs of both lane-start parities now (capture records
// the launches without running them), so that the first moss_step that
// replays one does not pay for capture and instantiation.  A failed capture
// leaves graphs off: steps are then launched directly.
static void prepare_graphs(moss_sim *h)
{
    if (h->graph_steps <= 0 || !h->graphs_ok || h->stream == nullptr)
        return;
    for (int p = 0; p < 2; ++p) {
        if (h->graph[p])
            continue;
        if (capture_graph(h, p, &h->graph[p]) != hipSuccess) {
            (void)hipGetLastError();
            h->graph[p] = nullptr;
            h->graphs_ok = false;
            drop_graphs(h);
            return;
        }
    }
}

static void fill_dev(moss_sim *h)
{
    const Layout &L = h->lay;
    char *w = h->ws;
    Dev &d = h->dev;
    auto F = [&](size_t o) { return (float *)(w + o); };
    auto U = [&](size_t o) { return (uint32_t *)(w + o); };
    auto I = [&](size_t o) { return (int32_t *)(w + o); };
    SoA *sets[3] = {&d.S, &d.Pr, &d.J};
    const size_t *offs[3] = {L.S, L.Pr, L.J};
    for (int k = 0; k < 3; ++k) {
        SoA &x = *sets[k];
        x.s = F(offs[k][0]);
        x.v = F(offs[k][1]);
        x.a = F(offs[k][2]);
        x.id = U(offs[k][3]);
        x.lane = U(offs[k][4]);
        x.ptr = U(offs[k][5]);
        x.next = I(offs[k][6]);
        x.v0 = F(offs[k][7]);
    }
    d.J.lane = U(L.jslane);
    // id and v0 of parity 0 (step_dev selects the buffers of a parity)
    d.S.id = d.Pr.id = U(L.idv[0][0]);
    d.S.v0 = d.Pr.v0 = F(L.idv[0][1]);
    d.id_next = U(L.idv[1][0]);
    d.v0_next = F(L.idv[1][1]);
    d.n_lanes = L.n_lanes;
    d.n_scen = L.n_scen;
    d.cap = L.cap;
    d.n_qlanes = L.n_qlanes;
    d.lanes = (const LaneInfo *)(w + L.lanes);
    d.roads = (const RoadInfo *)(w + L.roads);
    d.route = I(L.route);
    d.tails = (Tail *)(w + L.tails);
    d.leave = I(L.leave);
    d.chunk = (int4 *)(w + L.chunk);
    d.jcount = I(L.jcount);
    d.joff = I(L.joff);
    d.blk = I(L.blk);
    d.jlist = U(L.jlist);
    d.jlane = U(L.jlane);
    d.jidx = U(L.jidx);
    d.jslane = U(L.jslane);
    d.jins_list = U(L.jins_list);
    d.jins_lane = U(L.jins_lane);
    d.jcnt = I(L.jcnt);
    d.jcur = I(L.jcur);
    d.lane_red = (uint8_t *)(w + L.lane_red);
    int32_t *sc = I(L.scal);
    d.n_cur = sc + 0;
    d.n_next = sc + 1;
    d.n_dbg = sc + 2;
    d.n_ins = (uint32_t *)(sc + 3);
    d.err = (uint32_t *)(sc + 5);
    d.t = (int64_t *)(sc + 8);
    d.qlanes = I(L.qlanes);
    d.q_hdep = I(L.q_hdep);
    d.q_head = I(L.q_head);
    d.q_end = I(L.q_end);
    d.q_id = U(L.q_id);
    d.q_dep = I(L.q_dep);
    d.q_v0 = F(L.q_v0);
    d.q_ptr = U(L.q_ptr);
    d.q_next = I(L.q_next);
    d.n_veh = L.n_veh;
    d.vt_id = U(L.vt_id);
    d.vt_dep = I(L.vt_dep);
    d.vt_rstart = U(L.vt_rstart);
    d.vt_dist0 = (const double *)(w + L.vt_dist0);
    d.succ_off = I(L.succ_off);
    d.succ = (const Succ *)(w + L.succ);
    d.conf_off = I(L.conf_off);
    d.conf = (const Succ *)(w + L.conf);
    d.conf_feed = I(L.conf_feed);
    d.busy = (uint8_t *)(w + L.busy);
    d.cnt = (unsigned long long *)(w + L.cnt);
    d.sumv = (unsigned long long *)(w + L.sumv);
    d.cnt_stride = stripe_elems((int64_t)h->n_scen * C_N);
    d.sv_stride = stripe_elems(h->n_scen);
    d.mlp_theta = F(L.mlp_theta);
    d.mlp_norm = F(L.mlp_norm);
    d.mlp_pack = w + L.mlp_pack;
    d.mlp_sq = (double *)(w + L.mlp_sq);
    d.tr_feat = F(L.tr_feat);
    d.tr_label = F(L.tr_label);
    d.d_id = U(L.dbg[0]);
    d.d_leader = U(L.dbg[1]);
    d.d_flags = I(L.dbg[2]);
    d.d_margin = F(L.dbg[3]);
    d.d_tl = U(L.dbg[4]);
    d.d_tf = U(L.dbg[5]);
}

static Dev step_dev(const moss_sim *h, int parity)
{
    Dev d = h->dev;
    d.ls_old = (const int32_t *)(h->ws + h->lay.ls[parity]);
    d.ls_new = (int32_t *)(h->ws + h->lay.ls[1 - parity]);
    d.S.id = d.Pr.id = (uint32_t *)(h->ws + h->lay.idv[parity][0]);
    d.S.v0 = d.Pr.v0 = (float *)(h->ws + h->lay.idv[parity][1]);
    d.id_next = (uint32_t *)(h->ws + h->lay.idv[1 - parity][0]);
    d.v0_next = (float *)(h->ws + h->lay.idv[1 - parity][1]);
    return d;
}

// Whether lane l lets a vehicle continue onto road rd: no successor list, or
// a successor on rd (junction internal lanes).
static bool lane_permits(const moss_network *net, int32_t l, int32_t rd)
{
    if (!net->lane_succ_off || net->lane_succ_off[l] == net->lane_succ_off[l + 1])
        return true;
    for (int32_t q = net->lane_succ_off[l]; q < net->lane_succ_off[l + 1]; ++q) {
        const int32_t y = net->lane_succ[q];
        if (y >= net->road_lane0[rd] && y < net->road_lane0[rd] + net->road_nlanes[rd])
            return true;
    }
    return false;
}

// Origin lane of pending vehicle i: among the lanes of its first road that
// continue along its route (all of them without junction lanes, or for a
// one-road route), the one of index id mod their number.
static int32_t origin_lane(const moss_network *net, const moss_vehicles *veh, int32_t i)
{
    const int64_t a = veh->route_off[i];
    const int32_t r0 = veh->route_roads[a], l0 = net->road_lane0[r0], n = net->road_nlanes[r0];
    int32_t ok[256], cnt = 0;
    if (veh->route_off[i + 1] - a > 1)
        for (int32_t k = 0; k < n; ++k)
            if (lane_permits(net, l0 + k, veh->route_roads[a + 1]))
                ok[cnt++] = l0 + k;
    if (cnt == 0)
        return l0 + (int32_t)(veh->id[i] % (uint32_t)n);
    return ok[veh->id[i] % (uint32_t)cnt];
}

static void plan_layout(const moss_network *net, const moss_vehicles *veh, const moss_params *prm,
                        Layout *L)
{
    L->n_lanes = net->n_lanes;
    L->n_roads = net->n_roads;
    L->n_scen = net->n_scen > 0 ? net->n_scen : 1;
    L->n_veh = veh->n;
    L->cap = veh->n;
    L->n_route = veh->n > 0 ? veh->route_off[veh->n] : 0;
    int32_t n_pl = 0;
    std::vector<char> is_q(net->n_lanes, 0);
    for (int32_t i = 0; i < veh->n; ++i) {
        if (veh->placed && veh->placed[i])
            ++n_pl;
        else
            is_q[origin_lane(net, veh, i)] = 1;
    }
    L->n_succ = net->lane_succ_off ? net->lane_succ_off[net->n_lanes] : 0;
    L->n_conf = net->lane_conf_off ? net->lane_conf_off[net->n_lanes] : 0;
    L->n_pend = veh->n - n_pl;
    L->n_qlanes = (int32_t)std::count(is_q.begin(), is_q.end(), 1);
    L->nblk = (net->n_lanes + kScanBlockLanes - 1) / kScanBlockLanes;
    L->debug = (prm->flags & MOSS_FLAG_DEBUG) != 0;
    L->trace = (prm->flags & MOSS_FLAG_TRACE) != 0;
    L->mlp = prm->mode == MOSS_MODE_MLP;
    L->xy = net->node_x != nullptr && net->node_y != nullptr;
    L->plan();
}

extern "C" {

const char *moss_last_error(void) { return g_err.c_str(); }

int moss_query_workspace(const moss_network *net, const moss_signals *sig,
                         const moss_vehicles *veh, const moss_params *prm, size_t *bytes)
{
    g_err.clear();
    if (!bytes)
        return fail(MOSS_EINVAL, "bytes is null");
    int rc = validate(net, sig, veh, prm);
    if (rc)
        return rc;
    Layout L;
    plan_layout(net, veh, prm, &L);
    rc = check_array_sizes(L);
    if (rc)
        return rc;
    *bytes = L.total;
    return MOSS_OK;
}

int moss_create(const moss_network *net, const moss_signals *sig, const moss_vehicles *veh,
                const moss_params *prm, void *d_ws, size_t ws_bytes, void *hip_stream,
                moss_sim **out)
{
    g_err.clear();
    if (!out)
        return fail(MOSS_EINVAL, "out is null");
    *out = nullptr;
    int rc = validate(net, sig, veh, prm);
    if (rc)
        return rc;
    if (!d_ws)
        return fail(MOSS_EINVAL, "workspace is null");
    Layout L;
    plan_layout(net, veh, prm, &L);
    rc = check_array_sizes(L);
    if (rc)
        return rc;
    if (ws_bytes < L.total)
        return fail(MOSS_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    if (((uintptr_t)d_ws & 255) != 0)
        return fail(MOSS_EINVAL, "workspace must be 256-byte aligned");

    hipPointerAttribute_t attr;
    HIP_TRY(hipPointerGetAttributes(&attr, d_ws));
    if (attr.type != hipMemoryTypeDevice)
        return fail(MOSS_EINVAL, "workspace is not device memory");
    HIP_TRY(hipSetDevice(attr.device));

    const int32_t NL = net->n_lanes, NR = net->n_roads, N = veh->n;
    const moss_params &p = *prm;

    // --- static tables
    std::vector<LaneInfo> lanes(NL);
    std::vector<RoadInfo> roads(NR);
    for (int32_t r = 0; r < NR; ++r) {
        roads[r] = {net->road_lane0[r], net->road_nlanes[r], net->road_length[r], 0};
        int32_t j = net->road_to[r];
        int8_t g = sig->road_group[r];
        bool signalised = g >= 0 && sig->node_cycle[j] > 0;
        for (int32_t k = 0; k < net->road_nlanes[r]; ++k) {
            int32_t l = net->road_lane0[r] + k;
            LaneInfo &li = lanes[l];
            std::memset(&li, 0, sizeof li);
            li.L = net->road_length[r];
            li.vlim = net->lane_vlim[l];
            li.lane0 = net->road_lane0[r];
            li.scen = net->lane_scen ? net->lane_scen[l] : 0;
            li.k = (uint8_t)k;
            li.nlanes = (uint8_t)net->road_nlanes[r];
            li.group = signalised ? g : (int8_t)-1;
            li.cycle = (uint16_t)(signalised ? sig->node_cycle[j] : 1);
            li.phase = (uint16_t)(signalised ? sig->node_phase[j] : 1);
            li.offset = (uint16_t)(signalised ? sig->node_offset[j] % sig->node_cycle[j] : 0);
            li.manual = -1;
            li.road = r;
            li.lflags = (net->road_internal && net->road_internal[r]) ? kLaneInternal : 0;
        }
    }

    // --- red lights at the first step: phase ((t + offset) mod cycle) div
    // phase_len differs from the road's group
    std::vector<uint8_t> red0(NL, 0);
    for (int32_t l = 0; l < NL; ++l)
        red0[l] = lane_flags_at(lanes[l], (uint32_t)p.t0);

    // --- routes, each followed by -1, the vehicle's departure step and its
    // arrival step (-1 until it arrives)
    std::vector<int32_t> route((size_t)L.n_route + 3 * (size_t)N + 1);
    std::vector<uint32_t> rstart(N);
    {
        size_t w = 0;
        for (int32_t i = 0; i < N; ++i) {
            rstart[i] = (uint32_t)w;
            for (int64_t k = veh->route_off[i]; k < veh->route_off[i + 1]; ++k)
                route[w++] = veh->route_roads[k];
            route[w++] = -1;
            route[w++] = veh->depart[i];
            route[w++] = -1;
        }
        route[w] = -1;
    }

    // --- placed vehicles in lane order
    std::vector<int32_t> placed;
    std::vector<int32_t> pend;
    for (int32_t i = 0; i < N; ++i)
        ((veh->placed && veh->placed[i]) ? placed : pend).push_back(i);
    std::sort(placed.begin(), placed.end(), [&](int32_t x, int32_t y) {
        if (veh->lane[x] != veh->lane[y]) return veh->lane[x] < veh->lane[y];
        if (veh->s[x] != veh->s[y]) return veh->s[x] < veh->s[y];
        return veh->id[x] < veh->id[y];
    });
    const int32_t NP = (int32_t)placed.size();
    std::vector<float> hs(NP), hv(NP), ha(NP), hv0(NP);
    std::vector<uint32_t> hid(NP), hlane(NP), hptr(NP);
    std::vector<int32_t> hnext(NP), ls(NL + 1, 0);
    for (int32_t k = 0; k < NP; ++k) {
        int32_t i = placed[k];
        hs[k] = veh->s[i];
        hv[k] = veh->v[i];
        ha[k] = veh->a[i];
        hv0[k] = veh->v0[i];
        hid[k] = veh->id[i];
        hlane[k] = (uint32_t)veh->lane[i];
        hptr[k] = rstart[i] + (uint32_t)veh->cursor[i];
        hnext[k] = route[hptr[k] + 1];
        ls[veh->lane[i] + 1]++;
    }
    for (int32_t l = 0; l < NL; ++l)
        ls[l + 1] += ls[l];

    // --- departure queues: origin lane, then (depart, id)
    auto origin = [&](int32_t i) { return origin_lane(net, veh, i); };
    std::vector<int32_t> olane(N, -1);
    for (int32_t i : pend)
        olane[i] = origin(i);
    std::sort(pend.begin(), pend.end(), [&](int32_t x, int32_t y) {
        if (olane[x] != olane[y]) return olane[x] < olane[y];
        if (veh->depart[x] != veh->depart[y]) return veh->depart[x] < veh->depart[y];
        return veh->id[x] < veh->id[y];
    });
    const int32_t NQ = (int32_t)pend.size();
    std::vector<uint32_t> qid(NQ), qptr(NQ);
    std::vector<int32_t> qdep(NQ), qnext(NQ), qhead(NL, 0), qend(NL, 0), qlanes;
    std::vector<float> qv0(NQ);
    for (int32_t k = 0; k < NQ; ++k) {
        int32_t i = pend[k];
        qid[k] = veh->id[i];
        qdep[k] = veh->depart[i];
        qv0[k] = veh->v0[i];
        qptr[k] = rstart[i];
        qnext[k] = route[rstart[i] + 1];
        qend[olane[i]]++;
    }
    {
        int32_t acc = 0;
        for (int32_t l = 0; l < NL; ++l) {
            qhead[l] = acc;
            acc += qend[l];
            qend[l] = acc;
            if (qend[l] > qhead[l])
                qlanes.push_back(l);
        }
    }

    // --- vehicle table by id
    std::vector<int32_t> byid(N);
    std::iota(byid.begin(), byid.end(), 0);
    std::sort(byid.begin(), byid.end(), [&](int32_t x, int32_t y) { return veh->id[x] < veh->id[y]; });
    std::vector<uint32_t> vtid(N), vtr(N);
    std::vector<int32_t> vtdep(N);
    std::vector<double> vtd0(N, 0.0);
    for (int32_t k = 0; k < N; ++k) {
        const int32_t i = byid[k];
        vtid[k] = veh->id[i];
        vtdep[k] = veh->depart[i];
        vtr[k] = rstart[i];
        // route distance where the vehicle enters the simulation: the road
        // lengths before its starting road (FP64, route order) plus its
        // starting position; 0 at a route start
        if (veh->placed && veh->placed[i]) {
            double d0 = 0.0;
            for (int32_t c = 0; c < veh->cursor[i]; ++c)
                d0 += (double)net->road_length[veh->route_roads[veh->route_off[i] + c]];
            vtd0[k] = d0 + (double)veh->s[i];
        }
    }

    moss_sim *h = new moss_sim();
    h->lay = L;
    h->ws = (char *)d_ws;
    h->stream = (hipStream_t)hip_stream;
    h->device = attr.device;
    h->parity = 0;
    h->t = p.t0;
    h->n_scen = L.n_scen;
    h->err_seen = 0;
    fill_dev(h);
    Params &P = h->dev.P;
    P.dt = p.dt;
    P.a_max = p.a_max;
    P.s0 = p.s0;
    P.T = p.T;
    P.len = p.length;
    P.b_max = p.b_max;
    P.b_safe = p.b_safe;
    P.pol = p.politeness;
    P.a_thr = p.a_thr;
    P.p_lc = p.p_lc;
    P.d_look = p.d_look;
    P.inv_tsab = (float)(1.0 / (2.0 * std::sqrt((double)p.a_max * (double)p.b)));
    P.inv_2bmax = (float)(1.0 / (2.0 * (double)p.b_max));
    P.h_look = p.h_look;
    P.b_mand = p.b_mand;
    P.tau_yield = p.tau_yield;
    P.key0 = (uint32_t)(p.seed & 0xFFFFFFFFu);
    P.key1 = (uint32_t)(p.seed >> 32);
    P.debug = L.debug ? 1u : 0u;
    P.trace = L.trace ? 1u : 0u;
    h->dev.mode = L.mlp ? 1 : 0;
    h->dev.junctions = net->lane_succ_off ? 1 : 0;

    hipStream_t st = h->stream;
    char *w = h->ws;
    auto up = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, st);
    };
    int32_t scal[16] = {0};
    scal[0] = NP;
    int64_t t0 = p.t0;
    std::memcpy(&scal[8], &t0, 8);
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(hipMemsetAsync(w, 0, L.total, st));
    chk(up(L.S[0], hs.data(), 4 * (size_t)NP));
    chk(up(L.S[1], hv.data(), 4 * (size_t)NP));
    chk(up(L.S[2], ha.data(), 4 * (size_t)NP));
    chk(up(L.idv[0][0], hid.data(), 4 * (size_t)NP));
    chk(up(L.S[4], hlane.data(), 4 * (size_t)NP));
    chk(up(L.S[5], hptr.data(), 4 * (size_t)NP));
    chk(up(L.S[6], hnext.data(), 4 * (size_t)NP));
    chk(up(L.idv[0][1], hv0.data(), 4 * (size_t)NP));
    chk(up(L.ls[0], ls.data(), 4 * (size_t)(NL + 1)));
    chk(up(L.scal, scal, sizeof scal));
    chk(up(L.lanes, lanes.data(), sizeof(LaneInfo) * NL));
    chk(up(L.lane_red, red0.data(), (size_t)NL));
    chk(up(L.roads, roads.data(), sizeof(RoadInfo) * NR));
    {
        // incoming lanes of each node, for signal control
        const int32_t NN = net->n_nodes;
        h->in_off.assign((size_t)NN + 1, 0);
        h->node_sig.assign((size_t)NN, 0);
        for (int32_t j = 0; j < NN; ++j)
            h->node_sig[j] = sig->node_cycle[j] > 0;
        for (int32_t r = 0; r < NR; ++r)
            h->in_off[net->road_to[r] + 1] += net->road_nlanes[r];
        for (int32_t j = 0; j < NN; ++j)
            h->in_off[j + 1] += h->in_off[j];
        h->in_lanes.resize((size_t)h->in_off[NN]);
        std::vector<int32_t> fill(h->in_off.begin(), h->in_off.end() - 1);
        for (int32_t r = 0; r < NR; ++r)
            for (int32_t k = 0; k < net->road_nlanes[r]; ++k)
                h->in_lanes[fill[net->road_to[r]]++] = net->road_lane0[r] + k;
        h->lanes_h = lanes;
        h->roads_h = roads;
    }
    if (L.xy) {
        // each road's segment (upstream node, downstream node) for positions
        std::vector<double> ab(4 * (size_t)NR);
        for (int32_t r = 0; r < NR; ++r) {
            ab[4 * r + 0] = net->node_x[net->road_from[r]];
            ab[4 * r + 1] = net->node_y[net->road_from[r]];
            ab[4 * r + 2] = net->node_x[net->road_to[r]];
            ab[4 * r + 3] = net->node_y[net->road_to[r]];
        }
        chk(up(L.road_ab, ab.data(), 8 * ab.size()));
    }
    std::vector<Succ> succ_keep;
    std::vector<int32_t> succ_off_keep;
    if (net->lane_succ_off) {
        // junction internal lanes: successors as (lane, road) pairs
        std::vector<int32_t> road_of(NL);
        for (int32_t r = 0; r < NR; ++r)
            for (int32_t k = 0; k < net->road_nlanes[r]; ++k)
                road_of[net->road_lane0[r] + k] = r;
        std::vector<Succ> sv((size_t)L.n_succ);
        for (int64_t q = 0; q < L.n_succ; ++q)
            sv[q] = Succ{net->lane_succ[q], road_of[net->lane_succ[q]]};
        std::vector<Succ> cv((size_t)L.n_conf);
        for (int64_t q = 0; q < L.n_conf; ++q)
            cv[q] = Succ{net->lane_conf[q], road_of[net->lane_conf[q]]};
        chk(up(L.succ_off, net->lane_succ_off, 4 * ((size_t)NL + 1)));
        chk(up(L.succ, sv.data(), sizeof(Succ) * sv.size()));
        succ_keep = sv;
        succ_off_keep.assign(net->lane_succ_off, net->lane_succ_off + NL + 1);
        chk(up(L.conf_off, net->lane_conf_off, 4 * ((size_t)NL + 1)));
        chk(up(L.conf, cv.data(), sizeof(Succ) * cv.size()));
        chk(up(L.conf_feed, net->lane_conf_feed, 4 * (size_t)L.n_conf));
    }
    chk(up(L.route, route.data(), 4 * route.size()));
    chk(up(L.qlanes, qlanes.data(), 4 * qlanes.size()));
    {
        std::vector<int32_t> hdep(qlanes.size());
        for (size_t q = 0; q < qlanes.size(); ++q)
            hdep[q] = qdep[qhead[qlanes[q]]];
        chk(up(L.q_hdep, hdep.data(), 4 * hdep.size()));
    }
    chk(up(L.q_head, qhead.data(), 4 * (size_t)NL));
    chk(up(L.q_end, qend.data(), 4 * (size_t)NL));
    chk(up(L.q_id, qid.data(), 4 * (size_t)NQ));
    chk(up(L.q_dep, qdep.data(), 4 * (size_t)NQ));
    chk(up(L.q_v0, qv0.data(), 4 * (size_t)NQ));
    chk(up(L.q_ptr, qptr.data(), 4 * (size_t)NQ));
    chk(up(L.q_next, qnext.data(), 4 * (size_t)NQ));
    chk(up(L.vt_id, vtid.data(), 4 * (size_t)N));
    chk(up(L.vt_dep, vtdep.data(), 4 * (size_t)N));
    chk(up(L.vt_rstart, vtr.data(), 4 * (size_t)N));
    chk(up(L.vt_dist0, vtd0.data(), 8 * (size_t)N));
    if (L.mlp) {
        chk(up(L.mlp_theta, p.mlp_theta, 4 * (size_t)MOSS_MLP_PARAMS));
        chk(up(L.mlp_norm, p.mlp_norm, 4 * (size_t)MOSS_MLP_NORM));
    }
    if (e == hipSuccess)
        e = launch_tails(step_dev(h, 0), st);
    if (e == hipSuccess && h->dev.junctions)
        e = launch_yield(step_dev(h, 0), st);
    if (e == hipSuccess && L.mlp)
        e = launch_mlp_pack(step_dev(h, 0), st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    h->succ_h.swap(succ_keep);
    h->succ_off_h.swap(succ_off_keep);
    if (e != hipSuccess) {
        delete h;
        return fail(MOSS_EDEVICE, "device setup failed: %s", hipGetErrorString(e));
    }
    prepare_graphs(h);
    *out = h;
    return MOSS_OK;
}

int moss_step(moss_sim *h, int32_t n)
{
    g_err.clear();
    if (!h)
        return fail(MOSS_EINVAL, "null handle");
    if (n < 0)
        return fail(MOSS_EINVAL, "negative step count");
    if (h->err_seen)
        return fail(MOSS_ESTATE, "device error word 0x%x", h->err_seen);
    if (h->t + n >= (int64_t)1 << 31)
        return fail(MOSS_EINVAL, "step index would exceed 2^31");
    HIP_TRY(hipSetDevice(h->device));
    int32_t left = n;
    // whole graphs first (not on the legacy null stream, which cannot capture)
    const int32_t gs = h->graph_steps;
    while (gs > 0 && left >= gs && h->graphs_ok && h->stream != nullptr) {
        hipGraphExec_t &g = h->graph[h->parity];
        if (!g && capture_graph(h, h->parity, &g) != hipSuccess) {
            (void)hipGetLastError();
            g = nullptr;
            h->graphs_ok = false;
            break;
        }
        HIP_TRY(hipGraphLaunch(g, h->stream));
        left -= gs;
        h->t += gs;
    }
    for (; left > 0; --left) {
        HIP_TRY(launch_step(step_dev(h, h->parity), h->stream));
        h->parity ^= 1;
        h->t += 1;
    }
    return MOSS_OK;
}

int moss_set_launch(moss_sim *h, const moss_launch *cfg)
{
    g_err.clear();
    if (!h || !cfg)
        return fail(MOSS_EINVAL, "null argument");
    if (cfg->graph_steps < 0 || cfg->graph_steps > 256 || (cfg->graph_steps & 1))
        return fail(MOSS_EINVAL, "graph_steps %d: even, 0..256", cfg->graph_steps);
    if (cfg->update_blocks < 0 || cfg->update_blocks > 65535)
        return fail(MOSS_EINVAL, "update_blocks %d: 0..65535", cfg->update_blocks);
    if (cfg->scatter_blocks < 0 || cfg->scatter_blocks > 65535)
        return fail(MOSS_EINVAL, "scatter_blocks %d: 0..65535", cfg->scatter_blocks);
    if (cfg->xcd_remap != 0 && cfg->xcd_remap != 1)
        return fail(MOSS_EINVAL, "xcd_remap %d: 0 or 1", cfg->xcd_remap);
    HIP_TRY(hipSetDevice(h->device));
    // replays already enqueued keep their own executable graphs alive until
    // they finish only if the stream is drained first
    HIP_TRY(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    h->graphs_ok = true;
    h->graph_steps = cfg->graph_steps;
    h->dev.upd_blocks = cfg->update_blocks;
    h->dev.jsc_blocks = cfg->scatter_blocks;
    h->dev.xcd_remap = cfg->xcd_remap;
    prepare_graphs(h);
    return MOSS_OK;
}

int moss_get_launch(const moss_sim *h, moss_launch *cfg)
{
    g_err.clear();
    if (!h || !cfg)
        return fail(MOSS_EINVAL, "null argument");
    cfg->graph_steps = h->graph_steps;
    cfg->update_blocks = h->dev.upd_blocks;
    cfg->scatter_blocks = h->dev.jsc_blocks;
    cfg->xcd_remap = h->dev.xcd_remap;
    return MOSS_OK;
}

int moss_step_timed(moss_sim *h, int32_t n, double *kernel_ms, int32_t capacity,
                    int32_t *n_kernels)
{
    g_err.clear();
    if (!h || !kernel_ms || !n_kernels)
        return fail(MOSS_EINVAL, "null argument");
    const int K = step_kernel_count();
    *n_kernels = K;
    if (capacity < K)
        return fail(MOSS_ENOMEM, "%d kernels, capacity %d", K, capacity);
    if (n < 0)
        return fail(MOSS_EINVAL, "negative step count");
    if (h->err_seen)
        return fail(MOSS_ESTATE, "device error word 0x%x", h->err_seen);
    if (h->t + n >= (int64_t)1 << 31)
        return fail(MOSS_EINVAL, "step index would exceed 2^31");
    HIP_TRY(hipSetDevice(h->device));
    // steps are enqueued back to back in groups of kChunk with their events
    // (K + 1 per step) and synchronised once per group, so that a step's
    // first kernel does not include the host's submission after a sync
    constexpr int kChunk = 64;
    std::vector<hipEvent_t> ev((size_t)(K + 1) * kChunk, nullptr);
    int rc = MOSS_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            rc = fail(MOSS_EDEVICE, "event creation failed");
            break;
        }
    for (int k = 0; k < K; ++k)
        kernel_ms[k] = 0.0;
    for (int32_t s0 = 0; s0 < n && rc == MOSS_OK; s0 += kChunk) {
        const int m = std::min<int32_t>(kChunk, n - s0);
        hipError_t e = hipSuccess;
        int j = 0;
        for (; j < m && e == hipSuccess; ++j) {
            e = launch_step(step_dev(h, h->parity), h->stream, &ev[(size_t)j * (K + 1)]);
            h->parity ^= 1;
            h->t += 1;
        }
        if (e == hipSuccess)
            e = hipEventSynchronize(ev[(size_t)(m - 1) * (K + 1) + K]);
        if (e != hipSuccess) {
            rc = fail(MOSS_EDEVICE, "timed step failed: %s", hipGetErrorString(e));
            break;
        }
        for (j = 0; j < m; ++j)
            for (int k = 0; k < K; ++k) {
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, ev[(size_t)j * (K + 1) + k],
                                          ev[(size_t)j * (K + 1) + k + 1]);
                kernel_ms[k] += ms;
            }
    }
    for (auto &e : ev)
        if (e)
            (void)hipEventDestroy(e);
    // kernels this workload does not launch: the gap between their two
    // events is event overhead, not work
    for (int k = 0; k < K; ++k) {
        const std::string name = step_kernel_name(k);
        if ((name == "k_yield" && !h->dev.junctions) ||
            (name == "k_scan_reduce" && h->dev.n_lanes <= step_scan_block_lanes()))
            kernel_ms[k] = 0.0;
    }
    return rc;
}

const char *moss_kernel_name(int32_t i) { return step_kernel_name(i); }

static int sync_and_check(moss_sim *h)
{
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(hipStreamSynchronize(h->stream));
    uint32_t err = 0;
    HIP_TRY(hipMemcpy(&err, h->dev.err, 4, hipMemcpyDeviceToHost));
    h->err_seen |= err;
    return MOSS_OK;
}

// Copies made by the read functions run on the simulator's stream, so that
// they are ordered before every later step (whose kernels rewrite the buffers
// being read), and the read waits for them before it returns.  A device
// destination may be memory that work on another stream used until just now
// (a caching allocator's block), so device reads drain the device first.
struct ReadCopies {
    moss_sim *h;
    hipMemcpyKind kind;
    hipError_t e;
    ReadCopies(moss_sim *h_, bool device)
        : h(h_), kind(device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost), e(hipSuccess)
    {
        if (device)
            e = hipDeviceSynchronize();
    }
    void copy(void *dst, const void *src, size_t bytes)
    {
        if (e == hipSuccess && dst && bytes)
            e = hipMemcpyAsync(dst, src, bytes, kind, h->stream);
    }
    hipError_t finish()
    {
        if (e == hipSuccess)
            e = hipStreamSynchronize(h->stream);
        return e;
    }
};

int moss_read_state(moss_sim *h, moss_state_out *out)
{
    g_err.clear();
    if (!h || !out)
        return fail(MOSS_EINVAL, "null argument");
    int rc = sync_and_check(h);
    if (rc)
        return rc;
    int32_t n = 0;
    HIP_TRY(hipMemcpy(&n, h->dev.n_cur, 4, hipMemcpyDeviceToHost));
    out->n = n;
    out->t = h->t;
    if (n > out->capacity)
        return fail(MOSS_ENOMEM, "%d active vehicles, capacity %d", n, out->capacity);
    const size_t b = 4 * (size_t)n;
    const Dev dc = step_dev(h, h->parity);
    const SoA &S = dc.S;
    if (n > 0) {
        ReadCopies rc_(h, out->device != 0);
        rc_.copy(out->id, S.id, b);
        rc_.copy(out->lane, S.lane, b);
        rc_.copy(out->s, S.s, b);
        rc_.copy(out->v, S.v, b);
        rc_.copy(out->a, S.a, b);
        if (out->cursor && rc_.e == hipSuccess) {
            int32_t *tmp = (int32_t *)(h->ws + h->lay.cursor);
            rc_.e = launch_cursor(dc, S.id, S.ptr, tmp, n, h->stream);
            rc_.copy(out->cursor, tmp, b);
        }
        HIP_TRY(rc_.finish());
    }
    if (h->err_seen)
        return fail(MOSS_ESTATE, "device error word 0x%x", h->err_seen);
    return MOSS_OK;
}

// Per-scenario sums of the kStripes copies of a double observable, added in
// stripe order (a fixed order, so that a read is reproducible for a given
// device state).
static hipError_t sum_stripes(const moss_sim *h, const double *dev, double *out)
{
    const size_t st = (size_t)h->dev.sv_stride;
    std::vector<double> all(kStripes * st);
    hipError_t e = hipMemcpy(all.data(), dev, 8 * all.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return e;
    for (int32_t q = 0; q < h->n_scen; ++q) {
        double s = 0.0;
        for (int k = 0; k < kStripes; ++k)
            s += all[k * st + q];
        out[q] = s;
    }
    return hipSuccess;
}

int moss_read_counters(moss_sim *h, int64_t *counters, double *sum_v, uint32_t *error_word)
{
    g_err.clear();
    if (!h)
        return fail(MOSS_EINVAL, "null handle");
    int rc = sync_and_check(h);
    if (rc)
        return rc;
    if (counters) {
        const size_t m = (size_t)h->n_scen * C_N, st = (size_t)h->dev.cnt_stride;
        std::vector<unsigned long long> all(kStripes * st);
        HIP_TRY(hipMemcpy(all.data(), h->dev.cnt, 8 * all.size(), hipMemcpyDeviceToHost));
        for (size_t q = 0; q < m; ++q) {
            unsigned long long s = 0;
            for (int k = 0; k < kStripes; ++k)
                s += all[k * st + q];
            counters[q] = (int64_t)s;
        }
    }
    if (sum_v) {
        // integer stripes: exact in any order; the total in m/s rounded once
        const size_t st = (size_t)h->dev.sv_stride;
        std::vector<unsigned long long> all(kStripes * st);
        HIP_TRY(hipMemcpy(all.data(), h->dev.sumv, 8 * all.size(), hipMemcpyDeviceToHost));
        for (int32_t q = 0; q < h->n_scen; ++q) {
            unsigned long long s = 0;
            for (int k = 0; k < kStripes; ++k)
                s += all[k * st + q];
            sum_v[q] = (double)s / 1048576.0;
        }
    }
    if (error_word)
        *error_word = h->err_seen;
    return MOSS_OK;
}

int moss_read_pending(moss_sim *h, int32_t capacity, uint32_t *id, int32_t *n)
{
    g_err.clear();
    if (!h || !n)
        return fail(MOSS_EINVAL, "null argument");
    int rc = sync_and_check(h);
    if (rc)
        return rc;
    const int32_t nl = h->lay.n_lanes, np = h->lay.n_pend;
    *n = 0;
    if (np == 0)
        return MOSS_OK;
    // each lane's queue is q_id[q_head[l] .. q_end[l]); insertion advances the head
    std::vector<int32_t> head(nl), end(nl);
    std::vector<uint32_t> qid(np);
    HIP_TRY(hipMemcpy(head.data(), h->dev.q_head, 4 * (size_t)nl, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(end.data(), h->dev.q_end, 4 * (size_t)nl, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(qid.data(), h->dev.q_id, 4 * (size_t)np, hipMemcpyDeviceToHost));
    int32_t m = 0;
    for (int32_t l = 0; l < nl; ++l)
        m += end[l] - head[l];
    *n = m;
    if (m > capacity)
        return fail(MOSS_ENOMEM, "%d pending vehicles, capacity %d", m, capacity);
    if (m > 0 && !id)
        return fail(MOSS_EINVAL, "null id buffer");
    int32_t k = 0;
    for (int32_t l = 0; l < nl; ++l)
        for (int32_t q = head[l]; q < end[l]; ++q)
            id[k++] = qid[q];
    return MOSS_OK;
}

int moss_read_debug(moss_sim *h, int32_t capacity, uint32_t *id, uint32_t *leader,
                    int32_t *flags, float *margin, uint32_t *t_leader, uint32_t *t_follower,
                    int32_t *n)
{
    g_err.clear();
    if (!h || !n)
        return fail(MOSS_EINVAL, "null argument");
    if (!h->lay.debug)
        return fail(MOSS_EINVAL, "created without MOSS_FLAG_DEBUG");
    int rc = sync_and_check(h);
    if (rc)
        return rc;
    int32_t m = 0;
    HIP_TRY(hipMemcpy(&m, h->dev.n_dbg, 4, hipMemcpyDeviceToHost));
    *n = m;
    if (m > capacity)
        return fail(MOSS_ENOMEM, "%d rows, capacity %d", m, capacity);
    const size_t b = 4 * (size_t)m;
    if (m > 0) {
        if (id) HIP_TRY(hipMemcpy(id, h->dev.d_id, b, hipMemcpyDeviceToHost));
        if (leader) HIP_TRY(hipMemcpy(leader, h->dev.d_leader, b, hipMemcpyDeviceToHost));
        if (flags) HIP_TRY(hipMemcpy(flags, h->dev.d_flags, b, hipMemcpyDeviceToHost));
        if (margin) HIP_TRY(hipMemcpy(margin, h->dev.d_margin, b, hipMemcpyDeviceToHost));
        if (t_leader) HIP_TRY(hipMemcpy(t_leader, h->dev.d_tl, b, hipMemcpyDeviceToHost));
        if (t_follower) HIP_TRY(hipMemcpy(t_follower, h->dev.d_tf, b, hipMemcpyDeviceToHost));
    }
    return MOSS_OK;
}

int moss_read_trace(moss_sim *h, int32_t capacity, int32_t device, float *feat, float *label,
                    int32_t *n)
{
    g_err.clear();
    if (!h || !n)
        return fail(MOSS_EINVAL, "null argument");
    if (!h->lay.trace)
        return fail(MOSS_EINVAL, "created without MOSS_FLAG_TRACE");
    int rc = sync_and_check(h);
    if (rc)
        return rc;
    int32_t m = 0;
    HIP_TRY(hipMemcpy(&m, h->dev.n_dbg, 4, hipMemcpyDeviceToHost));
    *n = m;
    if (m > capacity)
        return fail(MOSS_ENOMEM, "%d rows, capacity %d", m, capacity);
    if (m > 0) {
        ReadCopies rc_(h, device != 0);
        rc_.copy(feat, h->dev.tr_feat, 4 * 8 * (size_t)m);
        rc_.copy(label, h->dev.tr_label, 4 * (size_t)m);
        HIP_TRY(rc_.finish());
    }
    return MOSS_OK;
}

// Uploads the staged lane records and patches them on the simulator's
// stream (ordered with the steps around it).
static int upload_patch(moss_sim *h)
{
    const int32_t n = (int32_t)h->patch_idx.size();
    if (n == 0)
        return MOSS_OK;
    HIP_TRY(hipSetDevice(h->device));
    int32_t *di = (int32_t *)(h->ws + h->lay.ctl_idx);
    LaneInfo *dr = (LaneInfo *)(h->ws + h->lay.ctl_rec);
    // the staging area may still be read by a patch enqueued before
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpyAsync(di, h->patch_idx.data(), 4 * (size_t)n, hipMemcpyHostToDevice,
                           h->stream));
    HIP_TRY(hipMemcpyAsync(dr, h->patch_rec.data(), sizeof(LaneInfo) * (size_t)n,
                           hipMemcpyHostToDevice, h->stream));
    HIP_TRY(launch_lane_patch(step_dev(h, h->parity), di, dr, n, h->stream));
    // the yield flags depend on the red flags just rewritten
    if (h->dev.junctions)
        HIP_TRY(launch_yield(step_dev(h, h->parity), h->stream));
    // the host staging vectors are reused by the next call
    HIP_TRY(hipStreamSynchronize(h->stream));
    return MOSS_OK;
}

// Each changed lane once (a lane named twice carries the last change), with
// its final record.
static int stage_and_upload(moss_sim *h)
{
    std::sort(h->patch_idx.begin(), h->patch_idx.end());
    h->patch_idx.erase(std::unique(h->patch_idx.begin(), h->patch_idx.end()),
                       h->patch_idx.end());
    h->patch_rec.clear();
    for (int32_t l : h->patch_idx)
        h->patch_rec.push_back(h->lanes_h[l]);
    return upload_patch(h);
}

int moss_set_signal_phase(moss_sim *h, const int32_t *node, const int32_t *phase, int32_t n)
{
    g_err.clear();
    if (!h || (n > 0 && (!node || !phase)) || n < 0)
        return fail(MOSS_EINVAL, "null argument or negative count");
    const int32_t NN = (int32_t)h->node_sig.size();
    for (int32_t i = 0; i < n; ++i) {
        if (node[i] < 0 || node[i] >= NN)
            return fail(MOSS_EINVAL, "node %d out of range", node[i]);
        if (!h->node_sig[node[i]])
            return fail(MOSS_EINVAL, "node %d has no signal", node[i]);
        if (phase[i] < -1 || phase[i] > 32767)
            return fail(MOSS_EINVAL, "node %d: phase %d not in -1..32767", node[i], phase[i]);
    }
    h->patch_idx.clear();
    for (int32_t i = 0; i < n; ++i)
        for (int32_t q = h->in_off[node[i]]; q < h->in_off[node[i] + 1]; ++q) {
            const int32_t l = h->in_lanes[q];
            h->lanes_h[l].manual = (int16_t)phase[i];
            h->patch_idx.push_back(l);
        }
    return stage_and_upload(h);
}

int moss_set_lane_turns(moss_sim *h, const int32_t *lane, const int32_t *road,
                        const int32_t *allowed, int32_t n)
{
    g_err.clear();
    if (!h || (n > 0 && (!lane || !road || !allowed)) || n < 0)
        return fail(MOSS_EINVAL, "null argument or negative count");
    if (h->succ_off_h.empty())
        return fail(MOSS_EINVAL, "the network has no junction lanes");
    const int32_t NL = (int32_t)h->succ_off_h.size() - 1;
    std::vector<int32_t> entry(n);
    for (int32_t i = 0; i < n; ++i) {
        if (lane[i] < 0 || lane[i] >= NL)
            return fail(MOSS_EINVAL, "lane %d out of range", lane[i]);
        entry[i] = -1;
        for (int32_t q = h->succ_off_h[lane[i]]; q < h->succ_off_h[lane[i] + 1]; ++q) {
            const int32_t r = h->succ_h[q].road;
            if ((r >= 0 ? r : -1 - r) == road[i])
                entry[i] = q;
        }
        if (entry[i] < 0)
            return fail(MOSS_EINVAL, "lane %d has no successor on road %d", lane[i], road[i]);
    }
    for (int32_t i = 0; i < n; ++i) {
        Succ &sx = h->succ_h[entry[i]];
        const int32_t r = sx.road >= 0 ? sx.road : -1 - sx.road;
        sx.road = allowed[i] ? r : -1 - r;
    }
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(h->ws + h->lay.succ, h->succ_h.data(), sizeof(Succ) * h->succ_h.size(),
                      hipMemcpyHostToDevice));
    return MOSS_OK;
}

int moss_set_lane_closed(moss_sim *h, const int32_t *lane, const int32_t *closed, int32_t n)
{
    g_err.clear();
    if (!h || (n > 0 && (!lane || !closed)) || n < 0)
        return fail(MOSS_EINVAL, "null argument or negative count");
    const int32_t NL = (int32_t)h->lanes_h.size();
    for (int32_t i = 0; i < n; ++i)
        if (lane[i] < 0 || lane[i] >= NL)
            return fail(MOSS_EINVAL, "lane %d out of range", lane[i]);
    // the masks after the whole batch, checked before anything changes
    std::map<int32_t, uint32_t> mask;
    for (int32_t i = 0; i < n; ++i) {
        const LaneInfo &li = h->lanes_h[lane[i]];
        if (!mask.count(li.road))
            mask[li.road] = h->roads_h[li.road].closed;
        if (li.nlanes > 32 && closed[i])
            return fail(MOSS_EINVAL, "lane %d: roads of more than 32 lanes cannot close lanes",
                        lane[i]);
        const uint32_t bit = li.nlanes > 32 ? 0u : 1u << li.k;
        mask[li.road] = closed[i] ? (mask[li.road] | bit) : (mask[li.road] & ~bit);
    }
    for (const auto &rm : mask) {
        const int32_t nl = h->roads_h[rm.first].nlanes;
        const uint32_t all = nl >= 32 ? 0xFFFFFFFFu : ((1u << nl) - 1u);
        if ((rm.second & all) == all)
            return fail(MOSS_EINVAL, "road %d would have no open lane", rm.first);
    }
    h->patch_idx.clear();
    for (int32_t i = 0; i < n; ++i) {
        uint8_t &lf = h->lanes_h[lane[i]].lflags;
        lf = (uint8_t)(closed[i] ? (lf | kLaneClosed) : (lf & ~kLaneClosed));
        h->patch_idx.push_back(lane[i]);
    }
    h->rpatch_idx.clear();
    h->rpatch_rec.clear();
    for (const auto &rm : mask) {
        h->roads_h[rm.first].closed = rm.second;
        h->rpatch_idx.push_back(rm.first);
        h->rpatch_rec.push_back(h->roads_h[rm.first]);
    }
    const int32_t nr = (int32_t)h->rpatch_idx.size();
    if (nr > 0) {
        HIP_TRY(hipSetDevice(h->device));
        int32_t *di = (int32_t *)(h->ws + h->lay.ctl_ridx);
        RoadInfo *dr = (RoadInfo *)(h->ws + h->lay.ctl_rrec);
        HIP_TRY(hipStreamSynchronize(h->stream));
        HIP_TRY(hipMemcpyAsync(di, h->rpatch_idx.data(), 4 * (size_t)nr, hipMemcpyHostToDevice,
                               h->stream));
        HIP_TRY(hipMemcpyAsync(dr, h->rpatch_rec.data(), sizeof(RoadInfo) * (size_t)nr,
                               hipMemcpyHostToDevice, h->stream));
        HIP_TRY(launch_road_patch(step_dev(h, h->parity), di, dr, nr, h->stream));
    }
    int32_t any = 0;
    for (const RoadInfo &rd : h->roads_h)
        any |= rd.closed != 0u;
    const int rc = stage_and_upload(h);
    if (rc)
        return rc;
    if (any != h->dev.closures) {
        // the step's update kernel changes: graphs captured with the other
        // one are redone
        HIP_TRY(hipStreamSynchronize(h->stream));
        drop_graphs(h);
        h->dev.closures = any;
        h->graphs_ok = true;
        prepare_graphs(h);
    }
    return MOSS_OK;
}

int moss_set_lane_vlim(moss_sim *h, const int32_t *lane, const float *vlim, int32_t n)
{
    g_err.clear();
    if (!h || (n > 0 && (!lane || !vlim)) || n < 0)
        return fail(MOSS_EINVAL, "null argument or negative count");
    const int32_t NL = (int32_t)h->lanes_h.size();
    for (int32_t i = 0; i < n; ++i) {
        if (lane[i] < 0 || lane[i] >= NL)
            return fail(MOSS_EINVAL, "lane %d out of range", lane[i]);
        if (!finite_pos(vlim[i]))
            return fail(MOSS_EINVAL, "lane %d: speed limit must be finite and > 0", lane[i]);
    }
    h->patch_idx.clear();
    for (int32_t i = 0; i < n; ++i) {
        h->lanes_h[lane[i]].vlim = vlim[i];
        h->patch_idx.push_back(lane[i]);
    }
    return stage_and_upload(h);
}

int moss_read_road_stats(moss_sim *h, int32_t device, int32_t *count, float *mean_v)
{
    g_err.clear();
    if (!h)
        return fail(MOSS_EINVAL, "null handle");
    int rc = sync_and_check(h);
    if (rc)
        return rc;
    const int32_t R = h->lay.n_roads;
    const Dev d = step_dev(h, h->parity);
    if (device) {
        HIP_TRY(hipDeviceSynchronize());     // destinations may have been in use elsewhere
        HIP_TRY(launch_road_stats(d, R, count, mean_v, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    } else {
        int32_t *dc = (int32_t *)(h->ws + h->lay.out_buf);
        float *dm = (float *)(dc + R);
        HIP_TRY(launch_road_stats(d, R, dc, dm, h->stream));
        ReadCopies rc_(h, false);
        rc_.copy(count, dc, 4 * (size_t)R);
        rc_.copy(mean_v, dm, 4 * (size_t)R);
        HIP_TRY(rc_.finish());
    }
    if (h->err_seen)
        return fail(MOSS_ESTATE, "device error word 0x%x", h->err_seen);
    return MOSS_OK;
}

int moss_read_positions(moss_sim *h, int32_t capacity, int32_t device, double *x, double *y,
                        double *heading, int32_t *n)
{
    g_err.clear();
    if (!h || !n || !x || !y || !heading)
        return fail(MOSS_EINVAL, "null argument");
    if (!h->lay.xy)
        return fail(MOSS_EINVAL, "created without node coordinates (node_x, node_y)");
    int rc = sync_and_check(h);
    if (rc)
        return rc;
    int32_t m = 0;
    HIP_TRY(hipMemcpy(&m, h->dev.n_cur, 4, hipMemcpyDeviceToHost));
    *n = m;
    if (m > capacity)
        return fail(MOSS_ENOMEM, "%d active vehicles, capacity %d", m, capacity);
    const Dev d = step_dev(h, h->parity);
    const double *ab = (const double *)(h->ws + h->lay.road_ab);
    if (m > 0) {
        if (device) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(launch_positions(d, m, ab, x, y, heading, h->stream));
            HIP_TRY(hipStreamSynchronize(h->stream));
        } else {
            double *bx = (double *)(h->ws + h->lay.out_buf);
            double *by = bx + m, *bh = by + m;
            HIP_TRY(launch_positions(d, m, ab, bx, by, bh, h->stream));
            ReadCopies rc_(h, false);
            rc_.copy(x, bx, 8 * (size_t)m);
            rc_.copy(y, by, 8 * (size_t)m);
            rc_.copy(heading, bh, 8 * (size_t)m);
            HIP_TRY(rc_.finish());
        }
    }
    if (h->err_seen)
        return fail(MOSS_ESTATE, "device error word 0x%x", h->err_seen);
    return MOSS_OK;
}

int moss_read_trips(moss_sim *h, int32_t capacity, int32_t device, uint32_t *id,
                    int32_t *status, int32_t *travel_time, double *distance, int32_t *n)
{
    g_err.clear();
    if (!h || !n)
        return fail(MOSS_EINVAL, "null argument");
    const int32_t N = h->lay.n_veh;
    *n = N;
    if (capacity < N)
        return fail(MOSS_ENOMEM, "%d vehicles, capacity %d", N, capacity);
    int rc = sync_and_check(h);
    if (rc)
        return rc;
    if (N == 0)
        return MOSS_OK;
    int32_t n_act = 0;
    HIP_TRY(hipMemcpy(&n_act, h->dev.n_cur, 4, hipMemcpyDeviceToHost));
    const Dev dc = step_dev(h, h->parity);
    // device destinations are written in place; host ones are staged
    char *tb = h->ws + h->lay.trip_buf;
    int32_t *d_st = device && status ? status : (int32_t *)tb;
    int32_t *d_tt = device && travel_time ? travel_time : (int32_t *)(tb + 4 * (size_t)N);
    double *d_ds = device && distance ? distance : (double *)(tb + 8 * (size_t)N);
    ReadCopies rc_(h, device != 0);
    if (rc_.e == hipSuccess)
        rc_.e = launch_trips(dc, n_act, d_st, d_tt, d_ds, h->stream);
    rc_.copy(id, dc.vt_id, 4 * (size_t)N);
    if (!device) {
        rc_.copy(status, d_st, 4 * (size_t)N);
        rc_.copy(travel_time, d_tt, 4 * (size_t)N);
        rc_.copy(distance, d_ds, 8 * (size_t)N);
    }
    HIP_TRY(rc_.finish());
    if (h->err_seen)
        return fail(MOSS_ESTATE, "device error word 0x%x", h->err_seen);
    return MOSS_OK;
}

int moss_read_mlp_error(moss_sim *h, double *sum_sq)
{
    g_err.clear();
    if (!h || !sum_sq)
        return fail(MOSS_EINVAL, "null argument");
    int rc = sync_and_check(h);
    if (rc)
        return rc;
    HIP_TRY(sum_stripes(h, h->dev.mlp_sq, sum_sq));
    return MOSS_OK;
}

int moss_destroy(moss_sim *h)
{
    g_err.clear();
    if (!h)
        return fail(MOSS_EINVAL, "null handle");
    if (h->device >= 0) {
        (void)hipSetDevice(h->device);
        (void)hipStreamSynchronize(h->stream);
        drop_graphs(h);
    }
    delete h;
    return MOSS_OK;
}

}  // extern "C"

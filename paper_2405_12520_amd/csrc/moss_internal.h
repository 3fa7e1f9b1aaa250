// Internal layout shared by the host runtime and the kernels of libmoss.
//
// Vehicle state is a structure of arrays kept in lane order: lane 0's
// vehicles by ascending front position, then lane 1's, ...; lane_start[l]
// gives the first row of lane l.  This is the per-lane spatial index of the
// paper's prepare phase (Sec. III-A), stored as a compact sorted array
// instead of linked lists so that the update phase reads it with coalesced
// loads and finds in-lane neighbours at row +-1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace moss {

constexpr uint32_t kNone = 0xFFFFFFFFu;      // "no vehicle" id
constexpr uint32_t kJoinBit = 0x80000000u;   // proposal lane: vehicle leaves its lane

// Per-lane constants, 32 bytes, read with one broadcast load per lane.  The
// fixed-time plan of the downstream junction is folded in (group < 0: the
// lane's road never waits for a signal).
struct LaneInfo {
    float L;            // road length
    float vlim;         // speed limit
    int32_t lane0;      // first lane of the road
    int32_t scen;       // scenario of the lane
    uint8_t k;          // index in the road
    uint8_t nlanes;
    int8_t group;       // signal group of the road at its downstream node, -1 none
    uint8_t lflags;     // kLaneClosed (control: closed to entering vehicles), kLaneInternal
    uint16_t cycle, phase, offset;         // plan of the downstream node (offset < cycle)
    int16_t manual;     // phase held by signal control, -1: the fixed-time plan
    int32_t road;
};

constexpr uint8_t kLaneClosed = 1u, kLaneInternal = 2u;

// Red light for the lanes of a road at step t: the road waits unless the
// phase its downstream junction shows (held by control, else of the
// fixed-time plan) is its group.
__host__ __device__ inline bool lane_red_at(const LaneInfo &li, uint32_t t)
{
    if (li.group < 0)
        return false;
    const int ph = li.manual >= 0 ? (int)li.manual
                                  : (int)(((t + (uint32_t)li.offset) % (uint32_t)li.cycle) /
                                          (uint32_t)li.phase);
    return ph != (int)li.group;
}

// Per-road constants used when following a route.
struct RoadInfo {
    int32_t lane0;
    int32_t nlanes;
    float L;
    uint32_t closed;    // bit k: lane k closed by control (roads of at most 32 lanes)
};

// Lane index taken on a road of n lanes (closed-lane mask `closed`) by a
// vehicle coming from lane index k: min(k, n - 1), or when control has
// closed that lane, the open lane nearest to it, the lower of two equally
// near.  A road always keeps an open lane, and only roads of at most 32
// lanes close lanes.  Branch-free: the nearest open lanes below and above
// come from the highest and lowest set bits of the open-lane mask.
__host__ __device__ inline int pick_lane(int k, int n, uint32_t closed)
{
    const int kk = k < n - 1 ? k : n - 1;
    const uint32_t nmask = n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
    const uint32_t open = ~closed & nmask;
    const uint32_t bit = 1u << (kk & 31);
    const uint32_t lo = open & (bit - 1u);
    const uint32_t hi = open & ~(bit | (bit - 1u));
    const int l = lo ? 31 - __builtin_clz(lo) : -64;
    const int h = hi ? __builtin_ctz(hi) : 64;
    const int near = (kk - l <= h - kk) ? l : h;
    return (closed == 0u || (open & bit)) ? kk : near;
}

// Per-lane flags of the current step (lane_red): the lane's road waits at a
// red light, the lane is closed, the lane lies inside a junction.
constexpr uint8_t kRedBit = 1u, kClosedBit = 2u, kInternalBit = 4u;

// Flags byte of a lane at step t (kRedBit, kClosedBit).
__host__ __device__ inline uint8_t lane_flags_at(const LaneInfo &li, uint32_t t)
{
    return (uint8_t)((lane_red_at(li, t) ? kRedBit : 0u) |
                     ((li.lflags & kLaneClosed) ? kClosedBit : 0u) |
                     ((li.lflags & kLaneInternal) ? kInternalBit : 0u));
}

// A lane's successor on another road (junction internal lanes).
struct Succ {
    int32_t lane, road;
};

// Last vehicle (lowest position) of each lane; id == kNone when empty.
struct Tail {
    float s, v;
    uint32_t id;
    int32_t pad;
};

// Hot per-vehicle state, structure of arrays (32 bytes per vehicle).
struct SoA {
    float *s, *v, *a;
    uint32_t *id;
    uint32_t *lane;     // in proposals: lane at step start, | kJoinBit if the vehicle leaves it
    uint32_t *ptr;      // absolute index of the current road in the route array
    int32_t *next;      // next road of the route, -1 on the last road
    float *v0;
};

struct Params {
    float dt, a_max, s0, T, len, b_max, b_safe, pol, a_thr, p_lc, d_look;
    float inv_tsab;     // fl32(1 / (2 sqrt(a_max b))) formed in double on the host
    float inv_2bmax;    // fl32(1 / (2 b_max)) formed in double on the host
    float b_mand, tau_yield;
    int32_t h_look;
    uint32_t key0, key1;
    uint32_t debug;
    uint32_t trace;
};

// Everything a kernel needs, passed by value.
struct Dev {
    Params P;
    int32_t n_lanes, n_scen, cap, n_qlanes;
    const LaneInfo *lanes;
    const RoadInfo *roads;
    // routes, each followed by -1, the departure step and the arrival step
    // (-1 until the vehicle arrives; written by the update at arrival)
    int32_t *route;
    SoA S;                        // state at the start of a step
    SoA Pr;                       // proposals, indexed by row at step start (+ insertions)
    // id and v0 never change in a step: they alternate between two buffers
    // by step parity instead of passing through the proposals.  S.id / S.v0
    // and Pr.id / Pr.v0 are the current buffer (which also holds the
    // insertion rows), id_next / v0_next the one the merge writes.
    uint32_t *id_next;
    float *v0_next;
    const int32_t *ls_old;        // lane_start of the state being read
    int32_t *ls_new;              // lane_start being built
    Tail *tails;
    int32_t *leave, *jcount;      // vehicles leaving / joining each lane (zeroed by the scan)
    int32_t *joff;                // exclusive scan of jcount
    int32_t *blk;                 // scan block sums
    // chunk[w] = (first lane, its new start, its old start, its joiner
    // offset) of merge chunk w: the first lane l with chunk_of(l, new start)
    // >= w (written by the lane-count scan);
    // [cap / kMergeRows + n_lanes / kMergeLanes + 3]
    int4 *chunk;
    // joiners (lane changers, road transfers, insertions).  Update tile b
    // (rows [b*kUpdateRows, (b+1)*kUpdateRows)) lists its jcnt[b] joiners in
    // jlist/jlane[b*kUpdateRows ...]; queue lane q lists its insertion (from
    // proposal row n_cur + q) in jins_list/jins_lane[q], lane kNone if none;
    // k_jscatter groups all of them by target lane into jidx/jslane using the
    // per-lane cursors jcur (initialised to joff by the scan).
    uint32_t *jlist, *jlane, *jidx, *jslane, *jins_list, *jins_lane;
    // the joiners' proposal records in the same lane-grouped order (J.lane is
    // jslane), copied by k_jscatter so that the merge reads them coalesced
    SoA J;
    int32_t *jcnt, *jcur;
    uint8_t *lane_red;            // lane flags of the current step (kRedBit, kClosedBit)
    int32_t *n_cur, *n_next, *n_dbg;
    uint32_t *n_ins;
    int64_t *t;
    // departure queues
    const int32_t *qlanes;
    int32_t *q_hdep;              // [n_qlanes] departure step of queue qlanes[q]'s head, INT32_MAX when empty
    int32_t *q_head;
    const int32_t *q_end;
    const uint32_t *q_id;
    const int32_t *q_dep;
    const float *q_v0;
    const uint32_t *q_ptr;
    const int32_t *q_next;
    // vehicle table sorted by id (arrival bookkeeping, cursor output)
    int32_t n_veh;
    const uint32_t *vt_id;
    const int32_t *vt_dep;
    const uint32_t *vt_rstart;
    const double *vt_dist0;       // route distance at which the vehicle entered
    // observables, each in kStripes copies (stripe k at k * cnt_stride /
    // sv_stride elements) so that concurrent waves add to different lines;
    // readers sum the copies
    unsigned long long *cnt;      // [kStripes][n_scen][C_N]
    unsigned long long *sumv;     // [kStripes][n_scen] speeds in 2^-20 m/s units
    int32_t cnt_stride, sv_stride;
    uint32_t *err;
    // launch shape (results do not depend on it): update and scatter grid
    // sizes (0 = default) and XCD-contiguous tile order
    int32_t upd_blocks, jsc_blocks, xcd_remap;
    // some lane is closed by control: the update variant that applies
    // closures is launched (set between steps; captured graphs are redone)
    int32_t closures;
    // junction internal lanes: successor lists (CSR over lanes), per
    // connector lane the conflicting lanes with priority and their feeders,
    // and the lanes' yield flags written after every step (k_yield)
    int32_t junctions;
    const int32_t *succ_off, *conf_off, *conf_feed;
    const Succ *succ, *conf;
    uint8_t *busy;
    // learned closure (mode 1) and its training trace
    int32_t mode;
    const float *mlp_theta, *mlp_norm;
    const void *mlp_pack;         // network image in the kernels' layout (mlp_pack_bytes())
    double *mlp_sq;               // [kStripes][n_scen] (stride sv_stride)
    float *tr_feat, *tr_label;    // [cap][8], [cap]
    // debug per row at step start
    uint32_t *d_id, *d_leader, *d_tl, *d_tf;
    int32_t *d_flags;
    float *d_margin;
};

// Merge chunks: a boundary every kMergeRows new rows and every kMergeLanes
// lanes, so that a chunk of a sparse state does not own tens of thousands of
// empty lanes.  chunk_of(l, s) is the chunk of lane l whose new start is s
// (the boundaries at or before it; non-decreasing along the lanes).
constexpr int kMergeRows = 512;
constexpr int kMergeLanes = 2048;
__host__ __device__ inline int chunk_of(int l, int s) { return s / kMergeRows + l / kMergeLanes; }
// Copies of the counters and sums; a wave adds to copy (4 * block + wave)
// mod kStripes.
constexpr int kStripes = 64;
// Elements per copy, padded to whole 256-byte lines.
inline int32_t stripe_elems(int64_t n) { return (int32_t)((n + 31) / 32 * 32); }

// Rows per update block (one joiner region per such tile).
constexpr int kUpdateRows = 256;
// Lanes per block of the lane-count scan (one pair of block sums each).
constexpr int kScanBlockLanes = 256;

enum { C_INSERTED = 0, C_INSERT_FAIL, C_ARRIVED, C_TRIP_TIME, C_CLAMPS, C_LANE_CHANGES,
       C_VEH_STEPS, C_MLP_EVAL, C_MLP_FALLBACK, C_N };

// Error text of the calling thread (moss_last_error): set_error stores a
// formatted message and returns code; clear_error empties it.
int set_error(int code, const char *fmt, ...);
void clear_error();

// Kernel launchers (moss_kernels.hip).
hipError_t launch_step(const Dev &d, hipStream_t st, hipEvent_t *ev = nullptr);
int step_kernel_count();
int step_scan_block_lanes();     // lanes per lane-count scan block
const char *step_kernel_name(int i);
hipError_t launch_tails(const Dev &d, hipStream_t st);
// Yield flags of the current state for the step about to run (junction
// internal lanes; after creation and after a change of the red flags).
hipError_t launch_yield(const Dev &d, hipStream_t st);
// Overwrites n lane records (signal control, speed limits) and recomputes
// their red flags for the step about to run.
hipError_t launch_lane_patch(const Dev &d, const int32_t *idx, const LaneInfo *rec, int32_t n,
                             hipStream_t st);
// Overwrites n road records (lane closures).
hipError_t launch_road_patch(const Dev &d, const int32_t *idx, const RoadInfo *rec, int32_t n,
                             hipStream_t st);
// Road measures and positions of the current state (read functions).
hipError_t launch_road_stats(const Dev &d, int32_t n_roads, int32_t *count, float *mean_v,
                             hipStream_t st);
hipError_t launch_positions(const Dev &d, int32_t n, const double *road_ab, double *x,
                            double *y, double *heading, hipStream_t st);
// Builds the packed network image from mlp_theta / mlp_norm (once per simulator).
hipError_t launch_mlp_pack(const Dev &d, hipStream_t st);
size_t mlp_pack_bytes();
// Trips of every vehicle in id order (status, travel time, distance; see
// moss_read_trips) from the current state of n_act rows.
hipError_t launch_trips(const Dev &d, int32_t n_act, int32_t *status, int32_t *travel,
                        double *dist, hipStream_t st);
hipError_t launch_cursor(const Dev &d, const uint32_t *ids, const uint32_t *ptrs, int32_t *out,
                         int32_t n, hipStream_t st);

}  // namespace moss

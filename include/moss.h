/*
 * moss.h -- C ABI of the MI355X (gfx950) microscopic traffic simulator.
 *
 * The library advances a road network full of vehicles in fixed time steps.
 * Each step follows the two-phase iteration of the paper's GPU simulator
 * (Sec. III-A): a prepare phase that orders every lane's vehicles by
 * position and keeps a read-only copy of their motion state, then an update
 * phase in which every vehicle, reading only that copy, finds its leader,
 * evaluates IDM car-following and a randomised MOBIL lane change, and moves
 * by Newton's equations of motion.  Inputs are a road network and travel
 * demand, outputs the per-vehicle state and road-level measures (Sec. III-A,
 * last paragraphs).
 *
 * Conventions
 * -----------
 * - All functions return MOSS_OK (0) or a negative MOSS_E* code; the text of
 *   the last error of the calling thread is returned by moss_last_error().
 * - Input structs hold HOST pointers; moss_create copies everything it needs,
 *   so the caller may free them when it returns.
 * - Device memory is owned by the caller: moss_create receives a workspace of
 *   at least moss_query_workspace() bytes (e.g. a uint8 torch tensor) that must
 *   stay allocated, and untouched, until moss_destroy.
 * - All device work is enqueued on the HIP stream given to moss_create
 *   (hipStream_t passed as void*, NULL = the null stream).  moss_step is
 *   asynchronous; the read functions synchronise that stream.
 * - A handle is not thread-safe; distinct handles are independent.
 *
 * Units: metres, seconds, m/s, m/s^2; time in integer steps of dt seconds.
 */
#ifndef MOSS_H
#define MOSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MOSS_OK 0
#define MOSS_EINVAL (-1)   /* malformed input or argument */
#define MOSS_ENOMEM (-2)   /* workspace or output buffer too small */
#define MOSS_EDEVICE (-3)  /* a HIP call failed */
#define MOSS_ESTATE (-4)   /* the device flagged an invalid state (see moss_read_counters) */

/* Flags for moss_params.flags */
#define MOSS_FLAG_DEBUG 1u /* record per-vehicle decisions of each step (moss_read_debug) */
#define MOSS_FLAG_TRACE 2u /* record the closure's inputs and IDM label (moss_read_trace) */

/* moss_params.mode */
#define MOSS_MODE_IDM 0
#define MOSS_MODE_MLP 1    /* learned closure inside its envelope, IDM outside */

/* Road network.  Roads are directed; road r has road_nlanes[r] lanes numbered
 * road_lane0[r] .. road_lane0[r]+road_nlanes[r]-1 (lane index k inside the
 * road = lane - road_lane0[r]); lanes must be numbered road by road without
 * gaps.  All lanes of a road have the road's length.  lane_scen (optional)
 * labels each lane with a scenario id in [0, n_scen) when several independent
 * scenarios are simulated as one disjoint network; counters are kept per
 * scenario. */
typedef struct {
    int32_t n_nodes, n_roads, n_lanes, n_scen;
    const int32_t *road_from;    /* [n_roads] upstream node */
    const int32_t *road_to;      /* [n_roads] downstream node */
    const int32_t *road_nlanes;  /* [n_roads] 1..255 */
    const int32_t *road_lane0;   /* [n_roads] */
    const float *road_length;    /* [n_roads] m, > 0 */
    const float *lane_vlim;      /* [n_lanes] speed limit, m/s, > 0 */
    const int32_t *lane_scen;    /* [n_lanes] or NULL (all 0) */
    const double *node_x;        /* [n_nodes] m, or NULL (then moss_read_positions fails) */
    const double *node_y;        /* [n_nodes] m, or NULL */
    /* Junction internal lanes (the map builder's lane connectivity inside
     * intersections, Sec. III-C-1), all NULL without them.  road_internal[r]
     * = 1 marks a connector road inside a junction (no lane changes on it).
     * lane_succ[lane_succ_off[l] .. lane_succ_off[l+1]-1] are the lanes a
     * vehicle on lane l may continue on, at most one per road; a vehicle whose
     * next route road is r takes l's successor on r, and a lane without a
     * list takes lane min(k, n-1) of r as without junction lanes.
     * lane_conf[lane_conf_off[c] .. ] are the connector lanes whose paths
     * conflict with connector lane c and that have priority over it, and
     * lane_conf_feed[] the lane feeding each of them. */
    const uint8_t *road_internal;       /* [n_roads] */
    const int32_t *lane_succ_off;       /* [n_lanes+1] */
    const int32_t *lane_succ;           /* [lane_succ_off[n_lanes]] */
    const int32_t *lane_conf_off;       /* [n_lanes+1] */
    const int32_t *lane_conf;           /* [lane_conf_off[n_lanes]] */
    const int32_t *lane_conf_feed;      /* [lane_conf_off[n_lanes]] */
} moss_network;

/* Fixed-time signal plans.  Node j with node_cycle[j] > 0 shows phase
 * ((t + node_offset[j]) mod node_cycle[j]) div node_phase[j] at step t.
 * A road r ending at a signalised node may enter the junction only while
 * that phase equals road_group[r]; road_group[r] = -1 means always green. */
typedef struct {
    const int32_t *node_cycle;   /* [n_nodes] steps, 0 = unsignalised */
    const int32_t *node_phase;   /* [n_nodes] steps per phase, > 0 if signalised */
    const int32_t *node_offset;  /* [n_nodes] steps, >= 0 */
    const int8_t *road_group;    /* [n_roads] */
} moss_signals;

/* Travel demand.  Vehicle i follows route_roads[route_off[i] ..
 * route_off[i+1]-1], a chain of at least one road where each road starts at
 * the node the previous one ends.  Vehicle ids must be unique and differ from
 * 0xFFFFFFFF.  A vehicle with placed[i] = 0 (or placed = NULL) enters its first
 * road at s = 0 at or after step depart[i]: it queues on lane id mod nlanes of
 * that road.  A vehicle with placed[i] = 1 starts on lane[i] at front-bumper
 * position s[i] with speed v[i], previous acceleration a[i] and route index
 * cursor[i]; placed vehicles of a lane must keep at least one vehicle length
 * between consecutive fronts. */
typedef struct {
    int32_t n;
    const uint32_t *id;          /* [n] */
    const int32_t *depart;       /* [n] step of departure (trip time counts from it) */
    const float *v0;             /* [n] desired speed, m/s, > 0 */
    const int64_t *route_off;    /* [n+1] */
    const int32_t *route_roads;  /* [route_off[n]] */
    const uint8_t *placed;       /* [n] or NULL */
    const int32_t *lane;         /* [n] used where placed */
    const int32_t *cursor;       /* [n] */
    const float *s, *v, *a;      /* [n] */
} moss_vehicles;

/* Model parameters (IDM: a_max, b, s0, T with exponent 4; MOBIL: politeness,
 * a_thr, b_safe; lane changes that pass are executed with probability p_lc
 * using Philox4x32-10 keyed by seed and counted by (step, vehicle id)). */
typedef struct {
    float dt;          /* s */
    float a_max, b, s0, T;
    float length;      /* vehicle length, m */
    float b_max;       /* braking limit, m/s^2 */
    float b_safe;      /* MOBIL safe braking of the new follower, m/s^2 */
    float politeness, a_thr, p_lc;
    float d_look;      /* m, lookahead range beyond the lane end */
    int32_t h_look;    /* roads scanned ahead, >= 0 */
    int32_t t0;        /* index of the first step, >= 0 */
    uint64_t seed;
    uint32_t flags;    /* MOSS_FLAG_* */
    int32_t mode;      /* MOSS_MODE_* */
    const float *mlp_theta;  /* host float[MOSS_MLP_PARAMS], used when mode = MLP */
    const float *mlp_norm;   /* host float[MOSS_MLP_NORM] */
    /* junction internal lanes: lane-change bias toward lanes that continue
     * the route (m/s^2, >= 0) and the approach time within which a vehicle
     * with priority makes a vehicle yield (s, >= 0) */
    float b_mand, tau_yield;
} moss_params;

typedef struct moss_sim moss_sim;

/* Per-vehicle state rows in lane order (lane ascending, then position).
 * Any pointer may be NULL to skip the field.  device = 1: pointers are device
 * memory of the simulator's GPU, 0: host memory.  capacity = rows available;
 * n receives the number of active vehicles (MOSS_ENOMEM if above capacity,
 * nothing written), t the index of the next step. */
typedef struct {
    int32_t capacity;
    int32_t device;
    uint32_t *id;
    int32_t *lane;
    float *s, *v, *a;
    int32_t *cursor;             /* index into the vehicle's route */
    int32_t n;                   /* out */
    int64_t t;                   /* out */
} moss_state_out;

/* Counter indices of moss_read_counters (per scenario). */
enum {
    MOSS_CNT_INSERTED = 0,   /* vehicles that entered the network */
    MOSS_CNT_INSERT_FAIL,    /* due queue heads that found no gap */
    MOSS_CNT_ARRIVED,        /* vehicles that completed their route */
    MOSS_CNT_TRIP_TIME,      /* sum over arrivals of (arrival step - depart) */
    MOSS_CNT_CLAMPS,         /* overlap corrections */
    MOSS_CNT_LANE_CHANGES,
    MOSS_CNT_VEH_STEPS,      /* sum over steps of active vehicles after the step */
    MOSS_CNT_MLP_EVAL,       /* learned-closure evaluations inside its envelope */
    MOSS_CNT_MLP_FALLBACK,   /* vehicle-steps that fell back to IDM */
    MOSS_N_COUNTERS
};

/* Device bytes a simulation of these inputs needs: the road network and the
 * travel demand, the simulator's two inputs (Sec. III-A, last paragraphs),
 * plus the per-step index and proposal arrays of the two-phase step.
 * Validates like moss_create (host-only work, no device call). */
int moss_query_workspace(const moss_network *net, const moss_signals *sig,
                         const moss_vehicles *veh, const moss_params *prm, size_t *bytes);

/* Starts a simulation of a road network and its travel demand (Sec. III-A,
 * last paragraphs: the inputs of the GPU simulator).  Validates and copies
 * the inputs into the workspace and returns a handle.
 * Errors: MOSS_EINVAL (inconsistent network, route that is not a chain,
 * overlapping placed vehicles, non-finite or non-positive parameters),
 * MOSS_ENOMEM (ws_bytes too small), MOSS_EDEVICE. */
int moss_create(const moss_network *net, const moss_signals *sig, const moss_vehicles *veh,
                const moss_params *prm, void *d_ws, size_t ws_bytes, void *hip_stream,
                moss_sim **out);

/* Enqueues n >= 0 steps.  Each step is the paper's iteration (Sec. III-A,
 * second paragraph): the update phase (every vehicle reads the state the
 * step started from, finds its leader, takes IDM and randomised-MOBIL
 * decisions and moves by Newton's equations), then the prepare phase that
 * orders every lane's vehicles by position for the next step.  Asynchronous.
 * MOSS_ESTATE if an earlier read found the device error word set. */
int moss_step(moss_sim *h, int32_t n);

/* The per-vehicle output of the simulator after the last step: position and
 * speed (Sec. III-A, last paragraph), with lane, previous acceleration and
 * route index.  Synchronises the stream and copies the requested state rows.  The copies
 * run on the simulator's stream and are complete on return; with device
 * destinations the whole device is synchronised first, so that a destination
 * just released by work on another stream is not written early. */
int moss_read_state(moss_sim *h, moss_state_out *out);

/* Synchronises and copies host arrays counters[n_scen][MOSS_N_COUNTERS] and
 * sum_v[n_scen] and the device error word (0 = healthy; bit 0 lane capacity
 * exceeded, bit 1 non-finite state).  Any pointer may be NULL.  sum_v is the
 * sum over steps and active vehicles of speed, from which the mean speed is
 * formed (Sec. III-A, last paragraph; Sec. IV-A): each vehicle adds its
 * speed in whole units of 2^-20 m/s (truncated; 0 for speeds <= 0, 2^32 - 1
 * from 4096 m/s on) to a 64-bit integer, exact and independent of the order
 * of the additions, and sum_v is that integer / 2^20 rounded to double. */
int moss_read_counters(moss_sim *h, int64_t *counters, double *sum_v, uint32_t *error_word);

/* Ids of the vehicles that have not entered the network yet (host buffer of
 * capacity entries), lane by lane of their first road, each lane in (depart,
 * id) order; n receives the count (MOSS_ENOMEM if above capacity, nothing
 * written).  Together with moss_read_state (rows with cursor and previous
 * acceleration) and the step index, this is a checkpoint: moss_create with the
 * rows as placed vehicles, these as pending ones and t0 = that step continues
 * the run exactly (the inputs of a step are the state and the queues, Sec.
 * III-A; arrived vehicles leave nothing behind; counters restart at zero).
 * Phases held by moss_set_signal_phase and limits set by moss_set_lane_vlim
 * are not part of it: the caller applies them again to the new simulator. */
int moss_read_pending(moss_sim *h, int32_t capacity, uint32_t *id, int32_t *n);

/* With MOSS_FLAG_DEBUG: per-vehicle decisions of the most recent step, in the
 * row order of the state that step started from (host pointers, capacity
 * rows, NULL to skip): vehicle id, leader id (0xFFFFFFFF = none), flags
 * (bits 0-1: 0 no lane-change evaluation, 1 evaluated and kept, 2 changed;
 * bit 2 red-light obstacle applied; bit 3 leader found beyond the lane end;
 * bit 4 arrived), MOBIL margin (incentive minus threshold), target-lane
 * leader and follower ids.  *n receives the row count. */
int moss_read_debug(moss_sim *h, int32_t capacity, uint32_t *id, uint32_t *leader,
                    int32_t *flags, float *margin, uint32_t *t_leader, uint32_t *t_follower,
                    int32_t *n);

/* Runs n steps like moss_step, each kernel launched directly between two HIP
 * events on the simulator's stream, and adds each kernel's duration to
 * kernel_ms[k] (milliseconds; array of capacity entries, zeroed first).
 * Steps are enqueued back to back and synchronised every 64 steps.
 * *n_kernels receives the number of kernels per step; moss_kernel_name(k)
 * names kernel k (NULL if out of range); a kernel the workload does not
 * launch (yield flags without junction lanes, the lane-count block reduction
 * on networks of at most 256 lanes) reports 0.  Departures are
 * inserted by workgroups of the update's launch, so their time is part of
 * k_update's.  Meant for measurement: the events and direct launches make it
 * slower than moss_step. */
int moss_step_timed(moss_sim *h, int32_t n, double *kernel_ms, int32_t capacity,
                    int32_t *n_kernels);
const char *moss_kernel_name(int32_t i);

/* Launch shape of the step kernels (batch APIs, Sec. III-C: the same step
 * serves many scenarios, so its shape is tuned per workload class).  Every
 * setting computes bit-identical states; the fields change only how the step
 * is grouped into graphs and workgroups:
 *   graph_steps     steps per captured hipGraph replay: even, 2..256; 0 turns
 *                   graphs off (every step launched directly).  Default 16.
 *   update_blocks   workgroups of the update kernel; each loops over 256-row
 *                   tiles.  0 = one per tile (capped at 16384).  1..65535.
 *   scatter_blocks  workgroups of the joiner scatter (4 tiles per workgroup
 *                   per pass).  0 = default (capped at 2048).  1..65535.
 *   xcd_remap       1: the tiles that have work in a step are split into 8
 *                   contiguous ranges, one per XCD (XCDs receive workgroups
 *                   round-robin, so workgroup b takes tile (b mod 8) * (g / 8)
 *                   + b / 8 with g the tile count rounded up to 8, or the grid
 *                   if smaller), so that each XCD's L2 holds the halo rows its
 *                   tiles share; applies to the update and merge kernels.
 *                   0: tile = b.  Default 0.
 * moss_set_launch validates (MOSS_EINVAL, state unchanged) and drops captured
 * graphs; it must not be called while steps enqueued on the handle's stream
 * are being captured elsewhere. */
typedef struct {
    int32_t graph_steps;
    int32_t update_blocks;
    int32_t scatter_blocks;
    int32_t xcd_remap;
} moss_launch;

int moss_set_launch(moss_sim *h, const moss_launch *cfg);
int moss_get_launch(const moss_sim *h, moss_launch *cfg);

/* ---- learned car-following closure (the project's extension) ----
 * An 8 -> 64 -> 64 -> 1 network with GELU (tanh form) that, inside its
 * training envelope, replaces the IDM acceleration of the vehicle update
 * (moss_params.mode = MOSS_MODE_MLP).  Parameters: float[MOSS_MLP_PARAMS] =
 * W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3; input description:
 * float[MOSS_MLP_NORM] = mean[8], inv_std[8], lo[8], hi[8] of the inputs
 * (leader gap, speed, leader speed, effective desired speed, distance to a red
 * stop line, previous acceleration, distance to the lane end, speed limit).
 * The simulator evaluates it with bfloat16 weights and activations and FP32
 * accumulation on the matrix cores.  All pointers below are device pointers
 * and all calls are asynchronous on the given stream. */
#define MOSS_MLP_PARAMS 4801
#define MOSS_MLP_NORM 32

/* Scratch bytes moss_mlp_grad needs for a batch of n samples. */
size_t moss_mlp_scratch_bytes(int32_t n);

/* Mean squared error of the network's output limited to [out_lo, out_hi]
 * (as the simulator limits it: -b_max, a_max) on n samples (features
 * feat[idx[b]][8], labels label[idx[b]]; idx = NULL means b itself) and its
 * gradient with respect to theta (float[MOSS_MLP_PARAMS]); the distance inputs
 * 0, 4 and 6 enter as ln(max(x, 0.5)) before normalisation.  bf16 = 1 rounds
 * weights and layer inputs to bfloat16 as the simulator does.  loss may be
 * NULL.  MOSS_EINVAL on bad arguments, MOSS_ENOMEM if scratch is too small. */
int moss_mlp_grad(const float *feat, const float *label, const int32_t *idx, int32_t n,
                  const float *theta, const float *norm, int32_t bf16, float out_lo,
                  float out_hi, float *grad, float *loss, void *scratch, size_t scratch_bytes,
                  void *hip_stream);

/* Largest batch moss_mlp_grad_static accepts. */
#define MOSS_MLP_STATIC_MAX_SAMPLES 8192

/* moss_mlp_grad without a scratch argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight training loops, hosts
 * that forbid hipMalloc): the same kernels and the same result, bit for bit,
 * as moss_mlp_grad, on a scratch area the library holds as a static device
 * array of moss_mlp_scratch_bytes(MOSS_MLP_STATIC_MAX_SAMPLES) bytes (about
 * 9.3 MB), one copy per GPU, kept until the process ends.  It runs on the
 * current device; the first call on a device looks up that device's copy.
 * It allocates nothing.  Every call on one GPU shares that GPU's copy: calls
 * that overlap in time on one GPU (different streams, or threads) race and
 * must be serialised by the caller; calls in order on one stream are safe.
 * Nothing needs to start at zero (each call writes every scratch value it
 * reads).  MOSS_EINVAL for n > MOSS_MLP_STATIC_MAX_SAMPLES (use moss_mlp_grad
 * with a workspace) and the argument errors of moss_mlp_grad; MOSS_EDEVICE if
 * the device copy cannot be found. */
int moss_mlp_grad_static(const float *feat, const float *label, const int32_t *idx, int32_t n,
                         const float *theta, const float *norm, int32_t bf16, float out_lo,
                         float out_hi, float *grad, float *loss, void *hip_stream);

/* One Adam step (Kingma & Ba) on theta with moments m, v (all
 * float[MOSS_MLP_PARAMS]); step counts from 1. */
int moss_mlp_adam(float *theta, float *m, float *v, const float *grad, int32_t step, float lr,
                  float beta1, float beta2, float eps, void *hip_stream);

/* Network outputs for n feature rows with the simulator's inference path. */
int moss_mlp_predict(const float *feat, int32_t n, const float *theta, const float *norm,
                     float *out, void *hip_stream);

/* With MOSS_FLAG_TRACE: the inputs of the network and the IDM acceleration of
 * every vehicle in the most recent step, in the row order of the state that
 * step started from, copied to feat[n][8] and label[n] (host or device
 * pointers per device flag).  Copies are ordered and completed as in
 * moss_read_state. */
int moss_read_trace(moss_sim *h, int32_t capacity, int32_t device, float *feat, float *label,
                    int32_t *n);

/* Runtime control (batch writes between steps, Sec. III-C).  Both calls
 * synchronise the handle's stream and take effect from the next step.
 *
 * moss_set_signal_phase: for each of the n signalised nodes node[i],
 * phase[i] >= 0 holds that phase (roads whose signal group differs wait)
 * until changed; phase[i] = -1 returns the node to its fixed-time plan.
 * MOSS_EINVAL for a node out of range or without a signal, or a phase
 * outside -1..32767 (nothing is changed then).  A node named twice takes
 * the last phase given.
 *
 * moss_set_lane_vlim: speed limits (m/s, finite, > 0) of n lanes; a lane
 * named twice takes the last value.
 *
 * moss_set_lane_closed: lane restrictions (Sec. III-C-4): closed[i] != 0
 * closes lane[i], 0 opens it (a lane named twice takes the last value).  A
 * closed lane admits no vehicle: it is never a lane-change target, a vehicle
 * entering its road (or looking ahead along its route) takes the open lane
 * nearest to the lane index it would take, the lower of two equally near,
 * and its departure queue waits (counted as insertion failures); vehicles
 * already on it carry on and may leave it.  MOSS_EINVAL, changing nothing,
 * for a lane out of range, a road of more than 32 lanes, or a batch that
 * would leave a road without an open lane.
 *
 * Host arrays for all three. */
int moss_set_signal_phase(moss_sim *h, const int32_t *node, const int32_t *phase, int32_t n);
int moss_set_lane_vlim(moss_sim *h, const int32_t *lane, const float *vlim, int32_t n);
int moss_set_lane_closed(moss_sim *h, const int32_t *lane, const int32_t *closed, int32_t n);

/* Dynamic lanes (Sec. III-C-4), with junction internal lanes: from the next
 * step on, lane[i] lets vehicles continue onto road[i] (allowed[i] != 0) or
 * no longer does, by taking its successor on that road in or out of use; the
 * movements of a lane are those its successor list holds (the map builder's
 * connectors).  Lane changes, the lane-change bias and the lanes vehicles
 * take follow the change; a lane none of whose successors is in use
 * continues nowhere (its vehicles change lanes, or go through on the nearest
 * connector lane).  Departure lanes stay those chosen at creation.
 * Synchronises the stream.  MOSS_EINVAL, changing nothing, without junction
 * lanes, for a lane out of range or a lane without a successor on the road.
 * Host arrays. */
int moss_set_lane_turns(moss_sim *h, const int32_t *lane, const int32_t *road,
                        const int32_t *allowed, int32_t n);

/* Road measures of the current state (the simulator's road outputs, Sec.
 * III-A: average speed per road): count[r] vehicles on road r (all lanes) and
 * mean_v[r] their mean speed (0 for an empty road), the sum taken in FP64
 * over the road's rows in state order.  Arrays of n_roads, host or device
 * pointers per the device flag; either may be NULL.  Synchronises like
 * moss_read_state. */
int moss_read_road_stats(moss_sim *h, int32_t device, int32_t *count, float *mean_v);

/* Position and heading of every vehicle of the current state (the
 * simulator's per-vehicle outputs, Sec. III-A), in state row order: a road is
 * the straight segment from its upstream to its downstream node; a vehicle
 * at s on lane k of road r (length L) is at A + (B - A) s / L, moved
 * (k + 1/2) * 3.5 m to the right of the direction of travel; heading =
 * atan2(By - Ay, Bx - Ax) in radians.  FP64.  Needs node_x / node_y at
 * creation (MOSS_EINVAL otherwise).  Arrays of capacity >= n rows, host or
 * device pointers per the device flag; *n receives the row count. */
int moss_read_positions(moss_sim *h, int32_t capacity, int32_t device, double *x, double *y,
                        double *heading, int32_t *n);

/* Travel time and distance of every vehicle (the paper's query APIs for
 * traffic participants, Sec. III-C-4), in ascending id order: id, status (0
 * waiting to depart, 1 on the network, 2 arrived), travel time in steps
 * (arrival step - depart once arrived; the index of the next step - depart
 * on the network; 0 while waiting) and distance in metres along the route
 * since the vehicle entered the simulation (the whole route once arrived; the
 * roads before its current one plus its position while on the network; for a
 * vehicle placed at creation, less the route distance of its placement; 0
 * while waiting), road lengths summed in FP64 in route order.  Arrays of
 * capacity >= the number of vehicles given at creation (*n receives it;
 * MOSS_ENOMEM if larger, nothing written), host or device pointers per the
 * device flag; any array may be NULL.  Synchronises like moss_read_state. */
int moss_read_trips(moss_sim *h, int32_t capacity, int32_t device, uint32_t *id,
                    int32_t *status, int32_t *travel_time, double *distance, int32_t *n);

/* Sum over the network's evaluations of (a_network - a_IDM)^2, per scenario
 * (host array double[n_scen]). */
int moss_read_mlp_error(moss_sim *h, double *sum_sq);

/* Ends the simulation started by moss_create: frees host-side resources of
 * the handle (captured step graphs, host copies of the lane records); the
 * workspace stays the caller's and may be freed after this returns. */
int moss_destroy(moss_sim *h);

/* Message of the calling thread's last error ("" if none). */
const char *moss_last_error(void);

#ifdef __cplusplus
}
#endif
#endif

/*
 * CPU oracle for the per-step microscopic vehicle update (test infrastructure).
 *
 * This is the slow, plain reference that the HIP simulator is checked
 * against.  It is only used by the test-suite, the smoke check and the CPU
 * baseline of the benchmark; the product path never calls it.  It shares no
 * code, header or table with the HIP library: the only thing the two have in
 * common is the seeded scenario generator that produces their inputs.
 *
 * What it computes follows the paper's simulator description (Sec. III-A):
 * each step has a prepare phase (per-lane spatial ordering plus a read-only
 * copy of the motion state) and an update phase in which every vehicle senses
 * its leader through that ordering, applies IDM car-following and a
 * randomised MOBIL lane-change rule, and advances by Newton's equations of
 * motion.  Points the paper leaves open (insertion, junctions, signals,
 * randomisation, collisions) follow the readings written next to each rule
 * in moss_oracle.c.
 */
#ifndef MOSS_ORACLE_H
#define MOSS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    /* network */
    int32_t n_nodes, n_roads, n_lanes, n_scen;
    const int32_t *road_from, *road_to, *road_nlanes, *road_lane0;
    const float *road_length, *lane_vlim;
    const int32_t *lane_scen;          /* may be NULL: one scenario */
    const double *node_x, *node_y;     /* may be NULL: no positions */
    /* signals */
    const int32_t *node_cycle, *node_phase, *node_offset;
    const int8_t *road_group;
    /* vehicles */
    int32_t n_veh;
    const uint32_t *veh_id;
    const int32_t *depart;
    const float *v0;
    const int64_t *route_off;
    const int32_t *route_roads;
    const uint8_t *placed;             /* may be NULL: nobody pre-placed */
    const int32_t *lane, *cursor;
    const float *s, *v, *a;
    /* parameters */
    float dt, a_max, b, s0, T, length, b_max, b_safe, politeness, a_thr, p_lc, d_look;
    int32_t h_look;
    int32_t t0;
    uint64_t seed;
    /* learned car-following closure (mode 1): parameters W1[64][8], b1[64],
     * W2[64][64], b2[64], w3[64], b3 (4801 floats) and norm = mean[8],
     * inv_std[8], lo[8], hi[8] of the inputs */
    int32_t mode;
    const float *mlp_theta;
    const float *mlp_norm;
    /* junction internal lanes (all NULL without): internal-road flags,
     * lane successors (CSR over lanes) and, per connector lane, the
     * conflicting connector lanes with priority over it and the lane feeding
     * each; b_mand (m/s^2) biases lane changes toward lanes that continue
     * along the route; tau_yield (s) is the time within which an approaching
     * vehicle with priority makes a vehicle yield */
    const uint8_t *road_internal;
    const int32_t *lane_succ_off, *lane_succ;
    const int32_t *lane_conf_off, *lane_conf, *lane_conf_feed;
    float b_mand, tau_yield;
} orc_input;

typedef struct orc_sim orc_sim;

/* counters per scenario, in this order */
enum { ORC_INSERTED = 0, ORC_INSERT_FAIL, ORC_ARRIVED, ORC_TRIP_TIME, ORC_CLAMPS,
       ORC_LANE_CHANGES, ORC_VEH_STEPS, ORC_MLP_EVAL, ORC_MLP_FALLBACK, ORC_N_COUNTERS };

#define ORC_NONE 0xFFFFFFFFu

orc_sim *orc_create(const orc_input *in);
const char *orc_error(void);
void orc_destroy(orc_sim *m);
int orc_step(orc_sim *m, int32_t n);
/* Threads for the update and merge loops (default 1).  Results are the same
 * bits for any count: vehicles and lanes are independent within a step and
 * every sum is taken afterwards in a fixed order. */
void orc_set_threads(orc_sim *m, int32_t n);
/* Threads OpenMP would use by default (1 without OpenMP). */
int32_t orc_max_threads(void);
int32_t orc_n_active(const orc_sim *m);
int64_t orc_time(const orc_sim *m);
/* State in lane order (lane ascending, then position ascending). */
void orc_read(const orc_sim *m, uint32_t *id, int32_t *lane, float *s, float *v, float *a,
              int32_t *cursor);
/* Per-vehicle decisions of the last step, in the order of the state the step
 * started from: vehicle id, leader id (ORC_NONE if none), flags (bits 0-1:
 * 0 no lane-change evaluation, 1 evaluated and kept, 2 changed; bit 2 red
 * light obstacle applied; bit 3 leader found by lookahead; bit 4 arrived),
 * MOBIL margin (incentive minus threshold, 0 when not evaluated), target-lane
 * leader and follower ids. */
int32_t orc_read_debug(const orc_sim *m, uint32_t *id, uint32_t *leader, int32_t *flags,
                       float *margin, uint32_t *t_leader, uint32_t *t_follower);
/* counters: int64 [n_scen][ORC_N_COUNTERS], sum of speeds [n_scen] */
void orc_counters(const orc_sim *m, int64_t *cnt, double *sum_v);
/* sum over network evaluations of (a_mlp - a_idm)^2 [n_scen] */
void orc_mlp_sq(const orc_sim *m, double *sum_sq);
/* network output for one normalised input vector z[8] (FP64; weights and
 * hidden layer inputs rounded to bfloat16, each input z as the pair
 * bf16(z) + bf16(z - bf16(z))) */
double orc_mlp_forward(const float *theta, const float *z);
/* Network mode: the raw closure inputs feat[n][8] of each vehicle of the last
 * step and their use (1 evaluated, 2 outside the envelope), in the order of
 * orc_read_debug.  Returns n (0 outside network mode). */
int32_t orc_read_mlp_inputs(const orc_sim *m, float *feat, int8_t *use);
/* Every network output an FP32 evaluation of the closure may correctly give
 * for raw inputs f[8] (normalised with norm[32] as in the step), limited to
 * [lo, hi]: bfloat16 roundings of hidden activations whose FP32 error
 * interval holds a rounding boundary are taken both ways, and the logarithm
 * of a distance may be any float within two ulps.  out[0] is the oracle's own
 * output.  info[4]: tied units of layer 1 and of layer 2 (with the oracle's
 * own choices), input combinations, first tied unit (64 * layer + unit, -1).
 * Returns the number of distinct outputs (at most cap). */
int32_t orc_mlp_candidates(const float *theta, const float *norm, const float *f, float lo,
                           float hi, int32_t cap, double *out, int32_t *info);
/* The same for n input rows (out[n][cap], n_out[n], info[n][4]). */
void orc_mlp_candidates_batch(const float *theta, const float *norm, int32_t n, const float *feat,
                              float lo, float hi, int32_t cap, double *out, int32_t *n_out,
                              int32_t *info, int32_t threads);
int32_t orc_pending(const orc_sim *m);
/* Signal control: node shows `phase` from the next step on (-1: its
 * fixed-time plan again).  Returns -1 for a node without a signal. */
int orc_set_signal_phase(orc_sim *m, int32_t node, int32_t phase);
/* Speed limit of a lane from the next step on. */
void orc_set_lane_vlim(orc_sim *m, int32_t lane, float vlim);
/* Lane restriction from the next step on: lane[q] is closed (closed[q] != 0)
 * or opened, in order (a lane named twice takes the last value).  A closed
 * lane is never a lane change target, vehicles entering its road take the
 * nearest open lane (pick_lane), and its departure queue waits; vehicles on
 * it carry on.  Returns -1, changing nothing, for a lane out of range or
 * when a road would be left without an open lane. */
int orc_set_lane_closed(orc_sim *m, int32_t n, const int32_t *lane, const int32_t *closed);
/* Dynamic lanes (junction internal lanes): from the next step on, lane[q]
 * lets vehicles continue onto road[q] (allowed[q] != 0) or not, by taking
 * its successor entry on that road in or out of use.  A lane with entries
 * none of which are in use continues nowhere.  Returns -1, changing nothing,
 * without junction lanes or when a lane has no successor on the road. */
int orc_set_lane_turns(orc_sim *m, int32_t n, const int32_t *lane, const int32_t *road,
                       const int32_t *allowed);
/* Vehicles and mean speed (FP64 sum in state order, 0 if empty) per road. */
void orc_road_stats(const orc_sim *m, int32_t *count, float *mean_v);
/* Position and heading of each state row: on the segment from the road's
 * upstream node A to its downstream node B at A + (B - A) s / L, moved
 * (k + 1/2) * 3.5 m to the right of the direction of travel; heading
 * atan2(By - Ay, Bx - Ax).  Returns -1 without node coordinates. */
int orc_positions(const orc_sim *m, double *x, double *y, double *heading);

/* Trips of all n_veh vehicles in ascending id order: status (0 waiting to
 * depart, 1 on the network, 2 arrived), travel time in steps (arrival -
 * depart; current step index - depart on the network; 0 waiting) and the
 * distance along the route since the vehicle entered the simulation (FP64,
 * road lengths summed in route order). */
void orc_read_trips(const orc_sim *m, uint32_t *id, int32_t *status, int32_t *travel,
                    double *dist);

/* Philox4x32 with 10 rounds (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* IDM acceleration in FP32 (has_leader = 0: free road); inv_tsab is the
 * FP32 reciprocal of 2 sqrt(a_max b), formed in double. */
float orc_idm(float v, float v0e, int has_leader, float v_lead, float gap, float a_max,
              float inv_tsab, float s0, float T, float b_max);

#ifdef __cplusplus
}
#endif
#endif

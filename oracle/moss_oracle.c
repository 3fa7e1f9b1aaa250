/*
 * CPU oracle for the per-step microscopic vehicle update.
 *
 * TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the simulator library.
 *
 * The paper (Sec. III-A) fixes the skeleton of one simulation step:
 *   prepare  - build a per-lane spatial index of the vehicles and take a
 *              read-only copy of their motion state;
 *   update   - every vehicle reads its leader through the index, computes
 *              its acceleration from IDM [Treiber et al. 2000], decides on
 *              a lane change with a randomised MOBIL rule [Kesting et al.
 *              2007], and moves by Newton's equations of motion.
 * It also fixes the 1 s step, the inputs (road network plus demand) and the
 * outputs (per-vehicle position and speed, road averages).  Everything else is
 * a reading of this project, marked [reading] below; the HIP library follows
 * the same readings.
 *
 * Arithmetic is FP32, each expression evaluated in the written order; the
 * file is compiled without FP contraction or fast-math so that every rounding
 * is a plain IEEE single-precision operation.
 *
 * The implementation is deliberately plain: the whole state is rebuilt every
 * step, neighbour searches are linear scans, joiners are ordered with qsort.
 */
#include "moss_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static char g_err[256];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *orc_error(void) { return g_err; }

/* ---------------------------------------------------------------- RNG --- */

/* Philox4x32-10 as published by Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64 bit
 * multiplications with a Weyl-sequence key schedule. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A speed in fixed point for the summed-speed observable (Sec. III-A: the
 * simulator reports speeds, from which the mean speed is formed): the whole
 * number of 2^-20 m/s units in v, 0 for v <= 0 (speeds are never negative)
 * and saturated at 2^32 - 1 from 4096 m/s on.
 * Scaling by a power of two is exact and the conversion truncates, so each
 * vehicle adds an exact integer and the sum is the same in any order. */
static uint64_t speed_fx(float v)
{
    if (v >= 4096.0f)
        return 0xFFFFFFFFull;
    return v > 0.0f ? (uint64_t)(uint32_t)(v * 1048576.0f) : 0u;
}

/* ---------------------------------------------------------------- IDM --- */

static float fmin32(float x, float y) { return x < y ? x : y; }
static float fmax32(float x, float y) { return x > y ? x : y; }

/* IDM acceleration (Treiber, Hennecke, Helbing 2000) with exponent 4:
 *   a_max * (1 - (v/v0)^4 - (s*(v, dv) / gap)^2),
 *   s* = s0 + max(0, v*T + v*dv / (2*sqrt(a_max*b))),
 * the last term evaluated as v*dv times the FP32 reciprocal of 2*sqrt(a_max*b)
 * formed in double [reading: the paper prints no formula].
 * Without a leader only the free-road term remains.  A non-positive gap
 * returns the braking limit [reading: guards the division]. */
float orc_idm(float v, float v0e, int has_leader, float v_lead, float gap, float a_max,
              float inv_tsab, float s0, float T, float b_max)
{
    float r = v / v0e;
    float r2 = r * r;
    float r4 = r2 * r2;
    float free_term = 1.0f - r4;
    if (!has_leader)
        return a_max * free_term;
    if (gap <= 0.0f)
        return -b_max;
    float dv = v - v_lead;
    float t1 = v * T;
    float t2 = (v * dv) * inv_tsab;
    float tt = t1 + t2;
    float ss = s0 + (tt > 0.0f ? tt : 0.0f);
    float q = ss / gap;
    return a_max * (free_term - q * q);
}

/* ---------------------------------------------------- learned closure --- */

/* bfloat16 rounding of a float (nearest, ties to even), as a double */
static double bf16r(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    float r;
    memcpy(&r, &u, 4);
    return (double)r;
}

/* GELU, tanh form (Hendrycks & Gimpel 2016) */
static double gelu_d(double x)
{
    const double k0 = 0.7978845608028654, k1 = 0.044715;
    return 0.5 * x * (1.0 + tanh(k0 * (x + k1 * x * x * x)));
}

/* Network input as a pair of bfloat16 numbers: hi = bf16(z), lo = bf16(z - hi)
 * (the difference taken in float, where it is exact); the first layer sees
 * hi + lo. */
static double bf16x2r(float z)
{
    const float hi = (float)bf16r(z);
    return (double)hi + bf16r(z - hi);
}

/* 8 -> 64 -> 64 -> 1 network; inputs as bfloat16 pairs, weights and hidden
 * layer inputs rounded to bfloat16, sums in double. */
double orc_mlp_forward(const float *theta, const float *z)
{
    const float *W1 = theta, *b1 = theta + 512, *W2 = theta + 576, *b2 = theta + 4672,
                *w3 = theta + 4736, *b3 = theta + 4800;
    double zq[8], h1[64], h2[64];
    for (int i = 0; i < 8; ++i) zq[i] = bf16x2r(z[i]);
    for (int j = 0; j < 64; ++j) {
        double acc = b1[j];
        for (int i = 0; i < 8; ++i) acc += bf16r(W1[j * 8 + i]) * zq[i];
        h1[j] = bf16r((float)gelu_d(acc));
    }
    for (int j = 0; j < 64; ++j) {
        double acc = b2[j];
        for (int i = 0; i < 64; ++i) acc += bf16r(W2[j * 64 + i]) * h1[i];
        h2[j] = bf16r((float)gelu_d(acc));
    }
    double y = b3[0];
    for (int i = 0; i < 64; ++i) y += bf16r(w3[i]) * h2[i];
    return y;
}

/* ---------------------------- closure parity: admissible outputs --- *
 *
 * The closure rounds its hidden activations to bfloat16.  An evaluation that
 * sums in FP32 in another order, evaluates GELU to within a few FP32 ulps and
 * takes the logarithm of a distance input to within one FP32 ulp reaches each
 * activation before rounding only to within a bounded error.  Where that
 * interval around this oracle's FP64 value holds a bfloat16 rounding
 * boundary, both roundings are correct results of the definition.
 * orc_mlp_candidates lists the network outputs of every such choice (each
 * limited to [lo, hi] like the simulator's acceleration); the first is the
 * oracle's own value.  Error model (u = 2^-24):
 *   - a sum of K exact products plus a bias: (K + 3) u times the sum of the
 *     magnitudes of its terms (K = 16 bfloat16 halves in layer 1, 64 in
 *     layer 2), the classical bound for recursive summation, any order;
 *   - GELU: derivative times the input error, plus (4 |a| + 8) u relative
 *     for the form x / (1 + 2^a), a = -2 sqrt(2/pi)(x + 0.044715 x^3) log2 e,
 *     with FP32 constants, exp2 and reciprocal each within one ulp;
 *   - ln of a distance: any float within two ulps of the exact value, i.e.
 *     this oracle's rounded value or one of the two floats on either side. */

#define ORC_U32 5.9604644775390625e-08

static double gelu_tol(double x, double ex)
{
    const double k0 = 0.7978845608028654, k1 = 0.044715;
    const double w = k0 * (x + k1 * x * x * x);
    const double th = tanh(w);
    const double g = 0.5 * x * (1.0 + th);
    const double dg = 0.5 * (1.0 + th) + 0.5 * x * (1.0 - th * th) * k0 * (1.0 + 3.0 * k1 * x * x);
    const double a = fabs(2.0 * w * 1.4426950408889634);
    return fabs(dg) * ex + (4.0 * a + 8.0) * ORC_U32 * fabs(g);
}

/* bfloat16 value of g and, if some value within e of g rounds (to float, then
 * to bfloat16) differently, that other value in *alt; returns 1 then */
static int bf16_window(double g, double e, double *nom, double *alt)
{
    *nom = bf16r((float)g);
    const double rl = bf16r((float)(g - e)), rh = bf16r((float)(g + e));
    if (rl != *nom) { *alt = rl; return 1; }
    if (rh != *nom) { *alt = rh; return 1; }
    return 0;
}

typedef struct {
    double *y;
    int32_t n, cap;
    double lo, hi;
} cand_t;

static void cand_add(cand_t *c, double y)
{
    y = y < c->lo ? c->lo : (y > c->hi ? c->hi : y);
    for (int32_t q = 0; q < c->n; ++q)
        if (c->y[q] == y) return;
    if (c->n < c->cap) c->y[c->n++] = y;
}

/* choices over a layer's tied units: every subset when there are at most 4,
 * else none and each one alone */
static int32_t n_choices(int32_t nt) { return nt <= 4 ? (1 << nt) : nt + 1; }
static int flipped(int32_t nt, int32_t choice, int32_t k)
{
    return nt <= 4 ? (choice >> k) & 1 : choice == k + 1;
}

/* all outputs from one input vector zq (bfloat16 pairs); ties of the first
 * choice counted in info[0] (layer 1) and info[1] (layer 2), the first tied
 * unit in info[3] (64 * layer + unit, -1 none) */
static void mlp_tied_outputs(const float *theta, const double *zq, cand_t *c, int32_t *info)
{
    const float *W1 = theta, *b1 = theta + 512, *W2 = theta + 576, *b2 = theta + 4672,
                *w3 = theta + 4736, *b3 = theta + 4800;
    double h1n[64], h1a[64], h1[64], h2n[64], h2a[64], h2[64];
    int32_t t1[64], nt1 = 0;
    for (int j = 0; j < 64; ++j) {
        double acc = b1[j], mag = fabs((double)b1[j]);
        for (int i = 0; i < 8; ++i) {
            const double w = bf16r(W1[j * 8 + i]);
            acc += w * zq[i];
            mag += fabs(w * zq[i]);
        }
        const double e = gelu_tol(acc, (16 + 3) * ORC_U32 * mag);
        if (bf16_window(gelu_d(acc), e, &h1n[j], &h1a[j])) t1[nt1++] = j;
    }
    if (info && info[0] < 0) {
        info[0] = nt1;
        if (nt1 && info[3] < 0) info[3] = t1[0];
    }
    for (int32_t c1 = 0; c1 < n_choices(nt1); ++c1) {
        memcpy(h1, h1n, sizeof h1);
        for (int32_t k = 0; k < nt1; ++k)
            if (flipped(nt1, c1, k)) h1[t1[k]] = h1a[t1[k]];
        int32_t t2[64], nt2 = 0;
        for (int j = 0; j < 64; ++j) {
            double acc = b2[j], mag = fabs((double)b2[j]);
            for (int i = 0; i < 64; ++i) {
                const double w = bf16r(W2[j * 64 + i]);
                acc += w * h1[i];
                mag += fabs(w * h1[i]);
            }
            const double e = gelu_tol(acc, (64 + 3) * ORC_U32 * mag);
            if (bf16_window(gelu_d(acc), e, &h2n[j], &h2a[j])) t2[nt2++] = j;
        }
        if (info && c1 == 0 && info[1] < 0) {
            info[1] = nt2;
            if (nt2 && info[3] < 0) info[3] = 64 + t2[0];
        }
        for (int32_t c2 = 0; c2 < n_choices(nt2); ++c2) {
            memcpy(h2, h2n, sizeof h2);
            for (int32_t k = 0; k < nt2; ++k)
                if (flipped(nt2, c2, k)) h2[t2[k]] = h2a[t2[k]];
            double y = b3[0];
            for (int i = 0; i < 64; ++i) y += bf16r(w3[i]) * h2[i];
            cand_add(c, y);
        }
    }
}

int32_t orc_mlp_candidates(const float *theta, const float *norm, const float *f, float lo,
                           float hi, int32_t cap, double *out, int32_t *info)
{
    const float *mean = norm, *inv = norm + 8;
    /* distinct input pairs per input: the five logarithm candidates of a
     * distance may give up to five */
    double zc[8][5];
    int32_t nz[8];
    for (int q = 0; q < 8; ++q) {
        nz[q] = 0;
        const int is_log = q == 0 || q == 4 || q == 6;
        float xs[5];
        int nx = 1;
        if (is_log) {
            const float c = (float)log(fmax32(f[q], 0.5f));
            xs[0] = c;
            xs[1] = nextafterf(c, -INFINITY);
            xs[2] = nextafterf(c, INFINITY);
            xs[3] = nextafterf(xs[1], -INFINITY);
            xs[4] = nextafterf(xs[2], INFINITY);
            nx = 5;
        } else {
            xs[0] = f[q];
        }
        for (int k = 0; k < nx; ++k) {
            const double zq = bf16x2r((xs[k] - mean[q]) * inv[q]);
            int seen = 0;
            for (int r = 0; r < nz[q]; ++r) seen |= zc[q][r] == zq;
            if (!seen) zc[q][nz[q]++] = zq;
        }
    }
    int32_t inf[4] = {-1, -1, 1, -1};
    for (int q = 0; q < 8; ++q) inf[2] *= nz[q];
    cand_t c = {out, 0, cap, lo, hi};
    /* every combination of the inputs' pairs, the oracle's own first */
    for (int32_t combo = 0; combo < inf[2]; ++combo) {
        double zq[8];
        int32_t r = combo;
        for (int q = 0; q < 8; ++q) {
            zq[q] = zc[q][r % nz[q]];
            r /= nz[q];
        }
        mlp_tied_outputs(theta, zq, &c, inf);
    }
    if (info) memcpy(info, inf, sizeof inf);
    return c.n;
}

void orc_mlp_candidates_batch(const float *theta, const float *norm, int32_t n, const float *feat,
                              float lo, float hi, int32_t cap, double *out, int32_t *n_out,
                              int32_t *info, int32_t threads)
{
#pragma omp parallel for schedule(dynamic, 256) num_threads(threads > 0 ? threads : 1)
    for (int32_t i = 0; i < n; ++i)
        n_out[i] = orc_mlp_candidates(theta, norm, feat + (size_t)i * 8, lo, hi, cap,
                                      out + (size_t)i * cap, info ? info + (size_t)i * 4 : NULL);
}

/* -------------------------------------------------------------- model --- */

typedef struct {
    float dt, a_max, b, s0, T, len, b_max, b_safe, p, a_thr, p_lc, d_look;
    float inv_tsab;        /* fl32(1/(2*sqrt(a_max*b))), formed in double */
    float inv_2bmax;       /* fl32(1/(2*b_max)), formed in double */
    float b_mand, tau_yield;
    int32_t h_look;
    uint32_t key0, key1;
} params_t;

enum { ST_STAY = 0, ST_JOIN = 1, ST_ARRIVE = 2 };

typedef struct {
    float s, v, a;
    int32_t lane, cur;
    int32_t veh;       /* vehicle table index */
    int32_t status;
    int32_t src_lane;  /* lane at step start (-1 for an insertion) */
    /* per-vehicle contributions to the counters, added up in row order
     * after the update phase: lane change made, closure use (1 evaluated,
     * 2 fell back to IDM), squared closure-vs-IDM difference */
    int32_t changed, mlp;
    double mlp_e2;
} prop_t;

struct orc_sim {
    params_t P;
    int32_t n_nodes, n_roads, n_lanes, n_scen, n_veh;
    int32_t *road_from, *road_to, *road_nlanes, *road_lane0;
    float *road_length, *lane_vlim;
    int32_t *lane_scen, *lane_road, *lane_k;
    double *node_x, *node_y;          /* NULL without coordinates */
    int32_t *node_cycle, *node_phase, *node_offset;
    int32_t *node_manual;             /* phase held by control, -1: fixed-time plan */
    uint8_t *lane_closed;             /* lane restriction by control: 1 closed */
    /* junction internal lanes (NULL without) */
    uint8_t *road_internal;
    int32_t *succ_off, *succ, *conf_off, *conf, *conf_feed;
    uint8_t *succ_en;                 /* successor entry in use (dynamic lanes) */
    int8_t *road_group;
    uint32_t *vid;
    int32_t *depart;
    float *v0;
    int64_t *route_off;
    int32_t *route_len;
    int32_t *routes;
    /* trips: arrival step (-1 before arrival) and the route distance at which
     * each vehicle entered the simulation (road lengths before its starting
     * road plus its starting position; 0 for a vehicle inserted at a route
     * start) */
    int64_t *arr;
    double *dist0;
    /* active state, lane order */
    int32_t n_act;
    int32_t *ls;       /* lane segment starts, n_lanes+1 */
    int32_t *sl;       /* lane of each slot */
    int32_t *vi;
    float *s, *v, *a;
    int32_t *cur;
    /* departure queues per origin lane */
    int32_t *q_start, *q_end, *q_head, *q_list;
    int64_t t;
    int64_t *cnt;      /* [n_scen][ORC_N_COUNTERS] */
    uint64_t *sumv;    /* [n_scen] sum of speed_fx over steps and vehicles */
    double *mlp_sq;    /* [n_scen] */
    int32_t mode;
    int32_t threads;   /* OpenMP threads of the update and merge loops */
    float mlp_theta[4801];
    float mlp_norm[32];
    /* decisions of the last step, indexed by slot at step start */
    int32_t dbg_n;
    uint32_t *d_id, *d_leader, *d_tl, *d_tf;
    int32_t *d_flags;
    float *d_margin;
    /* network mode: raw inputs [8] of each vehicle's closure and its use
     * (1 evaluated, 2 outside the envelope), same order */
    float *d_feat;
    int8_t *d_use;
};

/* copies an input array; size 0 or NULL source yields a zero-filled block */
static void *dup_arr(const void *src, size_t n, size_t elt)
{
    size_t bytes = n * elt;
    void *p = malloc(bytes ? bytes : 1);
    if (!p)
        return NULL;
    if (src && bytes)
        memcpy(p, src, bytes);
    else
        memset(p, 0, bytes ? bytes : 1);
    return p;
}

static void free_sim(orc_sim *m)
{
    if (!m)
        return;
    void *ptrs[] = {m->road_from, m->road_to, m->road_nlanes, m->road_lane0, m->road_length,
                    m->lane_vlim, m->lane_scen, m->lane_road, m->lane_k, m->node_cycle,
                    m->node_phase, m->node_offset, m->road_group, m->vid, m->depart, m->v0,
                    m->route_off, m->route_len, m->routes, m->ls, m->sl, m->vi, m->s, m->v,
                    m->a, m->cur, m->q_start, m->q_end, m->q_head, m->q_list, m->cnt, m->sumv, m->mlp_sq,
                    m->d_id, m->d_leader, m->d_tl, m->d_tf, m->d_flags, m->d_margin,
                    m->node_x, m->node_y, m->node_manual, m->d_feat, m->d_use, m->arr,
                    m->dist0, m->lane_closed, m->road_internal, m->succ_off, m->succ,
                    m->conf_off, m->conf, m->conf_feed, m->succ_en};
    for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; ++i)
        free(ptrs[i]);
    free(m);
}

void orc_destroy(orc_sim *m) { free_sim(m); }

/* ------------------------------------------------------------ create --- */

typedef struct { int32_t lane; float s; uint32_t id; int32_t veh; } place_t;

static int cmp_place(const void *x, const void *y)
{
    const place_t *p = x, *q = y;
    if (p->lane != q->lane) return p->lane < q->lane ? -1 : 1;
    if (p->s != q->s) return p->s < q->s ? -1 : 1;
    return p->id < q->id ? -1 : (p->id > q->id);
}

typedef struct { int32_t lane, depart; uint32_t id; int32_t veh; } pend_t;

static int cmp_pend(const void *x, const void *y)
{
    const pend_t *p = x, *q = y;
    if (p->lane != q->lane) return p->lane < q->lane ? -1 : 1;
    if (p->depart != q->depart) return p->depart < q->depart ? -1 : 1;
    return p->id < q->id ? -1 : (p->id > q->id);
}

static int permits(const orc_sim *m, int32_t x, int32_t rd);

/* Origin lane of a pending vehicle i (see the departure queues in orc_create). */
static int32_t origin_lane(const orc_sim *m, int32_t i)
{
    const int32_t r0 = m->routes[m->route_off[i]], l0 = m->road_lane0[r0];
    const int32_t n = m->road_nlanes[r0];
    int32_t ok[256], cnt = 0;
    if (m->route_len[i] > 1) {
        const int32_t r1 = m->routes[m->route_off[i] + 1];
        for (int32_t k = 0; k < n; ++k)
            if (permits(m, l0 + k, r1))
                ok[cnt++] = l0 + k;
    }
    if (cnt == 0)
        return l0 + (int32_t)(m->vid[i] % (uint32_t)n);
    return ok[m->vid[i] % (uint32_t)cnt];
}

/* Length of the first c roads of vehicle i's route, summed in FP64 in route
 * order. */
static double route_dist(const orc_sim *m, int32_t i, int32_t c)
{
    double d = 0.0;
    for (int32_t k = 0; k < c; ++k)
        d += (double)m->road_length[m->routes[m->route_off[i] + k]];
    return d;
}

orc_sim *orc_create(const orc_input *in)
{
    orc_sim *m = calloc(1, sizeof *m);
    if (!m) { set_err("out of memory"); return NULL; }
    m->n_nodes = in->n_nodes; m->n_roads = in->n_roads; m->n_lanes = in->n_lanes;
    m->n_scen = in->n_scen > 0 ? in->n_scen : 1; m->n_veh = in->n_veh;
    int32_t R = m->n_roads, Lc = m->n_lanes, N = m->n_veh;

    m->road_from = dup_arr(in->road_from, R, 4);
    m->road_to = dup_arr(in->road_to, R, 4);
    m->road_nlanes = dup_arr(in->road_nlanes, R, 4);
    m->road_lane0 = dup_arr(in->road_lane0, R, 4);
    m->road_length = dup_arr(in->road_length, R, 4);
    m->lane_vlim = dup_arr(in->lane_vlim, Lc, 4);
    m->lane_scen = dup_arr(in->lane_scen, Lc, 4);
    if (in->node_x && in->node_y) {
        m->node_x = dup_arr(in->node_x, m->n_nodes, 8);
        m->node_y = dup_arr(in->node_y, m->n_nodes, 8);
    }
    m->lane_closed = calloc((size_t)Lc + 1, 1);
    if (in->lane_succ_off) {
        m->road_internal = dup_arr(in->road_internal, R, 1);
        m->succ_off = dup_arr(in->lane_succ_off, (size_t)Lc + 1, 4);
        m->succ = dup_arr(in->lane_succ, (size_t)m->succ_off[Lc], 4);
        m->conf_off = dup_arr(in->lane_conf_off, (size_t)Lc + 1, 4);
        m->conf = dup_arr(in->lane_conf, (size_t)m->conf_off[Lc], 4);
        m->conf_feed = dup_arr(in->lane_conf_feed, (size_t)m->conf_off[Lc], 4);
        m->succ_en = malloc((size_t)m->succ_off[Lc] + 1);
        memset(m->succ_en, 1, (size_t)m->succ_off[Lc] + 1);
    }
    m->node_manual = malloc(sizeof(int32_t) * ((size_t)m->n_nodes + 1));
    for (int32_t j = 0; j < m->n_nodes; ++j)
        m->node_manual[j] = -1;
    m->node_cycle = dup_arr(in->node_cycle, m->n_nodes, 4);
    m->node_phase = dup_arr(in->node_phase, m->n_nodes, 4);
    m->node_offset = dup_arr(in->node_offset, m->n_nodes, 4);
    m->road_group = dup_arr(in->road_group, R, 1);
    m->vid = dup_arr(in->veh_id, N, 4);
    m->depart = dup_arr(in->depart, N, 4);
    m->v0 = dup_arr(in->v0, N, 4);
    m->route_off = dup_arr(in->route_off, (size_t)N + 1, 8);
    m->route_len = malloc(sizeof(int32_t) * (N ? N : 1));
    int64_t n_route = N ? in->route_off[N] : 0;
    m->routes = dup_arr(in->route_roads, (size_t)n_route, 4);
    m->lane_road = malloc(sizeof(int32_t) * (Lc ? Lc : 1));
    m->lane_k = malloc(sizeof(int32_t) * (Lc ? Lc : 1));
    for (int32_t r = 0; r < R; ++r)
        for (int32_t k = 0; k < m->road_nlanes[r]; ++k) {
            m->lane_road[m->road_lane0[r] + k] = r;
            m->lane_k[m->road_lane0[r] + k] = k;
        }
    for (int32_t i = 0; i < N; ++i)
        m->route_len[i] = (int32_t)(m->route_off[i + 1] - m->route_off[i]);
    m->arr = malloc(sizeof(int64_t) * (N ? N : 1));
    m->dist0 = calloc(N ? N : 1, sizeof(double));
    for (int32_t i = 0; i < N; ++i)
        m->arr[i] = -1;

    params_t *P = &m->P;
    P->dt = in->dt; P->a_max = in->a_max; P->b = in->b; P->s0 = in->s0; P->T = in->T;
    P->len = in->length; P->b_max = in->b_max; P->b_safe = in->b_safe; P->p = in->politeness;
    P->a_thr = in->a_thr; P->p_lc = in->p_lc; P->d_look = in->d_look; P->h_look = in->h_look;
    P->b_mand = in->b_mand; P->tau_yield = in->tau_yield;
    P->inv_tsab = (float)(1.0 / (2.0 * sqrt((double)in->a_max * (double)in->b)));
    P->inv_2bmax = (float)(1.0 / (2.0 * (double)in->b_max));
    P->key0 = (uint32_t)(in->seed & 0xFFFFFFFFu);
    P->key1 = (uint32_t)(in->seed >> 32);
    m->t = in->t0;

    /* pre-placed vehicles: ordered by (lane, s, id) */
    int32_t n_pl = 0;
    for (int32_t i = 0; i < N; ++i)
        if (in->placed && in->placed[i]) ++n_pl;
    place_t *pl = malloc(sizeof(place_t) * (n_pl ? n_pl : 1));
    int32_t j = 0;
    for (int32_t i = 0; i < N; ++i)
        if (in->placed && in->placed[i]) {
            pl[j].lane = in->lane[i]; pl[j].s = in->s[i]; pl[j].id = m->vid[i]; pl[j].veh = i; ++j;
        }
    qsort(pl, n_pl, sizeof(place_t), cmp_place);
    size_t cap = (size_t)N + (size_t)Lc + 1;
    m->ls = calloc((size_t)Lc + 1, 4);
    m->sl = malloc(4 * cap); m->vi = malloc(4 * cap); m->cur = malloc(4 * cap);
    m->s = malloc(4 * cap); m->v = malloc(4 * cap); m->a = malloc(4 * cap);
    m->d_id = malloc(4 * cap); m->d_leader = malloc(4 * cap); m->d_tl = malloc(4 * cap);
    m->d_tf = malloc(4 * cap); m->d_flags = malloc(4 * cap); m->d_margin = malloc(4 * cap);
    for (int32_t k = 0; k < n_pl; ++k) {
        int32_t i = pl[k].veh;
        m->sl[k] = pl[k].lane; m->vi[k] = i; m->s[k] = in->s[i]; m->v[k] = in->v[i];
        m->a[k] = in->a[i]; m->cur[k] = in->cursor[i];
        m->ls[pl[k].lane + 1]++;
        if (pl[k].lane < 0 || pl[k].lane >= Lc || m->cur[k] < 0 || m->cur[k] >= m->route_len[i]
            || m->routes[m->route_off[i] + m->cur[k]] != m->lane_road[pl[k].lane]) {
            set_err("pre-placed vehicle is not on the road its route cursor names");
            free(pl); free_sim(m); return NULL;
        }
        if (k > 0 && pl[k - 1].lane == pl[k].lane && !(m->s[k - 1] <= m->s[k] - P->len)) {
            set_err("pre-placed vehicles overlap");
            free(pl); free_sim(m); return NULL;
        }
    }
    for (int32_t l = 0; l < Lc; ++l)
        m->ls[l + 1] += m->ls[l];
    m->n_act = n_pl;
    for (int32_t k = 0; k < n_pl; ++k) {
        int32_t i = m->vi[k];
        m->dist0[i] = route_dist(m, i, m->cur[k]) + (double)m->s[k];
    }
    free(pl);

    /* pending vehicles queue on an origin lane of their first road [reading]:
     * among the lanes of that road that continue along the route (all of them
     * without junction lanes, or for a one-road route), the one of index id
     * mod their number; in (depart, id) order */
    int32_t n_pe = N - n_pl;
    pend_t *pe = malloc(sizeof(pend_t) * (n_pe ? n_pe : 1));
    j = 0;
    for (int32_t i = 0; i < N; ++i)
        if (!(in->placed && in->placed[i])) {
            pe[j].lane = origin_lane(m, i);
            pe[j].depart = m->depart[i]; pe[j].id = m->vid[i]; pe[j].veh = i; ++j;
        }
    qsort(pe, n_pe, sizeof(pend_t), cmp_pend);
    m->q_start = calloc((size_t)Lc + 1, 4);
    m->q_end = calloc((size_t)Lc + 1, 4);
    m->q_head = calloc((size_t)Lc + 1, 4);
    m->q_list = malloc(4 * (size_t)(n_pe ? n_pe : 1));
    for (int32_t k = 0; k < n_pe; ++k) {
        m->q_list[k] = pe[k].veh;
        m->q_end[pe[k].lane]++;
    }
    int32_t acc = 0;
    for (int32_t l = 0; l < Lc; ++l) {
        m->q_start[l] = acc; m->q_head[l] = acc; acc += m->q_end[l]; m->q_end[l] = acc;
    }
    free(pe);
    m->cnt = calloc((size_t)m->n_scen * ORC_N_COUNTERS, 8);
    m->sumv = calloc((size_t)m->n_scen, 8);
    m->mlp_sq = calloc((size_t)m->n_scen, 8);
    m->mode = in->mode;
    m->threads = 1;
    if (in->mode == 1) {
        memcpy(m->mlp_theta, in->mlp_theta, sizeof m->mlp_theta);
        memcpy(m->mlp_norm, in->mlp_norm, sizeof m->mlp_norm);
        size_t capd = (size_t)N + (size_t)Lc + 1;
        m->d_feat = malloc(4 * 8 * capd);
        m->d_use = malloc(capd);
    }
    return m;
}

/* ------------------------------------------------------------ helpers --- */

static float road_len(const orc_sim *m, int32_t lane) { return m->road_length[m->lane_road[lane]]; }

/* Signal reading [reading]: a node with cycle C, phase length P and offset O
 * shows phase ((t + O) mod C) div P; an in-road of group g may enter the
 * junction only while that phase equals g.  Group -1, unsignalised nodes and
 * the last road of a route are always green. */
static int red_for(const orc_sim *m, int32_t road, int64_t t)
{
    int32_t g = m->road_group[road];
    int32_t node = m->road_to[road];
    if (g < 0 || m->node_cycle[node] <= 0)
        return 0;
    if (m->node_manual[node] >= 0)        /* held by signal control */
        return m->node_manual[node] != g;
    int64_t c = m->node_cycle[node];
    int64_t ph = ((t + m->node_offset[node]) % c) / m->node_phase[node];
    return ph != g;
}

/* Lane index taken on road rd by a vehicle coming from lane index k
 * [reading]: min(k, lanes-1); when control has closed that lane, the open
 * lane nearest to it, the lower one of two equally near (a road always keeps
 * an open lane). */
static int32_t pick_lane(const orc_sim *m, int32_t rd, int32_t k)
{
    const int32_t n = m->road_nlanes[rd], l0 = m->road_lane0[rd];
    int32_t kk = k > n - 1 ? n - 1 : k;
    if (!m->lane_closed[l0 + kk])
        return kk;
    for (int32_t dd = 1; dd < n; ++dd) {
        if (kk - dd >= 0 && !m->lane_closed[l0 + kk - dd])
            return kk - dd;
        if (kk + dd < n && !m->lane_closed[l0 + kk + dd])
            return kk + dd;
    }
    return kk;
}

/* Lane connectivity inside junctions [reading; junction internal lanes].
 * succ_on: the successor of lane x on road rd in x's successor list, -1 if
 * x has a list without an entry in use on rd or has no list (control may
 * take entries out of use: dynamic lanes). */
static int32_t succ_on(const orc_sim *m, int32_t x, int32_t rd)
{
    if (!m->succ_off)
        return -1;
    for (int32_t q = m->succ_off[x]; q < m->succ_off[x + 1]; ++q)
        if (m->succ_en[q] && m->lane_road[m->succ[q]] == rd)
            return m->succ[q];
    return -1;
}

/* Whether lane x lets a vehicle continue onto road rd: x has no successor
 * list (every lane continues), or its list has a lane on rd. */
static int permits(const orc_sim *m, int32_t x, int32_t rd)
{
    if (!m->succ_off || m->succ_off[x] == m->succ_off[x + 1])
        return 1;
    return succ_on(m, x, rd) >= 0;
}

/* The lane a vehicle takes on road rd after lane x: x's successor there
 * (the open lane nearest to it if control closed it), else the lane of
 * index pick_lane(k) with k the index of x in its road. */
static int32_t step_lane(const orc_sim *m, int32_t x, int32_t rd)
{
    int32_t y = succ_on(m, x, rd);
    if (y >= 0)
        return m->lane_closed[y] ? m->road_lane0[rd] + pick_lane(m, rd, m->lane_k[y]) : y;
    return m->road_lane0[rd] + pick_lane(m, rd, m->lane_k[x]);
}

typedef struct { int has; float v, gap; uint32_t id; } leader_t;

/* Leader beyond the end of the vehicle's lane [reading]: follow the route for
 * at most h_look roads and while the distance already covered is within
 * d_look; on each next road take the lane step_lane gives after the previous one and
 * use its last vehicle (lowest position) as leader.  A vehicle never leads
 * itself (a ring road with one vehicle). */
static leader_t lookahead(const orc_sim *m, int32_t lane, float s, int32_t veh, int32_t cur)
{
    leader_t L = {0, 0.0f, 0.0f, ORC_NONE};
    float dist = road_len(m, lane) - s;
    int32_t y = lane;
    int32_t c = cur;
    for (int32_t h = 0; h < m->P.h_look; ++h) {
        if (c + 1 >= m->route_len[veh])
            break;
        if (dist > m->P.d_look)
            break;
        c += 1;
        int32_t rd = m->routes[m->route_off[veh] + c];
        y = step_lane(m, y, rd);
        if (m->ls[y] < m->ls[y + 1]) {
            int32_t tail = m->ls[y];
            if (m->vi[tail] != veh) {
                L.has = 1;
                L.v = m->v[tail];
                L.gap = (dist + m->s[tail]) - m->P.len;
                L.id = m->vid[m->vi[tail]];
            }
            return L;
        }
        dist = dist + m->road_length[rd];
    }
    return L;
}

static float idm_p(const params_t *P, float v, float v0e, int has, float vl, float gap)
{
    return orc_idm(v, v0e, has, vl, gap, P->a_max, P->inv_tsab, P->s0, P->T, P->b_max);
}

/* Yield rule at a junction [reading]: connector lane cl is busy when one of
 * the conflicting connector lanes with priority over it holds a vehicle, or
 * the lane feeding such a connector has a first vehicle that is headed into
 * it, not held by a red light, and within tau_yield seconds of its stop line
 * at its current speed (L - s <= v * tau_yield; a standing vehicle is not
 * approaching).  Everything read is the state at the start of the step. */
static int conflict_busy(const orc_sim *m, int32_t cl, int64_t t)
{
    for (int32_t q = m->conf_off[cl]; q < m->conf_off[cl + 1]; ++q) {
        const int32_t c2 = m->conf[q], f = m->conf_feed[q];
        if (m->ls[c2] < m->ls[c2 + 1])
            return 1;
        if (m->ls[f] < m->ls[f + 1]) {
            const int32_t hd = m->ls[f + 1] - 1, hv = m->vi[hd], hc = m->cur[hd];
            if (hc + 1 < m->route_len[hv] &&
                m->routes[m->route_off[hv] + hc + 1] == m->lane_road[c2] &&
                !red_for(m, m->lane_road[f], t) &&
                road_len(m, f) - m->s[hd] <= m->v[hd] * m->P.tau_yield)
                return 1;
        }
    }
    return 0;
}

/* --------------------------------------------------------- update phase --- */

/* One vehicle of the snapshot: everything read here belongs to the state at
 * the start of the step; the result goes to the proposal only. */
static void update_vehicle(orc_sim *m, int32_t i, prop_t *out)
{
    const params_t *P = &m->P;
    const int64_t t = m->t;
    int32_t l = m->sl[i];
    int32_t r = m->lane_road[l];
    int32_t k = m->lane_k[l];
    int32_t nl = m->road_nlanes[r];
    float L = m->road_length[r];
    int32_t veh = m->vi[i];
    uint32_t id = m->vid[veh];
    float s = m->s[i], v = m->v[i];
    out->changed = 0; out->mlp = 0; out->mlp_e2 = 0.0;
    float v0 = m->v0[veh];
    int32_t c = m->cur[i];
    int has_next = c + 1 < m->route_len[veh];
    int32_t lo = m->ls[l], hi = m->ls[l + 1];

    m->d_id[i] = id; m->d_leader[i] = ORC_NONE; m->d_tl[i] = ORC_NONE; m->d_tf[i] = ORC_NONE;
    m->d_flags[i] = 0; m->d_margin[i] = 0.0f;

    int32_t nr = has_next ? m->routes[m->route_off[veh] + c + 1] : -1;

    /* in-lane neighbours through the ordering */
    int32_t Lc = (i + 1 < hi) ? i + 1 : -1;
    int32_t o = (i - 1 >= lo) ? i - 1 : -1;

    /* --- randomised MOBIL (Kesting, Treiber, Helbing 2007) ---
     * [reading] one side per step: even steps look at lane k-1, odd steps at
     * k+1; only vehicles at s >= 0; neighbours within the same road only,
     * accelerations from IDM without signal or lookahead. */
    int change = 0;
    int32_t lt = -1, Lt = -1, nb = -1;
    /* no lane changes inside a junction (internal roads) */
    if (s >= 0.0f && !(m->road_internal && m->road_internal[r])) {
        int32_t kt = (t % 2 == 0) ? k - 1 : k + 1;
        /* a lane closed by control is never a target */
        if (kt >= 0 && kt < nl && !m->lane_closed[m->road_lane0[r] + kt]) {
            lt = m->road_lane0[r] + kt;
            /* brute force over the target lane: leader = lowest s_j >= s,
             * follower = highest s_j < s */
            for (int32_t j = m->ls[lt]; j < m->ls[lt + 1]; ++j) {
                if (m->s[j] >= s) {
                    if (Lt < 0 || m->s[j] < m->s[Lt]) Lt = j;
                } else {
                    if (nb < 0 || m->s[j] > m->s[nb]) nb = j;
                }
            }
            float vlim_c = m->lane_vlim[l], vlim_t = m->lane_vlim[lt];
            float v0e_c = fmin32(v0, vlim_c), v0e_t = fmin32(v0, vlim_t);
            float a_c = Lc >= 0 ? idm_p(P, v, v0e_c, 1, m->v[Lc], (m->s[Lc] - P->len) - s)
                                : idm_p(P, v, v0e_c, 0, 0.0f, 0.0f);
            float at_c = Lt >= 0 ? idm_p(P, v, v0e_t, 1, m->v[Lt], (m->s[Lt] - P->len) - s)
                                 : idm_p(P, v, v0e_t, 0, 0.0f, 0.0f);
            float d_o = 0.0f, d_n = 0.0f;
            int safe = 1;
            if (o >= 0) {
                float vo = m->v[o], so = m->s[o];
                float v0e_o = fmin32(m->v0[m->vi[o]], vlim_c);
                float a_o = idm_p(P, vo, v0e_o, 1, v, (s - P->len) - so);
                float at_o = Lc >= 0 ? idm_p(P, vo, v0e_o, 1, m->v[Lc], (m->s[Lc] - P->len) - so)
                                     : idm_p(P, vo, v0e_o, 0, 0.0f, 0.0f);
                d_o = at_o - a_o;
            }
            if (nb >= 0) {
                float vn = m->v[nb], sn = m->s[nb];
                float v0e_n = fmin32(m->v0[m->vi[nb]], vlim_t);
                float a_n = Lt >= 0 ? idm_p(P, vn, v0e_n, 1, m->v[Lt], (m->s[Lt] - P->len) - sn)
                                    : idm_p(P, vn, v0e_n, 0, 0.0f, 0.0f);
                float at_n = idm_p(P, vn, v0e_n, 1, v, (s - P->len) - sn);
                d_n = at_n - a_n;
                float gap_b = (s - P->len) - sn;
                if (!(gap_b > 0.0f)) safe = 0;
                if (!(at_n >= -P->b_safe)) safe = 0;
            }
            if (Lt >= 0) {
                float gap_f = (m->s[Lt] - P->len) - s;
                if (!(gap_f > 0.0f)) safe = 0;
            }
            float inc = (at_c - a_c) + P->p * (d_n + d_o);
            /* lanes that continue the route [reading]: a target lane that
             * does, when the own lane does not, adds b_mand to the incentive
             * (mandatory lane change); a target lane that does not, when the
             * own lane does, is never taken */
            int allowed = 1;
            if (has_next && m->succ_off) {
                const int pc = permits(m, l, nr), pt = permits(m, lt, nr);
                if (pt && !pc)
                    inc = inc + P->b_mand;
                else if (pc && !pt)
                    allowed = 0;
            }
            uint32_t ctr[4] = {(uint32_t)t, id, 0u, 0u}, key[2] = {P->key0, P->key1}, rnd[4];
            orc_philox4x32_10(ctr, key, rnd);
            float u = (float)(rnd[0] >> 8) * (1.0f / 16777216.0f);
            change = safe && allowed && inc > P->a_thr && u < P->p_lc;
            m->d_margin[i] = inc - P->a_thr;
            m->d_flags[i] |= change ? 2 : 1;
            m->d_tl[i] = Lt >= 0 ? m->vid[m->vi[Lt]] : ORC_NONE;
            m->d_tf[i] = nb >= 0 ? m->vid[m->vi[nb]] : ORC_NONE;
        }
    }

    /* --- car-following in the final lane --- */
    int32_t lf = change ? lt : l;
    leader_t ld = {0, 0.0f, 0.0f, ORC_NONE};
    int32_t lead_slot = change ? Lt : Lc;
    if (lead_slot >= 0) {
        ld.has = 1; ld.v = m->v[lead_slot]; ld.gap = (m->s[lead_slot] - P->len) - s;
        ld.id = m->vid[m->vi[lead_slot]];
    } else {
        ld = lookahead(m, lf, s, veh, c);
        if (ld.has) m->d_flags[i] |= 8;
    }
    m->d_leader[i] = ld.id;

    /* stop line [reading]: the end of the final lane is an obstacle (a
     * standing vehicle at the line) when the road's signal is red, or when
     * the vehicle, first in its lane, would enter a connector lane whose
     * conflicts with priority are busy; applied only if the vehicle can still
     * stop with the braking limit.  The last road of a route never stops.  A
     * vehicle still in a lane that does not continue its route (flag 32) is
     * not held: it takes the route's connector on the lane step_lane gives. */
    int red = 0;
    if (has_next) {
        int line = red_for(m, r, t);
        if (m->succ_off) {
            if (!permits(m, lf, nr))
                m->d_flags[i] |= 32;
            if (lead_slot < 0) {
                const int32_t cl = step_lane(m, lf, nr);
                if (conflict_busy(m, cl, t)) {
                    line = 1;
                    m->d_flags[i] |= 64;
                }
            }
        }
        if (line) {
            float stop_dist = (v * v) * P->inv_2bmax;
            if (L - s >= stop_dist)
                red = 1;
        }
    }
    float v0e = fmin32(v0, m->lane_vlim[lf]);
    float acc = idm_p(P, v, v0e, ld.has, ld.v, ld.gap);
    if (red) {
        float acc_red = idm_p(P, v, v0e, 1, 0.0f, L - s);
        acc = fmin32(acc, acc_red);
        m->d_flags[i] |= 4;
    }
    float a = fmax32(-P->b_max, acc);

    /* --- learned closure [reading]: inputs are the leader gap (d_look when
     * there is none or farther), own speed, leader speed (own speed when
     * none), effective desired speed, distance to a red stop line (d_look
     * when none), previous acceleration, distance to the lane end (at most
     * d_look) and the speed limit; inside the training envelope the network's
     * output, limited to [-b_max, a_max], replaces the IDM acceleration. --- */
    if (m->mode == 1) {
        float f[8];
        f[0] = ld.has ? fmin32(ld.gap, P->d_look) : P->d_look;
        f[1] = v;
        f[2] = ld.has ? ld.v : v;
        f[3] = v0e;
        f[4] = red ? fmin32(L - s, P->d_look) : P->d_look;
        f[5] = m->a[i];
        f[6] = fmin32(L - s, P->d_look);
        f[7] = m->lane_vlim[lf];
        const float *mean = m->mlp_norm, *inv = m->mlp_norm + 8, *lo = m->mlp_norm + 16,
                    *hi = m->mlp_norm + 24;
        int inside = 1;
        float z[8];
        for (int q = 0; q < 8; ++q) {
            if (!(f[q] >= lo[q] && f[q] <= hi[q])) inside = 0;
            /* distances (inputs 0, 4, 6) enter as ln(max(x, 0.5)) */
            float xt = (q == 0 || q == 4 || q == 6) ? (float)log(fmax32(f[q], 0.5f)) : f[q];
            z[q] = (xt - mean[q]) * inv[q];
        }
        memcpy(m->d_feat + (size_t)i * 8, f, sizeof f);
        m->d_use[i] = inside ? 1 : 2;
        if (inside) {
            float am = (float)orc_mlp_forward(m->mlp_theta, z);
            am = fmax32(-P->b_max, fmin32(am, P->a_max));
            double e = (double)am - (double)a;
            out->mlp_e2 = e * e;
            out->mlp = 1;
            a = am;
        } else {
            out->mlp = 2;
        }
    }

    /* --- Newton's equations over one step, stopping at v = 0 --- */
    float vn = v + a * P->dt;
    float dx;
    if (vn < 0.0f) {
        dx = -((v * v) / (2.0f * a));
        vn = 0.0f;
    } else {
        dx = v * P->dt + (0.5f * a) * (P->dt * P->dt);
    }
    float sp = s + dx;

    /* --- transfer along the route; arrival at the end of the last road --- */
    int32_t x = lf, c2 = c;
    while (sp >= road_len(m, x) && c2 + 1 < m->route_len[veh]) {
        sp = sp - road_len(m, x);
        c2 += 1;
        int32_t rd = m->routes[m->route_off[veh] + c2];
        x = step_lane(m, x, rd);
    }
    int arrived = sp >= road_len(m, x);
    out->s = sp; out->v = vn; out->a = a; out->lane = x; out->cur = c2; out->veh = veh;
    out->src_lane = l;
    out->status = arrived ? ST_ARRIVE : ((x == l && c2 == c) ? ST_STAY : ST_JOIN);
    if (arrived) m->d_flags[i] |= 16;
    out->changed = change;
}

/* ------------------------------------------------------- prepare phase --- */

static const orc_sim *g_sort_sim;
static int cmp_joiner(const void *x, const void *y)
{
    const prop_t *p = x, *q = y;
    if (p->lane != q->lane) return p->lane < q->lane ? -1 : 1;
    if (p->s != q->s) return p->s < q->s ? -1 : 1;
    uint32_t a = g_sort_sim->vid[p->veh], b = g_sort_sim->vid[q->veh];
    return a < b ? -1 : (a > b);
}

/* key order (s, id) used by the merge */
static int key_less(const orc_sim *m, const prop_t *p, const prop_t *q)
{
    if (p->s != q->s) return p->s < q->s;
    return m->vid[p->veh] < m->vid[q->veh];
}

static void one_step(orc_sim *m)
{
    const params_t *P = &m->P;
    const int64_t t = m->t;
    int32_t Lc = m->n_lanes;
    int32_t n = m->n_act;

    /* --- insertion [reading]: the head of each origin-lane queue may enter
     * when due, at most one per lane and step, if the lane is empty or the
     * gap behind its last vehicle is at least s0 + v*T for the entry speed
     * v = min(v0, speed limit, speed of that vehicle).  It joins the lane at
     * s = 0 at the end of the step. --- */
    prop_t *ins = malloc(sizeof(prop_t) * ((size_t)Lc + 1));
    int32_t n_ins = 0;
    for (int32_t l = 0; l < Lc; ++l) {
        if (m->q_head[l] >= m->q_end[l])
            continue;
        int32_t veh = m->q_list[m->q_head[l]];
        if (m->depart[veh] > t)
            continue;
        float v0e = fmin32(m->v0[veh], m->lane_vlim[l]);
        int ok;
        float vins;
        if (m->lane_closed[l]) {
            /* a closed lane holds its departure queue */
            ok = 0; vins = 0.0f;
        } else if (m->ls[l] == m->ls[l + 1]) {
            ok = 1; vins = v0e;
        } else {
            int32_t tail = m->ls[l];
            vins = fmin32(v0e, m->v[tail]);
            ok = (m->s[tail] - P->len) >= (P->s0 + vins * P->T);
        }
        size_t sc = (size_t)m->lane_scen[l] * ORC_N_COUNTERS;
        if (ok) {
            prop_t *q = &ins[n_ins++];
            q->s = 0.0f; q->v = vins; q->a = 0.0f; q->lane = l; q->cur = 0; q->veh = veh;
            q->status = ST_JOIN; q->src_lane = -1;
            m->q_head[l]++;
            m->cnt[sc + ORC_INSERTED]++;
        } else {
            m->cnt[sc + ORC_INSERT_FAIL]++;
        }
    }

    /* --- update phase: every vehicle reads the snapshot --- */
    prop_t *pr = malloc(sizeof(prop_t) * ((size_t)n + 1));
    /* vehicles are independent (each reads the snapshot and writes its own
     * proposal and debug row), so the loop may run on several threads */
#pragma omp parallel for schedule(dynamic, 1024) num_threads(m->threads)
    for (int32_t i = 0; i < n; ++i)
        update_vehicle(m, i, &pr[i]);
    m->dbg_n = n;
    for (int32_t i = 0; i < n; ++i) {
        size_t sc = (size_t)m->lane_scen[pr[i].src_lane];
        if (pr[i].changed) m->cnt[sc * ORC_N_COUNTERS + ORC_LANE_CHANGES]++;
        if (pr[i].mlp == 1) {
            m->mlp_sq[sc] += pr[i].mlp_e2;
            m->cnt[sc * ORC_N_COUNTERS + ORC_MLP_EVAL]++;
        } else if (pr[i].mlp == 2) {
            m->cnt[sc * ORC_N_COUNTERS + ORC_MLP_FALLBACK]++;
        }
    }

    /* --- arrivals --- */
    for (int32_t i = 0; i < n; ++i)
        if (pr[i].status == ST_ARRIVE) {
            size_t sc = (size_t)m->lane_scen[pr[i].src_lane] * ORC_N_COUNTERS;
            m->cnt[sc + ORC_ARRIVED]++;
            m->cnt[sc + ORC_TRIP_TIME] += (t + 1) - m->depart[pr[i].veh];
            m->arr[pr[i].veh] = t + 1;
        }

    /* --- joiners (lane changers, road transfers, insertions) by (lane, s, id) --- */
    int32_t n_join = 0;
    for (int32_t i = 0; i < n; ++i)
        if (pr[i].status == ST_JOIN) ++n_join;
    prop_t *jn = malloc(sizeof(prop_t) * ((size_t)n_join + n_ins + 1));
    int32_t nj = 0;
    for (int32_t i = 0; i < n; ++i)
        if (pr[i].status == ST_JOIN) jn[nj++] = pr[i];
    for (int32_t q = 0; q < n_ins; ++q)
        jn[nj++] = ins[q];
    g_sort_sim = m;
    qsort(jn, nj, sizeof(prop_t), cmp_joiner);

    /* --- per lane: stayers keep their order, joiners are merged in by
     * (s, id), then overlaps are removed from the head of the lane backwards
     * [reading: the paper does not model collisions] --- */
    size_t cap = (size_t)m->n_veh + (size_t)Lc + 1;
    int32_t *ls2 = calloc((size_t)Lc + 1, 4);
    int32_t *sl2 = malloc(4 * cap), *vi2 = malloc(4 * cap), *cur2 = malloc(4 * cap);
    float *s2 = malloc(4 * cap), *v2 = malloc(4 * cap), *a2 = malloc(4 * cap);
    prop_t *lanebuf = malloc(sizeof(prop_t) * ((size_t)n + nj + 1));
    /* each lane's joiners are jn[js[l] .. js[l+1]) (jn is sorted by lane);
     * its new rows start at ls2[l] = the rows of the lanes before it */
    int32_t *js = calloc((size_t)Lc + 1, 4);
    int64_t *clamps = calloc((size_t)Lc + 1, 8);
    for (int32_t q = 0; q < nj; ++q) js[jn[q].lane + 1]++;
    for (int32_t l = 0; l < Lc; ++l) {
        int32_t stay = 0;
        for (int32_t i = m->ls[l]; i < m->ls[l + 1]; ++i) stay += pr[i].status == ST_STAY;
        js[l + 1] += js[l];
        ls2[l + 1] = ls2[l] + stay + (js[l + 1] - js[l]);
    }
    /* lanes are independent: each merges into its own rows */
#pragma omp parallel for schedule(dynamic, 256) num_threads(m->threads)
    for (int32_t l = 0; l < Lc; ++l) {
        prop_t *buf = lanebuf + ls2[l];
        int32_t nb = 0;
        int32_t ip = m->ls[l], jp = js[l], jend = js[l + 1];
        for (;;) {
            while (ip < m->ls[l + 1] && pr[ip].status != ST_STAY) ++ip;
            int has_s = ip < m->ls[l + 1];
            int has_j = jp < jend;
            if (!has_s && !has_j) break;
            if (has_s && (!has_j || key_less(m, &pr[ip], &jn[jp])))
                buf[nb++] = pr[ip++];
            else
                buf[nb++] = jn[jp++];
        }
        for (int32_t f = nb - 2; f >= 0; --f) {
            float lim = buf[f + 1].s - P->len;
            if (buf[f].s > lim) {
                buf[f].s = lim;
                buf[f].v = fmin32(buf[f].v, buf[f + 1].v);
                clamps[l]++;
            }
        }
        for (int32_t q = 0; q < nb; ++q) {
            int32_t w = ls2[l] + q;
            sl2[w] = l; vi2[w] = buf[q].veh; cur2[w] = buf[q].cur;
            s2[w] = buf[q].s; v2[w] = buf[q].v; a2[w] = buf[q].a;
        }
    }
    for (int32_t l = 0; l < Lc; ++l)
        m->cnt[(size_t)m->lane_scen[l] * ORC_N_COUNTERS + ORC_CLAMPS] += clamps[l];
    int32_t w = ls2[Lc];
    free(js); free(clamps);
    free(m->ls); free(m->sl); free(m->vi); free(m->cur); free(m->s); free(m->v); free(m->a);
    m->ls = ls2; m->sl = sl2; m->vi = vi2; m->cur = cur2; m->s = s2; m->v = v2; m->a = a2;
    m->n_act = w;
    m->t = t + 1;

    /* --- observables on the new state --- */
    for (int32_t q = 0; q < w; ++q) {
        size_t sc = (size_t)m->lane_scen[m->sl[q]];
        m->cnt[sc * ORC_N_COUNTERS + ORC_VEH_STEPS]++;
        m->sumv[sc] += speed_fx(m->v[q]);
    }
    free(lanebuf); free(jn); free(pr); free(ins);
}

int orc_step(orc_sim *m, int32_t n)
{
    for (int32_t k = 0; k < n; ++k)
        one_step(m);
    return 0;
}

void orc_set_threads(orc_sim *m, int32_t n) { m->threads = n > 0 ? n : 1; }

int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int32_t orc_n_active(const orc_sim *m) { return m->n_act; }
int64_t orc_time(const orc_sim *m) { return m->t; }

int32_t orc_pending(const orc_sim *m)
{
    int32_t p = 0;
    for (int32_t l = 0; l < m->n_lanes; ++l) p += m->q_end[l] - m->q_head[l];
    return p;
}

void orc_read(const orc_sim *m, uint32_t *id, int32_t *lane, float *s, float *v, float *a,
              int32_t *cursor)
{
    for (int32_t q = 0; q < m->n_act; ++q) {
        if (id) id[q] = m->vid[m->vi[q]];
        if (lane) lane[q] = m->sl[q];
        if (s) s[q] = m->s[q];
        if (v) v[q] = m->v[q];
        if (a) a[q] = m->a[q];
        if (cursor) cursor[q] = m->cur[q];
    }
}

int orc_set_signal_phase(orc_sim *m, int32_t node, int32_t phase)
{
    if (node < 0 || node >= m->n_nodes || m->node_cycle[node] <= 0)
        return -1;
    m->node_manual[node] = phase < 0 ? -1 : phase;
    return 0;
}

void orc_set_lane_vlim(orc_sim *m, int32_t lane, float vlim)
{
    m->lane_vlim[lane] = vlim;
}

int orc_set_lane_turns(orc_sim *m, int32_t n, const int32_t *lane, const int32_t *road,
                       const int32_t *allowed)
{
    if (!m->succ_off)
        return -1;
    int32_t *at = malloc(sizeof(int32_t) * (n > 0 ? (size_t)n : 1));
    for (int32_t q = 0; q < n; ++q) {
        at[q] = -1;
        if (lane[q] < 0 || lane[q] >= m->n_lanes) {
            free(at);
            return -1;
        }
        for (int32_t e = m->succ_off[lane[q]]; e < m->succ_off[lane[q] + 1]; ++e)
            if (m->lane_road[m->succ[e]] == road[q])
                at[q] = e;
        if (at[q] < 0) {
            free(at);
            return -1;
        }
    }
    for (int32_t q = 0; q < n; ++q)
        m->succ_en[at[q]] = allowed[q] ? 1 : 0;
    free(at);
    return 0;
}

int orc_set_lane_closed(orc_sim *m, int32_t n, const int32_t *lane, const int32_t *closed)
{
    for (int32_t q = 0; q < n; ++q)
        if (lane[q] < 0 || lane[q] >= m->n_lanes)
            return -1;
    uint8_t *next = malloc((size_t)m->n_lanes + 1);
    memcpy(next, m->lane_closed, (size_t)m->n_lanes);
    for (int32_t q = 0; q < n; ++q)
        next[lane[q]] = closed[q] ? 1 : 0;
    for (int32_t q = 0; q < n; ++q) {
        const int32_t r = m->lane_road[lane[q]], l0 = m->road_lane0[r];
        int32_t open = 0;
        for (int32_t k = 0; k < m->road_nlanes[r]; ++k)
            open += !next[l0 + k];
        if (open == 0) {             /* a road keeps an open lane */
            free(next);
            return -1;
        }
    }
    memcpy(m->lane_closed, next, (size_t)m->n_lanes);
    free(next);
    return 0;
}

void orc_road_stats(const orc_sim *m, int32_t *count, float *mean_v)
{
    double *sum = calloc((size_t)m->n_roads + 1, sizeof(double));
    for (int32_t r = 0; r < m->n_roads; ++r)
        count[r] = 0;
    for (int32_t q = 0; q < m->n_act; ++q) {
        const int32_t r = m->lane_road[m->sl[q]];
        count[r] += 1;
        sum[r] += (double)m->v[q];
    }
    for (int32_t r = 0; r < m->n_roads; ++r)
        mean_v[r] = count[r] > 0 ? (float)(sum[r] / (double)count[r]) : 0.0f;
    free(sum);
}

int orc_positions(const orc_sim *m, double *x, double *y, double *heading)
{
    if (!m->node_x || !m->node_y)
        return -1;
    for (int32_t q = 0; q < m->n_act; ++q) {
        const int32_t l = m->sl[q], r = m->lane_road[l];
        const double ax = m->node_x[m->road_from[r]], ay = m->node_y[m->road_from[r]];
        const double bx = m->node_x[m->road_to[r]], by = m->node_y[m->road_to[r]];
        const double dx = bx - ax, dy = by - ay;
        const double len = sqrt(dx * dx + dy * dy);
        const double ux = len > 0.0 ? dx / len : 1.0, uy = len > 0.0 ? dy / len : 0.0;
        const double f = (double)m->s[q] / (double)m->road_length[r];
        const double off = ((double)m->lane_k[l] + 0.5) * 3.5;   /* lane width 3.5 m */
        x[q] = ax + dx * f + uy * off;
        y[q] = ay + dy * f - ux * off;
        heading[q] = atan2(dy, dx);
    }
    return 0;
}

int32_t orc_read_debug(const orc_sim *m, uint32_t *id, uint32_t *leader, int32_t *flags,
                       float *margin, uint32_t *t_leader, uint32_t *t_follower)
{
    for (int32_t q = 0; q < m->dbg_n; ++q) {
        if (id) id[q] = m->d_id[q];
        if (leader) leader[q] = m->d_leader[q];
        if (flags) flags[q] = m->d_flags[q];
        if (margin) margin[q] = m->d_margin[q];
        if (t_leader) t_leader[q] = m->d_tl[q];
        if (t_follower) t_follower[q] = m->d_tf[q];
    }
    return m->dbg_n;
}

int32_t orc_read_mlp_inputs(const orc_sim *m, float *feat, int8_t *use)
{
    if (m->mode != 1) return 0;
    if (feat) memcpy(feat, m->d_feat, sizeof(float) * 8 * (size_t)m->dbg_n);
    if (use) memcpy(use, m->d_use, (size_t)m->dbg_n);
    return m->dbg_n;
}

void orc_mlp_sq(const orc_sim *m, double *sum_sq)
{
    memcpy(sum_sq, m->mlp_sq, sizeof(double) * (size_t)m->n_scen);
}

static int cmp_u32_idx(const void *x, const void *y)
{
    const uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return a < b ? -1 : (a > b);
}

/* Trips of all vehicles in ascending id order [reading of the paper's query
 * APIs for travel time and distance, Sec. III-C-4]: status 0 while waiting
 * to depart, 1 on the network, 2 arrived; travel time in steps (arrival step
 * minus departure step once arrived, the current step index minus the
 * departure step on the network, 0 while waiting); distance in metres along
 * the route from where the vehicle entered the simulation (the whole route
 * once arrived; the roads before its current one plus its position while on
 * the network; 0 while waiting), in FP64 with road lengths summed in route
 * order. */
void orc_read_trips(const orc_sim *m, uint32_t *id, int32_t *status, int32_t *travel,
                    double *dist)
{
    const int32_t N = m->n_veh;
    uint64_t *ord = malloc(sizeof(uint64_t) * (N ? N : 1));
    int32_t *row = malloc(sizeof(int32_t) * (N ? N : 1));
    for (int32_t i = 0; i < N; ++i) {
        ord[i] = ((uint64_t)m->vid[i] << 32) | (uint32_t)i;
        row[i] = -1;
    }
    qsort(ord, N, sizeof(uint64_t), cmp_u32_idx);
    for (int32_t q = 0; q < m->n_act; ++q)
        row[m->vi[q]] = q;
    for (int32_t k = 0; k < N; ++k) {
        const int32_t i = (int32_t)(ord[k] & 0xFFFFFFFFu);
        int32_t st = 0, tt = 0;
        double d = 0.0;
        if (m->arr[i] >= 0) {
            st = 2;
            tt = (int32_t)(m->arr[i] - m->depart[i]);
            d = route_dist(m, i, m->route_len[i]) - m->dist0[i];
        } else if (row[i] >= 0) {
            const int32_t q = row[i];
            st = 1;
            tt = (int32_t)(m->t - m->depart[i]);
            d = (route_dist(m, i, m->cur[q]) + (double)m->s[q]) - m->dist0[i];
        }
        if (id) id[k] = m->vid[i];
        if (status) status[k] = st;
        if (travel) travel[k] = tt;
        if (dist) dist[k] = d;
    }
    free(ord);
    free(row);
}

void orc_counters(const orc_sim *m, int64_t *cnt, double *sum_v)
{
    memcpy(cnt, m->cnt, sizeof(int64_t) * (size_t)m->n_scen * ORC_N_COUNTERS);
    for (int32_t q = 0; q < m->n_scen; ++q)
        sum_v[q] = (double)m->sumv[q] / 1048576.0;
}

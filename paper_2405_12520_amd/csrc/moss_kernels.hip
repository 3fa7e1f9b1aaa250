// Kernels of one simulation step on gfx950.
//
// A step is the paper's two-phase iteration (Sec. III-A):
//   update  - k_update: every vehicle reads only the state S the step
//             started from (the read-only copy) and writes a proposal (new
//             position, speed, lane, route index) to its own row of Pr;
//             workgroups after the update's own insert departures;
//   prepare - k_scan_*, k_jscatter, k_merge: the proposals are re-ordered per
//             lane into the next state S (the spatial index of the next step).
// No kernel writes what another thread of the same kernel reads, so the
// result does not depend on thread scheduling; atomics only count and
// allocate slots, and every order they create is re-sorted by (position, id).
//
// Arithmetic is FP32 in the source order, compiled without contraction, so
// that decisions (leaders, lane changes, lanes) reproduce bit for bit.
#include "moss_internal.h"
#include "moss_mlp.h"

namespace moss {

// Element idx of a device array, addressed as the array's base plus a 32-bit
// byte offset: the access then uses the scalar base register with one 32-bit
// vector offset instead of 64-bit address arithmetic per array.  Every array
// of the workspace is below 4 GiB (checked at creation).
template <class T>
__device__ __forceinline__ T &at(T *base, uint32_t idx)
{
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + idx * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ const T &at(const T *base, uint32_t idx)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                        idx * (uint32_t)sizeof(T));
}

__device__ __forceinline__ float fmin32(float x, float y) { return x < y ? x : y; }
__device__ __forceinline__ float fmax32(float x, float y) { return x > y ? x : y; }

// IDM acceleration (Treiber, Hennecke, Helbing 2000), exponent 4:
//   a_max (1 - (v/v0)^4 - (s*/gap)^2),  s* = s0 + max(0, v T + v dv / (2 sqrt(a b))),
// the last term as v dv times the FP32 reciprocal of 2 sqrt(a b) formed in
// double on the host (no division per evaluation).
// idm_free gives the free-road factor 1 - (v/v0)^4, idm_lead the acceleration
// behind a leader from that factor (a non-positive gap returns the braking
// limit); without a leader the acceleration is a_max times the factor.  The
// split lets one factor serve every evaluation with the same (v, v0) -- the
// same operations on the same operands, so the same bits.
__device__ __forceinline__ float idm_free(float v, float v0e)
{
    float r = v / v0e;
    float r2 = r * r;
    float r4 = r2 * r2;
    return 1.0f - r4;
}

__device__ __forceinline__ float idm_lead(const Params &P, float free_term, float v, float vl,
                                          float gap)
{
    if (gap <= 0.0f)
        return -P.b_max;
    float dv = v - vl;
    float t1 = v * P.T;
    float t2 = (v * dv) * P.inv_tsab;
    float tt = t1 + t2;
    float ss = P.s0 + (tt > 0.0f ? tt : 0.0f);
    float q = ss / gap;
    return P.a_max * (free_term - q * q);
}

__device__ __forceinline__ float idm_any(const Params &P, float free_term, bool has, float v,
                                         float vl, float gap)
{
    return has ? idm_lead(P, free_term, v, vl, gap) : P.a_max * free_term;
}

// First output word of Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ uint32_t philox_x0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = c0 * 0xD2511F53u, hi0 = __umulhi(c0, 0xD2511F53u);
        uint32_t lo1 = c2 * 0xCD9E8D57u, hi1 = __umulhi(c2, 0xCD9E8D57u);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c0;
}

// DPP lane moves (row_shr:n reads lane - n of the same row of 16,
// row_bcast:15 / :31 read lane 15 / 31 of the row before), so that the wave
// scans below stay in the vector ALU instead of going through LDS.  Lanes
// that the move does not write (no source lane, or a row outside ROWS) get
// `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_move(uint32_t old, uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, CTRL, ROWS, 0xF, false);
}
constexpr int kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr4 = 0x114, kDppShr8 = 0x118;
constexpr int kDppBcast15 = 0x142, kDppBcast31 = 0x143;

// One step of the segmented prefix maximum: take the (key, row) the move
// reads if it is larger and its lane lies in this lane's segment.
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_max_step(uint64_t &v, uint32_t &vi, bool in_seg)
{
    const uint32_t lo = dpp_move<CTRL, ROWS>((uint32_t)v, (uint32_t)v);
    const uint32_t hi = dpp_move<CTRL, ROWS>((uint32_t)(v >> 32), (uint32_t)(v >> 32));
    const uint32_t oi = dpp_move<CTRL, ROWS>(vi, vi);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    if (in_seg && o > v) {
        v = o;
        vi = oi;
    }
}

// Sum over the wave, complete in lane 63 (inclusive scan by row shifts, then
// row broadcasts).
__device__ __forceinline__ double wave_sum_f64_l63(double x)
{
    auto step = [&](auto mv) {
        const uint64_t b = (uint64_t)__double_as_longlong(x);
        const uint32_t lo = mv((uint32_t)b), hi = mv((uint32_t)(b >> 32));
        x += __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
    };
    step([](uint32_t u) { return dpp_move<kDppShr1, 0xF>(0u, u); });
    step([](uint32_t u) { return dpp_move<kDppShr2, 0xF>(0u, u); });
    step([](uint32_t u) { return dpp_move<kDppShr4, 0xF>(0u, u); });
    step([](uint32_t u) { return dpp_move<kDppShr8, 0xF>(0u, u); });
    step([](uint32_t u) { return dpp_move<kDppBcast15, 0xA>(0u, u); });
    step([](uint32_t u) { return dpp_move<kDppBcast31, 0xC>(0u, u); });
    return x;
}

// The same for 64-bit integers.
__device__ __forceinline__ uint64_t wave_sum_u64_l63(uint64_t x)
{
    auto step = [&](auto mv) {
        const uint32_t lo = mv((uint32_t)x), hi = mv((uint32_t)(x >> 32));
        x += ((uint64_t)hi << 32) | lo;
    };
    step([](uint32_t u) { return dpp_move<kDppShr1, 0xF>(0u, u); });
    step([](uint32_t u) { return dpp_move<kDppShr2, 0xF>(0u, u); });
    step([](uint32_t u) { return dpp_move<kDppShr4, 0xF>(0u, u); });
    step([](uint32_t u) { return dpp_move<kDppShr8, 0xF>(0u, u); });
    step([](uint32_t u) { return dpp_move<kDppBcast15, 0xA>(0u, u); });
    step([](uint32_t u) { return dpp_move<kDppBcast31, 0xC>(0u, u); });
    return x;
}

// A vehicle's term of the summed speed (Sec. III-A: speeds are the output
// the mean speed is formed from), in whole units of 2^-20 m/s: v * 2^20 is
// exact and the conversion truncates, 0 for v <= 0, 2^32 - 1 from 4096 m/s
// on.  Integer terms make the sum independent of the order of the atomics.
__device__ __forceinline__ uint64_t speed_fx(float v)
{
    const uint32_t q = v > 0.0f ? (uint32_t)(v * 1048576.0f) : 0u;
    return v >= 4096.0f ? 0xFFFFFFFFull : (uint64_t)q;
}

// Inclusive scan over the wave: lane i gets the sum of lanes 0..i (lane 63
// the wave's sum).
__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t x)
{
    x += dpp_move<kDppShr1, 0xF>(0u, x);
    x += dpp_move<kDppShr2, 0xF>(0u, x);
    x += dpp_move<kDppShr4, 0xF>(0u, x);
    x += dpp_move<kDppShr8, 0xF>(0u, x);
    x += dpp_move<kDppBcast15, 0xA>(0u, x);
    x += dpp_move<kDppBcast31, 0xC>(0u, x);
    return x;
}

struct Lead {
    bool has;
    float v, gap;
    uint32_t id;
};

// Lane taken on road rd (record rdi, next road of the route) by a vehicle
// leaving lane y (index kk in its road).  EXT handles control's lane
// closures and junction internal lanes: y's successor on rd when y has a
// successor list (the nearest open lane if it is closed), else lane index
// min(kk, n-1), or with closures the open lane nearest to it.  Without EXT
// the lane index is min(kk, n-1).
template <bool EXT>
__device__ __forceinline__ int next_lane(const Dev &d, int y, int kk, int rd, const RoadInfo &rdi)
{
    if constexpr (EXT) {
        if (d.junctions) {
            const int a = at(d.succ_off, y), b = at(d.succ_off, y + 1);
            for (int q = a; q < b; ++q) {
                const Succ sx = at(d.succ, q);
                if (sx.road == rd) {
                    const int k2 = sx.lane - rdi.lane0;
                    return rdi.lane0 + (d.closures ? pick_lane(k2, rdi.nlanes, rdi.closed) : k2);
                }
            }
        }
        return rdi.lane0 +
               (d.closures ? pick_lane(kk, rdi.nlanes, rdi.closed) : min(kk, rdi.nlanes - 1));
    } else {
        return rdi.lane0 + min(kk, rdi.nlanes - 1);
    }
}

// Whether lane y lets a vehicle continue onto road rd (junction internal
// lanes): y has no successor list, or a successor on rd.
__device__ __forceinline__ bool lane_permits(const Dev &d, int y, int rd)
{
    const int a = at(d.succ_off, y), b = at(d.succ_off, y + 1);
    bool ok = a == b;
    for (int q = a; q < b; ++q)
        ok = ok || at(d.succ, q).road == rd;
    return ok;
}

// Leader beyond the lane end: follow the route for at most h_look roads while
// the distance covered is within d_look; on each road take the lane
// next_lane gives and use its last vehicle (lane tail).  A vehicle never
// leads itself.  lf is the vehicle's (final) lane, li its record; rd0 is the
// record of the next road nxt (already loaded by the caller); with pre, tl0
// is the tail the first road gives (loaded by the caller too).
template <bool EXT>
__device__ Lead lookahead(const Dev &d, int lf, const LaneInfo &li, float s, uint32_t id,
                          uint32_t ptr, int32_t nxt, RoadInfo rd0, bool pre, Tail tl0)
{
    Lead r = {false, 0.0f, 0.0f, kNone};
    float dist = li.L - s;
    int kk = li.k;
    int y = lf;
    uint32_t p = ptr;
    int32_t nr = nxt;
    RoadInfo rd = rd0;
    for (int h = 0; h < d.P.h_look; ++h) {
        if (nr < 0)
            break;
        if (dist > d.P.d_look)
            break;
        if (h > 0)
            rd = at(d.roads, nr);
        y = next_lane<EXT>(d, y, kk, nr, rd);
        kk = y - rd.lane0;
        Tail tl;
        if (h == 0 && pre)
            tl = tl0;
        else
            tl = at(d.tails, y);
        if (tl.id != kNone) {
            if (tl.id != id) {
                r.has = true;
                r.v = tl.v;
                r.gap = (dist + tl.s) - d.P.len;
                r.id = tl.id;
            }
            return r;
        }
        dist = dist + rd.L;
        p += 1;
        nr = at(d.route, p + 1);
    }
    return r;
}

// This wave's copy of the counters and sums.
__device__ __forceinline__ int wave_stripe()
{
    return (int)(((blockIdx.x << 2) + (threadIdx.x >> 6)) & (kStripes - 1));
}
__device__ __forceinline__ unsigned long long *cnt_at(const Dev &d, int scen, int c)
{
    return d.cnt + (size_t)wave_stripe() * d.cnt_stride + (size_t)scen * C_N + c;
}
__device__ __forceinline__ double *sv_at(const Dev &d, double *base, int scen)
{
    return base + (size_t)wave_stripe() * d.sv_stride + scen;
}
__device__ __forceinline__ unsigned long long *sumv_at(const Dev &d, int scen)
{
    return d.sumv + (size_t)wave_stripe() * d.sv_stride + scen;
}

// Adds the wave's count of pred to counter c (one atomic per wave when the
// wave's vehicles are all of one scenario).
// For each scenario among the wave's lanes with pred, adds their number to
// counter c of that scenario: one atomic per scenario present, where
// per-lane atomics would meet on one address 64 times.  Wave-uniform call.
__device__ __forceinline__ void wave_count_scen(const Dev &d, int c, bool pred, int scen)
{
    unsigned long long todo = __ballot(pred);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int s0 = __builtin_amdgcn_readlane(scen, leader);
        const unsigned long long mm = __ballot(pred && scen == s0);
        if (__lane_id() == leader)
            atomicAdd(cnt_at(d, s0, c), (unsigned long long)__popcll(mm));
        todo &= ~mm;
    }
}

// The same for the summed speed of each scenario (one wave sum per scenario
// present).  Wave-uniform call.
__device__ __forceinline__ void wave_sumv_scen(const Dev &d, bool pred, int scen, uint64_t x)
{
    unsigned long long todo = __ballot(pred);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int s0 = __builtin_amdgcn_readlane(scen, leader);
        const bool mine = pred && scen == s0;
        const unsigned long long mm = __ballot(mine);
        const uint64_t sum = wave_sum_u64_l63(mine ? x : 0ull);
        if (__lane_id() == 63)
            atomicAdd(sumv_at(d, s0), (unsigned long long)sum);
        todo &= ~mm;
    }
}

// Wave-aggregated counter increment for waves whose vehicles are all in one
// scenario (the common case); other waves use one atomic per lane.
__device__ __forceinline__ void wave_count(const Dev &d, int c, bool pred, int scen, int scen0,
                                           bool uniform)
{
    if (uniform) {
        const unsigned long long m = __ballot(pred);
        if (m && __lane_id() == __ffsll((long long)m) - 1)
            atomicAdd(cnt_at(d, scen0, c), (unsigned long long)__popcll(m));
    } else if (pred) {
        atomicAdd(cnt_at(d, scen, c), 1ull);
    }
}

// ----------------------------------------------------------------- insert --

// Head of each origin-lane queue enters when due, if the lane is empty or the
// gap behind its last vehicle is at least s0 + v T for the entry speed
// v = min(v0, limit, speed of that vehicle); it joins the lane at s = 0 at
// the end of the step.  Queue lane q; run by whole workgroups of the update
// launch (insertion reads only the start-of-step state, writes proposal rows
// from n_cur on and its own joiner list, and only adds to the lane counts,
// so it runs beside the update).
__device__ __forceinline__ void insert_lane(const Dev &d, const int q)
{
    const Params &P = d.P;
    bool ins = false, fail = false;
    int l = 0, h = 0, scen = 0;
    float vins = 0.0f;
    // the head's departure step is kept per queue, so that lanes with nothing
    // due leave after one coalesced load
    if (q < d.n_qlanes && (int64_t)at(d.q_hdep, q) <= *d.t) {
        l = at(d.qlanes, q);
        h = at(d.q_head, l);
        {
            const LaneInfo li = at(d.lanes, l);
            const float v0e = fmin32(at(d.q_v0, h), li.vlim);
            const int lo = at(d.ls_old, l), hi = at(d.ls_old, l + 1);
            bool ok;
            if (li.lflags & kLaneClosed) {
                ok = false;     // a closed lane holds its departure queue
            } else if (lo == hi) {
                ok = true;
                vins = v0e;
            } else {
                vins = fmin32(v0e, at(d.S.v, lo));
                ok = (at(d.S.s, lo) - P.len) >= (P.s0 + vins * P.T);
            }
            scen = li.scen;
            ins = ok;
            fail = !ok;
        }
    }
    // Queue lane q owns proposal row n_cur + q and entry q of the insertion
    // list (a lane inserts at most one vehicle per step), so no slot is
    // allocated (a shared slot counter, taken once per wave, serialised on
    // one address across the grid); entries of lanes that insert nothing
    // are marked kNone.
    if (q < d.n_qlanes) {
        const uint32_t slot = (uint32_t)(*d.n_cur) + (uint32_t)q;
        at(d.jins_list, q) = slot;
        at(d.jins_lane, q) = ins ? (uint32_t)l : kNone;
        if (ins) {
            at(d.Pr.s, slot) = 0.0f;
            at(d.Pr.v, slot) = vins;
            at(d.Pr.a, slot) = 0.0f;
            at(d.Pr.id, slot) = at(d.q_id, h);
            at(d.Pr.lane, slot) = (uint32_t)l | kJoinBit;
            at(d.Pr.ptr, slot) = at(d.q_ptr, h);
            at(d.Pr.next, slot) = at(d.q_next, h);
            at(d.Pr.v0, slot) = at(d.q_v0, h);
            atomicAdd(&at(d.jcount, l), 1);
            at(d.q_head, l) = h + 1;
            at(d.q_hdep, q) = h + 1 < at(d.q_end, l) ? at(d.q_dep, h + 1) : INT32_MAX;
        }
    }
    if (q == 0)
        *d.n_ins = (uint32_t)d.n_qlanes;
    wave_count_scen(d, C_INSERT_FAIL, fail, scen);
    wave_count_scen(d, C_INSERTED, ins, scen);
}

// ----------------------------------------------------------------- update --

constexpr int kUT = kUpdateRows;       // rows per update block
constexpr int kUH = 128;               // rows staged before and after them
constexpr int kUW = kUT + 2 * kUH;

__device__ __forceinline__ int lds_lower_bound_f32(const float *a, int lo, int hi, float x)
{
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] >= x)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Tile taken by workgroup blockIdx.x when ntiles tiles have work.
// Workgroups are dealt round-robin to the 8 XCDs; with remap on (and a grid
// that is a multiple of 8) the first g = min(grid, ntiles rounded up to 8)
// workgroups split those tiles into 8 contiguous ranges, one per XCD, so that
// neighbouring tiles' shared rows meet in the same L2.  Workgroups from g on
// keep their own index, which is past the last tile (g >= ntiles there).  A
// bijection of [0, grid) either way; with a persistent loop (grid below
// ntiles) each round adds grid.
__device__ __forceinline__ int xcd_tile(int remap, int ntiles, int grid)
{
    const int b = blockIdx.x;
    if (!remap || (grid & 7))
        return b;
    const int g = min(grid, ((ntiles + 7) >> 3) << 3);
    if (b >= g)
        return b;
    return (b & 7) * (g >> 3) + (b >> 3);
}

// Update phase for kUT rows per block.  The block stages the rows around its
// own (s, v, v0, id, lane of rows [base-kUH, base+kUT+kUH)) in LDS; in-lane
// neighbours are the adjacent rows and the target lane of a lane change is
// found by binary search in that window, falling back to global memory when
// the lane does not fit in it.  Records needed later (the side lane, the next
// road of lane heads) are loaded up front so that their latencies overlap.
// Joiners are listed in the tile's own region of jlist, so no atomic result
// is waited for.  MODE 1 evaluates the learned closure for the wave's 64
// vehicles on the matrix cores between the acceleration and the integration.
template <int MODE, bool AUX, bool EXT, bool INS>
__global__ void __launch_bounds__(kUT, 4) k_update(Dev d)
{
    __shared__ float w_s[kUW], w_v[kUW], w_v0[kUW];
    __shared__ uint32_t w_id[kUW], w_ln[kUW];
    __shared__ uint32_t s_jn;

    // the workgroups after the update's own insert departures (INS: the
    // variant for networks with departure queues; without them the code is
    // left out, which keeps scalar registers free)
    const int gu = INS ? (int)gridDim.x - (d.n_qlanes + kUT - 1) / kUT : (int)gridDim.x;
    if constexpr (INS) {
        if ((int)blockIdx.x >= gu) {
            insert_lane(d, ((int)blockIdx.x - gu) * kUT + (int)threadIdx.x);
            return;
        }
    }
    const int n = *d.n_cur;
    const int64_t t = *d.t;
    // lane closures by control and junction internal lanes change the lane
    // taken on the next road, the lane-change rule and the stop line; the
    // variant without them (EXT false) is launched when neither is present
    const bool junctions = EXT && d.junctions;
    const Params &P = d.P;
    const uint32_t tt = (uint32_t)t;
    const int tid = threadIdx.x;
    const int side = ((t & 1) == 0) ? -1 : 1;     // MOBIL looks at lane k-1 on even steps
    // AUX instantiations carry the debug and trace records (P.debug, P.trace);
    // the others never touch those buffers
    const bool dbg = AUX && P.debug, trc = AUX && P.trace;
    const bool want_feat = MODE == 1 || trc;

    MlpLds *mw = nullptr;
    uint16_t *mz = nullptr;
    if constexpr (MODE == 1) {
        __shared__ MlpLds s_mlp;
        __shared__ __attribute__((aligned(16))) uint16_t s_z[(kUT / 64) * kMlpStage];
        mlp_copy(s_mlp, static_cast<const MlpLds *>(d.mlp_pack));
        mw = &s_mlp;
        mz = s_z + (tid >> 6) * kMlpStage;
    }

    for (int base = xcd_tile(d.xcd_remap, (n + kUT - 1) / kUT, gu) * kUT; base < n;
         base += gu * kUT) {
        const int ws = max(base - kUH, 0), we = min(base + kUT + kUH, n);
        const int i = base + tid;
        const bool act = i < n;
        uint32_t ptr = 0;
        int32_t nxt = -1;
        float a_prev = 0.0f;
        if (act) {
            ptr = at(d.S.ptr, i);
            nxt = at(d.S.next, i);
            if (want_feat)
                a_prev = at(d.S.a, i);
        }
        __syncthreads();
        if (tid == 0)
            s_jn = 0;
        // the window (at most 2 kUT rows): every load is issued before the
        // first LDS store waits for one; indices are clamped into the window
        static_assert(2 * kUH <= kUT, "window rows fit two per thread");
        {
            const int r0 = ws + tid, r1 = ws + tid + kUT;
            const int q0 = min(r0, we - 1), q1 = min(r1, we - 1);
            const float s0 = at(d.S.s, q0), v0a = at(d.S.v, q0), v00 = at(d.S.v0, q0);
            const uint32_t id0 = at(d.S.id, q0), ln0 = at(d.S.lane, q0);
            const float s1 = at(d.S.s, q1), v1a = at(d.S.v, q1), v01 = at(d.S.v0, q1);
            const uint32_t id1 = at(d.S.id, q1), ln1 = at(d.S.lane, q1);
            if (r0 < we) {
                w_s[r0 - ws] = s0;
                w_v[r0 - ws] = v0a;
                w_v0[r0 - ws] = v00;
                w_id[r0 - ws] = id0;
                w_ln[r0 - ws] = ln0;
            }
            if (r1 < we) {
                w_s[r1 - ws] = s1;
                w_v[r1 - ws] = v1a;
                w_v0[r1 - ws] = v01;
                w_id[r1 - ws] = id1;
                w_ln[r1 - ws] = ln1;
            }
        }
        __syncthreads();

        const int x_i = i - ws;
        const uint32_t l = act ? w_ln[x_i] : 0u;
        const bool hasLc = act && (i + 1 < n) && w_ln[x_i + 1] == l;
        // independent loads of the second round, all issued before any is
        // waited for: indices are made valid (lane l, road 0) instead of
        // skipping the load, and the values are selected afterwards
        const int ls_side = (int)l + side;
        const bool side_ok = act && ls_side >= 0 && ls_side < d.n_lanes;
        const int ls_c = side_ok ? ls_side : (int)l;
        const bool head_next = act && !hasLc && nxt >= 0;
        const LaneInfo li = at(d.lanes, l);
        const uint8_t red_raw = at(d.lane_red, l);
        const float vlim_c_side = at(d.lanes, ls_c).vlim;
        const uint8_t side_flags = EXT ? at(d.lane_red, ls_c) : (uint8_t)0;
        const int r0_c = at(d.ls_old, ls_c), r1_c = at(d.ls_old, ls_c + 1);
        const RoadInfo rd_c = at(d.roads, (act && nxt >= 0) ? nxt : 0);
        const bool red_now = act && (red_raw & kRedBit) != 0;
        // a lane closed by control is never a lane-change target
        const bool side_open = (side_flags & kClosedBit) == 0;
        const float vlim_side = side_ok ? vlim_c_side : 0.0f;
        // rows of the side lane (the MOBIL target when it is on the same road)
        const int side_r0 = side_ok ? r0_c : 0;
        const int side_r1 = side_ok ? r1_c : 0;
        RoadInfo rd_next = {0, 1, 0.0f, 0};
        bool rd_ok = false;       // rd_next holds roads[nxt]
        if (act && nxt >= 0) {
            rd_next = rd_c;
            rd_ok = true;
        }
        // a lane head's first lookahead tail, in its own lane and in the side
        // lane, loaded now so that the load overlaps the acceleration (entry
        // 0 for the other vehicles)
        Tail tl_own, tl_side;
        {
            int ln_own = 0, ln_side = 0;
            if (head_next) {
                ln_own = next_lane<EXT>(d, (int)l, (int)li.k, nxt, rd_c);
                ln_side = next_lane<EXT>(d, side_ok ? ls_side : (int)l,
                                         max((int)li.k + side, 0), nxt, rd_c);
            }
            tl_own = at(d.tails, ln_own);
            tl_side = at(d.tails, ln_side);
        }
        // a vehicle that may pass its lane's end this step: the route entry
        // after its next road, loaded now so that the transfer does not wait
        // for it (s + v dt + a_max dt^2 / 2 bounds the new position, the
        // metre covers rounding; the others load entry 0)
        bool pre = false;
        int32_t nr_pre = -1;
        if constexpr (MODE == 0) {
            if (act && nxt >= 0)
                pre = w_s[x_i] + w_v[x_i] * P.dt + 0.5f * P.a_max * (P.dt * P.dt) + 1.0f >= li.L;
            nr_pre = at(d.route, pre ? ptr + 2u : 0u);
        }
        const int scen0 = __builtin_amdgcn_readlane(li.scen, 0);
        const bool uni_scen = __all(!act || li.scen == scen0);

        // values carried from the acceleration to the integration
        bool arrived = false, change = false, joins = false;
        int x = 0, lf = (int)l;
        uint32_t p = ptr;
        float sp = 0.0f, vn = 0.0f, a = 0.0f, a_idm = 0.0f;
        int32_t nr = nxt;
        uint32_t id = 0, lead_id = kNone, tl_id = kNone, tf_id = kNone;
        float v0 = 0.0f, s = 0.0f, v = 0.0f, margin = 0.0f;
        int32_t flags = 0;
        LaneInfo lif = li;
        float feat[kMlpIn];
#pragma unroll
        for (int q = 0; q < kMlpIn; ++q)
            feat[q] = 0.0f;

        if (act) {
            s = w_s[x_i];
            v = w_v[x_i];
            id = w_id[x_i];
            v0 = w_v0[x_i];
            const float L = li.L;

            // red light at the stop line, applied if the vehicle can still stop
            bool red = false;
            if (nxt >= 0 && red_now) {
                float stop_dist = (v * v) * P.inv_2bmax;
                if (L - s >= stop_dist)
                    red = true;
            }

            // in-lane neighbours are the adjacent rows
            const bool hasO = (i >= 1) && w_ln[x_i - 1] == l;
            float sLc = 0.0f, vLc = 0.0f;
            if (hasLc) {
                sLc = w_s[x_i + 1];
                vLc = w_v[x_i + 1];
            }
            const float v0e_c = fmin32(v0, li.vlim);
            const float free_c = idm_free(v, v0e_c);
            float acc_c = 0.0f, acc_t = 0.0f, free_t = 0.0f;   // valid when MOBIL ran
            bool mobil = false;

            // randomised MOBIL on one side per step (even: k-1, odd: k+1)
            int lt = -1;
            bool hasLt = false, hasN = false;
            float sLt = 0.0f, vLt = 0.0f;
            uint32_t idLt = kNone;
            // no lane changes inside a junction
            if (s >= 0.0f && (!EXT || !(red_raw & kInternalBit))) {
                const int kt = (int)li.k + side;
                if (kt >= 0 && kt < (int)li.nlanes && side_open) {
                    mobil = true;
                    lt = ls_side;
                    float sN = 0.0f, vN = 0.0f, v0N = 0.0f;
                    uint32_t idN = kNone;
                    // the target lane's rows from the lane starts; searched in
                    // the window when they all lie in it
                    const int g0 = side_r0, g1 = side_r1;
                    const int a0 = g0 - ws, a1 = g1 - ws;
                    if (g0 >= ws && g1 <= we) {
                        const int j = lds_lower_bound_f32(w_s, a0, a1, s);
                        if (j < a1) {
                            hasLt = true; sLt = w_s[j]; vLt = w_v[j]; idLt = w_id[j];
                        }
                        if (j - 1 >= a0) {
                            hasN = true; sN = w_s[j - 1]; vN = w_v[j - 1]; v0N = w_v0[j - 1];
                            idN = w_id[j - 1];
                        }
                    } else {
                        int lo2 = g0, hi2 = g1;
                        while (lo2 < hi2) {
                            int mid = (lo2 + hi2) >> 1;
                            if (at(d.S.s, mid) >= s)
                                hi2 = mid;
                            else
                                lo2 = mid + 1;
                        }
                        if (lo2 < g1) {
                            hasLt = true; sLt = at(d.S.s, lo2); vLt = at(d.S.v, lo2); idLt = at(d.S.id, lo2);
                        }
                        if (lo2 - 1 >= g0) {
                            hasN = true; sN = at(d.S.s, lo2 - 1); vN = at(d.S.v, lo2 - 1);
                            v0N = at(d.S.v0, lo2 - 1); idN = at(d.S.id, lo2 - 1);
                        }
                    }
                    const float vlim_c = li.vlim, vlim_t = vlim_side;
                    const float v0e_t = fmin32(v0, vlim_t);
                    free_t = (v0e_t == v0e_c) ? free_c : idm_free(v, v0e_t);
                    acc_c = idm_any(P, free_c, hasLc, v, vLc, (sLc - P.len) - s);
                    acc_t = idm_any(P, free_t, hasLt, v, vLt, (sLt - P.len) - s);
                    float d_o = 0.0f, d_n = 0.0f;
                    bool safe = true;
                    if (hasO) {
                        const float vo = w_v[x_i - 1], so = w_s[x_i - 1];
                        const float free_o = idm_free(vo, fmin32(w_v0[x_i - 1], vlim_c));
                        float a_o = idm_lead(P, free_o, vo, v, (s - P.len) - so);
                        float at_o = idm_any(P, free_o, hasLc, vo, vLc, (sLc - P.len) - so);
                        d_o = at_o - a_o;
                    }
                    if (hasN) {
                        const float free_n = idm_free(vN, fmin32(v0N, vlim_t));
                        float a_n = idm_any(P, free_n, hasLt, vN, vLt, (sLt - P.len) - sN);
                        float at_n = idm_lead(P, free_n, vN, v, (s - P.len) - sN);
                        d_n = at_n - a_n;
                        float gap_b = (s - P.len) - sN;
                        if (!(gap_b > 0.0f)) safe = false;
                        if (!(at_n >= -P.b_safe)) safe = false;
                    }
                    if (hasLt) {
                        float gap_f = (sLt - P.len) - s;
                        if (!(gap_f > 0.0f)) safe = false;
                    }
                    float inc = (acc_t - acc_c) + P.pol * (d_n + d_o);
                    // lanes that continue the route: a target lane that does,
                    // when the own lane does not, adds b_mand to the incentive;
                    // one that does not, when the own lane does, is never taken
                    bool allowed = true;
                    if (junctions && nxt >= 0) {
                        const bool pc = lane_permits(d, (int)l, nxt);
                        const bool pt = lane_permits(d, lt, nxt);
                        if (pt && !pc)
                            inc = inc + P.b_mand;
                        else if (pc && !pt)
                            allowed = false;
                    }
                    const bool cand = safe && allowed && inc > P.a_thr;
                    if (cand) {       // the random draw only matters for candidates
                        uint32_t x0 = philox_x0(tt, id, 0u, 0u, P.key0, P.key1);
                        float u = (float)(x0 >> 8) * (1.0f / 16777216.0f);
                        change = u < P.p_lc;
                    }
                    margin = inc - P.a_thr;
                    flags |= change ? 2 : 1;
                    tl_id = idLt;
                    tf_id = idN;
                }
            }

            // car-following in the final lane
            lf = change ? lt : (int)l;
            if (change) {
                lif.vlim = vlim_side;
                lif.k = (uint8_t)((int)li.k + side);
            }
            const float free_f = change ? free_t : free_c;
            const bool inlane = change ? hasLt : hasLc;
            if (junctions && nxt >= 0 && !lane_permits(d, lf, nxt))
                flags |= 32;        // final lane does not continue the route
            float acc;
            bool has_lead;
            float lead_v, lead_gap;
            if (inlane) {
                // same operands as MOBIL's own-lane / target-lane evaluation
                has_lead = true;
                lead_v = change ? vLt : vLc;
                lead_gap = ((change ? sLt : sLc) - P.len) - s;
                acc = mobil ? (change ? acc_t : acc_c) : idm_lead(P, free_f, v, vLc, lead_gap);
                lead_id = change ? idLt : w_id[x_i + 1];
            } else {
                if (!rd_ok && nxt >= 0) {
                    rd_next = at(d.roads, nxt);
                    rd_ok = true;
                }
                const Lead ld = lookahead<EXT>(d, lf, lif, s, id, ptr, nxt, rd_next, head_next,
                                               change ? tl_side : tl_own);
                // yield at a junction: the first vehicle of its lane stops at
                // the line when the connector lane it would take has busy
                // conflicts with priority (applied if it can still stop)
                if (junctions && nxt >= 0) {
                    const int cl = next_lane<EXT>(d, lf, (int)lif.k, nxt, rd_next);
                    if (at(d.busy, cl)) {
                        flags |= 64;
                        if (!red) {
                            float stop_dist = (v * v) * P.inv_2bmax;
                            if (L - s >= stop_dist)
                                red = true;
                        }
                    }
                }
                if (ld.has) flags |= 8;
                has_lead = ld.has;
                lead_v = ld.v;
                lead_gap = ld.gap;
                acc = idm_any(P, free_f, ld.has, v, ld.v, ld.gap);
                lead_id = ld.id;
            }
            if (red) {
                float acc_red = idm_lead(P, free_f, v, 0.0f, L - s);
                acc = fmin32(acc, acc_red);
                flags |= 4;
            }
            a = fmax32(-P.b_max, acc);
            a_idm = a;
            if (want_feat) {
                // inputs of the learned closure
                feat[0] = has_lead ? fmin32(lead_gap, P.d_look) : P.d_look;
                feat[1] = v;
                feat[2] = has_lead ? lead_v : v;
                feat[3] = fmin32(v0, lif.vlim);
                feat[4] = red ? fmin32(L - s, P.d_look) : P.d_look;
                feat[5] = a_prev;
                feat[6] = fmin32(L - s, P.d_look);
                feat[7] = lif.vlim;
            }
        }

        uint32_t ptr0 = ptr;     // route position at step start
        if constexpr (MODE == 1) {
            // records that do not depend on the network are written first,
            // so that little of the update's state is held across it
            if (act && trc) {
#pragma unroll
                for (int q = 0; q < kMlpIn; ++q)
                    at(d.tr_feat, (size_t)i * kMlpIn + q) = feat[q];
                at(d.tr_label, i) = a_idm;
            }
            if (act && dbg) {
                at(d.d_id, i) = id;
                at(d.d_leader, i) = lead_id;
                at(d.d_margin, i) = margin;
                at(d.d_tl, i) = tl_id;
                at(d.d_tf, i) = tf_id;
            }
            // learned closure for the whole wave; inside the envelope it
            // replaces the IDM acceleration, limited to [-b_max, a_max]
            const float *nm = mw->norm;
            bool inside = act;
            float z[kMlpIn];
#pragma unroll
            for (int q = 0; q < kMlpIn; ++q) {
                if (!(feat[q] >= nm[16 + q] && feat[q] <= nm[24 + q]))
                    inside = false;
                z[q] = act ? mlp_in(q, feat[q], nm) : 0.0f;
            }
            const float y = wave_mlp(*mw, mz, z);
            double e2 = 0.0;
            if (inside) {
                const float am = fmax32(-P.b_max, fmin32(y, P.a_max));
                const double e = (double)am - (double)a;
                e2 = e * e;
                a = am;
            }
            wave_count(d, C_MLP_EVAL, inside, li.scen, scen0, uni_scen);
            wave_count(d, C_MLP_FALLBACK, act && !inside, li.scen, scen0, uni_scen);
            if (uni_scen) {
                e2 = wave_sum_f64_l63(e2);
                if (__lane_id() == 63 && e2 != 0.0)
                    atomicAdd(sv_at(d, d.mlp_sq, scen0), e2);
            } else if (inside) {
                atomicAdd(sv_at(d, d.mlp_sq, li.scen), e2);
            }
            // the rest of the update re-reads its inputs: the window rows are
            // unchanged until the next tile, the rest comes from the tables
            if (act) {
                s = w_s[x_i];
                v = w_v[x_i];
                id = w_id[x_i];
                v0 = w_v0[x_i];
                ptr0 = at(d.S.ptr, i);
                p = ptr0;
                nr = at(d.S.next, i);
                rd_ok = false;
                const LaneInfo lr = at(d.lanes, l);
                lif.L = lr.L;
                lif.k = (uint8_t)((int)lr.k + (change ? side : 0));
            }
        }

        if (act) {
            // Newton's equations over one step, stopping at v = 0
            vn = v + a * P.dt;
            float dx;
            if (vn < 0.0f) {
                dx = -((v * v) / (2.0f * a));
                vn = 0.0f;
            } else {
                dx = v * P.dt + (0.5f * a) * (P.dt * P.dt);
            }
            sp = s + dx;

            // transfer along the route, arrival at the end of the last road
            x = lf;
            int kk = lif.k;
            float Lx = lif.L;
            bool first = true;
            while (sp >= Lx && nr >= 0) {
                sp = sp - Lx;
                p += 1;
                const RoadInfo rd = (first && rd_ok) ? rd_next : at(d.roads, nr);
                x = next_lane<EXT>(d, x, kk, nr, rd);
                kk = x - rd.lane0;
                Lx = rd.L;
                nr = (first && pre) ? nr_pre : at(d.route, p + 1);
                first = false;
            }
            arrived = sp >= Lx;
            joins = !arrived && !(x == (int)l && p == ptr0);
            if (!(isfinite(sp) && isfinite(vn)))
                atomicOr(d.err, 2u);
            if (arrived)
                flags |= 16;
            if (dbg) {
                at(d.d_flags, i) = flags;
                if constexpr (MODE == 0) {
                    at(d.d_id, i) = id;
                    at(d.d_leader, i) = lead_id;
                    at(d.d_margin, i) = margin;
                    at(d.d_tl, i) = tl_id;
                    at(d.d_tf, i) = tf_id;
                }
            }
            if (MODE == 0 && trc) {
#pragma unroll
                for (int q = 0; q < kMlpIn; ++q)
                    at(d.tr_feat, (size_t)i * kMlpIn + q) = feat[q];
                at(d.tr_label, i) = a_idm;
            }
        }

        // bookkeeping: joiners in the tile's region, per-lane leave/join
        // counts (no returned values awaited), counters
        const unsigned long long jm = __ballot(joins);
        uint32_t jbase = 0;
        if (jm) {
            const int leader = __ffsll((long long)jm) - 1;
            if (__lane_id() == leader)
                jbase = atomicAdd(&s_jn, (uint32_t)__popcll(jm));
            jbase = (uint32_t)__builtin_amdgcn_readlane((int)jbase, leader);
        }
        if (act) {
            if (arrived || joins)
                atomicAdd(&at(d.leave, l), 1);
            if (arrived) {
                // the route array stores the departure step after the -1 that
                // ends the route
                const int32_t dep = at(d.route, p + 2);
                at(d.route, p + 3) = (int32_t)(t + 1);      // arrival step
                atomicAdd(cnt_at(d, li.scen, C_TRIP_TIME),
                          (unsigned long long)((t + 1) - (int64_t)dep));
            } else if (joins) {
                const int lane_id = __lane_id();
                const unsigned long long below = lane_id ? (~0ull >> (64 - lane_id)) : 0ull;
                const uint32_t slot = (uint32_t)base + jbase + (uint32_t)__popcll(jm & below);
                at(d.jlist, slot) = (uint32_t)i;
                at(d.jlane, slot) = (uint32_t)x;
                atomicAdd(&at(d.jcount, x), 1);
            }
            // (id and v0 of the row are already in Pr: the step's id/v0 buffer)
            at(d.Pr.s, i) = sp;
            at(d.Pr.v, i) = vn;
            at(d.Pr.a, i) = a;
            at(d.Pr.lane, i) = l | ((arrived || joins) ? kJoinBit : 0u);
            at(d.Pr.ptr, i) = p;
            at(d.Pr.next, i) = nr;
        }
        wave_count(d, C_ARRIVED, arrived, li.scen, scen0, uni_scen);
        wave_count(d, C_LANE_CHANGES, change, li.scen, scen0, uni_scen);
        __syncthreads();
        if (tid == 0)
            at(d.jcnt, base / kUT) = (int32_t)s_jn;
    }
}

// --------------------------------------------------------- lane-count scan --

constexpr int kScanThreads = 256;
constexpr int kScanPer = 1;
constexpr int kScanLanes = kScanThreads * kScanPer;
static_assert(kScanLanes == kScanBlockLanes, "block sums are sized for kScanBlockLanes");

// Inclusive scan of two ints over the block: within each wave by DPP moves,
// then the totals of the waves before it are added (one LDS round).
__device__ __forceinline__ void block_scan2(int &x, int &y, int *sh)
{
    const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
    x = (int)wave_scan_u32((uint32_t)x);
    y = (int)wave_scan_u32((uint32_t)y);
    if (lane == 63) {
        sh[wv] = x;
        sh[kScanThreads / 64 + wv] = y;
    }
    __syncthreads();
    for (int k = 0; k < wv; ++k) {
        x += sh[k];
        y += sh[kScanThreads / 64 + k];
    }
}

// new lane size = old size - vehicles leaving + vehicles joining
__device__ __forceinline__ int new_count(const Dev &d, int l, int &j)
{
    j = at(d.jcount, l);
    return (at(d.ls_old, l + 1) - at(d.ls_old, l)) - at(d.leave, l) + j;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(Dev d)
{
    __shared__ int sh[2 * kScanThreads];
    const int base = blockIdx.x * kScanLanes + threadIdx.x * kScanPer;
    int tot = 0, tj = 0;
    for (int q = 0; q < kScanPer; ++q) {
        int l = base + q;
        if (l < d.n_lanes) {
            int j;
            tot += new_count(d, l, j);
            tj += j;
        }
    }
    block_scan2(tot, tj, sh);
    if (threadIdx.x == kScanThreads - 1) {
        at(d.blk, 2 * blockIdx.x) = tot;
        at(d.blk, 2 * blockIdx.x + 1) = tj;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(Dev d)
{
    __shared__ int sh[2 * kScanThreads];
    const int b = blockIdx.x;
    int off = 0, offj = 0;
    for (int q = threadIdx.x; q < b; q += kScanThreads) {
        off += at(d.blk, 2 * q);
        offj += at(d.blk, 2 * q + 1);
    }
    block_scan2(off, offj, sh);
    __shared__ int base_tot, base_j;
    if (threadIdx.x == kScanThreads - 1) {
        base_tot = off;
        base_j = offj;
    }
    __syncthreads();
    const int b0 = base_tot, bj = base_j;
    const uint32_t tnext = (uint32_t)(*d.t + 1);
    const int base = b * kScanLanes + threadIdx.x * kScanPer;
    int cnt[kScanPer], jc[kScanPer];
    int tot = 0, tj = 0;
    for (int q = 0; q < kScanPer; ++q) {
        int l = base + q;
        cnt[q] = 0;
        jc[q] = 0;
        if (l < d.n_lanes)
            cnt[q] = new_count(d, l, jc[q]);
        tot += cnt[q];
        tj += jc[q];
    }
    int inc = tot, incj = tj;
    block_scan2(inc, incj, sh);
    int run = b0 + inc - tot, runj = bj + incj - tj;
    for (int q = 0; q < kScanPer; ++q) {
        int l = base + q;
        if (l < d.n_lanes) {
            at(d.ls_new, l) = run;
            at(d.joff, l) = runj;
            at(d.jcur, l) = runj;
            at(d.leave, l) = 0;
            at(d.jcount, l) = 0;
            // red light of the lane's road at the next step
            at(d.lane_red, l) = lane_flags_at(at(d.lanes, l), tnext);
            // chunks past lane l's and up to lane l+1's begin at lane l+1:
            // record its lane, new start, old start and joiner offset
            for (int w = chunk_of(l, run) + 1; w <= chunk_of(l + 1, run + cnt[q]); ++w)
                at(d.chunk, w) = make_int4(l + 1, run + cnt[q], at(d.ls_old, l + 1), runj + jc[q]);
        }
        run += cnt[q];
        runj += jc[q];
    }
    if (b == 0 && threadIdx.x == 0)
        at(d.chunk, 0) = make_int4(0, 0, 0, 0);
    if (b == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) {
        at(d.ls_new, d.n_lanes) = run;
        at(d.joff, d.n_lanes) = runj;
        *d.n_next = run;
        // upper bound of the last chunk (merge blocks past it read nothing)
        at(d.chunk, chunk_of(d.n_lanes, run) + 1) =
            make_int4(d.n_lanes, run, at(d.ls_old, d.n_lanes), runj);
    }
}

// ----------------------------------------------------- joiners by lane --

// One wave per update tile (then per kUpdateRows queue lanes' insertion
// entries, kNone for a lane that inserted nothing): each joiner takes
// the next slot of its target lane's bucket.
__global__ void __launch_bounds__(256) k_jscatter(Dev d)
{
    const int ntiles = (*d.n_cur + kUpdateRows - 1) / kUpdateRows;
    // insertion entries (one per queue lane) in tiles of kUpdateRows after
    // the update tiles
    const int nins = (int)*d.n_ins;
    const int itiles = (nins + kUpdateRows - 1) / kUpdateRows;
    const int lane = __lane_id();
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int tile = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); tile < ntiles + itiles;
         tile += waves) {
        const bool ins = tile >= ntiles;
        const int k0 = ins ? (tile - ntiles) * kUpdateRows : 0;
        const int cnt = ins ? min(kUpdateRows, nins - k0) : at(d.jcnt, tile);
        const uint32_t *lst = ins ? d.jins_list + k0 : d.jlist + (size_t)tile * kUpdateRows;
        const uint32_t *lan = ins ? d.jins_lane + k0 : d.jlane + (size_t)tile * kUpdateRows;
        for (int k = lane; k < cnt; k += 64) {
            const uint32_t x = lan[k], src = lst[k];
            if (x == kNone)
                continue;       // a queue lane that inserted nothing
            // the record's loads do not wait for the slot
            const float s = at(d.Pr.s, src), v = at(d.Pr.v, src), a = at(d.Pr.a, src), v0 = at(d.Pr.v0, src);
            const uint32_t id = at(d.Pr.id, src), ptr = at(d.Pr.ptr, src);
            const int32_t next = at(d.Pr.next, src);
            const int pos = atomicAdd(&at(d.jcur, x), 1);
            at(d.jidx, pos) = src;
            at(d.J.lane, pos) = x;
            at(d.J.s, pos) = s;
            at(d.J.v, pos) = v;
            at(d.J.a, pos) = a;
            at(d.J.id, pos) = id;
            at(d.J.ptr, pos) = ptr;
            at(d.J.next, pos) = next;
            at(d.J.v0, pos) = v0;
        }
    }
}

// ------------------------------------------------------------------ merge --
//
// The next order of lane l is the merge of its stayers (rows of l that stay,
// in their old order) with its joiners (by (s, id)): walking both lists from
// the tail, the smaller (s, id) key goes first.  Stayers need not be sorted by
// their new positions, and the walk is then characterised by prefix maxima:
// with pm_p the largest stayer key among stayers 0..p, stayer p is preceded by
// exactly the joiners whose key is below pm_p, and a joiner by exactly the
// stayers up to the first one with pm above its key.  k_merge evaluates those
// counts in parallel; overlaps are then removed from the lane head backwards,
// starting at the highest overlapping pair (rows above it keep their values).

__device__ __forceinline__ bool key_less(const Dev &d, uint32_t a, uint32_t b)
{
    float sa = at(d.Pr.s, a), sb = at(d.Pr.s, b);
    if (sa != sb)
        return sa < sb;
    return at(d.Pr.id, a) < at(d.Pr.id, b);
}

// (s, id) as one unsigned key with the order of the float comparison followed
// by the id; -0 is first made +0 because the two compare equal.
__device__ __forceinline__ uint64_t okey(float s, uint32_t id)
{
    uint32_t b = __float_as_uint(s + 0.0f);
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((uint64_t)b << 32) | id;
}

__device__ __forceinline__ void write_row(const Dev &d, int w, uint32_t src, uint32_t lane, float s,
                                          float v)
{
    at(d.S.s, w) = s;
    at(d.S.v, w) = v;
    at(d.S.a, w) = at(d.Pr.a, src);
    at(d.id_next, w) = at(d.Pr.id, src);
    at(d.S.lane, w) = lane;
    at(d.S.ptr, w) = at(d.Pr.ptr, src);
    at(d.S.next, w) = at(d.Pr.next, src);
    at(d.v0_next, w) = at(d.Pr.v0, src);
}

__device__ __forceinline__ void write_tail(const Dev &d, int l, bool any, float s, float v,
                                           uint32_t id)
{
    Tail tl;
    tl.pad = 0;
    tl.s = any ? s : 0.0f;
    tl.v = any ? v : 0.0f;
    tl.id = any ? id : kNone;
    at(d.tails, l) = tl;
}

// Merge of one lane straight from global memory, walking both lists (used for
// chunks too large for the LDS tile).
__device__ void merge_lane_global(const Dev &d, int l, uint64_t &vsum, unsigned long long &clamps)
{
    vsum = 0;
    clamps = 0;
    const int o0 = at(d.ls_old, l), o1 = at(d.ls_old, l + 1);
    const int j0 = at(d.joff, l), j1 = at(d.joff, l + 1);
    const int w0 = at(d.ls_new, l), w1 = at(d.ls_new, l + 1);
    for (int a = j0 + 1; a < j1; ++a) {
        uint32_t xk = at(d.jidx, a);
        int b = a - 1;
        while (b >= j0 && key_less(d, xk, at(d.jidx, b))) {
            at(d.jidx, b + 1) = at(d.jidx, b);
            --b;
        }
        at(d.jidx, b + 1) = xk;
    }
    int ip = o0, jp = j0, w = w0;
    for (;;) {
        while (ip < o1 && (at(d.Pr.lane, ip) & kJoinBit))
            ++ip;
        const bool hs = ip < o1, hj = jp < j1;
        if (!hs && !hj)
            break;
        if (w >= w1) {          // counts disagree with the scan: never write past the lane
            atomicOr(d.err, 1u);
            break;
        }
        uint32_t src;
        if (hs && (!hj || key_less(d, (uint32_t)ip, at(d.jidx, jp))))
            src = (uint32_t)ip++;
        else
            src = at(d.jidx, jp++);
        write_row(d, w, src, (uint32_t)l, at(d.Pr.s, src), at(d.Pr.v, src));
        ++w;
    }
    if (w != w1)
        atomicOr(d.err, 1u);
    for (int f = w1 - 2; f >= w0; --f) {
        float lim = at(d.S.s, f + 1) - d.P.len;
        if (at(d.S.s, f) > lim) {
            at(d.S.s, f) = lim;
            at(d.S.v, f) = fmin32(at(d.S.v, f), at(d.S.v, f + 1));
            ++clamps;
        }
    }
    write_tail(d, l, w1 > w0, at(d.S.s, w0), at(d.S.v, w0), at(d.id_next, w0));
    for (int f = w0; f < w1; ++f)
        vsum += speed_fx(at(d.S.v, f));
}

constexpr int kMT = 256;          // threads per merge block (4 waves)
constexpr int kMC = kMergeRows;   // new rows per chunk
constexpr int kOldCap = 3 * kMT;  // old rows staged per chunk (3 per thread)
constexpr int kNewCap = 3 * kMT;  // new rows staged per chunk
constexpr int kJCap = 160;        // joiners staged per chunk (at most 1 per thread)
constexpr int kLaneCap = 128;     // owned lanes whose starts are cached in LDS
// Sources of placed rows (w_src): an old row index, a joiner index | kTagJ,
// or kNoSrc; both indices are below 2^15.
constexpr uint16_t kTagJ = 0x8000u;
constexpr uint16_t kNoSrc = 0xFFFFu;
// Lanes of staged rows and joiners are kept relative to the chunk's first
// owned lane, in 15 bits, with kLeave16 marking old rows that leave the lane.
constexpr uint16_t kLeave16 = 0x8000u;
constexpr int kRelLanes = 0x8000;

// Segmented scan over one wave of old rows: inclusive prefix maximum of the
// stayer keys (returned as the row index holding it, kNoRow before the
// lane's first stayer) and exclusive count of stayers, restarting at lane
// heads and continuing from the carry when the wave's first rows continue a
// lane.
constexpr uint32_t kNoRow = 0xFFFFu;
static_assert(2 * kOldCap + kJCap <= 4 * kNewCap, "o_p, o_pi and j_ord share u_buf");
static_assert(kOldCap < 0x8000 && kJCap < 0x8000, "row sources are 15-bit indices");

__device__ __forceinline__ void wave_seg_scan(bool valid, bool head, bool st, uint64_t key,
                                              uint32_t row, uint64_t &c_pm, uint32_t &c_pi,
                                              uint32_t &c_p, uint32_t &pi_out, uint32_t &p_out)
{
    const int lane = __lane_id();
    const unsigned long long hm = __ballot(valid && head);
    const unsigned long long sm = __ballot(valid && st);
    const unsigned long long upto = (lane == 63) ? hm : (hm & ((2ull << lane) - 1ull));
    const int h = upto ? 63 - __clzll(upto) : -1;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const unsigned long long seg = (h < 0) ? below : (below & ~((1ull << h) - 1ull));
    uint32_t p = (uint32_t)__popcll(sm & seg);
    uint64_t v = (valid && st) ? key : 0ull;
    uint32_t vi = (valid && st) ? row : kNoRow;
    // Hillis-Steele within rows of 16, then across rows; a lane without a
    // source keeps its own value, which never wins (o > v fails)
    seg_max_step<kDppShr1, 0xF>(v, vi, lane - 1 >= h);
    seg_max_step<kDppShr2, 0xF>(v, vi, lane - 2 >= h);
    seg_max_step<kDppShr4, 0xF>(v, vi, lane - 4 >= h);
    seg_max_step<kDppShr8, 0xF>(v, vi, lane - 8 >= h);
    seg_max_step<kDppBcast15, 0xA>(v, vi, (lane & ~15) - 1 >= h);
    seg_max_step<kDppBcast31, 0xC>(v, vi, 31 >= h);
    if (h < 0) {
        p += c_p;
        if (c_pm > v) {
            v = c_pm;
            vi = c_pi;
        }
    }
    pi_out = vi;
    p_out = p;
    // carry for the next wave of rows: the state after row 63
    c_pm = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    c_pi = (uint32_t)__builtin_amdgcn_readlane((int)vi, 63);
    c_p = (uint32_t)__builtin_amdgcn_readlane((int)p, 63) + (uint32_t)((sm >> 63) & 1ull);
}

// Merge of the whole lanes [la, lb) -- new rows [n0, n1), old rows [o0, o1),
// joiners [j0, j1), which the caller has checked to fit the LDS tile.  Their
// old rows and joiners are staged in LDS (their other fields in registers of
// the staging thread), positions are computed in parallel (see above),
// overlaps are removed per lane, and the rows are written out.
__device__ __forceinline__ void merge_group(const Dev &d, const int la, const int lb, const int n0,
                                            const int n1, const int o0, const int o1,
                                            const int j0, const int j1, const bool one_scen,
                                            uint64_t &vsum, unsigned long long &clamps)
{
    __shared__ float o_s[kOldCap], o_v[kOldCap];
    __shared__ uint32_t o_id[kOldCap];
    __shared__ uint16_t o_ln[kOldCap];
    // stayer ranks, prefix-maximum rows and the joiners in key order per lane
    // (scan to stayer placement), then the overlap markers of the lanes'
    // first rows (overlap removal)
    __shared__ uint32_t u_buf[2 * kNewCap];
    uint16_t *const o_p = reinterpret_cast<uint16_t *>(u_buf);
    uint16_t *const o_pi = o_p + kOldCap;
    uint16_t *const j_ord = o_pi + kOldCap;
    int *const w_top = reinterpret_cast<int *>(u_buf);
    int *const w_bot = w_top + kNewCap;
    __shared__ float j_s[kJCap], j_v[kJCap];
    __shared__ uint32_t j_id[kJCap];
    __shared__ uint16_t j_ln[kJCap];
    __shared__ uint16_t w_src[kNewCap];
    __shared__ int lt_old[kLaneCap + 1], lt_new[kLaneCap + 1], lt_jo[kLaneCap + 1];
    __shared__ int wave_start[5];

    const int tid = threadIdx.x;
    const int lane = __lane_id();
    const int wv = tid >> 6;
    const int no = o1 - o0, nw = n1 - n0, nj = j1 - j0;
    const float len = d.P.len;
    // ---- owned lanes' old starts, new starts and joiner offsets, old rows
    // (3 per thread) and joiners (1 per thread): every load is issued before
    // the first LDS store waits for one, from indices clamped to valid
    // entries, rows and joiners (row 0 and joiner 0 when there are none)
    const bool lt_ok = lb - la <= kLaneCap;
    static_assert(kLaneCap + 1 <= kMT, "one lane-table entry per thread");
    const int qc = la + min(tid, lb - la);
    const int lt_o = at(d.ls_old, qc), lt_n = at(d.ls_new, qc), lt_j = at(d.joff, qc);
    float rs[3], rv[3], ra[3], rv0[3];
    uint32_t rl[3], rid[3], rptr[3];
    int32_t rnext[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int r = no > 0 ? o0 + min(tid + k * kMT, no - 1) : 0;
        rs[k] = at(d.Pr.s, r);
        rv[k] = at(d.Pr.v, r);
        rl[k] = at(d.Pr.lane, r);
        rid[k] = at(d.Pr.id, r);
        ra[k] = at(d.Pr.a, r);
        rptr[k] = at(d.Pr.ptr, r);
        rnext[k] = at(d.Pr.next, r);
        rv0[k] = at(d.Pr.v0, r);
    }
    const int qj = nj > 0 ? j0 + min(tid, nj - 1) : 0;
    const float js = at(d.J.s, qj), jv = at(d.J.v, qj);
    const uint32_t jid = at(d.J.id, qj), jl = at(d.J.lane, qj);
    const float ja = at(d.J.a, qj), jv0 = at(d.J.v0, qj);
    const uint32_t jptr = at(d.J.ptr, qj);
    const int32_t jnext = at(d.J.next, qj);
    if (lt_ok && tid <= lb - la) {
        lt_old[tid] = lt_o;
        lt_new[tid] = lt_n;
        lt_jo[tid] = lt_j;
    }
    auto LO = [&](int l) { return lt_ok ? lt_old[l - la] : at(d.ls_old, l); };
    auto LN = [&](int l) { return lt_ok ? lt_new[l - la] : at(d.ls_new, l); };
    auto JO = [&](int l) { return lt_ok ? lt_jo[l - la] : at(d.joff, l); };
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int r = tid + k * kMT;
        if (r < no) {
            o_s[r] = rs[k];
            o_v[r] = rv[k];
            o_ln[r] = (uint16_t)(((rl[k] & ~kJoinBit) - (uint32_t)la) |
                                 ((rl[k] & kJoinBit) ? kLeave16 : 0u));
            o_id[r] = rid[k];
        }
    }
    if (tid < nj) {
        j_s[tid] = js;
        j_v[tid] = jv;
        j_id[tid] = jid;
        j_ln[tid] = (uint16_t)(jl - (uint32_t)la);
    }
    for (int k = tid; k < nw; k += kMT)
        w_src[k] = kNoSrc;
    __syncthreads();
    // ---- split the old rows among the 4 waves at lane boundaries (first
    // lane start at or after an even share, found 64 rows at a time)
    {
        int r = (no * wv) / 4;
        if (wv > 0 && r > 0) {
            for (;;) {
                const int q = r + lane;
                const bool bnd = q >= no || (o_ln[q] & ~kLeave16) != (o_ln[q - 1] & ~kLeave16);
                const unsigned long long m = __ballot(bnd);
                if (m) {
                    r += __ffsll((long long)m) - 1;
                    break;
                }
                r += 64;
            }
        }
        if (lane == 0) {
            wave_start[wv] = (wv == 0) ? 0 : min(r, no);
            if (wv == 3)
                wave_start[4] = no;
        }
    }
    // ---- joiners: rank among the lane's joiners, which orders them by key
    int jq = 0;
    if (tid < nj) {
        const uint32_t l = (uint32_t)la + j_ln[tid];
        const uint64_t key = okey(j_s[tid], j_id[tid]);
        const int jl = JO(l) - j0, jh = JO(l + 1) - j0;
        for (int e2 = jl; e2 < jh; ++e2)
            jq += okey(j_s[e2], j_id[e2]) < key;
        j_ord[jl + jq] = (uint16_t)tid;
    }
    __syncthreads();
    // ---- stayer ranks and prefix maxima, one wave per row range
    {
        const int ra0 = wave_start[wv], rb0 = max(wave_start[wv + 1], ra0);
        uint64_t c_pm = 0;
        uint32_t c_pi = kNoRow, c_p = 0;
        for (int r0 = ra0; r0 < rb0; r0 += 64) {
            const int r = r0 + lane;
            const bool valid = r < rb0;
            bool head = false, st = false;
            uint64_t key = 0;
            if (valid) {
                const uint32_t ln = o_ln[r];
                st = (ln & kLeave16) == 0;
                head = (r == ra0) || ((o_ln[r - 1] & ~kLeave16) != (ln & ~kLeave16));
                key = okey(o_s[r], o_id[r]);
            }
            uint32_t pi, p;
            wave_seg_scan(valid, head, st, key, (uint32_t)r, c_pm, c_pi, c_p, pi, p);
            if (valid) {
                o_p[r] = (uint16_t)p;
                o_pi[r] = (uint16_t)pi;
            }
        }
    }
    __syncthreads();
    // ---- joiners: the stayers before them (the first old row of the lane
    // whose prefix maximum exceeds the key); stayers below
    if (tid < nj) {
        const int e = tid;
        const uint32_t l = (uint32_t)la + j_ln[e];
        const uint64_t key = okey(j_s[e], j_id[e]);
        const int jl = JO(l) - j0, jh = JO(l + 1) - j0;
        const int q = jq;
        const int lo = LO(l) - o0, hi = LO(l + 1) - o0;
        int a = lo, b = hi;       // first old row of l with prefix max > key
        while (a < b) {
            const int mid = (a + b) >> 1;
            const uint32_t pr = o_pi[mid];
            const uint64_t pm = (pr == kNoRow) ? 0ull : okey(o_s[pr], o_id[pr]);
            if (pm > key)
                b = mid;
            else
                a = mid + 1;
        }
        const int wl = LN(l) - n0;
        const int stay_total = (LN(l + 1) - LN(l)) - (jh - jl);
        const int f = (a < hi) ? (int)o_p[a] : stay_total;
        const int pos = wl + f + q;
        if (pos >= 0 && pos < nw) {
            w_src[pos] = (uint16_t)(kTagJ | e);
            const int g = n0 + pos;
            at(d.S.a, g) = ja;
            at(d.id_next, g) = j_id[e];
            at(d.S.lane, g) = l;
            at(d.S.ptr, g) = jptr;
            at(d.S.next, g) = jnext;
            at(d.v0_next, g) = jv0;
        } else {
            atomicOr(d.err, 1u);
        }
    }
    // ---- stayers: joiners with a smaller key than their prefix maximum
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int r = tid + k * kMT;
        if (r >= no)
            continue;
        if (o_ln[r] & kLeave16)
            continue;
        const uint32_t ln = (uint32_t)la + o_ln[r];
        const uint32_t pr = o_pi[r];    // a stayer: its own row or one before it
        const uint64_t pm = okey(o_s[pr], o_id[pr]);
        const int jl = JO(ln) - j0, jh = JO(ln + 1) - j0;
        int a = jl, b = jh;       // joiners of the lane with key < pm (sorted keys)
        while (a < b) {
            const int mid = (a + b) >> 1;
            const uint32_t je = j_ord[mid];
            const uint64_t kk = okey(j_s[je], j_id[je]);
            if (kk < pm)
                a = mid + 1;
            else
                b = mid;
        }
        const int pos = (LN(ln) - n0) + (int)o_p[r] + (a - jl);
        if (pos >= 0 && pos < nw) {
            w_src[pos] = (uint16_t)r;
            const int g = n0 + pos;
            at(d.S.a, g) = ra[k];
            at(d.id_next, g) = o_id[r];
            at(d.S.lane, g) = ln;
            at(d.S.ptr, g) = rptr[k];
            at(d.S.next, g) = rnext[k];
            at(d.v0_next, g) = rv0[k];
        } else {
            atomicOr(d.err, 1u);
        }
    }
    __syncthreads();
    // lane of a placed row (stayers carry no leave bit)
    auto lane_of = [&](uint32_t x) {
        return (uint32_t)la + ((x & kTagJ) ? j_ln[x & ~kTagJ] : o_ln[x]);
    };
    for (int k = tid; k < nw; k += kMT) {
        w_top[k] = -1;
        w_bot[k] = 0x7FFFFFFF;
    }
    __syncthreads();
    // ---- overlaps: highest offending pair of each lane
    for (int k = tid; k < nw; k += kMT) {
        const uint32_t x = w_src[k];
        if (x == kNoSrc) {
            atomicOr(d.err, 1u);
            continue;
        }
        const uint32_t lk = lane_of(x);
        if (k + 1 < nw && w_src[k + 1] != kNoSrc && lane_of(w_src[k + 1]) == lk) {
            const uint32_t y = w_src[k + 1];
            const float sk = (x & kTagJ) ? j_s[x & ~kTagJ] : o_s[x];
            const float sn = (y & kTagJ) ? j_s[y & ~kTagJ] : o_s[y];
            if (sk > sn - len) {
                const int first = LN((int)lk) - n0;
                atomicMax(&w_top[first], k);
                atomicMin(&w_bot[first], k);
            }
        }
    }
    __syncthreads();
    // ---- sequential removal from there down towards the lane tail.  Below
    // the lowest offending pair of raw positions, a row left unchanged
    // leaves every row behind it unchanged, so the walk stops there.
    for (int k = tid; k < nw; k += kMT) {
        const int top = w_top[k];
        if (top < 0)
            continue;     // set only at a lane's first row
        const int bot = w_bot[k];
        const uint32_t y = w_src[top + 1];
        float sl = (y & kTagJ) ? j_s[y & ~kTagJ] : o_s[y];
        float vl = (y & kTagJ) ? j_v[y & ~kTagJ] : o_v[y];
        for (int f = top; f >= k; --f) {
            const uint32_t xf = w_src[f];
            const bool jf = (xf & kTagJ) != 0;
            const uint32_t kf = xf & ~kTagJ;
            float sf = jf ? j_s[kf] : o_s[kf];
            float vf = jf ? j_v[kf] : o_v[kf];
            const float lim = sl - len;
            if (sf > lim) {
                sf = lim;
                vf = fmin32(vf, vl);
                if (jf) { j_s[kf] = sf; j_v[kf] = vf; }
                else { o_s[kf] = sf; o_v[kf] = vf; }
                ++clamps;
                if (!one_scen)
                    atomicAdd(cnt_at(d, at(d.lanes, lane_of(w_src[k])).scen, C_CLAMPS), 1ull);
            } else if (f < bot) {
                break;
            }
            sl = sf;
            vl = vf;
        }
    }
    __syncthreads();
    // ---- lane tails (empty lanes too)
    for (int l = la + tid; l < lb; l += kMT) {
        const int wl = LN(l) - n0, wh = LN(l + 1) - n0;
        if (wh > wl && w_src[wl] != kNoSrc) {
            const uint32_t x = w_src[wl];
            if (x & kTagJ)
                write_tail(d, l, true, j_s[x & ~kTagJ], j_v[x & ~kTagJ], j_id[x & ~kTagJ]);
            else
                write_tail(d, l, true, o_s[x], o_v[x], o_id[x]);
        } else {
            write_tail(d, l, false, 0.0f, 0.0f, kNone);
        }
    }
    // ---- positions and speeds of the chunk's rows, coalesced (a chunk of
    // several scenarios counts per scenario present in each wave)
    for (int k0 = 0; k0 < nw; k0 += kMT) {
        const int k = k0 + tid;
        const uint32_t x = k < nw ? w_src[k] : kNoSrc;
        const bool ok = x != kNoSrc;
        float v = 0.0f;
        int sc = 0;
        if (ok) {
            const bool jx = (x & kTagJ) != 0;
            const uint32_t e = x & ~kTagJ;
            const float s = jx ? j_s[e] : o_s[e];
            v = jx ? j_v[e] : o_v[e];
            at(d.S.s, n0 + k) = s;
            at(d.S.v, n0 + k) = v;
            if (one_scen)
                vsum += speed_fx(v);
            else
                sc = at(d.lanes, lane_of(x)).scen;
        }
        if (!one_scen) {
            wave_count_scen(d, C_VEH_STEPS, ok, sc);
            wave_sumv_scen(d, ok, sc, speed_fx(v));
        }
    }
}

// Lanes [la, lb) one per thread, straight from global memory.
__device__ void merge_lanes_global(const Dev &d, const int la, const int lb, const bool one_scen,
                                   uint64_t &vsum, unsigned long long &clamps)
{
    const int tid = threadIdx.x;
    for (int l = la + tid; l < lb; l += kMT) {
        uint64_t ls;
        unsigned long long lc;
        merge_lane_global(d, l, ls, lc);
        const int cnt = at(d.ls_new, l + 1) - at(d.ls_new, l);
        if (one_scen) {
            vsum += ls;
            clamps += lc;
        } else {
            unsigned long long *c = cnt_at(d, at(d.lanes, l).scen, 0);
            if (cnt) {
                atomicAdd(c + C_VEH_STEPS, (unsigned long long)cnt);
                atomicAdd(sumv_at(d, at(d.lanes, l).scen), (unsigned long long)ls);
            }
            if (lc) atomicAdd(c + C_CLAMPS, lc);
        }
    }
}

__device__ __forceinline__ bool group_fits(int new_rows, int old_rows, int joiners, int lanes)
{
    return new_rows <= kNewCap && old_rows <= kOldCap && joiners <= kJCap && lanes < kRelLanes;
}

// Next state, one chunk per block: the lanes between two chunk boundaries
// (every kMC new rows and every kMergeLanes lanes), merged with merge_group.
// A chunk that does not fit the LDS tile is merged in consecutive groups of
// whole lanes that do (at most two); the lanes from one that alone exceeds
// the tile on, or beyond the two groups, take merge_lanes_global.
__global__ void __launch_bounds__(kMT) k_merge(Dev d)
{
    __shared__ uint64_t red_d[kMT / 64];
    __shared__ unsigned long long red_k[kMT / 64];
    __shared__ int s_gb;

    const int tid = threadIdx.x;
    const int lane = __lane_id();
    const int wv = tid >> 6;
    // The chunk of this block when the rows fill the grid (the usual case)
    // is loaded together with the row count, and loaded again only when that
    // guess is wrong; w is uniform, every thread reads the same records.
    const int wg = min(xcd_tile(d.xcd_remap, (int)gridDim.x, (int)gridDim.x),
                       d.cap / kMC + d.n_lanes / kMergeLanes + 1);
    int4 ca = at(d.chunk, wg), cb = at(d.chunk, wg + 1);
    const int n_next = *d.n_next;
    const int nch = chunk_of(d.n_lanes, n_next);     // the last chunk
    const int w = xcd_tile(d.xcd_remap, nch + 1, (int)gridDim.x);
    if (w > nch)
        return;
    if (w != wg) {
        ca = at(d.chunk, w);
        cb = at(d.chunk, w + 1);
    }
    const int la = ca.x, lb = cb.x;
    const int n0 = ca.y, n1 = cb.y, o0 = ca.z, o1 = cb.z, j0 = ca.w, j1 = cb.w;
    const int nw = n1 - n0;
    const bool one_scen = (lb <= la) || at(d.lanes, la).scen == at(d.lanes, lb - 1).scen;
    uint64_t vsum = 0;
    unsigned long long clamps = 0;

    // the longest run of whole lanes from ga that fits the tile (ga itself
    // when lane ga alone exceeds it); uniform, computed by one thread
    auto longest_fit = [&](int ga, int g_n0, int g_o0, int g_j0) {
        if (tid == 0) {
            int lo = ga, hi = lb;      // [ga, lo) fits, [ga, hi) does not
            while (hi - lo > 1) {
                const int mid = lo + ((hi - lo) >> 1);
                if (group_fits(at(d.ls_new, mid) - g_n0, at(d.ls_old, mid) - g_o0, at(d.joff, mid) - g_j0,
                               mid - ga))
                    lo = mid;
                else
                    hi = mid;
            }
            s_gb = lo;
        }
        __syncthreads();
        const int gb = __builtin_amdgcn_readfirstlane(s_gb);
        __syncthreads();               // s_gb may be written again
        return gb;
    };
    // At most two groups through the tile (written out rather than looped:
    // a loop around the tile code costs it about 40 VGPRs).  The lanes left
    // after them -- from a lane that alone exceeds the tile on, or beyond
    // two tiles' worth -- are merged one per thread.
    int ga = la;
    int gb = group_fits(nw, o1 - o0, j1 - j0, lb - la) ? lb : longest_fit(la, n0, o0, j0);
    if (gb > ga) {
        const int g_n1 = gb == lb ? n1 : __builtin_amdgcn_readfirstlane(at(d.ls_new, gb));
        const int g_o1 = gb == lb ? o1 : __builtin_amdgcn_readfirstlane(at(d.ls_old, gb));
        const int g_j1 = gb == lb ? j1 : __builtin_amdgcn_readfirstlane(at(d.joff, gb));
        merge_group(d, ga, gb, n0, g_n1, o0, g_o1, j0, g_j1, one_scen, vsum, clamps);
        ga = gb;
    }
    if (ga < lb) {
        __syncthreads();               // the LDS tile is reused
        const int g_n0 = __builtin_amdgcn_readfirstlane(at(d.ls_new, ga));
        const int g_o0 = __builtin_amdgcn_readfirstlane(at(d.ls_old, ga));
        const int g_j0 = __builtin_amdgcn_readfirstlane(at(d.joff, ga));
        gb = group_fits(n1 - g_n0, o1 - g_o0, j1 - g_j0, lb - ga) ? lb
                                                                  : longest_fit(ga, g_n0, g_o0, g_j0);
        if (gb > ga) {
            const int g_n1 = __builtin_amdgcn_readfirstlane(at(d.ls_new, gb));
            const int g_o1 = __builtin_amdgcn_readfirstlane(at(d.ls_old, gb));
            const int g_j1 = __builtin_amdgcn_readfirstlane(at(d.joff, gb));
            merge_group(d, ga, gb, g_n0, g_n1, g_o0, g_o1, g_j0, g_j1, one_scen, vsum, clamps);
            ga = gb;
        }
        if (ga < lb)
            merge_lanes_global(d, ga, lb, one_scen, vsum, clamps);
    }

    if (one_scen) {
        vsum = wave_sum_u64_l63(vsum);
        const uint32_t ck32 = wave_scan_u32((uint32_t)clamps);
        if (lane == 63) {
            red_d[wv] = vsum;
            red_k[wv] = ck32;
        }
        __syncthreads();
        if (tid == 0 && lb > la) {
            uint64_t sv = 0;
            unsigned long long ck = 0;
            for (int q = 0; q < kMT / 64; ++q) {
                sv += red_d[q];
                ck += red_k[q];
            }
            const int sc = at(d.lanes, la).scen;
            unsigned long long *c = cnt_at(d, sc, 0);
            if (nw) atomicAdd(c + C_VEH_STEPS, (unsigned long long)nw);
            if (ck) atomicAdd(c + C_CLAMPS, ck);
            if (nw) atomicAdd(sumv_at(d, sc), (unsigned long long)sv);
        }
    }
    if (w == 0 && tid == 0) {
        *d.n_dbg = *d.n_cur;
        *d.n_cur = n_next;
        *d.n_ins = 0u;
        *d.t = *d.t + 1;
    }
}

// -------------------------------------------------------------- utilities --

__global__ void k_tails(Dev d)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= d.n_lanes)
        return;
    const int w0 = at(d.ls_old, l), w1 = at(d.ls_old, l + 1);
    const bool any = w1 > w0;
    write_tail(d, l, any, any ? at(d.S.s, w0) : 0.0f, any ? at(d.S.v, w0) : 0.0f,
               any ? at(d.S.id, w0) : kNone);
}

// Yield flags of the step about to run (junction internal lanes), one per
// lane: connector lane cl is busy when a conflicting connector lane with
// priority over it holds a vehicle (its tail), or the lane feeding such a
// connector has a first vehicle (highest position) headed into it, not held
// by a red light, and within tau_yield seconds of its stop line at its speed
// (L - s <= v tau_yield); lanes without conflicts are never busy.  Computed
// once per step from the state with lane starts ls, its tails and the red
// flags of the step, so that a lane head reads one flag instead of walking
// the conflict list.
__global__ void k_yield(Dev d, const int32_t *ls)
{
    const int cl = blockIdx.x * blockDim.x + threadIdx.x;
    if (cl >= d.n_lanes)
        return;
    const int a = at(d.conf_off, cl), b = at(d.conf_off, cl + 1);
    uint8_t busy = 0;
    for (int q = a; q < b && !busy; ++q) {
        const Succ c2 = at(d.conf, q);
        if (at(d.tails, c2.lane).id != kNone) {
            busy = 1;
            break;
        }
        const int f = at(d.conf_feed, q);
        const int w0 = at(ls, f), w1 = at(ls, f + 1);
        if (w1 > w0 && at(d.S.next, w1 - 1) == c2.road && !(at(d.lane_red, f) & kRedBit) &&
            at(d.lanes, f).L - at(d.S.s, w1 - 1) <= at(d.S.v, w1 - 1) * d.P.tau_yield)
            busy = 1;
    }
    at(d.busy, cl) = busy;
}

__device__ __forceinline__ int find_vehicle(const Dev &d, uint32_t id)
{
    int lo = 0, hi = d.n_veh;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (at(d.vt_id, mid) < id)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ void k_cursor(Dev d, const uint32_t *ids, const uint32_t *ptrs, int32_t *out, int32_t n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int vi = find_vehicle(d, ids[i]);
    out[i] = (int32_t)(ptrs[i] - at(d.vt_rstart, vi));
}

// Trips, first pass, one thread per vehicle in id order: a vehicle whose
// arrival step is recorded after its route has arrived (status 2; trip time;
// its whole route's length, summed in FP64 in route order, less the route
// distance where it entered).  Every other vehicle is set to waiting (status
// 0), and the second pass overwrites those on the network.
__global__ void k_trips_all(Dev d, int32_t *status, int32_t *travel, double *dist)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.n_veh)
        return;
    uint32_t p = at(d.vt_rstart, k);
    double acc = 0.0;
    for (int32_t r = at(d.route, p); r >= 0; r = at(d.route, p)) {
        acc += (double)at(d.roads, r).L;
        ++p;
    }
    const int32_t dep = at(d.route, p + 1), arr = at(d.route, p + 2);
    const bool done = arr >= 0;
    at(status, k) = done ? 2 : 0;
    at(travel, k) = done ? arr - dep : 0;
    at(dist, k) = done ? acc - at(d.vt_dist0, k) : 0.0;
}

// Trips, second pass, one thread per state row: the vehicle is on the network
// (status 1); travel time = current step index - departure step; distance =
// lengths of the roads before its current one (FP64, route order) plus its
// position, less the route distance where it entered.
__global__ void k_trips_active(Dev d, int32_t n, int32_t *status, int32_t *travel, double *dist)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int k = find_vehicle(d, at(d.S.id, i));
    const uint32_t r0 = at(d.vt_rstart, k), ptr = at(d.S.ptr, i);
    double acc = 0.0;
    for (uint32_t p = r0; p < ptr; ++p)
        acc += (double)at(d.roads, at(d.route, p)).L;
    at(status, k) = 1;
    at(travel, k) = (int32_t)(*d.t - (int64_t)at(d.vt_dep, k));
    at(dist, k) = (acc + (double)at(d.S.s, i)) - at(d.vt_dist0, k);
}

static inline unsigned blocks_for(long long n, int per)
{
    long long b = (n + per - 1) / per;
    return (unsigned)(b < 1 ? 1 : b);
}

static const char *const kStepKernels[] = {"k_update", "k_scan_reduce", "k_scan_apply",
                                            "k_jscatter", "k_merge", "k_yield"};

int step_kernel_count() { return (int)(sizeof kStepKernels / sizeof kStepKernels[0]); }
int step_scan_block_lanes() { return kScanLanes; }
const char *step_kernel_name(int i)
{
    return (i >= 0 && i < step_kernel_count()) ? kStepKernels[i] : nullptr;
}

// The update kernel with or without the insertion workgroups.
template <int MODE, bool AUX, bool EXT>
static void (*update_variant(bool ins))(Dev)
{
    return ins ? k_update<MODE, AUX, EXT, true> : k_update<MODE, AUX, EXT, false>;
}

// Enqueues one step.  With ev != nullptr, ev[0] is recorded before the first
// kernel and ev[k+1] after kernel k (in kStepKernels order).
hipError_t launch_step(const Dev &d, hipStream_t st, hipEvent_t *ev)
{
    auto mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], st);
    };
    mark(0);
    unsigned gu = blocks_for(d.cap, kUT);
    if (gu > 16384) gu = 16384;
    if (d.upd_blocks > 0) gu = (unsigned)d.upd_blocks;
    if (d.xcd_remap) gu = (gu + 7u) & ~7u;     // workgroups past the last tile find no work
    const bool aux = d.P.debug || d.P.trace;
    const bool ins = d.n_qlanes > 0;
    void (*ku)(Dev);
    if (d.closures || d.junctions)
        ku = d.mode == 1 ? (aux ? update_variant<1, true, true>(ins) : update_variant<1, false, true>(ins))
                         : (aux ? update_variant<0, true, true>(ins) : update_variant<0, false, true>(ins));
    else
        ku = d.mode == 1 ? (aux ? update_variant<1, true, false>(ins) : update_variant<1, false, false>(ins))
                         : (aux ? update_variant<0, true, false>(ins) : update_variant<0, false, false>(ins));
    // insertion: one more workgroup per kUT queue lanes
    const unsigned gi = ins ? (unsigned)((d.n_qlanes + kUT - 1) / kUT) : 0u;
    hipLaunchKernelGGL(ku, dim3(gu + gi), dim3(kUT), 0, st, d);
    mark(1);
    // with one scan block the apply kernel needs no block sums (its prefix
    // over earlier blocks is empty), so the reduction is not launched
    const unsigned gs = blocks_for(d.n_lanes, kScanLanes);
    if (gs > 1)
        hipLaunchKernelGGL(k_scan_reduce, dim3(gs), dim3(kScanThreads), 0, st, d);
    mark(2);
    hipLaunchKernelGGL(k_scan_apply, dim3(gs), dim3(kScanThreads), 0, st, d);
    mark(3);
    unsigned gj = blocks_for((long long)d.cap / kUpdateRows + 1, 4);
    if (gj > 2048) gj = 2048;
    if (d.jsc_blocks > 0) gj = (unsigned)d.jsc_blocks;
    hipLaunchKernelGGL(k_jscatter, dim3(gj), dim3(256), 0, st, d);
    mark(4);
    unsigned gm = (unsigned)(d.cap / kMC + d.n_lanes / kMergeLanes + 1);
    if (d.xcd_remap) gm = (gm + 7u) & ~7u;     // chunks past the last one return at once
    hipLaunchKernelGGL(k_merge, dim3(gm), dim3(kMT), 0, st, d);
    mark(5);
    if (d.junctions)
        hipLaunchKernelGGL(k_yield, dim3(blocks_for(d.n_lanes, 256)), dim3(256), 0, st, d,
                           (const int32_t *)d.ls_new);
    mark(6);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_mlp_pack(Dev d)
{
    mlp_pack(*static_cast<MlpLds *>(const_cast<void *>(d.mlp_pack)), d.mlp_theta, d.mlp_norm);
}

size_t mlp_pack_bytes() { return sizeof(MlpLds); }

__global__ void k_lane_patch(Dev d, const int32_t *idx, const LaneInfo *rec, int32_t n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int l = idx[i];
    const_cast<LaneInfo *>(d.lanes)[l] = rec[i];
    at(d.lane_red, l) = lane_flags_at(rec[i], (uint32_t)*d.t);
}

__global__ void k_road_patch(Dev d, const int32_t *idx, const RoadInfo *rec, int32_t n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        const_cast<RoadInfo *>(d.roads)[idx[i]] = rec[i];
}

hipError_t launch_road_patch(const Dev &d, const int32_t *idx, const RoadInfo *rec, int32_t n,
                             hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL(k_road_patch, dim3(blocks_for(n, 256)), dim3(256), 0, st, d, idx, rec,
                           n);
    return hipGetLastError();
}

hipError_t launch_lane_patch(const Dev &d, const int32_t *idx, const LaneInfo *rec, int32_t n,
                             hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL(k_lane_patch, dim3(blocks_for(n, 256)), dim3(256), 0, st, d, idx, rec,
                           n);
    return hipGetLastError();
}

// Vehicles and mean speed per road of the current state: the rows of road r
// are those of its lanes, [ls[lane0], ls[lane0 + nlanes]); the speeds are
// summed in FP64 in row order.
__global__ void k_road_stats(Dev d, int32_t n_roads, int32_t *count, float *mean_v)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_roads)
        return;
    const RoadInfo rd = at(d.roads, r);
    const int a = at(d.ls_old, rd.lane0), b = at(d.ls_old, rd.lane0 + rd.nlanes);
    double sum = 0.0;
    for (int i = a; i < b; ++i)
        sum += (double)at(d.S.v, i);
    if (count)
        count[r] = b - a;
    if (mean_v)
        mean_v[r] = b > a ? (float)(sum / (double)(b - a)) : 0.0f;
}

// Position and heading of each state row: along the straight segment from
// the road's upstream node A to its downstream node B in proportion s / L,
// (k + 1/2) lane widths of 3.5 m to the right of the direction of travel.
// road_ab[r] = (Ax, Ay, Bx, By).
__global__ void k_positions(Dev d, int32_t n, const double4 *road_ab, double *x, double *y,
                            double *heading)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const LaneInfo li = at(d.lanes, d.S.lane[i]);
    const double4 ab = road_ab[li.road];
    const double dx = ab.z - ab.x, dy = ab.w - ab.y;
    const double len = sqrt(dx * dx + dy * dy);
    const double ux = len > 0.0 ? dx / len : 1.0, uy = len > 0.0 ? dy / len : 0.0;
    const double f = (double)at(d.S.s, i) / (double)li.L;
    const double off = ((double)li.k + 0.5) * 3.5;
    x[i] = ab.x + dx * f + uy * off;
    y[i] = ab.y + dy * f - ux * off;
    heading[i] = atan2(dy, dx);
}

hipError_t launch_road_stats(const Dev &d, int32_t n_roads, int32_t *count, float *mean_v,
                             hipStream_t st)
{
    if (n_roads > 0)
        hipLaunchKernelGGL(k_road_stats, dim3(blocks_for(n_roads, 256)), dim3(256), 0, st, d,
                           n_roads, count, mean_v);
    return hipGetLastError();
}

hipError_t launch_positions(const Dev &d, int32_t n, const double *road_ab, double *x,
                            double *y, double *heading, hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL(k_positions, dim3(blocks_for(n, 256)), dim3(256), 0, st, d, n,
                           (const double4 *)road_ab, x, y, heading);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(const Dev &d, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_yield(const Dev &d, hipStream_t st)
{
    hipLaunchKernelGGL(k_yield, dim3(blocks_for(d.n_lanes, 256)), dim3(256), 0, st, d, d.ls_old);
    return hipGetLastError();
}

hipError_t launch_tails(const Dev &d, hipStream_t st)
{
    hipLaunchKernelGGL(k_tails, dim3(blocks_for(d.n_lanes, 256)), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_trips(const Dev &d, int32_t n_act, int32_t *status, int32_t *travel,
                        double *dist, hipStream_t st)
{
    if (d.n_veh > 0)
        hipLaunchKernelGGL(k_trips_all, dim3(blocks_for(d.n_veh, 256)), dim3(256), 0, st, d,
                           status, travel, dist);
    if (n_act > 0)
        hipLaunchKernelGGL(k_trips_active, dim3(blocks_for(n_act, 256)), dim3(256), 0, st, d,
                           n_act, status, travel, dist);
    return hipGetLastError();
}

hipError_t launch_cursor(const Dev &d, const uint32_t *ids, const uint32_t *ptrs, int32_t *out,
                         int32_t n, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_cursor, dim3(blocks_for(n, 256)), dim3(256), 0, st, d, ids, ptrs, out, n);
    return hipGetLastError();
}

}  // namespace moss

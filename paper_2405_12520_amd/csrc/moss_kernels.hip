// Kernels of one simulation step on gfx950.
//
// A step is the paper's two-phase iteration (Sec. III-A):
//   update  - k_insert, k_update: every vehicle reads only the state S the
//             step started from (the read-only copy) and writes a proposal
//             (new position, speed, lane, route index) to its own row of Pr;
//   prepare - k_scan_*, k_jscatter, k_merge: the proposals are re-ordered per
//             lane into the next state S (the spatial index of the next step).
// No kernel writes what another thread of the same kernel reads, so the
// result does not depend on thread scheduling; atomics only count and
// allocate slots, and every order they create is re-sorted by (position, id).
//
// Arithmetic is FP32 in the source order, compiled without contraction, so
// that decisions (leaders, lane changes, lanes) reproduce bit for bit.
#include "moss_internal.h"

namespace moss {

__device__ __forceinline__ float fmin32(float x, float y) { return x < y ? x : y; }
__device__ __forceinline__ float fmax32(float x, float y) { return x > y ? x : y; }

// IDM acceleration (Treiber, Hennecke, Helbing 2000), exponent 4.  Without a
// leader only the free-road term a(1 - (v/v0)^4) remains; a non-positive gap
// returns the braking limit.
__device__ __forceinline__ float idm(const Params &P, float v, float v0e, bool has, float vl,
                                     float gap)
{
    float r = v / v0e;
    float r2 = r * r;
    float r4 = r2 * r2;
    float free_term = 1.0f - r4;
    if (!has)
        return P.a_max * free_term;
    if (gap <= 0.0f)
        return -P.b_max;
    float dv = v - vl;
    float t1 = v * P.T;
    float t2 = (v * dv) / P.two_sqrt_ab;
    float tt = t1 + t2;
    float ss = P.s0 + (tt > 0.0f ? tt : 0.0f);
    float q = ss / gap;
    return P.a_max * (free_term - q * q);
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

struct Lead {
    bool has;
    float v, gap;
    uint32_t id;
};

// Leader beyond the lane end: follow the route for at most h_look roads while
// the distance covered is within d_look; on each road take lane min(k, n-1)
// and use its last vehicle (lane tail).  A vehicle never leads itself.
__device__ Lead lookahead(const Dev &d, const LaneInfo &li, float s, uint32_t id, uint32_t ptr,
                          int32_t nxt)
{
    Lead r = {false, 0.0f, 0.0f, kNone};
    float dist = li.L - s;
    int kk = li.k;
    uint32_t p = ptr;
    int32_t nr = nxt;
    for (int h = 0; h < d.P.h_look; ++h) {
        if (nr < 0)
            break;
        if (dist > d.P.d_look)
            break;
        RoadInfo rd = d.roads[nr];
        if (kk > rd.nlanes - 1)
            kk = rd.nlanes - 1;
        Tail tl = d.tails[rd.lane0 + kk];
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
        nr = d.route[p + 1];
    }
    return r;
}

__device__ __forceinline__ int find_vehicle(const Dev &d, uint32_t id)
{
    int lo = 0, hi = d.n_veh;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (d.vt_id[mid] < id)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// ----------------------------------------------------------------- insert --

// Head of each origin-lane queue enters when due, if the lane is empty or the
// gap behind its last vehicle is at least s0 + v T for the entry speed
// v = min(v0, limit, speed of that vehicle); it joins the lane at s = 0 at
// the end of the step.
__global__ void k_insert(Dev d)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.n_qlanes)
        return;
    const int l = d.qlanes[q];
    const int h = d.q_head[l];
    if (h >= d.q_end[l])
        return;
    const int64_t t = *d.t;
    if ((int64_t)d.q_dep[h] > t)
        return;
    const Params &P = d.P;
    const LaneInfo li = d.lanes[l];
    float v0e = fmin32(d.q_v0[h], li.vlim);
    int lo = d.ls_old[l], hi = d.ls_old[l + 1];
    bool ok;
    float vins;
    if (lo == hi) {
        ok = true;
        vins = v0e;
    } else {
        vins = fmin32(v0e, d.S.v[lo]);
        ok = (d.S.s[lo] - P.len) >= (P.s0 + vins * P.T);
    }
    unsigned long long *c = d.cnt + (size_t)li.scen * C_N;
    if (!ok) {
        atomicAdd(c + C_INSERT_FAIL, 1ull);
        return;
    }
    uint32_t slot = (uint32_t)(*d.n_cur) + atomicAdd(d.n_ins, 1u);
    d.Pr.s[slot] = 0.0f;
    d.Pr.v[slot] = vins;
    d.Pr.a[slot] = 0.0f;
    d.Pr.id[slot] = d.q_id[h];
    d.Pr.lane[slot] = (uint32_t)l | kJoinBit;
    d.Pr.ptr[slot] = d.q_ptr[h];
    d.Pr.next[slot] = d.q_next[h];
    d.Pr.v0[slot] = d.q_v0[h];
    d.jrank[slot] = (uint32_t)atomicAdd(d.jcount + l, 1);
    d.jlist[atomicAdd(d.n_join, 1u)] = slot;
    d.q_head[l] = h + 1;
    atomicAdd(c + C_INSERTED, 1ull);
}

// ----------------------------------------------------------------- update --

__global__ void __launch_bounds__(256) k_update(Dev d)
{
    const int n = *d.n_cur;
    const int64_t t = *d.t;
    const Params &P = d.P;
    const uint32_t tt = (uint32_t)t;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t l = d.S.lane[i];
        const LaneInfo li = d.lanes[l];
        const float s = d.S.s[i], v = d.S.v[i];
        const uint32_t id = d.S.id[i], ptr = d.S.ptr[i];
        const int32_t nxt = d.S.next[i];
        const float v0 = d.S.v0[i];
        const int lo = d.ls_old[l], hi = d.ls_old[l + 1];
        const float L = li.L;
        int32_t flags = 0;
        float margin = 0.0f;
        uint32_t tl_id = kNone, tf_id = kNone;

        // red light at the stop line, applied if the vehicle can still stop
        bool red = false;
        if (nxt >= 0 && li.sig >= 0) {
            SigInfo g = d.sigs[li.sig];
            uint32_t ph = ((tt + (uint32_t)g.offset) % (uint32_t)g.cycle) / (uint32_t)g.phase;
            if ((int)ph != g.group) {
                float stop_dist = (v * v) / (2.0f * P.b_max);
                if (L - s >= stop_dist)
                    red = true;
            }
        }

        const int Lc = (i + 1 < hi) ? i + 1 : -1;
        const int o = (i - 1 >= lo) ? i - 1 : -1;

        // randomised MOBIL on one side per step (even: k-1, odd: k+1)
        bool change = false;
        int lt = -1, Lt = -1, nb = -1;
        if (s >= 0.0f) {
            int kt = ((t & 1) == 0) ? li.k - 1 : li.k + 1;
            if (kt >= 0 && kt < li.nlanes) {
                lt = li.lane0 + kt;
                const int a0 = d.ls_old[lt], a1 = d.ls_old[lt + 1];
                int lo2 = a0, hi2 = a1;
                while (lo2 < hi2) {
                    int mid = (lo2 + hi2) >> 1;
                    if (d.S.s[mid] >= s)
                        hi2 = mid;
                    else
                        lo2 = mid + 1;
                }
                Lt = lo2 < a1 ? lo2 : -1;
                nb = lo2 - 1 >= a0 ? lo2 - 1 : -1;
                const float vlim_c = li.vlim, vlim_t = d.lanes[lt].vlim;
                const float v0e_c = fmin32(v0, vlim_c), v0e_t = fmin32(v0, vlim_t);
                float sLc = 0.0f, vLc = 0.0f, sLt = 0.0f, vLt = 0.0f;
                if (Lc >= 0) { sLc = d.S.s[Lc]; vLc = d.S.v[Lc]; }
                if (Lt >= 0) { sLt = d.S.s[Lt]; vLt = d.S.v[Lt]; }
                float a_c = Lc >= 0 ? idm(P, v, v0e_c, true, vLc, (sLc - P.len) - s)
                                    : idm(P, v, v0e_c, false, 0.0f, 0.0f);
                float at_c = Lt >= 0 ? idm(P, v, v0e_t, true, vLt, (sLt - P.len) - s)
                                     : idm(P, v, v0e_t, false, 0.0f, 0.0f);
                float d_o = 0.0f, d_n = 0.0f;
                bool safe = true;
                if (o >= 0) {
                    const float vo = d.S.v[o], so = d.S.s[o];
                    const float v0e_o = fmin32(d.S.v0[o], vlim_c);
                    float a_o = idm(P, vo, v0e_o, true, v, (s - P.len) - so);
                    float at_o = Lc >= 0 ? idm(P, vo, v0e_o, true, vLc, (sLc - P.len) - so)
                                         : idm(P, vo, v0e_o, false, 0.0f, 0.0f);
                    d_o = at_o - a_o;
                }
                if (nb >= 0) {
                    const float vn = d.S.v[nb], sn = d.S.s[nb];
                    const float v0e_n = fmin32(d.S.v0[nb], vlim_t);
                    float a_n = Lt >= 0 ? idm(P, vn, v0e_n, true, vLt, (sLt - P.len) - sn)
                                        : idm(P, vn, v0e_n, false, 0.0f, 0.0f);
                    float at_n = idm(P, vn, v0e_n, true, v, (s - P.len) - sn);
                    d_n = at_n - a_n;
                    float gap_b = (s - P.len) - sn;
                    if (!(gap_b > 0.0f)) safe = false;
                    if (!(at_n >= -P.b_safe)) safe = false;
                }
                if (Lt >= 0) {
                    float gap_f = (sLt - P.len) - s;
                    if (!(gap_f > 0.0f)) safe = false;
                }
                float inc = (at_c - a_c) + P.pol * (d_n + d_o);
                uint32_t x0 = philox_x0(tt, id, 0u, 0u, P.key0, P.key1);
                float u = (float)(x0 >> 8) * (1.0f / 16777216.0f);
                change = safe && inc > P.a_thr && u < P.p_lc;
                margin = inc - P.a_thr;
                flags |= change ? 2 : 1;
                if (Lt >= 0) tl_id = d.S.id[Lt];
                if (nb >= 0) tf_id = d.S.id[nb];
            }
        }

        // car-following in the final lane
        const int lf = change ? lt : (int)l;
        const LaneInfo lif = change ? d.lanes[lf] : li;
        const int lead = change ? Lt : Lc;
        Lead ld;
        if (lead >= 0) {
            ld.has = true;
            ld.v = d.S.v[lead];
            ld.gap = (d.S.s[lead] - P.len) - s;
            ld.id = d.S.id[lead];
        } else {
            ld = lookahead(d, lif, s, id, ptr, nxt);
            if (ld.has) flags |= 8;
        }
        const float v0e = fmin32(v0, lif.vlim);
        float acc = idm(P, v, v0e, ld.has, ld.v, ld.gap);
        if (red) {
            float acc_red = idm(P, v, v0e, true, 0.0f, L - s);
            acc = fmin32(acc, acc_red);
            flags |= 4;
        }
        const float a = fmax32(-P.b_max, acc);

        // Newton's equations over one step, stopping at v = 0
        float vn = v + a * P.dt;
        float dx;
        if (vn < 0.0f) {
            dx = -((v * v) / (2.0f * a));
            vn = 0.0f;
        } else {
            dx = v * P.dt + (0.5f * a) * (P.dt * P.dt);
        }
        float sp = s + dx;

        // transfer along the route, arrival at the end of the last road
        int x = lf;
        uint32_t p = ptr;
        int32_t nr = nxt;
        int kk = lif.k;
        float Lx = lif.L;
        while (sp >= Lx && nr >= 0) {
            sp = sp - Lx;
            p += 1;
            RoadInfo rd = d.roads[nr];
            if (kk > rd.nlanes - 1)
                kk = rd.nlanes - 1;
            x = rd.lane0 + kk;
            Lx = rd.L;
            nr = d.route[p + 1];
        }
        const bool arrived = sp >= Lx;
        if (!(isfinite(sp) && isfinite(vn)))
            atomicOr(d.err, 2u);

        unsigned long long *c = d.cnt + (size_t)li.scen * C_N;
        uint32_t plane;
        if (arrived) {
            plane = kArrived;
            flags |= 16;
            int vi = find_vehicle(d, id);
            atomicAdd(c + C_ARRIVED, 1ull);
            atomicAdd(c + C_TRIP_TIME, (unsigned long long)((t + 1) - (int64_t)d.vt_dep[vi]));
        } else if (x == (int)l && p == ptr) {
            plane = l;
            atomicAdd(d.scount + l, 1);
        } else {
            plane = (uint32_t)x | kJoinBit;
            d.jrank[i] = (uint32_t)atomicAdd(d.jcount + x, 1);
            d.jlist[atomicAdd(d.n_join, 1u)] = (uint32_t)i;
        }
        if (change)
            atomicAdd(c + C_LANE_CHANGES, 1ull);
        d.Pr.s[i] = sp;
        d.Pr.v[i] = vn;
        d.Pr.a[i] = a;
        d.Pr.id[i] = id;
        d.Pr.lane[i] = plane;
        d.Pr.ptr[i] = p;
        d.Pr.next[i] = nr;
        d.Pr.v0[i] = v0;
        if (P.debug) {
            d.d_id[i] = id;
            d.d_leader[i] = ld.id;
            d.d_flags[i] = flags;
            d.d_margin[i] = margin;
            d.d_tl[i] = tl_id;
            d.d_tf[i] = tf_id;
        }
    }
}

// --------------------------------------------------------- lane-count scan --

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanLanes = kScanThreads * kScanPer;

// inclusive scan of two ints over a 256-thread block
__device__ void block_scan2(int &x, int &y, int *sh)
{
    const int tid = threadIdx.x;
    sh[tid] = x;
    sh[kScanThreads + tid] = y;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int ax = 0, ay = 0;
        if (tid >= off) {
            ax = sh[tid - off];
            ay = sh[kScanThreads + tid - off];
        }
        __syncthreads();
        sh[tid] += ax;
        sh[kScanThreads + tid] += ay;
        __syncthreads();
    }
    x = sh[tid];
    y = sh[kScanThreads + tid];
    __syncthreads();
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(Dev d)
{
    __shared__ int sh[2 * kScanThreads];
    const int base = blockIdx.x * kScanLanes + threadIdx.x * kScanPer;
    int tot = 0, tj = 0;
    for (int q = 0; q < kScanPer; ++q) {
        int l = base + q;
        if (l < d.n_lanes) {
            int j = d.jcount[l];
            tot += d.scount[l] + j;
            tj += j;
        }
    }
    block_scan2(tot, tj, sh);
    if (threadIdx.x == kScanThreads - 1) {
        d.blk[2 * blockIdx.x] = tot;
        d.blk[2 * blockIdx.x + 1] = tj;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(Dev d)
{
    __shared__ int sh[2 * kScanThreads];
    const int b = blockIdx.x;
    int off = 0, offj = 0;
    for (int q = threadIdx.x; q < b; q += kScanThreads) {
        off += d.blk[2 * q];
        offj += d.blk[2 * q + 1];
    }
    block_scan2(off, offj, sh);
    __shared__ int base_tot, base_j;
    if (threadIdx.x == kScanThreads - 1) {
        base_tot = off;
        base_j = offj;
    }
    __syncthreads();
    const int b0 = base_tot, bj = base_j;
    const int base = b * kScanLanes + threadIdx.x * kScanPer;
    int cnt[kScanPer], jc[kScanPer];
    int tot = 0, tj = 0;
    for (int q = 0; q < kScanPer; ++q) {
        int l = base + q;
        cnt[q] = 0;
        jc[q] = 0;
        if (l < d.n_lanes) {
            jc[q] = d.jcount[l];
            cnt[q] = d.scount[l] + jc[q];
        }
        tot += cnt[q];
        tj += jc[q];
    }
    int inc = tot, incj = tj;
    block_scan2(inc, incj, sh);
    int run = b0 + inc - tot, runj = bj + incj - tj;
    for (int q = 0; q < kScanPer; ++q) {
        int l = base + q;
        if (l < d.n_lanes) {
            d.ls_new[l] = run;
            d.joff[l] = runj;
            d.scount[l] = 0;
            d.jcount[l] = 0;
        }
        run += cnt[q];
        runj += jc[q];
    }
    if (b == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) {
        d.ls_new[d.n_lanes] = run;
        d.joff[d.n_lanes] = runj;
        *d.n_next = run;
    }
}

// ----------------------------------------------------- joiners by lane --

__global__ void k_jscatter(Dev d)
{
    const int n = (int)*d.n_join;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint32_t p = d.jlist[i];
        uint32_t x = d.Pr.lane[p] & ~kJoinBit;
        d.jidx[d.joff[x] + d.jrank[p]] = p;
    }
}

// ------------------------------------------------------------------ merge --

__device__ __forceinline__ bool key_less(const Dev &d, uint32_t a, uint32_t b)
{
    float sa = d.Pr.s[a], sb = d.Pr.s[b];
    if (sa != sb)
        return sa < sb;
    return d.Pr.id[a] < d.Pr.id[b];
}

// One thread per lane: stayers keep their order, joiners are sorted by
// (s, id) and merged in, then overlaps are removed from the lane head
// backwards (a follower is put one vehicle length behind its leader and
// takes the leader's speed if faster).
__global__ void __launch_bounds__(256) k_merge_lane(Dev d)
{
    __shared__ double s_sum[256];
    __shared__ unsigned long long s_cnt[256], s_clamp[256];
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    double vsum = 0.0;
    unsigned long long count = 0, clamps = 0;
    if (l < d.n_lanes) {
        const int o0 = d.ls_old[l], o1 = d.ls_old[l + 1];
        const int j0 = d.joff[l], j1 = d.joff[l + 1];
        const int w0 = d.ls_new[l], w1 = d.ls_new[l + 1];
        for (int a = j0 + 1; a < j1; ++a) {
            uint32_t xk = d.jidx[a];
            int b = a - 1;
            while (b >= j0 && key_less(d, xk, d.jidx[b])) {
                d.jidx[b + 1] = d.jidx[b];
                --b;
            }
            d.jidx[b + 1] = xk;
        }
        int ip = o0, jp = j0, w = w0;
        for (;;) {
            while (ip < o1 && d.Pr.lane[ip] != (uint32_t)l)
                ++ip;
            const bool hs = ip < o1, hj = jp < j1;
            if (!hs && !hj)
                break;
            if (w >= w1) {          // counts disagree with the scan: never write past the lane
                atomicOr(d.err, 1u);
                break;
            }
            uint32_t src;
            if (hs && (!hj || key_less(d, (uint32_t)ip, d.jidx[jp])))
                src = (uint32_t)ip++;
            else
                src = d.jidx[jp++];
            d.S.s[w] = d.Pr.s[src];
            d.S.v[w] = d.Pr.v[src];
            d.S.a[w] = d.Pr.a[src];
            d.S.id[w] = d.Pr.id[src];
            d.S.lane[w] = (uint32_t)l;
            d.S.ptr[w] = d.Pr.ptr[src];
            d.S.next[w] = d.Pr.next[src];
            d.S.v0[w] = d.Pr.v0[src];
            ++w;
        }
        if (w != w1)
            atomicOr(d.err, 1u);
        for (int f = w1 - 2; f >= w0; --f) {
            float lim = d.S.s[f + 1] - d.P.len;
            if (d.S.s[f] > lim) {
                d.S.s[f] = lim;
                d.S.v[f] = fmin32(d.S.v[f], d.S.v[f + 1]);
                ++clamps;
            }
        }
        Tail tl;
        tl.pad = 0;
        if (w1 > w0) {
            tl.s = d.S.s[w0];
            tl.v = d.S.v[w0];
            tl.id = d.S.id[w0];
        } else {
            tl.s = 0.0f;
            tl.v = 0.0f;
            tl.id = kNone;
        }
        d.tails[l] = tl;
        for (int f = w0; f < w1; ++f)
            vsum += (double)d.S.v[f];
        count = (unsigned long long)(w1 - w0);
    }
    // reduce per block when all its lanes belong to one scenario
    const int lfirst = blockIdx.x * blockDim.x;
    const int llast = min(lfirst + (int)blockDim.x, d.n_lanes) - 1;
    const int sc0 = d.lanes[lfirst].scen;
    if (sc0 == d.lanes[llast].scen) {
        s_sum[threadIdx.x] = vsum;
        s_cnt[threadIdx.x] = count;
        s_clamp[threadIdx.x] = clamps;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) {
                s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
                s_cnt[threadIdx.x] += s_cnt[threadIdx.x + off];
                s_clamp[threadIdx.x] += s_clamp[threadIdx.x + off];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            unsigned long long *c = d.cnt + (size_t)sc0 * C_N;
            if (s_cnt[0]) atomicAdd(c + C_VEH_STEPS, s_cnt[0]);
            if (s_clamp[0]) atomicAdd(c + C_CLAMPS, s_clamp[0]);
            if (s_cnt[0]) atomicAdd(d.sumv + sc0, s_sum[0]);
        }
    } else if (l < d.n_lanes) {
        const int sc = d.lanes[l].scen;
        unsigned long long *c = d.cnt + (size_t)sc * C_N;
        if (count) atomicAdd(c + C_VEH_STEPS, count);
        if (clamps) atomicAdd(c + C_CLAMPS, clamps);
        if (count) atomicAdd(d.sumv + sc, vsum);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *d.n_dbg = *d.n_cur;
        *d.n_cur = *d.n_next;
        *d.n_ins = 0u;
        *d.n_join = 0u;
        *d.t = *d.t + 1;
    }
}

// -------------------------------------------------------------- utilities --

__global__ void k_tails(Dev d)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= d.n_lanes)
        return;
    const int w0 = d.ls_old[l], w1 = d.ls_old[l + 1];
    Tail tl;
    tl.pad = 0;
    if (w1 > w0) {
        tl.s = d.S.s[w0];
        tl.v = d.S.v[w0];
        tl.id = d.S.id[w0];
    } else {
        tl.s = 0.0f;
        tl.v = 0.0f;
        tl.id = kNone;
    }
    d.tails[l] = tl;
}

__global__ void k_cursor(Dev d, const uint32_t *ids, const uint32_t *ptrs, int32_t *out, int32_t n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int vi = find_vehicle(d, ids[i]);
    out[i] = (int32_t)(ptrs[i] - d.vt_rstart[vi]);
}

static inline unsigned blocks_for(long long n, int per)
{
    long long b = (n + per - 1) / per;
    return (unsigned)(b < 1 ? 1 : b);
}

static const char *const kStepKernels[] = {"k_insert", "k_update", "k_scan_reduce",
                                            "k_scan_apply", "k_jscatter", "k_merge_lane"};

int step_kernel_count() { return (int)(sizeof kStepKernels / sizeof kStepKernels[0]); }
const char *step_kernel_name(int i)
{
    return (i >= 0 && i < step_kernel_count()) ? kStepKernels[i] : nullptr;
}

// Enqueues one step.  With ev != nullptr, ev[0] is recorded before the first
// kernel and ev[k+1] after kernel k (in kStepKernels order).
hipError_t launch_step(const Dev &d, hipStream_t st, hipEvent_t *ev)
{
    auto mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], st);
    };
    mark(0);
    if (d.n_qlanes > 0)
        hipLaunchKernelGGL(k_insert, dim3(blocks_for(d.n_qlanes, 256)), dim3(256), 0, st, d);
    mark(1);
    unsigned gu = blocks_for(d.cap, 256);
    if (gu > 16384) gu = 16384;
    hipLaunchKernelGGL(k_update, dim3(gu), dim3(256), 0, st, d);
    mark(2);
    const unsigned gs = blocks_for(d.n_lanes, kScanLanes);
    hipLaunchKernelGGL(k_scan_reduce, dim3(gs), dim3(kScanThreads), 0, st, d);
    mark(3);
    hipLaunchKernelGGL(k_scan_apply, dim3(gs), dim3(kScanThreads), 0, st, d);
    mark(4);
    unsigned gj = blocks_for((long long)d.cap + d.n_lanes, 256);
    if (gj > 4096) gj = 4096;
    hipLaunchKernelGGL(k_jscatter, dim3(gj), dim3(256), 0, st, d);
    mark(5);
    hipLaunchKernelGGL(k_merge_lane, dim3(blocks_for(d.n_lanes, 256)), dim3(256), 0, st, d);
    mark(6);
    return hipGetLastError();
}

hipError_t launch_tails(const Dev &d, hipStream_t st)
{
    hipLaunchKernelGGL(k_tails, dim3(blocks_for(d.n_lanes, 256)), dim3(256), 0, st, d);
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

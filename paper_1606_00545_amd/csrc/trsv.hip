// Level-scheduled triangular solves (Sec. 2.6, Alg. 3), as one persistent
// launch per triangle in which rows of successive levels are solved inside a
// workgroup with their dependencies held in LDS.
//
// Plan (built once per factor on the host by plan.hpp's make_plan):
//  * the rows are cut into parts: x-y tiles spanning all z for a recognised
//    grid stencil, otherwise contiguous row ranges, numbered in the order the
//    triangle is solved. Every dependency of a row lies in its own part or in an
//    earlier part, so the parts can be claimed in order from a ticket counter:
//    a part only ever waits for parts already claimed by running workgroups,
//    hence no deadlock at any occupancy or grid size;
//  * inside a part the rows are laid out by (level, row) (Alg. 3's order) and
//    cut into sub-segments of at most 64 rows of one level.
//
// Execution (k_trsv_blk): one workgroup per part: solver wavefronts (one by
// default), a writer wavefront and prefetching wavefronts.
//  * Prefetchers stream the next sub-segments into a ring of LDS slots: the
//    right-hand side (gathered by row, or read in plan order for the upper
//    solve of an L-then-U chain), the row's entries, and the values of
//    dependencies in earlier parts, polled from global memory until final;
//  * the solver takes sub-segments in order, reads dependencies inside the part
//    from a small LDS ring of recent results and dependencies outside it from
//    the slot, and publishes each result to the polled copy (below). It never
//    waits on global memory itself;
//  * the writer copies the part's results from the polled copy to the outputs
//    by row or in the other triangle's order, scattered stores kept off the
//    solver's path.
//  * Every wait is bounded: a wave that has polled `spin` times (the limit set by
//    hec_set_spin_limit) gives up, records the failure in the schedule's error
//    word and in its workgroup's abort flag, and every wave then leaves its loops
//    and the launch ends normally, with garbage in its outputs; the host reports
//    the failure (HEC_ERR_TIMEOUT) at its next synchronisation. Only a broken plan,
//    a lost store or a misuse (two streams on one schedule) can get there.
//  * Readiness of a value across parts is the value itself: each triangle
//    keeps an internal copy of its results in plan order, pre-filled with a
//    signalling-NaN bit pattern that arithmetic never produces; results are
//    stored to it and polled from it with device-coherent (agent scope)
//    accesses, so only single-location coherence is needed and no cache-wide
//    fence is issued. A sub-segment's results are 64 consecutive positions, so
//    these stores are whole cache lines; the outputs by row (or in the other
//    triangle's order) are plain stores. In an L-then-U chain the lower launch
//    fills the upper solve's copy and the upper launch refills the lower one
//    for the next chain, so the chain is exactly two launches.
#include <algorithm>
#include <climits>
#include <cmath>
#include <type_traits>

#include "hec_internal.hpp"

namespace hec {

namespace {

constexpr int kWaves = 16;  // solver wavefronts first, then prefetching wavefronts, the writer last
constexpr int kWriterBatch = 8;  // sub-segments' worth of positions the writer copies at a time
constexpr int kBlkThreads = 64 * kWaves;
constexpr int kBatch = 8;           // entries loaded per batch by a prefetcher lane
using plan::kPad;
using plan::kSub;
using plan::align16;
using plan::ctrl_bytes;
using plan::ctrl_head;
using plan::lds_bytes;
using plan::Slot;

template <class T> struct Sentinel;
template <> struct Sentinel<double> {
    using U = unsigned long long;
    static constexpr U bits = 0x7FF4DEADBEEF1234ull;  // signalling NaN: never produced by arithmetic
    static constexpr U qnan = 0x7FF8000000000000ull;
};
template <> struct Sentinel<float> {
    using U = unsigned int;
    static constexpr U bits = 0x7FA0BEEFu;
    static constexpr U qnan = 0x7FC00000u;
};

template <class T>
__device__ __forceinline__ typename Sentinel<T>::U load_coherent(const T *p) {
    using U = typename Sentinel<T>::U;
    return __hip_atomic_load((U *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publishes a solved value. A right-hand side that carries the sentinel's own
// bit pattern (and reaches the output untouched by arithmetic) is replaced by
// a quiet NaN, so no waiting row can mistake a final value for "not ready".
template <class T>
__device__ __forceinline__ void store_coherent(T *p, T v) {
    using U = typename Sentinel<T>::U;
    U u;
    __builtin_memcpy(&u, &v, sizeof(T));
    if (u == Sentinel<T>::bits) u = Sentinel<T>::qnan;
    __hip_atomic_store((U *)p, u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ T from_bits(typename Sentinel<T>::U u) {
    T v;
    __builtin_memcpy(&v, &u, sizeof(T));
    return v;
}

// Vectors of one triangular solve. b: right-hand side, read at bmap[q] for
// position q when bmap is given, else by row (b_by_row) or in plan order; xq:
// the results in plan order, the copy dependent rows poll (pre-filled with the
// sentinel); x: optional output by row; yother: optional output at the plan's
// per-position index (`other`, -1: not written) -- the other triangle's plan
// order, or a caller's vector; fill: a vector of nfill elements the kernel sets
// to the sentinel for the next solve (the polled copy of the other triangle of
// an L-then-U chain).
template <class T>
struct SolveIO {
    const T *b;
    const int32_t *bmap;
    int32_t b_by_row;
    T *xq, *x, *yother, *fill;
    int64_t nfill;
};

// Sets io.fill to the sentinel: a grid-stride loop at kernel start.
template <class T>
__device__ __forceinline__ void fill_sentinel(const SolveIO<T> &io) {
    if (!io.fill) return;
    const T s = from_bits<T>(Sentinel<T>::bits);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < io.nfill; i += (int64_t)gridDim.x * blockDim.x)
        io.fill[i] = s;
}

struct PlanArgs {
    int32_t nparts, K, ldq, W, D, S;  // S: most sub-segments in one part
    const int32_t *part_ss, *part_pos, *ss_pos, *ss_need, *grow, *other, *enc;
    uint32_t *err;  // the schedule's error word: set when a wait gives up
    uint32_t spin;  // polls a wait makes before it gives up
};

// Records a wait that gave up: the schedule's error word (read by the host).
__device__ __forceinline__ void record_timeout(uint32_t *err) {
    __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Another wave gave up somewhere on the device (checked now and then by long waits).
__device__ __forceinline__ bool timed_out(const uint32_t *err) {
    return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

// First poll of a dependency outside the part: only lanes whose entry has one
// load (a lane-masked load); the others get 0, which is never the sentinel. (A
// shared dummy address for those lanes would send a device-coherent load per
// wavefront and entry to one cache line from every compute unit: a hot spot that
// slows every access mapped to the same memory channel.)
template <class T>
__device__ __forceinline__ typename Sentinel<T>::U first_poll(const T *x, int e) {
    return e >= 0 ? load_coherent(x + e) : (typename Sentinel<T>::U)0;
}

template <class T, bool UPPER, int KC, int NS>
__global__ __launch_bounds__(kBlkThreads) void k_trsv_blk(PlanArgs P, const T *__restrict__ val,
                                                          const T *__restrict__ piv, SolveIO<T> io,
                                                          uint32_t *sync, const int32_t *skip) {
    using U = typename Sentinel<T>::U;
    constexpr U SENT = Sentinel<T>::bits;
    if (skip && *skip) return;  // uniform: no workgroup touches the counters
    fill_sentinel(io);
    T *const xq = io.xq;
    T *const x = io.x;
    T *const yother = io.yother;
    extern __shared__ __align__(16) char smem[];
    constexpr int NP = kWaves - NS - 1;
    const int D = P.D, K = P.K, W = P.W;
    int *done = (int *)smem;  // per solver wavefront: the next sub-segment it solves
    int *filled = done + plan::kMaxSolvers;
    int *s_part = filled + D;
    int *s_abort = s_part + 1;  // a wave of this workgroup gave up a wait
    const uint32_t zero_off = (uint32_t)(ctrl_head(D) - 16);
    int *sspos = (int *)(smem + ctrl_head(D));
    int *ssneed = (int *)(smem + ctrl_head(D) + plan::ss_bytes(P.S));
    const uint32_t sx_off = (uint32_t)ctrl_bytes(D, P.S, NS);
    T *sx = (T *)(smem + sx_off);
    const uint32_t slots_off = sx_off + (uint32_t)align16((size_t)W * sizeof(T));
    const Slot<T, UPPER> L{KC};
    const uint32_t sb = (uint32_t)L.bytes();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (threadIdx.x < 4) ((int *)(smem + zero_off))[threadIdx.x] = 0;
    if (threadIdx.x == 0) *s_abort = 0;
    // every slot's dependency addresses start at the zero word: a solver that gave up a
    // wait may still read the header of a slot that was never filled (the reads stay in
    // range; nothing it computes is published)
    for (int t = threadIdx.x; t < D * KC * kSub; t += blockDim.x)
        ((uint32_t *)(smem + slots_off + (t / (KC * kSub)) * sb + L.a()))[t % (KC * kSub)] = zero_off;
    // A wait that has spun `spin` times gives up: it marks the workgroup and the device.
    // Waves of the workgroup see the mark within 64 polls; other workgroups' long polls
    // look at the device's error word as often.
    // (every calling lane stores the mark: callers are wave-uniform, so lane 0 may not be among them)
    auto give_up = [&]() {
        __hip_atomic_store(s_abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        record_timeout(P.err);
    };
    auto wg_aborted = [&]() { return __hip_atomic_load(s_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0; };
    // one more poll of a wait: true when the wait must stop (given up here or elsewhere).
    // Called in wave-uniform control flow only, so a wave stops as a whole; the answer
    // is made a scalar (read from the first lane) so that the compiler keeps the loops
    // and flags that depend on it uniform (scalar branches, no exec-mask bookkeeping)
    auto spun_out = [&](uint32_t &it, bool device_wide) {
        ++it;
        bool stop = it > P.spin;
        if (!stop && (it & 63) == 0) stop = wg_aborted() || (device_wide && timed_out(P.err));
        stop = __builtin_amdgcn_readfirstlane((int)stop) != 0;
        if (stop) give_up();
        return stop;
    };

    for (;;) {
        __syncthreads();
        if (*s_abort) break;  // uniform: read by every thread after the barrier
        if (threadIdx.x == 0) *s_part = (int)atomicAdd(&sync[0], 1u);
        if ((int)threadIdx.x < plan::kMaxSolvers) done[threadIdx.x] = (int)threadIdx.x < NS ? (int)threadIdx.x : INT_MAX;
        if ((int)threadIdx.x < D) filled[threadIdx.x] = -1;
        __syncthreads();
        const int p = *s_part;
        if (p >= P.nparts) break;
        const int kb = P.part_ss[p], nss = P.part_ss[p + 1] - kb, pos0 = P.part_pos[p];
        for (int t = threadIdx.x; t <= nss; t += blockDim.x) {
            sspos[t] = P.ss_pos[kb + t];
            if constexpr (NS > 1)
                if (t < nss) ssneed[t] = P.ss_need[kb + t];
        }
        __syncthreads();

        if (wave < NS) {
            // ---------------- solvers: one LDS round trip and KC fused multiply-adds per row.
            // Solver wavefront w takes the part's sub-segments w, w + NS, ...; with NS > 1 a
            // sub-segment first waits until every sub-segment below its dependency bound is
            // solved (the `done` counters), which orders its reads of the ring of results
            // after their writes. The next own sub-segment's header and dependency
            // addresses are read while the current one is computed (two register sets used
            // alternately), so the only dependent LDS access of a step is the read of its
            // dependencies' values.
            __builtin_amdgcn_s_setprio(3);
            struct Head {
                T b, d;
                int q0, cnt, need;
                uint32_t ad[KC];
            };
            const int w0 = wave;
            auto adv = [&](int sl) {  // slot of the next own sub-segment (NS <= D)
                sl += NS;
                return sl >= D ? sl - D : sl;
            };
            int ready = w0;  // own sub-segments below `ready` are known to be filled
            bool bail = false;  // a wait gave up: stop taking sub-segments
            // Waits until own sub-segment r (in slot sl) is filled; returns one past the
            // run of consecutive own filled sub-segments starting at r (at most 8 looked
            // at). Lane u reads the flag of own sub-segment r + u*NS, so the eight flags
            // take one LDS round trip; relaxed loads suffice: a slot's contents are
            // complete before its flag is written (the prefetcher waits for its LDS
            // writes first), LDS accesses of one wavefront complete in order, and the
            // signal fence keeps the compiler from moving slot reads above the check.
            auto scan = [&](int r, int sl) -> int {
                const int u = lane & 7, want = r + u * NS;
                int s2 = sl + u * NS;
                s2 -= D * (int)((unsigned)s2 / (unsigned)D);
                uint32_t it = 0;
                for (;;) {
                    const int f = __hip_atomic_load(&filled[s2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    const uint64_t m = __ballot(lane < 8 && want < nss && f == want);
                    const int ok = __builtin_ctzll(~m);  // own filled sub-segments r, r + NS, ... in a row
                    if (ok > 0) {
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        return r + ok * NS;
                    }
                    if (spun_out(it, false)) {
                        bail = true;
                        return r;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            };
            // With several solvers: waits until every sub-segment below `need` is solved.
            // done[v] only grows and holds the next sub-segment solver v takes, so all below
            // `need` are solved once every counter reaches it (unused counters hold
            // INT_MAX; lane v reads counter v & 7). Relaxed loads suffice as in scan.
            auto wait_need = [&](int need) {
                if constexpr (NS == 1) return;  // one solver: its own earlier sub-segments are solved
                const int v = lane & (plan::kMaxSolvers - 1);
                uint32_t it = 0;
                for (;;) {
                    const int dv = __hip_atomic_load(&done[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (__ballot(dv < need) == 0) break;
                    if (spun_out(it, false)) {
                        bail = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
            };
            auto load_head = [&](int r, int sl, Head &H) {
                const char *p2 = smem + slots_off + sl * sb;
                H.q0 = sspos[r];
                H.cnt = sspos[r + 1] - H.q0;
                H.need = 0;
                if constexpr (NS > 1) H.need = ssneed[r];
                H.b = ((const T *)(p2 + L.b()))[lane];
                H.d = (T)1;
                if constexpr (UPPER) H.d = ((const T *)(p2 + L.d()))[lane];
#pragma unroll
                for (int u = 0; u < KC; ++u) H.ad[u] = ((const uint32_t *)(p2 + L.a()))[u * kSub + lane];
            };
            // Two register sets fit the 128-VGPR budget of a 1024-thread workgroup for
            // rows of up to 64 bytes of values; longer rows load the next header after
            // the step instead (nxt is then cur).
            constexpr bool kPipe = KC * sizeof(T) <= 64;
            // One sub-segment: cur is loaded; nxt receives own sub-segment rel + NS.
            auto step = [&](int rel, int slot, Head &cur, Head &nxt) {
                const int nslot = adv(slot);
                const char *p2 = smem + slots_off + slot * sb;
                const bool pre = kPipe && rel + NS < ready;
                T acc = cur.b;
                // entries in chunks of at most 8 (bounds the live registers of long rows)
                constexpr int CH = KC < 8 ? KC : 8;
#pragma unroll
                for (int c0 = 0; c0 < KC; c0 += CH) {
                    T xv[CH], av[CH];
#pragma unroll
                    for (int u = 0; u < CH; ++u) av[u] = ((const T *)(p2 + L.v()))[(c0 + u) * kSub + lane];
                    if (c0 == 0) wait_need(cur.need);
#pragma unroll
                    for (int u = 0; u < CH; ++u) xv[u] = *(const T *)(smem + cur.ad[c0 + u]);
                    if (c0 == 0 && pre) load_head(rel + NS, nslot, nxt);
#pragma unroll
                    for (int u = 0; u < CH; ++u) acc -= av[u] * xv[u];
                }
                if constexpr (UPPER) acc = acc * cur.d;  // the pivot's reciprocal, formed by the prefetcher
                if (lane < cur.cnt && !bail) {  // (after a give-up nothing more is published)
                    sx[(cur.q0 - pos0 + lane) & (W - 1)] = acc;
                    store_coherent(xq + cur.q0 + lane, acc);
                }
                // publish: the results in the ring are readable and the slot is free. A lone
                // solver releases every 4 sub-segments (only prefetchers wait on it).
                if (NS > 1 || (rel & 3) == 3 || rel + NS >= nss) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    if (lane == 0) __hip_atomic_store(&done[w0], rel + NS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                if (kPipe && !pre && rel + NS < nss) {
                    ready = scan(rel + NS, nslot);
                    load_head(rel + NS, nslot, nxt);  // (after a give-up: read, never used)
                }
                return nslot;
            };
            int slot = w0 % D;
            if constexpr (kPipe) {
                // A give-up is looked at once per pair of steps: the data flow between the
                // two register sets stays the same on every path (a check between the
                // steps made the compiler copy one set into the other, measured 7% slower
                // on the 128^3 pair); the second step of a pair then publishes nothing.
                Head h0, h1;
                if (w0 < nss) {
                    ready = scan(w0, slot);
                    load_head(w0, slot, h0);
                }
                for (int rel = w0; rel < nss && !bail; rel += 2 * NS) {
                    slot = step(rel, slot, h0, h1);
                    if (rel + NS < nss) slot = step(rel + NS, slot, h1, h0);
                }
            } else {
                for (int rel = w0; rel < nss; rel += NS) {
                    if (rel >= ready) ready = scan(rel, slot);
                    if (bail) break;
                    Head h;
                    load_head(rel, slot, h);
                    slot = step(rel, slot, h, h);
                }
            }
            __builtin_amdgcn_s_setprio(0);
        } else if (wave == kWaves - 1) {
            // ---------------- writer: the part's results go to the outputs by row (x) and in the
            // other order (yother), read back from the polled copy, where a final value is
            // its own ready flag. The part's positions are consecutive; each lane takes
            // every 64th of kWriterBatch * 64 at a time, once the solvers' progress counters
            // have passed them.
            if (x || yother) {
                const int pend_part = P.part_pos[p + 1];
                constexpr int WB = kWriterBatch;
                for (int c = pos0; c < pend_part; c += WB * kSub) {
                    const int cend = min(c + WB * kSub, pend_part);
                    U v[WB];
                    int gi[WB], po[WB];
#pragma unroll
                    for (int k = 0; k < WB; ++k) {
                        const int q = c + k * kSub + lane;
                        const bool live = q < cend;
                        gi[k] = live && x ? P.grow[q] : -1;
                        po[k] = live && yother && P.other ? P.other[q] : -1;
                        v[k] = live ? SENT : (U)0;
                    }
                    bool quit = false;
                    uint32_t it = 0;
                    for (;;) {  // all sub-segments below the smallest counter are solved
                        int m = INT_MAX;
#pragma unroll
                        for (int u = 0; u < plan::kMaxSolvers; ++u)
                            m = min(m, __hip_atomic_load(&done[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                        if (sspos[min(m, nss)] >= cend) break;
                        if (spun_out(it, false)) {
                            quit = true;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                    if (quit) break;
                    bool pend = true;
                    it = 0;
                    while (pend) {  // the solvers' coherent stores may still be on their way
#pragma unroll
                        for (int k = 0; k < WB; ++k)
                            if (v[k] == SENT) v[k] = load_coherent(xq + c + k * kSub + lane);
                        bool mine = false;
#pragma unroll
                        for (int k = 0; k < WB; ++k) mine |= v[k] == SENT;
                        pend = __ballot(mine) != 0;  // uniform: the wave waits as a whole
                        if (pend && spun_out(it, true)) {
                            quit = true;
                            break;
                        }
                        if (pend) __builtin_amdgcn_s_sleep(2);
                    }
                    if (quit) break;
#pragma unroll
                    for (int k = 0; k < WB; ++k) {
                        const T r = from_bits<T>(v[k]);
                        if (gi[k] >= 0) x[gi[k]] = r;
                        if (po[k] >= 0) yother[po[k]] = r;
                    }
                }
            }
        } else {
            // ---------------- prefetchers: every lane of a slot is written (idle lanes get padding)
            // Each prefetching wavefront keeps two of its sub-segments in flight: while
            // the right-hand side and the polls of one are outstanding, the row data and
            // first entries of its next one (NP later) are already loading.
            // Only the LDS writes wait for the solver to release the slot.
            constexpr int B = KC < kBatch ? KC : kBatch;
            constexpr bool kPfPipe = KC == 4;  // two register sets fit the 128-VGPR budget for short rows only
            struct Pre {
                int q0, cnt, gi, po;
                T dd;
                int es[B];
                T vs[B];
            };
            auto issue = [&](int r, Pre &R) {  // everything indexed by position: one round trip
                R.q0 = sspos[r];
                R.cnt = sspos[r + 1] - R.q0;
                const bool live = lane < R.cnt;
                const int q = R.q0 + (live ? lane : 0);
                R.gi = live && io.b_by_row && !io.bmap ? P.grow[q] : 0;
                // upper: the reciprocal of u_ii (correctly rounded), so that the solver's
                // step multiplies instead of dividing; the result is within about one
                // rounding of the quotient
                R.dd = (T)1;
                if constexpr (UPPER) R.dd = live ? (T)1 / piv[q] : (T)1;
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    R.es[u] = kPad;
                    R.vs[u] = (T)0;
                    if (live && u < K) {
                        R.es[u] = P.enc[(size_t)u * P.ldq + q];
                        R.vs[u] = val[(size_t)u * P.ldq + q];
                    }
                }
            };
            // every lane polls all its entries at once; entries without an outside
            // dependency read a constant zero. A repeated poll reloads only the entries
            // still pending (a load per entry and lane that is already final, or that
            // has no outside dependency, was measured slower: 420 against 353 us for the
            // 128^3 pair, the extra device-coherent loads crowding the memory side)
            bool quit = false;  // a wait gave up: stop filling slots
            auto poll = [&](const int (&es)[B], U (&xs)[B]) {
                bool pend = false;
#pragma unroll
                for (int u = 0; u < B; ++u) pend |= xs[u] == SENT;
                uint32_t it = 0;
                while (__ballot(pend) != 0) {  // uniform: the wave polls as a whole
                    if (spun_out(it, true)) {
                        quit = true;
                        return;
                    }
                    __builtin_amdgcn_s_sleep(1);
#pragma unroll
                    for (int u = 0; u < B; ++u)
                        if (xs[u] == SENT) xs[u] = load_coherent(xq + es[u]);
                    pend = false;
#pragma unroll
                    for (int u = 0; u < B; ++u) pend |= xs[u] == SENT;
                }
            };
            // entries and dependency addresses (known before any poll completes)
            auto put = [&](char *sl, uint32_t so, int s0, const int (&es)[B], const T (&vs)[B]) {
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int s = s0 + u;
                    const uint32_t xe_at = so + (uint32_t)(L.xe() + (size_t)(s * kSub + lane) * sizeof(T));
                    uint32_t at = zero_off;  // padding: value 0 times a zero
                    if (es[u] >= 0) at = xe_at;
                    else if (es[u] != kPad) at = sx_off + (uint32_t)(((-1 - es[u]) & (W - 1)) * sizeof(T));
                    ((uint32_t *)(sl + L.a()))[s * kSub + lane] = at;
                    ((T *)(sl + L.v()))[s * kSub + lane] = vs[u];
                }
            };
            // the polled values of dependencies outside the part (other entries never read theirs)
            auto put_xe = [&](char *sl, int s0, const int (&es)[B], const U (&xs)[B]) {
#pragma unroll
                for (int u = 0; u < B; ++u)
                    if (es[u] >= 0) ((T *)(sl + L.xe()))[(s0 + u) * kSub + lane] = from_bits<T>(xs[u]);
            };
            auto process = [&](int rel, Pre &cur, Pre &nxt) {
                const int slot = rel % D;
                const uint32_t so = slots_off + slot * sb;
                char *sl = smem + so;
                const bool live = lane < cur.cnt;
                const int q = cur.q0 + (live ? lane : 0);
                const T bb = live ? io.b[io.bmap ? io.bmap[q] : io.b_by_row ? cur.gi : q] : (T)0;
                U xs[B];
#pragma unroll
                for (int u = 0; u < B; ++u) xs[u] = first_poll(xq, cur.es[u]);
                if (kPfPipe && rel + NP < nss) issue(rel + NP, nxt);
                // the slot's previous sub-segment, rel - D, must be solved; everything but the
                // outside values goes in before the polls, so that only those and the flag
                // follow the last poll
                const int prev = rel - D;
                if (prev >= 0) {
                    uint32_t it = 0;
                    while (__hip_atomic_load(&done[prev & (NS - 1)], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) <= prev) {
                        if (spun_out(it, false)) {
                            quit = true;
                            return;
                        }
                        __builtin_amdgcn_s_sleep(4);
                    }
                }
                put(sl, so, 0, cur.es, cur.vs);
                ((T *)(sl + L.b()))[lane] = bb;
                if constexpr (UPPER) ((T *)(sl + L.d()))[lane] = cur.dd;
                poll(cur.es, xs);
                if (quit) return;
                put_xe(sl, 0, cur.es, xs);
                for (int s0 = B; s0 < KC; s0 += B) {  // rows longer than one batch
                    int es[B];
                    T vs[B];
#pragma unroll
                    for (int u = 0; u < B; ++u) {
                        es[u] = kPad;
                        vs[u] = (T)0;
                        if (live && s0 + u < K) {
                            es[u] = P.enc[(size_t)(s0 + u) * P.ldq + q];
                            vs[u] = val[(size_t)(s0 + u) * P.ldq + q];
                        }
                    }
                    U xs2[B];
#pragma unroll
                    for (int u = 0; u < B; ++u) xs2[u] = first_poll(xq, es[u]);
                    put(sl, so, s0, es, vs);
                    poll(es, xs2);
                    if (quit) return;
                    put_xe(sl, s0, es, xs2);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (lane == 0) __hip_atomic_store(&filled[slot], rel, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            };
            const int w = wave - NS;
            if constexpr (kPfPipe) {
                Pre p0, p1;
                if (w < nss) issue(w, p0);
                for (int rel = w; rel < nss && !quit; rel += 2 * NP) {
                    process(rel, p0, p1);
                    if (rel + NP < nss && !quit) process(rel + NP, p1, p0);
                }
            } else {
                for (int rel = w; rel < nss && !quit; rel += NP) {
                    Pre p0;
                    issue(rel, p0);
                    process(rel, p0, p0);
                }
            }
        }
    }
    if (threadIdx.x == 0) {
        uint32_t d = atomicAdd(&sync[1], 1u);
        if (d == gridDim.x - 1) {
            __hip_atomic_store(&sync[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&sync[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Fallback for triangles whose rows are too long for the LDS slots: rows in
// level order cut into 64-row chunks inside a level, wavefronts take chunks in
// increasing order from a ticket counter and poll every dependency in global
// memory (a chunk only waits for chunks taken by running wavefronts).
template <class T, bool UPPER>
__global__ __launch_bounds__(256) void k_trsv_sf(int32_t nchunks, const int32_t *__restrict__ chunk_ptr, int32_t K,
                                                 int32_t ldq, const int32_t *__restrict__ grow,
                                                 const int32_t *__restrict__ other, const int32_t *__restrict__ enc,
                                                 const T *__restrict__ val, const T *__restrict__ piv,
                                                 SolveIO<T> io, uint32_t *sync, const int32_t *skip,
                                                 uint32_t *err, uint32_t spin) {
    using U = typename Sentinel<T>::U;
    constexpr U SENT = Sentinel<T>::bits;
    if (skip && *skip) return;
    fill_sentinel(io);
    T *const xq = io.xq;
    T *const x = io.x;
    T *const yother = io.yother;
    const int lane = threadIdx.x & 63;
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(&sync[0], 1u);
        t = __shfl(t, 0);
        if (t >= (uint32_t)nchunks) break;
        const int32_t q = chunk_ptr[t] + lane;
        bool quit = false;  // this lane's wait gave up (here or, through the error word, elsewhere)
        if (q < chunk_ptr[t + 1]) {
            const int32_t gi = grow[q];
            T acc = io.b[io.bmap ? io.bmap[q] : io.b_by_row ? gi : q];
            for (int32_t s0 = 0; s0 < K; s0 += kBatch) {
                const int nb = min(kBatch, K - s0);
                int es[kBatch];
                T vs[kBatch];
                U xs[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    es[u] = kPad;
                    vs[u] = (T)0;
                    if (u < nb) {
                        es[u] = enc[(size_t)(s0 + u) * ldq + q];
                        vs[u] = val[(size_t)(s0 + u) * ldq + q];
                    }
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) xs[u] = u < nb ? first_poll(xq, es[u]) : (U)0;
                bool pend = false;
#pragma unroll
                for (int u = 0; u < kBatch; ++u) pend |= u < nb && xs[u] == SENT;
                uint32_t it = 0;
                while (pend) {  // only the pending entries are reloaded
                    ++it;
                    if (it > spin || ((it & 63) == 0 && timed_out(err))) {
                        record_timeout(err);
                        quit = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
#pragma unroll
                    for (int u = 0; u < kBatch; ++u)
                        if (u < nb && xs[u] == SENT) xs[u] = load_coherent(xq + es[u]);
                    pend = false;
#pragma unroll
                    for (int u = 0; u < kBatch; ++u) pend |= u < nb && xs[u] == SENT;
                }
                if (quit) break;
#pragma unroll
                for (int u = 0; u < kBatch; ++u)
                    if (u < nb && es[u] != kPad) acc -= vs[u] * from_bits<T>(xs[u]);
            }
            if (!quit) {  // (after a give-up nothing more is published)
                if constexpr (UPPER) acc = acc / piv[q];
                store_coherent(xq + q, acc);
                if (x) x[gi] = acc;
                if (yother) {
                    const int32_t o = other[q];
                    if (o >= 0) yother[o] = acc;
                }
            }
        }
        if (__ballot(quit) != 0) break;  // every lane is back here: the wave stops as a whole
    }
    if (lane == 0) {
        const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
        uint32_t d = atomicAdd(&sync[1], 1u);
        if (d == nwaves - 1) {
            __hip_atomic_store(&sync[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&sync[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// Wavefront solve of a grid triangle (plan.hpp's GridPlan): one tile of TA x TB
// columns per workgroup (8 x 8 on a 3D grid, which the description below follows;
// 64 x 1 on a 2D grid), tiles claimed in order from a ticket counter (a tile only
// waits for tiles claimed before it, held by running workgroups).
//  * Wavefront 0 solves. At step s lane (ma, mb) solves the row at c-index
//    s - ma - mb of its column; that row's dependencies were solved at step s - 1:
//    the one behind it along c by the lane itself (a register), the ones along a
//    and b by lanes (ma - 1, mb) and (ma, mb - 1), or, on the tile's low faces, by
//    the tiles before it. Each step has a 9 x 9 grid of cells in LDS, a cell per
//    lane (row mb, column ma; row and column 8 take the high faces' writes)
//    holding the two values the lane reads: from the left and from below. A lane
//    writes its result into the left slot of the cell to its right and the below
//    slot of the cell above in the next step's grid (one LDS instruction), the
//    face poller fills the slots no lane writes (the left slots of column 0, the
//    below slots of row 0), and a lane reads its cell in one instruction. A single wavefront issues
//    at most one instruction every 4 cycles, so the step is kept to a few dozen
//    instructions: the dependency chain is one LDS round trip and three fused
//    multiply-adds. Steps run as unrolled blocks of 8 with ring offsets fixed at
//    compile time and one release per block: about 20 instructions a step where a
//    whole tile's 64 rows are all valid for the 8 steps (the bulk of a long column),
//    a few more with validity masks elsewhere (0.13 us a step against 0.19 us for
//    the general step, which only a column's last, partial block takes).
//  * Wavefronts 1..kGridPollers poll the tile's incoming face values (8 on the
//    a-face, 8 on the b-face per step) for a window of the next 4 * HEC_GRID_POLL_R
//    steps, one lane per value and step, with device-coherent loads until they are
//    not the sentinel, write each into its step's grid, and raise the count of
//    leading steps that have all of theirs. (Several pollers would poll the same
//    window independently; a wider window or more pollers send more device-coherent
//    loads, and a poll takes longer the more lines it reads: at 128^3 every wider
//    window or second poller measured slower.) A 2D tile's poller polls its one
//    face value per step, 32 steps at a time.
//  * The other wavefronts load the coefficients (packed by claim, step and lane, so
//    every load is a whole line) and the right-hand side of runs of steps into a
//    ring of LDS slots. They depend on nothing but the ring, so they run ahead.
//  * The solver stores each result to the output (by row, or in padded tile-step
//    order for the intermediate of an L-then-U chain) and, on the tile's high
//    faces, to the face buffer with a device-coherent store, at the index of the
//    step at which the next tile needs it (the corner lane's value only on the
//    a-face, where the tile above also reads it).
// Readiness is the value itself, as in the blocked kernel: the face buffer holds
// the sentinel before the launch (filled by the previous launch of an L-then-U
// chain, or by a fill kernel before a lone solve).
#ifndef HEC_GRID_POLL_R
#define HEC_GRID_POLL_R 1
#endif
#ifndef HEC_GRID_POLLERS
#define HEC_GRID_POLLERS 1
#endif
#ifndef HEC_GRID_POLL_SLEEP
#define HEC_GRID_POLL_SLEEP 2
#endif
constexpr int kGridWaves = 8;    // the solver, the face pollers, then loaders
constexpr int kGridPollers = HEC_GRID_POLLERS;
constexpr int kGridLoaders = kGridWaves - 1 - kGridPollers;
constexpr int kGridBatch = 3;   // consecutive steps a loader has in flight
constexpr int kGridRing = 32;   // steps in LDS (slots and grids): how far loads run ahead
static_assert((kGridRing & (kGridRing - 1)) == 0 && kGridRing % 8 == 0 && kGridBatch <= kGridRing, "ring");

struct GridArgs {
    int32_t NA, NB, NC, PA, PB, S, nclaims;
    int64_t sa, sb, sc;
    uint32_t *err;  // the schedule's error word
    uint32_t spin;  // polls before a wait gives up
};

// b: right-hand side by row; x: results by row; face: the triangle's face buffer
// ([claim][face][step][8], sentinel-filled); fill: nfill elements set to the
// sentinel for a later solve (may be NULL). bpad / xpad: b / x in padded tile-step
// order instead, the lower plan's position (claim * S + step) * 64 + lane, which the
// upper plan visits in reverse (its claim c, step s, lane l is the lower plan's
// position total - 1 - (c S + s) 64 - l): the intermediate of an L-then-U chain, read
// and written 512 contiguous bytes a step instead of a row-by-row gather.
template <class T>
struct GridIO {
    const T *b;
    T *x;
    T *face;
    T *fill;
    int64_t nfill;
    int32_t bpad, xpad;
};

// Dynamic LDS of k_trsv_grid: control words, slots [ring][NCOEF + 1][64], grids
// [ring][TB + 1][TA + 1][2] (a cell: the value from the left, the value from below).
constexpr size_t kGridCtrl = 256;
template <class T, bool UPPER, int TA>
constexpr size_t grid_lds_bytes() {
    constexpr int NCOEF = UPPER ? plan::kGridCoefUpper : plan::kGridCoefLower;
    return kGridCtrl + (size_t)kGridRing * (NCOEF + 1) * 64 * sizeof(T) +
           (size_t)kGridRing * (TA + 1) * (64 / TA + 1) * 2 * sizeof(T);
}

// TA: tile side along a (8: 8 x 8 tiles of a 3D grid; 64: 64 x 1 tiles of a 2D grid,
// whose b-face is empty: its cells are zeroed once per tile and never written again).
template <class T, bool UPPER, int TA>
__global__ __launch_bounds__(64 * kGridWaves) void k_trsv_grid(GridArgs G, const T *__restrict__ coef, GridIO<T> io,
                                                               uint32_t *sync, const int32_t *skip) {
    using U = typename Sentinel<T>::U;
    constexpr U SENT = Sentinel<T>::bits;
    constexpr int NCOEF = UPPER ? plan::kGridCoefUpper : plan::kGridCoefLower;
    static_assert(TA == plan::kGT || TA == plan::kGT2, "tile shape");
    constexpr int TB = 64 / TA, GG = TA + 1, GA = (TA + 1) * (TB + 1) * 2, RM = kGridRing - 1;
    // face entries per step in the face buffer: 8 and 8 on a 3D grid, the one a-face entry
    // on a 2D grid (no tile has a tile above it there)
    constexpr int FS = TA == TB ? TA : TB;
    constexpr int SLOT = (NCOEF + 1) * 64;  // elements of a slot: [NCOEF][64] coefficients, [64] rhs
    if (skip && *skip) return;  // uniform: no workgroup touches the counters
    if (io.fill) {
        const T sv = from_bits<T>(SENT);
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < io.nfill;
             i += (int64_t)gridDim.x * blockDim.x)
            io.fill[i] = sv;
    }
    extern __shared__ __align__(16) char gsm[];
    int *const filled = (int *)gsm;          // [ring]: step whose coefficients and rhs a slot holds
    int *const s_done = filled + kGridRing;  // steps the solver has finished (slots and grids below are free)
    int *const s_faces = s_done + 1;         // leading steps whose face values are all in their grids
    int *const s_claim = s_done + 2;
    int *const s_abort = s_done + 3;
    T *const slots = (T *)(gsm + kGridCtrl);
    T *const xg = slots + kGridRing * SLOT;  // [ring][9][9][2]: row mb, column ma; left, below
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ma = lane % TA, mb = lane / TA;
    if (threadIdx.x == 0) *s_abort = 0;
    auto give_up = [&]() {
        __hip_atomic_store(s_abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        record_timeout(G.err);
    };
    // one more poll of a wait (wave-uniform callers): true when the wait must stop
    auto spun_out = [&](uint32_t &it, bool device_wide) {
        ++it;
        bool stop = it > G.spin;
        if (!stop && (it & 63) == 0)
            stop = __hip_atomic_load(s_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0 ||
                   (device_wide && timed_out(G.err));
        stop = __builtin_amdgcn_readfirstlane((int)stop) != 0;
        if (stop) give_up();
        return stop;
    };
    auto lds_load = [](const int *p) {
        return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
    };
    // waits until the solver has finished step `below` (its slot is free); false: gave up
    auto wait_done = [&](int below) {
        uint32_t it = 0;
        while (lds_load(s_done) <= below) {
            if (spun_out(it, false)) return false;
            __builtin_amdgcn_s_sleep(2);
        }
        return true;
    };
    for (;;) {
        __syncthreads();
        if (*s_abort) break;  // uniform: read by every thread after the barrier
        if (threadIdx.x == 0) {
            *s_claim = (int)atomicAdd(&sync[0], 1u);
            *s_done = 0;
            *s_faces = 0;
        }
        if (threadIdx.x < kGridRing) filled[threadIdx.x] = -1;
        // step 0: no previous results (a 2D tile: every grid, whose b-face cells stay zero)
        for (int t = threadIdx.x; t < (TB == 1 ? kGridRing * GA : GA); t += blockDim.x) xg[t] = (T)0;
        __syncthreads();
        const int c = *s_claim;
        if (c >= G.nclaims) break;
        const int mta = c % G.PA, mtb = c / G.PA;
        const int32_t ta = UPPER ? G.PA - 1 - mta : mta, tb = UPPER ? G.PB - 1 - mtb : mtb;
        // global a and b of the column of lane (ma', mb')
        auto col_a = [&](int m) { return ta * TA + (UPPER ? TA - 1 - m : m); };
        auto col_b = [&](int m) { return tb * TB + (UPPER ? TB - 1 - m : m); };
        const bool act = col_a(ma) < G.NA && col_b(mb) < G.NB;
        const int64_t base = (int64_t)col_a(ma) * G.sa + (int64_t)col_b(mb) * G.sb;
        auto row_at = [&](int32_t mc) { return base + (int64_t)(UPPER ? G.NC - 1 - mc : mc) * G.sc; };
        // this lane's padded tile-step position at step 0, and its change per step
        const int64_t pq = (int64_t)c * G.S * 64 + lane;
        const int64_t p0 = UPPER ? (int64_t)G.nclaims * G.S * 64 - 1 - pq : pq, pd = UPPER ? -64 : 64;

        if (wave == 0) {
            // ---------------- solver
            __builtin_amdgcn_s_setprio(3);
            const bool has_u = mtb < G.PB - 1;  // a tile above reads the b-face
            // this lane's face store (if any): a-face by mb (the corner too), b-face by ma
            const bool fst = ma == TA - 1 || (mb == TB - 1 && has_u);
            T *const fp = io.face + ((int64_t)c * 2 + (ma == TA - 1 ? 0 : 1)) * G.S * 8 +
                          (ma == TA - 1 ? mb - (TA - 1) * FS : ma - (TB - 1) * FS);  // + FS s: the entry of step s
            T xp = (T)0;  // this lane's result of the previous step (0: none)
            int ready = 0, fready = 0;
            bool bail = false;
            // waits until step s is loaded; returns one past the run of loaded steps from s
            // (8 flags, one per lane, in one LDS round trip)
            auto scan = [&](int s) -> int {
                const int u = lane & 7;
                uint32_t it = 0;
                for (;;) {
                    const int want = s + u;
                    const int f = __hip_atomic_load(&filled[want & RM], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP);
                    const uint64_t m = __ballot(lane < 8 && want < G.S && f == want);
                    const int ok = __builtin_ctzll(~m);
                    if (ok > 0) {
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        return s + ok;
                    }
                    if (spun_out(it, false)) {
                        bail = true;
                        return s;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            };
            auto wait_faces = [&](int s) -> int {  // until step s has its face values
                uint32_t it = 0;
                for (;;) {
                    const int f = lds_load(s_faces);
                    if (f > s) {
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        return f;
                    }
                    if (spun_out(it, false)) {
                        bail = true;
                        return s;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            };
            auto ensure = [&](int s) {  // step s loaded and its faces in; false: gave up
                if (s >= ready) ready = scan(s);
                if (s >= fready && !bail) fready = wait_faces(s);
                return !bail;
            };
            struct Step {  // one step's coefficients and right-hand side
                T cv[NCOEF];
                T bv;
            };
            auto load_step = [&](int s, Step &H) {
                const T *sl = slots + (s & RM) * SLOT + lane;
#pragma unroll
                for (int k = 0; k < NCOEF; ++k) H.cv[k] = sl[k * 64];
                H.bv = sl[NCOEF * 64];
            };
            // the lane's row at step s: c-index s - ma - mb, valid for (unsigned)(s - moff) < ncl
            const int moff = ma + mb;
            const uint32_t ncl = act ? (uint32_t)G.NC : 0u;
            const int64_t dsc = io.xpad ? pd : UPPER ? -G.sc : G.sc;
            int64_t roff = io.xpad ? p0 : row_at(-moff);  // the output of step 0, advanced by dsc a step
            const int gl = (mb * GG + ma) * 2;  // this lane's cell
            // One step: cur holds its inputs; the next step's are read into nxt while it
            // computes. That read is speculative (unconditional, so that the compiler
            // counts it exactly when it waits for the neighbours' values) and is repeated
            // after the wait when the next step was not yet known to be ready. After a
            // give-up the step still runs (so the two register sets keep one data flow)
            // but stores nothing.
            auto step = [&](int s, Step &cur, Step &nxt, bool odd) {
                const T *g = xg + (s & RM) * GA + gl;
                const T left = g[0], below = g[1];
                const bool more = s + 1 < G.S;
                const bool early = more && s + 1 < ready && s + 1 < fready;
                load_step(s + 1, nxt);  // (when s + 1 = S: a slot in range, unused)
                T acc;
                if constexpr (!UPPER) {  // columns ascending (c along z): back, below, left
                    acc = cur.bv - cur.cv[0] * xp;
                    acc -= cur.cv[1] * below;
                    acc -= cur.cv[2] * left;
                } else {  // left, below, back; then the reciprocal pivot
                    acc = cur.bv - cur.cv[2] * left;
                    acc -= cur.cv[1] * below;
                    acc -= cur.cv[0] * xp;
                    acc *= cur.cv[3];
                }
                const bool valid = (uint32_t)(s - moff) < ncl;
                const T xn = valid ? acc : (T)0;
                T *gn = xg + ((s + 1) & RM) * GA + gl;
                gn[2] = xn;           // left slot of the cell to the right
                gn[2 * GG + 1] = xn;  // below slot of the cell above
                if (valid && !bail) {
                    io.x[roff] = xn;
                    if (fst) store_coherent(fp + (int64_t)s * FS, xn);  // the next tile reads it at step s - TA + 1
                }
                xp = xn;
                roff += dsc;
                // slots and grids up to s are free once read: LDS accesses of one wavefront
                // complete in order, so the reads issued above are done before this store
                if (odd || !more) {
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    if (lane == 0) __hip_atomic_store(s_done, s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                if (more && !early && ensure(s + 1)) load_step(s + 1, nxt);
            };
            // Eight steps s0 .. s0 + 7 (s0 + 8 < S) with the coefficients of all of them and
            // the next loaded: no load bookkeeping, ring offsets fixed at compile time (the
            // ring holds whole blocks of 8), one release of the slots at the end; only the
            // face values are checked step by step, as they arrive. MASKED: lanes whose row
            // at a step is not valid publish zeros and store nothing; unmasked blocks are
            // those at which every lane's row is valid (a tile with all 64 columns in the
            // grid, TA + TB - 2 <= s0 and s0 + 8 <= NC: the bulk of a long column).
            // On entry H0 holds step s0's coefficients; on exit step s0 + 8's.
            auto block8 = [&](auto masked, int s0, Step &H0, Step &H1) {
                constexpr bool MASKED = decltype(masked)::value;
                T *const gb = xg + (s0 & RM) * GA + gl;
                T *const gx = xg + ((s0 + 8) & RM) * GA + gl;
                const T *const sb = slots + (s0 & RM) * SLOT + lane;
                const T *const sx = slots + ((s0 + 8) & RM) * SLOT + lane;
                T *const fb = fp + (int64_t)s0 * FS;
                T *xo = io.x + roff;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int s = s0 + u;
                    if (s >= fready) {
                        fready = wait_faces(s);
                        if (bail) break;
                    }
                    Step &cur = (u & 1) ? H1 : H0;
                    Step &nxt = (u & 1) ? H0 : H1;
                    const T *g = gb + u * GA;
                    const T left = g[0], below = g[1];
                    const T *sl = u < 7 ? sb + (u + 1) * SLOT : sx;
#pragma unroll
                    for (int k = 0; k < NCOEF; ++k) nxt.cv[k] = sl[k * 64];
                    nxt.bv = sl[NCOEF * 64];
                    T acc;
                    if constexpr (!UPPER) {
                        acc = cur.bv - cur.cv[0] * xp;
                        acc -= cur.cv[1] * below;
                        acc -= cur.cv[2] * left;
                    } else {
                        acc = cur.bv - cur.cv[2] * left;
                        acc -= cur.cv[1] * below;
                        acc -= cur.cv[0] * xp;
                        acc *= cur.cv[3];
                    }
                    const bool valid = !MASKED || (uint32_t)(s - moff) < ncl;
                    if constexpr (MASKED) acc = valid ? acc : (T)0;
                    T *gn = u < 7 ? gb + (u + 1) * GA : gx;
                    gn[2] = acc;
                    gn[2 * GG + 1] = acc;
                    if (valid) *xo = acc;
                    xo += dsc;
                    // an arithmetic result is never the signalling-NaN sentinel (IEEE mode
                    // quiets NaN operands), so no check is needed before publishing it
                    if (valid && fst) {
                        U bits;
                        __builtin_memcpy(&bits, &acc, sizeof(T));
                        __hip_atomic_store((U *)(fb + u * FS), bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    xp = acc;
                }
                roff += 8 * dsc;
                if (!bail) {
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    if (lane == 0) __hip_atomic_store(s_done, s0 + 8, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            };
            const bool full = __ballot(act) == ~0ull;
            Step h0, h1;
            if (ensure(0)) load_step(0, h0);
            for (int s0 = 0; s0 < G.S && !bail; s0 += 8) {
                const bool whole = full && s0 >= TA + TB - 2 && s0 + 8 <= G.NC;
                if (whole || s0 + 8 < G.S) {
                    while (ready <= s0 + 8 && !bail) ready = scan(ready);
                    if (bail) break;
                    if (whole)
                        block8(std::integral_constant<bool, false>{}, s0, h0, h1);
                    else
                        block8(std::integral_constant<bool, true>{}, s0, h0, h1);
                } else {  // the last, partial block
                    for (int s = s0; s < min(s0 + 8, G.S) && !bail; s += 2) {
                        if (s >= ready || s >= fready) ensure(s);  // after a block: step s's faces
                        step(s, h0, h1, false);
                        if (s + 1 < G.S) step(s + 1, h1, h0, true);
                    }
                }
            }
            __builtin_amdgcn_s_setprio(0);
        } else if (TB == 1 && wave <= kGridPollers) {
            // ---------------- face poller of a 2D tile: its one face value per step (the left
            // value of lane 0), from the tile before along a. Lane l < 32 polls step w + l; a
            // value goes into its step's grid once, when it has arrived and the solver is done
            // with the grid's previous use; the window moves on by the leading steps that have
            // their value, whose count is published.
            if (wave == 1) {
                const bool has = mta > 0;
                const T *const fsrc = has ? io.face + (int64_t)(c - 1) * 2 * G.S * 8 : io.face;
                int w = 0, pub = 0;
                bool wr = false;  // this lane's value of step w + lane is in its grid
                uint32_t it = 0;
                while (pub < G.S) {
                    const int dn = lds_load(s_done);
                    const int st = w + lane;
                    const bool can = lane < 32 && !wr && st < G.S && st < dn + kGridRing;
                    const bool need = can && has && st < G.NC;
                    const U v = need ? load_coherent(fsrc + st) : (U)0;
                    if (can && (!need || v != SENT)) {
                        xg[(st & RM) * GA] = need ? from_bits<T>(v) : (T)0;
                        wr = true;
                    }
                    const uint64_t m = __ballot(wr || (lane < 32 && st >= G.S)) & 0xFFFFFFFFull;
                    const int k = __builtin_ctzll(~m);  // leading steps of the window with their value
                    if (w + k > pub) {
                        pub = min(w + k, G.S);
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // after this wave's writes
                        if (lane == 0) __hip_atomic_store(s_faces, pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        it = 0;
                    } else {
                        if (spun_out(it, true)) break;
                        __builtin_amdgcn_s_sleep(HEC_GRID_POLL_SLEEP);
                    }
                    if (k > 0) {  // lane l takes over lane l + k's step
                        const int from = lane + k;
                        const int nw = __shfl((int)wr, from < 64 ? from : lane);
                        wr = from < 32 && nw != 0;
                        w += k;
                    }
                }
            }
        } else if (wave <= kGridPollers) {
            // ---------------- face pollers: a window of 4R steps from w, step w + q + 4r in
            // lane 16q + i for r < R; i < 8: a-face entry i (lane (0, i)), i >= 8:
            // b-face entry i - 8 (lane (i - 8, 0)). A value goes into its step's grid once,
            // when it has arrived and the solver is done with the grid's previous step; the
            // window moves on by whole groups of 4 steps, and the count of leading steps
            // with all their values is published as it grows.
            constexpr int R = HEC_GRID_POLL_R;
            const int q = lane >> 4, i = lane & 15, j = i & 7;
            const bool on_a = i < 8;
            const bool has = on_a ? mta > 0 && col_b(j) < G.NB : mtb > 0 && col_a(j) < G.NA;
            // a-face entry j: a-face of the tile before along a; b-face entry j: b-face of the
            // tile below, its corner (j = 7) on that tile's a-face
            const T *const fsrc = !has              ? io.face  // (not read)
                                  : on_a            ? io.face + ((int64_t)(c - 1) * 2 + 0) * G.S * 8 + j
                                  : j == TA - 1     ? io.face + ((int64_t)(c - G.PA) * 2 + 0) * G.S * 8 + j
                                                    : io.face + ((int64_t)(c - G.PA) * 2 + 1) * G.S * 8 + j;
            // a-face: left slot of lane (0, j)'s cell; b-face: below slot of lane (j, 0)'s cell
            const int gpos = on_a ? j * GG * 2 : j * 2 + 1;
            int w = 0, pub = 0;
            bool wr[R] = {};  // this lane's value of step w + q + 4r is in its grid
            uint32_t it = 0;
            while (pub < G.S) {
                const int dn = lds_load(s_done);
                U v[R];
                bool need[R], can[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {  // all loads first, then one wait
                    const int st = w + q + 4 * r;
                    can[r] = !wr[r] && st < G.S && st < dn + kGridRing;
                    need[r] = can[r] && has && st - j >= 0 && st - j < G.NC;
                    v[r] = need[r] ? load_coherent(fsrc + (int64_t)st * 8) : (U)0;
                }
                uint64_t okm[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int st = w + q + 4 * r;
                    if (can[r] && (!need[r] || v[r] != SENT)) {
                        xg[(st & RM) * GA + gpos] = need[r] ? from_bits<T>(v[r]) : (T)0;
                        wr[r] = true;
                    }
                    okm[r] = __ballot(wr[r] || st >= G.S);
                }
                int k = 0;  // leading steps of the window with all their values
                if constexpr (R == 1) {
                    uint64_t t = okm[0];  // bit 16 q ends up set when all 16 lanes of step w + q are in
                    t &= t >> 8;
                    t &= t >> 4;
                    t &= t >> 2;
                    t &= t >> 1;
                    const uint32_t g = (uint32_t)((t & 1) | ((t >> 15) & 2) | ((t >> 30) & 4) | ((t >> 45) & 8));
                    k = __builtin_ctz(~g);
                } else {
                    bool gap = false;
#pragma unroll
                    for (int r = 0; r < R; ++r)
#pragma unroll
                        for (int qq = 0; qq < 4; ++qq) {
                            gap = gap || ((okm[r] >> (16 * qq)) & 0xFFFFull) != 0xFFFFull;
                            k += gap ? 0 : 1;
                        }
                }
                if (w + k > pub) {
                    pub = min(w + k, G.S);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // after this wave's writes
                    if (lane == 0) {  // one poller: its count only grows; several: the largest
                        if constexpr (kGridPollers == 1)
                            __hip_atomic_store(s_faces, pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        else
                            __hip_atomic_fetch_max(s_faces, pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    it = 0;
                } else {
                    if (spun_out(it, true)) break;
                    __builtin_amdgcn_s_sleep(HEC_GRID_POLL_SLEEP);
                }
                const int gsh = k >> 2;  // whole groups done: the window moves on
                if (gsh > 0) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        bool nw = false;
#pragma unroll
                        for (int u = 1; u < R; ++u) nw = u == gsh && r + u < R ? wr[r + u] : nw;
                        wr[r] = nw;
                    }
                    w += 4 * gsh;
                }
            }
        } else {
            // ---------------- loaders: wavefront 1 + kGridPollers + l takes runs of kGridBatch consecutive
            // steps, l * kGridBatch + i * L * kGridBatch (L loaders), each run in flight at
            // once; a run only waits for its own slots, so loads run up to the ring's
            // depth ahead of the solver
            constexpr int NL = kGridLoaders, B = kGridBatch;
            for (int s0 = (wave - 1 - kGridPollers) * B; s0 < G.S; s0 += NL * B) {
                if (!wait_done(min(s0 + B, G.S) - 1 - kGridRing)) break;
                T cv[B][NCOEF], bv[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int s = s0 + u;
                    const bool in = s < G.S;
                    const T *cp = coef + ((int64_t)c * G.S + (in ? s : s0)) * NCOEF * 64 + lane;
#pragma unroll
                    for (int k = 0; k < NCOEF; ++k) cv[u][k] = cp[k * 64];
                    const int32_t mc = s - ma - mb;
                    bv[u] = in && act && mc >= 0 && mc < G.NC ? io.b[io.bpad ? p0 + s * pd : row_at(mc)] : (T)0;
                }
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int s = s0 + u;
                    if (s < G.S) {
                        T *sl = slots + (s & RM) * SLOT + lane;
#pragma unroll
                        for (int k = 0; k < NCOEF; ++k) sl[k * 64] = cv[u][k];
                        sl[NCOEF * 64] = bv[u];
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (lane < B && s0 + lane < G.S)
                    __hip_atomic_store(&filled[(s0 + lane) & RM], s0 + lane, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // the last workgroup out resets the counters for the next launch
        const uint32_t d = atomicAdd(&sync[1], 1u);
        if (d == gridDim.x - 1) {
            __hip_atomic_store(&sync[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&sync[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Packed coefficients of a wavefront plan: out[q] = value map[q] of the factor (0
// where map[q] < 0); slot k = 3 of each step holds the reciprocal of the pivot.
template <class T>
__global__ __launch_bounds__(256) void k_grid_coef(size_t n, int ncoef, const int32_t *__restrict__ map,
                                                   const double *__restrict__ src, T *__restrict__ out) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int32_t m = map[q];
    const int k = (int)((q / 64) % (size_t)ncoef);
    T v = m >= 0 ? (T)src[m] : (T)0;
    if (k == 3 && m >= 0) v = (T)1 / v;
    out[q] = v;
}

// Before a single-triangle solve: the output filled with the sentinel.
template <class T>
__global__ __launch_bounds__(256) void k_trsv_fill(int64_t n, T *x, const int32_t *skip) {
    if (skip && *skip) return;
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) x[q] = from_bits<T>(Sentinel<T>::bits);
}

// dst[q] = src[map[q]] (0 where map[q] < 0), optional FP32 copy.
__global__ __launch_bounds__(256) void k_gather(size_t n, const int32_t *__restrict__ map,
                                                const double *__restrict__ src, double *__restrict__ dst,
                                                float *__restrict__ dst32) {
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int32_t m = map[q];
    double v = m >= 0 ? src[m] : 0.0;
    dst[q] = v;
    if (dst32) dst32[q] = (float)v;
}

int max_lds_per_block() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 64 * 1024;
    return std::min(v, 160 * 1024);
}

template <class T, bool UPPER>
void launch_blk(const hec_tri &tri, uint32_t *sync, uint32_t *err, const SolveIO<T> &io, hipStream_t s,
                const int32_t *skip) {
    const uint32_t spin = spin_limit();
    T *const yother = io.yother;
    if (tri.nparts == 0 && tri.nchunks == 0) return;
    const bool f64 = sizeof(T) == 8;
    if (!tri.blocked) {
        const T *val = f64 ? (const T *)tri.val.get() : (const T *)tri.val32.get();
        const T *piv = UPPER ? (f64 ? (const T *)tri.piv.get() : (const T *)tri.piv32.get()) : nullptr;
        int waves = std::min(tri.nchunks, 1024);
        k_trsv_sf<T, UPPER><<<(waves + 3) / 4, 256, 0, s>>>(tri.nchunks, tri.chunk_ptr.get(), tri.K, tri.ldq,
                                                          tri.grow.get(), yother ? tri.other.get() : nullptr,
                                                          tri.enc.get(), val, piv, io, sync, skip, err, spin);
        HEC_CHECK_LAUNCH();
        return;
    }
    const size_t lds = f64 ? tri.lds64 : tri.lds32;
    PlanArgs P{tri.nparts, tri.K, tri.ldq, tri.W, f64 ? tri.D64 : tri.D32, tri.S,
               tri.part_ss.get(), tri.part_pos.get(), tri.ss_pos.get(), tri.ss_need.get(), tri.grow.get(),
               yother ? tri.other.get() : nullptr, tri.enc.get(), err, spin};
    const T *val, *piv = nullptr;
    if constexpr (sizeof(T) == 8) {
        val = tri.val.get();
        if (UPPER) piv = tri.piv.get();
    } else {
        val = tri.val32.get();
        if (UPPER) piv = tri.piv32.get();
    }
    const int grid = std::min(tri.nparts, 256);
    auto go = [&](auto kc, auto ns) {
        constexpr int KC = decltype(kc)::value, NS = decltype(ns)::value;
        static bool attr_set = false;  // one per instantiation
        if (!attr_set) {
            HEC_HIP(hipFuncSetAttribute((const void *)k_trsv_blk<T, UPPER, KC, NS>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_per_block()));
            attr_set = true;
        }
        k_trsv_blk<T, UPPER, KC, NS><<<grid, kBlkThreads, lds, s>>>(P, val, piv, io, sync, skip);
    };
    // the planner gives 1 or plan::kSolvers solver wavefronts
    auto go_kc = [&](auto ns) {
        switch (tri.KC) {
            case 4: go(std::integral_constant<int, 4>(), ns); break;
            case 8: go(std::integral_constant<int, 8>(), ns); break;
            case 16: go(std::integral_constant<int, 16>(), ns); break;
            default: go(std::integral_constant<int, 32>(), ns); break;
        }
    };
    if (tri.NS == 1)
        go_kc(std::integral_constant<int, 1>());
    else if constexpr (plan::kSolvers > 1)
        go_kc(std::integral_constant<int, plan::kSolvers>());
    HEC_CHECK_LAUNCH();
}

template <class T, bool UPPER>
void launch_grid(const hec_grid &g, uint32_t *sync, uint32_t *err, const GridIO<T> &io, hipStream_t s,
                 const int32_t *skip) {
    const int32_t nclaims = g.PA * g.PB;
    GridArgs G{g.NA, g.NB, g.NC, g.PA, g.PB, g.S, nclaims, g.sa, g.sb, g.sc, err, spin_limit()};
    const T *coef;
    if constexpr (sizeof(T) == 8)
        coef = g.coef.get();
    else
        coef = g.coef32.get();
    const int grid = std::min(nclaims, 1024);
    auto go = [&](auto ta) {
        constexpr int TA = decltype(ta)::value;
        constexpr size_t lds = grid_lds_bytes<T, UPPER, TA>();
        static_assert(lds <= 160 * 1024, "LDS");
        static bool attr_set = false;  // one per instantiation
        if (!attr_set) {
            HEC_HIP(hipFuncSetAttribute((const void *)k_trsv_grid<T, UPPER, TA>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            attr_set = true;
        }
        k_trsv_grid<T, UPPER, TA><<<grid, 64 * kGridWaves, lds, s>>>(G, coef, io, sync, skip);
    };
    if (g.TA == plan::kGT)
        go(std::integral_constant<int, plan::kGT>());
    else
        go(std::integral_constant<int, plan::kGT2>());
    HEC_CHECK_LAUNCH();
}

// The wavefront path of trsv_launch (both triangles have grid plans; not RAS).
template <class T>
void trsv_launch_grid(const hec_levels_s &lv, uint32_t which, const T *b, T *x, hipStream_t s,
                      const int32_t *skip) {
    T *fL, *fU, *yp;
    if constexpr (sizeof(T) == 8) {
        fL = lv.fL64.get();
        fU = lv.fU64.get();
        yp = lv.yp64.get();
    } else {
        fL = lv.fL32.get();
        fU = lv.fU32.get();
        yp = lv.yp32.get();
    }
    const int64_t nface = lv.lower.grid.face_elems();
    uint32_t *sync = const_cast<uint32_t *>(lv.sync.get());
    uint32_t *err = sync + kLevelsErrWord;
    if (which == HEC_LU) {
        // fL is sentinel-filled between chains (by level_schedule, then by every upper
        // launch); the lower launch fills fU for the upper one
        // the intermediate goes through yp in padded tile-step order
        launch_grid<T, false>(lv.lower.grid, sync, err, GridIO<T>{b, yp, fL, fU, nface, 0, 1}, s, skip);
        launch_grid<T, true>(lv.upper.grid, sync + 2, err, GridIO<T>{yp, x, fU, fL, nface, 1, 0}, s, skip);
        return;
    }
    // a lone triangle: fU, free between calls, is filled right before
    k_trsv_fill<T><<<ceil_div(nface, 256), 256, 0, s>>>(nface, fU, skip);
    HEC_CHECK_LAUNCH();
    if (which == HEC_LOWER)
        launch_grid<T, false>(lv.lower.grid, sync, err, GridIO<T>{b, x, fU, nullptr, 0}, s, skip);
    else
        launch_grid<T, true>(lv.upper.grid, sync + 2, err, GridIO<T>{b, x, fU, nullptr, 0}, s, skip);
}

}  // namespace

template <class T>
void trsv_launch(const hec_levels_s &lv, uint32_t which, const T *b, T *x, hipStream_t s, const int32_t *skip) {
    const int64_t n = lv.n, nf = lv.nf;
    if (n == 0) return;
    T *qL, *qU, *yp;
    if constexpr (sizeof(T) == 8) {
        qL = lv.qL64.get();
        qU = lv.qU64.get();
        yp = lv.yp64.get();
    } else {
        qL = lv.qL32.get();
        qU = lv.qU32.get();
        yp = lv.yp32.get();
    }
    if (lv.lower.grid.on && lv.upper.grid.on) {
        trsv_launch_grid<T>(lv, which, b, x, s, skip);
        return;
    }
    uint32_t *sync = const_cast<uint32_t *>(lv.sync.get());
    uint32_t *err = sync + kLevelsErrWord;
    if (which == HEC_LU) {
        // qL is sentinel-filled between calls (by level_schedule, then by every upper
        // launch); the lower launch fills qU for the upper one: two launches in all.
        // Restricted additive Schwarz: the lower solve reads b through the stacked
        // rows' system rows (bmap); the upper solve writes each owned row's result to
        // x through `other`, overlap rows nowhere.
        if (lv.ras) {
            launch_blk<T, false>(lv.lower, sync, err, SolveIO<T>{b, lv.lower.bmap.get(), 0, qL, nullptr, yp, qU, nf}, s,
                                 skip);
            launch_blk<T, true>(lv.upper, sync + 2, err, SolveIO<T>{yp, nullptr, 0, qU, nullptr, x, qL, nf}, s, skip);
        } else {
            launch_blk<T, false>(lv.lower, sync, err, SolveIO<T>{b, nullptr, 1, qL, nullptr, yp, qU, nf}, s, skip);
            launch_blk<T, true>(lv.upper, sync + 2, err, SolveIO<T>{yp, nullptr, 0, qU, x, nullptr, qL, nf}, s, skip);
        }
        return;
    }
    // one triangle: qU, free between calls, holds the polled copy; qL keeps its fill
    k_trsv_fill<T><<<ceil_div(nf, 256), 256, 0, s>>>(nf, qU, skip);
    HEC_CHECK_LAUNCH();
    if (which == HEC_LOWER)
        launch_blk<T, false>(lv.lower, sync, err, SolveIO<T>{b, nullptr, 1, qU, x, nullptr, nullptr, 0}, s, skip);
    else
        launch_blk<T, true>(lv.upper, sync + 2, err, SolveIO<T>{b, nullptr, 1, qU, x, nullptr, nullptr, 0}, s, skip);
}

void trsv_init_levels(hec_levels_s &lv, hipStream_t s) {
    const int64_t n = lv.nf;
    if (n == 0) return;
    k_trsv_fill<double><<<ceil_div(n, 256), 256, 0, s>>>(n, lv.qL64.get(), nullptr);
    HEC_CHECK_LAUNCH();
    if (lv.qL32.get()) {
        k_trsv_fill<float><<<ceil_div(n, 256), 256, 0, s>>>(n, lv.qL32.get(), nullptr);
        HEC_CHECK_LAUNCH();
    }
    const int64_t nface = lv.fL64.get() ? lv.lower.grid.face_elems() : 0;
    if (nface) {
        k_trsv_fill<double><<<ceil_div(nface, 256), 256, 0, s>>>(nface, lv.fL64.get(), nullptr);
        HEC_CHECK_LAUNCH();
        if (lv.fL32.get()) {
            k_trsv_fill<float><<<ceil_div(nface, 256), 256, 0, s>>>(nface, lv.fL32.get(), nullptr);
            HEC_CHECK_LAUNCH();
        }
    }
}

void level_only(const hec_ilu_s &M, bool upper, hec_tri &tri) {
    tri.nlev = plan::compute_levels(M.n, M.hLUp.data(), M.hLUj.data(), M.hdiag.data(), upper, tri.hlevel_ptr,
                                    tri.hperm);
}

void build_grid(const hec_ilu_s &M, bool upper, hec_grid &g, hipStream_t s) {
    g = hec_grid();
    plan::GridPlan P;
    if (!plan::make_grid_plan(M.n, M.hLUp.data(), M.hLUj.data(), M.hdiag.data(), M.gnx, M.gny, M.gnz, upper, P))
        return;
    g.TA = P.TA;
    g.NA = P.NA;
    g.NB = P.NB;
    g.NC = P.NC;
    g.PA = P.PA;
    g.PB = P.PB;
    g.S = P.S;
    g.sa = P.sa;
    g.sb = P.sb;
    g.sc = P.sc;
    const size_t m = P.src.size();
    DevBuf<int32_t> dsrc(m);
    dsrc.upload(P.src.data(), m, s);
    g.coef.alloc(m);
    k_grid_coef<double><<<ceil_div(m, 256), 256, 0, s>>>(m, P.ncoef, dsrc.get(), M.LUx.get(), g.coef.get());
    HEC_CHECK_LAUNCH();
    if (M.has_f32) {
        g.coef32.alloc(m);
        k_grid_coef<float><<<ceil_div(m, 256), 256, 0, s>>>(m, P.ncoef, dsrc.get(), M.LUx.get(), g.coef32.get());
        HEC_CHECK_LAUNCH();
    }
    HEC_HIP(hipStreamSynchronize(s));  // dsrc and the host map end here
    g.on = true;
}

template void trsv_launch<double>(const hec_levels_s &, uint32_t, const double *, double *, hipStream_t,
                                  const int32_t *);
template void trsv_launch<float>(const hec_levels_s &, uint32_t, const float *, float *, hipStream_t,
                                 const int32_t *);

void build_tri(const hec_ilu_s &M, bool upper, hec_tri &tri, const hec_tri *upper_plan, hipStream_t s) {
    const int32_t n = M.n;
    plan::HostPlan P;
    plan::make_plan(n, M.hLUp.data(), M.hLUj.data(), M.hdiag.data(), M.gnx, M.gny, M.gnz, upper, M.has_f32,
                    max_lds_per_block() - 256, P, false, M.hblocks.empty() ? nullptr : &M.hblocks);
    tri.nlev = P.nlev;
    tri.hlevel_ptr = std::move(P.level_ptr);
    tri.hperm = std::move(P.perm);
    tri.K = P.K;
    tri.KC = P.KC;
    tri.ldq = P.ldq;
    if (n == 0) return;
    tri.blocked = P.blocked;
    tri.nparts = P.nparts;
    tri.nss = P.nss;
    tri.W = P.W;
    tri.S = P.S;
    tri.D64 = P.D64;
    tri.D32 = P.D32;
    tri.lds64 = P.lds64;
    tri.lds32 = P.lds32;
    if (!P.blocked) {
        tri.nchunks = (int32_t)P.chunks.size() - 1;
        tri.chunk_ptr.alloc(P.chunks.size());
        tri.chunk_ptr.upload(P.chunks.data(), P.chunks.size(), s);
    }
    tri.part_ss.alloc(P.part_ss.size());
    tri.part_ss.upload(P.part_ss.data(), P.part_ss.size(), s);
    tri.part_pos.alloc(P.part_pos.size());
    tri.part_pos.upload(P.part_pos.data(), P.part_pos.size(), s);
    tri.ss_pos.alloc(P.ss_pos.size());
    tri.ss_pos.upload(P.ss_pos.data(), P.ss_pos.size(), s);
    tri.NS = P.NS;
    if (!P.ss_need.empty()) {
        tri.ss_need.alloc(P.ss_need.size());
        tri.ss_need.upload(P.ss_need.data(), P.ss_need.size(), s);
    }
    tri.grow.alloc(n);
    tri.grow.upload(P.grow.data(), n, s);
    const bool ras = !M.hext_row.empty();
    if (ras && !upper) {  // right-hand side of each position: the system row of its stacked row
        std::vector<int32_t> bm(n);
        for (int32_t q = 0; q < n; ++q) bm[q] = M.hext_row[P.grow[q]];
        tri.bmap.alloc(n);
        tri.bmap.upload(bm.data(), n, s);
        HEC_HIP(hipStreamSynchronize(s));
    }
    if (ras && upper) {  // owned rows write their result to the system vector, overlap rows nowhere
        std::vector<int32_t> om(n);
        for (int32_t q = 0; q < n; ++q) {
            const int32_t row = P.grow[q], sys = M.hext_row[row];
            om[q] = M.hown[sys] == row ? sys : -1;
        }
        tri.other.alloc(n);
        tri.other.upload(om.data(), n, s);
        HEC_HIP(hipStreamSynchronize(s));
    }
    if (!upper && upper_plan) {
        // position of each lower-plan row in the upper plan
        std::vector<int32_t> up_pos(n), other(n);
        for (int32_t q = 0; q < n; ++q) up_pos[upper_plan->hgrow[q]] = q;
        for (int32_t q = 0; q < n; ++q) other[q] = up_pos[P.grow[q]];
        tri.other.alloc(n);
        tri.other.upload(other.data(), n, s);
        HEC_HIP(hipStreamSynchronize(s));  // `other` is uploaded from host memory that ends here
    }
    const size_t slab = (size_t)P.K * P.ldq;
    tri.enc.alloc(slab);
    tri.enc.upload(P.enc.data(), slab, s);
    tri.val.alloc(slab);
    if (M.has_f32) tri.val32.alloc(slab);
    DevBuf<int32_t> dsrc(slab);
    if (slab) {
        dsrc.upload(P.src.data(), slab, s);
        k_gather<<<ceil_div(slab, 256), 256, 0, s>>>(slab, dsrc.get(), M.LUx.get(), tri.val.get(), tri.val32.get());
        HEC_CHECK_LAUNCH();
    }
    DevBuf<int32_t> dp;
    if (upper) {
        tri.piv.alloc(tri.ldq);
        if (M.has_f32) tri.piv32.alloc(tri.ldq);
        dp.alloc(tri.ldq);
        dp.upload(P.psrc.data(), tri.ldq, s);
        k_gather<<<ceil_div(tri.ldq, 256), 256, 0, s>>>(tri.ldq, dp.get(), M.LUx.get(), tri.piv.get(),
                                                        tri.piv32.get());
        HEC_CHECK_LAUNCH();
    }
    HEC_HIP(hipStreamSynchronize(s));
    tri.hgrow = std::move(P.grow);
}

void build_flat(const hec_ilu_s &M, bool upper, hec_tri &tri, hipStream_t s) {
    const int32_t n = M.n;
    plan::HostPlan P;
    plan::make_plan(n, M.hLUp.data(), M.hLUj.data(), M.hdiag.data(), 0, 0, 0, upper, M.has_f32, 0, P, true);
    hec_flat &f = tri.flat;
    f.K = P.K;
    f.ldq = P.ldq;
    f.nchunks = n ? (int32_t)P.chunks.size() - 1 : 0;
    if (n == 0) return;
    f.chunk_ptr.alloc(P.chunks.size());
    f.chunk_ptr.upload(P.chunks.data(), P.chunks.size(), s);
    f.row.alloc(n);
    f.row.upload(P.grow.data(), n, s);
    const size_t slab = (size_t)P.K * P.ldq;
    f.col.alloc(slab);
    f.col.upload(P.enc.data(), slab, s);
    f.val.alloc(slab);
    if (M.has_f32) f.val32.alloc(slab);
    DevBuf<int32_t> dsrc(slab);
    if (slab) {
        dsrc.upload(P.src.data(), slab, s);
        k_gather<<<ceil_div(slab, 256), 256, 0, s>>>(slab, dsrc.get(), M.LUx.get(), f.val.get(), f.val32.get());
        HEC_CHECK_LAUNCH();
    }
    DevBuf<int32_t> dp;
    if (upper) {
        f.piv.alloc(P.ldq);
        if (M.has_f32) f.piv32.alloc(P.ldq);
        dp.alloc(P.ldq);
        dp.upload(P.psrc.data(), P.ldq, s);
        k_gather<<<ceil_div(P.ldq, 256), 256, 0, s>>>(P.ldq, dp.get(), M.LUx.get(), f.piv.get(), f.piv32.get());
        HEC_CHECK_LAUNCH();
    }
    HEC_HIP(hipStreamSynchronize(s));
}

}  // namespace hec

// Host-side planning of the level-scheduled triangular solves (Sec. 2.6,
// Eq. (11), Alg. 3): levels, grid recognition, and the blocked execution plan.
// Pure C++ (no HIP): the GPU library builds its plans with it, and a CPU-only
// checker library built from the same header lets the plan be verified without
// a GPU.
#pragma once

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <vector>

#if defined(__HIPCC__)
#define HEC_HD __host__ __device__
#else
#define HEC_HD
#endif

namespace hec {
namespace plan {

constexpr int kSub = 64;          // rows per sub-segment (one solver wavefront)
constexpr int kPad = INT_MIN;     // padding entry of a row shorter than K
// Partitioning parameters (overridable at compile time for tuning sweeps).
#ifndef HEC_TRSV_TARGET_PARTS
#define HEC_TRSV_TARGET_PARTS 64
#endif
#ifndef HEC_TRSV_MIN_PART_ROWS
#define HEC_TRSV_MIN_PART_ROWS 4096
#endif
#ifndef HEC_TRSV_TILE_PARTS
#define HEC_TRSV_TILE_PARTS 256
#endif
#ifndef HEC_TRSV_MAX_RING
#define HEC_TRSV_MAX_RING 32
#endif
#ifndef HEC_TRSV_SOLVERS
#define HEC_TRSV_SOLVERS 2
#endif
#ifndef HEC_TRSV_TILE
#define HEC_TRSV_TILE 0
#endif
#ifndef HEC_TRSV_SHEAR
#define HEC_TRSV_SHEAR 1  // 0: grid tiles on the x-y axes only (sheared axes off)
#endif
constexpr int kTargetParts = HEC_TRSV_TARGET_PARTS;  // contiguous parts: about this many ...
constexpr int kMinPartRows = HEC_TRSV_MIN_PART_ROWS;  // ... of at least this many rows
constexpr int kTileParts = HEC_TRSV_TILE_PARTS;      // grid tiles: at most about this many
constexpr int kMaxRing = HEC_TRSV_MAX_RING;          // most LDS slots in the ring
constexpr int kMaxSolvers = 8;                       // solver wavefronts per workgroup: 1, 2, 4 or 8 ...
constexpr int kSolvers = HEC_TRSV_SOLVERS;           // ... the kernels are built for (the planner's default)
constexpr int kTile = HEC_TRSV_TILE;                 // grid tile side (0: the planner chooses)
static_assert(kSolvers == 1 || kSolvers == 2 || kSolvers == 4 || kSolvers == 8, "solver count");

HEC_HD constexpr size_t align16(size_t b) { return (b + 15) / 16 * 16; }

// Byte offsets inside one LDS slot (64 rows of one sub-segment, KC entries per
// row: the row's entries padded to a compile-time width).
template <class T, bool UPPER>
struct Slot {
    int KC;
    HEC_HD size_t b() const { return 0; }                                       // T[64]
    HEC_HD size_t xe() const { return b() + kSub * sizeof(T); }                 // T[KC][64]
    HEC_HD size_t v() const { return xe() + (size_t)KC * kSub * sizeof(T); }    // T[KC][64]
    HEC_HD size_t d() const { return v() + (size_t)KC * kSub * sizeof(T); }     // T[64] (U: 1 / u_ii)
    HEC_HD size_t a() const { return d() + (UPPER ? kSub * sizeof(T) : 0); }    // int[KC][64]
    HEC_HD size_t bytes() const { return align16(a() + (size_t)KC * kSub * sizeof(int)); }
};

// LDS: [done[kMaxSolvers] | filled[D] | part | abort | zero (16 B)] [part's
//      sub-segment starts, S+1] [their dependency bounds, S+1, with NS > 1 only]
//      [ring of recent results, W] [D slots]
HEC_HD inline size_t ctrl_head(int D) { return align16((size_t)(kMaxSolvers + D + 2) * sizeof(int)) + 16; }
HEC_HD inline size_t ss_bytes(int S) { return align16((size_t)(S + 1) * sizeof(int)); }
HEC_HD inline size_t ctrl_bytes(int D, int S, int NS) { return ctrl_head(D) + (NS > 1 ? 2 : 1) * ss_bytes(S); }

template <class T, bool UPPER>
size_t lds_bytes(int KC, int W, int D, int S, int NS) {
    return ctrl_bytes(D, S, NS) + align16((size_t)W * sizeof(T)) + (size_t)D * Slot<T, UPPER>{KC}.bytes();
}

// Eq. (11): level of each row, 0-based, for the strict lower (upper == false)
// or strict upper triangle of a pattern with known diagonal positions, then
// Alg. 3's grouping: level_ptr and perm with rows ascending inside each level
// (stable counting sort). Returns the number of levels.
inline int32_t compute_levels(int32_t n, const int32_t *LUp, const int32_t *LUj, const int32_t *diag, bool upper,
                              std::vector<int32_t> &level_ptr, std::vector<int32_t> &perm,
                              std::vector<int32_t> *lev_out = nullptr) {
    std::vector<int32_t> lev(n);
    int32_t nlev = 0;
    if (!upper) {
        for (int32_t i = 0; i < n; ++i) {
            int32_t l = 0;
            for (int32_t e = LUp[i]; e < diag[i]; ++e) l = std::max(l, lev[LUj[e]] + 1);
            lev[i] = l;
            nlev = std::max(nlev, l + 1);
        }
    } else {
        for (int32_t i = n - 1; i >= 0; --i) {
            int32_t l = 0;
            for (int32_t e = diag[i] + 1; e < LUp[i + 1]; ++e) l = std::max(l, lev[LUj[e]] + 1);
            lev[i] = l;
            nlev = std::max(nlev, l + 1);
        }
    }
    level_ptr.assign(nlev + 1, 0);
    for (int32_t i = 0; i < n; ++i) level_ptr[lev[i] + 1]++;
    for (int32_t l = 0; l < nlev; ++l) level_ptr[l + 1] += level_ptr[l];
    std::vector<int32_t> next(level_ptr.begin(), level_ptr.end() - 1);
    perm.resize(n);
    for (int32_t i = 0; i < n; ++i) perm[next[lev[i]]++] = i;
    if (lev_out) lev_out->swap(lev);
    return nlev;
}

// Recognises a natural-order 5- or 7-point stencil (cell x + nx*(y + ny*z)):
// the strictly lower entries of A have offsets i - j in {1, nx, nx*ny} only,
// with exactly the counts such a grid gives. The answer only steers how the
// triangular solves are partitioned (a performance choice; any answer is correct).
inline void detect_grid(int32_t n, const int32_t *Ap, const int32_t *Aj, int32_t &nx, int32_t &ny, int32_t &nz) {
    nx = ny = nz = 0;
    int64_t off[3] = {0, 0, 0}, cnt[3] = {0, 0, 0};
    int nd = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t e = Ap[i]; e < Ap[i + 1] && Aj[e] < i; ++e) {
            int64_t d = (int64_t)i - Aj[e];
            int k = 0;
            while (k < nd && off[k] != d) ++k;
            if (k == nd) {
                if (nd == 3) return;
                off[nd++] = d;
            }
            cnt[k]++;
        }
    }
    for (int a = 0; a < nd; ++a)
        for (int b = a + 1; b < nd; ++b)
            if (off[b] < off[a]) {
                std::swap(off[a], off[b]);
                std::swap(cnt[a], cnt[b]);
            }
    if (nd < 2 || off[0] != 1) return;
    if (nd == 3 && off[2] % off[1] != 0) return;
    int64_t X = off[1], Y = nd == 3 ? off[2] / off[1] : (int64_t)n / off[1];
    int64_t plane = X * Y;
    if (plane <= 0 || n % plane != 0) return;
    int64_t Z = n / plane;
    if (cnt[0] != (X - 1) * Y * Z || cnt[1] != X * (Y - 1) * Z) return;
    if (nd == 3 && cnt[2] != X * Y * (Z - 1)) return;
    if (nd == 2 && Z != 1) return;
    nx = (int32_t)X;
    ny = (int32_t)Y;
    nz = (int32_t)Z;
}

// Tile axes of a grid triangle: two combinations a = ca . (x, y, z), b = cb . (x, y, z)
// with coefficients in 0..cmax such that every dependency of the triangle sits at a
// and b no larger (lower triangle; no smaller for the upper one). Tiles T wide in a
// and in b, numbered b-tile major, then never wait on a later tile. Among the valid
// pairs, the one whose tiles (at about `target` of them) are crossed least often by a
// path through the grid: about (range_a + range_b) / T boundaries, T = sqrt(count /
// target) with `count` the (a, b) pairs that hold a cell (ranked by the bound
// min((range_a + 1)(range_b + 1), n), counted exactly for the chosen pair). For ILU(0) of a 7-point
// stencil this is (x, y), the x-y pencils; ILU(1) fill (row x depends on x + 1 in
// the plane below) rules x-y pencils out, and a sheared pair such as (x + y + z, z)
// takes over. Returns false when no pair is valid.
struct TileAxes {
    int ca[3] = {1, 0, 0}, cb[3] = {0, 1, 0};
    int32_t T = 1;
    int64_t ra = 0, rb = 0;  // largest a and b on the grid (both start at 0)
};

inline bool choose_tile_axes(int32_t n, const int32_t *LUp, const int32_t *LUj, const int32_t *diag, int32_t gnx,
                             int32_t gny, int32_t gnz, bool upper, int64_t target, TileAxes &best) {
    // the triangle's dependency offsets (dx, dy, dz), each once: the distinct index
    // offsets j - i first, each with a row that has it (a grid factor's entries join
    // grid neighbours, so an index offset stands for one grid offset)
    std::vector<std::pair<int32_t, int32_t>> off;  // (j - i, i)
    for (int32_t i = 0; i < n; ++i) {
        const int32_t a = upper ? diag[i] + 1 : LUp[i], b = upper ? LUp[i + 1] : diag[i];
        for (int32_t e = a; e < b; ++e) {
            const int32_t o = LUj[e] - i;
            bool have = false;
            for (const auto &w : off) have = have || w.first == o;
            if (!have) {
                if (off.size() >= 256) return false;
                off.push_back({o, i});
            }
        }
    }
    std::vector<std::array<int, 3>> D;
    for (const auto &w : off) {
        const int32_t i = w.second, j = i + w.first;
        const std::array<int, 3> d{j % gnx - i % gnx, (j / gnx) % gny - (i / gnx) % gny,
                                   j / (gnx * gny) - i / (gnx * gny)};
        if (std::find(D.begin(), D.end(), d) == D.end()) D.push_back(d);
    }
    const int sg = upper ? -1 : 1;
    double best_score = 0.0;
    bool found = false;
    for (int cmax = 1; cmax <= 2 && !found; ++cmax) {
        std::vector<std::array<int, 3>> C;  // valid coefficient vectors, (1,0,0) and (0,1,0) first
        for (int c2 = 0; c2 <= cmax; ++c2)
            for (int c1 = 0; c1 <= cmax; ++c1)
                for (int c0 = 0; c0 <= cmax; ++c0) {
                    if (!c0 && !c1 && !c2) continue;
                    if (!HEC_TRSV_SHEAR && c0 + c1 + c2 != 1) continue;
                    bool ok = true;
                    for (const auto &d : D) ok = ok && sg * (c0 * d[0] + c1 * d[1] + c2 * d[2]) <= 0;
                    if (ok) C.push_back({c0, c1, c2});
                }
        for (size_t u = 0; u < C.size(); ++u)
            for (size_t v = u + 1; v < C.size(); ++v) {
                const auto &p = C[u], &q = C[v];
                const int64_t cx = (int64_t)p[1] * q[2] - (int64_t)p[2] * q[1],
                              cy = (int64_t)p[2] * q[0] - (int64_t)p[0] * q[2],
                              cz = (int64_t)p[0] * q[1] - (int64_t)p[1] * q[0];
                if (!cx && !cy && !cz) continue;  // parallel: not two axes
                const int64_t ra = (int64_t)p[0] * (gnx - 1) + (int64_t)p[1] * (gny - 1) + (int64_t)p[2] * (gnz - 1);
                const int64_t rb = (int64_t)q[0] * (gnx - 1) + (int64_t)q[1] * (gny - 1) + (int64_t)q[2] * (gnz - 1);
                const double bound = (double)std::min<int64_t>((ra + 1) * (rb + 1), n);
                const double score = (double)(ra + rb) / std::max(1.0, std::sqrt(bound / (double)target));
                if (!found || score < best_score) {
                    found = true;
                    best_score = score;
                    for (int k = 0; k < 3; ++k) {
                        best.ca[k] = p[k];
                        best.cb[k] = q[k];
                    }
                    best.ra = ra;
                    best.rb = rb;
                }
            }
    }
    if (!found) return false;
    // the (a, b) pairs that hold a cell, for the tile side
    std::vector<uint8_t> seen((size_t)((best.ra + 1) * (best.rb + 1)), 0);
    int64_t count = 0;
    for (int32_t z = 0; z < gnz; ++z)
        for (int32_t y = 0; y < gny; ++y)
            for (int32_t x = 0; x < gnx; ++x) {
                const int64_t a = (int64_t)best.ca[0] * x + (int64_t)best.ca[1] * y + (int64_t)best.ca[2] * z;
                const int64_t b = (int64_t)best.cb[0] * x + (int64_t)best.cb[1] * y + (int64_t)best.cb[2] * z;
                uint8_t &f = seen[(size_t)(a * (best.rb + 1) + b)];
                count += !f;
                f = 1;
            }
    best.T = (int32_t)std::max<int64_t>(1, std::lround(std::sqrt((double)count / (double)target)));
    return true;
}

// Tile side for the chosen axes. A path through the triangle runs through every
// level; inside a tile a level takes ceil(rows / kSub) solver steps, and each tile
// boundary the path crosses, about (ra + rb) / T of them, costs about kHopSteps
// steps more (a result handed between workgroups arrives some eight solver steps
// after it was solved, measured at 128^3, one of which overlaps). Sides from
// tmax down are tried, tmax the side that gives about `target` tiles (fewer tiles
// would idle workgroups), while the hops alone still beat the best cost so far.
constexpr int kHopSteps = 7;

inline int32_t choose_tile_side(int32_t n, const std::vector<int32_t> &lev, int32_t nlev, const std::vector<int32_t> &ga,
                                const std::vector<int32_t> &gb, const TileAxes &ax, int32_t tmax) {
    int32_t best = std::max<int32_t>(1, tmax);
    double best_cost = 0.0;
    std::vector<int32_t> lo, hi, cnt;
    std::vector<int64_t> off;
    for (int32_t T = best; T >= std::max<int32_t>(1, tmax / 4); --T) {
        const double hops = (double)(ax.ra + ax.rb) / T;
        if (T < best && nlev + kHopSteps * hops >= best_cost) break;
        const int64_t PA = ax.ra / T + 1, PB = ax.rb / T + 1, nt = PA * PB;
        lo.assign((size_t)nt, INT_MAX);
        hi.assign((size_t)nt, -1);
        for (int32_t i = 0; i < n; ++i) {
            const int64_t t = ga[i] / T + PA * (gb[i] / T);
            lo[(size_t)t] = std::min(lo[(size_t)t], lev[i]);
            hi[(size_t)t] = std::max(hi[(size_t)t], lev[i]);
        }
        off.assign((size_t)nt + 1, 0);
        for (int64_t t = 0; t < nt; ++t) off[(size_t)t + 1] = off[(size_t)t] + (hi[(size_t)t] >= 0 ? hi[(size_t)t] - lo[(size_t)t] + 1 : 0);
        if (off[(size_t)nt] > 8 * (int64_t)n) continue;  // levels scattered over the tiles: not a candidate
        cnt.assign((size_t)off[(size_t)nt], 0);
        for (int32_t i = 0; i < n; ++i) {
            const int64_t t = ga[i] / T + PA * (gb[i] / T);
            ++cnt[(size_t)(off[(size_t)t] + lev[i] - lo[(size_t)t])];
        }
        int64_t groups = 0, steps = 0;
        for (int32_t c : cnt)
            if (c) {
                ++groups;
                steps += (c + kSub - 1) / kSub;
            }
        const double cost = (double)nlev * (double)steps / (double)std::max<int64_t>(1, groups) + kHopSteps * hops;
        if (T == tmax || cost < best_cost) {
            best = T;
            best_cost = cost;
        }
    }
    return best;
}

// The blocked execution plan of one triangle.
//  * Parts: with a recognised grid, tiles of two axes (choose_tile_axes: x-y
//    pencils spanning all z for ILU(0), sheared prisms for fill), about
//    kTileParts of them, numbered in the order the triangle is solved, kept only
//    if every dependency then lies in the same or an earlier part; otherwise
//    contiguous row ranges in that order. Parts are claimed in order at run time.
//  * Positions: each part's rows at consecutive positions, by (level, row).
//  * Sub-segments: runs of one level inside a part, at most kSub rows.
//  * enc[s*ldq + q]: the dependency of entry s of position q: -(local position
//    + 1) inside the part, its position outside it (its row in a flat plan),
//    kPad for padding.
//  * NS: solver wavefronts per workgroup. With NS > 1 they take a part's
//    sub-segments round-robin, and sub-segment t starts once every sub-segment
//    of its part below ss_need[t] (relative to the part's first one, one past
//    the last holding a dependency of t) is solved. NS > 1 is chosen when a
//    part's levels span several sub-segments on average.
//  * W: size of the ring of recent results, a power of two that spans the
//    longest distance from a row to an in-part dependency, plus kSub; with
//    NS > 1 also wide enough that the results of a sub-segment never replace
//    an entry that a sub-segment which may still run reads.
//  * D64/D32: LDS ring depth for the FP64/FP32 solves; 0 when the plan does not
//    fit in LDS (more than 32 entries per row): then blocked == false and the
//    solve polls every dependency (level-order positions in 64-row chunks).
//    flat == true asks for that level-order layout directly.
struct HostPlan {
    int32_t n = 0, nlev = 0, K = 0, KC = 4, ldq = 0, nparts = 0, nss = 0, W = 64, S = 0, D64 = 0, D32 = 0, NS = 1;
    bool blocked = false;
    size_t lds64 = 0, lds32 = 0;
    std::vector<int32_t> level_ptr, perm, lev;
    std::vector<int32_t> part_ss, part_pos, ss_pos, ss_need, grow, part_of, pos, chunks;
    std::vector<int32_t> enc, src, psrc;  // src/psrc: index into the factor's value array
};

inline void make_plan(int32_t n, const int32_t *LUp, const int32_t *LUj, const int32_t *diag, int32_t gnx,
                      int32_t gny, int32_t gnz, bool upper, bool has_f32, int64_t lds_max, HostPlan &P,
                      bool flat = false, const std::vector<int32_t> *blocks = nullptr, int solvers = kSolvers,
                      int32_t tile = 0) {
    P = HostPlan();
    P.n = n;
    P.nlev = compute_levels(n, LUp, LUj, diag, upper, P.level_ptr, P.perm, &P.lev);
    int32_t K = 0;
    for (int32_t i = 0; i < n; ++i) K = std::max(K, upper ? LUp[i + 1] - diag[i] - 1 : diag[i] - LUp[i]);
    P.K = K;
    P.KC = K <= 4 ? 4 : K <= 8 ? 8 : K <= 16 ? 16 : 32;
    P.ldq = (int32_t)(((int64_t)n + 63) / 64 * 64);
    if (n == 0) return;
    auto deps = [&](int32_t i, int32_t &a, int32_t &b) {
        a = upper ? diag[i] + 1 : LUp[i];
        b = upper ? LUp[i + 1] : diag[i];
    };

    std::vector<int32_t> &part_of = P.part_of, &pos = P.pos, &grow = P.grow;
    part_of.assign(n, 0);
    pos.assign(n, 0);
    grow.assign(n, 0);
    if (!flat) {  // flat: level order only (the layout of the per-row polling solves)
        int64_t R = std::max<int64_t>(kMinPartRows, (n + kTargetParts - 1) / kTargetParts);
        R = std::min<int64_t>(R, n);
        bool tiled = false;
        int32_t ntiles = 0;
        // explicit blocks (rows blocks[b] .. blocks[b+1]-1, no dependency between blocks): enough
        // of them make independent parts -- one block per part, or consecutive blocks grouped so
        // that about kTileParts parts remain (grouped blocks share sub-segments level by level);
        // a few large blocks are cut like any factor
        const int32_t nbk = blocks && blocks->size() >= 2 && blocks->back() == n ? (int32_t)blocks->size() - 1 : 0;
        const bool by_block = nbk >= kTileParts / 8;
        if (by_block) {
            const int32_t group = (nbk + kTileParts - 1) / kTileParts;
            ntiles = (nbk + group - 1) / group;
            for (int32_t b = 0; b < nbk; ++b) {
                const int32_t t = b / group;
                for (int32_t i = (*blocks)[b]; i < (*blocks)[b + 1]; ++i) part_of[i] = upper ? ntiles - 1 - t : t;
            }
            tiled = true;
            for (int32_t i = 0; i < n && tiled; ++i) {
                int32_t a, b2;
                deps(i, a, b2);
                for (int32_t e = a; e < b2; ++e)
                    if (part_of[LUj[e]] > part_of[i]) {
                        tiled = false;
                        break;
                    }
            }
        } else if (gnx > 0 && (int64_t)gnx * gny * gnz == n && n >= 2 * kMinPartRows) {
            const int64_t target = std::min<int64_t>(kTileParts, n / kMinPartRows);
            TileAxes ax;
            if (choose_tile_axes(n, LUp, LUj, diag, gnx, gny, gnz, upper, target, ax)) {
                // each row's coordinates on the two axes
                std::vector<int32_t> ga(n), gb(n);
                for (int32_t i = 0; i < n; ++i) {
                    const int64_t xx = i % gnx, yy = (i / gnx) % gny, zz = i / ((int64_t)gnx * gny);
                    ga[i] = (int32_t)(ax.ca[0] * xx + ax.ca[1] * yy + ax.ca[2] * zz);
                    gb[i] = (int32_t)(ax.cb[0] * xx + ax.cb[1] * yy + ax.cb[2] * zz);
                }
                // no wider than the part count allows: wider tiles hold levels of more than
                // kSub rows and lengthen each tile's lead on its neighbours (measured slower
                // at 128^3 ILU(0)); narrower where the steps saved outweigh the extra hops
                // (sheared ILU(1) tiles: 8 instead of 17 at 192^3, measured)
                const int32_t T = tile > 0 ? tile : kTile > 0 ? kTile : choose_tile_side(n, P.lev, P.nlev, ga, gb, ax, ax.T);
                const int64_t PA = ax.ra / T + 1, PB = ax.rb / T + 1;
                // tile index b-major, then empty tiles dropped (numbering kept in order)
                std::vector<int32_t> tid((size_t)(PA * PB), -1);
                for (int32_t i = 0; i < n; ++i) {
                    const int64_t t = ga[i] / T + PA * (gb[i] / T);
                    part_of[i] = (int32_t)t;
                    tid[(size_t)t] = 0;
                }
                for (size_t t = 0; t < tid.size(); ++t)
                    if (tid[t] == 0) tid[t] = ntiles++;
                for (int32_t i = 0; i < n; ++i) {
                    const int32_t t = tid[(size_t)part_of[i]];
                    part_of[i] = upper ? ntiles - 1 - t : t;
                }
                tiled = ntiles > 1;
            }
            for (int32_t i = 0; i < n && tiled; ++i) {
                int32_t a, b;
                deps(i, a, b);
                for (int32_t e = a; e < b; ++e)
                    if (part_of[LUj[e]] > part_of[i]) {
                        tiled = false;
                        break;
                    }
            }
        }
        for (;;) {
            int32_t nparts;
            if (tiled) {
                nparts = ntiles;
            } else {
                nparts = (int32_t)((n + R - 1) / R);
                for (int32_t i = 0; i < n; ++i) part_of[i] = (int32_t)((upper ? (int64_t)(n - 1 - i) : (int64_t)i) / R);
            }
            P.part_pos.assign(nparts + 1, 0);
            for (int32_t i = 0; i < n; ++i) P.part_pos[part_of[i] + 1]++;
            for (int32_t p = 0; p < nparts; ++p) P.part_pos[p + 1] += P.part_pos[p];
            std::vector<int32_t> fillp(P.part_pos.begin(), P.part_pos.end() - 1);
            for (int32_t t = 0; t < n; ++t) {
                int32_t i = P.perm[t];
                int32_t q = fillp[part_of[i]]++;
                pos[i] = q;
                grow[q] = i;
            }
            P.part_ss.assign(nparts + 1, 0);
            P.ss_pos.clear();
            for (int32_t p = 0; p < nparts; ++p) {
                P.part_ss[p] = (int32_t)P.ss_pos.size();
                int32_t q = P.part_pos[p];
                while (q < P.part_pos[p + 1]) {
                    P.ss_pos.push_back(q);
                    int32_t l = P.lev[grow[q]];
                    int32_t e = q + 1;
                    while (e < P.part_pos[p + 1] && e - q < kSub && P.lev[grow[e]] == l) ++e;
                    q = e;
                }
            }
            P.part_ss[nparts] = (int32_t)P.ss_pos.size();
            P.ss_pos.push_back(n);
            const int32_t nss = (int32_t)P.ss_pos.size() - 1;
            std::vector<int32_t> ss_of(n);
            for (int32_t t = 0; t < nss; ++t)
                for (int32_t q = P.ss_pos[t]; q < P.ss_pos[t + 1]; ++q) ss_of[q] = t;
            // in-part dependencies: longest distance, and per sub-segment the dependency
            // bound and the lowest position read
            P.ss_need.assign(nss, 0);
            std::vector<int32_t> mindep(nss, INT_MAX);
            int64_t maxd = 0;
            for (int32_t i = 0; i < n; ++i) {
                int32_t a, b;
                deps(i, a, b);
                const int32_t t = ss_of[pos[i]], t0 = P.part_ss[part_of[i]];
                for (int32_t e = a; e < b; ++e) {
                    int32_t j = LUj[e];
                    if (part_of[j] != part_of[i]) continue;
                    maxd = std::max<int64_t>(maxd, (int64_t)pos[i] - pos[j]);
                    P.ss_need[t] = std::max(P.ss_need[t], ss_of[pos[j]] - t0 + 1);
                    mindep[t] = std::min(mindep[t], pos[j]);
                }
            }
            int64_t groups = 0;  // (part, level) pairs
            for (int32_t p = 0; p < nparts; ++p)
                for (int32_t t = P.part_ss[p]; t < P.part_ss[p + 1]; ++t)
                    if (t == P.part_ss[p] || P.lev[grow[P.ss_pos[t]]] != P.lev[grow[P.ss_pos[t - 1]]]) ++groups;
            P.NS = solvers > 1 && 2 * (int64_t)nss >= 3 * groups ? solvers : 1;
            int64_t span = maxd + kSub;
            if (P.NS > 1) {
                // sub-segment t starts when all below its bound are solved, so those from
                // the bound up to t - 1 may still run and read down to their lowest
                // dependency: t's results must not wrap onto it (range minima by a sparse table)
                std::vector<std::vector<int32_t>> mn(1, mindep);
                for (int32_t h = 1; (2 << (h - 1)) <= nss; ++h) {
                    const std::vector<int32_t> &lo = mn[h - 1];
                    std::vector<int32_t> nx(nss - (1 << h) + 1);
                    for (size_t t = 0; t < nx.size(); ++t) nx[t] = std::min(lo[t], lo[t + (1 << (h - 1))]);
                    mn.push_back(std::move(nx));
                }
                for (int32_t p = 0; p < nparts; ++p)
                    for (int32_t t = P.part_ss[p]; t < P.part_ss[p + 1]; ++t) {
                        const int32_t a = P.part_ss[p] + P.ss_need[t];
                        if (a >= t) continue;
                        int h = 0;
                        while ((2 << h) <= t - a) ++h;
                        const int32_t lo = std::min(mn[h][a], mn[h][t - (1 << h)]);
                        if (lo != INT_MAX) span = std::max<int64_t>(span, (int64_t)P.ss_pos[t + 1] - lo);
                    }
            }
            P.W = 64;
            while (P.W < span) P.W *= 2;
            P.S = 0;
            for (int32_t p = 0; p < nparts; ++p) P.S = std::max(P.S, P.part_ss[p + 1] - P.part_ss[p]);
            auto fit = [&](auto tag) {
                using T = decltype(tag);
                int best = 0;
                for (int D = std::max(4, P.NS); D <= kMaxRing; ++D) {
                    size_t bb = upper ? lds_bytes<T, true>(P.KC, P.W, D, P.S, P.NS)
                                      : lds_bytes<T, false>(P.KC, P.W, D, P.S, P.NS);
                    if ((int64_t)bb <= lds_max) best = D;
                }
                return best;
            };
            P.D64 = fit(double());
            P.D32 = has_f32 ? fit(float()) : 4;
            P.nparts = nparts;
            if ((P.D64 >= 4 && P.D32 >= 4) || R <= kSub || K > 32) break;
            tiled = false;                       // fall back to (smaller) contiguous parts
            R = std::max<int64_t>(kSub, R / 2);  // a smaller part keeps the ring of results smaller
        }
        P.blocked = P.D64 >= 4 && P.D32 >= 4 && K <= 32;
    }
    if (!P.blocked) {
        for (int32_t t = 0; t < n; ++t) {
            grow[t] = P.perm[t];
            pos[P.perm[t]] = t;
            part_of[P.perm[t]] = t;
        }
        P.part_pos.assign(2, 0);
        P.part_pos[1] = n;
        P.chunks.assign(1, 0);
        for (int32_t l = 0; l < P.nlev; ++l)
            for (int32_t q = P.level_ptr[l]; q < P.level_ptr[l + 1]; q += kSub)
                P.chunks.push_back(std::min(q + kSub, P.level_ptr[l + 1]));
        P.part_ss.assign(2, 0);
        P.ss_pos.assign(1, 0);
        P.ss_need.clear();
        P.nparts = 0;
        P.NS = 1;
    }
    P.nss = (int32_t)P.ss_pos.size() - 1;
    P.lds64 = upper ? lds_bytes<double, true>(P.KC, P.W, P.D64, P.S, P.NS)
                    : lds_bytes<double, false>(P.KC, P.W, P.D64, P.S, P.NS);
    P.lds32 = upper ? lds_bytes<float, true>(P.KC, P.W, P.D32, P.S, P.NS)
                    : lds_bytes<float, false>(P.KC, P.W, P.D32, P.S, P.NS);
    const size_t slab = (size_t)K * P.ldq;
    P.enc.assign(slab, kPad);
    P.src.assign(slab, -1);
    if (upper) P.psrc.assign(P.ldq, -1);
    for (int32_t q = 0; q < n; ++q) {
        int32_t i = grow[q];
        int32_t a, b;
        deps(i, a, b);
        int32_t pstart = P.blocked ? P.part_pos[part_of[i]] : 0;
        for (int32_t e = a, s2 = 0; e < b; ++e, ++s2) {
            int32_t j = LUj[e];
            P.enc[(size_t)s2 * P.ldq + q] = P.blocked && part_of[j] == part_of[i] ? -(pos[j] - pstart + 1)
                                             : flat                                   ? j
                                                                                      : pos[j];
            P.src[(size_t)s2 * P.ldq + q] = e;
        }
        if (upper) P.psrc[q] = diag[i];
    }
}

// ---------------------------------------------------------------------------
// Wavefront plan of a grid triangle whose every dependency is one of the three grid
// neighbours behind a row (lower: x-1, y-1, z-1; upper: x+1, y+1, z+1), as ILU(0)
// of a 7-point stencil gives (Sec. 2.6: the level of a row is then the sum of its
// coordinates, Eq. (11)).
//
// The grid is cut into tiles of TA x TB columns along two axes (a, b); the columns
// run along the third (c, the longest): 8 x 8 on a 3D grid, 64 x 1 on a 2D grid (b
// is then the unit axis, and a tile is 64 columns side by side). One wavefront takes
// a tile: lane (ma, mb) = (lane % TA, lane / TA) solves its column's rows in order,
// the row at c-index mc at step s = mc + ma + mb.
// The three dependencies of that row were solved one step earlier: the one behind
// it along c by the lane itself, the ones along a and b by lanes (ma - 1, mb) and
// (ma, mb - 1), or, on the tile's low faces, by the tiles before it, which hand the
// values over through face buffers in global memory. The upper triangle runs the
// same schedule in mirrored coordinates (m = TA - 1, TB - 1 - local index along a
// and b, c reversed, tiles claimed in reverse order), so one kernel serves both.
//
// Tiles are claimed in order: claim t is the m-tile (t % PA, t / PA); its
// dependencies lie in claims t - 1 and t - PA, both earlier.
constexpr int kGT = 8;                       // tile side on a 3D grid: kGT * kGT = 64 lanes
constexpr int kGT2 = 64;                     // tile side along a on a 2D grid (64 x 1)
constexpr int kGT2Min = 16;                  // a 2D grid needs this many columns along a
constexpr int kGridCoefLower = 3;            // per lane and step: back (c), below (b), left (a)
constexpr int kGridCoefUpper = 4;            // ... and the reciprocal pivot

struct GridPlan {
    int32_t NA = 0, NB = 0, NC = 0;  // extents along a, b and c
    int64_t sa = 0, sb = 0, sc = 0;  // row strides along a, b and c
    int32_t TA = kGT, TB = kGT;      // tile sides along a and b (TA * TB = 64)
    int32_t PA = 0, PB = 0;          // tiles along a and b
    int32_t S = 0;                   // steps of one tile: NC + (TA - 1) + (TB - 1)
    int32_t ncoef = 0;               // kGridCoefLower or kGridCoefUpper
    // [claim][step][k][lane]: index into the factor's values of coefficient k of the
    // lane's row at that step (k = 3: the pivot, whose reciprocal is used), -1: none
    std::vector<int32_t> src;
    int64_t nclaims() const { return (int64_t)PA * PB; }
};

// Grid coordinates of a claim's lane at a step: false when the lane holds no row then.
// (ta, tb): the tile; (la, lb): the lane's column in it; mc: the c-index in solve order.
struct GridCell {
    int32_t ga, gb, gc;
    bool valid;
};
HEC_HD inline GridCell grid_cell(int32_t NA, int32_t NB, int32_t NC, int32_t PA, int32_t PB, int TA, bool upper,
                                 int64_t claim, int lane, int32_t s) {
    const int TB = 64 / TA;
    const int32_t mta = (int32_t)(claim % PA), mtb = (int32_t)(claim / PA);
    const int32_t ta = upper ? PA - 1 - mta : mta, tb = upper ? PB - 1 - mtb : mtb;
    const int ma = lane % TA, mb = lane / TA;
    const int la = upper ? TA - 1 - ma : ma, lb = upper ? TB - 1 - mb : mb;
    const int32_t mc = s - ma - mb;
    GridCell g;
    g.ga = ta * TA + la;
    g.gb = tb * TB + lb;
    g.gc = upper ? NC - 1 - mc : mc;
    g.valid = g.ga < NA && g.gb < NB && mc >= 0 && mc < NC;
    return g;
}

// Builds the wavefront plan of the strict lower (upper) triangle of the factor pattern
// on the nx x ny x nz grid. Returns false (G untouched) when it does not apply: no
// grid, fewer than kGT columns along a tile axis of a 3D grid (kGT2Min along a of a
// 2D one), or an entry that is not one of the neighbours behind its row.
inline bool make_grid_plan(int32_t n, const int32_t *LUp, const int32_t *LUj, const int32_t *diag, int32_t gnx,
                           int32_t gny, int32_t gnz, bool upper, GridPlan &G) {
    if (gnx <= 0 || gny <= 0 || gnz <= 0 || (int64_t)gnx * gny * gnz != n) return false;
    const int32_t ext[3] = {gnx, gny, gnz};
    const int64_t str[3] = {1, gnx, (int64_t)gnx * gny};
    int c = 2;  // the longest axis runs along the columns (ties: the largest stride)
    for (int k = 1; k >= 0; --k)
        if (ext[k] > ext[c]) c = k;
    const int a = c == 0 ? 1 : 0, b = c == 2 ? 1 : 2;  // the others, by stride
    const bool flat = ext[b] == 1;  // a 2D grid (b the unit axis): tiles of 64 x 1
    if (flat ? ext[a] < kGT2Min : ext[a] < kGT || ext[b] < kGT) return false;
    // every strict-triangle entry must be a neighbour behind the row
    for (int32_t i = 0; i < n; ++i) {
        const int32_t co[3] = {i % gnx, (i / gnx) % gny, i / (gnx * gny)};
        const int32_t e0 = upper ? diag[i] + 1 : LUp[i], e1 = upper ? LUp[i + 1] : diag[i];
        for (int32_t e = e0; e < e1; ++e) {
            const int64_t d = (int64_t)LUj[e] - i;
            bool ok = false;
            for (int k = 0; k < 3 && !ok; ++k) {
                const int64_t want = upper ? str[k] : -str[k];
                ok = d == want && (upper ? co[k] + 1 < ext[k] : co[k] > 0);
            }
            if (!ok) return false;
        }
    }
    GridPlan P;
    P.NA = ext[a];
    P.NB = ext[b];
    P.NC = ext[c];
    P.sa = str[a];
    P.sb = str[b];
    P.sc = str[c];
    P.TA = flat ? kGT2 : kGT;
    P.TB = 64 / P.TA;
    P.PA = (P.NA + P.TA - 1) / P.TA;
    P.PB = (P.NB + P.TB - 1) / P.TB;
    P.S = P.NC + (P.TA - 1) + (P.TB - 1);
    P.ncoef = upper ? kGridCoefUpper : kGridCoefLower;
    const int64_t nc = P.nclaims();
    P.src.assign((size_t)(nc * P.S * P.ncoef * 64), -1);
    const int64_t sg = upper ? 1 : -1;
    for (int64_t t = 0; t < nc; ++t)
        for (int32_t s = 0; s < P.S; ++s)
            for (int lane = 0; lane < 64; ++lane) {
                const GridCell g = grid_cell(P.NA, P.NB, P.NC, P.PA, P.PB, P.TA, upper, t, lane, s);
                if (!g.valid) continue;
                const int64_t row = g.ga * P.sa + g.gb * P.sb + g.gc * P.sc;
                const int64_t dep[3] = {row + sg * P.sc, row + sg * P.sb, row + sg * P.sa};  // back, below, left
                int32_t *o = &P.src[(size_t)(((t * P.S + s) * P.ncoef) * 64 + lane)];
                const int32_t e0 = upper ? diag[row] + 1 : LUp[row], e1 = upper ? LUp[row + 1] : diag[row];
                for (int32_t e = e0; e < e1; ++e)
                    for (int k = 0; k < 3; ++k)
                        if (LUj[e] == dep[k]) o[k * 64] = e;
                if (upper) o[3 * 64] = diag[row];
            }
    G = std::move(P);
    return true;
}

}  // namespace plan
}  // namespace hec

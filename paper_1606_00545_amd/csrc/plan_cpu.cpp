// CPU build of the triangular-solve planner (plan.hpp) with a small C ABI, so
// that a plan can be built and inspected without a GPU: the test suite replays
// it on the host (ordering, ring and LDS limits, deadlock freedom) against the
// reference triangular solves. Built with the host compiler into libhecplan.so.
#include <cstring>
#include <new>

#include "plan.hpp"

using hec::plan::HostPlan;

extern "C" {

// Builds the plan of the strict lower (upper == 0) or strict upper triangle of
// the factor pattern (LUp, LUj, diag: row pointers, columns, diagonal
// positions; 0-based) with the grid sizes detected from A (all 0: none) and
// lds_max bytes of LDS per workgroup; flat != 0 asks for the level-order layout;
// blocks (nbounds entries, may be NULL): first rows of independent row blocks
// followed by n, to be used as parts; solvers: solver wavefronts per workgroup
// for parts with wide levels (1, 2, 4 or 8; 0: the library's default); tile: the
// side of grid tiles (0: the planner's choice). Returns NULL on allocation
// failure or a bad solver count.
void *hecplan_make(int32_t n, const int32_t *LUp, const int32_t *LUj, const int32_t *diag, int32_t gnx,
                   int32_t gny, int32_t gnz, int32_t upper, int32_t has_f32, int64_t lds_max, int32_t flat,
                   const int32_t *blocks, int32_t nbounds, int32_t solvers, int32_t tile) {
    if (solvers == 0) solvers = hec::plan::kSolvers;
    if (solvers != 1 && solvers != 2 && solvers != 4 && solvers != 8) return nullptr;
    HostPlan *P = new (std::nothrow) HostPlan();
    if (!P) return nullptr;
    try {
        std::vector<int32_t> bv;
        if (blocks && nbounds > 0) bv.assign(blocks, blocks + nbounds);
        hec::plan::make_plan(n, LUp, LUj, diag, gnx, gny, gnz, upper != 0, has_f32 != 0, lds_max, *P, flat != 0,
                             bv.empty() ? nullptr : &bv, solvers, tile < 0 ? 0 : tile);
    } catch (...) {
        delete P;
        return nullptr;
    }
    return P;
}

// meta[0..16] = n, nlev, K, KC, ldq, nparts, nss, W, S, D64, D32, blocked,
// lds64, lds32, kSub, kPad, NS.
void hecplan_meta(const void *h, int64_t *meta) {
    const HostPlan &P = *(const HostPlan *)h;
    const int64_t m[17] = {P.n, P.nlev, P.K, P.KC, P.ldq, P.nparts, P.nss, P.W, P.S, P.D64, P.D32,
                           P.blocked ? 1 : 0, (int64_t)P.lds64, (int64_t)P.lds32, hec::plan::kSub,
                           hec::plan::kPad, P.NS};
    std::memcpy(meta, m, sizeof(m));
}

// Copies the named array (level_ptr, perm, lev, part_ss, part_pos, ss_pos,
// ss_need, grow, part_of, pos, chunks, enc, src, psrc) into dst when dst != NULL.
// Returns its length, or -1 for an unknown name.
int64_t hecplan_array(const void *h, const char *name, int32_t *dst) {
    const HostPlan &P = *(const HostPlan *)h;
    const std::vector<int32_t> *v = nullptr;
    if (!std::strcmp(name, "level_ptr")) v = &P.level_ptr;
    else if (!std::strcmp(name, "perm")) v = &P.perm;
    else if (!std::strcmp(name, "lev")) v = &P.lev;
    else if (!std::strcmp(name, "part_ss")) v = &P.part_ss;
    else if (!std::strcmp(name, "part_pos")) v = &P.part_pos;
    else if (!std::strcmp(name, "ss_pos")) v = &P.ss_pos;
    else if (!std::strcmp(name, "ss_need")) v = &P.ss_need;
    else if (!std::strcmp(name, "grow")) v = &P.grow;
    else if (!std::strcmp(name, "part_of")) v = &P.part_of;
    else if (!std::strcmp(name, "pos")) v = &P.pos;
    else if (!std::strcmp(name, "chunks")) v = &P.chunks;
    else if (!std::strcmp(name, "enc")) v = &P.enc;
    else if (!std::strcmp(name, "src")) v = &P.src;
    else if (!std::strcmp(name, "psrc")) v = &P.psrc;
    if (!v) return -1;
    if (dst && !v->empty()) std::memcpy(dst, v->data(), v->size() * sizeof(int32_t));
    return (int64_t)v->size();
}

void hecplan_free(void *h) { delete (HostPlan *)h; }

// Wavefront plan of the strict lower (upper) triangle on the nx x ny x nz grid
// (make_grid_plan); NULL when none applies or on allocation failure.
void *hecplan_grid_make(int32_t n, const int32_t *LUp, const int32_t *LUj, const int32_t *diag, int32_t gnx,
                        int32_t gny, int32_t gnz, int32_t upper) {
    auto *G = new (std::nothrow) hec::plan::GridPlan();
    if (!G) return nullptr;
    try {
        if (hec::plan::make_grid_plan(n, LUp, LUj, diag, gnx, gny, gnz, upper != 0, *G)) return G;
    } catch (...) {
    }
    delete G;
    return nullptr;
}

// meta[0..11] = NA, NB, NC, sa, sb, sc, PA, PB, S, ncoef, TA, TB.
void hecplan_grid_meta(const void *h, int64_t *meta) {
    const auto &G = *(const hec::plan::GridPlan *)h;
    const int64_t m[12] = {G.NA, G.NB, G.NC, G.sa, G.sb, G.sc, G.PA, G.PB, G.S, G.ncoef, G.TA, G.TB};
    std::memcpy(meta, m, sizeof(m));
}

// Copies the coefficient map ([claim][step][k][lane]) into dst when dst != NULL;
// returns its length.
int64_t hecplan_grid_src(const void *h, int32_t *dst) {
    const auto &G = *(const hec::plan::GridPlan *)h;
    if (dst && !G.src.empty()) std::memcpy(dst, G.src.data(), G.src.size() * sizeof(int32_t));
    return (int64_t)G.src.size();
}

void hecplan_grid_free(void *h) { delete (hec::plan::GridPlan *)h; }

// Grid recognition used to choose tiled parts: out = {nx, ny, nz}, all 0 when
// the pattern is not a natural-order 5/7-point stencil.
void hecplan_detect_grid(int32_t n, const int32_t *Ap, const int32_t *Aj, int32_t *out) {
    hec::plan::detect_grid(n, Ap, Aj, out[0], out[1], out[2]);
}

}  // extern "C"

// Shared pieces of the render orchestration: the per-call frame of view
// tables and buffers, and the two halves of a forward pass.
#pragma once

#include "ctx.h"

namespace vcgs {

struct Frame {
    int V = 0;
    int64_t n = 0, E = 0;
    ProjTab pt;
    EmitTab et;
    ViewTab vt;
    uint32_t total_tiles = 0;
    ProjTab* pt_dev = nullptr;
    Splat* rec = nullptr;
    uint32_t* depth_key = nullptr;
    uint2* rect = nullptr;
    uint32_t* count = nullptr;
    uint32_t* ranges = nullptr;
    uint32_t* gids = nullptr;
    int64_t cap = 0;  // pair capacity (exact pair count in the synchronising path)
    int64_t pair_hint = 0;  // expected pair count when cap is a generous bound (0: cap)
    // the projection takes pt as a kernel argument and writes it to pt_dev
    // (false: the caller uploads pt_dev, e.g. for a captured graph)
    bool tab_by_value = false;
    // per-entry gradient sums of the backward: the projection zeroes the
    // slots of the visible entries when this is set (no separate fill)
    float* g2 = nullptr;
};

struct Work {
    uint32_t *dk, *order, *kaltE, *valtE, *headE, *stateE, *scanE, *cnt, *offs, *total, *overflow;
    uint32_t *headP;  // the pair sort's counters (entry-sized work, so that one launch can zero it early)
    uint32_t *tile_ids, *kaltP, *valtP, *stateP, *scanP;  // scanP: emission chunk starts
    int64_t stateP_words = 0;  // words at stateP
    const uint32_t* nvis;  // device count of entries in the depth order (culled ones are dropped)
};

int check_camera(const vcgs_camera* c);
int check_gaussians(const vcgs_gaussians* g, int V);
// Fills the projection, emission and compositing tables of V views (outputs,
// final transmittance and upstream-gradient pointers of vt are left null).
void build_tables(int V, int64_t n, const vcgs_camera* cams, const vcgs_pose* poses, const float bg[3], Frame& f);
// Zeroes, in one launch, what a pass needs at zero: both sorts' counters, the
// pair scan's look-back words, the tile ranges and (unless keep_overflow) the
// overflow flag.
void zero_pass(Frame& f, Work& w, hipStream_t s, bool keep_overflow = false);
// zero_pass's clearing (done by the projection launch), projection, depth
// order of all entries, pair offsets; the pair count ends up in w.total on the
// device.  Returns the depth order.
const uint32_t* phase_a(Prof& pf, const vcgs_gaussians& g, Frame& f, Work& w, hipStream_t s,
                        bool keep_overflow = false, uint32_t* host_total = nullptr);
// Pairs (at most f.cap, overflow flagged in w.overflow), stable tile sort,
// tile ranges, forward compositing (after phase_a, or zero_pass when there
// are no entries).
void phase_b(Prof& pf, Frame& f, Work& w, const uint32_t* ord, hipStream_t s);

// Significant bits of v (at least 1).
inline int bits_for(uint32_t v)
{
    int b = 1;
    while (b < 32 && (v >> b) != 0u) ++b;
    return b;
}

// Allocation of the entry-sized work buffers through `get` (a pool or a plan).
template <class Get>
inline void alloc_work_e(Work& w, int64_t E, Get get)
{
    w.dk = get(E);
    w.order = get(E);
    w.kaltE = get(E);
    w.valtE = get(E);
    w.headE = get(sort_head_words());
    w.stateE = get(sort_state_words(E));
    w.headP = get(sort_head_words());
    w.scanE = get(pair_scan_words(E));
    w.cnt = get(E);
    w.offs = get(E);
    w.total = get(8);
    w.overflow = w.total + 1;  // adjacent: one 8-byte copy reads both
}

template <class Get>
inline void alloc_work_p(Work& w, int64_t cap, Get get)
{
    w.tile_ids = get(cap);
    w.kaltP = get(cap);
    w.valtP = get(cap);
    w.stateP = get(sort_state_words(cap));
    w.stateP_words = sort_state_words(cap);
    w.scanP = get(emit_chunk_words(cap));
}

}  // namespace vcgs

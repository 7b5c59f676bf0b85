// Host-side plan object (internal).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/nolsm.h"
#include "nolsm_internal.h"

struct HostChunk {
    std::vector<SubMeta> meta;
    std::vector<uint32_t> t_subst, t_conv, t_ns, t_ns64, t_rows;
    int32_t max_m = 0, max_np = 0, max_own = 1;
    size_t n_ns_real = 0, n_ns64_real = 0;   // task counts before padding
    size_t ws_used = 0;       // bytes of the workspace this chunk uses
    size_t off_ctl = 0;       // workspace offset of the SubCtl array
    size_t off_ictl = 0;      // workspace offset of the InvCtl array (0: none)
    size_t off_q = 0;         // workspace offset of the queue counters
    size_t base = 0;          // offset of the chunk's region in the workspace
                              // (pipeline schedule: two regions in turn)
    // metadata image offsets (bytes from d_meta)
    size_t o_meta = 0, o_subst = 0, o_conv = 0, o_ns = 0, o_ns64 = 0, o_rows = 0;
};

struct nolsm_plan {
    int32_t nb = 0, bs = 0;
    std::vector<int32_t> Krp, Kci, Srp, Sci;
    std::vector<int32_t> sub_ptr, sub_blk, self_pos, scatter_pos;
    int32_t m_min = 0, m_max = 0;
    double sum_n3 = 0.0;
    // submatrices: groups of molecules (one per molecule unless combined).
    // Group g: row blocks grp_blk[grp_ptr[g] ..) and owned molecules
    // own_J[own_ptr[g] ..); own_pos: position of each owned molecule's block
    // in its group's rows; rowpos[sub_ptr[J] + a]: position of N(J)_a there.
    std::vector<int32_t> grp_ptr, grp_blk, own_ptr, own_J, own_pos, rowpos;
    int32_t g_m_max = 0;
    double sum_gn3 = 0.0;

    // configuration
    bool configured = false;
    bool bound = false;
    int32_t prec = -1, sched = -1, max_iter = 0, ns_tile = 0, elem = 0;
    int32_t inverse = 0, inv_max_iter = 0, sym = 0;
    size_t ws_bytes = 0, ws_min = 0, ws_full = 0;
    std::vector<HostChunk> chunks;
    std::vector<char> image;              // metadata image uploaded by bind
    size_t o_Krp = 0, o_Kci = 0, o_Srp = 0, o_Sci = 0, o_sub_ptr = 0, o_sub_blk = 0,
           o_self = 0, o_scatter = 0, o_grp_blk = 0, o_own_J = 0, o_own_pos = 0, o_rowpos = 0;
    void *d_meta = nullptr;
    int device = -1;
    int32_t pgrid = 512;      // persistent-launch grid (2 x CUs), set by bind
    // graph cache
    void *graph_exec = nullptr;
    const void *g_key[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    double g_mu = 0.0;
    nolsm_solve_opts g_opts;
    void *g_stream = nullptr;
    // pipeline schedule: the library's second stream and its order events
    void *aux_stream = nullptr;
    std::vector<void *> events;
    nolsm_profile prof = {};
};

// Internal helpers implemented in plan.cpp
size_t nolsm_slot_bytes(int32_t np, int32_t ns_tile, int32_t elem, int32_t max_iter, int32_t inverse,
                        int32_t nown, int32_t sym);
int nolsm_ns_tile_for(int32_t prec, int32_t np, uint64_t small_mask);
int nolsm_elem_for(int32_t prec);
void nolsm_set_last_error(const std::string &s);

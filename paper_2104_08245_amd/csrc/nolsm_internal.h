// Internal layout shared by the host runtime (plan.cpp, api.cpp) and the HIP
// kernels. Not part of the public ABI.
#pragma once
#include <stdint.h>

#include "../../include/nolsm.h"

#define NOLSM_TILE 64          // FP64 setup tile (Cholesky, substitution)
#define NOLSM_NFEAT 12
#define NOLSM_MAX_ITER_CAP 128
#define NOLSM_NVEC 12          // finishing-iteration vectors per submatrix

// One submatrix slot of a chunk. Byte offsets are into the workspace.
struct SubMeta {
    int32_t J;        // first owned column block (molecule)
    int32_t m;        // row blocks of the submatrix (N(J), or the union over a group)
    int32_t n;        // bs * m
    int32_t np;       // n rounded up to NOLSM_TILE
    int32_t p;        // position of J's block in the submatrix rows
    int32_t P;        // np / NOLSM_TILE
    int32_t sub_off;  // offset of the submatrix rows in the group row list
    int32_t ntile_ns; // NS GEMM tiles of this slot (for residual partials)
    int32_t ldx;      // leading dimension of the X / R buffers: np rounded up
                      // to the NS tile, so tile loads never leave the buffer
    int32_t nown;     // molecules owned by this submatrix (1 unless combined)
    int32_t own_off;  // their offset in the owned-molecule list
    int32_t pmin;     // smallest block position of an owned molecule (first
                      // nonzero row block of the E columns)
    int32_t kf32;     // the K buffer holds FP32 values (the substitution runs
                      // in FP32 arithmetic), else FP64
    int32_t pad_;
    int64_t offL;     // np*np doubles (FP32 Cholesky route: floats): S -> L; later X buffer 0
    int64_t offK;     // np*(np+64) values (FP64, or FP32 if kf32): K -> W -> [A | Y]
    int64_t offDinv;  // P*64*64 doubles (or floats): inverses of the diagonal tiles of L
    int64_t offRow;   // (P+1)*np doubles: partial |A| row sums per column tile
    int64_t offCol;   // np doubles col sums of |A|, then 64 more: P frob partials
    int64_t offX1;    // ldx*ldx elements of the NS precision: X buffer 1
    int64_t offB;     // ldx*ldx elements: R = I - X^2
    int64_t offVec;   // nown * NOLSM_NVEC * np * 6 floats/doubles: finishing vectors
    int64_t offX0;    // X buffer 0: offL, or its own ldx*ldx buffer on the
                      // symmetric route (which keeps L until the extraction)
    int64_t offRes;   // max(max_iter, inv_max_iter) * ntile_ns doubles: residual partials
    // coupled Newton-Schulz inverse only (0 otherwise): ldx*ldx elements each
    int64_t offY0, offY1;   // Y_k ping-pong; after convergence S^-1 and K in 16 bits
    int64_t offZ0, offZ1;   // Z_k ping-pong
    // FP64 factor applied in FP32 only (0 otherwise): FP32 copies of L
    // (np*np, tiles on and below the diagonal) and of the diagonal-tile
    // inverses (P*64*64), written by the FP64 Cholesky, read by the
    // substitutions
    int64_t offL32, offDinv32;
};

// Per-slot control state, written by kernels only.
struct SubCtl {
    int32_t done;       // sign iteration finished (or failed)
    int32_t iters;      // index K of the returned iterate X_K
    int32_t status;     // NOLSM_MOL_*
    int32_t fallback;   // Gershgorin restart used
    int32_t restart_at; // iteration of the restart, -1 if none
    uint32_t kmax;      // bits of max |T_J(K)| (FP32, non-negative), from the gather
    int32_t pad_[2];
    double scale;       // c_J actually used
    double scale_g;     // Gershgorin scale 1/rho_G
    double resid;       // residual of the returned iterate
    double rhist[NOLSM_MAX_ITER_CAP];
};

// Per-slot state of the coupled Newton-Schulz inverse, written by kernels only.
struct InvCtl {
    int32_t done;       // iteration finished (or failed)
    int32_t iters;      // index K of the returned Z_K
    int32_t pad_[2];
    double scale;       // c = 1 / max row sum of |S_J|
    double rhist[NOLSM_MAX_ITER_CAP];
};

// First 256 bytes of the workspace: values that change between calls without
// changing the captured launch sequence.
struct WsHeader {
    double mu;          // chemical potential of the current solve
    double sumN;        // sum_J N_J (FP64), written by the trace reduction
    double sumE;        // sum_J E_J
    int32_t n_bad;      // molecules with status != OK
    int32_t pad_;
};
#define NOLSM_WS_HEADER 256

// Packed task: slot (16 bits) | a (8 bits) | b (8 bits); 0xFFFFFFFF = no-op.
#define NOLSM_TASK(slot, a, b) (((uint32_t)(slot) << 16) | ((uint32_t)(a) << 8) | (uint32_t)(b))
#define NOLSM_TASK_NONE 0xFFFFFFFFu

// Device addresses of one chunk's metadata and lists (inside d_meta).
struct ChunkDev {
    const SubMeta *meta;
    const uint32_t *t_subst;   // (slot, column tile 0..P)
    const uint32_t *t_conv;    // (slot, 64x64 tile i, j) for X_0
    const uint32_t *t_ns;      // (slot, NS tile i, j): 64x64 (FP64/FP32) or 128x128 (FP16/BF16) tiles
    const uint32_t *t_ns64;    // FP16/BF16 slots that use 64x64 tiles
    const uint32_t *t_rows;    // (slot, 256-row block, owned molecule) for the skinny products
    SubCtl *ctl;               // in the workspace
    InvCtl *ictl;              // in the workspace (coupled inverse), else null
    int32_t *queues;           // persistent launches: [max_iter][2][2][8] counters
    int32_t nqueue;            // number of counters
    int32_t nsub, n_subst, n_conv, n_ns, n_ns64, n_rows, max_m, max_np, max_own;
};

// Launchers of the HIP kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "nolsm_internal.h"

struct GatherArgs {
    const int32_t *Krp, *Kci, *Srp, *Sci;
    const int32_t *grp_blk;   // row blocks of every submatrix (SubMeta::sub_off)
    const int32_t *own_pos;   // position of each owned molecule in its rows (SubMeta::own_off)
    const int32_t *own_J;     // the owned molecules themselves (SubMeta::own_off)
    const double *Kval, *Sval;
    int32_t s_fp32;           // write T_J(S) as FP32 (FP32 Cholesky route), else FP64
    int32_t bs;
    int32_t poison_J;
    int32_t s_lower;          // write T_J(S) only on and below its diagonal 64-tiles
    int32_t k_upper;          // write T_J(K) only on and above its diagonal 64-tiles
    int32_t pad_;
};

struct BoundsArgs {
    const float *d_mlp;
    const float *d_norm;
    float *d_features;
    const int32_t *own_J;     // molecules owned by each submatrix (SubMeta::own_off)
    float safety;
    int32_t learned;
    double scale_mult;
    int32_t sym;              // symmetric sign iteration: X_0 from the upper triangle
    int32_t pad_;
};

// control of the sign iteration, identical for every workgroup of a launch
struct NsArgs {
    int32_t prec;          // nolsm_prec
    int32_t max_iter;
    int32_t fixed_iters;   // > 0: stop exactly after this many updates
    int32_t allow_restart; // Gershgorin restart on divergence
    double tol;            // stop when r < tol (0: unused)
    double theta, rmax;    // stagnation switch: r_k > theta r_{k-1} and r_k < rmax
    int32_t persistent;    // queue-driven fixed grid instead of one workgroup per tile
    int32_t pgrid;         // workgroups of a persistent launch
    int32_t sym;           // symmetric sign iteration: upper tiles, mirrored (FP16/BF16)
    int32_t force_stall;   // molecule taken as diverged at iteration NOLSM_STALL_IT (-1: none)
};
#define NOLSM_STALL_IT 2

// Coupled Newton-Schulz inverse (Eq. inv1-inv3), stop rule as for the sign
// iteration in 16 bits: stagnation r_k > theta r_{k-1} with r_k < rmax.
struct InvArgs {
    int32_t prec;          // NOLSM_FP16 or NOLSM_BF16
    int32_t max_iter;      // iteration slots
    double theta, rmax;
    const int32_t *own_pos;   // block position of each owned molecule (SubMeta::own_off)
    int32_t bs;
};

struct FinishArgs {
    int32_t prec;
    int32_t nfinal;        // 0, 1, 2 column-restricted finishing iterations
    int32_t rows;          // FP16: the row-streaming kernel instead of the fused one
    int32_t pad_;
};

struct ExtractArgs {
    const int32_t *Krp, *Kci, *Srp, *Sci, *sub_blk, *scatter_pos;
    const int32_t *sub_ptr;   // N(J) of molecule J: sub_blk[sub_ptr[J] ..)
    const int32_t *rowpos;    // position of N(J)_a in the rows of J's submatrix
    const int32_t *own_J, *own_pos;
    const int32_t *grp_blk;   // submatrix row blocks (SubMeta::sub_off)
    const double *Kval, *Sval;
    double *Dcols;         // [36 * sum_m] for bs = 6
    double *Dval;          // optional
    double *Wcols;         // optional, Dcols layout: owned columns of T_J(W)
    void *stats;           // nolsm_mol_stats[nb]
    int32_t bs;
    int32_t prec;
    int32_t nfinal;
    int32_t sym;           // symmetric sign iteration: apply L^-T to the column block
    int32_t L_fp32;        // the factor is stored in FP32 (else FP64)
};

hipError_t launch_gather(const ChunkDev &cd, char *ws, const GatherArgs &ga, hipStream_t st);
hipError_t launch_wcols(const ChunkDev &cd, char *ws, const ExtractArgs &ea, hipStream_t st);
hipError_t launch_inverse(const ChunkDev &cd, char *ws, const InvArgs &ia, hipStream_t st);
// fp32: arithmetic on the FP32 matrix cores (FP64 storage either way)
hipError_t launch_chol(const ChunkDev &cd, char *ws, bool fp32, hipStream_t st);
hipError_t launch_subst(const ChunkDev &cd, char *ws, bool fp32, hipStream_t st);
// symmetric sign iteration: [W | y] = L^-1 [K | E], then A~ = W L^-T - mu I in place
hipError_t launch_subst_sym(const ChunkDev &cd, char *ws, bool fp32, bool split16, hipStream_t st);
hipError_t launch_set_header(char *ws, double mu, hipStream_t st);
int finish_launches(const FinishArgs &fa);
hipError_t launch_trace_sums(const void *stats, int32_t nb, char *ws, hipStream_t st);
hipError_t launch_bounds(const ChunkDev &cd, char *ws, const BoundsArgs &ba, int prec, hipStream_t st);
hipError_t launch_convert(const ChunkDev &cd, char *ws, int prec, int use_scale_g, int sym, hipStream_t st);
hipError_t launch_ns_iter(const ChunkDev &cd, char *ws, const NsArgs &na, int it, hipStream_t st);
hipError_t launch_finish(const ChunkDev &cd, char *ws, const FinishArgs &fa, hipStream_t st);
hipError_t launch_extract(const ChunkDev &cd, char *ws, const ExtractArgs &ea, hipStream_t st);
hipError_t launch_assemble(const double *Dcols, double *Dval, const int32_t *scatter_pos, int64_t sum_m,
                           int32_t bs, hipStream_t st);
hipError_t nolsm_kernels_init();
hipError_t nolsm_finish_init();

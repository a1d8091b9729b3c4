// mlp_internal.h -- internal interface of the surrogate kernels (libdpps).
#pragma once

#include <stdint.h>

#include "dpps_internal.h"

namespace dpps {

enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3, EPI_PARTIAL = 4 };

#define TOPK_SORT 4096   // most cells per frame for the top-k (>= coarse lattice size)
#define TOPK_MAX 256     // largest k (one workgroup thread per winner)

struct GemmArgs {
    const uint16_t *A;   // bf16
    const uint16_t *B;   // bf16
    int lda, ldb, ldc;
    int M, N, K;
    const float *bias;   // EPI_BIAS, EPI_BIAS_GELU
    const float *Zin;    // EPI_GELU_GRAD: pre-activation, [M][ldc]
    float *Cf;           // f32 output
    uint16_t *Cb;        // bf16 output
    float *work;         // optional workspace for a K split (EPI_NONE only), work_elems floats
    int64_t work_elems;
    int k_slice;         // set by the dispatcher
};

int gemm(const GemmArgs &g, bool a_k, bool b_k, int epi, void *stream);
// Inference GEMM of a few rows (A, B k-contiguous; EPI_BIAS or EPI_BIAS_GELU),
// bit-identical per element to gemm(g, true, true, epi, stream).
int gemm_rows(const GemmArgs &g, int epi, void *stream);
// Column sums (bias gradients); part holds colsum_chunks(M) x N floats.
int launch_colsum(const uint16_t *dz, int M, int N, int ld, float *db, float *part, void *st);
int colsum_chunks(int M);
int launch_loss(const float *y, int ldy, const float *tgt, int ldt, int rows, int outs, int rows_pad,
                int outs_pad, float pos_weight, float ce_weight, float tau, uint16_t *dz,
                float *partial, void *st);
int launch_pool(const float *fine, int n_frames, int fnx, int fny, float *coarse, int cnx, int cny,
                void *st);
int launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                float eps, float c1, float c2, float wd, uint16_t *wb, uint16_t *wbt, int rows,
                int cols, void *st);
int launch_cast(const float *w, int64_t n, uint16_t *wb, uint16_t *wbt, int rows, int cols, void *st);
int launch_featurize(const FrameDev *frames, const dpps_robot *robots, int n_frames, int rows_pad,
                     int in_pad, float inv_hl, float inv_hw, float inv_v, uint16_t *x, void *st);
// Re-score tables written by the top-k kernel: per frame f, its copy
// frames[f] (n_windows = tile_count = k), k windows and k tiles.
struct RescoreTables {
    const FrameDev *src;
    int coarse_nx, fine_nx, fine_ny;
    float fine_h;
    FrameDev *frames;
    WinDev *wins;
    TileDev *tiles;
    int32_t *zero_word;     // cleared by the kernel (may be NULL)
};
// Top-k cells of each frame's map into out [n_frames][k]; with rt, also the
// re-score tables of those cells.
int launch_topk(const float *y, int ldy, int n_frames, int n_cells, int k, int32_t *out,
                const RescoreTables *rt, void *st);

}  // namespace dpps

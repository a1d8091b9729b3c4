// mlp_api.hip -- the learned surrogate behind the C ABI (include/dpps.h):
// parameters, forward and backward passes, Adam, top-k and the surrogate
// search (network proposals re-scored by the exact kernel, exact fallback).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <new>
#include <random>
#include <vector>

#include "mlp_internal.h"
#include "runtime.h"

using namespace dpps;

namespace {

constexpr int NL = 4;
constexpr int IN = 66, IN_PAD = 96, HID = 512, OUT = 2806, OUT_PAD = 2816;
constexpr int IN_DIM[NL] = {IN_PAD, HID, HID, HID};
constexpr int IN_REAL[NL] = {IN, HID, HID, HID};
constexpr int OUT_DIM[NL] = {HID, HID, HID, OUT_PAD};
constexpr int OUT_REAL[NL] = {HID, HID, HID, OUT};
// workspace of the split weight-gradient products (partial sums, floats)
constexpr int64_t GWORK_ELEMS = 3 * 1024 * 1024;
constexpr double COARSE_H = 0.2, FINE_H = 0.05;

int64_t real_count()
{
    int64_t n = 0;
    for (int l = 0; l < NL; ++l) n += (int64_t)OUT_REAL[l] * IN_REAL[l] + OUT_REAL[l];
    return n;
}

}  // namespace

struct dpps_mlp {
    dpps_ctx *ctx = nullptr;
    int rows_cap = 0;       // padded to 64
    int k_cap = 0;
    void *arena = nullptr;
    size_t arena_bytes = 0;
    float *w[NL], *b[NL], *gw[NL], *gb[NL], *mw[NL], *vw[NL], *mb[NL], *vb[NL];
    uint16_t *wb[NL], *wbt[NL];
    uint16_t *x0;
    float *z[3];
    uint16_t *a[3];
    float *y;
    uint16_t *dz4;
    uint16_t *dz[3];
    float *partial;
    float *colpart;          // partial column sums of the bias gradients
    float *gwork;            // partial weight-gradient products
    int64_t step = 0;
    // re-score tables
    int32_t *cells;
    FrameDev *rf;
    WinDev *rw;
    TileDev *rt;
    TileRec *rrec;
    uint32_t *rcounter;
    int coarse_nx = 0, fine_nx = 0, fine_ny = 0;
    // exact fallback built on the device: the frames whose proposals are all
    // infeasible, their full-lattice windows, per-tile records, the frame
    // map, the frame count and the work counter
    FrameDev *ff;
    WinDev *fw;
    TileRec *frec;
    int32_t *fmap;
    int32_t *fcount;
    uint32_t *fcounter;
    int32_t *h_count = nullptr;  // pinned landing word of the fallback count
};

// Points per tile of the device-side exact fallback (its tiles are implicit).
static constexpr int FB_TILE = 64;

static size_t carve(size_t &off, size_t bytes)
{
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
}

static int rows_pad(int n) { return (n + 63) / 64 * 64; }

static int refresh_bf16(dpps_mlp *m, hipStream_t st)
{
    for (int l = 0; l < NL; ++l) {
        int64_t n = (int64_t)OUT_DIM[l] * IN_DIM[l];
        if (launch_cast(m->w[l], n, m->wb[l], m->wbt[l], OUT_DIM[l], IN_DIM[l], (void *)st))
            return fail(DPPS_E_DEVICE, "cast kernel launch failed");
    }
    return DPPS_OK;
}

// copy between the real parameter layout on the host (W0 [512][66], b0,
// W1, b1, W2, b2, W3 [2806][512], b3 [2806]) and the padded device tensors
static int params_xfer(dpps_mlp *m, float *const *dw, float *const *db, float *host, bool to_dev)
{
    int64_t o = 0;
    for (int l = 0; l < NL; ++l) {
        size_t wrow = (size_t)IN_REAL[l] * 4, dpitch = (size_t)IN_DIM[l] * 4;
        if (to_dev)
            HIP_OK(hipMemcpy2D(dw[l], dpitch, host + o, wrow, wrow, OUT_REAL[l], hipMemcpyHostToDevice));
        else
            HIP_OK(hipMemcpy2D(host + o, wrow, dw[l], dpitch, wrow, OUT_REAL[l], hipMemcpyDeviceToHost));
        o += (int64_t)OUT_REAL[l] * IN_REAL[l];
        if (to_dev)
            HIP_OK(hipMemcpy(db[l], host + o, (size_t)OUT_REAL[l] * 4, hipMemcpyHostToDevice));
        else
            HIP_OK(hipMemcpy(host + o, db[l], (size_t)OUT_REAL[l] * 4, hipMemcpyDeviceToHost));
        o += OUT_REAL[l];
    }
    return DPPS_OK;
}

// Batches of at most SMALL_ROWS frames are run, for inference, by the few-row
// GEMM over the frames' rows rounded up to 16 (identical results, one wave
// per output tile instead of a handful of 64 x 64 tiles); training needs
// every padded row and uses the tiled GEMM.
constexpr int SMALL_ROWS = 64;

static int forward(dpps_mlp *m, const dpps_batch *bt, hipStream_t st, bool training)
{
    const int nf = bt->n_frames, R = rows_pad(nf);
    const bool small = !training && nf >= 1 && nf <= SMALL_ROWS;
    if (nf > m->rows_cap) return fail(DPPS_E_INVALID, "batch of %d frames exceeds the network's %d",
                                      nf, m->rows_cap);
    const dpps_params &p = m->ctx->p;
    if (launch_featurize(bt->d_frames, bt->d_robots, nf, R, IN_PAD, 2.0f / p.field_len,
                         2.0f / p.field_wid, 1.0f / p.vmax, m->x0, (void *)st))
        return fail(DPPS_E_DEVICE, "featurize launch failed");
    const uint16_t *in = m->x0;
    for (int l = 0; l < NL; ++l) {
        GemmArgs g;
        memset(&g, 0, sizeof g);
        g.A = in;
        g.lda = IN_DIM[l];
        g.B = m->wb[l];
        g.ldb = IN_DIM[l];
        g.M = small ? (nf + 15) / 16 * 16 : R;
        g.N = OUT_DIM[l];
        g.K = IN_DIM[l];
        g.ldc = OUT_DIM[l];
        g.bias = m->b[l];
        int epi;
        if (l < NL - 1) {
            g.Cf = m->z[l];
            g.Cb = m->a[l];
            epi = EPI_BIAS_GELU;
            in = m->a[l];
        } else {
            g.Cf = m->y;
            epi = EPI_BIAS;
        }
        if (small ? gemm_rows(g, epi, (void *)st) : gemm(g, true, true, epi, (void *)st))
            return fail(DPPS_E_DEVICE, "gemm launch failed");
    }
    return DPPS_OK;
}

struct LossCfg {
    float pos_weight, ce_weight, tau;
};

// gradients of the training loss against targets [nf][ld_t] (after forward)
static int backward_loss(dpps_mlp *m, int nf, const float *tgt, int64_t ld_t, LossCfg lc,
                         hipStream_t st)
{
    const int R = rows_pad(nf);
    if (launch_loss(m->y, OUT_PAD, tgt, (int)ld_t, nf, OUT, R, OUT_PAD, lc.pos_weight, lc.ce_weight,
                    lc.tau, m->dz4, m->partial, (void *)st))
        return fail(DPPS_E_DEVICE, "loss launch failed");
    const uint16_t *dz_top = m->dz4;
    for (int l = NL - 1; l >= 0; --l) {
        const uint16_t *act = l == 0 ? m->x0 : m->a[l - 1];
        // dW_l = dZ_l^T act  ([out][in], reduction over rows)
        GemmArgs g;
        memset(&g, 0, sizeof g);
        g.A = dz_top;
        g.lda = OUT_DIM[l];
        g.B = act;
        g.ldb = IN_DIM[l];
        g.M = OUT_DIM[l];
        g.N = IN_DIM[l];
        g.K = R;
        g.ldc = IN_DIM[l];
        g.Cf = m->gw[l];
        g.work = m->gwork;  // the reduction over the batch may be split
        g.work_elems = GWORK_ELEMS;
        if (gemm(g, false, false, EPI_NONE, (void *)st)) return fail(DPPS_E_DEVICE, "gemm failed");
        if (launch_colsum(dz_top, R, OUT_DIM[l], OUT_DIM[l], m->gb[l], m->colpart, (void *)st))
            return fail(DPPS_E_DEVICE, "colsum failed");
        if (l == 0) break;
        // dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1})
        GemmArgs h;
        memset(&h, 0, sizeof h);
        h.A = dz_top;
        h.lda = OUT_DIM[l];
        h.B = m->wbt[l];
        h.ldb = OUT_DIM[l];
        h.M = R;
        h.N = IN_DIM[l];
        h.K = OUT_DIM[l];
        h.ldc = IN_DIM[l];
        h.Zin = m->z[l - 1];
        h.Cb = m->dz[l - 1];
        if (gemm(h, true, true, EPI_GELU_GRAD, (void *)st)) return fail(DPPS_E_DEVICE, "gemm failed");
        dz_top = m->dz[l - 1];
    }
    return DPPS_OK;
}

static int read_loss(dpps_mlp *m, int nf, float ce_weight, hipStream_t st, float *loss)
{
    if (!loss) return DPPS_OK;
    const int R = rows_pad(nf);
    std::vector<float> part(2 * (size_t)R);
    HIP_OK(hipMemcpyAsync(part.data(), m->partial, (size_t)R * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    double s = 0.0, e = 0.0;
    for (int r = 0; r < nf; ++r) {
        s += part[2 * r];
        e += part[2 * r + 1];
    }
    *loss = (float)(s / ((double)nf * OUT) + ce_weight * e / nf);
    return DPPS_OK;
}

extern "C" {

int64_t dpps_mlp_param_count(void) { return real_count(); }

int dpps_mlp_create(dpps_ctx *c, int32_t max_frames, int32_t max_k, uint64_t seed, dpps_mlp **out)
{
    if (!c || !out) return fail(DPPS_E_INVALID, "NULL argument");
    *out = nullptr;
    if (max_frames < 1 || max_frames > (1 << 20)) return fail(DPPS_E_INVALID, "max_frames out of range");
    if (max_k < 1 || max_k > TOPK_MAX) return fail(DPPS_E_INVALID, "max_k must be in [1, %d]", TOPK_MAX);
    int32_t cnx, cny, fnx, fny;
    if (lattice_dim(c->p.field_len, (float)COARSE_H, &cnx) || lattice_dim(c->p.field_wid, (float)COARSE_H, &cny) ||
        lattice_dim(c->p.field_len, (float)FINE_H, &fnx) || lattice_dim(c->p.field_wid, (float)FINE_H, &fny) ||
        cnx * cny != OUT)
        return fail(DPPS_E_UNSUPPORTED, "the surrogate maps the 12 m x 9 m field at 20 cm (2806 cells)");
    HIP_OK(hipSetDevice(c->device));
    dpps_mlp *m = new (std::nothrow) dpps_mlp();
    if (!m) return fail(DPPS_E_NOMEM, "allocation failed");
    m->ctx = c;
    m->rows_cap = rows_pad(max_frames);
    m->k_cap = max_k;
    m->coarse_nx = cnx;
    m->fine_nx = fnx;
    m->fine_ny = fny;
    const size_t R = (size_t)m->rows_cap;
    size_t off = 0, ow[NL], ob[NL], ogw[NL], ogb[NL], omw[NL], ovw[NL], omb[NL], ovb[NL], owb[NL], owbt[NL];
    for (int l = 0; l < NL; ++l) {
        size_t nw = (size_t)OUT_DIM[l] * IN_DIM[l], nb = OUT_DIM[l];
        ow[l] = carve(off, nw * 4); ob[l] = carve(off, nb * 4);
        ogw[l] = carve(off, nw * 4); ogb[l] = carve(off, nb * 4);
        omw[l] = carve(off, nw * 4); ovw[l] = carve(off, nw * 4);
        omb[l] = carve(off, nb * 4); ovb[l] = carve(off, nb * 4);
        owb[l] = carve(off, nw * 2); owbt[l] = carve(off, nw * 2);
    }
    size_t ox0 = carve(off, R * IN_PAD * 2), oz[3], oa[3], odz[3];
    for (int l = 0; l < 3; ++l) {
        oz[l] = carve(off, R * HID * 4);
        oa[l] = carve(off, R * HID * 2);
        odz[l] = carve(off, R * HID * 2);
    }
    size_t oy = carve(off, R * OUT_PAD * 4), odz4 = carve(off, R * OUT_PAD * 2);
    size_t opart = carve(off, R * 8);
    size_t ocol = carve(off, (size_t)colsum_chunks((int)R) * OUT_PAD * 4);
    size_t ogwork = carve(off, (size_t)GWORK_ELEMS * 4);
    size_t ocells = carve(off, R * max_k * 4);
    size_t orf = carve(off, R * sizeof(FrameDev));
    size_t orw = carve(off, R * max_k * sizeof(WinDev));
    size_t ort = carve(off, R * max_k * sizeof(TileDev));
    size_t orrec = carve(off, R * max_k * sizeof(TileRec));
    size_t octr = carve(off, 256);
    const size_t fb_tpf = ((size_t)fnx * fny + FB_TILE - 1) / FB_TILE;
    size_t off_ff = carve(off, R * sizeof(FrameDev));
    size_t off_fw = carve(off, R * sizeof(WinDev));
    size_t off_frec = carve(off, R * fb_tpf * sizeof(TileRec));
    size_t off_fmap = carve(off, R * sizeof(int32_t));
    size_t off_fcnt = carve(off, 256);
    size_t off_fctr = carve(off, 256);
    if (c->p.hbm_budget_bytes && c->budget_used + off > c->p.hbm_budget_bytes) {
        delete m;
        return fail(DPPS_E_BUDGET, "network needs %zu device bytes", off);
    }
    if (hipMalloc(&m->arena, off) != hipSuccess) {
        (void)hipGetLastError();
        delete m;
        return fail(DPPS_E_NOMEM, "hipMalloc(%zu) failed", off);
    }
    m->arena_bytes = off;
    c->budget_used += off;
    char *A = (char *)m->arena;
    for (int l = 0; l < NL; ++l) {
        m->w[l] = (float *)(A + ow[l]); m->b[l] = (float *)(A + ob[l]);
        m->gw[l] = (float *)(A + ogw[l]); m->gb[l] = (float *)(A + ogb[l]);
        m->mw[l] = (float *)(A + omw[l]); m->vw[l] = (float *)(A + ovw[l]);
        m->mb[l] = (float *)(A + omb[l]); m->vb[l] = (float *)(A + ovb[l]);
        m->wb[l] = (uint16_t *)(A + owb[l]); m->wbt[l] = (uint16_t *)(A + owbt[l]);
    }
    m->x0 = (uint16_t *)(A + ox0);
    for (int l = 0; l < 3; ++l) {
        m->z[l] = (float *)(A + oz[l]);
        m->a[l] = (uint16_t *)(A + oa[l]);
        m->dz[l] = (uint16_t *)(A + odz[l]);
    }
    m->y = (float *)(A + oy);
    m->dz4 = (uint16_t *)(A + odz4);
    m->partial = (float *)(A + opart);
    m->colpart = (float *)(A + ocol);
    m->gwork = (float *)(A + ogwork);
    m->cells = (int32_t *)(A + ocells);
    m->rf = (FrameDev *)(A + orf);
    m->rw = (WinDev *)(A + orw);
    m->rt = (TileDev *)(A + ort);
    m->rrec = (TileRec *)(A + orrec);
    m->rcounter = (uint32_t *)(A + octr);
    m->ff = (FrameDev *)(A + off_ff);
    m->fw = (WinDev *)(A + off_fw);
    m->frec = (TileRec *)(A + off_frec);
    m->fmap = (int32_t *)(A + off_fmap);
    m->fcount = (int32_t *)(A + off_fcnt);
    m->fcounter = (uint32_t *)(A + off_fctr);
    if (hipMemset(m->arena, 0, off) != hipSuccess) {
        dpps_mlp_destroy(m);
        return fail(DPPS_E_DEVICE, "hipMemset failed");
    }
    if (hipHostMalloc((void **)&m->h_count, 64, hipHostMallocDefault) != hipSuccess) {
        m->h_count = nullptr;
        dpps_mlp_destroy(m);
        return fail(DPPS_E_NOMEM, "hipHostMalloc of the fallback count failed");
    }
    // He-uniform initialisation of the real weights (bound sqrt(6 / fan_in)),
    // zero biases; padding rows and columns stay zero
    std::mt19937_64 rng(seed);
    std::vector<float> host(real_count());
    int64_t o = 0;
    for (int l = 0; l < NL; ++l) {
        double bound = sqrt(6.0 / IN_REAL[l]);
        std::uniform_real_distribution<double> U(-bound, bound);
        for (int64_t i = 0; i < (int64_t)OUT_REAL[l] * IN_REAL[l]; ++i) host[o++] = (float)U(rng);
        for (int i = 0; i < OUT_REAL[l]; ++i) host[o++] = 0.0f;
    }
    int rc = dpps_mlp_set_params(m, host.data(), (int64_t)host.size());
    if (rc) {
        dpps_mlp_destroy(m);
        return rc;
    }
    *out = m;
    return DPPS_OK;
}

void dpps_mlp_destroy(dpps_mlp *m)
{
    if (!m) return;
    if (m->ctx && m->ctx->stream) (void)hipStreamSynchronize(m->ctx->stream);
    if (m->arena) {
        (void)hipFree(m->arena);
        if (m->ctx) m->ctx->budget_used -= m->arena_bytes;
    }
    if (m->h_count) (void)hipHostFree(m->h_count);
    delete m;
}

int dpps_mlp_set_params(dpps_mlp *m, const float *host, int64_t n)
{
    if (!m || !host) return fail(DPPS_E_INVALID, "NULL argument");
    if (n != real_count()) return fail(DPPS_E_INVALID, "expected %lld parameters", (long long)real_count());
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(host[i])) return fail(DPPS_E_INVALID, "parameter %lld not finite", (long long)i);
    HIP_OK(hipSetDevice(m->ctx->device));
    HIP_OK(hipStreamSynchronize(m->ctx->stream));
    int rc = params_xfer(m, m->w, m->b, const_cast<float *>(host), true);
    if (rc) return rc;
    rc = refresh_bf16(m, m->ctx->stream);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(m->ctx->stream));
    return DPPS_OK;
}

int dpps_mlp_get_params(dpps_mlp *m, float *host, int64_t n)
{
    if (!m || !host) return fail(DPPS_E_INVALID, "NULL argument");
    if (n != real_count()) return fail(DPPS_E_INVALID, "expected %lld parameters", (long long)real_count());
    HIP_OK(hipStreamSynchronize(m->ctx->stream));
    return params_xfer(m, m->w, m->b, host, false);
}

int dpps_mlp_get_grads(dpps_mlp *m, float *host, int64_t n)
{
    if (!m || !host) return fail(DPPS_E_INVALID, "NULL argument");
    if (n != real_count()) return fail(DPPS_E_INVALID, "expected %lld parameters", (long long)real_count());
    HIP_OK(hipStreamSynchronize(m->ctx->stream));
    return params_xfer(m, m->gw, m->gb, host, false);
}

int dpps_mlp_get_adam(dpps_mlp *m, float *host_m, float *host_v, int64_t n, int64_t *step)
{
    if (!m || !host_m || !host_v || !step) return fail(DPPS_E_INVALID, "NULL argument");
    if (n != real_count()) return fail(DPPS_E_INVALID, "expected %lld parameters", (long long)real_count());
    HIP_OK(hipStreamSynchronize(m->ctx->stream));
    int rc = params_xfer(m, m->mw, m->mb, host_m, false);
    if (rc) return rc;
    *step = m->step;
    return params_xfer(m, m->vw, m->vb, host_v, false);
}

int dpps_mlp_set_adam(dpps_mlp *m, const float *host_m, const float *host_v, int64_t n, int64_t step)
{
    if (!m || !host_m || !host_v) return fail(DPPS_E_INVALID, "NULL argument");
    if (n != real_count() || step < 0) return fail(DPPS_E_INVALID, "bad Adam state");
    HIP_OK(hipStreamSynchronize(m->ctx->stream));
    int rc = params_xfer(m, m->mw, m->mb, const_cast<float *>(host_m), true);
    if (rc) return rc;
    m->step = step;
    return params_xfer(m, m->vw, m->vb, const_cast<float *>(host_v), true);
}

int dpps_mlp_forward(dpps_mlp *m, dpps_batch *b, float *d_out, int64_t ld_out, void *hip_stream)
{
    if (!m || !b) return fail(DPPS_E_INVALID, "NULL argument");
    if (d_out && ld_out < OUT) return fail(DPPS_E_INVALID, "ld_out must be >= %d", OUT);
    HIP_OK(hipSetDevice(m->ctx->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : m->ctx->stream;
    int rc = forward(m, b, st, false);
    if (rc) return rc;
    if (d_out && b->n_frames > 0)
        HIP_OK(hipMemcpy2DAsync(d_out, (size_t)ld_out * 4, m->y, (size_t)OUT_PAD * 4, (size_t)OUT * 4,
                                b->n_frames, hipMemcpyDeviceToDevice, st));
    return DPPS_OK;
}

int dpps_mlp_loss_grad(dpps_mlp *m, dpps_batch *b, const float *d_target, int64_t ld_target,
                       float pos_weight, float ce_weight, float tau, float *loss, void *hip_stream)
{
    if (!m || !b || !d_target) return fail(DPPS_E_INVALID, "NULL argument");
    if (!(pos_weight >= 0.0f) || !isfinite(pos_weight) || !(ce_weight >= 0.0f) ||
        !isfinite(ce_weight) || !(tau > 0.0f) || !isfinite(tau))
        return fail(DPPS_E_INVALID, "loss weights must be >= 0 and tau > 0");
    if (b->n_frames < 1) return fail(DPPS_E_INVALID, "empty batch");
    if (ld_target < OUT) return fail(DPPS_E_INVALID, "ld_target must be >= %d", OUT);
    HIP_OK(hipSetDevice(m->ctx->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : m->ctx->stream;
    int rc = forward(m, b, st, true);
    if (rc) return rc;
    rc = backward_loss(m, b->n_frames, d_target, ld_target, LossCfg{pos_weight, ce_weight, tau}, st);
    if (rc) return rc;
    return read_loss(m, b->n_frames, ce_weight, st, loss);
}

int dpps_mlp_adam(dpps_mlp *m, float lr, float beta1, float beta2, float eps, float weight_decay,
                  void *hip_stream)
{
    if (!m) return fail(DPPS_E_INVALID, "NULL argument");
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f) || !(weight_decay >= 0.0f))
        return fail(DPPS_E_INVALID, "bad Adam hyper-parameters");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : m->ctx->stream;
    m->step += 1;
    float c1 = (float)(1.0 - pow((double)beta1, (double)m->step));
    float c2 = (float)(1.0 - pow((double)beta2, (double)m->step));
    for (int l = 0; l < NL; ++l) {
        int64_t nw = (int64_t)OUT_DIM[l] * IN_DIM[l];
        if (launch_adam(m->w[l], m->gw[l], m->mw[l], m->vw[l], nw, lr, beta1, beta2, eps, c1, c2,
                        weight_decay, m->wb[l], m->wbt[l], OUT_DIM[l], IN_DIM[l], (void *)st) ||
            launch_adam(m->b[l], m->gb[l], m->mb[l], m->vb[l], OUT_DIM[l], lr, beta1, beta2, eps, c1,
                        c2, 0.0f, nullptr, nullptr, 1, OUT_DIM[l], (void *)st))
            return fail(DPPS_E_DEVICE, "adam launch failed");
    }
    return DPPS_OK;
}

int dpps_pool_cells(const float *d_fine, int32_t n_frames, int32_t fine_nx, int32_t fine_ny,
                    float *d_coarse, int32_t coarse_nx, int32_t coarse_ny, void *hip_stream)
{
    if (!d_fine || !d_coarse) return fail(DPPS_E_INVALID, "NULL argument");
    if (n_frames < 0 || fine_nx < 1 || fine_ny < 1 || coarse_nx < 1 || coarse_ny < 1 ||
        4 * (coarse_nx - 1) > fine_nx + 1 || 4 * (coarse_ny - 1) > fine_ny + 1)
        return fail(DPPS_E_INVALID, "bad pooling shape");
    if (launch_pool(d_fine, n_frames, fine_nx, fine_ny, d_coarse, coarse_nx, coarse_ny, hip_stream))
        return fail(DPPS_E_DEVICE, "pool launch failed");
    return DPPS_OK;
}

int dpps_mlp_train_step(dpps_mlp *m, dpps_batch *b, const float *d_target, int64_t ld_target,
                        float lr, float pos_weight, float ce_weight, float tau, float *loss,
                        void *hip_stream)
{
    int rc = dpps_mlp_loss_grad(m, b, d_target, ld_target, pos_weight, ce_weight, tau, loss,
                                hip_stream);
    if (rc) return rc;
    return dpps_mlp_adam(m, lr, 0.9f, 0.999f, 1e-8f, 0.0f, hip_stream);
}

int dpps_mlp_features(dpps_mlp *m, dpps_batch *b, uint16_t *d_x, void *hip_stream)
{
    if (!m || !b || !d_x) return fail(DPPS_E_INVALID, "NULL argument");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : m->ctx->stream;
    const int nf = b->n_frames;
    if (nf > m->rows_cap) return fail(DPPS_E_INVALID, "batch too large");
    const dpps_params &p = m->ctx->p;
    if (launch_featurize(b->d_frames, b->d_robots, nf, rows_pad(nf), IN_PAD, 2.0f / p.field_len,
                         2.0f / p.field_wid, 1.0f / p.vmax, m->x0, (void *)st))
        return fail(DPPS_E_DEVICE, "featurize launch failed");
    if (nf > 0)
        HIP_OK(hipMemcpy2DAsync(d_x, IN * 2, m->x0, IN_PAD * 2, IN * 2, nf, hipMemcpyDeviceToDevice, st));
    return DPPS_OK;
}

int dpps_mlp_topk(dpps_mlp *m, int32_t n_frames, int32_t k, int32_t *d_cells, void *hip_stream)
{
    if (!m || !d_cells) return fail(DPPS_E_INVALID, "NULL argument");
    if (k < 1 || k > m->k_cap || n_frames < 0 || n_frames > m->rows_cap)
        return fail(DPPS_E_INVALID, "bad top-k request");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : m->ctx->stream;
    if (n_frames > 0 && launch_topk(m->y, OUT_PAD, n_frames, OUT, k, d_cells, nullptr, (void *)st))
        return fail(DPPS_E_DEVICE, "top-k launch failed");
    return DPPS_OK;
}

}  // extern "C"

// Forward pass, top-k cells, re-score tables and the exact re-score of the
// proposed windows (kernel launches only), best records into res.
static int propose(dpps_ctx *c, dpps_mlp *m, dpps_batch *b, int32_t k, dpps_best *res,
                   hipStream_t st, bool fallback = false, float fallback_below = -INFINITY)
{
    const int nf = b->n_frames;
    int rc = forward(m, b, st, false);
    if (rc) return rc;
    // top-k cells and, in the same kernel, their re-score tables
    RescoreTables rt;
    rt.src = b->d_frames;
    rt.coarse_nx = m->coarse_nx;
    rt.fine_nx = m->fine_nx;
    rt.fine_ny = m->fine_ny;
    rt.fine_h = (float)FINE_H;
    rt.frames = m->rf;
    rt.wins = m->rw;
    rt.tiles = m->rt;
    rt.zero_word = m->fcount;  // the fallback list starts empty
    if (launch_topk(m->y, OUT_PAD, nf, OUT, k, m->cells, &rt, (void *)st))
        return fail(DPPS_E_DEVICE, "top-k launch failed");
    // exact re-score of the proposed windows: one 16-point tile per window
    LaunchArgs a;
    memset(&a, 0, sizeof a);
    a.P = c->P;
    a.P.out_flags = 0;
    a.frames = m->rf;
    a.robots = b->d_robots;
    a.variants = b->d_variants;
    a.wins = m->rw;
    a.tiles = m->rt;
    a.n_tiles = nf * k;
    a.n_frames = nf;
    a.tile_points = 16;
    a.persistent = 1;
    a.counter = m->rcounter;
    a.tile_rec = m->rrec;
    a.best = res;
    if (fallback) {
        // frames without a feasible proposal (or below the threshold) are
        // listed for the exact fallback by the re-score's finalize
        a.fb_on = 1;
        a.fb.below = fallback_below;
        a.fb.nx = m->fine_nx;
        a.fb.ny = m->fine_ny;
        a.fb.h = (float)FINE_H;
        a.fb.tiles_per_frame = (m->fine_nx * m->fine_ny + FB_TILE - 1) / FB_TILE;
        a.fb.frames = m->ff;
        a.fb.wins = m->fw;
        a.fb.map = m->fmap;
        a.fb.count = m->fcount;
    }
    // few windows (small batches): eight waves share each window's 16
    // points, two points per wave, instead of the context's shape
    const int wv = (int64_t)a.n_tiles <= (int64_t)c->n_cu ? 8 : c->waves;
    int per_cu = search_occupancy(c->p.n_samples, wv, a.tile_points);
    int64_t cap = (int64_t)c->n_cu * per_cu;
    int grid = (int)(a.n_tiles < cap ? a.n_tiles : cap);
    if (launch_search(a, wv, grid, (void *)st, nullptr, nullptr))
        return fail(DPPS_E_DEVICE, "re-score launch failed");
    return DPPS_OK;
}

// The surrogate search of a staged batch; with h_best the records also go to
// host memory and the call returns after the stream has finished them.
static int surrogate_core(dpps_ctx *c, dpps_mlp *m, dpps_batch *b, int32_t k, dpps_best *d_best,
                          int fallback, float fallback_below, int32_t *n_fallback,
                          dpps_best *h_best, void *hip_stream)
{
    if (!c || !m || !b || !d_best) return fail(DPPS_E_INVALID, "NULL argument");
    if (fallback_below != fallback_below) return fail(DPPS_E_INVALID, "fallback_below is NaN");
    if (m->ctx != c) return fail(DPPS_E_INVALID, "network belongs to another context");
    if (k < 1 || k > m->k_cap) return fail(DPPS_E_INVALID, "k must be in [1, %d]", m->k_cap);
    HIP_OK(hipSetDevice(c->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
    const int nf = b->n_frames;
    if (n_fallback) *n_fallback = 0;
    if (nf == 0) return DPPS_OK;
    int rc = propose(c, m, b, k, d_best, st, fallback != 0, fallback_below);
    if (rc) return rc;
    if (!fallback) return h_best ? read_best(c, h_best, d_best, nf, st) : DPPS_OK;
    // frames whose proposals are all infeasible (or score below the
    // threshold), listed by the re-score's finalize: the exact search of the
    // full fine lattice with the frame's own variants, its records placed on
    // the device in stream order (no host round trip)
    const int tpf = (m->fine_nx * m->fine_ny + FB_TILE - 1) / FB_TILE;
    LaunchArgs a;
    memset(&a, 0, sizeof a);
    a.P = c->P;
    a.P.out_flags = 0;
    a.frames = m->ff;
    a.robots = b->d_robots;
    a.variants = b->d_variants;
    a.wins = m->fw;
    a.tiles = nullptr;
    a.tiles_per_frame = tpf;
    a.n_frames_dev = m->fcount;
    a.best_map = m->fmap;
    a.n_tiles = nf * tpf;
    a.n_frames = nf;
    a.tile_points = FB_TILE;
    a.persistent = 1;
    a.counter = m->fcounter;
    a.tile_rec = m->frec;
    a.best = d_best;
    const int per_cu = search_occupancy(c->p.n_samples, c->waves, a.tile_points);
    const int64_t cap = (int64_t)c->n_cu * per_cu;
    const int grid = (int)((int64_t)a.n_tiles < cap ? a.n_tiles : cap);
    if (launch_search(a, c->waves, grid, (void *)st, nullptr, nullptr))
        return fail(DPPS_E_DEVICE, "fallback search launch failed");
    if (n_fallback)
        HIP_OK(hipMemcpyAsync(m->h_count, m->fcount, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (h_best) {
        rc = read_best(c, h_best, d_best, nf, st);
        if (rc) return rc;
    } else if (n_fallback) {
        HIP_OK(hipStreamSynchronize(st));
    }
    if (n_fallback) *n_fallback = *m->h_count;
    return DPPS_OK;
}

extern "C" {

int dpps_surrogate_search(dpps_ctx *c, dpps_mlp *m, dpps_batch *b, int32_t k, dpps_best *d_best,
                          int fallback, float fallback_below, int32_t *n_fallback,
                          void *hip_stream)
{
    return surrogate_core(c, m, b, k, d_best, fallback, fallback_below, n_fallback, nullptr,
                          hip_stream);
}

int dpps_surrogate_search_frames(dpps_ctx *c, dpps_mlp *m, int32_t n_frames,
                                 const dpps_frame *frames, const dpps_robot *robots,
                                 const dpps_window *windows, const dpps_variant *variants,
                                 int32_t k, dpps_best *d_best, int fallback, float fallback_below,
                                 int32_t *n_fallback, dpps_best *h_best, void *hip_stream)
{
    if (!c || !m) return fail(DPPS_E_INVALID, "NULL argument");
    if (m->ctx != c) return fail(DPPS_E_INVALID, "network belongs to another context");
    HIP_OK(hipSetDevice(c->device));
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
    // the windows are validated but not searched: tables without tiles
    dpps_batch *b = &c->scratch;
    int rc = build_tables(&c->p, n_frames, frames, robots, windows, variants, 0, b->T);
    if (rc) return rc;
    b->n_frames = n_frames;
    b->tile_points = c->tile_points;
    rc = stage_tables(c, b, st);
    if (rc) return rc;
    return surrogate_core(c, m, b, k, d_best, fallback, fallback_below, n_fallback, h_best,
                          hip_stream);
}

}  // extern "C"

// C ABI of the coupling flow (declared in include/msx_flow.h): parameter and
// work-buffer ownership, the layer schedule of the forward, inverse and
// reverse-mode passes, and the fused sampling path.
#include "../../include/msx_flow.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "flow_launch.h"

using namespace msx;

struct msx_flow {
    int device = 0;
    int d = 0, L = 0, K = 0, H = 0, type = FT_BF16;
    int nh = 0, n_out = 0;
    int64_t per_layer = 0, P = 0;
    int64_t per_layer_t = 0;   // layer block of the operand copy (multiple of 8 elements)
    int64_t off[8] = {};  // W1 b1 W2 b2 W3 b3 W4 b4 within a layer
    std::vector<std::vector<int32_t>> trans, cond;
    float* params = nullptr;   // FP32 master
    void* params_t = nullptr;  // operand copy (BF16 or FP32), layer blocks of per_layer_t
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    int64_t adam_t = 0;
    // work buffers, grown on demand
    int64_t cap = 0;
    float* z = nullptr;      // [(L + 1)][d][cap]
    void* x0 = nullptr;      // [L][cap][nh]
    void* h = nullptr;       // [L][3][cap][H]
    float* theta = nullptr;  // [L][cap][n_out]
    float* logq = nullptr;   // [cap]
    float* G = nullptr;      // [cap]
    void* dtheta = nullptr;  // [cap][n_out]
    void* dha = nullptr;     // [cap][H]
    void* dhb = nullptr;     // [cap][H]
    float* dx0 = nullptr;    // [cap][nh]
    float* adj = nullptr;    // [d][cap]
    float* ldp = nullptr;    // [nh][cap] per-coordinate log-det terms
    float* part = nullptr;   // split-K partials
    int64_t part_cap = 0;
    double* lpart = nullptr;  // loss partials (1024) + loss (1)
    // sampling scratch
    int64_t scap = 0;
    float* su = nullptr;
    double* syd = nullptr;
    double* sjac = nullptr;
    float* sld = nullptr;
    std::string err;
};

namespace {

thread_local std::string g_ferr;

msx_status ffail(msx_flow* f, msx_status st, const std::string& msg) {
    if (f) f->err = msg;
    else g_ferr = msg;
    return st;
}

msx_status fdev(msx_flow* f, hipError_t e, const char* what) {
    return ffail(f, e == hipErrorOutOfMemory ? MSX_ERR_OOM : MSX_ERR_DEVICE,
                 std::string(what) + ": " + hipGetErrorString(e));
}

#define FHIP(f, call, what)                                 \
    do {                                                    \
        hipError_t _e = (call);                             \
        if (_e != hipSuccess) return fdev(f, _e, what);     \
    } while (0)

size_t tsize(int type) { return type == FT_BF16 ? 2 : 4; }

template <class T>
hipError_t fmalloc(T** p, size_t bytes) {
    return hipMalloc((void**)p, std::max<size_t>(bytes, 16));
}

void ffree(void* p) {
    if (p) (void)hipFree(p);
}

void free_work(msx_flow* f) {
    ffree(f->z);
    ffree(f->x0);
    ffree(f->h);
    ffree(f->theta);
    ffree(f->logq);
    ffree(f->G);
    ffree(f->dtheta);
    ffree(f->dha);
    ffree(f->dhb);
    ffree(f->dx0);
    ffree(f->adj);
    ffree(f->ldp);
    f->ldp = nullptr;
    f->z = nullptr;
    f->x0 = f->h = f->dtheta = f->dha = f->dhb = nullptr;
    f->theta = f->logq = f->G = f->dx0 = f->adj = nullptr;
    f->cap = 0;
}

// Work buffers for n events (all layers kept, as the reverse pass needs them).
msx_status ensure_work(msx_flow* f, int64_t n) {
    if (n <= f->cap) return MSX_OK;
    free_work(f);
    const size_t ts = tsize(f->type);
    const size_t N = (size_t)n;
    FHIP(f, fmalloc(&f->z, sizeof(float) * (size_t)(f->L + 1) * f->d * N), "flow work");
    FHIP(f, fmalloc(&f->x0, ts * (size_t)f->L * N * f->nh), "flow work");
    FHIP(f, fmalloc(&f->h, ts * (size_t)f->L * 3 * N * f->H), "flow work");
    FHIP(f, fmalloc(&f->theta, sizeof(float) * (size_t)f->L * N * f->n_out), "flow work");
    FHIP(f, fmalloc(&f->logq, sizeof(float) * N), "flow work");
    FHIP(f, fmalloc(&f->G, sizeof(float) * N), "flow work");
    FHIP(f, fmalloc(&f->dtheta, ts * N * f->n_out), "flow work");
    FHIP(f, fmalloc(&f->dha, ts * N * f->H), "flow work");
    FHIP(f, fmalloc(&f->dhb, ts * N * f->H), "flow work");
    FHIP(f, fmalloc(&f->dx0, sizeof(float) * N * f->nh), "flow work");
    FHIP(f, fmalloc(&f->adj, sizeof(float) * (size_t)f->d * N), "flow work");
    FHIP(f, fmalloc(&f->ldp, sizeof(float) * (size_t)f->nh * N), "flow work");
    f->cap = n;
    return MSX_OK;
}

// Split-K chunks of a weight-gradient GEMM over n events with an M x N
// output: about 1024 workgroups in all (64 x 128 output tiles), chunks of at
// least 256 events.
int splits_for(int64_t n, int M, int N) {
    const int64_t tiles = (int64_t)((M + 63) / 64) * ((N + 127) / 128);
    const int64_t want = std::max<int64_t>(1, 1024 / tiles);
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, n / 256));
}

msx_status ensure_part(msx_flow* f, int64_t floats) {
    if (floats <= f->part_cap) return MSX_OK;
    ffree(f->part);
    f->part = nullptr;
    f->part_cap = 0;
    FHIP(f, fmalloc(&f->part, sizeof(float) * (size_t)floats), "flow partials");
    f->part_cap = floats;
    return MSX_OK;
}

const char* tptr(const msx_flow* f, const void* base, int64_t elems) {
    return (const char*)base + (size_t)elems * tsize(f->type);
}
char* tptr(const msx_flow* f, void* base, int64_t elems) {
    return (char*)base + (size_t)elems * tsize(f->type);
}

GemmArgs gemm(const msx_flow* f, int M, int N, int K, const void* A, int64_t a_m, int64_t a_k, const void* B,
              int64_t b_k, int64_t b_n, int epi, void* out, int64_t ldc) {
    GemmArgs g{};
    g.type = f->type;
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = A;
    g.a_m = a_m;
    g.a_k = a_k;
    g.B = B;
    g.b_k = b_k;
    g.b_n = b_n;
    g.splits = 1;
    g.epi = epi;
    g.out = out;
    g.ldc = ldc;
    return g;
}

// MLP of layer l on the conditioning coordinates of z ([d][n]); hidden
// activations to h3 (3 consecutive [n][H] arrays), parameters to theta.
msx_status run_mlp(msx_flow* f, int l, const float* z, int64_t n, void* x0, void* h3, float* theta, hipStream_t s) {
    const int H = f->H, nh = f->nh;
    const int64_t base = l * f->per_layer;
    const void* W = tptr(f, f->params_t, l * f->per_layer_t - base);  // W + base + off = layer block + off
    FHIP(f, launch_gather(f->type, z, n, nh, f->cond[l].data(), x0, s), "flow gather");
    void* h1 = h3;
    void* h2 = tptr(f, h3, n * H);
    void* h3p = tptr(f, h3, 2 * n * H);
    GemmArgs g = gemm(f, (int)n, H, nh, x0, nh, 1, tptr(f, W, base + f->off[0]), 1, nh, EPI_BIAS_RELU, h1, H);
    g.bias = f->params + base + f->off[1];
    FHIP(f, launch_gemm(g, s), "flow gemm 1");
    g = gemm(f, (int)n, H, H, h1, H, 1, tptr(f, W, base + f->off[2]), 1, H, EPI_BIAS_RELU, h2, H);
    g.bias = f->params + base + f->off[3];
    FHIP(f, launch_gemm(g, s), "flow gemm 2");
    g = gemm(f, (int)n, H, H, h2, H, 1, tptr(f, W, base + f->off[4]), 1, H, EPI_BIAS_RELU, h3p, H);
    g.bias = f->params + base + f->off[5];
    FHIP(f, launch_gemm(g, s), "flow gemm 3");
    g = gemm(f, (int)n, f->n_out, H, h3p, H, 1, tptr(f, W, base + f->off[6]), 1, H, EPI_BIAS_F32, theta, f->n_out);
    g.bias = f->params + base + f->off[7];
    FHIP(f, launch_gemm(g, s), "flow gemm 4");
    return MSX_OK;
}

// dW[M][N] = sum_b A(b, m) B(b, n) over the batch (split-K), into grad.
msx_status weight_grad(msx_flow* f, int M, int N, int64_t n, const void* A, int64_t lda, const void* B, int64_t ldb,
                       float* out, hipStream_t s) {
    const int splits = splits_for(n, M, N);
    if (msx_status st = ensure_part(f, (int64_t)splits * M * N)) return st;
    GemmArgs g = gemm(f, M, N, (int)n, A, 1, lda, B, ldb, 1, EPI_PARTIAL, f->part, N);
    g.splits = splits;
    FHIP(f, launch_gemm(g, s), "flow weight gradient");
    FHIP(f, launch_reduce_partials(f->part, splits, M, N, out, N, s), "flow reduce");
    return MSX_OK;
}

msx_status bias_grad(msx_flow* f, const void* X, int64_t n, int N, float* out, hipStream_t s) {
    const int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(256, n / 256));
    if (msx_status st = ensure_part(f, (int64_t)chunks * N)) return st;
    FHIP(f, launch_colsum(f->type, X, n, N, N, f->part, chunks, out, s), "flow bias gradient");
    return MSX_OK;
}

// The one-kernel coupling layer covers BF16 conditioners of hidden width 128
// with up to 16 bins.
bool fused_ok(const msx_flow* f) {
    return f->type == FT_BF16 && f->H == kFusedHidden && f->K <= kFusedMaxBins;
}

// Inverse pass over all layers keeping every intermediate: z[L] = y, z[l] =
// layer l inverted from z[l + 1]; logq accumulates log |du/dy|.
msx_status inverse_saving(msx_flow* f, int64_t n, const float* y, hipStream_t s) {
    const size_t zs = (size_t)f->d * n;
    float* zl = f->z + (size_t)f->L * zs;
    FHIP(f, hipMemcpyAsync(zl, y, sizeof(float) * zs, hipMemcpyDeviceToDevice, s), "flow copy");
    FHIP(f, hipMemsetAsync(f->logq, 0, sizeof(float) * n, s), "flow clear");
    for (int l = f->L - 1; l >= 0; --l) {
        float* zin = f->z + (size_t)(l + 1) * zs;
        float* zout = f->z + (size_t)l * zs;
        void* x0 = tptr(f, f->x0, (int64_t)l * n * f->nh);
        void* h = tptr(f, f->h, (int64_t)l * 3 * n * f->H);
        float* th = f->theta + (size_t)l * n * f->n_out;
        if (fused_ok(f)) {
            FHIP(f, hipMemcpyAsync(zout, zin, sizeof(float) * zs, hipMemcpyDeviceToDevice, s), "flow copy");
            FHIP(f,
                 launch_flow_layer(true, zout, n, tptr(f, f->params_t, l * f->per_layer_t),
                                   f->params + (int64_t)l * f->per_layer, f->off, f->nh, f->trans[l].data(),
                                   f->cond[l].data(), f->K, f->logq, x0, h, th, s),
                 "flow layer");
            continue;
        }
        if (msx_status st = run_mlp(f, l, zin, n, x0, h, th, s)) return st;
        FHIP(f, hipMemcpyAsync(zout, zin, sizeof(float) * zs, hipMemcpyDeviceToDevice, s), "flow copy");
        FHIP(f, launch_spline(true, zout, n, th, f->n_out, f->nh, f->trans[l].data(), f->K, f->logq, f->ldp, s),
             "flow spline");
    }
    return MSX_OK;
}

msx_status gradient(msx_flow* f, int64_t n, const float* y, const double* wfj, const float* logq_old, float* grad,
                    double* loss, bool log_loss, hipStream_t s) {
    if (msx_status st = ensure_work(f, n)) return st;
    if (!f->lpart) FHIP(f, fmalloc(&f->lpart, sizeof(double) * 1025), "flow loss partials");
    if (msx_status st = inverse_saving(f, n, y, s)) return st;
    FHIP(f, launch_flow_loss(n, wfj, f->logq, logq_old, f->G, f->lpart, loss ? loss : f->lpart + 1024, log_loss, s),
         "flow loss");
    const size_t zs = (size_t)f->d * n;
    FHIP(f, hipMemsetAsync(f->adj, 0, sizeof(float) * zs, s), "flow clear");
    const int H = f->H, nh = f->nh, no = f->n_out;
    for (int l = 0; l < f->L; ++l) {
        const int64_t base = l * f->per_layer;
        const void* W = tptr(f, f->params_t, l * f->per_layer_t - base);  // W + base + off = layer block + off
        const float* zin = f->z + (size_t)(l + 1) * zs;
        const float* th = f->theta + (size_t)l * n * no;
        const void* x0 = tptr(f, f->x0, (int64_t)l * n * nh);
        const void* h1 = tptr(f, f->h, (int64_t)l * 3 * n * H);
        const void* h2 = tptr(f, h1, n * H);
        const void* h3 = tptr(f, h1, 2 * n * H);
        FHIP(f,
             launch_spline_backward(f->type, zin, f->adj, n, th, no, nh, f->trans[l].data(), f->K, f->G, f->dtheta, s),
             "flow spline backward");
        // layer 4
        if (msx_status st = weight_grad(f, no, H, n, f->dtheta, no, h3, H, grad + base + f->off[6], s)) return st;
        if (msx_status st = bias_grad(f, f->dtheta, n, no, grad + base + f->off[7], s)) return st;
        GemmArgs g = gemm(f, (int)n, H, no, f->dtheta, no, 1, tptr(f, W, base + f->off[6]), H, 1, EPI_RELU_MASK,
                          f->dha, H);
        g.mask = h3;
        g.ldm = H;
        FHIP(f, launch_gemm(g, s), "flow backward gemm 4");
        // layer 3
        if (msx_status st = weight_grad(f, H, H, n, f->dha, H, h2, H, grad + base + f->off[4], s)) return st;
        if (msx_status st = bias_grad(f, f->dha, n, H, grad + base + f->off[5], s)) return st;
        g = gemm(f, (int)n, H, H, f->dha, H, 1, tptr(f, W, base + f->off[4]), H, 1, EPI_RELU_MASK, f->dhb, H);
        g.mask = h2;
        g.ldm = H;
        FHIP(f, launch_gemm(g, s), "flow backward gemm 3");
        // layer 2
        if (msx_status st = weight_grad(f, H, H, n, f->dhb, H, h1, H, grad + base + f->off[2], s)) return st;
        if (msx_status st = bias_grad(f, f->dhb, n, H, grad + base + f->off[3], s)) return st;
        g = gemm(f, (int)n, H, H, f->dhb, H, 1, tptr(f, W, base + f->off[2]), H, 1, EPI_RELU_MASK, f->dha, H);
        g.mask = h1;
        g.ldm = H;
        FHIP(f, launch_gemm(g, s), "flow backward gemm 2");
        // layer 1 and the conditioning coordinates
        if (msx_status st = weight_grad(f, H, nh, n, f->dha, H, x0, nh, grad + base + f->off[0], s)) return st;
        if (msx_status st = bias_grad(f, f->dha, n, H, grad + base + f->off[1], s)) return st;
        g = gemm(f, (int)n, nh, H, f->dha, H, 1, tptr(f, W, base + f->off[0]), nh, 1, EPI_F32, f->dx0, nh);
        FHIP(f, launch_gemm(g, s), "flow backward gemm 1");
        FHIP(f, launch_scatter_add(f->adj, f->dx0, n, nh, f->cond[l].data(), s), "flow scatter");
    }
    return MSX_OK;
}

msx_status check_events(msx_flow* f, int64_t n) {
    if (n < 0) return ffail(f, MSX_ERR_ARG, "n < 0");
    if (n > (int64_t)INT32_MAX) return ffail(f, MSX_ERR_ARG, "n exceeds 2^31 - 1 events per call");
    return MSX_OK;
}

}  // namespace

extern "C" {

const char* msx_flow_last_error(const msx_flow* f) { return f ? f->err.c_str() : g_ferr.c_str(); }

msx_status msx_flow_create(int32_t dims, int32_t layers, int32_t bins, int32_t hidden, int32_t mlp_type,
                           int32_t device, msx_flow** out) {
    if (!out) return ffail(nullptr, MSX_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (dims < 2 || dims > 2 * kFlowMaxHalf || dims % 2) return ffail(nullptr, MSX_ERR_ARG, "dims must be even, 2..64");
    if (layers < 1 || layers > 64) return ffail(nullptr, MSX_ERR_ARG, "layers must be 1..64");
    if (bins < 1 || bins > kFlowMaxBins) return ffail(nullptr, MSX_ERR_ARG, "bins must be 1..32");
    if (hidden < 1 || hidden > 1024) return ffail(nullptr, MSX_ERR_ARG, "hidden must be 1..1024");
    if (mlp_type != MSX_FLOW_BF16 && mlp_type != MSX_FLOW_FP32)
        return ffail(nullptr, MSX_ERR_ARG, "mlp_type must be MSX_FLOW_BF16 or MSX_FLOW_FP32");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return ffail(nullptr, MSX_ERR_DEVICE, "no such HIP device");
    if (hipSetDevice(device) != hipSuccess) return ffail(nullptr, MSX_ERR_DEVICE, "hipSetDevice failed");
    msx_flow* f = new msx_flow();
    f->device = device;
    f->d = dims;
    f->L = layers;
    f->K = bins;
    f->H = hidden;
    f->type = mlp_type == MSX_FLOW_BF16 ? FT_BF16 : FT_F32;
    f->nh = dims / 2;
    f->n_out = f->nh * (3 * bins + 1);
    const int64_t H = hidden, nh = f->nh, no = f->n_out;
    const int64_t sizes[8] = {H * nh, H, H * H, H, H * H, H, no * H, no};
    int64_t o = 0;
    for (int i = 0; i < 8; ++i) {
        f->off[i] = o;
        o += sizes[i];
    }
    f->per_layer = o;
    f->per_layer_t = (o + 7) / 8 * 8;
    f->P = o * layers;
    for (int l = 0; l < layers; ++l) {
        std::vector<int32_t> t, c;
        const int md = l % 4;
        for (int i = 0; i < dims; ++i) {
            bool tr = md == 0 ? i < dims / 2 : md == 1 ? i >= dims / 2 : md == 2 ? (i % 2 == 0) : (i % 2 == 1);
            (tr ? t : c).push_back(i);
        }
        f->trans.push_back(t);
        f->cond.push_back(c);
    }
    const size_t P = (size_t)f->P;
    hipError_t e = hipSuccess;
    const size_t PT = (size_t)f->per_layer_t * layers;
    if ((e = fmalloc(&f->params, 4 * P)) != hipSuccess || (e = fmalloc(&f->params_t, tsize(f->type) * PT)) != hipSuccess ||
        (e = fmalloc(&f->m, 4 * P)) != hipSuccess || (e = fmalloc(&f->v, 4 * P)) != hipSuccess ||
        (e = fmalloc(&f->grad, 4 * P)) != hipSuccess) {
        msx_flow_destroy(f);
        return ffail(nullptr, e == hipErrorOutOfMemory ? MSX_ERR_OOM : MSX_ERR_DEVICE, "flow parameters");
    }
    if (hipMemset(f->params, 0, 4 * P) != hipSuccess || hipMemset(f->params_t, 0, tsize(f->type) * PT) != hipSuccess ||
        hipMemset(f->m, 0, 4 * P) != hipSuccess || hipMemset(f->v, 0, 4 * P) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        msx_flow_destroy(f);
        return ffail(nullptr, MSX_ERR_DEVICE, "flow parameter initialisation");
    }
    *out = f;
    return MSX_OK;
}

msx_status msx_flow_destroy(msx_flow* f) {
    if (!f) return MSX_OK;
    (void)hipSetDevice(f->device);
    free_work(f);
    ffree(f->params);
    ffree(f->params_t);
    ffree(f->m);
    ffree(f->v);
    ffree(f->grad);
    ffree(f->part);
    ffree(f->lpart);
    ffree(f->su);
    ffree(f->syd);
    ffree(f->sjac);
    ffree(f->sld);
    delete f;
    return MSX_OK;
}

msx_status msx_flow_param_count(const msx_flow* f, int64_t* n) {
    if (!f || !n) return ffail(nullptr, MSX_ERR_ARG, "flow and n are required");
    *n = f->P;
    return MSX_OK;
}

msx_status msx_flow_set_params(msx_flow* f, const float* host, int64_t n) {
    if (!f) return ffail(nullptr, MSX_ERR_ARG, "flow is NULL");
    if (!host || n != f->P) return ffail(f, MSX_ERR_ARG, "expected host pointer and n == parameter count");
    FHIP(f, hipSetDevice(f->device), "hipSetDevice");
    FHIP(f, hipDeviceSynchronize(), "flow synchronise");
    FHIP(f, hipMemcpy(f->params, host, sizeof(float) * n, hipMemcpyHostToDevice), "flow set params");
    FHIP(f, hipMemset(f->m, 0, sizeof(float) * n), "flow clear");
    FHIP(f, hipMemset(f->v, 0, sizeof(float) * n), "flow clear");
    f->adam_t = 0;
    FHIP(f, launch_cast(n, f->params, f->type, f->params_t, f->per_layer, f->per_layer_t, nullptr), "flow cast");
    FHIP(f, hipDeviceSynchronize(), "flow synchronise");
    return MSX_OK;
}

msx_status msx_flow_get_params(msx_flow* f, float* host, int64_t n) {
    if (!f) return ffail(nullptr, MSX_ERR_ARG, "flow is NULL");
    if (!host || n != f->P) return ffail(f, MSX_ERR_ARG, "expected host pointer and n == parameter count");
    FHIP(f, hipSetDevice(f->device), "hipSetDevice");
    FHIP(f, hipDeviceSynchronize(), "flow synchronise");
    FHIP(f, hipMemcpy(host, f->params, sizeof(float) * n, hipMemcpyDeviceToHost), "flow get params");
    return MSX_OK;
}

namespace {
// Layout of a serialised flow state: this header, then the FP32 master
// parameters, Adam's first and second moments (P floats each).
struct FlowStateHeader {
    char magic[8];  // "MSXFLOW1"
    int32_t d, L, K, H, type, pad;
    int64_t P, adam_t;
};
constexpr char kFlowMagic[8] = {'M', 'S', 'X', 'F', 'L', 'O', 'W', '1'};
}  // namespace

msx_status msx_flow_get_state(msx_flow* f, void* buf, size_t* size) {
    if (!f) return ffail(nullptr, MSX_ERR_ARG, "flow is NULL");
    if (!size) return ffail(f, MSX_ERR_ARG, "size is NULL");
    const size_t need = sizeof(FlowStateHeader) + 3 * sizeof(float) * (size_t)f->P;
    if (!buf) {
        *size = need;
        return MSX_OK;
    }
    if (*size < need) return ffail(f, MSX_ERR_ARG, "state buffer too small");
    FlowStateHeader h{};
    std::memcpy(h.magic, kFlowMagic, 8);
    h.d = f->d;
    h.L = f->L;
    h.K = f->K;
    h.H = f->H;
    h.type = f->type;
    h.P = f->P;
    h.adam_t = f->adam_t;
    char* b = (char*)buf;
    std::memcpy(b, &h, sizeof h);
    float* body = (float*)(b + sizeof h);
    FHIP(f, hipSetDevice(f->device), "hipSetDevice");
    FHIP(f, hipDeviceSynchronize(), "flow synchronise");
    FHIP(f, hipMemcpy(body, f->params, sizeof(float) * f->P, hipMemcpyDeviceToHost), "flow state");
    FHIP(f, hipMemcpy(body + f->P, f->m, sizeof(float) * f->P, hipMemcpyDeviceToHost), "flow state");
    FHIP(f, hipMemcpy(body + 2 * f->P, f->v, sizeof(float) * f->P, hipMemcpyDeviceToHost), "flow state");
    *size = need;
    return MSX_OK;
}

msx_status msx_flow_set_state(msx_flow* f, const void* buf, size_t size) {
    if (!f) return ffail(nullptr, MSX_ERR_ARG, "flow is NULL");
    if (!buf || size < sizeof(FlowStateHeader)) return ffail(f, MSX_ERR_ARG, "state buffer too small");
    FlowStateHeader h;
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, kFlowMagic, 8) != 0) return ffail(f, MSX_ERR_STATE, "not a flow state");
    if (h.d != f->d || h.L != f->L || h.K != f->K || h.H != f->H || h.type != f->type || h.P != f->P)
        return ffail(f, MSX_ERR_STATE, "flow state of a different shape");
    if (size != sizeof h + 3 * sizeof(float) * (size_t)f->P) return ffail(f, MSX_ERR_STATE, "flow state size");
    if (h.adam_t < 0) return ffail(f, MSX_ERR_STATE, "negative Adam step count");
    const float* body = (const float*)((const char*)buf + sizeof h);
    for (int64_t i = 0; i < 3 * f->P; ++i)
        if (!std::isfinite(body[i])) return ffail(f, MSX_ERR_STATE, "flow state holds a non-finite value");
    FHIP(f, hipSetDevice(f->device), "hipSetDevice");
    FHIP(f, hipDeviceSynchronize(), "flow synchronise");
    FHIP(f, hipMemcpy(f->params, body, sizeof(float) * f->P, hipMemcpyHostToDevice), "flow state");
    FHIP(f, hipMemcpy(f->m, body + f->P, sizeof(float) * f->P, hipMemcpyHostToDevice), "flow state");
    FHIP(f, hipMemcpy(f->v, body + 2 * f->P, sizeof(float) * f->P, hipMemcpyHostToDevice), "flow state");
    f->adam_t = h.adam_t;
    FHIP(f, launch_cast(f->P, f->params, f->type, f->params_t, f->per_layer, f->per_layer_t, nullptr), "flow cast");
    FHIP(f, hipDeviceSynchronize(), "flow synchronise");
    return MSX_OK;
}

msx_status msx_flow_dims(const msx_flow* f, int32_t* dims) {
    if (!f || !dims) return ffail(nullptr, MSX_ERR_ARG, "flow and dims are required");
    *dims = f->d;
    return MSX_OK;
}

msx_status msx_flow_forward(msx_flow* f, int64_t n, const float* u, float* y, float* logdet, void* stream) {
    if (!f) return ffail(nullptr, MSX_ERR_ARG, "flow is NULL");
    if (msx_status st = check_events(f, n)) return st;
    if (n == 0) return MSX_OK;
    if (!u || !y || !logdet) return ffail(f, MSX_ERR_ARG, "u, y and logdet are required");
    hipStream_t s = (hipStream_t)stream;
    FHIP(f, hipSetDevice(f->device), "hipSetDevice");
    // whole layers in one kernel where the shape allows it (BF16, hidden 128,
    // <= 16 bins, 16-byte aligned layer blocks); no work buffers then
    const bool fused = fused_ok(f);
    if (!fused)
        if (msx_status st = ensure_work(f, n)) return st;
    if (y != u) FHIP(f, hipMemcpyAsync(y, u, sizeof(float) * (size_t)f->d * n, hipMemcpyDeviceToDevice, s), "flow copy");
    FHIP(f, hipMemsetAsync(logdet, 0, sizeof(float) * n, s), "flow clear");
    for (int l = 0; l < f->L; ++l) {
        if (fused) {
            const int64_t base = l * f->per_layer;
            FHIP(f,
                 launch_flow_layer(false, y, n, tptr(f, f->params_t, l * f->per_layer_t), f->params + base, f->off,
                                   f->nh, f->trans[l].data(), f->cond[l].data(), f->K, logdet, nullptr, nullptr,
                                   nullptr, s),
                 "flow layer");
            continue;
        }
        if (msx_status st = run_mlp(f, l, y, n, f->x0, f->h, f->theta, s)) return st;
        FHIP(f, launch_spline(false, y, n, f->theta, f->n_out, f->nh, f->trans[l].data(), f->K, logdet, f->ldp, s),
             "flow spline");
    }
    return MSX_OK;
}

msx_status msx_flow_inverse(msx_flow* f, int64_t n, const float* y, float* u, float* logq, void* stream) {
    if (!f) return ffail(nullptr, MSX_ERR_ARG, "flow is NULL");
    if (msx_status st = check_events(f, n)) return st;
    if (n == 0) return MSX_OK;
    if (!u || !y || !logq) return ffail(f, MSX_ERR_ARG, "y, u and logq are required");
    hipStream_t s = (hipStream_t)stream;
    FHIP(f, hipSetDevice(f->device), "hipSetDevice");
    const bool fused = fused_ok(f);
    if (!fused)
        if (msx_status st = ensure_work(f, n)) return st;
    if (y != u) FHIP(f, hipMemcpyAsync(u, y, sizeof(float) * (size_t)f->d * n, hipMemcpyDeviceToDevice, s), "flow copy");
    FHIP(f, hipMemsetAsync(logq, 0, sizeof(float) * n, s), "flow clear");
    for (int l = f->L - 1; l >= 0; --l) {
        if (fused) {
            FHIP(f,
                 launch_flow_layer(true, u, n, tptr(f, f->params_t, l * f->per_layer_t),
                                   f->params + (int64_t)l * f->per_layer, f->off, f->nh, f->trans[l].data(),
                                   f->cond[l].data(), f->K, logq, nullptr, nullptr, nullptr, s),
                 "flow layer");
            continue;
        }
        if (msx_status st = run_mlp(f, l, u, n, f->x0, f->h, f->theta, s)) return st;
        FHIP(f, launch_spline(true, u, n, f->theta, f->n_out, f->nh, f->trans[l].data(), f->K, logq, f->ldp, s),
             "flow spline");
    }
    return MSX_OK;
}

msx_status msx_flow_gradient(msx_flow* f, int64_t n, const float* y, const double* wfj, const float* logq_old,
                             float* grad, double* loss, void* stream) {
    if (!f) return ffail(nullptr, MSX_ERR_ARG, "flow is NULL");
    if (msx_status st = check_events(f, n)) return st;
    if (n == 0) return ffail(f, MSX_ERR_ARG, "empty batch");
    if (!y || !wfj || !logq_old || !grad) return ffail(f, MSX_ERR_ARG, "y, wfj, logq_old and grad are required");
    FHIP(f, hipSetDevice(f->device), "hipSetDevice");
    return gradient(f, n, y, wfj, logq_old, grad, loss, false, (hipStream_t)stream);
}

msx_status msx_flow_train_step(msx_flow* f, int64_t n, const float* y, const double* wfj, const float* logq_old,
                               float lr, double* loss, void* stream) {
    if (!f) return ffail(nullptr, MSX_ERR_ARG, "flow is NULL");
    if (msx_status st = check_events(f, n)) return st;
    if (n == 0) return ffail(f, MSX_ERR_ARG, "empty batch");
    if (!y || !wfj || !logq_old) return ffail(f, MSX_ERR_ARG, "y, wfj and logq_old are required");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return ffail(f, MSX_ERR_ARG, "lr must be positive");
    hipStream_t s = (hipStream_t)stream;
    FHIP(f, hipSetDevice(f->device), "hipSetDevice");
    if (msx_status st = gradient(f, n, y, wfj, logq_old, f->grad, loss, true, s)) return st;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    f->adam_t += 1;
    const double c1 = 1.0 - std::pow(b1, (double)f->adam_t), c2 = 1.0 - std::pow(b2, (double)f->adam_t);
    const float lr_t = (float)(lr * std::sqrt(c2) / c1), eps_t = (float)(eps * std::sqrt(c2));
    FHIP(f, launch_adam(f->P, f->params, f->grad, f->m, f->v, (float)b1, (float)b2, lr_t, eps_t, f->type, f->params_t,
                        f->per_layer, f->per_layer_t, s),
         "flow adam");
    return MSX_OK;
}

msx_status msx_flow_sample(msx_flow* f, msx_ctx* ctx, int32_t channel, int64_t n, uint64_t seed, uint64_t stream_id,
                           uint64_t counter_offset, float* y, float* logq, double* p, double* x1x2, double* wfj,
                           double* w, void* stream) {
    if (!f) return ffail(nullptr, MSX_ERR_ARG, "flow is NULL");
    if (!ctx) return ffail(f, MSX_ERR_ARG, "ctx is NULL");
    if (msx_status st = check_events(f, n)) return st;
    int64_t dims = 0;
    if (msx_get_meta(ctx, MSX_META_DIMS, channel, &dims) != MSX_OK)
        return ffail(f, MSX_ERR_ARG, std::string("channel: ") + msx_last_error(ctx));
    if (dims != f->d) return ffail(f, MSX_ERR_ARG, "the channel's dimension differs from the flow's");
    if (n == 0) return MSX_OK;
    if (!y || !logq || !p || !wfj || !w) return ffail(f, MSX_ERR_ARG, "y, logq, p, wfj and w are required");
    if (counter_offset > UINT64_MAX - (uint64_t)n) return ffail(f, MSX_ERR_ARG, "event ids overflow the counter");
    hipStream_t s = (hipStream_t)stream;
    FHIP(f, hipSetDevice(f->device), "hipSetDevice");
    if (n > f->scap) {
        ffree(f->su);
        ffree(f->syd);
        ffree(f->sjac);
        ffree(f->sld);
        f->su = nullptr;
        f->syd = nullptr;
        f->sjac = nullptr;
        f->sld = nullptr;
        f->scap = 0;
        FHIP(f, fmalloc(&f->su, sizeof(float) * (size_t)f->d * n), "flow sample scratch");
        FHIP(f, fmalloc(&f->syd, sizeof(double) * (size_t)f->d * n), "flow sample scratch");
        FHIP(f, fmalloc(&f->sjac, sizeof(double) * (size_t)n), "flow sample scratch");
        FHIP(f, fmalloc(&f->sld, sizeof(float) * (size_t)n), "flow sample scratch");
        f->scap = n;
    }
    FHIP(f, launch_uniform_f32(seed, stream_id, counter_offset, n, f->d, f->su, s), "flow uniforms");
    if (msx_status st = msx_flow_forward(f, n, f->su, y, f->sld, stream)) return st;
    FHIP(f, launch_widen((int64_t)f->d * n, y, f->syd, s), "flow widen");
    if (msx_status st = msx_map(ctx, channel, n, f->syd, p, x1x2, f->sjac, wfj, stream))
        return ffail(f, st, std::string("map: ") + msx_last_error(ctx));
    FHIP(f, launch_flow_weight(n, wfj, f->sld, w, logq, s), "flow weight");
    return MSX_OK;
}

}  // extern "C"

// The learned cost models of libhb: 16 -> 64 -> 64 -> 2 MLPs (ReLU), trained
// on the GPU by this library's kernels (matrix-core GEMM with bf16 operands
// and fp32 accumulation, Adam).  Two of the same shape: the block model over
// per-(block, predicate) features predicting (pass rate, cost), which the
// learned plan reads, and the paper's per-pair network over features of a
// predicate and two tuples' values predicting (satisfied, time of the
// check), whose summed estimates give the predicates' costs (Section 4.2,
// "Shallow NNs", "Estimated cost"; Adam and ReLU as in the paper's
// defaults, Section 6).
#include <cmath>
#include <cstdio>

#include "hb_ctx.h"

namespace hb {

// Parameter layout (fp32, row-major, used as x W + b).
constexpr int kIn = 16, kHid = 64, kOut = 2;
constexpr int kW1 = 0, kB1 = kW1 + kIn * kHid, kW2 = kB1 + kHid, kB2 = kW2 + kHid * kHid;
constexpr int kW3 = kB2 + kHid, kB3 = kW3 + kHid * kOut, kParams = kB3 + kOut;
static_assert(kParams == HB_MLP_PARAMS, "parameter count");

CostModel& selected_model(Ctx* c) { return c->model_sel == HB_MODEL_PAIR ? c->pair_model : c->model; }

namespace {

// Activations of one batch of `n` rows.
struct Acts {
    DevBuf z1, h1, z2, h2, y, dy, dz2, dz1, grad, sse;
    int cap = 0;
    void ensure(Ctx* c, int n) {
        if (n <= cap) return;
        z1.alloc(c, sizeof(float) * n * kHid);
        h1.alloc(c, sizeof(float) * n * kHid);
        z2.alloc(c, sizeof(float) * n * kHid);
        h2.alloc(c, sizeof(float) * n * kHid);
        y.alloc(c, sizeof(float) * n * kOut);
        dy.alloc(c, sizeof(float) * n * kOut);
        dz2.alloc(c, sizeof(float) * n * kHid);
        dz1.alloc(c, sizeof(float) * n * kHid);
        grad.alloc(c, sizeof(float) * kParams);
        sse.alloc(c, sizeof(float));
        cap = n;
    }
};

GemmArgs gemm(const float* A, int lda, int ta, const float* B, int ldb, int tb, float* C, int ldc, int M, int N,
              int K) {
    GemmArgs g{};
    g.A = A; g.lda = lda; g.transA = ta;
    g.B = B; g.ldb = ldb; g.transB = tb;
    g.C = C; g.ldc = ldc;
    g.M = M; g.N = N; g.K = K;
    return g;
}

void forward(Ctx* c, const float* W, const float* x, int n, Acts& a) {
    GemmArgs g = gemm(x, kIn, 0, W + kW1, kHid, 0, a.z1.as<float>(), kHid, n, kHid, kIn);
    g.bias = W + kB1;
    g.relu = a.h1.as<float>();
    HB_HIP(launch_gemm(g, c->stream));
    g = gemm(a.h1.as<float>(), kHid, 0, W + kW2, kHid, 0, a.z2.as<float>(), kHid, n, kHid, kHid);
    g.bias = W + kB2;
    g.relu = a.h2.as<float>();
    HB_HIP(launch_gemm(g, c->stream));
    g = gemm(a.h2.as<float>(), kHid, 0, W + kW3, kOut, 0, a.y.as<float>(), kOut, n, kOut, kHid);
    g.bias = W + kB3;
    HB_HIP(launch_gemm(g, c->stream));
}

// gradients of the mean squared error of the batch into a.grad
void backward(Ctx* c, const float* W, const float* x, const float* t, int n, Acts& a) {
    float* G = a.grad.as<float>();
    zero(c, a.sse.get(), sizeof(float));
    HB_HIP(launch_mse_grad(a.y.as<float>(), t, n * kOut, 1.f / (float)(n * kOut), a.dy.as<float>(), a.sse.as<float>(),
                           c->stream));
    HB_HIP(launch_gemm(gemm(a.h2.as<float>(), kHid, 1, a.dy.as<float>(), kOut, 0, G + kW3, kOut, kHid, kOut, n),
                       c->stream));
    HB_HIP(launch_colsum(a.dy.as<float>(), n, kOut, G + kB3, c->stream));
    GemmArgs g = gemm(a.dy.as<float>(), kOut, 0, W + kW3, kOut, 1, a.dz2.as<float>(), kHid, n, kHid, kOut);
    g.mask = a.z2.as<float>();
    HB_HIP(launch_gemm(g, c->stream));
    HB_HIP(launch_gemm(gemm(a.h1.as<float>(), kHid, 1, a.dz2.as<float>(), kHid, 0, G + kW2, kHid, kHid, kHid, n),
                       c->stream));
    HB_HIP(launch_colsum(a.dz2.as<float>(), n, kHid, G + kB2, c->stream));
    g = gemm(a.dz2.as<float>(), kHid, 0, W + kW2, kHid, 1, a.dz1.as<float>(), kHid, n, kHid, kHid);
    g.mask = a.z1.as<float>();
    HB_HIP(launch_gemm(g, c->stream));
    HB_HIP(launch_gemm(gemm(x, kIn, 1, a.dz1.as<float>(), kHid, 0, G + kW1, kHid, kIn, kHid, n), c->stream));
    HB_HIP(launch_colsum(a.dz1.as<float>(), n, kHid, G + kB1, c->stream));
}

void adam(Ctx* c, const float* grad, float lr) {
    CostModel& m = selected_model(c);
    m.adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)m.adam_t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)m.adam_t)));
    HB_HIP(launch_adam(m.params.as<float>(), grad, m.m.as<float>(), m.v.as<float>(), kParams, lr, (float)b1,
                       (float)b2, 1e-8f, c1, c2, c->stream));
}

void ensure_model(Ctx* c) {
    CostModel& m = selected_model(c);
    if (m.params.get()) return;
    m.params.alloc(c, sizeof(float) * kParams);
    m.m.alloc(c, sizeof(float) * kParams);
    m.v.alloc(c, sizeof(float) * kParams);
    zero(c, m.params.get(), sizeof(float) * kParams);
    zero(c, m.m.get(), sizeof(float) * kParams);
    zero(c, m.v.get(), sizeof(float) * kParams);
}

void reset_adam(Ctx* c) {
    CostModel& m = selected_model(c);
    zero(c, m.m.get(), sizeof(float) * kParams);
    zero(c, m.v.get(), sizeof(float) * kParams);
    m.adam_t = 0;
}

uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// device copy of host or device rows
const float* rows_on_device(Ctx* c, const float* p, size_t count, int on_device, DevBuf& hold) {
    if (on_device) return p;
    hold.alloc(c, sizeof(float) * std::max<size_t>(count, 1));
    if (count) HB_HIP(hipMemcpyAsync(hold.get(), p, sizeof(float) * count, hipMemcpyHostToDevice, c->stream));
    return hold.as<float>();
}

}  // namespace

void costmodel_init(Ctx* c, uint64_t seed) {
    ensure_model(c);
    std::vector<float> w(kParams, 0.f);
    uint64_t s = seed;
    auto fill = [&](int off, int fan_in, int count) {
        const double lim = std::sqrt(6.0 / fan_in);
        for (int x = 0; x < count; ++x) {
            const double u = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
            w[off + x] = (float)((2.0 * u - 1.0) * lim);
        }
    };
    fill(kW1, kIn, kIn * kHid);
    fill(kW2, kHid, kHid * kHid);
    fill(kW3, kHid, kHid * kOut);
    HB_HIP(hipMemcpyAsync(selected_model(c).params.get(), w.data(), sizeof(float) * kParams, hipMemcpyHostToDevice, c->stream));
    reset_adam(c);
    selected_model(c).ready = true;
    c->sync();
}

void costmodel_set(Ctx* c, const float* p, uint32_t n) {
    if (!p || n != (uint32_t)kParams) fail(HB_ERR_INVALID_ARG, "expected HB_MLP_PARAMS floats");
    ensure_model(c);
    HB_HIP(hipMemcpyAsync(selected_model(c).params.get(), p, sizeof(float) * kParams, hipMemcpyHostToDevice, c->stream));
    reset_adam(c);
    selected_model(c).ready = true;
    c->sync();
}

void costmodel_get(Ctx* c, float* p, uint32_t n) {
    if (!p || n != (uint32_t)kParams) fail(HB_ERR_INVALID_ARG, "expected HB_MLP_PARAMS floats");
    if (!selected_model(c).ready) fail(HB_ERR_STATE, "no cost model (hb_costmodel_init / set / train first)");
    HB_HIP(hipMemcpyAsync(p, selected_model(c).params.get(), sizeof(float) * kParams, hipMemcpyDeviceToHost, c->stream));
    c->sync();
}

void costmodel_train(Ctx* c, const float* x, const float* t, uint64_t n, int on_device, uint32_t epochs,
                     uint32_t batch, float lr, float* final_loss) {
    if (!x || !t || n == 0 || batch == 0) fail(HB_ERR_INVALID_ARG, "empty training set");
    if (n > (1ull << 30)) fail(HB_ERR_LIMIT, "more than 2^30 training rows");
    if (!selected_model(c).ready) costmodel_init(c, 0x48420007ull);
    DevBuf hx, ht;
    const float* dx = rows_on_device(c, x, n * kIn, on_device, hx);
    const float* dt = rows_on_device(c, t, n * kOut, on_device, ht);
    Acts a;
    const int b = (int)std::min<uint64_t>(batch, n);
    a.ensure(c, b);
    double last = 0.0;
    for (uint32_t e = 0; e < epochs; ++e) {
        double sse = 0.0;
        for (uint64_t r0 = 0; r0 < n; r0 += b) {
            const int nb = (int)std::min<uint64_t>(b, n - r0);
            const float* xb = dx + r0 * kIn;
            const float* tb = dt + r0 * kOut;
            forward(c, selected_model(c).params.as<float>(), xb, nb, a);
            backward(c, selected_model(c).params.as<float>(), xb, tb, nb, a);
            adam(c, a.grad.as<float>(), lr);
            if (e + 1 == epochs) sse += read1(c, a.sse.as<float>());
        }
        last = sse / (double)(n * kOut);
    }
    c->sync();
    if (final_loss) *final_loss = (float)last;
}

void model_forward(Ctx* c, const CostModel& m, const float* x, uint64_t n, float* y) {
    HB_HIP(launch_mlp_forward(m.params.as<float>(), x, n, y, c->stream));
}

void costmodel_predict(Ctx* c, const float* x, uint64_t n, int on_device, float* y, int y_on_device) {
    if (!selected_model(c).ready) fail(HB_ERR_STATE, "no cost model");
    if (!x || !y) fail(HB_ERR_INVALID_ARG, "NULL buffer");
    DevBuf hx, hy;
    const float* dx = rows_on_device(c, x, n * kIn, on_device, hx);
    float* dy = y;
    if (!y_on_device) {
        hy.alloc(c, sizeof(float) * kOut * std::max<uint64_t>(n, 1));
        dy = hy.as<float>();
    }
    HB_HIP(launch_mlp_forward(selected_model(c).params.as<float>(), dx, n, dy, c->stream));
    if (!y_on_device) {
        HB_HIP(hipMemcpyAsync(y, dy, sizeof(float) * kOut * n, hipMemcpyDeviceToHost, c->stream));
        c->sync();
    }
}

void costmodel_trace(Ctx* c, const float* x, const float* t, uint32_t n, float* out, uint64_t out_len) {
    if (!selected_model(c).ready) fail(HB_ERR_STATE, "no cost model");
    const uint64_t need = (uint64_t)n * (kHid * 6 + kOut * 2) + kParams;
    if (!x || !t || !out || n == 0 || out_len < need) fail(HB_ERR_INVALID_ARG, "trace buffer too small");
    DevBuf hx, ht;
    const float* dx = rows_on_device(c, x, (size_t)n * kIn, 0, hx);
    const float* dt = rows_on_device(c, t, (size_t)n * kOut, 0, ht);
    Acts a;
    a.ensure(c, (int)n);
    forward(c, selected_model(c).params.as<float>(), dx, (int)n, a);
    backward(c, selected_model(c).params.as<float>(), dx, dt, (int)n, a);
    float* o = out;
    const DevBuf* parts[] = {&a.z1, &a.h1, &a.z2, &a.h2, &a.y, &a.dy, &a.dz2, &a.dz1};
    const size_t sizes[] = {(size_t)n * kHid, (size_t)n * kHid, (size_t)n * kHid, (size_t)n * kHid,
                            (size_t)n * kOut, (size_t)n * kOut, (size_t)n * kHid, (size_t)n * kHid};
    for (int k = 0; k < 8; ++k) {
        HB_HIP(hipMemcpyAsync(o, parts[k]->get(), sizeof(float) * sizes[k], hipMemcpyDeviceToHost, c->stream));
        o += sizes[k];
    }
    HB_HIP(hipMemcpyAsync(o, a.grad.get(), sizeof(float) * kParams, hipMemcpyDeviceToHost, c->stream));
    c->sync();
}

// Model file (little-endian): the 8 bytes "HBCMODEL", u32 version (1),
// u32 inputs, hidden width, outputs and parameter count (16, 64, 2, 5378),
// u32 model kind (0 block, 1 per pair), the fp32 parameters in hb.h's order,
// and the FNV-1a 64 hash of the parameter bytes.
namespace {
constexpr char kMagic[8] = {'H', 'B', 'C', 'M', 'O', 'D', 'E', 'L'};
constexpr uint32_t kFileVersion = 1;

uint64_t fnv1a64(const uint8_t* p, size_t n) {
    uint64_t h = 0xCBF29CE484222325ull;
    for (size_t x = 0; x < n; ++x) {
        h ^= p[x];
        h *= 0x100000001B3ull;
    }
    return h;
}

struct FileCloser {
    FILE* f;
    ~FileCloser() {
        if (f) std::fclose(f);
    }
};
}  // namespace

void costmodel_save(Ctx* c, const char* path) {
    if (!path || !*path) fail(HB_ERR_INVALID_ARG, "NULL or empty path");
    std::vector<float> w(kParams);
    costmodel_get(c, w.data(), kParams);
    const uint32_t head[6] = {kFileVersion, (uint32_t)kIn, (uint32_t)kHid, (uint32_t)kOut, (uint32_t)kParams,
                              (uint32_t)c->model_sel};
    const uint64_t sum = fnv1a64((const uint8_t*)w.data(), sizeof(float) * kParams);
    // write a temporary file beside the target, then rename it over the target
    const std::string tmp = std::string(path) + ".tmp";
    {
        FileCloser fc{std::fopen(tmp.c_str(), "wb")};
        if (!fc.f) fail(HB_ERR_INVALID_ARG, "cannot open " + tmp + " for writing");
        const bool ok = std::fwrite(kMagic, 1, sizeof(kMagic), fc.f) == sizeof(kMagic) &&
                        std::fwrite(head, sizeof(uint32_t), 6, fc.f) == 6 &&
                        std::fwrite(w.data(), sizeof(float), kParams, fc.f) == (size_t)kParams &&
                        std::fwrite(&sum, sizeof(sum), 1, fc.f) == 1;
        const bool closed = std::fclose(fc.f) == 0;
        fc.f = nullptr;
        if (!ok || !closed) {
            std::remove(tmp.c_str());
            fail(HB_ERR_INVALID_ARG, "write to " + tmp + " failed");
        }
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        fail(HB_ERR_INVALID_ARG, std::string("cannot rename the model file to ") + path);
    }
}

void costmodel_load(Ctx* c, const char* path) {
    if (!path || !*path) fail(HB_ERR_INVALID_ARG, "NULL or empty path");
    FileCloser fc{std::fopen(path, "rb")};
    if (!fc.f) fail(HB_ERR_INVALID_ARG, std::string("cannot open ") + path);
    char magic[8];
    uint32_t head[6];
    std::vector<float> w(kParams);
    uint64_t sum = 0;
    if (std::fread(magic, 1, 8, fc.f) != 8 || std::memcmp(magic, kMagic, 8) != 0)
        fail(HB_ERR_INVALID_ARG, std::string(path) + " is not a cost-model file");
    if (std::fread(head, sizeof(uint32_t), 6, fc.f) != 6 || head[0] != kFileVersion)
        fail(HB_ERR_INVALID_ARG, std::string(path) + ": unknown cost-model file version");
    if (head[1] != (uint32_t)kIn || head[2] != (uint32_t)kHid || head[3] != (uint32_t)kOut ||
        head[4] != (uint32_t)kParams || head[5] > 1u)
        fail(HB_ERR_INVALID_ARG, std::string(path) + ": the model's shape is not 16 -> 64 -> 64 -> 2");
    if (head[5] != (uint32_t)c->model_sel)
        fail(HB_ERR_INVALID_ARG, std::string(path) + (head[5] ? ": holds a per-pair model, the block model is selected"
                                                              : ": holds a block model, the per-pair model is selected"));
    if (std::fread(w.data(), sizeof(float), kParams, fc.f) != (size_t)kParams ||
        std::fread(&sum, sizeof(sum), 1, fc.f) != 1)
        fail(HB_ERR_INVALID_ARG, std::string(path) + ": truncated cost-model file");
    char extra;
    if (std::fread(&extra, 1, 1, fc.f) != 0) fail(HB_ERR_INVALID_ARG, std::string(path) + ": trailing bytes");
    if (fnv1a64((const uint8_t*)w.data(), sizeof(float) * kParams) != sum)
        fail(HB_ERR_INVALID_ARG, std::string(path) + ": parameter checksum mismatch");
    costmodel_set(c, w.data(), kParams);
}

void costmodel_adam(Ctx* c, const float* grad_host, float lr) {
    if (!selected_model(c).ready) fail(HB_ERR_STATE, "no cost model");
    DevBuf g;
    const float* dg = rows_on_device(c, grad_host, kParams, 0, g);
    adam(c, dg, lr);
    c->sync();
}

}  // namespace hb

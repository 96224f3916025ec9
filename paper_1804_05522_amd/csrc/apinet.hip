// C ABI of the learned warm start's network (see convnet.hip).
#include "internal.hpp"

struct fde_net_s {
  bool bf16 = true;            // activations in BF16 (matrix cores) or FP32
  int64_t cap = 0;             // pixel capacity of the activation buffers
  float* par = nullptr;        // FP32 master weights (hfde::kNetParams)
  float* grad = nullptr;
  float* am = nullptr;         // Adam moments
  float* av = nullptr;
  void* a1 = nullptr;          // activations, cap x 32
  void* a2 = nullptr;
  void* a3 = nullptr;
  float* g3 = nullptr;         // FP32 gradients wrt pre-activations, cap x 32
  float* g2 = nullptr;
  float* g1 = nullptr;
  float* gpred = nullptr;      // cap
  double* lpart = nullptr;     // loss partials
  float* wpart = nullptr;      // weight-gradient partials
  int adam_t = 0;
  std::vector<void*> allocs;
};

namespace {

template <typename T>
hodlr_status nalloc(fde_net n, T** p, size_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return HODLR_ENOMEM;
  n->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return HODLR_OK;
}

template <typename TA>
void net_forward(fde_net n, NetImg g, const float* u, float* pred, hipStream_t s) {
  const int64_t P = g.pixels();
  const unsigned blocks = unsigned((P + 255) / 256);
  TA* a1 = static_cast<TA*>(n->a1);
  TA* a2 = static_cast<TA*>(n->a2);
  TA* a3 = static_cast<TA*>(n->a3);
  HFDE_LAUNCH(k_net_conv1<TA>, dim3(blocks), dim3(256), 0, s, g, u, n->par, a1);
  if constexpr (std::is_same<TA, bf16>::value) {
    const unsigned mb = unsigned((P + 127) / 128);
    HFDE_LAUNCH(k_net_conv32_mfma, dim3(mb), dim3(256), 0, s, g, a1, n->par, kNW2, kNB2, a2);
    HFDE_LAUNCH(k_net_conv32_mfma, dim3(mb), dim3(256), 0, s, g, a2, n->par, kNW3, kNB3, a3);
  } else {
    HFDE_LAUNCH((k_net_conv32<float, float, float, false>), dim3(blocks), dim3(256), 0, s, g, a1, n->par, kNW2, kNB2,
                (const float*)nullptr, a2);
    HFDE_LAUNCH((k_net_conv32<float, float, float, false>), dim3(blocks), dim3(256), 0, s, g, a2, n->par, kNW3, kNB3,
                (const float*)nullptr, a3);
  }
  HFDE_LAUNCH(k_net_conv4<TA>, dim3(blocks), dim3(256), 0, s, g, a3, u, n->par, pred);
}

template <typename TA>
void net_backward(fde_net n, NetImg g, const float* u, hipStream_t s) {
  const int64_t P = g.pixels();
  const unsigned blocks = unsigned((P + 255) / 256);
  const int chunks = int((P + kNetChunk - 1) / kNetChunk);
  const TA* a1 = static_cast<const TA*>(n->a1);
  const TA* a2 = static_cast<const TA*>(n->a2);
  const TA* a3 = static_cast<const TA*>(n->a3);
  constexpr int kS32 = kNetC * kNetC * 9 + kNetC, kS4 = kNetC * 9 + 1, kS1 = kNetC * 9 + kNetC;
  // layer 4
  HFDE_LAUNCH(k_net_bwd4<TA>, dim3(blocks), dim3(256), 0, s, g, n->gpred, a3, n->par, n->g3);
  HFDE_LAUNCH((k_net_wgrad_edge<TA, false>), dim3(chunks), dim3(288), 0, s, g, n->gpred, a3, u, n->wpart);
  HFDE_LAUNCH(k_net_reduce, dim3((kS4 + 255) / 256), dim3(256), 0, s, n->wpart, chunks, kS4, n->grad, kNW4);
  // layer 3
  HFDE_LAUNCH(k_net_wgrad32<TA>, dim3(chunks), dim3(256), 0, s, g, n->g3, a2, n->wpart);
  HFDE_LAUNCH(k_net_reduce, dim3((kS32 + 255) / 256), dim3(256), 0, s, n->wpart, chunks, kS32, n->grad, kNW3);
  HFDE_LAUNCH((k_net_conv32<float, float, TA, true>), dim3(blocks), dim3(256), 0, s, g, n->g3, n->par, kNW3, 0, a2,
              n->g2);
  // layer 2
  HFDE_LAUNCH(k_net_wgrad32<TA>, dim3(chunks), dim3(256), 0, s, g, n->g2, a1, n->wpart);
  HFDE_LAUNCH(k_net_reduce, dim3((kS32 + 255) / 256), dim3(256), 0, s, n->wpart, chunks, kS32, n->grad, kNW2);
  HFDE_LAUNCH((k_net_conv32<float, float, TA, true>), dim3(blocks), dim3(256), 0, s, g, n->g2, n->par, kNW2, 0, a1,
              n->g1);
  // layer 1
  HFDE_LAUNCH((k_net_wgrad_edge<TA, true>), dim3(chunks), dim3(288), 0, s, g, n->g1, a1, u, n->wpart);
  HFDE_LAUNCH(k_net_reduce, dim3((kS1 + 255) / 256), dim3(256), 0, s, n->wpart, chunks, kS1, n->grad, kNW1);
}

hodlr_status net_check_image(hodlr_ctx ctx, fde_net n, int nimg, int h, int w, int first_arg) {
  if (nimg < 1) return set_arg(ctx, first_arg);
  if (h < 1) return set_arg(ctx, first_arg + 1);
  if (w < 1) return set_arg(ctx, first_arg + 2);
  if (int64_t(nimg) * h * w > n->cap) return set_arg(ctx, first_arg);
  return HODLR_OK;
}

}  // namespace

extern "C" {

int fde_net_param_count(void) { return kNetParams; }

hodlr_status fde_net_create(hodlr_ctx ctx, int act_bf16, int64_t max_pixels, fde_net* out) {
  if (!ctx) return HODLR_EINVAL;
  if (max_pixels < 1) return set_arg(ctx, 3);
  if (!out) return set_arg(ctx, 4);
  fde_net n = new (std::nothrow) fde_net_s;
  if (!n) return HODLR_ENOMEM;
  n->bf16 = act_bf16 != 0;
  n->cap = max_pixels;
  const size_t asz = size_t(max_pixels) * kNetC * (n->bf16 ? sizeof(bf16) : sizeof(float));
  const int64_t chunks = (max_pixels + kNetChunk - 1) / kNetChunk;
  char *a1 = nullptr, *a2 = nullptr, *a3 = nullptr;
  bool ok = nalloc(n, &n->par, kNetParams) == HODLR_OK && nalloc(n, &n->grad, kNetParams) == HODLR_OK &&
            nalloc(n, &n->am, kNetParams) == HODLR_OK && nalloc(n, &n->av, kNetParams) == HODLR_OK &&
            nalloc(n, &a1, asz) == HODLR_OK && nalloc(n, &a2, asz) == HODLR_OK && nalloc(n, &a3, asz) == HODLR_OK &&
            nalloc(n, &n->g3, size_t(max_pixels) * kNetC) == HODLR_OK &&
            nalloc(n, &n->g2, size_t(max_pixels) * kNetC) == HODLR_OK &&
            nalloc(n, &n->g1, size_t(max_pixels) * kNetC) == HODLR_OK &&
            nalloc(n, &n->gpred, size_t(max_pixels)) == HODLR_OK &&
            nalloc(n, &n->lpart, size_t((max_pixels + 255) / 256)) == HODLR_OK &&
            nalloc(n, &n->wpart, size_t(chunks) * (kNetC * kNetC * 9 + kNetC)) == HODLR_OK;
  if (!ok) {
    fde_net_destroy(n);
    return HODLR_ENOMEM;
  }
  n->a1 = a1;
  n->a2 = a2;
  n->a3 = a3;
  hipStream_t s = ctx->stream;
  if (hipMemsetAsync(n->par, 0, kNetParams * sizeof(float), s) != hipSuccess ||
      hipMemsetAsync(n->am, 0, kNetParams * sizeof(float), s) != hipSuccess ||
      hipMemsetAsync(n->av, 0, kNetParams * sizeof(float), s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    fde_net_destroy(n);
    return HODLR_EHIP;
  }
  *out = n;
  return HODLR_OK;
}

void fde_net_destroy(fde_net n) {
  if (!n) return;
  for (void* p : n->allocs) (void)hipFree(p);
  delete n;
}

hodlr_status fde_net_set_params(hodlr_ctx ctx, fde_net n, const float* host, int count) {
  if (!ctx) return HODLR_EINVAL;
  if (!n) return set_arg(ctx, 2);
  if (!host) return set_arg(ctx, 3);
  if (count != kNetParams) return set_arg(ctx, 4);
  HIP_TRY(hipMemcpyAsync(n->par, host, kNetParams * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipMemsetAsync(n->am, 0, kNetParams * sizeof(float), ctx->stream));
  HIP_TRY(hipMemsetAsync(n->av, 0, kNetParams * sizeof(float), ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  n->adam_t = 0;
  return HODLR_OK;
}

hodlr_status fde_net_get_params(hodlr_ctx ctx, fde_net n, float* host, int count) {
  if (!ctx) return HODLR_EINVAL;
  if (!n) return set_arg(ctx, 2);
  if (!host) return set_arg(ctx, 3);
  if (count != kNetParams) return set_arg(ctx, 4);
  HIP_TRY(hipMemcpyAsync(host, n->par, kNetParams * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return HODLR_OK;
}

hodlr_status fde_net_get_grads(hodlr_ctx ctx, fde_net n, float* host, int count) {
  if (!ctx) return HODLR_EINVAL;
  if (!n) return set_arg(ctx, 2);
  if (!host) return set_arg(ctx, 3);
  if (count != kNetParams) return set_arg(ctx, 4);
  HIP_TRY(hipMemcpyAsync(host, n->grad, kNetParams * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return HODLR_OK;
}

hodlr_status fde_net_forward(hodlr_ctx ctx, fde_net n, const float* u, int nimg, int h, int w, float* pred) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!n) return set_arg(ctx, 2);
  if (!u) return set_arg(ctx, 3);
  TRY(net_check_image(ctx, n, nimg, h, w, 4));
  if (!pred) return set_arg(ctx, 7);
  const NetImg g{nimg, h, w};
  if (n->bf16) net_forward<bf16>(n, g, u, pred, ctx->stream);
  else net_forward<float>(n, g, u, pred, ctx->stream);
  HIP_TRY(hipGetLastError());
  return HODLR_OK;
}

hodlr_status fde_net_train_step(hodlr_ctx ctx, fde_net n, const float* u, const float* target, int nimg, int h, int w,
                                int margin, float lr, int update, double* loss) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!n) return set_arg(ctx, 2);
  if (!u) return set_arg(ctx, 3);
  if (!target) return set_arg(ctx, 4);
  TRY(net_check_image(ctx, n, nimg, h, w, 5));
  if (margin < 0 || 2 * margin >= h || 2 * margin >= w) return set_arg(ctx, 8);
  if (!(lr >= 0.0f)) return set_arg(ctx, 9);
  hipStream_t s = ctx->stream;
  const NetImg g{nimg, h, w};
  const int64_t P = g.pixels();
  const unsigned blocks = unsigned((P + 255) / 256);
  float* pred = n->gpred;                 // the prediction is overwritten by dL/dpred below
  if (n->bf16) net_forward<bf16>(n, g, u, pred, s);
  else net_forward<float>(n, g, u, pred, s);
  const double count = double(nimg) * (h - 2 * margin) * (w - 2 * margin);
  HFDE_LAUNCH(k_net_loss, dim3(blocks), dim3(256), 0, s, g, pred, target, margin, 1.0 / count, n->gpred, n->lpart);
  if (n->bf16) net_backward<bf16>(n, g, u, s);
  else net_backward<float>(n, g, u, s);
  if (update) {
    n->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, float(n->adam_t)), c2 = 1.0f - std::pow(b2, float(n->adam_t));
    HFDE_LAUNCH(k_net_adam, dim3((kNetParams + 255) / 256), dim3(256), 0, s, n->par, n->grad, n->am, n->av, kNetParams,
                lr, b1, b2, 1e-8f, c1, c2);
  }
  if (loss) {
    std::vector<double> lp(blocks);
    HIP_TRY(hipMemcpyAsync(lp.data(), n->lpart, blocks * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double sum = 0.0;
    for (double v : lp) sum += v;
    *loss = sum;
  }
  HIP_TRY(hipGetLastError());
  return HODLR_OK;
}

}  // extern "C"

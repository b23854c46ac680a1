// rst_cnn.hip -- driver of the learned correction network: weight packing,
// forward pass with kept activations, backward pass, loss and Adam.
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "rst_cnn.hpp"
#include "rst_cnn_api.hpp"

namespace rst {
namespace cnn {

namespace {

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

hipError_t ensure(Buf& b, size_t bytes) {
  if (bytes <= b.cap && b.p) return hipSuccess;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) return e;
    b.p = nullptr;
    b.cap = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes < 256 ? 256 : bytes);
  if (e == hipSuccess) b.cap = bytes;
  return e;
}

void release(Buf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

Lvl coarse(const Lvl& f) {
  Lvl c;
  c.nz = (f.nz + 1) / 2;
  c.nb = (f.nb + 1) / 2;
  c.na = (f.na + 1) / 2;
  c.n = (long long)c.nz * c.nb * c.na;
  return c;
}

size_t packed_size(int l) { return (size_t)NTAP * kLayerCin[l] * 16; }
size_t packed_off(int l) {
  size_t o = 0;
  for (int k = 0; k < l; ++k) o += packed_size(k);
  return o;
}
size_t natural_size(int l) { return (size_t)kLayerCout[l] * kLayerCin[l] * NTAP; }
size_t natural_off(int l) {
  size_t o = 0;
  for (int k = 0; k < l; ++k) o += natural_size(k);
  return o;
}
int flip_rows(int l) { return kLayerCout[l] == 2 ? 4 : 16; }  // input channels of the adjoint conv
size_t flip_size(int l) { return (size_t)NTAP * flip_rows(l) * 16; }
size_t flip_off(int l) {
  size_t o = 0;
  for (int k = 0; k < l; ++k) o += flip_size(k);
  return o;
}

}  // namespace

size_t natural_count() { return natural_off(NLAYER); }

class Engine {
 public:
  hipStream_t s = nullptr;
  bool has_w = false;
  int t_adam = 0;
  Buf w, wt, gw, am, av, part, lossp;
  // kept activations (ncol columns): level 0 h0a h0 g0; level 1 p1 h1a h1 g1; level 2 p2 h2a h2
  Buf h0a, h0, g0, p1, h1a, h1, g1, p2, h2a, h2;
  // gradient scratch per level
  Buf gA0, gB0, gA1, gB1, gA2, gB2;
  Buf outb, g4;  // network output and widened output gradient of the training step
  const float* x_kept = nullptr;
  int ncol = 0;
  Lvl L0{}, L1{}, L2{};

  float* W(int l) const { return (float*)w.p + packed_off(l); }
  float* Wt(int l) const { return (float*)wt.p + flip_off(l); }
  float* GW(int l) const { return (float*)gw.p + packed_off(l); }

  hipError_t alloc_params() {
    const size_t np = packed_off(NLAYER) * 4;
    hipError_t e;
    if ((e = ensure(w, np)) != hipSuccess) return e;
    if ((e = ensure(gw, np)) != hipSuccess) return e;
    if ((e = ensure(am, np)) != hipSuccess) return e;
    if ((e = ensure(av, np)) != hipSuccess) return e;
    if ((e = ensure(wt, flip_off(NLAYER) * 4)) != hipSuccess) return e;
    return hipSuccess;
  }

  hipError_t alloc_acts(int nc, const Lvl& l0) {
    ncol = nc;
    L0 = l0;
    L1 = coarse(L0);
    L2 = coarse(L1);
    const size_t b0 = (size_t)nc * L0.n * 16 * 4, b1 = (size_t)nc * L1.n * 16 * 4, b2 = (size_t)nc * L2.n * 16 * 4;
    Buf* l0b[] = {&h0a, &h0, &g0};
    Buf* l1b[] = {&p1, &h1a, &h1, &g1};
    Buf* l2b[] = {&p2, &h2a, &h2};
    hipError_t e;
    for (Buf* b : l0b)
      if ((e = ensure(*b, b0)) != hipSuccess) return e;
    for (Buf* b : l1b)
      if ((e = ensure(*b, b1)) != hipSuccess) return e;
    for (Buf* b : l2b)
      if ((e = ensure(*b, b2)) != hipSuccess) return e;
    return hipSuccess;
  }

  template <int CIN, int COUT, int MODE, bool RELU, bool ACCUM>
  hipError_t conv(const float* X, const float* Y, const float* Wl, float* out, const Lvl& L, const Lvl& Lc) {
    ConvArgs A;
    A.X = X;
    A.Y = Y;
    A.W = Wl;
    A.out = out;
    A.L = L;
    A.Lc = Lc;
    A.ncol = ncol;
    const unsigned gx = (unsigned)((L.n + 63) / 64);
    hipLaunchKernelGGL((k_conv<CIN, COUT, MODE, RELU, ACCUM>), dim3(gx, (unsigned)ncol), dim3(256), 0, s, A);
    return hipGetLastError();
  }

  template <int CIN, int GC, int MODE>
  hipError_t bwdw(const float* X, const float* Y, const float* G, const float* M, const Lvl& L, const Lvl& Lc,
                  int layer) {
    BwArgs A;
    A.X = X;
    A.Y = Y;
    A.G = G;
    A.M = M;
    A.L = L;
    A.Lc = Lc;
    A.ncol = ncol;
    A.total = (long long)ncol * L.n;
    long long chunk = (A.total + 1023) / 1024;
    chunk = ((chunk + 3) / 4) * 4;
    if (chunk < 64) chunk = 64;
    A.chunk = chunk;
    const long long nw = (A.total + chunk - 1) / chunk;
    const unsigned blocks = (unsigned)((nw + 3) / 4);
    const long long nw_alloc = (long long)blocks * 4;
    hipError_t e = ensure(part, (size_t)nw_alloc * NTAP * 256 * 4);
    if (e != hipSuccess) return e;
    A.part = (float*)part.p;
    hipLaunchKernelGGL((k_conv_bwdw<CIN, GC, MODE>), dim3(blocks), dim3(256), 0, s, A);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bwdw_reduce, dim3((NTAP * 256 + 255) / 256), dim3(256), 0, s, (const float*)part.p,
                       nw_alloc, kLayerCin[layer], GW(layer));
    return hipGetLastError();
  }

  hipError_t up_adj(const float* gf, float* gc, const Lvl& f, const Lvl& c, int accum) {
    const long long tot = (long long)ncol * c.n * 16;
    hipLaunchKernelGGL(k_up_adj, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, gf, gc, f, c, ncol, accum);
    return hipGetLastError();
  }

  hipError_t pool_adj_acc(const float* gc, float* gf, const Lvl& f, const Lvl& c) {
    const long long tot = (long long)ncol * f.n * 16;
    hipLaunchKernelGGL(k_pool_adj_acc, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, gc, gf, f, c, ncol);
    return hipGetLastError();
  }

  hipError_t pool(const float* x, float* y, const Lvl& f, const Lvl& c) {
    const long long tot = (long long)ncol * c.n * 16;
    hipLaunchKernelGGL(k_pool, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x, y, f, c, ncol);
    return hipGetLastError();
  }
};

#define CNN_CHK(x)                   \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

Engine* engine_create(hipStream_t s) {
  Engine* e = new Engine();
  e->s = s;
  return e;
}

void engine_destroy(Engine* e) {
  if (!e) return;
  Buf* all[] = {&e->w, &e->wt, &e->gw, &e->am, &e->av, &e->part, &e->lossp, &e->h0a, &e->h0, &e->g0,
                &e->p1, &e->h1a, &e->h1, &e->g1, &e->p2, &e->h2a, &e->h2, &e->gA0, &e->gB0, &e->gA1,
                &e->gB1, &e->gA2, &e->gB2, &e->outb, &e->g4};
  for (Buf* b : all) release(*b);
  delete e;
}

bool engine_has_weights(const Engine* e) { return e && e->has_w; }

void engine_reset_adam(Engine* e) { e->t_adam = 0; }

hipError_t engine_set_weights(Engine* e, const float* nat) {
  CNN_CHK(e->alloc_params());
  std::vector<float> pk(packed_off(NLAYER), 0.f);
  for (int l = 0; l < NLAYER; ++l) {
    const int ci = kLayerCin[l], co = kLayerCout[l];
    const float* src = nat + natural_off(l);
    float* dst = pk.data() + packed_off(l);
    for (int o = 0; o < co; ++o)
      for (int i = 0; i < ci; ++i)
        for (int t = 0; t < NTAP; ++t) dst[(t * ci + i) * 16 + o] = src[((size_t)o * ci + i) * NTAP + t];
  }
  CNN_CHK(hipMemcpyAsync(e->w.p, pk.data(), pk.size() * 4, hipMemcpyHostToDevice, e->s));
  std::vector<float> z(pk.size(), 0.f);
  CNN_CHK(hipMemcpyAsync(e->am.p, z.data(), z.size() * 4, hipMemcpyHostToDevice, e->s));
  CNN_CHK(hipMemcpyAsync(e->av.p, z.data(), z.size() * 4, hipMemcpyHostToDevice, e->s));
  CNN_CHK(hipMemcpyAsync(e->gw.p, z.data(), z.size() * 4, hipMemcpyHostToDevice, e->s));
  CNN_CHK(hipStreamSynchronize(e->s));
  e->t_adam = 0;
  e->has_w = true;
  return hipSuccess;
}

static hipError_t unpack(Engine* e, const Buf& b, float* nat) {
  std::vector<float> pk(packed_off(NLAYER));
  CNN_CHK(hipMemcpyAsync(pk.data(), b.p, pk.size() * 4, hipMemcpyDeviceToHost, e->s));
  CNN_CHK(hipStreamSynchronize(e->s));
  for (int l = 0; l < NLAYER; ++l) {
    const int ci = kLayerCin[l], co = kLayerCout[l];
    const float* src = pk.data() + packed_off(l);
    float* dst = nat + natural_off(l);
    for (int o = 0; o < co; ++o)
      for (int i = 0; i < ci; ++i)
        for (int t = 0; t < NTAP; ++t) dst[((size_t)o * ci + i) * NTAP + t] = src[(t * ci + i) * 16 + o];
  }
  return hipSuccess;
}

hipError_t engine_get_weights(Engine* e, float* nat) {
  if (!e->has_w) return hipErrorInvalidValue;
  return unpack(e, e->w, nat);
}

hipError_t engine_get_grad(Engine* e, float* nat) {
  if (!e->has_w) return hipErrorInvalidValue;
  return unpack(e, e->gw, nat);
}

hipError_t engine_seed(Engine* e, uint64_t seed) {
  std::mt19937_64 gen(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<float> nat(natural_count());
  for (int l = 0; l < NLAYER; ++l) {
    const double sd = std::sqrt(2.0 / (NTAP * kLayerCin[l])) * (l == NLAYER - 1 ? 0.1 : 1.0);
    float* d = nat.data() + natural_off(l);
    for (size_t j = 0; j < natural_size(l); ++j) d[j] = (float)(sd * nd(gen));
  }
  return engine_set_weights(e, nat.data());
}

hipError_t engine_forward(Engine* e, const float* x, float* out, int ncol, int nz, int nb, int na, bool keep) {
  (void)keep;  // the activations are always kept: the inference buffers are the training ones
  if (!e->has_w) return hipErrorInvalidValue;
  Lvl L0{nz, nb, na, (long long)nz * nb * na};
  CNN_CHK(e->alloc_acts(ncol, L0));
  const Lvl &l0 = e->L0, &l1 = e->L1, &l2 = e->L2;
  float *h0a = (float*)e->h0a.p, *h0 = (float*)e->h0.p, *g0 = (float*)e->g0.p;
  float *p1 = (float*)e->p1.p, *h1a = (float*)e->h1a.p, *h1 = (float*)e->h1.p, *g1 = (float*)e->g1.p;
  float *p2 = (float*)e->p2.p, *h2a = (float*)e->h2a.p, *h2 = (float*)e->h2.p;
  CNN_CHK((e->conv<4, 16, CIN_PLAIN, true, false>(x, nullptr, e->W(0), h0a, l0, l0)));
  CNN_CHK((e->conv<16, 16, CIN_PLAIN, true, false>(h0a, nullptr, e->W(1), h0, l0, l0)));
  CNN_CHK(e->pool(h0, p1, l0, l1));
  CNN_CHK((e->conv<16, 16, CIN_PLAIN, true, false>(p1, nullptr, e->W(2), h1a, l1, l1)));
  CNN_CHK((e->conv<16, 16, CIN_PLAIN, true, false>(h1a, nullptr, e->W(3), h1, l1, l1)));
  CNN_CHK(e->pool(h1, p2, l1, l2));
  CNN_CHK((e->conv<16, 16, CIN_PLAIN, true, false>(p2, nullptr, e->W(4), h2a, l2, l2)));
  CNN_CHK((e->conv<16, 16, CIN_PLAIN, true, false>(h2a, nullptr, e->W(5), h2, l2, l2)));
  CNN_CHK((e->conv<16, 16, CIN_UPADD, true, false>(h1, h2, e->W(6), g1, l1, l2)));
  CNN_CHK((e->conv<16, 16, CIN_UPADD, true, false>(h0, g1, e->W(7), g0, l0, l1)));
  CNN_CHK((e->conv<16, 2, CIN_PLAIN, false, false>(g0, nullptr, e->W(8), out, l0, l0)));
  e->x_kept = x;
  return hipSuccess;
}

hipError_t engine_backward(Engine* e, const float* gout4) {
  if (!e->has_w || !e->x_kept) return hipErrorInvalidValue;
  const int nc = e->ncol;
  const Lvl &l0 = e->L0, &l1 = e->L1, &l2 = e->L2;
  const size_t b0 = (size_t)nc * l0.n * 16 * 4, b1 = (size_t)nc * l1.n * 16 * 4, b2 = (size_t)nc * l2.n * 16 * 4;
  CNN_CHK(ensure(e->gA0, b0));
  CNN_CHK(ensure(e->gB0, b0));
  CNN_CHK(ensure(e->gA1, b1));
  CNN_CHK(ensure(e->gB1, b1));
  CNN_CHK(ensure(e->gA2, b2));
  CNN_CHK(ensure(e->gB2, b2));
  // adjoint-convolution weights
  for (int l = 1; l < NLAYER; ++l) {
    const int cnt = (int)flip_size(l);
    hipLaunchKernelGGL(k_flip, dim3((cnt + 255) / 256), dim3(256), 0, e->s, (const float*)e->W(l), kLayerCin[l],
                       kLayerCout[l], flip_rows(l), e->Wt(l));
    CNN_CHK(hipGetLastError());
  }
  const float* x = e->x_kept;
  float *h0a = (float*)e->h0a.p, *h0 = (float*)e->h0.p, *g0 = (float*)e->g0.p;
  float *p1 = (float*)e->p1.p, *h1a = (float*)e->h1a.p, *h1 = (float*)e->h1.p, *g1 = (float*)e->g1.p;
  float *p2 = (float*)e->p2.p, *h2a = (float*)e->h2a.p, *h2 = (float*)e->h2.p;
  float *gA0 = (float*)e->gA0.p, *gB0 = (float*)e->gB0.p, *gA1 = (float*)e->gA1.p, *gB1 = (float*)e->gB1.p;
  float *gA2 = (float*)e->gA2.p, *gB2 = (float*)e->gB2.p;
  // W8 (no activation): gW8 from g0 and gout; gA0 = d/dg0
  CNN_CHK((e->bwdw<16, 4, CIN_PLAIN>(g0, nullptr, gout4, nullptr, l0, l0, 8)));
  CNN_CHK((e->conv<4, 16, CIN_PLAIN, false, false>(gout4, nullptr, e->Wt(8), gA0, l0, l0)));
  // W7: input u0 = h0 + up(g1), output g0; gB0 = d/du0 (the h0 skip), gA1 = up-adjoint (d/dg1)
  CNN_CHK((e->bwdw<16, 16, CIN_UPADD>(h0, g1, gA0, g0, l0, l1, 7)));
  CNN_CHK((e->conv<16, 16, CIN_MASK, false, false>(gA0, g0, e->Wt(7), gB0, l0, l0)));
  CNN_CHK(e->up_adj(gB0, gA1, l0, l1, 0));
  // W6: input u1 = h1 + up(h2), output g1; gB1 = d/du1 (the h1 skip), gA2 = d/dh2
  CNN_CHK((e->bwdw<16, 16, CIN_UPADD>(h1, h2, gA1, g1, l1, l2, 6)));
  CNN_CHK((e->conv<16, 16, CIN_MASK, false, false>(gA1, g1, e->Wt(6), gB1, l1, l1)));
  CNN_CHK(e->up_adj(gB1, gA2, l1, l2, 0));
  // W5: h2a -> h2
  CNN_CHK((e->bwdw<16, 16, CIN_PLAIN>(h2a, nullptr, gA2, h2, l2, l2, 5)));
  CNN_CHK((e->conv<16, 16, CIN_MASK, false, false>(gA2, h2, e->Wt(5), gB2, l2, l2)));
  // W4: p2 -> h2a; gA2 = d/dp2, then d/dh1 += pool-adjoint
  CNN_CHK((e->bwdw<16, 16, CIN_PLAIN>(p2, nullptr, gB2, h2a, l2, l2, 4)));
  CNN_CHK((e->conv<16, 16, CIN_MASK, false, false>(gB2, h2a, e->Wt(4), gA2, l2, l2)));
  CNN_CHK(e->pool_adj_acc(gA2, gB1, l1, l2));
  // W3: h1a -> h1
  CNN_CHK((e->bwdw<16, 16, CIN_PLAIN>(h1a, nullptr, gB1, h1, l1, l1, 3)));
  CNN_CHK((e->conv<16, 16, CIN_MASK, false, false>(gB1, h1, e->Wt(3), gA1, l1, l1)));
  // W2: p1 -> h1a; gB1 = d/dp1, then d/dh0 += pool-adjoint
  CNN_CHK((e->bwdw<16, 16, CIN_PLAIN>(p1, nullptr, gA1, h1a, l1, l1, 2)));
  CNN_CHK((e->conv<16, 16, CIN_MASK, false, false>(gA1, h1a, e->Wt(2), gB1, l1, l1)));
  CNN_CHK(e->pool_adj_acc(gB1, gB0, l0, l1));
  // W1: h0a -> h0
  CNN_CHK((e->bwdw<16, 16, CIN_PLAIN>(h0a, nullptr, gB0, h0, l0, l0, 1)));
  CNN_CHK((e->conv<16, 16, CIN_MASK, false, false>(gB0, h0, e->Wt(1), gA0, l0, l0)));
  // W0: x -> h0a
  CNN_CHK((e->bwdw<4, 16, CIN_PLAIN>(x, nullptr, gA0, h0a, l0, l0, 0)));
  return hipSuccess;
}

hipError_t engine_loss(Engine* e, const float* out, const float* tgt, float* gout4, int ncol, long long n,
                       double* loss) {
  const long long npts = (long long)ncol * n;
  const unsigned blocks = (unsigned)((npts + 255) / 256);
  CNN_CHK(ensure(e->lossp, (size_t)blocks * 8));
  hipLaunchKernelGGL(k_loss, dim3(blocks), dim3(256), 0, e->s, out, tgt, gout4, (double*)e->lossp.p, npts,
                     1.0f / (float)ncol);
  CNN_CHK(hipGetLastError());
  std::vector<double> lp(blocks);
  CNN_CHK(hipMemcpyAsync(lp.data(), e->lossp.p, blocks * 8, hipMemcpyDeviceToHost, e->s));
  CNN_CHK(hipStreamSynchronize(e->s));
  double s = 0.0;
  for (double v : lp) s += v;
  *loss = s / ncol;
  return hipSuccess;
}

hipError_t engine_adam(Engine* e, float lr) {
  if (!e->has_w) return hipErrorInvalidValue;
  e->t_adam += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)e->t_adam), c2 = 1.f - std::pow(b2, (float)e->t_adam);
  const int cnt = (int)packed_off(NLAYER);
  hipLaunchKernelGGL(k_adam, dim3((cnt + 255) / 256), dim3(256), 0, e->s, (float*)e->w.p, (const float*)e->gw.p,
                     (float*)e->am.p, (float*)e->av.p, cnt, lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

hipError_t engine_gradient(Engine* e, const float* x, const float* g2, int ncol, int nz, int nb, int na) {
  const long long npts = (long long)ncol * nz * nb * na;
  CNN_CHK(ensure(e->outb, (size_t)npts * 2 * 4));
  CNN_CHK(ensure(e->g4, (size_t)npts * 4 * 4));
  CNN_CHK(engine_forward(e, x, (float*)e->outb.p, ncol, nz, nb, na, true));
  hipLaunchKernelGGL(k_pad24, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, e->s, g2, (float*)e->g4.p, npts);
  CNN_CHK(hipGetLastError());
  return engine_backward(e, (const float*)e->g4.p);
}

hipError_t engine_train_step(Engine* e, const float* x, const float* tgt, int ncol, int nz, int nb, int na,
                             float lr, double* loss) {
  const long long n = (long long)nz * nb * na;
  const long long npts = (long long)ncol * n;
  CNN_CHK(ensure(e->outb, (size_t)npts * 2 * 4));
  CNN_CHK(ensure(e->g4, (size_t)npts * 4 * 4));
  CNN_CHK(engine_forward(e, x, (float*)e->outb.p, ncol, nz, nb, na, true));
  CNN_CHK(engine_loss(e, (const float*)e->outb.p, tgt, (float*)e->g4.p, ncol, n, loss));
  CNN_CHK(engine_backward(e, (const float*)e->g4.p));
  return engine_adam(e, lr);
}

}  // namespace cnn
}  // namespace rst

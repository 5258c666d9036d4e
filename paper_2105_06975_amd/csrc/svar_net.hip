// Host side of the sweep-correction network: the svar_net object (parameters, Adam state,
// kernel-layout weights, training workspace), its C ABI, and the in-place application inside
// a preconditioner program.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mem.h"
#include "net.h"
#include "svar_handle.h"

using namespace svar;

struct svar_net {
  int device = 0;
  svar_net_desc d{};
  NetLayout L;
  std::vector<void*> allocs;      // parameters and weights
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  int64_t t = 0;                  // Adam steps taken
  NetWeights W;
  // training / standalone-forward workspace
  std::vector<void*> ws_allocs;
  int64_t rows_cap = 0, tiles_cap = 0;
  float *X0 = nullptr, *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *gA = nullptr,
        *gB = nullptr, *outv = nullptr, *g4 = nullptr, *part = nullptr, *part2 = nullptr;
  double* lpart = nullptr;
  NetSample* smp = nullptr;
  NetTile* tiles = nullptr;
  std::vector<NetSample> hsmp;
  std::vector<NetTile> htiles;
};

namespace {

int inv(const std::string& m) { return inval_msg(m); }

int net_ensure(svar_net* n, int64_t rows, int64_t ntiles, hipStream_t st) {
  if (rows <= n->rows_cap && ntiles <= n->tiles_cap) return SVAR_OK;
  SVAR_HIP(hipStreamSynchronize(st));
  free_all(n->ws_allocs);
  n->rows_cap = std::max(rows, n->rows_cap);
  n->tiles_cap = std::max(ntiles, n->tiles_cap);
  auto& A = n->ws_allocs;
  const size_t R = (size_t)n->rows_cap, T = (size_t)n->tiles_cap;
  SVAR_TRY(dalloc(A, &n->X0, R * NET_CIN1));
  SVAR_TRY(dalloc(A, &n->a1, R * NET_C));
  SVAR_TRY(dalloc(A, &n->a2, R * NET_C));
  SVAR_TRY(dalloc(A, &n->a3, R * NET_C));
  SVAR_TRY(dalloc(A, &n->gA, R * NET_C));
  SVAR_TRY(dalloc(A, &n->gB, R * NET_C));
  SVAR_TRY(dalloc(A, &n->outv, R));
  SVAR_TRY(dalloc(A, &n->g4, R));
  SVAR_TRY(dalloc(A, &n->lpart, T));
  SVAR_TRY(dalloc(A, &n->smp, T));  // at most one sample per tile
  SVAR_TRY(dalloc(A, &n->tiles, T));
  SVAR_TRY(dalloc(A, &n->part, (size_t)net_grid_cap() * NET_WG_PART));
  SVAR_TRY(dalloc(A, &n->part2, (size_t)(net_grid_cap() / 16 + 1) * NET_WG_PART));
  return SVAR_OK;
}

// samples (pair, block) of a [npair][nb][s] pool, rows in sample order
int net_stage(svar_net* n, int nb, int s, int nsample, const int32_t* pairs_blocks, int npair,
              hipStream_t st, int* ntiles_out) {
  SVAR_HIP(hipStreamSynchronize(st));  // the host tables are reused
  const int tps = (s + NET_TILE - 1) / NET_TILE;
  const int64_t ntiles = (int64_t)nsample * tps;
  if (ntiles > (int64_t)1 << 30) return inv("too many tiles");
  SVAR_TRY(net_ensure(n, (int64_t)nsample * s, ntiles, st));
  n->hsmp.resize(nsample);
  n->htiles.resize(ntiles);
  for (int q = 0; q < nsample; ++q) {
    const int p = pairs_blocks[2 * q], b = pairs_blocks[2 * q + 1];
    if (p < 0 || p >= npair || b < 0 || b >= nb) return inv("sample out of range");
    NetSample S{};
    S.src = (int64_t)p * nb * s;
    S.row0 = (int64_t)q * s;
    S.s = s;
    S.nb = nb;
    S.blk = b;
    S.sys = p;
    n->hsmp[q] = S;
    for (int t = 0; t < tps; ++t) n->htiles[(int64_t)q * tps + t] = NetTile{q, t * NET_TILE};
  }
  SVAR_HIP(hipMemcpyAsync(n->smp, n->hsmp.data(), nsample * sizeof(NetSample),
                          hipMemcpyHostToDevice, st));
  SVAR_HIP(hipMemcpyAsync(n->tiles, n->htiles.data(), ntiles * sizeof(NetTile),
                          hipMemcpyHostToDevice, st));
  *ntiles_out = (int)ntiles;
  return SVAR_OK;
}

int check_shape(int npair, int nb, int s) {
  if (npair < 1 || nb < 1 || s < 1) return inv("need npair, nb, s >= 1");
  if ((int64_t)npair * nb * s > ((int64_t)1 << 40)) return inv("pool too large");
  return SVAR_OK;
}

}  // namespace

namespace svar {

// In-place correction base[...] += sigma * NN(features(base / sigma)) of every system of the
// program's vector (see add_net in the program builder).
int run_net(svar_handle* h, const NetApp& app, double* base, const int* skip, hipStream_t st) {
  svar_net* n = h->net;
  if (!n) return SVAR_OK;
  const int bf = n->d.precision == SVAR_NET_BF16 ? 1 : 0;
  const size_t es = bf ? 2 : 4;
  // bfloat16: the fused kernel needs one float per grid point; float32: the layer-by-layer
  // kernels need the layer-1 features and two hidden activations
  const int64_t need = bf ? app.max_rows * (int64_t)sizeof(float)
                          : app.max_rows * (NET_CIN1 + 2 * NET_C) * (int64_t)es;
  if (need > h->net_ws_bytes) {
    SVAR_HIP(hipStreamSynchronize(st));
    if (h->net_ws) {
      (void)hipFree(h->net_ws);
      auto it = std::find(h->allocs.begin(), h->allocs.end(), h->net_ws);
      if (it != h->allocs.end()) h->allocs.erase(it);
      h->net_ws = nullptr;
      h->net_ws_bytes = 0;
    }
    char* p = nullptr;
    SVAR_TRY(dalloc(h->allocs, &p, (size_t)need));
    h->net_ws = p;
    h->net_ws_bytes = need;
  }
  char* ws = (char*)h->net_ws;
  void* X0 = ws;
  void* A = ws + app.max_rows * NET_CIN1 * es;
  void* B = (char*)A + app.max_rows * NET_C * es;
  net_sumsq(base, app.chunks, app.nchunk, app.part, skip, st);
  net_sigma_impl(app.part, app.chunk0, app.chunks, app.nsys, app.sigma, app.inv_sigma, skip, st);
  const int nrc = (int)app.row0.size();
  if (bf) {
    float* corr = (float*)ws;
    for (int c = 0; c < nrc; ++c) {
      const int f0 = app.ftile0[c], nf = app.ftile0[c + 1] - f0;
      const int t0 = app.tile0[c], nt = app.tile0[c + 1] - t0;
      net_fused(base, app.inv_sigma, app.smp, app.ftiles + f0, nf, app.row0[c], n->d.k,
                n->d.n_bound, n->W, n->theta, n->L, corr, skip, h->net_off, st);
      net_apply(corr, app.smp, app.tiles + t0, nt, app.row0[c], base, app.sigma, h->net_off,
                skip, st);
    }
    return SVAR_OK;
  }
  const void* wl[3];
  for (int l = 0; l < 3; ++l) wl[l] = bf ? (const void*)n->W.wb[l] : (const void*)n->W.wf[l];
  for (int c = 0; c < nrc; ++c) {
    const int t0 = app.tile0[c], nt = app.tile0[c + 1] - t0;
    const NetTile* tl = app.tiles + t0;
    const int64_t rb = app.row0[c];
    const int* off = h->net_off;
    net_feat_d(base, app.inv_sigma, app.smp, tl, nt, rb, n->d.k, n->d.n_bound, bf, X0, skip, off,
               st);
    net_conv(bf, 1, 0, X0, A, wl[0], n->theta + n->L.b[0], nullptr, app.smp, tl, nt, rb, skip,
             off, st);
    net_conv(bf, 0, 0, A, B, wl[1], n->theta + n->L.b[1], nullptr, app.smp, tl, nt, rb, skip,
             off, st);
    net_conv(bf, 0, 0, B, A, wl[2], n->theta + n->L.b[2], nullptr, app.smp, tl, nt, rb, skip,
             off, st);
    net_out(bf, A, n->W.w4, n->theta + n->L.b[3], app.smp, tl, nt, rb, nullptr, base, app.sigma,
            h->net_off, skip, st);
  }
  return SVAR_OK;
}

}  // namespace svar

extern "C" {

int svar_net_create(const svar_net_desc* d, svar_net** out) {
  if (!out) return inv("out is NULL");
  *out = nullptr;
  if (!d) return inv("desc is NULL");
  if (d->k < 1) return inv("need k >= 1");
  if (d->n_bound < 0 || 1 + d->n_bound + d->k > NET_CIN1)
    return inv("need n_bound >= 0 and 1 + n_bound + k <= 32");
  if (d->precision != SVAR_NET_FP32 && d->precision != SVAR_NET_BF16)
    return inv("bad network precision");
  svar_net* n = new svar_net();
  n->d = *d;
  n->L.init(1 + d->n_bound + d->k);
  int rc = SVAR_OK;
  if (hipGetDevice(&n->device) != hipSuccess) rc = inv("no HIP device");
  auto& A = n->allocs;
  const size_t np = (size_t)n->L.n;
  if (rc == SVAR_OK) rc = dalloc(A, &n->theta, np);
  if (rc == SVAR_OK) rc = dalloc(A, &n->m, np);
  if (rc == SVAR_OK) rc = dalloc(A, &n->v, np);
  if (rc == SVAR_OK) rc = dalloc(A, &n->grad, np);
  for (int l = 0; l < 3 && rc == SVAR_OK; ++l) {
    const size_t ne = (size_t)NET_C * NET_W * (l == 0 ? NET_CIN1 : NET_C);
    rc = dalloc(A, &n->W.wf[l], ne);
    if (rc == SVAR_OK) rc = dalloc(A, &n->W.wb[l], ne);
  }
  for (int l = 0; l < 2 && rc == SVAR_OK; ++l)
    rc = dalloc(A, &n->W.wflip[l], (size_t)NET_C * NET_W * NET_C);
  if (rc == SVAR_OK) rc = dalloc(A, &n->W.w4, (size_t)NET_W * NET_C);
  if (rc == SVAR_OK) {
    std::vector<float> z(np, 0.0f);
    rc = svar_net_set_params(n, z.data());
  }
  if (rc != SVAR_OK) {
    svar_net_destroy(n);
    return rc;
  }
  *out = n;
  return SVAR_OK;
}

int svar_net_destroy(svar_net* n) {
  if (!n) return SVAR_OK;
  (void)hipDeviceSynchronize();
  free_all(n->ws_allocs);
  free_all(n->allocs);
  delete n;
  return SVAR_OK;
}

int64_t svar_net_nparams(const svar_net* n) { return n ? n->L.n : -1; }

int svar_net_set_params(svar_net* n, const float* theta) {
  if (!n || !theta) return inv("bad arguments");
  const size_t b = (size_t)n->L.n * sizeof(float);
  SVAR_HIP(hipMemcpy(n->theta, theta, b, hipMemcpyHostToDevice));
  SVAR_HIP(hipMemset(n->m, 0, b));
  SVAR_HIP(hipMemset(n->v, 0, b));
  n->t = 0;
  net_pack(n->theta, n->L, n->W, nullptr);
  SVAR_HIP(hipDeviceSynchronize());
  return SVAR_OK;
}

int svar_net_get_params(const svar_net* n, float* theta) {
  if (!n || !theta) return inv("bad arguments");
  SVAR_HIP(hipDeviceSynchronize());
  SVAR_HIP(hipMemcpy(theta, n->theta, (size_t)n->L.n * sizeof(float), hipMemcpyDeviceToHost));
  return SVAR_OK;
}

int svar_net_make_pairs(int32_t npair, int32_t nb, int32_t s, const double* chat,
                        const double* cexact, float* x, float* y, void* stream) {
  SVAR_TRY(check_shape(npair, nb, s));
  if (!chat || !cexact || !x || !y) return inv("NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  const int64_t len = (int64_t)nb * s;
  const int64_t CH = 1 << 13;
  std::vector<NetChunk> ch;
  std::vector<int32_t> c0(npair + 1);
  for (int p = 0; p < npair; ++p) {
    c0[p] = (int)ch.size();
    for (int64_t e = 0; e < len; e += CH) {
      NetChunk c{};
      c.sys = p;
      c.e0 = (int64_t)p * len + e;
      c.e1 = (int64_t)p * len + std::min(len, e + CH);
      ch.push_back(c);
    }
  }
  c0[npair] = (int)ch.size();
  std::vector<void*> tmp;
  NetChunk* dch = nullptr;
  int32_t* dc0 = nullptr;
  double *part = nullptr, *sg = nullptr, *isg = nullptr;
  int rc = upload(tmp, &dch, ch.data(), ch.size(), st);
  if (rc == SVAR_OK) rc = upload(tmp, &dc0, c0.data(), c0.size(), st);
  if (rc == SVAR_OK) rc = dalloc(tmp, &part, ch.size());
  if (rc == SVAR_OK) rc = dalloc(tmp, &sg, (size_t)npair);
  if (rc == SVAR_OK) rc = dalloc(tmp, &isg, (size_t)npair);
  if (rc == SVAR_OK) {
    net_sumsq(chat, dch, (int)ch.size(), part, nullptr, st);
    net_sigma_impl(part, dc0, dch, npair, sg, isg, nullptr, st);
    net_norm_pairs(chat, cexact, isg, len, npair, x, y, st);
    if (hipStreamSynchronize(st) != hipSuccess) rc = inv("make_pairs kernels failed");
  }
  free_all(tmp);
  return rc;
}

int svar_net_forward(svar_net* n, int32_t precision, int32_t npair, int32_t nb, int32_t s,
                     const float* x, float* out, void* stream) {
  if (!n || !x || !out) return inv("bad arguments");
  SVAR_TRY(check_shape(npair, nb, s));
  if (precision != SVAR_NET_FP32 && precision != SVAR_NET_BF16) return inv("bad precision");
  hipStream_t st = (hipStream_t)stream;
  const int64_t ns = (int64_t)npair * nb;
  if (ns > (1 << 24)) return inv("too many samples");
  std::vector<int32_t> pb(2 * ns);
  for (int64_t q = 0; q < ns; ++q) {
    pb[2 * q] = (int32_t)(q / nb);
    pb[2 * q + 1] = (int32_t)(q % nb);
  }
  int ntiles = 0;
  SVAR_TRY(net_stage(n, nb, s, (int)ns, pb.data(), npair, st, &ntiles));
  const int bf = precision == SVAR_NET_BF16;
  const void* wl[3];
  for (int l = 0; l < 3; ++l) wl[l] = bf ? (const void*)n->W.wb[l] : (const void*)n->W.wf[l];
  // bfloat16 activations reuse the float32 buffers (half of each is used)
  net_feat_f(x, n->smp, n->tiles, ntiles, 0, n->d.k, n->d.n_bound, bf, n->X0, st);
  net_conv(bf, 1, 0, n->X0, n->a1, wl[0], n->theta + n->L.b[0], nullptr, n->smp, n->tiles,
           ntiles, 0, nullptr, nullptr, st);
  net_conv(bf, 0, 0, n->a1, n->a2, wl[1], n->theta + n->L.b[1], nullptr, n->smp, n->tiles,
           ntiles, 0, nullptr, nullptr, st);
  net_conv(bf, 0, 0, n->a2, n->a3, wl[2], n->theta + n->L.b[2], nullptr, n->smp, n->tiles,
           ntiles, 0, nullptr, nullptr, st);
  net_out(bf, n->a3, n->W.w4, n->theta + n->L.b[3], n->smp, n->tiles, ntiles, 0, out, nullptr,
          nullptr, nullptr, nullptr, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return inv(std::string("network kernels failed: ") + hipGetErrorString(e));
  return SVAR_OK;
}

int svar_net_train_step(svar_net* n, int32_t npair, int32_t nb, int32_t s, const float* x,
                        const float* y, int32_t nsample, const int32_t* samples,
                        const svar_adam_opts* adam, double* loss, float* grad, void* stream) {
  if (!n || !x || !y || !samples || nsample < 1) return inv("bad arguments");
  SVAR_TRY(check_shape(npair, nb, s));
  if (adam && !(adam->lr > 0.0 && adam->beta1 >= 0.0 && adam->beta1 < 1.0 &&
                adam->beta2 >= 0.0 && adam->beta2 < 1.0 && adam->eps > 0.0))
    return inv("bad Adam options");
  hipStream_t st = (hipStream_t)stream;
  int ntiles = 0;
  SVAR_TRY(net_stage(n, nb, s, nsample, samples, npair, st, &ntiles));
  const NetSample* S = n->smp;
  const NetTile* T = n->tiles;
  const float* b = n->theta;
  // forward (float32), keeping the activations
  net_feat_f(x, S, T, ntiles, 0, n->d.k, n->d.n_bound, 0, n->X0, st);
  net_conv(0, 1, 0, n->X0, n->a1, n->W.wf[0], b + n->L.b[0], nullptr, S, T, ntiles, 0, nullptr,
           nullptr, st);
  net_conv(0, 0, 0, n->a1, n->a2, n->W.wf[1], b + n->L.b[1], nullptr, S, T, ntiles, 0, nullptr,
           nullptr, st);
  net_conv(0, 0, 0, n->a2, n->a3, n->W.wf[2], b + n->L.b[2], nullptr, S, T, ntiles, 0, nullptr,
           nullptr, st);
  net_out(0, n->a3, n->W.w4, b + n->L.b[3], S, T, ntiles, 0, n->outv, nullptr, nullptr, nullptr,
          nullptr, st);
  // loss and backward
  const double count = (double)nsample * s;
  net_loss(n->outv, y, S, T, ntiles, (float)(2.0 / count), n->g4, n->lpart, st);
  const int G = std::min(ntiles, net_grid_cap());
  net_out_bwd(n->g4, n->W.w4, n->a3, n->gA, S, T, ntiles, st);
  net_wgrad4(n->g4, n->a3, S, T, ntiles, G, n->part, st);
  net_wreduce(n->part, n->part2, G, 3, n->L, n->grad, st);
  net_wgrad(0, n->gA, n->a2, S, T, ntiles, G, n->part, st);
  net_wreduce(n->part, n->part2, G, 2, n->L, n->grad, st);
  net_conv(0, 0, 1, n->gA, n->gB, n->W.wflip[1], nullptr, n->a2, S, T, ntiles, 0, nullptr, nullptr,
           st);
  net_wgrad(0, n->gB, n->a1, S, T, ntiles, G, n->part, st);
  net_wreduce(n->part, n->part2, G, 1, n->L, n->grad, st);
  net_conv(0, 0, 1, n->gB, n->gA, n->W.wflip[0], nullptr, n->a1, S, T, ntiles, 0, nullptr, nullptr,
           st);
  net_wgrad(1, n->gA, n->X0, S, T, ntiles, G, n->part, st);
  net_wreduce(n->part, n->part2, G, 0, n->L, n->grad, st);
  if (grad)
    SVAR_HIP(hipMemcpyAsync(grad, n->grad, (size_t)n->L.n * sizeof(float),
                            hipMemcpyDeviceToHost, st));
  if (adam) {
    n->t += 1;
    const double bc1 = 1.0 - std::pow(adam->beta1, (double)n->t);
    const double bc2 = 1.0 - std::pow(adam->beta2, (double)n->t);
    net_adam(n->theta, n->grad, n->m, n->v, n->L.n, (float)adam->lr, (float)adam->beta1,
             (float)adam->beta2, (float)adam->eps, (float)bc1, (float)bc2, st);
    net_pack(n->theta, n->L, n->W, st);
  }
  if (loss) {
    std::vector<double> lp(ntiles);
    SVAR_HIP(hipMemcpyAsync(lp.data(), n->lpart, ntiles * sizeof(double), hipMemcpyDeviceToHost,
                            st));
    SVAR_HIP(hipStreamSynchronize(st));
    double acc = 0.0;
    for (double v : lp) acc += v;
    *loss = acc / count;
  } else if (grad) {
    SVAR_HIP(hipStreamSynchronize(st));
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return inv(std::string("network kernels failed: ") + hipGetErrorString(e));
  return SVAR_OK;
}

// ------------------------------------------------------------------ training driver
namespace {

// splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number generators"): the
// sample order of epoch e is a Fisher-Yates shuffle driven by the generator seeded with
// seed + e, so any epoch's order can be rebuilt when training resumes
uint64_t splitmix64(uint64_t& st) {
  uint64_t z = (st += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void epoch_order(int64_t nsamp, uint64_t seed, int64_t epoch, std::vector<int64_t>& ord) {
  ord.resize(nsamp);
  for (int64_t i = 0; i < nsamp; ++i) ord[i] = i;
  uint64_t st = seed + (uint64_t)epoch;
  for (int64_t i = nsamp - 1; i > 0; --i) {
    const int64_t j = (int64_t)(splitmix64(st) % (uint64_t)(i + 1));
    std::swap(ord[i], ord[j]);
  }
}

// checkpoint file: this header, then theta, m, v (nparams float32 each), little endian
struct CkptHeader {
  char magic[8];        // "SVARNET1"
  int32_t k, n_bound, precision, cin;
  int64_t nparams;
  int64_t adam_t;       // Adam steps taken
  int64_t epoch, pos;   // data cursor: next batch starts at sample pos of epoch's order
  uint64_t seed;
  int32_t npair, nb, s, batch;
};

int write_ckpt(const svar_net* n, const char* path, int64_t epoch, int64_t pos, uint64_t seed,
               int npair, int nb, int s, int batch) {
  CkptHeader H{};
  std::memcpy(H.magic, "SVARNET1", 8);
  H.k = n->d.k;
  H.n_bound = n->d.n_bound;
  H.precision = n->d.precision;
  H.cin = n->L.cin;
  H.nparams = n->L.n;
  H.adam_t = n->t;
  H.epoch = epoch;
  H.pos = pos;
  H.seed = seed;
  H.npair = npair;
  H.nb = nb;
  H.s = s;
  H.batch = batch;
  std::vector<float> buf((size_t)3 * n->L.n);
  const size_t b = (size_t)n->L.n * sizeof(float);
  SVAR_HIP(hipDeviceSynchronize());
  SVAR_HIP(hipMemcpy(buf.data(), n->theta, b, hipMemcpyDeviceToHost));
  SVAR_HIP(hipMemcpy(buf.data() + n->L.n, n->m, b, hipMemcpyDeviceToHost));
  SVAR_HIP(hipMemcpy(buf.data() + 2 * n->L.n, n->v, b, hipMemcpyDeviceToHost));
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return inv(std::string("cannot open ") + tmp + " for writing");
  const bool ok = std::fwrite(&H, sizeof(H), 1, f) == 1 &&
                  std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  const bool closed = std::fclose(f) == 0;
  if (!ok || !closed) return inv(std::string("writing ") + tmp + " failed");
  if (std::rename(tmp.c_str(), path) != 0) return inv(std::string("cannot rename to ") + path);
  return SVAR_OK;
}

int read_ckpt(svar_net* n, const char* path, CkptHeader* out) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return inv(std::string("cannot open ") + path);
  CkptHeader H{};
  std::vector<float> buf;
  bool ok = std::fread(&H, sizeof(H), 1, f) == 1 && std::memcmp(H.magic, "SVARNET1", 8) == 0;
  if (ok && (H.k != n->d.k || H.n_bound != n->d.n_bound || H.nparams != n->L.n)) {
    std::fclose(f);
    return inv("checkpoint was written for another network shape (k, n_bound or size)");
  }
  if (ok) {
    buf.resize((size_t)3 * H.nparams);
    ok = std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  }
  std::fclose(f);
  if (!ok) return inv(std::string(path) + " is not a network checkpoint");
  const size_t b = (size_t)n->L.n * sizeof(float);
  SVAR_HIP(hipMemcpy(n->theta, buf.data(), b, hipMemcpyHostToDevice));
  SVAR_HIP(hipMemcpy(n->m, buf.data() + n->L.n, b, hipMemcpyHostToDevice));
  SVAR_HIP(hipMemcpy(n->v, buf.data() + 2 * n->L.n, b, hipMemcpyHostToDevice));
  n->t = H.adam_t;
  net_pack(n->theta, n->L, n->W, nullptr);
  SVAR_HIP(hipDeviceSynchronize());
  if (out) *out = H;
  return SVAR_OK;
}

}  // namespace

int svar_train(svar_net* n, int32_t npair, int32_t nb, int32_t s, const float* x, const float* y,
               const svar_train_opts* o, const char* ckpt_path, double* loss_hist,
               void* stream) {
  if (!n || !x || !y || !o) return inv("bad arguments");
  SVAR_TRY(check_shape(npair, nb, s));
  if (o->epochs < 1 || o->batch < 1) return inv("need epochs >= 1 and batch >= 1");
  if (o->resume && !ckpt_path) return inv("resume needs a checkpoint path");
  const int64_t nsamp = (int64_t)npair * nb;
  if (nsamp > ((int64_t)1 << 31) - 1) return inv("too many samples");
  int64_t epoch = 0, pos = 0;
  if (o->resume) {
    FILE* f = std::fopen(ckpt_path, "rb");
    if (f) {
      std::fclose(f);
      CkptHeader H{};
      SVAR_TRY(read_ckpt(n, ckpt_path, &H));
      if (H.npair != npair || H.nb != nb || H.s != s || H.seed != o->seed ||
          H.batch != o->batch)
        return inv("checkpoint belongs to another pool, seed or batch size");
      epoch = H.epoch;
      pos = H.pos;
    }
  }
  std::vector<int64_t> ord;
  std::vector<int32_t> smp;
  int64_t steps = 0;
  for (; epoch < o->epochs; ++epoch, pos = 0) {
    epoch_order(nsamp, o->seed, epoch, ord);
    double tot = 0.0;
    int64_t cnt = 0;
    for (; pos < nsamp; pos += o->batch) {
      const int64_t e = std::min<int64_t>(nsamp, pos + o->batch);
      smp.resize(2 * (e - pos));
      for (int64_t q = pos; q < e; ++q) {
        smp[2 * (q - pos)] = (int32_t)(ord[q] / nb);
        smp[2 * (q - pos) + 1] = (int32_t)(ord[q] % nb);
      }
      double loss = 0.0;
      SVAR_TRY(svar_net_train_step(n, npair, nb, s, x, y, (int32_t)(e - pos), smp.data(),
                                   &o->adam, loss_hist ? &loss : nullptr, nullptr, stream));
      tot += loss * (double)(e - pos);
      cnt += e - pos;
      ++steps;
      if (ckpt_path && o->checkpoint_every > 0 && steps % o->checkpoint_every == 0)
        SVAR_TRY(write_ckpt(n, ckpt_path, epoch, e, o->seed, npair, nb, s, o->batch));
    }
    if (loss_hist) loss_hist[epoch] = cnt > 0 ? tot / (double)cnt : 0.0;
    if (ckpt_path)
      SVAR_TRY(write_ckpt(n, ckpt_path, epoch + 1, 0, o->seed, npair, nb, s, o->batch));
  }
  SVAR_HIP(hipStreamSynchronize((hipStream_t)stream));
  return SVAR_OK;
}

int svar_load_learned(svar_net* n, const char* path, int64_t* cursor) {
  if (!n || !path) return inv("bad arguments");
  CkptHeader H{};
  SVAR_TRY(read_ckpt(n, path, &H));
  if (cursor) {
    cursor[0] = H.epoch;
    cursor[1] = H.pos;
    cursor[2] = H.adam_t;
  }
  return SVAR_OK;
}

int svar_set_net(svar_handle* h, svar_net* n) {
  if (!h) return inv("handle is NULL");
  if (n) {
    if (h->popts.type == SVAR_PREC_NONE) return inv("the handle has no preconditioner");
    if (n->d.k != h->popts.k) return inv("the network's k differs from the handle's");
    if (n->device != h->device) return inv("the network lives on another device");
  }
  SVAR_HIP(hipDeviceSynchronize());
  h->net = n;
  h->net_off = nullptr;
  h->prog_gen += 1;
  // preconditioner programs are rebuilt with (or without) the correction
  for (auto it = h->progs.begin(); it != h->progs.end();) {
    if (it->first.op == PROG_P || it->first.op == PROG_PD)
      it = h->progs.erase(it);
    else
      ++it;
  }
  return SVAR_OK;
}

}  // extern "C"

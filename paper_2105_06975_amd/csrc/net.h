// Internal declarations of the sweep-correction network (forward, training, inference
// inside the preconditioner).  Layout conventions:
//   * an activation tensor is [row][channel] with the channel contiguous; the rows of one
//     sample (one block of one system) are its s grid points, consecutive;
//   * layer l's weights for the MFMA kernels are Wk[co][t * CIN + ci] (CIN = 32 padded
//     input channels for layer 1, 64 otherwise), t the tap of the width-5 stencil;
//   * the flat parameter vector keeps the host order W1 (64, cin, 5), b1, W2, b2, W3, b3,
//     W4 (1, 64, 5), b4.
#pragma once
#include <cstdint>
#include <vector>

#include "svar_impl.h"

struct svar_handle;
struct svar_net;

namespace svar {

#define NET_C 64                        // hidden channels
#define NET_W 5                         // stencil width
#define NET_HALO 2
#define NET_CIN1 32                     // padded input channels of layer 1
#define NET_TILE 64                     // grid points per tile
#define NET_FTILE 128                   // grid points per tile of the fused inference kernel
#define NET_ROWS (NET_TILE + NET_W - 1) // staged input rows per tile
#define NET_WG_PART (NET_C * NET_W * NET_C + NET_C)  // largest per-workgroup gradient part

struct NetSample {   // one block of one system
  int64_t src;       // element offset of the system's block 0 in the source vector
  int64_t row0;      // first activation row of the sample
  int32_t s, nb, blk, sys;
};
struct NetTile {
  int32_t sample, pos0;
};
struct NetChunk {    // a range of one system for the per-system sums of squares
  int32_t sys, pad;
  int64_t e0, e1;
};

// offsets of the parameter groups in the flat vector
struct NetLayout {
  int cin = 0;
  int64_t w[4], b[4], n = 0;
  void init(int cin_) {
    cin = cin_;
    const int ci[4] = {cin_, NET_C, NET_C, NET_C};
    const int co[4] = {NET_C, NET_C, NET_C, 1};
    int64_t o = 0;
    for (int l = 0; l < 4; ++l) {
      w[l] = o;
      o += (int64_t)co[l] * ci[l] * NET_W;
      b[l] = o;
      o += co[l];
    }
    n = o;
  }
};

// device weights in kernel layouts (refreshed from the flat parameters after each change)
struct NetWeights {
  float* wf[3] = {nullptr, nullptr, nullptr};        // [64][5 * CIN_l]
  uint16_t* wb[3] = {nullptr, nullptr, nullptr};     // bfloat16 copies
  float* wflip[2] = {nullptr, nullptr};              // layers 2, 3: [ci][t' * 64 + co] =
                                                     // W[co][ci][4 - t']
  float* w4 = nullptr;                               // [t][c]
};

// kernel launchers (k_net.hip)
void net_pack(const float* theta, const NetLayout& L, const NetWeights& W, hipStream_t st);
void net_sumsq(const double* v, const NetChunk* chunks, int nchunk, double* part,
               const int* skip, hipStream_t st);
void net_sigma_impl(const double* part, const int32_t* chunk0, const NetChunk* ch, int nsys,
                    double* sigma, double* inv_sigma, const int* skip, hipStream_t st);
void net_norm_pairs(const double* chat, const double* cex, const double* inv_sigma,
                    int64_t len, int npair, float* x, float* y, hipStream_t st);
// features of layer 1 (float source: training pool, no scaling; double source: vector with
// per-system 1/sigma)
void net_feat_f(const float* src, const NetSample* smp, const NetTile* tiles, int ntiles,
                int64_t row_base, int k, int S, int bf16, void* X0, hipStream_t st);
void net_feat_d(const double* src, const double* inv_sigma, const NetSample* smp,
                const NetTile* tiles, int ntiles, int64_t row_base, int k, int S, int bf16,
                void* X0, const int* skip, const int* off, hipStream_t st);
// hidden layer: out = relu(conv(in) + b) (fwd) or conv(in) * (mask > 0) (bwd, float only);
// tiles of systems whose off flag is set are skipped (off may be NULL)
void net_conv(int bf16, int cin16, int bwd, const void* in, void* out, const void* W,
              const float* bias, const float* mask, const NetSample* smp, const NetTile* tiles,
              int ntiles, int64_t row_base, const int* skip, const int* off, hipStream_t st);
// last layer: training output (outv) or in-place correction dst += sigma * NN (apply)
void net_out(int bf16, const void* a3, const float* w4, const float* b4, const NetSample* smp,
             const NetTile* tiles, int ntiles, int64_t row_base, float* outv, double* dst,
             const double* sigma, const int* off, const int* skip, hipStream_t st);
// fused bfloat16 inference: corr[row] = NN(features) (normalised, float32) for the fused
// tiles (NET_FTILE points), then dst += sigma * corr over the ordinary tiles
void net_fused(const double* src, const double* inv_sigma, const NetSample* smp,
               const NetTile* ftiles, int nftiles, int64_t row_base, int k, int S,
               const NetWeights& W, const float* theta, const NetLayout& L, float* corr,
               const int* skip, const int* off, hipStream_t st);
void net_apply(const float* corr, const NetSample* smp, const NetTile* tiles, int ntiles,
               int64_t row_base, double* dst, const double* sigma, const int* off,
               const int* skip, hipStream_t st);
// training
void net_loss(const float* outv, const float* y, const NetSample* smp, const NetTile* tiles,
              int ntiles, float scale, float* g4, double* lpart, hipStream_t st);
void net_out_bwd(const float* g4, const float* w4, const float* a3, float* g3,
                 const NetSample* smp, const NetTile* tiles, int ntiles, hipStream_t st);
void net_wgrad4(const float* g4, const float* a3, const NetSample* smp, const NetTile* tiles,
                int ntiles, int grid, float* part, hipStream_t st);
void net_wgrad(int cin16, const float* g, const float* a, const NetSample* smp,
               const NetTile* tiles, int ntiles, int grid, float* part, hipStream_t st);
// part2: scratch of ceil(grid / 16) partial rows
void net_wreduce(const float* part, float* part2, int grid, int layer, const NetLayout& L,
                 float* grad, hipStream_t st);
void net_adam(float* theta, const float* grad, float* m, float* v, int64_t n, float lr,
              float b1, float b2, float eps, float bc1, float bc2, hipStream_t st);
int net_grid_cap();
void net_fill_int(int* p, int n, int v, hipStream_t st);

// one in-place application of the network to the Lhat^{-T} output of a preconditioner
// program (host object owned by the handle; device tables in the handle's allocations)
struct NetApp {
  int base = 0;                      // Bases index of the corrected vector
  int nsys = 0, nchunk = 0, ntiles = 0;
  NetChunk* chunks = nullptr;        // device
  int32_t* chunk0 = nullptr;         // device, nsys + 1
  NetSample* smp = nullptr;          // device
  NetTile* tiles = nullptr;          // device
  NetTile* ftiles = nullptr;         // device: tiles of NET_FTILE points (fused kernel)
  int nftiles = 0;
  std::vector<int> ftile0;           // row chunks: first fused tile (size nrc + 1)
  double *part = nullptr, *sigma = nullptr, *inv_sigma = nullptr;
  std::vector<int> tile0;            // row chunks: first tile (size nrc + 1)
  std::vector<int64_t> row0;         // row chunks: first activation row
  int64_t max_rows = 0;              // rows of the largest row chunk
  std::vector<std::pair<int64_t, int64_t>> spans;  // [lo, hi) of every system (validation)
};

int run_net(svar_handle* h, const NetApp& app, double* base, const int* skip, hipStream_t st);

}  // namespace svar

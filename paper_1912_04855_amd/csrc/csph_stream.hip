// Streaming reference for the measurement of the stage kernels.
//
// A stage kernel reads some fields and writes others, each once per cell, plus
// the halos its stencil needs.  The rate HBM delivers for the same mix of read
// and write streams without any halo, in plain address order, is the practical
// ceiling that kernel's bytes can reach; the published peak of the memory is the
// other one.  csph_stream_probe times that mix.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "csph.h"

namespace {

constexpr int kMaxStreams = 16;

struct StreamSet {
  const float* r[kMaxStreams];
  float* w[kMaxStreams];
};

// every cell: the sum of the R read streams goes to each of the W write streams
// (R, W fixed, so that all loads of a cell are issued before the first use)
template <int R, int W>
__global__ void __launch_bounds__(256) k_stream(StreamSet s, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
    float t[R];
#pragma unroll
    for (int v = 0; v < R; ++v) t[v] = s.r[v][c];
    float a = 0.0f;
#pragma unroll
    for (int v = 0; v < R; ++v) a += t[v];
#pragma unroll
    for (int v = 0; v < W; ++v) s.w[v][c] = a + (float)v;
  }
}

// any other mix
__global__ void __launch_bounds__(256) k_stream_any(StreamSet s, int nr, int nw, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
    float a = 0.0f;
    for (int v = 0; v < nr; ++v) a += s.r[v][c];
    for (int v = 0; v < nw; ++v) s.w[v][c] = a + (float)v;
  }
}

// the mixes of the stage kernels (reads, writes): FP32 P (6, 5), C (10, 4),
// E (12, 5); FP64 P (6, 8), C (13, 7)
void launch_stream(const StreamSet& s, int nr, int nw, long long n, unsigned grid, hipStream_t st) {
  if (nr == 6 && nw == 5) k_stream<6, 5><<<grid, 256, 0, st>>>(s, n);
  else if (nr == 10 && nw == 4) k_stream<10, 4><<<grid, 256, 0, st>>>(s, n);
  else if (nr == 12 && nw == 5) k_stream<12, 5><<<grid, 256, 0, st>>>(s, n);
  else if (nr == 6 && nw == 8) k_stream<6, 8><<<grid, 256, 0, st>>>(s, n);
  else if (nr == 13 && nw == 7) k_stream<13, 7><<<grid, 256, 0, st>>>(s, n);
  else k_stream_any<<<grid, 256, 0, st>>>(s, nr, nw, n);
}

}  // namespace

extern "C" csph_status csph_stream_probe(int32_t reads, int32_t writes, int64_t words, int32_t reps,
                                         void* hip_stream, double* ms_per_pass) {
  if (reads < 1 || reads > kMaxStreams || writes < 1 || writes > kMaxStreams || words < 1 || reps < 1 ||
      !ms_per_pass)
    return CSPH_ERR_ARG;
  const hipStream_t st = (hipStream_t)hip_stream;
  const size_t bytes = (size_t)words * sizeof(float);
  StreamSet s{};
  void* bufs[2 * kMaxStreams] = {};
  const int nbuf = reads + writes;
  csph_status rc = CSPH_OK;
  for (int q = 0; q < nbuf && !rc; ++q) {
    if (hipMalloc(&bufs[q], bytes) != hipSuccess) {
      (void)hipGetLastError();
      rc = CSPH_ERR_NOMEM;
    } else if (hipMemsetAsync(bufs[q], 0, bytes, st) != hipSuccess) {
      rc = CSPH_ERR_DEVICE;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = CSPH_ERR_DEVICE;
  if (!rc) {
    for (int q = 0; q < reads; ++q) s.r[q] = (const float*)bufs[q];
    for (int q = 0; q < writes; ++q) s.w[q] = (float*)bufs[reads + q];
    const long long blocks = (words + 255) / 256;
    const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
    // one untimed pass, then `reps` timed ones
    launch_stream(s, reads, writes, words, grid, st);
    if (hipEventRecord(e0, st) != hipSuccess) rc = CSPH_ERR_DEVICE;
    for (int r = 0; r < reps && !rc; ++r) launch_stream(s, reads, writes, words, grid, st);
    if (!rc && (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess))
      rc = CSPH_ERR_DEVICE;
    float ms = 0.0f;
    if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = CSPH_ERR_DEVICE;
    if (!rc) *ms_per_pass = ms / reps;
  }
  (void)hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (int q = 0; q < nbuf; ++q)
    if (bufs[q]) (void)hipFree(bufs[q]);
  return rc;
}

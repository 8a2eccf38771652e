// Work list of the FV sub-cell operator: the elements with alpha > 0, in
// degree-bucket order, rebuilt on the device by every call that has alpha
// (alpha may change from call to call, e.g. once per Runge-Kutta step).
//
// Three small kernels, no atomics and no host round trip, so a captured graph
// replays them as they are:
//   count:   one 1024-lane workgroup per chunk of `order`, wave ballots
//   scan:    one workgroup: exclusive prefix sum of the chunk counts, and the
//            blended count before each degree bucket
//   scatter: each chunk writes its blended elements at its offset, ranked by
//            wave ballots
// The persistent FV kernels then walk blend_list[start[N], start[N + 1]).
#include "dgfv_internal.h"

namespace dgfv {
namespace {

constexpr int WAVES = LIST_CHUNK / 64;

__device__ inline bool blended_at(const MeshView& m, const double* alpha, int i) {
  return i < m.K && alpha[m.order[i]] > 0.0;
}

__global__ void __launch_bounds__(LIST_CHUNK) blend_count_kernel(MeshView m, const double* __restrict__ alpha) {
  __shared__ int wsum[WAVES];
  const int i = blockIdx.x * LIST_CHUNK + threadIdx.x;
  const unsigned long long b = __ballot(blended_at(m, alpha, i));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wsum[wave] = __popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    int sum = 0;
    for (int w = 0; w < WAVES; ++w) sum += wsum[w];
    m.chunk_cnt[blockIdx.x] = sum;
  }
}

__global__ void __launch_bounds__(LIST_CHUNK) blend_scan_kernel(MeshView m, const double* __restrict__ alpha) {
  __shared__ int s[LIST_CHUNK];
  __shared__ int carry;
  const int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < m.n_chunk; base += LIST_CHUNK) {
    const int x = base + t < m.n_chunk ? m.chunk_cnt[base + t] : 0;
    s[t] = x;
    __syncthreads();
    for (int off = 1; off < LIST_CHUNK; off <<= 1) {      // inclusive Hillis-Steele scan
      const int y = t >= off ? s[t - off] : 0;
      __syncthreads();
      s[t] += y;
      __syncthreads();
    }
    if (base + t < m.n_chunk) m.chunk_off[base + t] = carry + s[t] - x;
    __syncthreads();
    if (t == LIST_CHUNK - 1) carry += s[t];
    __syncthreads();
  }
  // blended elements before the first position of each degree bucket: the
  // chunks before its chunk plus the part of its chunk, summed by the whole
  // workgroup
  for (int N = 1; N <= MAXN + 1; ++N) {
    const int P = m.bucket_pos[N];
    const int c = P / LIST_CHUNK;
    int part = 0;
    for (int j = t; j < c; j += LIST_CHUNK) part += m.chunk_cnt[j];
    const int i = c * LIST_CHUNK + t;
    if (i < P && blended_at(m, alpha, i)) part += 1;
    s[t] = part;
    __syncthreads();
    for (int half = LIST_CHUNK / 2; half > 0; half >>= 1) {
      if (t < half) s[t] += s[t + half];
      __syncthreads();
    }
    if (t == 0) m.blend_start[N] = s[0];
    __syncthreads();
  }
  if (t == 0) m.blend_start[0] = 0;
}

__global__ void __launch_bounds__(LIST_CHUNK) blend_scatter_kernel(MeshView m, const double* __restrict__ alpha) {
  __shared__ int wsum[WAVES];
  const int i = blockIdx.x * LIST_CHUNK + threadIdx.x;
  const bool f = blended_at(m, alpha, i);
  const unsigned long long b = __ballot(f);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wsum[wave] = __popcll(b);
  __syncthreads();
  int woff = 0;
  for (int w = 0; w < wave; ++w) woff += wsum[w];
  const int rank = __popcll(b & ((1ull << lane) - 1ull));
  if (f) m.blend_list[m.chunk_off[blockIdx.x] + woff + rank] = m.order[i];
}

}  // namespace

hipError_t launch_blend_list(const MeshView& m, const double* alpha, hipStream_t s) {
  if (m.K == 0) return hipSuccess;
  hipLaunchKernelGGL(blend_count_kernel, dim3(m.n_chunk), dim3(LIST_CHUNK), 0, s, m, alpha);
  hipLaunchKernelGGL(blend_scan_kernel, dim3(1), dim3(LIST_CHUNK), 0, s, m, alpha);
  hipLaunchKernelGGL(blend_scatter_kernel, dim3(m.n_chunk), dim3(LIST_CHUNK), 0, s, m, alpha);
  return hipGetLastError();
}

}  // namespace dgfv

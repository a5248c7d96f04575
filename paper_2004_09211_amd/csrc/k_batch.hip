// Persistent batched kernel: many independent sequences of photon-list
// frames (uneven resolutions, bin counts and photon counts) in one launch.
//
// Work items are (frame n, sequence s, chunk c), a chunk being a band of
// image rows. Items are handed out by one atomic counter in frame-major
// order, so every item an item depends on was handed out before it. Item
// (n, s, c) needs frame n-1 of chunks c-1, c, c+1 of the same sequence (the
// 3x3 prior reads one row of halo): it waits on their done counters, which a
// finished item publishes with a release store at device scope after its
// writes (each wavefront first fences its own stores at device scope); the
// waiter reads them with an acquire, whose cache invalidation serves the whole
// block once the block barrier orders the other wavefronts after it. Waits are bounded (a spin
// limit the host sets); exceeding it records an error and goes on, so every
// wavefront always reaches the exit. Two state buffers alternate per frame:
// by the time an item of frame n+1 overwrites the buffer of frame n-1 for
// its rows, every item that read those rows (chunks c-1..c+1 of frame n)
// has finished, because the item depends on exactly them.
#include "r3d_batch.hpp"
#include "r3d_pixel.hpp"

namespace r3d {

__global__ void k_batch_reset(unsigned* queue, int* done, int ndone) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *queue = 0u;
  for (int k = i; k < ndone; k += gridDim.x * blockDim.x) done[k] = 0;
}

// 4 wavefronts per SIMD: the photon-list pixels are latency-bound
__global__ void __launch_bounds__(256, 4) k_batch(const SeqDesc* __restrict__ seqs, BatchGeom B) {
  extern __shared__ __align__(16) float smem[];
  __shared__ unsigned s_item;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // wave-uniform predicate (readfirstlane), so every branch that brackets a
  // block barrier is uniform and no lane of a wavefront can run ahead into
  // another iteration of the item loop
  const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) < 64u;
  float* sh_h = smem;
  float* sh_irf = smem + kMaxW;
  unsigned* hist = reinterpret_cast<unsigned*>(smem + 2 * kMaxW) + wave * B.hist_words;

  if (wave0 && lane == 0) s_item = atomicAdd(B.queue, 1u);
  __syncthreads();
  unsigned item = __builtin_amdgcn_readfirstlane(s_item);
  while (item < B.nitems) {
    const int n = (int)(item / (unsigned)B.chunks_total);
    const int rem = (int)(item - (unsigned)n * (unsigned)B.chunks_total);
    int s = 0;
    while (s + 1 < B.nseq && B.chunk_prefix[s + 1] <= rem) ++s;
    s = __builtin_amdgcn_readfirstlane(s);
    const SeqDesc& S = seqs[s];
    const int c = rem - B.chunk_prefix[s];
    const bool active = n < S.nframes;  // uniform
    int* const my_done = B.done + S.done_off + c;

    if (active) {
      // wait for frame n-1 of the neighbouring chunks (wavefront 0, uniform loop)
      if (wave0 && n > 0) {
        unsigned spins = 0;
        for (int cc = c - 1; cc <= c + 1; ++cc) {
          if (cc < 0 || cc >= S.nchunks) continue;
          const int* flag = B.done + S.done_off + cc;
          for (;;) {
            const int f = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (f >= n) break;
            if (++spins > B.spin_limit) {
              if (lane == 0) atomicOr(B.err, kErrTimeout);
              break;
            }
            __builtin_amdgcn_s_sleep(2);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      for (int j = threadIdx.x; j < S.M.W; j += blockDim.x) {
        sh_h[j] = S.M.h[j];
        sh_irf[j] = S.M.irf[j];
      }
      __syncthreads();

      StepIO io{};
      const int P = S.M.P;
      const int a = n & 1, b = a ^ 1;
      io.row_ptr = S.row_ptr[n];
      io.toa = S.toa[n];
      io.pi_in = S.pi_in ? S.pi_in + (size_t)n * P : nullptr;
      io.faulty = S.faulty;
      io.pm = S.st_m[a];
      io.pv = S.st_v[a];
      io.ppi = S.st_pi[a];
      io.pb = S.st_b[a];
      io.nm = S.st_m[b];
      io.nv = S.st_v[b];
      io.npi = S.st_pi[b];
      io.nb = S.st_b[b];
      const size_t off = (size_t)n * P;
      io.depth = S.depth ? S.depth + off : nullptr;
      io.var = S.var ? S.var + off : nullptr;
      io.intensity = S.intensity ? S.intensity + off : nullptr;
      io.background = S.background ? S.background + off : nullptr;
      io.pi0_next = S.pi0_next ? S.pi0_next + off : nullptr;
      io.argmax = S.argmax ? S.argmax + off : nullptr;
      DevModel M = S.M;
      M.err = B.err;
      const int r0 = c * S.chunk_rows;
      const int r1 = min(S.M.rows, r0 + S.chunk_rows);
      for (int p = r0 * S.M.cols + wave; p < r1 * S.M.cols; p += 4)
        pixel_step<false>(M, io, p, lane, hist, sh_h, sh_irf);
      // every wavefront makes its own stores visible at device scope before
      // the block publishes the item
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __syncthreads();
    // publish this item and fetch the next one in a single region between
    // two barriers
    if (wave0 && lane == 0) {
      if (active) __hip_atomic_store(my_done, n + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      s_item = atomicAdd(B.queue, 1u);
    }
    __syncthreads();
    item = __builtin_amdgcn_readfirstlane(s_item);
  }
}

hipError_t launch_batch(const SeqDesc* seqs, const BatchGeom& B, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(64), dim3(256), 0, s, B.queue, B.done, B.ndone);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch, dim3(blocks), dim3(256), batch_lds_bytes(B), s, seqs, B);
  return hipGetLastError();
}

size_t batch_lds_bytes(const BatchGeom& B) {
  return (size_t)(2 * kMaxW) * 4 + (size_t)4 * B.hist_words * 4;
}

int batch_blocks_per_cu(const BatchGeom& B) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch, 256, batch_lds_bytes(B)) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

}  // namespace r3d

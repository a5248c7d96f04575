// Descriptors of the persistent batched kernel.
#pragma once

#include "r3d_internal.hpp"

namespace r3d {

// One sequence, as the kernel reads it (device memory).
struct SeqDesc {
  DevModel M;
  int nframes;
  int chunk_rows;  // image rows per work item
  int nchunks;     // ceil(rows / chunk_rows)
  int done_off;    // first of this sequence's done counters
  const int32_t* const* row_ptr;  // [nframes] device pointers
  const int16_t* const* toa;      // [nframes] device pointers
  float* st_m[2];
  float* st_v[2];
  float* st_pi[2];
  float* st_b[2];
  float *depth, *var, *intensity, *background, *pi0_next;  // [nframes][P]
  int32_t* argmax;
  const float* pi_in;     // [nframes][P] or null
  const uint8_t* faulty;  // [P] or null
};

struct BatchGeom {
  int nseq;
  int chunks_total;        // sum of nchunks
  const int* chunk_prefix;  // device [nseq + 1]
  unsigned nitems;         // max frames * chunks_total
  int hist_words;          // LDS words per wavefront (pixel_lds_words of the largest T)
  unsigned spin_limit;     // bound on dependency polls per item
  unsigned* queue;         // work counter
  int* done;               // [ndone] frames completed per (sequence, chunk)
  int ndone;
  unsigned* err;           // error word of the batch
};

hipError_t launch_batch(const SeqDesc* seqs, const BatchGeom& B, int blocks, hipStream_t s);
size_t batch_lds_bytes(const BatchGeom& B);
int batch_blocks_per_cu(const BatchGeom& B);

}  // namespace r3d

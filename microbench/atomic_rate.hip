// Device-atomic and launch microbenchmarks for the MI355X roofline of the compounding
// kernels (gfx950).  Prints:
//   - no-return 32/64-bit global atomic adds per second when each wave instruction covers
//     runs of R consecutive words at random 128-byte-aligned places of a 645 MB buffer
//     (the accumulator size of the whole-spine grid), R = 1 .. 16, and the rate of
//     distinct 64-byte segments per instruction ("requests"); the same with workgroup,
//     agent and system memory scope, and on 2 / 16 / 128 MB footprints;
//   - read bandwidth of a grid-stride streaming kernel;
//   - time per back-to-back launch of an empty kernel.
// Build: hipcc --offload-arch=gfx950 -O3 -o microbench/atomic_rate microbench/atomic_rate.hip
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#define CK(x)                                                                       \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);   \
      return 1;                                                                     \
    }                                                                               \
  } while (0)

// lane l of a wave belongs to run l / R; a run starts at a pseudo-random 128-byte aligned
// line in [0, nlines) and covers R consecutive words
template <class T>
__global__ __launch_bounds__(256) void atomic_runs(T *base, uint32_t nlines, int R, int iters) {
  const uint32_t lane = threadIdx.x & 63, wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t run = lane / R, off = lane - run * R;
  const uint32_t per_line = 128 / sizeof(T);
  for (int it = 0; it < iters; ++it) {
    const uint32_t h = (wave * 64 + run + it * 7919u) * 2654435761u;
    atomicAdd(base + (uint64_t)(h % nlines) * per_line + off, (T)1);
  }
}


template <class T, int SCOPE>
__global__ __launch_bounds__(256) void atomic_runs_scoped(T *base, uint32_t nlines, int R, int iters) {
  const uint32_t lane = threadIdx.x & 63, wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t run = lane / R, off = lane - run * R;
  const uint32_t per_line = 128 / sizeof(T);
  for (int it = 0; it < iters; ++it) {
    const uint32_t h = (wave * 64 + run + it * 7919u) * 2654435761u;
    (void)__hip_atomic_fetch_add(base + (uint64_t)(h % nlines) * per_line + off, (T)1, __ATOMIC_RELAXED, SCOPE);
  }
}

__global__ __launch_bounds__(256) void stream_read(const uint4 *__restrict__ p, int64_t n, uint32_t *out) {
  uint32_t x = 0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint4 v = p[i];
    x ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (x == 0x9e3779b9u) out[0] = x;
}

__global__ void empty_kernel() {}

int main() {
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  const uint64_t bytes = 645120000ull;
  void *buf = nullptr;
  uint32_t *out = nullptr;
  CK(hipMalloc(&buf, bytes));
  CK(hipMalloc(&out, 64));
  CK(hipMemset(buf, 0, bytes));
  const uint32_t nlines = (uint32_t)(bytes / 128) - 1;
  const int blocks = 4096, iters = 4, reps = 20;
  const double n_atomics = (double)blocks * 256 * iters;
  float ms = 0.0f;
  std::printf("atomics: %d x 256 threads x %d per launch, runs at random lines of a %.0f MB buffer\n", blocks,
              iters, bytes / 1e6);
  for (int R : {1, 2, 4, 8, 16}) {
    for (int w = 0; w < 3; ++w) atomic_runs<unsigned long long><<<blocks, 256>>>((unsigned long long *)buf, nlines, R, iters);
    CK(hipEventRecord(e0));
    for (int r = 0; r < reps; ++r)
      atomic_runs<unsigned long long><<<blocks, 256>>>((unsigned long long *)buf, nlines, R, iters);
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    CK(hipEventElapsedTime(&ms, e0, e1));
    double rate = n_atomics * reps / (ms * 1e-3);
    std::printf("  u64 runs of %2d: %7.1f G atomics/s  %6.1f G 64-byte requests/s\n", R, rate / 1e9,
                rate * ((R * 8 + 63) / 64) / R / 1e9);
    for (int w = 0; w < 3; ++w) atomic_runs<unsigned int><<<blocks, 256>>>((unsigned int *)buf, nlines, R, iters);
    CK(hipEventRecord(e0));
    for (int r = 0; r < reps; ++r) atomic_runs<unsigned int><<<blocks, 256>>>((unsigned int *)buf, nlines, R, iters);
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    CK(hipEventElapsedTime(&ms, e0, e1));
    rate = n_atomics * reps / (ms * 1e-3);
    std::printf("  u32 runs of %2d: %7.1f G atomics/s  %6.1f G 64-byte requests/s\n", R, rate / 1e9,
                rate * ((R * 4 + 63) / 64) / R / 1e9);
  }

  for (int R : {1, 4, 16}) {
    for (int sc = 0; sc < 3; ++sc) {
      auto run = [&]() {
        if (sc == 0) atomic_runs_scoped<unsigned long long, __HIP_MEMORY_SCOPE_WORKGROUP><<<blocks, 256>>>((unsigned long long *)buf, nlines, R, iters);
        else if (sc == 1) atomic_runs_scoped<unsigned long long, __HIP_MEMORY_SCOPE_AGENT><<<blocks, 256>>>((unsigned long long *)buf, nlines, R, iters);
        else atomic_runs_scoped<unsigned long long, __HIP_MEMORY_SCOPE_SYSTEM><<<blocks, 256>>>((unsigned long long *)buf, nlines, R, iters);
      };
      for (int w = 0; w < 3; ++w) run();
      CK(hipEventRecord(e0));
      for (int r = 0; r < reps; ++r) run();
      CK(hipEventRecord(e1));
      CK(hipEventSynchronize(e1));
      CK(hipEventElapsedTime(&ms, e0, e1));
      double rate = n_atomics * reps / (ms * 1e-3);
      std::printf("  scope %s u64 runs of %2d: %7.1f G atomics/s  %6.1f G 64-byte requests/s\n",
                  sc == 0 ? "workgroup" : (sc == 1 ? "agent    " : "system   "), R, rate / 1e9,
                  rate * ((R * 8 + 63) / 64) / R / 1e9);
    }
  }
  for (uint64_t small : {2ull << 20, 16ull << 20, 128ull << 20}) {
    const uint32_t nl = (uint32_t)(small / 128) - 1;
    for (int R : {1, 16}) {
      for (int w = 0; w < 3; ++w) atomic_runs<unsigned long long><<<blocks, 256>>>((unsigned long long *)buf, nl, R, iters);
      CK(hipEventRecord(e0));
      for (int r = 0; r < reps; ++r) atomic_runs<unsigned long long><<<blocks, 256>>>((unsigned long long *)buf, nl, R, iters);
      CK(hipEventRecord(e1));
      CK(hipEventSynchronize(e1));
      CK(hipEventElapsedTime(&ms, e0, e1));
      double rate = n_atomics * reps / (ms * 1e-3);
      std::printf("  %4llu MB buffer, u64 runs of %2d: %7.1f G atomics/s  %6.1f G 64-byte requests/s\n",
                  (unsigned long long)(small >> 20), R, rate / 1e9, rate * ((R * 8 + 63) / 64) / R / 1e9);
    }
  }
  const int64_t n16 = (int64_t)(bytes / 16);
  for (int w = 0; w < 3; ++w) stream_read<<<8192, 256>>>((const uint4 *)buf, n16, out);
  CK(hipEventRecord(e0));
  for (int r = 0; r < reps; ++r) stream_read<<<8192, 256>>>((const uint4 *)buf, n16, out);
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  CK(hipEventElapsedTime(&ms, e0, e1));
  std::printf("stream read of %.0f MB: %.0f GB/s\n", bytes / 1e6, (double)bytes * reps / (ms * 1e-3) / 1e9);
  for (int grid : {2560, 10240}) {
    for (int w = 0; w < 10; ++w) empty_kernel<<<grid, 256>>>();
    CK(hipEventRecord(e0));
    for (int r = 0; r < 200; ++r) empty_kernel<<<grid, 256>>>();
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    CK(hipEventElapsedTime(&ms, e0, e1));
    std::printf("empty kernel, %5d blocks of 256: %.2f us per back-to-back launch\n", grid, ms * 1e3 / 200);
  }
  CK(hipDeviceSynchronize());
  CK(hipFree(buf));
  CK(hipFree(out));
  return 0;
}

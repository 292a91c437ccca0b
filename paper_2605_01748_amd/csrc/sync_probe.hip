// sync_probe.hip -- measurement of the two ways an iteration can separate its device-wide steps
// on the running GPU, used to choose the graph engine's structure:
//   (a) kernel boundaries: pairs of near-empty kernels with the grid shapes of the two per-iteration
//       kernels, captured in a HIP graph of 16 pairs and replayed;
//   (b) grid-wide barriers inside one cooperative (co-resident) kernel: every workgroup publishes
//       an arrival counter, then its first wavefront polls all of them.
// Every wait is bounded: a barrier that has not completed after a fixed number of polls sets an
// error flag and the kernel still runs to its end.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace te_probe {

__global__ void k_touch(int *out) {
  if (threadIdx.x == 0) out[blockIdx.x] = (int)blockIdx.x;
}

constexpr int kSpinLimit = 1 << 20;

// After a wait hits its bound, the failure flag makes every other wait of every workgroup return
// at once, so the kernel ends within about one bound.
__global__ void k_barriers(unsigned *arrive, int iters, int *failed) {
  const int nb = gridDim.x;
  for (int it = 1; it <= iters; ++it) {
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      __hip_atomic_store(&arrive[blockIdx.x], (unsigned)it, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x < 64) {
      // relaxed polls (no cache invalidation per poll), one acquire fence once all have arrived
      for (int b = threadIdx.x; b < nb; b += 64) {
        int spins = 0;
        while (__hip_atomic_load(&arrive[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)it) {
          if (++spins > kSpinLimit) {
            atomicExch(failed, 1);
            break;
          }
          if ((spins & 255) == 0 && __hip_atomic_load(failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        }
      }
      __atomic_thread_fence(__ATOMIC_ACQUIRE);
    }
    __syncthreads();
  }
}

}  // namespace te_probe

extern "C" {

// out[0] = microseconds per replayed kernel pair, out[1] = microseconds per grid barrier,
// out[2] = 1 if a barrier wait hit its bound (the measurement is then invalid).
// Returns 0, or a nonzero HIP error code.
int te_probe_sync(int blocks_a, int threads_a, int blocks_b, int threads_b, int iters, double *out) {
  hipError_t e = hipSuccess;
  int *touch = nullptr, *failed = nullptr;
  unsigned *arrive = nullptr;
  hipStream_t st = nullptr, cap = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.f;
  const int nmax = blocks_a > blocks_b ? blocks_a : blocks_b;
  int nbar = 0, dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
#define PCHK(x)                 \
  do {                          \
    e = (x);                    \
    if (e != hipSuccess) goto done; \
  } while (0)
  if (blocks_a < 1 || blocks_b < 1 || threads_a < 64 || threads_b < 64 || threads_a > 1024 || threads_b > 1024 ||
      iters < 1 || !out)
    return (int)hipErrorInvalidValue;
  PCHK(hipMalloc(&touch, sizeof(int) * nmax));
  PCHK(hipMalloc(&failed, sizeof(int)));
  PCHK(hipMemset(failed, 0, sizeof(int)));
  PCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  PCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  PCHK(hipEventCreate(&e0));
  PCHK(hipEventCreate(&e1));
  // (a) graph of 16 kernel pairs
  PCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < 16; ++i) {
    hipLaunchKernelGGL(te_probe::k_touch, dim3(blocks_a), dim3(threads_a), 0, cap, touch);
    hipLaunchKernelGGL(te_probe::k_touch, dim3(blocks_b), dim3(threads_b), 0, cap, touch);
  }
  PCHK(hipStreamEndCapture(cap, &g));
  PCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
  PCHK(hipGraphLaunch(ge, st));
  PCHK(hipEventRecord(e0, st));
  for (int i = 0; i < (iters + 15) / 16; ++i) PCHK(hipGraphLaunch(ge, st));
  PCHK(hipEventRecord(e1, st));
  PCHK(hipEventSynchronize(e1));
  PCHK(hipEventElapsedTime(&ms, e0, e1));
  out[0] = 1e3 * (double)ms / (16.0 * ((iters + 15) / 16));
  // (b) cooperative kernel with grid barriers: as many 1024-thread workgroups as can be co-resident,
  // at most blocks_b (the link kernel's grid)
  PCHK(hipGetDevice(&dev));
  PCHK(hipGetDeviceProperties(&prop, dev));
  PCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, te_probe::k_barriers, 1024, 0));
  nbar = per_cu * prop.multiProcessorCount;
  if (nbar > blocks_b) nbar = blocks_b;
  if (nbar < 1) nbar = 1;
  PCHK(hipMalloc(&arrive, sizeof(unsigned) * nbar));
  PCHK(hipMemset(arrive, 0, sizeof(unsigned) * nbar));
  {
    void *args[] = {&arrive, &iters, &failed};
    PCHK(hipEventRecord(e0, st));
    PCHK(hipLaunchCooperativeKernel((const void *)te_probe::k_barriers, dim3(nbar), dim3(1024), args, 0, st));
    PCHK(hipEventRecord(e1, st));
    PCHK(hipEventSynchronize(e1));
    PCHK(hipEventElapsedTime(&ms, e0, e1));
  }
  out[1] = 1e3 * (double)ms / iters;
  {
    int f = 0;
    PCHK(hipMemcpy(&f, failed, sizeof(int), hipMemcpyDeviceToHost));
    out[2] = (double)f;
  }
done:
  if (ge) (void)hipGraphExecDestroy(ge);
  if (g) (void)hipGraphDestroy(g);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (cap) (void)hipStreamDestroy(cap);
  if (st) (void)hipStreamDestroy(st);
  if (touch) (void)hipFree(touch);
  if (failed) (void)hipFree(failed);
  if (arrive) (void)hipFree(arrive);
#undef PCHK
  return (int)e;
}

}  // extern "C"

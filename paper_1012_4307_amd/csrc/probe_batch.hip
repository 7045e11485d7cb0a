// probe_batch.hip -- measurement probes of two organisations of the batched
// solve (many independent systems, Sec. 2.4) that the library does not use:
// one workgroup per (system, right-hand side) item, and a group of workgroups
// per item meeting at barriers between the phases of a cycle.  No solver call
// reaches these kernels; they exist so the measurements can be repeated.
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "ecsmg_probe.h"

namespace {

constexpr int kItemThreads = 1024;
constexpr int kGroupThreads = 256;
// bounded waits: wall_clock64() counts at a constant 100 MHz
constexpr uint64_t kWaitTicks = 100000000ull;

struct Z {
  double re, im;
};

// Red-black sweeps on independent n x n grids, one workgroup per grid: each
// wave relaxes whole rows (lane h takes column 2h or 2h + 1, whichever has
// the phase's colour), the workgroup meets at a barrier after every colour.
__global__ __launch_bounds__(kItemThreads) void k_probe_item_sweeps(Z *__restrict__ u, const Z *__restrict__ b,
                                                                    const double *__restrict__ k2, int n, int items,
                                                                    int sweeps) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nn = (int64_t)n * n;
  const int H = (n + 1) >> 1;
  for (int it = blockIdx.x; it < items; it += gridDim.x) {
    Z *U = u + it * nn;
    const Z *B = b + it * nn;
    const double *K = k2 + it * nn;
    for (int s = 0; s < sweeps; s++) {
      for (int c = 0; c < 2; c++) {
        for (int j = 1 + wave; j <= n - 2; j += kItemThreads / 64) {
          for (int h = lane; h < H; h += 64) {
            const int i = 2 * h + ((j + c) & 1);
            if (i < 1 || i > n - 2) continue;
            const int64_t p = (int64_t)j * n + i;
            const Z a = U[p - 1], e = U[p + 1], f = U[p - n], g = U[p + n], bv = B[p];
            const double dre = 4.0 - K[p], dim = 0.5;
            const double s2 = 1.0 / (dre * dre + dim * dim);
            const double ore = bv.re + a.re + e.re + f.re + g.re, oim = bv.im + a.im + e.im + f.im + g.im;
            U[p] = Z{(ore * dre + oim * dim) * s2, (oim * dre - ore * dim) * s2};
          }
        }
        __syncthreads();
      }
    }
  }
}

__global__ void k_probe_fill(double *p, int64_t n, double v) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    p[q] = v + 1e-9 * (double)(q & 1023);
}

// One phase barrier among all workgroups of the launch: a central counter
// and a generation number, both device-scope atomics; the last workgroup to
// arrive resets the counter and advances the generation.  The wait is
// bounded in time; a late or failed barrier sets *err, and every workgroup
// stops at its next barrier.
__device__ bool group_barrier(unsigned *count, unsigned *gen, int *err, unsigned blocks) {
  __shared__ int failed;
  __syncthreads();
  if (threadIdx.x == 0) {
    failed = 0;
    const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived = __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (arrived == blocks) {
      __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            wall_clock64() - t0 > kWaitTicks) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    failed = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  return failed == 0;
}

// rounds of (write this workgroup's output, barrier); GRID selects the
// device-wide barrier or a workgroup-local one
template <bool GRID>
__global__ __launch_bounds__(kGroupThreads) void k_probe_group(double *out, int words, int rounds, unsigned *count,
                                                               unsigned *gen, int *err) {
  double *mine = out + (int64_t)blockIdx.x * words;
  for (int r = 0; r < rounds; r++) {
    for (int k = threadIdx.x; k < words; k += kGroupThreads) mine[k] = (double)(r + k);
    if constexpr (GRID) {
      if (!group_barrier(count, gen, err, gridDim.x)) return;
    } else {
      __syncthreads();
    }
  }
}

int hip_fail(hipError_t e) { return e == hipSuccess ? 0 : -3; }

}  // namespace

extern "C" int ecs_probe_item_sweeps(int n, int items, int workgroups, int sweeps, double *ms) {
  if (!ms || n < 5 || n > 4097 || items < 1 || items > 4096 || workgroups < 1 || workgroups > items || sweeps < 1 ||
      sweeps > 64)
    return -1;
  const int64_t nn = (int64_t)n * n, tot = nn * items;
  if ((double)tot * 40.0 > 64.0 * (1ull << 30)) return -1;
  Z *u = nullptr, *b = nullptr;
  double *k2 = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 0;
  float t = 0;
  if ((rc = hip_fail(hipMalloc(&u, tot * sizeof(Z)))) || (rc = hip_fail(hipMalloc(&b, tot * sizeof(Z)))) ||
      (rc = hip_fail(hipMalloc(&k2, tot * sizeof(double)))) || (rc = hip_fail(hipEventCreate(&e0))) ||
      (rc = hip_fail(hipEventCreate(&e1))))
    goto done;
  hipLaunchKernelGGL(k_probe_fill, dim3(1024), dim3(256), 0, nullptr, reinterpret_cast<double *>(u), 2 * tot, 0.0);
  hipLaunchKernelGGL(k_probe_fill, dim3(1024), dim3(256), 0, nullptr, reinterpret_cast<double *>(b), 2 * tot, 1.0);
  hipLaunchKernelGGL(k_probe_fill, dim3(1024), dim3(256), 0, nullptr, k2, tot, 0.5);
  hipLaunchKernelGGL(k_probe_item_sweeps, dim3(workgroups), dim3(kItemThreads), 0, nullptr, u, b, k2, n, items, 1);
  if ((rc = hip_fail(hipEventRecord(e0, nullptr)))) goto done;
  hipLaunchKernelGGL(k_probe_item_sweeps, dim3(workgroups), dim3(kItemThreads), 0, nullptr, u, b, k2, n, items,
                     sweeps);
  if ((rc = hip_fail(hipEventRecord(e1, nullptr))) || (rc = hip_fail(hipEventSynchronize(e1))) ||
      (rc = hip_fail(hipEventElapsedTime(&t, e0, e1))) || (rc = hip_fail(hipGetLastError())))
    goto done;
  *ms = t;
done:
  (void)hipDeviceSynchronize();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(u);
  (void)hipFree(b);
  (void)hipFree(k2);
  return rc;
}

extern "C" int ecs_probe_group_barrier(int blocks, int rounds, int bytes_per_block, double *us_barrier,
                                       double *us_local) {
  if (!us_barrier || !us_local || blocks < 1 || rounds < 1 || rounds > 100000 || bytes_per_block < 0 ||
      bytes_per_block > (1 << 20))
    return -1;
  int dev = 0, cus = 0, per_cu = 0;
  if (hip_fail(hipGetDevice(&dev)) || hip_fail(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) ||
      hip_fail(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_probe_group<true>, kGroupThreads, 0)))
    return -3;
  if (blocks > per_cu * cus) return -1;
  int words = bytes_per_block / 8;
  double *out = nullptr;
  unsigned *sync = nullptr;  // count, generation, error flag
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 0, err = 0;
  float t = 0;
  if ((rc = hip_fail(hipMalloc(&out, (size_t)blocks * (words > 0 ? words : 1) * sizeof(double)))) ||
      (rc = hip_fail(hipMalloc(&sync, 3 * sizeof(unsigned)))) || (rc = hip_fail(hipMemset(sync, 0, 3 * sizeof(unsigned)))) ||
      (rc = hip_fail(hipEventCreate(&e0))) || (rc = hip_fail(hipEventCreate(&e1))))
    goto done;
  {
    unsigned *count = sync, *gen = sync + 1;
    int *errp = reinterpret_cast<int *>(sync + 2);
    for (int pass = 0; pass < 2 && rc == 0; pass++) {
      const bool grid = pass == 0;
      for (int rep = 0; rep < 2 && rc == 0; rep++) {  // rep 0: warm-up with a few rounds
        int rr = rep == 0 ? (rounds < 16 ? rounds : 16) : rounds;
        void *args[] = {&out, &words, &rr, &count, &gen, &errp};
        const void *fn = grid ? reinterpret_cast<const void *>(k_probe_group<true>)
                              : reinterpret_cast<const void *>(k_probe_group<false>);
        if ((rc = hip_fail(hipEventRecord(e0, nullptr)))) break;
        if ((rc = hip_fail(hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(kGroupThreads), args, 0, nullptr)))) break;
        if ((rc = hip_fail(hipEventRecord(e1, nullptr))) || (rc = hip_fail(hipEventSynchronize(e1))) ||
            (rc = hip_fail(hipEventElapsedTime(&t, e0, e1))))
          break;
        if ((rc = hip_fail(hipMemcpy(&err, errp, sizeof(int), hipMemcpyDeviceToHost)))) break;
        if (err) {
          rc = -4;
          break;
        }
        if (rep == 1) *(grid ? us_barrier : us_local) = 1000.0 * t / rounds;
      }
    }
  }
done:
  (void)hipDeviceSynchronize();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  (void)hipFree(sync);
  return rc;
}

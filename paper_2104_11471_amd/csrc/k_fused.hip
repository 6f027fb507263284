// Fused launches: one kernel runs any of the compiled row / column / plane
// variants, so a mixed batch needs one launch per pass level (or one in all)
// instead of one per (level, variant).
//
// The plan fixes a sequence of passes per transform once (Sec. 3.1, Fig. 1);
// a mixed batch is the union of those sequences.  The host lays the (job,
// pass) segments of a launch out as one run of tiles (one tile = one
// workgroup's share of the pass, the same share the pass kernels give
// blockIdx.x), a workgroup per tile; the workgroup finds its segment by binary
// search and runs the segment's variant body through a compile-time dispatch
// table (the same row_body / col_body / plane_body code as the per-variant
// kernels, so every result is bitwise the same).
//
// Two modes.  Level mode (ticketed = 0): one launch per pass level; tile =
// blockIdx.x, no waits (the stream orders the levels).  Dependency mode
// (ticketed = 1): one launch for all levels, segments in (level, job) order; a
// tile of pass l of a job reads what any tile of pass l-1 of that job wrote
// (the passes of Eq. 3 exchange data through global memory only, Sec. 3.2),
// so it takes its index from an atomic counter (arrival order) and first
// waits until that segment's finished-tile count reaches its tile count.  No
// deadlock: a tile waits only on tiles earlier in the queue, which running
// workgroups already hold (a pass-1 tile waits on nothing; by induction every
// held tile finishes); a workgroup that has not started holds no tile.  Every
// wait is still bounded by the wall clock (FusedHdr.wait_ticks): a wait that
// runs out sets the batch's failure flag and the device-wide failure count,
// after which the remaining dependent tiles give up at once, so the launch
// always drains.  Visibility: each wave of a tile that is waited on makes its
// stores visible at agent scope (release fence: on this GPU it writes back
// the XCD's L2, whose contents other XCDs do not see) before the workgroup
// barrier, then one lane counts the tile; the waiting lane reads the count
// with acquire semantics and every wave takes an acquire fence after the
// barrier that follows the wait.  Those fences and the ticket make the mode
// slower than level mode on MI355X (measured), so level mode is the default.
//
// One tile per workgroup rather than a persistent loop: with a loop around the
// variant dispatch the compiler keeps values live across variants and the
// register budget of two workgroups per CU spills.
#include "plane_body.h"

namespace tcfft {

namespace {

// Variants compiled into the fused kernels.  Rows: C = points per workgroup
// (0 = 16384), tstore = transposed store (second pass of a four-step
// transform).  Columns: C adjacent columns.  Plane: L = nz, C = ny.
struct FusedVariant {
  int kind, L, R0, C, split, xtw, tstore;
};

constexpr FusedVariant kFused[] = {
    // FP16 rows, 16384 points per workgroup
    {K_ROW, 16, 1, 0, 0, 0, 0},      {K_ROW, 32, 2, 0, 0, 0, 0},
    {K_ROW, 64, 4, 0, 0, 0, 0},      {K_ROW, 128, 8, 0, 0, 0, 0},
    {K_ROW, 256, 1, 0, 0, 0, 0},     {K_ROW, 512, 2, 0, 0, 0, 0},
    {K_ROW, 1024, 4, 0, 0, 0, 0},    {K_ROW, 2048, 8, 0, 0, 0, 0},
    {K_ROW, 4096, 1, 0, 0, 0, 0},    {K_ROW, 8192, 2, 0, 0, 0, 0},
    {K_ROW, 16384, 4, 0, 0, 0, 0},
    // FP16 rows, 8192 points per workgroup; transposed-store rows
    {K_ROW, 1024, 4, 8192, 0, 0, 0}, {K_ROW, 256, 1, 0, 0, 0, 1},
    {K_ROW, 512, 2, 0, 0, 0, 1},     {K_ROW, 1024, 4, 0, 0, 0, 1},
    // FP16 columns: four-step first passes (inter-pass twiddle, transposed
    // store or natural order), second passes and 2D columns
    {K_COL, 128, 8, 64, 0, 1, 1},    {K_COL, 128, 8, 64, 0, 1, 0},
    {K_COL, 256, 1, 64, 0, 1, 1},    {K_COL, 256, 1, 64, 0, 1, 0},
    {K_COL, 256, 1, 64, 0, 0, 0},    {K_COL, 512, 2, 64, 0, 1, 1},
    {K_COL, 512, 2, 64, 0, 0, 0},    {K_COL, 1024, 4, 32, 0, 1, 1},
    {K_COL, 1024, 4, 32, 0, 0, 0},   {K_COL, 2048, 8, 16, 0, 1, 1},
    {K_COL, 2048, 8, 16, 0, 0, 0},
    // FP16 planes (2D 128 x 128, 64 x 64)
    {K_PLANE, 128, 8, 128, 0, 0, 0}, {K_PLANE, 64, 4, 64, 0, 0, 0},
    // split rows
    {K_ROW, 16, 1, 0, 1, 0, 0},      {K_ROW, 32, 2, 0, 1, 0, 0},
    {K_ROW, 64, 4, 0, 1, 0, 0},      {K_ROW, 128, 8, 0, 1, 0, 0},
    {K_ROW, 256, 1, 8192, 1, 0, 0},  {K_ROW, 512, 2, 8192, 1, 0, 0},
    {K_ROW, 1024, 4, 8192, 1, 0, 0}, {K_ROW, 2048, 8, 8192, 1, 0, 0},
    {K_ROW, 4096, 1, 8192, 1, 0, 0}, {K_ROW, 8192, 2, 8192, 1, 0, 0},
    {K_ROW, 16384, 4, 0, 1, 0, 0},
    // split columns and plane
    {K_COL, 64, 4, 64, 1, 0, 0},     {K_COL, 128, 8, 64, 1, 1, 1},
    {K_COL, 256, 1, 64, 1, 1, 1},    {K_COL, 256, 1, 64, 1, 0, 0},
    {K_COL, 512, 2, 32, 1, 1, 1},    {K_COL, 512, 2, 32, 1, 0, 0},
    {K_COL, 1024, 4, 16, 1, 1, 1},   {K_COL, 1024, 4, 16, 1, 0, 0},
    {K_COL, 2048, 8, 8, 1, 1, 1},    {K_COL, 2048, 8, 8, 1, 0, 0},
    {K_PLANE, 128, 8, 128, 1, 0, 0},
};
constexpr int kNumFused = (int)(sizeof(kFused) / sizeof(kFused[0]));

constexpr int r0_for(int n) { return 1 << (ilog2c(n) % 4); }

template <bool SPLIT, int I = 0>
__device__ __forceinline__ void fused_run(int var, const KParams& kp, int64_t wg, uint32_t* lds) {
  if constexpr (I < kNumFused) {
    constexpr FusedVariant v = kFused[I];
    if constexpr ((v.split != 0) == SPLIT) {
      if (var == I) {
        if constexpr (v.kind == K_ROW)
          row_body<v.L, v.R0, 256, SPLIT, v.tstore != 0, 0, (v.C ? v.C : 16384)>(kp, wg, lds);
        else if constexpr (v.kind == K_COL)
          col_body<v.L, v.R0, v.C, 256, SPLIT, v.xtw != 0, v.tstore != 0>(kp, wg, lds);
        else
          plane_body<v.L, v.R0, v.C, r0_for(v.C), 256, SPLIT>(kp, wg, lds);
        return;
      }
    }
    fused_run<SPLIT, I + 1>(var, kp, wg, lds);
  }
}

typedef const TCFFT_CONST FusedHdr CFusedHdr;
typedef const TCFFT_CONST FusedSeg CFusedSeg;

__device__ unsigned g_fused_wait_failures;

__device__ __forceinline__ int find_seg(const TCFFT_CONST int32_t* starts, int nsegs, int t) {
  int lo = 0, hi = nsegs - 1;  // largest s with starts[s] <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (starts[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Waits until *done >= need; false when the batch has already failed or the
// wait ran past `ticks` of the wall clock (then the batch is marked failed).
__device__ bool wait_count(int* done, int need, int* failed, int64_t ticks) {
  if (__hip_atomic_load(done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
  const int64_t t0 = wall_clock64();
  for (;;) {
    if (__hip_atomic_load(failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (wall_clock64() - t0 > ticks) {
      if (__hip_atomic_fetch_add(failed, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        __hip_atomic_fetch_add(&g_fused_wait_failures, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
    if (__hip_atomic_load(done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
  }
}

template <bool SPLIT>
__global__ __launch_bounds__(256, SPLIT ? 1 : 2) void fused_kernel_t(const FusedHdr* __restrict__ hdr) {
  extern __shared__ uint32_t lds[];
  CFusedHdr* h = (CFusedHdr*)hdr;
  CFusedSeg* segs = (CFusedSeg*)h->segs;
  CKParams* kps = (CKParams*)h->kps;
  int* const head = h->ctr;
  int* const failed = h->ctr + 1;
  int* const done = h->ctr + 2;
  const int nsegs = (int)h->nsegs;
  const int64_t total = h->total;
  const int64_t ticks = h->wait_ticks;
  uint32_t* const slot = lds + h->lds_slot;  // [0] tile index, [1] wait result
  int64_t t = blockIdx.x;
  if (h->ticketed) {  // dependency waits: tiles in arrival order
    if (threadIdx.x == 0)
      slot[0] = (uint32_t)__hip_atomic_fetch_add(head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    t = slot[0];
  }
  if (t >= total) return;
  const int s = find_seg((const TCFFT_CONST int32_t*)h->starts, nsegs, (int)t);
  const int dep = segs[s].dep;
  bool ok = true;
  if (dep >= 0) {  // one lane waits and decides for the workgroup
    if (threadIdx.x == 0)
      slot[1] = wait_count(done + dep, (int)segs[dep].tiles, failed, ticks) ? 1u : 0u;
    __syncthreads();
    ok = slot[1] != 0;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  if (ok) {
    const KParams kp = load_job(kps, segs[s].kp);
    fused_run<SPLIT>(segs[s].var, kp, t - segs[s].start, lds);
  }
  // an agent-scope release writes back the XCD's L2 (the GPU's L2s are not
  // coherent with each other): only tiles that a later tile waits on pay it
  if (segs[s].waited) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();  // every wave's stores are visible before the tile counts
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(done + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

int fused_variant(const KernelKey& k) {
  if (k.NT != 256 || k.real != 0) return -1;
  for (int i = 0; i < kNumFused; ++i) {
    const FusedVariant& v = kFused[i];
    if (v.kind == k.kind && v.L == k.L && v.R0 == k.R0 && v.C == k.C && v.split == k.split &&
        v.xtw == k.xtw && v.tstore == k.tstore)
      return i;
  }
  return -1;
}

const void* fused_kernel(bool split) {
  return split ? (const void*)fused_kernel_t<true> : (const void*)fused_kernel_t<false>;
}

hipError_t fused_wait_failures(unsigned* count) {
  return hipMemcpyFromSymbol(count, HIP_SYMBOL(g_fused_wait_failures), sizeof(unsigned), 0,
                             hipMemcpyDeviceToHost);
}

}  // namespace tcfft

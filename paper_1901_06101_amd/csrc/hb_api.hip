// Host orchestration of H-BACA (Algorithm 3) behind the C ABI in hbaca.h.
//
// One call runs, on one stream:
//   setup      cluster trees, leaf descriptors, first column blocks (SplitMix64)
//   leaf BACA  one launch of the leaf kernel over every leaf of every problem
//   leaf SVD   TSQR of U and V^H, M = R_U R_V^H, Jacobi SVD, Q applied to X, Y
//   merges     for l = 1..L: horizontal merges, then vertical merges, each a
//              batch over all blocks of all problems (TSQR, SVD, block GEMM)
// The host reads back only ranks (to size the next step) and small records.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/hbaca.h"
#include "hb_common.h"
#include "hb_entries.h"
#include "hb_adj_plan.h"
#include "hb_internal.h"
#include "hb_merge.h"

namespace {

// ------------------------------------------------------------------ errors --
struct HbError {
  hb_status st;
};
// With HB_VERBOSE set in the environment, every failing HIP call or launch
// and every unsupported size is reported on stderr with its source line.
// set once the runtime has refused a cooperative launch in this process
static std::atomic<bool> g_coop_refused{false};

static void hb_report(const char* what, int code, const char* detail, int line) {
  static const bool on = std::getenv("HB_VERBOSE") != nullptr;
  if (on) std::fprintf(stderr, "[hbaca] %s failed (%d: %s) at hb_api.hip:%d\n", what, code, detail, line);
}
#define HB_HIP(call)                                                         \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      hb_report(#call, (int)e_, hipGetErrorString(e_), __LINE__);            \
      throw HbError{HB_EDEVICE};                                             \
    }                                                                        \
  } while (0)
#define HB_LAUNCH(call)                                                      \
  do {                                                                       \
    int e_ = (call);                                                         \
    if (e_ == -1) {                                                          \
      hb_report(#call, e_, "size outside the built kernels", __LINE__);      \
      throw HbError{HB_EUNSUPPORTED};                                        \
    }                                                                        \
    if (e_ != 0) {                                                           \
      hb_report(#call, e_, hipGetErrorString((hipError_t)e_), __LINE__);     \
      throw HbError{HB_EDEVICE};                                             \
    }                                                                        \
  } while (0)

// --------------------------------------------------------- device memory ---
// Caching device allocator.  Blocks are rounded up to size classes (four per
// octave, at least 256 bytes), obtained once with hipMalloc and never given
// back to the HIP runtime: a freed block goes to a free list tagged with the stream
// whose work last used it and is reused only by work on that same stream
// (stream order makes the reuse safe), or by any stream once the device has
// been synchronised (result memory).  This keeps allocation off the critical
// path: a call allocates and frees a few hundred buffers.
class BlockCache {
 public:
  static BlockCache& get() {
    static BlockCache c;
    return c;
  }
  void* alloc(size_t bytes, hipStream_t st) {
    const size_t cls = size_class(bytes);
    {
      std::lock_guard<std::mutex> g(mu_);
      int dev = 0;
      (void)hipGetDevice(&dev);
      auto& lst = free_[cls];
      for (size_t i = lst.size(); i-- > 0;) {
        const Entry& e = lst[i];
        if (e.dev == dev && (e.st == st || e.idle)) {
          void* p = e.ptr;
          lst.erase(lst.begin() + (ptrdiff_t)i);
          return p;
        }
      }
    }
    void* p = nullptr;
    if (hipMalloc(&p, cls) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      trim();
      if (hipMalloc(&p, cls) != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    std::lock_guard<std::mutex> g(mu_);
    size_[p] = cls;
    return p;
  }
  // `idle`: the device has finished every use of the block
  void release(void* p, hipStream_t st, bool idle) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = size_.find(p);
    if (it == size_.end()) return;
    int dev = 0;
    (void)hipGetDevice(&dev);
    free_[it->second].push_back(Entry{p, it->second, st, idle, dev});
  }

 private:
  struct Entry {
    void* ptr;
    size_t bytes;
    hipStream_t st;
    bool idle;
    int dev;
  };
  static size_t size_class(size_t b) {
    size_t c = 256;
    while (c < b) {
      // four classes per octave: c, 1.25c, 1.5c, 1.75c
      const size_t q = c / 4;
      if (c + q >= b) return c + q;
      if (c + 2 * q >= b) return c + 2 * q;
      if (c + 3 * q >= b) return c + 3 * q;
      c *= 2;
    }
    return c;
  }
  // out of memory: give every idle cached block back and try again
  void trim() {
    (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> g(mu_);
    for (auto& kv : free_)
      for (auto& e : kv.second) {
        (void)hipFree(e.ptr);
        size_.erase(e.ptr);
      }
    free_.clear();
  }
  std::mutex mu_;
  std::unordered_map<size_t, std::vector<Entry>> free_;  // by size class
  std::unordered_map<void*, size_t> size_;
};

struct DevMem {
  std::vector<void*> ptrs;
  hipStream_t st = nullptr;
  bool sync_free = false;  // results outlive the caller's stream
  void* alloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    void* p = BlockCache::get().alloc(bytes, st);
    if (p == nullptr) throw HbError{HB_ENOMEM};
    ptrs.push_back(p);
    return p;
  }
  template <typename T> T* get(size_t n) { return (T*)alloc(n * sizeof(T)); }
  // one allocation carved into 256-byte aligned pieces
  std::vector<char*> carve(const std::vector<size_t>& sizes) {
    size_t tot = 0;
    std::vector<size_t> off(sizes.size());
    for (size_t i = 0; i < sizes.size(); ++i) {
      off[i] = tot;
      tot += (std::max<size_t>(sizes[i], 1) + 255) & ~(size_t)255;
    }
    char* base = (char*)alloc(tot);
    std::vector<char*> out(sizes.size());
    for (size_t i = 0; i < sizes.size(); ++i) out[i] = base + off[i];
    return out;
  }
  void release() {
    if (ptrs.empty()) return;
    if (sync_free) (void)hipDeviceSynchronize();
    for (void* p : ptrs) BlockCache::get().release(p, st, sync_free);
    ptrs.clear();
  }
  ~DevMem() { release(); }
};

template <typename T>
static T* upload(DevMem& mem, const std::vector<T>& v, hipStream_t st) {
  T* d = mem.get<T>(v.size() ? v.size() : 1);
  if (!v.empty()) HB_HIP(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return d;
}

// The descriptors of several launches, sent to the device in one copy before
// the first of them: a copy queued between two kernels leaves the device idle
// while it runs.  Launches are recorded as callbacks and issued by run(),
// after the copy; at() gives the device address of a descriptor array there.
struct Batch {
  std::vector<unsigned char> h;
  unsigned char* d = nullptr;
  std::vector<std::function<void()>> launches;
  template <typename T>
  size_t add(const std::vector<T>& v) {
    static_assert(std::is_trivially_copyable<T>::value, "descriptors are copied bytewise");
    const size_t o = (h.size() + 255) & ~(size_t)255;
    h.insert(h.end(), o - h.size(), (unsigned char)0);
    const unsigned char* p = (const unsigned char*)v.data();
    if (v.empty()) h.insert(h.end(), sizeof(T), (unsigned char)0);
    else h.insert(h.end(), p, p + v.size() * sizeof(T));
    return o;
  }
  template <typename T> T* at(size_t o) const { return (T*)(d + o); }
  void then(std::function<void()> f) { launches.push_back(std::move(f)); }
  void run(DevMem& mem, hipStream_t st) {
    if (!h.empty()) {
      d = (unsigned char*)mem.alloc(h.size());
      HB_HIP(hipMemcpyAsync(d, h.data(), h.size(), hipMemcpyHostToDevice, st));
    }
    for (auto& f : launches) f();
    h.clear();
    launches.clear();
    d = nullptr;
  }
};

// Copies `bytes` from the device to `dst` after the stream's work, and waits:
// through a pinned buffer of the calling thread (grown as needed, kept for
// the life of the thread), so the copy is one transfer rather than a staged
// one.  The wait polls an event for up to 3 ms before it blocks: a rank
// read-back sits between two dependent launches, and polling wakes sooner.
static void d2h_sync(void* dst, const void* src, size_t bytes, hipStream_t st) {
  static thread_local void* pin = nullptr;
  static thread_local size_t cap = 0;
  if (bytes > cap) {
    const size_t want = std::max<size_t>(bytes, 64 * 1024);
    void* p = nullptr;
    if (hipHostMalloc(&p, want, hipHostMallocDefault) == hipSuccess) {
      if (pin) (void)hipHostFree(pin);  // idle: every use waits for its copy
      pin = p;
      cap = want;
    } else {
      (void)hipGetLastError();
    }
  }
  if (bytes <= cap) {
    HB_HIP(hipMemcpyAsync(pin, src, bytes, hipMemcpyDeviceToHost, st));
    static thread_local hipEvent_t ev = nullptr;
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      ev = nullptr;
    }
    bool done = false;
    if (ev && hipEventRecord(ev, st) == hipSuccess) {
      const auto t0 = std::chrono::steady_clock::now();
      while (true) {
        const hipError_t q = hipEventQuery(ev);
        if (q == hipSuccess) {
          done = true;
          break;
        }
        if (q != hipErrorNotReady) {  // the blocking wait below reports it
          (void)hipGetLastError();
          break;
        }
        if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(3000)) break;
      }
    } else {
      (void)hipGetLastError();
    }
    if (!done) HB_HIP(hipStreamSynchronize(st));
    std::memcpy(dst, pin, bytes);
  } else {
    HB_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
    HB_HIP(hipStreamSynchronize(st));
  }
}

// Applies through trees of more nodes than this issue every tree level as soon
// as its descriptors are built (the host prepares the next level while the
// device runs this one); smaller ones send all levels in one copy.
constexpr size_t kApplyBatchNodes = 512;
// TSQR factor levels of at least this many nodes (the CUs of the device) are
// launched once per register-width class
constexpr size_t kSplitNodes = 256;

// ------------------------------------------------------------ SplitMix64 ---
// J_1 of leaf b: SplitMix64 (Steele, Lea and Flood 2014) from
// seed + b * 0x632BE59BD9B4E019, partial Fisher-Yates over 0..n0-1.
static void first_column_block(uint64_t seed, uint64_t b, int n0, int d, int32_t* out) {
  const int q = std::min(d, n0);
  uint64_t s = seed + b * 0x632BE59BD9B4E019ull;
  // q steps of a Fisher-Yates shuffle of 0..n0-1, on an identity array kept
  // per thread: the swaps are undone afterwards, so a call costs O(q)
  static thread_local std::vector<int32_t> perm;
  static thread_local std::vector<int32_t> js;
  if ((int)perm.size() < n0) {
    const int old = (int)perm.size();
    perm.resize(n0);
    for (int i = old; i < n0; ++i) perm[i] = i;
  }
  if ((int)js.size() < q) js.resize(q);
  for (int t = 0; t < q; ++t) {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const int j = t + (int)(z % (uint64_t)(n0 - t));
    js[t] = j;
    std::swap(perm[t], perm[j]);
  }
  for (int t = 0; t < q; ++t) out[t] = perm[t];
  for (int t = q - 1; t >= 0; --t) std::swap(perm[t], perm[js[t]]);
}

// ------------------------------------------------------------ trees --------
static int tree_levels(int64_t m, int64_t n, int64_t leaf) {
  int L = 0;
  const int64_t big = std::max(m, n);
  while (leaf * ((int64_t)1 << L) < big) ++L;
  while (L > 0 && ((int64_t)1 << L) > std::min(m, n)) --L;
  return L;
}

struct Node {
  int64_t off, size;
};
static std::vector<std::vector<Node>> cluster_tree(int64_t size, int L) {
  std::vector<std::vector<Node>> lv(1, std::vector<Node>{{0, size}});
  for (int l = 0; l < L; ++l) {
    std::vector<Node> nx;
    for (const Node& nd : lv.back()) {
      const int64_t h = (nd.size + 1) / 2;
      nx.push_back({nd.off, h});
      nx.push_back({nd.off + h, nd.size - h});
    }
    lv.push_back(nx);
  }
  return lv;
}

// ------------------------------------------------------------ kernels ------
__global__ void aos_to_soa_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                  int64_t npts, int dim) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts) return;
  for (int c = 0; c < dim; ++c) dst[(int64_t)c * npts + i] = src[i * dim + c];
}

// FP32 vectors to FP64 and back (the adjoint's FP32 entry point).
__global__ void widen_kernel(const float* __restrict__ src, double* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

__global__ void narrow_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

// Compressed operator applied to a vector: y = U diag(S) Vh^H w, or its
// adjoint w~ = Vh diag(S) U^H y.  First t_j = S_j sum_i conj(X(i, j)) v_i for
// every column j of X (one workgroup per column, a deterministic tree sum),
// then out_i = sum_j Z(i, j) t_j (one thread per row, t staged in LDS).
constexpr int AP_NT = 256;
template <typename T>
__global__ __launch_bounds__(AP_NT) void apply_reduce_kernel(const T* __restrict__ X, int64_t len,
                                                             int r, const double* __restrict__ S,
                                                             const T* __restrict__ v,
                                                             T* __restrict__ t) {
  const int j = blockIdx.x;
  if (j >= r) return;
  const T* x = X + (int64_t)j * len;
  T acc = sc_zero<T>();
  for (int64_t i = threadIdx.x; i < len; i += AP_NT) sc_cfma(acc, x[i], v[i]);
  acc = group_sum_sc<64, T>(acc);
  __shared__ T part[AP_NT / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T sum = part[0];
    for (int w = 1; w < AP_NT / 64; ++w) sum = sc_add(sum, part[w]);
    t[j] = sc_scale(sum, S[j]);
  }
}
template <typename T>
__global__ __launch_bounds__(AP_NT) void apply_expand_kernel(const T* __restrict__ Z, int64_t len,
                                                             int r, const T* __restrict__ t,
                                                             T* __restrict__ out) {
  extern __shared__ unsigned char smem_ap[];
  T* st = (T*)smem_ap;
  for (int j = threadIdx.x; j < r; j += AP_NT) st[j] = t[j];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * AP_NT + threadIdx.x;
  if (i >= len) return;
  T acc = sc_zero<T>();
  for (int j = 0; j < r; ++j) sc_fma(acc, Z[(int64_t)j * len + i], st[j]);
  out[i] = acc;
}

// FP32 leaf factors of the mixed-precision path widened to FP64 for the
// re-compression and the merges (one grid row per factor).
struct CvtDev {
  const float* src;
  double* dst;
  int64_t n;
};
__global__ void cvt_f2d_kernel(const CvtDev* __restrict__ jobs) {
  const CvtDev J = jobs[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < J.n;
       i += (int64_t)gridDim.x * blockDim.x)
    J.dst[i] = (double)J.src[i];
}

// M = R_U R_V^H for one leaf: R_U (pu x r), R_V (pv x r) from TSQR top nodes.
template <typename T>
__global__ void rrh_kernel(const QRNodeDev* __restrict__ topU, const QRNodeDev* __restrict__ topV,
                           const T* __restrict__ store, const T* __restrict__ alpha,
                           T* const* __restrict__ Mout) {
  const QRNodeDev A = topU[blockIdx.x];
  const QRNodeDev B = topV[blockIdx.x];
  const int pu = A.steps, pv = B.steps, r = A.k;
  T* M = Mout[blockIdx.x];
  for (int e = threadIdx.x; e < pu * pv; e += blockDim.x) {
    const int i = e % pu, j = e / pu;
    T acc = sc_zero<T>();
    // R_U(i, t) nonzero for t >= i; R_V(j, t) nonzero for t >= j
    for (int t = max(i, j); t < r; ++t) {
      const T a = (i < t) ? store[A.store + (int64_t)t * 256 + i] : alpha[A.ab + t];
      const T b = (j < t) ? store[B.store + (int64_t)t * 256 + j] : alpha[B.ab + t];
      sc_fma(acc, a, sc_conj(b));
    }
    M[e] = acc;  // column-major pu x pv
  }
}

// Sums of |A - U S Vh^H|^2 and |A|^2 over rows i = stride * blockIdx.y... one
// workgroup per (row, column tile); partial sums per workgroup.
template <typename T>
__global__ void error_kernel(EntryDev E, int64_t row_base, int64_t col_base, int64_t m, int64_t n,
                             const T* __restrict__ U, const double* __restrict__ S,
                             const T* __restrict__ Vh, int r, int64_t stride, int64_t nrows_s,
                             double* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0.0, a2 = 0.0;
  if (j < n) {
    double yj[HB_MAXDIM];
    for (int q = 0; q < HB_MAXDIM; ++q) yj[q] = q < E.dim ? E.Y[(int64_t)q * E.ldy + col_base + j] : 0.0;
    for (int64_t rr = blockIdx.y; rr < nrows_s; rr += gridDim.y) {
      const int64_t i = rr * stride;
      double xi[HB_MAXDIM];
      for (int q = 0; q < HB_MAXDIM; ++q) xi[q] = q < E.dim ? E.X[(int64_t)q * E.ldx + row_base + i] : 0.0;
      const T a = eval_entry<T>(E, row_base + i, col_base + j, xi, yj);
      T ap = sc_zero<T>();
      for (int t = 0; t < r; ++t)
        sc_fma(ap, sc_scale(U[(int64_t)t * m + i], S[t]), sc_conj(Vh[(int64_t)t * n + j]));
      e2 += sc_abs2(sc_sub(a, ap));
      a2 += sc_abs2(a);
    }
  }
  __shared__ double r1[256], r2[256];
  r1[threadIdx.x] = e2;
  r2[threadIdx.x] = a2;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r1[threadIdx.x] += r1[threadIdx.x + s];
      r2[threadIdx.x] += r2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * (blockIdx.y * gridDim.x + blockIdx.x)] = r1[0];
    part[2 * (blockIdx.y * gridDim.x + blockIdx.x) + 1] = r2[0];
  }
}

// ------------------------------------------------------------ structures ---
struct Block {  // compressed block A_b ~ U diag(S) Vh^H on the device
  int64_t m = 0, n = 0;
  int r = 0;
  void* U = nullptr;   // m x r, ld m
  void* Vh = nullptr;  // n x r, ld n
  double* S = nullptr; // r
};

struct Problem {
  int64_t m, n, row_base, col_base;
  int L;
  uint64_t seed;
  std::vector<std::vector<Node>> rt, ct;
  Block root;
};

struct LeafHost {
  int problem, t, v;
  int64_t row0, col0;
  int m0, n0;
  int rank_baca = 0, rank_leaf = 0, iters = 0, status = 0;
  std::vector<int32_t> tape_rows, tape_cols, it_dk;
  std::vector<double> it_nu, it_mu;
  std::vector<int32_t> fz;  // frozen structure: iters records of fz_stride ints
};

}  // namespace

struct hb_result {
  int scalar = 0;  // 0 real, 1 complex
  int entry = 0;
  EntryDev E{};
  std::vector<Problem> problems;
  std::vector<LeafHost> leaves;
  std::vector<Block> out_blocks;  // what hb_result_copy returns
  DevMem keep;                     // device memory owned by the result
  hb_stats stats{};
  // frozen structure for the adjoint (record_tape == 2, single problem):
  // the stride of the per-iteration records, the ranks of the horizontal
  // merges of level l (block (ti, v), ti-major) and of the vertical merges
  // (block (t, v), t-major), and the kernel parameters
  int fz_stride = 0;
  bool fz_complete = false;  // set once the whole pipeline ran on one problem
  std::vector<std::vector<int>> fz_hrank, fz_vrank;
  double fz_h = 0.0, fz_c = 0.0;
};

struct hb_hodlr {
  int64_t N = 0;
  int levels = 0;                        // depth of the cluster tree
  hb_result* blocks = nullptr;           // H-BACA of every off-diagonal block
  std::vector<int> level;                // per block
  std::vector<int64_t> roff, rcnt, coff, ccnt;
  std::vector<std::vector<int>> by_level;  // block indices of each level
  int64_t nleaves = 0;
  void* leaves_dev = nullptr;            // HodlrLeafDev per leaf
  std::vector<int64_t> leaf_off, leaf_size;
  double* dense = nullptr;               // dense diagonal blocks
  int64_t dense_elems = 0;
  std::vector<void*> jobs_dev;           // HodlrJob arrays per level
  std::vector<int> level_rmax;
  std::vector<int64_t> level_rowmax;
  int64_t t_elems = 0;                   // products per matvec
  int64_t leaf_max = 0;
  DevMem keep;                           // device memory of this object
  ~hb_hodlr();
};

namespace {

static size_t scalar_bytes(int scalar) { return scalar == 1 ? 16 : 8; }

// ------------------------------------------------- batched truncated SVDs ---
// A "merge job" computes the truncated SVD of B = [P1 diag(S1), P2 diag(S2)]
// (rows x k) and applies it:  Pnew = Q X_r,  Onew = blockdiag(O1, O2) Y_r.
// With O1 == nullptr (leaf re-compression) the job is the SVD re-compression
// of U Vh^H instead (see run_recompress).
struct MergeJob {
  int64_t rows;           // rows of P1, P2
  const void* P1; int r1; const double* S1;
  const void* P2; int r2; const double* S2;
  const void* O1; int64_t n1;  // O1: n1 x r1
  const void* O2; int64_t n2;
  Block* outP_owner;  // filled: rank, S, P (as out->U or out->Vh), O
  bool p_is_u;        // true: P side is U (horizontal), false: P side is Vh
};

struct TreeBuild {
  std::vector<std::vector<QRNodeDev>> levels;  // per level, all trees concatenated
  std::vector<std::vector<int>> nmat;          // per level, the matrix of every node
  std::vector<int> top_level, top_index;       // per matrix
  std::vector<int> kmat;                       // per matrix
  size_t store_elems = 0;
  int ab_elems = 0;
};

static size_t tree_nodes(const TreeBuild& tb) {
  size_t n = 0;
  for (const auto& lv : tb.levels) n += lv.size();
  return n;
}

// Builds TSQR trees for a list of tall matrices given by their level-0 sources.
// The nodes of every level are laid out matrix by matrix in the order `ord`
// (all matrices in index order when it is empty).
static void build_trees(const std::vector<QRNodeDev>& mats, const std::vector<int64_t>& rows,
                        TreeBuild& tb, const std::vector<int>& ord = {}) {
  const int MC = 256;
  const size_t nm = mats.size();
  tb.top_level.assign(nm, -1);
  tb.top_index.assign(nm, -1);
  tb.kmat.assign(nm, 0);
  std::vector<int> seq(ord);
  if (seq.empty())
    for (size_t a = 0; a < nm; ++a) seq.push_back((int)a);
  // a matrix's nodes are contiguous on every level: first index and count
  std::vector<int> first(nm, 0), count(nm, 0);
  tb.levels.clear();
  tb.levels.emplace_back();
  tb.nmat.clear();
  tb.nmat.emplace_back();
  size_t n0 = 0;
  for (const int a : seq)
    if (mats[a].k > 0 && rows[a] > 0) n0 += (size_t)((rows[a] + MC - 1) / MC);
  tb.levels[0].reserve(n0);
  tb.nmat[0].reserve(n0);
  for (const int a : seq) {
    const int k = mats[a].k;
    tb.kmat[a] = k;
    if (k == 0 || rows[a] == 0) continue;
    first[a] = (int)tb.levels[0].size();
    for (int64_t r0 = 0; r0 < rows[a]; r0 += MC) {
      QRNodeDev nd = mats[a];
      nd.row0 = mats[a].row0 + r0;
      nd.rows = (int)std::min<int64_t>(MC, rows[a] - r0);
      nd.steps = std::min(nd.rows, k);
      nd.level0 = 1;
      nd.store = (int64_t)tb.store_elems;
      tb.store_elems += (size_t)MC * k;
      nd.ab = tb.ab_elems;
      tb.ab_elems += k;
      tb.levels[0].push_back(nd);
      tb.nmat[0].push_back(a);
      ++count[a];
    }
  }
  int lev = 0;
  while (true) {
    bool any = false;
    std::vector<QRNodeDev> next;
    std::vector<int> next_mat;
    const std::vector<QRNodeDev>& below = tb.levels[lev];
    for (const int a : seq) {
      if (count[a] == 0) continue;
      if (count[a] == 1) {
        if (tb.top_level[a] < 0) {
          tb.top_level[a] = lev;
          tb.top_index[a] = first[a];
        }
        count[a] = 0;
        continue;
      }
      any = true;
      const int k = tb.kmat[a];
      const int g = std::max(2, MC / k);
      const int nfirst = (int)next.size();
      int ncount = 0;
      for (int c0 = 0; c0 < count[a]; c0 += g) {
        const int nc = std::min(g, count[a] - c0);
        int rws = 0;
        for (int c = 0; c < nc; ++c) rws += below[first[a] + c0 + c].steps;
        QRNodeDev nd{};
        nd.rows = rws;
        nd.k = k;
        nd.steps = std::min(rws, k);
        nd.level0 = 0;
        nd.child0 = first[a] + c0;
        nd.nchild = nc;
        nd.store = (int64_t)tb.store_elems;
        tb.store_elems += (size_t)MC * k;
        nd.ab = tb.ab_elems;
        tb.ab_elems += k;
        next.push_back(nd);
        next_mat.push_back(a);
        ++ncount;
      }
      first[a] = nfirst;
      count[a] = ncount;
    }
    if (!any) break;
    tb.levels.push_back(std::move(next));
    tb.nmat.push_back(std::move(next_mat));
    ++lev;
  }
}

// Device time per kernel class of one call: HIP event pairs recorded on the
// call's stream around each launch of the class, read after the call's last
// synchronisation.  Events come from a process-wide pool, so a call creates
// none after the first few.
class EventPool {
 public:
  static EventPool& get() {
    static EventPool p;
    return p;
  }
  hipEvent_t take() {
    std::lock_guard<std::mutex> g(mu_);
    if (!free_.empty()) {
      hipEvent_t e = free_.back();
      free_.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }
  void give(hipEvent_t e) {
    if (!e) return;
    std::lock_guard<std::mutex> g(mu_);
    free_.push_back(e);
  }

 private:
  std::mutex mu_;
  std::vector<hipEvent_t> free_;
};

enum KClass { KC_SVD = 0, KC_QR = 1, KC_GEMM = 2, KC_N = 3 };

struct KernelClock {
  struct Span {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Span> spans;
  hipEvent_t begin(hipStream_t st) {
    hipEvent_t e = EventPool::get().take();
    if (e) (void)hipEventRecord(e, st);
    return e;
  }
  void end(int cls, hipEvent_t a, hipStream_t st) {
    hipEvent_t b = EventPool::get().take();
    if (b) (void)hipEventRecord(b, st);
    spans.push_back(Span{cls, a, b});
  }
  // after the stream has been synchronised
  void totals(double* ms, int* launches) {
    for (const Span& s : spans) {
      if (s.a && s.b) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, s.a, s.b) == hipSuccess) ms[s.cls] += t;
        else (void)hipGetLastError();
      }
      launches[s.cls] += 1;
    }
  }
  ~KernelClock() {
    for (const Span& s : spans) {
      EventPool::get().give(s.a);
      EventPool::get().give(s.b);
    }
  }
};

struct Engine {
  hipStream_t st;
  int scalar;
  double eps;
  DevMem& tmp;

  int panel = 0;        // merge panel width (0: the TSQR tile)
  int svd_sweeps_max = 0;
  int svd_storage = 0;  // forced SVD storage mode (diagnostics)
  double svd_flops = 0.0;  // algorithmic flops of the small SVDs run so far
  KernelClock clock;

  Engine(hipStream_t s, int sc, double e, DevMem& t) : st(s), scalar(sc), eps(e), tmp(t) {}

  int kcap() const { return panel > 0 ? panel : (scalar == 0 ? 128 : 64); }

  size_t sb() const { return scalar_bytes(scalar); }

  // Factor trees; returns device copies of each level's nodes.
  struct Factored {
    TreeBuild tb;
    std::vector<QRNodeDev*> dlev;
    // owner matrix of every node, offsets of the trailing rows, first chunk row
    // of every matrix: the tree walks of the applies, done once (walk())
    mutable std::vector<std::vector<int>> owner;
    mutable std::vector<std::vector<int64_t>> tofs;
    mutable std::vector<int64_t> first_row;
    void* store = nullptr;
    void* alpha = nullptr;
    double* beta = nullptr;
  };

  // With a batch, the launches join it (issued by its run()); without, they
  // are issued here.
  void factor(const std::vector<QRNodeDev>& mats, const std::vector<int64_t>& rows, Factored& F,
              Batch* batch = nullptr) {
    // Every matrix takes the narrowest register tile that holds its width:
    // the trees are laid out narrowest class first, and a large level is
    // launched once per class over its run of nodes (a batch of mostly
    // narrow matrices with a few wider ones keeps the narrow tile for most).
    const size_t nm = mats.size();
    std::vector<int> kvm(nm, 0), ord(nm);
    for (size_t a = 0; a < nm; ++a) {
      ord[a] = (int)a;
      if (mats[a].k == 0) continue;
      kvm[a] = hbk::tsqr_kmax_for(scalar, mats[a].k);
      if (kvm[a] < 0) throw HbError{HB_EUNSUPPORTED};
    }
    {
      // stable counting sort by width class (0, 16, 32, 64, 128 columns)
      auto cls = [](int kv) { return kv == 0 ? 0 : kv == 16 ? 1 : kv == 32 ? 2 : kv == 64 ? 3 : 4; };
      size_t start[6] = {0, 0, 0, 0, 0, 0};
      for (size_t a = 0; a < nm; ++a) ++start[cls(kvm[a]) + 1];
      for (int c = 0; c < 5; ++c) start[c + 1] += start[c];
      for (size_t a = 0; a < nm; ++a) ord[start[cls(kvm[a])]++] = (int)a;
    }
    build_trees(mats, rows, F.tb, ord);
    struct Seg {
      int level, first, count, kv;
    };
    // A level with fewer nodes than the device has CUs is one launch at the
    // widest tile of the level: its launches would run one after another,
    // each as long as its slowest node.
    std::vector<Seg> segs;
    for (size_t l = 0; l < F.tb.levels.size(); ++l) {
      const std::vector<int>& nmat = F.tb.nmat[l];
      if (nmat.size() < kSplitNodes) {
        int kvl = 0;
        for (int a : nmat) kvl = std::max(kvl, kvm[a]);
        if (!nmat.empty()) segs.push_back(Seg{(int)l, 0, (int)nmat.size(), kvl});
        continue;
      }
      for (size_t i = 0; i < nmat.size();) {
        size_t j = i + 1;
        while (j < nmat.size() && kvm[nmat[j]] == kvm[nmat[i]]) ++j;
        segs.push_back(Seg{(int)l, (int)i, (int)(j - i), kvm[nmat[i]]});
        i = j;
      }
    }
    F.store = tmp.alloc(std::max<size_t>(F.tb.store_elems, 1) * sb());
    F.alpha = tmp.alloc(std::max(F.tb.ab_elems, 1) * sb());
    F.beta = tmp.get<double>(std::max(F.tb.ab_elems, 1));
    Batch local;
    Batch& B = batch ? *batch : local;
    std::vector<size_t> off;
    for (auto& lv : F.tb.levels) off.push_back(B.add(lv));
    B.then([this, &F, &B, off, segs]() {
      F.dlev.clear();
      for (size_t o : off) F.dlev.push_back(B.at<QRNodeDev>(o));
      hipEvent_t t0 = clock.begin(st);
      for (const Seg& g : segs) {
        const int l = g.level;
        HB_LAUNCH(hbk::tsqr_factor_launch(scalar, g.kv, F.dlev[l] + g.first, g.count,
                                          l ? F.dlev[l - 1] : nullptr, F.store, F.alpha, F.beta,
                                          st));
      }
      clock.end(KC_QR, t0, st);
    });
    if (!batch) local.run(tmp, st);
  }

  // Zout(matrix a) = Q_a [Zin_a; 0]  (Zin_a: steps_top x r_a, ld ldin_a;
  // Zout_a: rows_a x r_a, ld ldout_a)
  // Q Z for any number of columns: groups of at most kcap columns
  // Q Z for any number of columns: groups of at most kcap columns.  With
  // `ztr`, rows beyond each node's steps come from the trailing block
  // (rows - steps_top rows, ld ldtr) instead of zeros.
  void apply(const Factored& F, const std::vector<const void*>& zin, const std::vector<int64_t>& ldin,
             const std::vector<int>& rr, const std::vector<void*>& zout,
             const std::vector<int64_t>& ldout, const std::vector<const void*>* ztr = nullptr,
             const std::vector<int64_t>* ldtr = nullptr, Batch* batch = nullptr) {
    const int kcap = scalar == 0 ? 128 : 64;
    int rmax = 0;
    for (int r : rr) rmax = std::max(rmax, r);
    if (rmax <= kcap) {
      apply_cols(F, zin, ldin, rr, zout, ldout, ztr, ldtr, batch);
      return;
    }
    for (int c0 = 0; c0 < rmax; c0 += kcap) {
      std::vector<const void*> zi(zin.size(), nullptr), zt(zin.size(), nullptr);
      std::vector<void*> zo(zout.size(), nullptr);
      std::vector<int> rc(rr.size(), 0);
      for (size_t a = 0; a < rr.size(); ++a) {
        rc[a] = std::max(0, std::min(kcap, rr[a] - c0));
        if (rc[a] == 0) continue;
        zi[a] = (const char*)zin[a] + (size_t)c0 * ldin[a] * sb();
        zo[a] = (char*)zout[a] + (size_t)c0 * ldout[a] * sb();
        if (ztr && (*ztr)[a]) zt[a] = (const char*)(*ztr)[a] + (size_t)c0 * (*ldtr)[a] * sb();
      }
      apply_cols(F, zi, ldin, rc, zo, ldout, ztr ? &zt : nullptr, ldtr, batch);
    }
  }

  // the tree walks the applies need (host only; once per factorisation)
  static void walk(const Factored& F) {
    if (!F.owner.empty() || F.tb.levels.empty()) return;
    F.owner = owners(F.tb);
    F.tofs = trailing_offsets(F.tb, F.owner);
    F.first_row.assign(F.tb.kmat.size(), -1);
    for (size_t id = 0; id < F.tb.levels[0].size(); ++id) {
      const int a = F.owner[0][id];
      if (a >= 0 && F.first_row[a] < 0) F.first_row[a] = F.tb.levels[0][id].row0;
    }
  }

  // per node: offset of its trailing rows in the matrix's trailing block
  static std::vector<std::vector<int64_t>> trailing_offsets(const TreeBuild& tb,
                                                            const std::vector<std::vector<int>>& owner) {
    const int nlev = (int)tb.levels.size();
    std::vector<std::vector<int64_t>> off(nlev);
    std::vector<int64_t> cur(tb.kmat.size(), 0);
    for (int l = 0; l < nlev; ++l) {
      off[l].assign(tb.levels[l].size(), 0);
      for (size_t id = 0; id < tb.levels[l].size(); ++id) {
        const int a = owner[l][id];
        if (a < 0) continue;
        off[l][id] = cur[a];
        cur[a] += tb.levels[l][id].rows - tb.levels[l][id].steps;
      }
    }
    return off;
  }

  static std::vector<std::vector<int>> owners(const TreeBuild& tb) {
    const int nlev = (int)tb.levels.size();
    std::vector<std::vector<int>> owner(nlev);
    for (int l = 0; l < nlev; ++l) owner[l].assign(tb.levels[l].size(), -1);
    for (size_t a = 0; a < tb.kmat.size(); ++a) {
      if (tb.top_level[a] < 0) continue;
      std::vector<int> cur{tb.top_index[a]};
      for (int l = tb.top_level[a]; l >= 0; --l) {
        std::vector<int> nx;
        for (int id : cur) {
          owner[l][id] = (int)a;
          if (l > 0)
            for (int c = 0; c < tb.levels[l][id].nchild; ++c) nx.push_back(tb.levels[l][id].child0 + c);
        }
        cur = nx;
      }
    }
    return owner;
  }

  // Q^H Z bottom-up through every tree: Z (rows_a x kk_a, ld ldin) -> the top
  // node's first steps rows into top (ld ldtop) and the remaining rows into
  // the trailing block trail (rows_a - steps_top rows, ld ldtrail).
  void apply_h(const Factored& F, const std::vector<const void*>& zin,
               const std::vector<int64_t>& ldin, const std::vector<int>& kk,
               const std::vector<void*>& top, const std::vector<int64_t>& ldtop,
               const std::vector<void*>& trail, const std::vector<int64_t>& ldtrail,
               Batch* batch = nullptr) {
    const auto& tb = F.tb;
    const int nlev = (int)tb.levels.size();
    const size_t nm = tb.kmat.size();
    int kmx = 1;
    for (size_t a = 0; a < nm; ++a) kmx = std::max(kmx, kk[a]);
    const int kv = hbk::tsqr_kmax_for(scalar, kmx);
    if (kv < 0) throw HbError{HB_EUNSUPPORTED};
    walk(F);
    const auto& owner = F.owner;
    const auto& toff = F.tofs;
    // stacked input buffers of levels >= 1
    std::vector<std::vector<char*>> sbuf(nlev);
    for (int l = 1; l < nlev; ++l) {
      std::vector<size_t> sz;
      for (size_t id = 0; id < tb.levels[l].size(); ++id) {
        const int a = owner[l][id];
        sz.push_back(a < 0 ? 0 : (size_t)tb.levels[l][id].rows * kk[a] * sb());
      }
      sbuf[l] = tmp.carve(sz);
    }
    // parent of every node and the child's row offset in the parent's stack
    std::vector<std::vector<int>> par(nlev), poff(nlev);
    for (int l = 0; l < nlev; ++l) {
      par[l].assign(tb.levels[l].size(), -1);
      poff[l].assign(tb.levels[l].size(), 0);
    }
    for (int l = 1; l < nlev; ++l)
      for (size_t id = 0; id < tb.levels[l].size(); ++id) {
        int off = 0;
        const QRNodeDev& nd = tb.levels[l][id];
        for (int c = 0; c < nd.nchild; ++c) {
          par[l - 1][nd.child0 + c] = (int)id;
          poff[l - 1][nd.child0 + c] = off;
          off += tb.levels[l - 1][nd.child0 + c].steps;
        }
      }
    const auto& first_row = F.first_row;
    const bool stream = tree_nodes(tb) > kApplyBatchNodes;
    Batch local;
    Batch& B = batch && !stream ? *batch : local;
    std::vector<std::pair<size_t, int>> lv;  // (descriptor offset, jobs) per level
    for (int l = 0; l < nlev; ++l) {
      std::vector<QRApplyHDev> jobs;
      for (size_t id = 0; id < tb.levels[l].size(); ++id) {
        const int a = owner[l][id];
        if (a < 0 || kk[a] == 0) continue;
        const QRNodeDev& nd = tb.levels[l][id];
        QRApplyHDev J{};
        J.rows = nd.rows;
        J.steps = nd.steps;
        J.r = kk[a];
        J.store = nd.store;
        J.ab = nd.ab;
        if (l == 0) {
          J.Zin = (const char*)zin[a] + (size_t)(nd.row0 - first_row[a]) * sb();
          J.ldin = ldin[a];
        } else {
          J.Zin = sbuf[l][id];
          J.ldin = nd.rows;
        }
        const bool is_top = (l == tb.top_level[a] && (int)id == tb.top_index[a]);
        if (is_top) {
          J.Zup = top[a];
          J.ldup = ldtop[a];
        } else {
          const int pid = par[l][id];
          J.Zup = sbuf[l + 1][pid] + (size_t)poff[l][id] * sb();
          J.ldup = tb.levels[l + 1][pid].rows;
        }
        J.Ztr = (char*)trail[a] + (size_t)toff[l][id] * sb();
        J.ldtr = ldtrail[a];
        jobs.push_back(J);
      }
      if (jobs.empty()) continue;
      if (stream) {
        QRApplyHDev* dj = upload(tmp, jobs, st);
        hipEvent_t t0 = clock.begin(st);
        HB_LAUNCH(hbk::tsqr_applyh_launch(scalar, kv, dj, (int)jobs.size(), F.store, F.beta, st));
        clock.end(KC_QR, t0, st);
      } else {
        lv.emplace_back(B.add(jobs), (int)jobs.size());
      }
    }
    if (!lv.empty())
      B.then([this, &F, &B, lv, kv]() {
        hipEvent_t t0 = clock.begin(st);
        for (const auto& e : lv)
          HB_LAUNCH(hbk::tsqr_applyh_launch(scalar, kv, B.at<QRApplyHDev>(e.first), e.second,
                                            F.store, F.beta, st));
        clock.end(KC_QR, t0, st);
      });
    if (&B == &local) local.run(tmp, st);
  }

  void apply_cols(const Factored& F, const std::vector<const void*>& zin,
                  const std::vector<int64_t>& ldin, const std::vector<int>& rr,
                  const std::vector<void*>& zout, const std::vector<int64_t>& ldout,
                  const std::vector<const void*>* ztr, const std::vector<int64_t>* ldtr,
                  Batch* batch) {
    const auto& tb = F.tb;
    const int nlev = (int)tb.levels.size();
    const size_t nm = tb.kmat.size();
    int rmax = 1;
    for (size_t a = 0; a < nm; ++a) rmax = std::max(rmax, rr[a]);
    const int kv = hbk::tsqr_kmax_for(scalar, rmax);
    if (kv < 0) throw HbError{HB_EUNSUPPORTED};
    // node -> matrix, then the input/output of every node, top down
    walk(F);
    const auto& owner = F.owner;
    const auto& tofs = F.tofs;
    const bool stream = tree_nodes(tb) > kApplyBatchNodes;
    Batch local;
    Batch& B = batch && !stream ? *batch : local;
    std::vector<std::pair<size_t, int>> lv;  // (descriptor offset, jobs) per level
    // per node Zin pointer/ld and Zout pointer/ld
    std::vector<std::vector<const void*>> nin(nlev);
    std::vector<std::vector<int64_t>> nldin(nlev);
    for (int l = 0; l < nlev; ++l) {
      nin[l].assign(tb.levels[l].size(), nullptr);
      nldin[l].assign(tb.levels[l].size(), 0);
    }
    for (size_t a = 0; a < nm; ++a)
      if (tb.top_level[a] >= 0 && rr[a] > 0) {
        nin[tb.top_level[a]][tb.top_index[a]] = zin[a];
        nldin[tb.top_level[a]][tb.top_index[a]] = ldin[a];
      }
    for (int l = nlev - 1; l >= 0; --l) {
      std::vector<QRApplyDev> jobs;
      std::vector<char*> lbuf;
      if (l > 0) {
        std::vector<size_t> sz;
        for (size_t id = 0; id < tb.levels[l].size(); ++id) {
          const int a = owner[l][id];
          sz.push_back((a < 0 || rr[a] == 0) ? 0 : (size_t)tb.levels[l][id].rows * rr[a] * sb());
        }
        lbuf = tmp.carve(sz);
      }
      for (size_t id = 0; id < tb.levels[l].size(); ++id) {
        const int a = owner[l][id];
        if (a < 0 || rr[a] == 0) continue;
        const QRNodeDev& nd = tb.levels[l][id];
        QRApplyDev J{};
        J.rows = nd.rows;
        J.steps = nd.steps;
        J.r = rr[a];
        J.store = nd.store;
        J.ab = nd.ab;
        J.Zin = nin[l][id];
        J.ldin = nldin[l][id];
        if (ztr && (*ztr)[a]) {
          J.Ztr = (const char*)(*ztr)[a] + (size_t)tofs[l][id] * sb();
          J.ldtr = (*ldtr)[a];
        }
        if (l == 0) {
          // rows [row0 - base, ...) of the destination
          const int64_t base = tb.levels[0][id].row0;  // absolute row in the source
          (void)base;
          J.Zout = (char*)zout[a] + 0;  // patched below with the chunk offset
          J.ldout = ldout[a];
        } else {
          void* buf = lbuf[id];
          J.Zout = buf;
          J.ldout = nd.rows;
          int off = 0;
          for (int c = 0; c < nd.nchild; ++c) {
            const int cid = nd.child0 + c;
            nin[l - 1][cid] = (const char*)buf + (size_t)off * sb();
            nldin[l - 1][cid] = nd.rows;
            off += tb.levels[l - 1][cid].steps;
          }
        }
        jobs.push_back(J);
      }
      if (l == 0) {
        // level-0 chunks write rows [chunk offset, ...) of their matrix
        size_t j = 0;
        for (size_t id = 0; id < tb.levels[0].size(); ++id) {
          const int a = owner[0][id];
          if (a < 0 || rr[a] == 0) continue;
          const int64_t off = tb.levels[0][id].row0 - F.first_row[a];
          jobs[j].Zout = (char*)zout[a] + (size_t)off * sb();
          ++j;
        }
      }
      if (jobs.empty()) continue;
      if (stream) {
        QRApplyDev* dj = upload(tmp, jobs, st);
        hipEvent_t t0 = clock.begin(st);
        HB_LAUNCH(hbk::tsqr_apply_launch(scalar, kv, dj, (int)jobs.size(), F.store, F.beta, st));
        clock.end(KC_QR, t0, st);
      } else {
        lv.emplace_back(B.add(jobs), (int)jobs.size());
      }
    }
    if (!lv.empty())
      B.then([this, &F, &B, lv, kv]() {
        hipEvent_t t0 = clock.begin(st);
        for (const auto& e : lv)
          HB_LAUNCH(hbk::tsqr_apply_launch(scalar, kv, B.at<QRApplyDev>(e.first), e.second,
                                           F.store, F.beta, st));
        clock.end(KC_QR, t0, st);
      });
    if (&B == &local) local.run(tmp, st);
  }
};

// Runs a batch of truncated SVDs of R matrices (explicit or TSQR tops).
struct SvdOut {
  void* Xr;
  void* Yr;
  double* S;
  int32_t* rank;
  int p, k;
};

// `batch` holds launches queued before the SVDs (they and the SVDs go out
// with one descriptor copy); `overlap` runs on the host while the device
// works, before the ranks are read back.
static void run_svds(Engine& E, std::vector<SVDJobDev>& jobs, const void* store, const void* alpha,
                     std::vector<SvdOut>& outs, std::vector<int>& ranks_host,
                     Batch* batch = nullptr, const std::function<void()>& overlap = nullptr) {
  const size_t nj = jobs.size();
  outs.assign(nj, SvdOut{});
  if (nj == 0) {
    if (batch) batch->run(E.tmp, E.st);
    if (overlap) overlap();
    ranks_host.clear();
    return;
  }
  int32_t* dr = E.tmp.get<int32_t>(2 * nj);
  int kmax = 0, pmax = 0;
  std::vector<size_t> sz;
  for (size_t a = 0; a < nj; ++a) {
    const size_t p = jobs[a].p, k = jobs[a].k;
    kmax = std::max(kmax, (int)k);
    pmax = std::max(pmax, (int)p);
    sz.push_back(p * k * E.sb());   // HBM workspace (R^H when it exceeds LDS)
    sz.push_back(k * 8);
    sz.push_back(k * 4);
    sz.push_back(p * k * E.sb());
    sz.push_back(k * k * E.sb());
    sz.push_back(p * k * E.sb());   // HBM workspace (R2^H)
    sz.push_back(p * 4);            // preconditioner row permutation
  }
  std::vector<char*> bufs = E.tmp.carve(sz);
  for (size_t a = 0; a < nj; ++a) {
    SVDJobDev& J = jobs[a];
    J.A = bufs[7 * a + 0];
    J.S = (double*)bufs[7 * a + 1];
    J.perm = (int32_t*)bufs[7 * a + 2];
    J.rank = dr + 2 * a;
    J.Xr = bufs[7 * a + 3];
    J.Yr = bufs[7 * a + 4];
    J.W = bufs[7 * a + 5];
    J.cperm = (int32_t*)bufs[7 * a + 6];
    outs[a] = SvdOut{J.Xr, J.Yr, J.S, J.rank, J.p, J.k};
  }
  Batch local;
  Batch& B = batch ? *batch : local;
  const size_t joff = B.add(jobs);
  // The multi-workgroup SVD takes batches of a few wide matrices (the top
  // merge levels), where one workgroup per matrix runs about k / 32 pairs
  // after one another in every round and leaves most of the chip idle: B
  // workgroups per matrix, when every matrix suits it (p >= k, p <= 512)
  // and the batch is small.  Storage mode 3 forces it wherever the shape
  // allows; 1 and 2 keep one workgroup per matrix.
  int wideB = 0;
  if (E.svd_storage == 0 || E.svd_storage == 3) {
    for (size_t a = 0; a < nj; ++a) {
      const int b = hbk::svd_wide_blocks(E.scalar, jobs[a].p, jobs[a].k);
      if (b == 0) {
        wideB = 0;
        break;
      }
      wideB = std::max(wideB, b);
    }
    // automatic: matrices wider than 160 columns, or batches of one or two
    // (the top merges) of at least 64 columns, and at most 256 workgroups.
    // Measured: below 160 columns several workgroups lose to one when the
    // batch has four or more matrices, and win for one or two (Gauss 3-D
    // 2000^2: small-SVD time 16.2 -> 13.2 ms; Helmholtz 20000^2: 6.9 -> 6.5).
    if (E.svd_storage == 0 &&
        ((int64_t)nj * wideB > 256 || (kmax <= 160 && !(nj <= 2 && kmax >= 64))))
      wideB = 0;
    if (wideB > 0 && !hbk::svd_wide_fits(E.scalar, (int)nj, wideB, pmax)) wideB = 0;
    if (g_coop_refused.load(std::memory_order_relaxed)) wideB = 0;
  }
  const int storage = E.svd_storage == 3 ? 2 : E.svd_storage;
  B.then([&]() {
  SVDJobDev* dj = B.at<SVDJobDev>(joff);
  hipEvent_t t0 = E.clock.begin(E.st);
  if (wideB > 0) {
    // the preconditioner on one workgroup per matrix, then the sweeps on B
    void* work = E.tmp.alloc(hbk::svd_wide_work_bytes((int)nj, wideB));
    HB_LAUNCH(hbk::svd_launch(E.scalar, dj, (int)nj, kmax, pmax, store, alpha, E.eps, E.st,
                              storage, true));
    const int we = hbk::svd_wide_launch(E.scalar, dj, (int)nj, wideB, pmax, store, alpha, E.eps,
                                        work, E.st);
    if (we != 0) {
      // The runtime can refuse a cooperative launch that fits (error 401 was
      // seen while another process on the device had made cooperative
      // launches). The preconditioner read the inputs only, so the
      // one-workgroup SVD starts over from them; the process keeps to it.
      hb_report("cooperative SVD launch (falling back to one workgroup per matrix)", we,
                we > 0 ? hipGetErrorString((hipError_t)we) : "grid does not fit", __LINE__);
      (void)hipGetLastError();
      g_coop_refused.store(true, std::memory_order_relaxed);
      HB_LAUNCH(hbk::svd_launch(E.scalar, dj, (int)nj, kmax, pmax, store, alpha, E.eps, E.st,
                                storage));
    }
  } else {
    HB_LAUNCH(hbk::svd_launch(E.scalar, dj, (int)nj, kmax, pmax, store, alpha, E.eps, E.st,
                              storage));
  }
  E.clock.end(KC_SVD, t0, E.st);
  });
  B.run(E.tmp, E.st);
  if (overlap) overlap();
  std::vector<int32_t> rh(2 * nj);
  d2h_sync(rh.data(), dr, 2 * nj * sizeof(int32_t), E.st);
  ranks_host.resize(nj);
  // algorithmic flops: QRCP of R^H (4 phi p k q) and per Jacobi sweep
  // q (q - 1) / 2 pairs, each a dot product and a rotation of two length-p
  // columns (8 phi p); q = min(p, k)
  const double phi = E.scalar ? 4.0 : 1.0;
  for (size_t a = 0; a < nj; ++a) {
    ranks_host[a] = rh[2 * a];
    E.svd_sweeps_max = std::max(E.svd_sweeps_max, (int)rh[2 * a + 1]);
    const double p = jobs[a].p, k = jobs[a].k, q = std::min(p, k);
    E.svd_flops += phi * (4.0 * p * k * q + (double)rh[2 * a + 1] * 4.0 * p * q * (q - 1.0));
  }
}

static void copy_sigmas(Engine& E, const std::vector<CopyDev>& cp, Batch* batch = nullptr) {
  if (cp.empty()) return;
  Batch local;
  Batch& B = batch ? *batch : local;
  const size_t off = B.add(cp);
  const int n = (int)cp.size();
  B.then([&E, &B, off, n]() { HB_LAUNCH(hbk::copy_list_launch(B.at<CopyDev>(off), n, E.st)); });
  if (!batch) local.run(E.tmp, E.st);
}

// Truncated SVD of the horizontal (p_is_u) or vertical concatenation of two
// blocks, for a batch of pairs.  Results are allocated in `out_mem`.
static void run_merges_direct(Engine& E, std::vector<MergeJob>& jobs, DevMem& out_mem) {
  const size_t nj = jobs.size();
  std::vector<QRNodeDev> mats;
  std::vector<int64_t> rows;
  std::vector<size_t> midx(nj, (size_t)-1);
  for (size_t a = 0; a < nj; ++a) {
    MergeJob& J = jobs[a];
    Block& B = *J.outP_owner;
    const int k = J.r1 + J.r2;
    if (J.p_is_u) {
      B.m = J.rows;
      B.n = J.n1 + J.n2;
    } else {
      B.n = J.rows;
      B.m = J.n1 + J.n2;
    }
    B.r = 0;
    if (k == 0) continue;
    QRNodeDev nd{};
    nd.k = k;
    nd.P1 = J.P1; nd.ld1 = J.rows; nd.n1 = J.r1; nd.S1 = J.S1;
    nd.P2 = J.P2; nd.ld2 = J.rows; nd.n2 = J.r2; nd.S2 = J.S2;
    nd.row0 = 0;
    midx[a] = mats.size();
    mats.push_back(nd);
    rows.push_back(J.rows);
  }
  Engine::Factored F;
  E.factor(mats, rows, F);  // at once: the device factors while the host plans the SVDs
  Batch pre;
  std::vector<SVDJobDev> sj;
  for (size_t a = 0; a < mats.size(); ++a) {
    const QRNodeDev& top = F.tb.levels[F.tb.top_level[a]][F.tb.top_index[a]];
    SVDJobDev J{};
    J.p = top.steps;
    J.k = top.k;
    J.from_node = 1;
    J.store = top.store;
    J.ab = top.ab;
    sj.push_back(J);
  }
  std::vector<SvdOut> so;
  std::vector<int> rk;
  run_svds(E, sj, F.store, F.alpha, so, rk, &pre, [&F]() { Engine::walk(F); });
  // allocate outputs
  std::vector<const void*> zin;
  std::vector<int64_t> ldin, ldout;
  std::vector<int> rr;
  std::vector<void*> zout;
  std::vector<BlockGemmDev> gj;
  int64_t max_rows = 0;
  int max_rin = 0;
  std::vector<size_t> osz;
  for (size_t a = 0; a < nj; ++a) {
    MergeJob& J = jobs[a];
    const int r = midx[a] == (size_t)-1 ? 0 : rk[midx[a]];
    osz.push_back((size_t)J.rows * r * E.sb());
    osz.push_back((size_t)(J.n1 + J.n2) * r * E.sb());
    osz.push_back((size_t)r * 8);
  }
  std::vector<char*> ob = out_mem.carve(osz);
  std::vector<CopyDev> scp;
  for (size_t a = 0; a < nj; ++a) {
    MergeJob& J = jobs[a];
    Block& B = *J.outP_owner;
    if (midx[a] == (size_t)-1) continue;
    const size_t i = midx[a];
    const int r = rk[i];
    B.r = r;
    if (r == 0) continue;
    const int64_t prow = J.rows, orow = J.n1 + J.n2;
    void* P = ob[3 * a];
    void* O = ob[3 * a + 1];
    B.S = (double*)ob[3 * a + 2];
    scp.push_back(CopyDev{so[i].S, B.S, (int64_t)r * 8});
    if (J.p_is_u) {
      B.U = P;
      B.Vh = O;
    } else {
      B.Vh = P;
      B.U = O;
    }
    zin.push_back(so[i].Xr);
    ldin.push_back(so[i].p);
    rr.push_back(r);
    zout.push_back(P);
    ldout.push_back(prow);
    BlockGemmDev g{};
    g.A1 = J.O1; g.lda1 = J.n1; g.n1 = (int)J.n1; g.r1 = J.r1;
    g.A2 = J.O2; g.lda2 = J.n2; g.n2 = (int)J.n2; g.r2 = J.r2;
    g.Y = so[i].Yr; g.ldy = so[i].k; g.r = r;
    g.C = O; g.ldc = orow;
    gj.push_back(g);
    max_rows = std::max(max_rows, orow);
    max_rin = std::max(max_rin, J.r1 + J.r2);
  }
  // Q [X_r; 0] for every matrix with a nonzero rank (zeros for rank 0 are skipped)
  std::vector<int> rr_all(mats.size(), 0);
  std::vector<const void*> zin_all(mats.size(), nullptr);
  std::vector<int64_t> ldin_all(mats.size(), 1), ldout_all(mats.size(), 1);
  std::vector<void*> zout_all(mats.size(), nullptr);
  {
    size_t c = 0;
    for (size_t a = 0; a < nj; ++a) {
      if (midx[a] == (size_t)-1) continue;
      const size_t i = midx[a];
      if (rk[i] == 0) continue;
      rr_all[i] = rr[c];
      zin_all[i] = zin[c];
      ldin_all[i] = ldin[c];
      zout_all[i] = zout[c];
      ldout_all[i] = ldout[c];
      ++c;
    }
  }
  Batch post;
  copy_sigmas(E, scp, &post);
  E.apply(F, zin_all, ldin_all, rr_all, zout_all, ldout_all, nullptr, nullptr, &post);
  if (!gj.empty()) {
    const size_t goff = post.add(gj);
    const int ng = (int)gj.size();
    post.then([&]() {
      hipEvent_t t0 = E.clock.begin(E.st);
      HB_LAUNCH(hbk::block_gemm_launch(E.scalar, post.at<BlockGemmDev>(goff), ng, (int)max_rows,
                                       max_rin, E.st));
      E.clock.end(KC_GEMM, t0, E.st);
    });
  }
  post.run(E.tmp, E.st);
}

// Householder QR of tall matrices wider than the register TSQR tile, by
// column panels (communication-avoiding QR).  Panel p is factored by TSQR;
// the Q^H of its tree is applied bottom-up to every later panel, whose top
// rows become the coupling block R_{p,j} and whose other rows form the next
// working matrix.  The inputs are only read.
struct PanelQR {
  size_t nj = 0;
  int kcap = 0, qmax = 0;
  std::vector<int> q, kk;
  std::vector<int64_t> rows;
  std::vector<std::vector<int64_t>> rows_at;  // working rows when panel p is factored
  std::vector<std::vector<int>> stepsp;       // R rows contributed by panel p
  std::vector<std::unique_ptr<Engine::Factored>> Fp;
  std::vector<std::vector<int>> midx;         // matrix index of job a in panel p's trees
  std::vector<int64_t> P;                     // rows of R (sum of the panel steps)
  std::vector<char*> R;                       // R compacted: P x k, column-major, ld P
  int pw(size_t a, int p) const { return std::min(kcap, kk[a] - p * kcap); }
};

// B_a: rows_a x k_a, column-major with ld rows_a.
static void panel_qr_factor(Engine& E, const std::vector<const void*>& B,
                            const std::vector<int64_t>& rows, const std::vector<int>& k,
                            PanelQR& S) {
  const size_t nj = B.size();
  const size_t sb = E.sb();
  S.nj = nj;
  S.kcap = E.kcap();
  S.kk = k;
  S.rows = rows;
  S.q.assign(nj, 0);
  S.qmax = 0;
  for (size_t a = 0; a < nj; ++a) {
    S.q[a] = (k[a] + S.kcap - 1) / S.kcap;
    S.qmax = std::max(S.qmax, S.q[a]);
  }
  S.rows_at.assign(nj, {});
  S.stepsp.assign(nj, {});
  S.Fp.clear();
  S.Fp.resize(S.qmax);
  S.midx.assign(S.qmax, std::vector<int>(nj, -1));
  std::vector<std::vector<const void*>> pin(nj);
  std::vector<int64_t> wrows(rows);
  for (size_t a = 0; a < nj; ++a) {
    pin[a].resize(S.q[a]);
    for (int p = 0; p < S.q[a]; ++p) pin[a][p] = (const char*)B[a] + (size_t)p * S.kcap * rows[a] * sb;
  }
  // R is written during the sweep at its upper bound (k x k, ld k) and
  // compacted to its P rows afterwards
  std::vector<size_t> rsz(nj);
  for (size_t a = 0; a < nj; ++a) rsz[a] = (size_t)k[a] * k[a] * sb;
  std::vector<char*> Rbuf = E.tmp.carve(rsz);
  {
    size_t tot = 0;
    for (size_t a = 0; a < nj; ++a) tot += (std::max<size_t>(rsz[a], 1) + 255) & ~(size_t)255;
    HB_LAUNCH(hbk::zero_fill_launch(Rbuf[0], tot, E.st));
  }
  std::vector<int64_t> roff(nj, 0);
  for (int p = 0; p < S.qmax; ++p) {
    std::vector<QRNodeDev> mats;
    std::vector<int64_t> mrows;
    for (size_t a = 0; a < nj; ++a) {
      if (p >= S.q[a]) continue;
      if (wrows[a] == 0) {  // no rows left: this panel adds no R rows
        S.rows_at[a].push_back(0);
        S.stepsp[a].push_back(0);
        continue;
      }
      QRNodeDev nd{};
      nd.k = S.pw(a, p);
      nd.P1 = pin[a][p];
      nd.ld1 = wrows[a];
      nd.n1 = nd.k;
      nd.P2 = pin[a][p];
      nd.ld2 = wrows[a];
      S.midx[p][a] = (int)mats.size();
      mats.push_back(nd);
      mrows.push_back(wrows[a]);
    }
    S.Fp[p].reset(new Engine::Factored());
    Engine::Factored& F = *S.Fp[p];
    if (mats.empty()) continue;
    E.factor(mats, mrows, F);
    // R_pp into R, coupling blocks of later panels, next working matrices
    std::vector<RCopyDev> rc;
    for (size_t a = 0; a < nj; ++a) {
      if (S.midx[p][a] < 0) continue;
      const int i = S.midx[p][a];
      const QRNodeDev& top = F.tb.levels[F.tb.top_level[i]][F.tb.top_index[i]];
      S.rows_at[a].push_back(wrows[a]);
      S.stepsp[a].push_back(top.steps);
      RCopyDev c{};
      c.store = top.store;
      c.ab = top.ab;
      c.p = top.steps;
      c.k = top.k;
      c.dst = Rbuf[a] + ((size_t)p * S.kcap * k[a] + roff[a]) * sb;
      c.ld = k[a];
      rc.push_back(c);
    }
    RCopyDev* drc = upload(E.tmp, rc, E.st);
    HB_LAUNCH(hbk::rcopy_launch(E.scalar, drc, (int)rc.size(), F.store, F.alpha, E.st));
    for (int j = p + 1; j < S.qmax; ++j) {
      std::vector<const void*> zin(mats.size(), nullptr);
      std::vector<int64_t> ldin(mats.size(), 1), ldtop(mats.size(), 1), ldtr(mats.size(), 1);
      std::vector<int> kj(mats.size(), 0);
      std::vector<void*> top(mats.size(), nullptr), trail(mats.size(), nullptr);
      std::vector<size_t> tsz(mats.size(), 0);
      std::vector<size_t> who;
      for (size_t a = 0; a < nj; ++a)
        if (S.midx[p][a] >= 0 && j < S.q[a]) who.push_back(a);
      if (who.empty()) continue;
      for (size_t a : who) {
        const int i = S.midx[p][a];
        tsz[i] = (size_t)(wrows[a] - S.stepsp[a][p]) * S.pw(a, j) * sb;
      }
      std::vector<char*> tb = E.tmp.carve(tsz);
      for (size_t a : who) {
        const int i = S.midx[p][a];
        kj[i] = S.pw(a, j);
        zin[i] = pin[a][j];
        ldin[i] = wrows[a];
        top[i] = Rbuf[a] + ((size_t)j * S.kcap * k[a] + roff[a]) * sb;
        ldtop[i] = k[a];
        trail[i] = tb[i];
        ldtr[i] = wrows[a] - S.stepsp[a][p];
      }
      E.apply_h(F, zin, ldin, kj, top, ldtop, trail, ldtr);
      for (size_t a : who) pin[a][j] = tb[S.midx[p][a]];
    }
    for (size_t a = 0; a < nj; ++a)
      if (S.midx[p][a] >= 0) {
        roff[a] += S.stepsp[a][p];
        wrows[a] -= S.stepsp[a][p];
      }
  }
  S.P = roff;
  std::vector<size_t> csz(nj);
  for (size_t a = 0; a < nj; ++a) csz[a] = (size_t)std::max<int64_t>(roff[a], 1) * k[a] * sb;
  S.R = E.tmp.carve(csz);
  std::vector<RCompactDev> rcj(nj);
  for (size_t a = 0; a < nj; ++a) rcj[a] = RCompactDev{Rbuf[a], k[a], S.R[a], (int)roff[a], k[a]};
  RCompactDev* drcj = upload(E.tmp, rcj, E.st);
  HB_LAUNCH(hbk::rcompact_launch(E.scalar, drcj, (int)nj, E.st));
}

// Zout_a (rows_a x r_a, ld rows_a) = Q_a [Zin_a; 0], Zin_a: P_a x r_a with
// leading dimension ldin_a.  Panel by panel from the last: Z_p = Q_p [rows
// of Zin for panel p; Z_{p+1}], the later panels' rows re-injected below.
static void panel_qr_apply(Engine& E, const PanelQR& S, const std::vector<const void*>& zin,
                           const std::vector<int64_t>& ldin, const std::vector<int>& rr,
                           const std::vector<void*>& zout) {
  const size_t nj = S.nj;
  const size_t sb = E.sb();
  std::vector<const void*> znext(nj, nullptr);
  std::vector<int64_t> ldnext(nj, 1);
  for (int p = S.qmax - 1; p >= 0; --p) {
    const Engine::Factored& F = *S.Fp[p];
    const size_t nm = F.tb.kmat.size();
    if (nm == 0) continue;
    std::vector<const void*> zi(nm, nullptr), ztr(nm, nullptr);
    std::vector<int64_t> li(nm, 1), lo(nm, 1), ltr(nm, 1);
    std::vector<int> rc(nm, 0);
    std::vector<void*> zo(nm, nullptr);
    std::vector<size_t> zsz(nm, 0);
    for (size_t a = 0; a < nj; ++a) {
      const int i = S.midx[p][a];
      if (i < 0 || rr[a] == 0) continue;
      if (p > 0) zsz[i] = (size_t)S.rows_at[a][p] * rr[a] * sb;
    }
    std::vector<char*> zb = E.tmp.carve(zsz);
    for (size_t a = 0; a < nj; ++a) {
      const int i = S.midx[p][a];
      if (i < 0 || rr[a] == 0) continue;
      int64_t r0 = 0;
      for (int pp = 0; pp < p; ++pp) r0 += S.stepsp[a][pp];
      rc[i] = rr[a];
      zi[i] = (const char*)zin[a] + (size_t)r0 * sb;
      li[i] = ldin[a];
      zo[i] = p == 0 ? zout[a] : (void*)zb[i];
      lo[i] = S.rows_at[a][p];
      if (p + 1 < S.q[a]) {
        ztr[i] = znext[a];
        ltr[i] = ldnext[a];
      }
    }
    E.apply(F, zi, li, rc, zo, lo, &ztr, &ltr);
    for (size_t a = 0; a < nj; ++a) {
      const int i = S.midx[p][a];
      if (i < 0 || rr[a] == 0) continue;
      znext[a] = zo[i];
      ldnext[a] = S.rows_at[a][p];
    }
  }
}

// Merges wider than the register TSQR tile: the panel QR of the materialised
// B = [P1 S1, P2 S2], the SVD of its R, Q [X_r; 0] and the block product on
// the other side.
static void run_merges_caqr(Engine& E, std::vector<MergeJob>& jobs, DevMem& out_mem) {
  const size_t nj = jobs.size();
  if (nj == 0) return;
  const size_t sb = E.sb();
  std::vector<int> kk(nj);
  std::vector<int64_t> rows(nj);
  for (size_t a = 0; a < nj; ++a) {
    MergeJob& J = jobs[a];
    Block& B = *J.outP_owner;
    if (J.p_is_u) {
      B.m = J.rows;
      B.n = J.n1 + J.n2;
    } else {
      B.n = J.rows;
      B.m = J.n1 + J.n2;
    }
    B.r = 0;
    kk[a] = J.r1 + J.r2;
    rows[a] = J.rows;
  }
  // materialised B = [P1 S1, P2 S2]
  std::vector<size_t> bsz(nj);
  for (size_t a = 0; a < nj; ++a) bsz[a] = (size_t)jobs[a].rows * kk[a] * sb;
  std::vector<char*> Bm = E.tmp.carve(bsz);
  {
    std::vector<ConcatDev> cj(nj);
    int64_t mm = 0;
    for (size_t a = 0; a < nj; ++a) {
      const MergeJob& J = jobs[a];
      cj[a] = ConcatDev{J.P1, J.P2, J.S1, J.S2, J.rows, J.r1, J.r2, Bm[a]};
      mm = std::max(mm, J.rows);
    }
    ConcatDev* d = upload(E.tmp, cj, E.st);
    HB_LAUNCH(hbk::concat_launch(E.scalar, d, (int)nj, mm, 0, E.st));
  }
  PanelQR S;
  panel_qr_factor(E, std::vector<const void*>(Bm.begin(), Bm.end()), rows, kk, S);
  std::vector<SVDJobDev> sj(nj);
  for (size_t a = 0; a < nj; ++a) {
    SVDJobDev J{};
    J.p = (int)S.P[a];
    J.k = kk[a];
    J.from_node = 0;
    J.R = S.R[a];
    sj[a] = J;
  }
  std::vector<SvdOut> so;
  std::vector<int> rk;
  run_svds(E, sj, nullptr, nullptr, so, rk);
  std::vector<size_t> osz;
  for (size_t a = 0; a < nj; ++a) {
    const int r = rk[a];
    osz.push_back((size_t)jobs[a].rows * r * sb);
    osz.push_back((size_t)(jobs[a].n1 + jobs[a].n2) * r * sb);
    osz.push_back((size_t)r * 8);
  }
  std::vector<char*> ob = out_mem.carve(osz);
  std::vector<BlockGemmDev> gj;
  int64_t max_rows = 0;
  int max_rin = 0;
  std::vector<const void*> zin(nj, nullptr);
  std::vector<int64_t> ldin(nj, 1);
  std::vector<int> rr(nj, 0);
  std::vector<void*> zout(nj, nullptr);
  std::vector<CopyDev> scp;
  for (size_t a = 0; a < nj; ++a) {
    MergeJob& J = jobs[a];
    Block& B = *J.outP_owner;
    const int r = rk[a];
    B.r = r;
    if (r == 0) continue;
    void* P = ob[3 * a];
    void* O = ob[3 * a + 1];
    B.S = (double*)ob[3 * a + 2];
    scp.push_back(CopyDev{so[a].S, B.S, (int64_t)r * 8});
    if (J.p_is_u) {
      B.U = P;
      B.Vh = O;
    } else {
      B.Vh = P;
      B.U = O;
    }
    zin[a] = so[a].Xr;
    ldin[a] = so[a].p;
    rr[a] = r;
    zout[a] = P;
    BlockGemmDev bg{};
    bg.A1 = J.O1; bg.lda1 = J.n1; bg.n1 = (int)J.n1; bg.r1 = J.r1;
    bg.A2 = J.O2; bg.lda2 = J.n2; bg.n2 = (int)J.n2; bg.r2 = J.r2;
    bg.Y = so[a].Yr; bg.ldy = so[a].k; bg.r = r;
    bg.C = O; bg.ldc = J.n1 + J.n2;
    gj.push_back(bg);
    max_rows = std::max<int64_t>(max_rows, J.n1 + J.n2);
    max_rin = std::max(max_rin, J.r1 + J.r2);
  }
  copy_sigmas(E, scp);
  panel_qr_apply(E, S, zin, ldin, rr, zout);
  if (!gj.empty()) {
    BlockGemmDev* dg = upload(E.tmp, gj, E.st);
    hipEvent_t t0 = E.clock.begin(E.st);
    HB_LAUNCH(hbk::block_gemm_launch(E.scalar, dg, (int)gj.size(), (int)max_rows, max_rin, E.st));
    E.clock.end(KC_GEMM, t0, E.st);
  }
}

// Algorithmic flops of a batch of merges (see hb_stats::merge_flops).
static double merge_job_flops(const std::vector<MergeJob>& jobs, int scalar) {
  const double phi = scalar ? 4.0 : 1.0;
  double f = 0.0;
  for (const MergeJob& J : jobs) {
    const double k = (double)J.r1 + J.r2, r = J.outP_owner ? J.outP_owner->r : 0;
    f += 2.0 * phi * (double)J.rows * k * k + 2.0 * phi * (double)J.rows * k * r +
         2.0 * phi * r * ((double)J.r1 * J.n1 + (double)J.r2 * J.n2);
  }
  return f;
}

static void run_merges(Engine& E, std::vector<MergeJob>& jobs, DevMem& out_mem) {
  const int kcap = E.kcap();
  std::vector<MergeJob> direct, split;
  for (auto& J : jobs) {
    const int k = J.r1 + J.r2;
    if (k <= kcap) direct.push_back(J);
    else if (k <= 512) split.push_back(J);
    else throw HbError{HB_EUNSUPPORTED};
  }
  run_merges_direct(E, direct, out_mem);
  run_merges_caqr(E, split, out_mem);
}

// SVD re-compression of BACA leaves: U (m0 x r), Vh (n0 x r) -> truncated SVD.
struct RecJob {
  const void* U;
  const void* Vh;
  int64_t m0, n0;
  int r;
  Block* out;
};

static void run_recompress_narrow(Engine& E, std::vector<RecJob>& jobs, DevMem& out_mem);

// Leaves whose BACA rank exceeds the register TSQR tile: the same steps as
// the narrow route (Section "Blocked Adaptive Cross Approximation", the SVD
// re-compression): Q_U T_U = QR(U), Q_V T_V = QR(V^H) by column panels,
// M = T_U T_V^H, the truncated SVD of M, then U' = Q_U Y_r and
// V'^H = Q_V X_r.  As on the narrow route the SVD is taken of
// M^H = T_V T_U^H, so that the side that becomes the next merge's
// orthonormal basis comes from the Jacobi iteration.
static void run_recompress_wide(Engine& E, std::vector<RecJob>& jobs, DevMem& out_mem) {
  const size_t nj = jobs.size();
  if (nj == 0) return;
  const size_t sb = E.sb();
  std::vector<const void*> B(2 * nj);
  std::vector<int64_t> rows(2 * nj);
  std::vector<int> k(2 * nj);
  for (size_t a = 0; a < nj; ++a) {
    B[2 * a] = jobs[a].U;
    rows[2 * a] = jobs[a].m0;
    B[2 * a + 1] = jobs[a].Vh;
    rows[2 * a + 1] = jobs[a].n0;
    k[2 * a] = k[2 * a + 1] = jobs[a].r;
  }
  PanelQR S;
  panel_qr_factor(E, B, rows, k, S);
  // M^H = T_V T_U^H (P_V x P_U) per leaf
  std::vector<size_t> msz(nj);
  for (size_t a = 0; a < nj; ++a) msz[a] = (size_t)S.P[2 * a] * S.P[2 * a + 1] * sb;
  std::vector<char*> MH = E.tmp.carve(msz);
  std::vector<RRhDev> mj(nj);
  std::vector<SVDJobDev> sj(nj);
  int64_t mmax = 0;
  for (size_t a = 0; a < nj; ++a) {
    const int pv = (int)S.P[2 * a + 1], pu = (int)S.P[2 * a];
    mj[a] = RRhDev{S.R[2 * a + 1], S.R[2 * a], MH[a], pv, pu, jobs[a].r, 0};
    mmax = std::max<int64_t>(mmax, (int64_t)pv * pu);
    SVDJobDev J{};
    J.p = pv;
    J.k = pu;
    J.from_node = 0;
    J.R = MH[a];
    sj[a] = J;
  }
  RRhDev* dmj = upload(E.tmp, mj, E.st);
  HB_LAUNCH(hbk::rrh_launch(E.scalar, dmj, (int)nj, mmax, E.st));
  std::vector<SvdOut> so;
  std::vector<int> rk;
  run_svds(E, sj, nullptr, nullptr, so, rk);
  std::vector<size_t> osz;
  for (size_t a = 0; a < nj; ++a) {
    osz.push_back((size_t)jobs[a].m0 * rk[a] * sb);
    osz.push_back((size_t)jobs[a].n0 * rk[a] * sb);
    osz.push_back((size_t)rk[a] * 8);
  }
  std::vector<char*> ob = out_mem.carve(osz);
  std::vector<const void*> zin(2 * nj, nullptr);
  std::vector<int64_t> ldin(2 * nj, 1);
  std::vector<int> rr(2 * nj, 0);
  std::vector<void*> zout(2 * nj, nullptr);
  std::vector<CopyDev> scp;
  for (size_t a = 0; a < nj; ++a) {
    Block& Bk = *jobs[a].out;
    const int r = rk[a];
    Bk.r = r;
    if (r == 0) continue;
    Bk.U = ob[3 * a];
    Bk.Vh = ob[3 * a + 1];
    Bk.S = (double*)ob[3 * a + 2];
    scp.push_back(CopyDev{so[a].S, Bk.S, (int64_t)r * 8});
    // M^H = X S Y^H  =>  M = Y S X^H: U side from Y, V side from X
    zin[2 * a] = so[a].Yr;
    ldin[2 * a] = so[a].k;
    rr[2 * a] = r;
    zout[2 * a] = Bk.U;
    zin[2 * a + 1] = so[a].Xr;
    ldin[2 * a + 1] = so[a].p;
    rr[2 * a + 1] = r;
    zout[2 * a + 1] = Bk.Vh;
  }
  copy_sigmas(E, scp);
  panel_qr_apply(E, S, zin, ldin, rr, zout);
}

static void run_recompress(Engine& E, std::vector<RecJob>& jobs, DevMem& out_mem) {
  std::vector<RecJob> narrow, wide;
  for (auto& J : jobs) {
    Block& B = *J.out;
    B.m = J.m0;
    B.n = J.n0;
    B.r = 0;
    if (J.r > 512) throw HbError{HB_EUNSUPPORTED};
    (J.r > E.kcap() ? wide : narrow).push_back(J);
  }
  run_recompress_narrow(E, narrow, out_mem);
  run_recompress_wide(E, wide, out_mem);
}

static void run_recompress_narrow(Engine& E, std::vector<RecJob>& jobs, DevMem& out_mem) {
  const size_t nj = jobs.size();
  std::vector<QRNodeDev> mats;
  std::vector<int64_t> rows;
  std::vector<size_t> live;
  for (size_t a = 0; a < nj; ++a) {
    Block& B = *jobs[a].out;
    B.m = jobs[a].m0;
    B.n = jobs[a].n0;
    B.r = 0;
    if (jobs[a].r == 0) continue;
    live.push_back(a);
    for (int side = 0; side < 2; ++side) {
      QRNodeDev nd{};
      nd.k = jobs[a].r;
      nd.P1 = side == 0 ? jobs[a].U : jobs[a].Vh;
      nd.ld1 = side == 0 ? jobs[a].m0 : jobs[a].n0;
      nd.n1 = jobs[a].r;
      nd.P2 = nd.P1;
      nd.ld2 = nd.ld1;
      nd.n2 = 0;
      mats.push_back(nd);
      rows.push_back(side == 0 ? jobs[a].m0 : jobs[a].n0);
    }
  }
  if (live.empty()) return;
  Engine::Factored F;
  E.factor(mats, rows, F);  // at once: the device factors while the host plans the rest
  Batch pre;
  const size_t nl = live.size();
  std::vector<QRNodeDev> topU(nl), topV(nl);
  std::vector<void*> Mptr(nl);
  std::vector<SVDJobDev> sj(nl);
  // The SVD is taken of M^H = R_V R_U^H: Jacobi's accurate (orthonormal to the
  // sweep tolerance) side then lands on V^H, which the first horizontal
  // merge uses as an orthonormal basis; U's side is R^H X / S.
  for (size_t i = 0; i < nl; ++i) {
    topU[i] = F.tb.levels[F.tb.top_level[2 * i]][F.tb.top_index[2 * i]];
    topV[i] = F.tb.levels[F.tb.top_level[2 * i + 1]][F.tb.top_index[2 * i + 1]];
    const int pu = topU[i].steps, pv = topV[i].steps;
    Mptr[i] = nullptr;
    SVDJobDev J{};
    J.p = pv;
    J.k = pu;
    J.from_node = 0;
    J.R = Mptr[i];
    sj[i] = J;
  }
  {
    std::vector<size_t> msz;
    for (size_t i = 0; i < nl; ++i) msz.push_back((size_t)topU[i].steps * topV[i].steps * E.sb());
    std::vector<char*> mb = E.tmp.carve(msz);
    for (size_t i = 0; i < nl; ++i) {
      Mptr[i] = mb[i];
      sj[i].R = mb[i];
    }
  }
  const size_t oU = pre.add(topV);  // first factor of M^H
  const size_t oV = pre.add(topU);
  const size_t oM = pre.add(Mptr);
  pre.then([&]() {
    QRNodeDev* dU = pre.at<QRNodeDev>(oU);
    QRNodeDev* dV = pre.at<QRNodeDev>(oV);
    void** dM = pre.at<void*>(oM);
    if (E.scalar == 0)
      hipLaunchKernelGGL((rrh_kernel<double>), dim3(nl), dim3(256), 0, E.st, dU, dV,
                         (const double*)F.store, (const double*)F.alpha, (double* const*)dM);
    else
      hipLaunchKernelGGL((rrh_kernel<hb_cplx>), dim3(nl), dim3(256), 0, E.st, dU, dV,
                         (const hb_cplx*)F.store, (const hb_cplx*)F.alpha, (hb_cplx* const*)dM);
    HB_HIP(hipGetLastError());
  });
  std::vector<SvdOut> so;
  std::vector<int> rk;
  run_svds(E, sj, F.store, F.alpha, so, rk, &pre, [&F]() { Engine::walk(F); });
  std::vector<int> rr(mats.size(), 0);
  std::vector<const void*> zin(mats.size(), nullptr);
  std::vector<int64_t> ldin(mats.size(), 1), ldout(mats.size(), 1);
  std::vector<void*> zout(mats.size(), nullptr);
  std::vector<size_t> osz;
  for (size_t i = 0; i < nl; ++i) {
    const RecJob& J = jobs[live[i]];
    osz.push_back((size_t)J.m0 * rk[i] * E.sb());
    osz.push_back((size_t)J.n0 * rk[i] * E.sb());
    osz.push_back((size_t)rk[i] * 8);
  }
  std::vector<char*> ob = out_mem.carve(osz);
  std::vector<CopyDev> scp;
  for (size_t i = 0; i < nl; ++i) {
    RecJob& J = jobs[live[i]];
    Block& B = *J.out;
    const int r = rk[i];
    B.r = r;
    if (r == 0) continue;
    B.U = ob[3 * i];
    B.Vh = ob[3 * i + 1];
    B.S = (double*)ob[3 * i + 2];
    scp.push_back(CopyDev{so[i].S, B.S, (int64_t)r * 8});
    // M^H = X S Y^H  =>  M = Y S X^H: U side from Y, V side from X
    rr[2 * i] = r;
    zin[2 * i] = so[i].Yr;
    ldin[2 * i] = so[i].k;
    zout[2 * i] = B.U;
    ldout[2 * i] = J.m0;
    rr[2 * i + 1] = r;
    zin[2 * i + 1] = so[i].Xr;
    ldin[2 * i + 1] = so[i].p;
    zout[2 * i + 1] = B.Vh;
    ldout[2 * i + 1] = J.n0;
  }
  Batch post;
  copy_sigmas(E, scp, &post);
  E.apply(F, zin, ldin, rr, zout, ldout, nullptr, nullptr, &post);
  post.run(E.tmp, E.st);
}

// ---------------------------------------------------------- the pipeline ---
struct CallSpec {
  int entry;
  const hb_params* prm;
  const double* X;  // row points (AoS)
  const double* Y;
  int64_t nx, ny;   // total points
  std::vector<int64_t> roff, rcnt, coff, ccnt;
  double tol;
  int d, leaf;
  hipStream_t st;
  bool batched;
};

static float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, a, b);
  return ms;
}

static hb_status validate(const CallSpec& c) {
  const hb_params* p = c.prm;
  if (!p) return HB_EINVAL;
  if (!(c.tol > 0.0 && c.tol < 1.0)) return std::isfinite(c.tol) ? HB_EINVAL : HB_ENONFINITE;
  if (c.d < 1 || c.leaf < 1) return HB_EINVAL;
  if (c.d > 32) return HB_EUNSUPPORTED;
  if (p->precision != HB_PREC_FP64 && p->precision != HB_PREC_MIXED) return HB_EINVAL;
  if (p->precision == HB_PREC_MIXED && (c.entry == HB_K_HELMHOLTZ3D || c.entry == HB_K_EFIE2D))
    return HB_EUNSUPPORTED;
  if (p->stop_after < 0 || p->stop_after > 2 + 2 * 30 || p->rank_cap < 0) return HB_EINVAL;
  if (p->record_tape < 0 || p->record_tape > 2) return HB_EINVAL;
  if (p->diag_panel < 0 || p->diag_panel > 128 || p->diag_svd_storage < 0 ||
      p->diag_svd_storage > 3)
    return HB_EINVAL;
  if (p->selector != HB_SEL_QRCP && p->selector != HB_SEL_STRONG) return HB_EINVAL;
  if (p->selector == HB_SEL_STRONG && !(std::isfinite(p->select_f) && p->select_f > 1.0))
    return HB_EINVAL;
  for (size_t b = 0; b < c.rcnt.size(); ++b) {
    if (c.rcnt[b] < 1 || c.ccnt[b] < 1 || c.roff[b] < 0 || c.coff[b] < 0) return HB_EINVAL;
    if (c.roff[b] + c.rcnt[b] > c.nx || c.coff[b] + c.ccnt[b] > c.ny) return HB_EINVAL;
  }
  switch (c.entry) {
    case HB_K_GAUSS:
      if (!std::isfinite(p->h) || !std::isfinite(p->gauss_c)) return HB_ENONFINITE;
      if (!(p->h > 0.0) || !(p->gauss_c > 0.0)) return HB_EINVAL;
      [[fallthrough]];
    case HB_K_LAPLACE:
    case HB_K_HELMHOLTZ3D:
    case HB_K_EFIE2D:
      if (c.entry == HB_K_HELMHOLTZ3D || c.entry == HB_K_EFIE2D) {
        if (!std::isfinite(p->wavenumber)) return HB_ENONFINITE;
        if (!(p->wavenumber > 0.0)) return HB_EINVAL;
      }
      if (p->dim < 1 || p->dim > HB_MAXDIM) return HB_EINVAL;
      if (!c.X || !c.Y) return HB_EINVAL;
      break;
    case HB_K_POLYNOMIAL:
      if (!std::isfinite(p->h)) return HB_ENONFINITE;
      if (p->dim < 1 || p->dim > HB_POLY_MAXDIM) return HB_EINVAL;
      if (!c.X || !c.Y) return HB_EINVAL;
      break;
    case HB_K_LOWRANK_SPIKES:
      if (c.batched) return HB_EINVAL;
      if (p->lr_rank < 1 || !p->lr_G1 || !p->lr_G2) return HB_EINVAL;
      if (p->n_spikes < 0 || (p->n_spikes > 0 && (!p->spike_lin || !p->spike_val))) return HB_EINVAL;
      break;
    default:
      return HB_EINVAL;
  }
  return HB_OK;
}

static hb_status run(const CallSpec& c, hb_result** out) {
  if (!out) return HB_EINVAL;
  *out = nullptr;
  hb_status vs = validate(c);
  if (vs != HB_OK) return vs;
  const hb_params& P = *c.prm;
  std::unique_ptr<hb_result> R(new (std::nothrow) hb_result());
  if (!R) return HB_ENOMEM;
  hipStream_t st = c.st;
  R->keep.st = st;
  R->keep.sync_free = true;
  DevMem tmp;
  tmp.st = st;
  hipEvent_t ev[6] = {};
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 6; ++i) EventPool::get().give(e[i]);
    }
  } evg{ev};
  for (auto& e : ev) {
    e = EventPool::get().take();
    if (!e) throw HbError{HB_EDEVICE};
  }
  HB_HIP(hipEventRecord(ev[0], st));

  const int scalar = (c.entry == HB_K_HELMHOLTZ3D || c.entry == HB_K_EFIE2D) ? 1 : 0;
  R->scalar = scalar;
  R->entry = c.entry;
  const size_t sbytes = scalar_bytes(scalar);
  // mixed precision: the leaf BACA runs on FP32 data (entries, residual
  // blocks, factors) with FP64 accumulation and norms; everything after it
  // is FP64
  const bool mixed = P.precision == HB_PREC_MIXED;
  const int bscalar = mixed ? 2 : scalar;
  const size_t bbytes = mixed ? 4 : sbytes;

  // ---- entry description (SoA points owned by the result)
  EntryDev E{};
  E.kind = c.entry;
  if (c.entry == HB_K_LOWRANK_SPIKES) {
    E.dim = 0;
    E.G1 = P.lr_G1;
    E.G2 = P.lr_G2;
    E.r0 = P.lr_rank;
    E.n_glob = c.ny;
    E.spike_lin = P.spike_lin;
    E.spike_val = P.spike_val;
    E.nspk = P.n_spikes;
  } else {
    // the polynomial kernel reads its coordinates by global index (any dim);
    // the others preload at most HB_MAXDIM of them per point
    E.dim = c.entry == HB_K_POLYNOMIAL ? 0 : P.dim;
    E.pdim = c.entry == HB_K_POLYNOMIAL ? P.dim : 0;
    E.poly_h = P.h;
    double* Xs = R->keep.get<double>((size_t)c.nx * P.dim);
    double* Ys = R->keep.get<double>((size_t)c.ny * P.dim);
    hipLaunchKernelGGL(aos_to_soa_kernel, dim3((c.nx + 255) / 256), dim3(256), 0, st, c.X, Xs,
                       c.nx, P.dim);
    hipLaunchKernelGGL(aos_to_soa_kernel, dim3((c.ny + 255) / 256), dim3(256), 0, st, c.Y, Ys,
                       c.ny, P.dim);
    HB_HIP(hipGetLastError());
    E.X = Xs;
    E.Y = Ys;
    E.ldx = c.nx;
    E.ldy = c.ny;
    E.neg_inv_ch2 = c.entry == HB_K_GAUSS ? -1.0 / (P.gauss_c * P.h * P.h) : 0.0;
    E.wavenumber = P.wavenumber;
  }
  R->E = E;

  // ---- problems, trees, leaves
  const size_t np = c.rcnt.size();
  R->problems.resize(np);
  int Lmax = 0;
  for (size_t p = 0; p < np; ++p) {
    Problem& pr = R->problems[p];
    pr.m = c.rcnt[p];
    pr.n = c.ccnt[p];
    pr.row_base = c.roff[p];
    pr.col_base = c.coff[p];
    pr.L = tree_levels(pr.m, pr.n, c.leaf);
    pr.seed = P.seed + (c.batched ? (uint64_t)p : 0ull);
    pr.rt = cluster_tree(pr.m, pr.L);
    pr.ct = cluster_tree(pr.n, pr.L);
    Lmax = std::max(Lmax, pr.L);
    const int nb = 1 << pr.L;
    for (int t = 0; t < nb; ++t)
      for (int v = 0; v < nb; ++v) {
        LeafHost lf;
        lf.problem = (int)p;
        lf.t = t;
        lf.v = v;
        lf.row0 = pr.row_base + pr.rt[pr.L][t].off;
        lf.col0 = pr.col_base + pr.ct[pr.L][v].off;
        lf.m0 = (int)pr.rt[pr.L][t].size;
        lf.n0 = (int)pr.ct[pr.L][v].size;
        R->leaves.push_back(lf);
      }
  }
  const size_t nleaves = R->leaves.size();
  int maxdim = 0;
  for (auto& lf : R->leaves) maxdim = std::max(maxdim, std::max(lf.m0, lf.n0));
  if (maxdim > 2048) return HB_EUNSUPPORTED;
  const int dmax = c.d <= 8 ? 8 : (c.d <= 16 ? 16 : 32);
  const int rpt = (maxdim + 511) / 512;
  int rpt_v = rpt <= 1 ? 1 : (rpt <= 2 ? 2 : 4);
  if (scalar == 1 && ((dmax == 16 && rpt_v > 2) || (dmax == 32 && rpt_v > 1))) return HB_EUNSUPPORTED;
  if (scalar == 0 && !mixed && dmax == 32 && rpt_v > 2) return HB_EUNSUPPORTED;

  // ---- leaf descriptors; largest leaves first
  std::vector<int> order(nleaves);
  for (size_t i = 0; i < nleaves; ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (int64_t)R->leaves[a].m0 * R->leaves[a].n0 > (int64_t)R->leaves[b].m0 * R->leaves[b].n0;
  });
  std::vector<BacaLeafDev> ld(nleaves);
  std::vector<int32_t> j1;
  int64_t uo = 0, vo = 0, co = 0, ro = 0;
  int32_t tapeo = 0, ito = 0;
  std::vector<int> caps(nleaves);
  for (size_t s = 0; s < nleaves; ++s) {
    const LeafHost& lf = R->leaves[order[s]];
    const Problem& pr = R->problems[lf.problem];
    BacaLeafDev& L = ld[s];
    std::memset(&L, 0, sizeof(L));
    L.m0 = lf.m0;
    L.n0 = lf.n0;
    L.row0 = lf.row0;
    L.col0 = lf.col0;
    int cap = std::min(lf.m0, lf.n0);
    if (P.rank_cap > 0) cap = std::min(cap, P.rank_cap);
    caps[s] = cap;
    L.cap = cap;
    L.u_off = uo;
    uo += (int64_t)lf.m0 * cap;
    L.v_off = vo;
    vo += (int64_t)lf.n0 * cap;
    L.c_off = co;
    co += (int64_t)lf.m0 * dmax;
    L.r_off = ro;
    ro += (int64_t)lf.n0 * dmax;
    L.tape_off = tapeo;
    tapeo += cap;
    L.it_off = ito;
    ito += cap + 1;
    L.j1_off = (int32_t)j1.size();
    L.nj1 = std::min(c.d, lf.n0);
    const uint64_t b = (uint64_t)lf.t * ((uint64_t)1 << pr.L) + (uint64_t)lf.v;
    std::vector<int32_t> jj(L.nj1);
    first_column_block(pr.seed, b, lf.n0, c.d, jj.data());
    j1.insert(j1.end(), jj.begin(), jj.end());
  }
  DevMem baca_mem;
  baca_mem.st = st;
  BacaArgs A{};
  A.leaves = upload(tmp, ld, st);
  A.out = tmp.get<BacaOutDev>(nleaves);
  A.E = E;
  A.U = baca_mem.alloc((size_t)std::max<int64_t>(uo, 1) * bbytes);
  A.V = baca_mem.alloc((size_t)std::max<int64_t>(vo, 1) * bbytes);
  A.C = tmp.alloc((size_t)std::max<int64_t>(co, 1) * bbytes);
  A.R = tmp.alloc((size_t)std::max<int64_t>(ro, 1) * bbytes);
  A.j1 = upload(tmp, j1, st);
  A.tape_rows = tmp.get<int32_t>(std::max(tapeo, 1));
  A.tape_cols = tmp.get<int32_t>(std::max(tapeo, 1));
  A.it_dk = tmp.get<int32_t>(std::max(ito, 1));
  A.it_nu = tmp.get<double>(std::max(ito, 1));
  A.it_mu = tmp.get<double>(std::max(ito, 1));
  const bool frozen = P.record_tape == 2;
  if (frozen) {
    A.fz_stride = 3 + 3 * dmax;
    A.fz = tmp.get<int32_t>((size_t)std::max(ito, 1) * A.fz_stride);
    R->fz_stride = A.fz_stride;
    R->fz_h = P.h;
    R->fz_c = P.gauss_c;
  }
  A.eps = c.tol;
  A.nleaves = (int32_t)nleaves;
  A.queue = tmp.get<int32_t>(2);
  A.selector = P.selector;
  A.select_f = P.select_f;
  HB_HIP(hipEventRecord(ev[1], st));
  HB_LAUNCH(hbk::baca_launch(bscalar, dmax, rpt_v, A, st));
  HB_HIP(hipEventRecord(ev[2], st));
  std::vector<BacaOutDev> bo(nleaves);
  HB_HIP(hipMemcpyAsync(bo.data(), A.out, nleaves * sizeof(BacaOutDev), hipMemcpyDeviceToHost, st));
  std::vector<int32_t> h_rows, h_cols, h_dk(std::max(ito, 1)), h_fz;
  std::vector<double> h_nu, h_mu;
  if (frozen) {
    h_fz.resize((size_t)std::max(ito, 1) * A.fz_stride);
    HB_HIP(hipMemcpyAsync(h_fz.data(), A.fz, (size_t)ito * A.fz_stride * 4, hipMemcpyDeviceToHost,
                          st));
  }
  HB_HIP(hipMemcpyAsync(h_dk.data(), A.it_dk, ito * 4, hipMemcpyDeviceToHost, st));
  if (P.record_tape) {
    h_rows.resize(tapeo);
    h_cols.resize(tapeo);
    h_nu.resize(ito);
    h_mu.resize(ito);
    HB_HIP(hipMemcpyAsync(h_rows.data(), A.tape_rows, tapeo * 4, hipMemcpyDeviceToHost, st));
    HB_HIP(hipMemcpyAsync(h_cols.data(), A.tape_cols, tapeo * 4, hipMemcpyDeviceToHost, st));
    HB_HIP(hipMemcpyAsync(h_nu.data(), A.it_nu, ito * 8, hipMemcpyDeviceToHost, st));
    HB_HIP(hipMemcpyAsync(h_mu.data(), A.it_mu, ito * 8, hipMemcpyDeviceToHost, st));
  }
  HB_HIP(hipStreamSynchronize(st));
  hb_stats& S = R->stats;
  S.n_leaves = (int32_t)nleaves;
  S.n_blocks = (int32_t)np;
  S.levels_max = Lmax;
  for (size_t s = 0; s < nleaves; ++s) {
    LeafHost& lf = R->leaves[order[s]];
    lf.rank_baca = bo[s].rank;
    lf.iters = bo[s].iters;
    lf.status = bo[s].status;
    if (bo[s].status == 1) return HB_ERANKCAP;
    if (bo[s].status != 0) {  // a pivot outside its candidate range (non-finite data)
      hb_report("leaf BACA", bo[s].status, "pivot index outside the candidate range", __LINE__);
      return HB_EDEVICE;
    }
    if (P.record_tape) {
      lf.tape_rows.assign(h_rows.begin() + ld[s].tape_off, h_rows.begin() + ld[s].tape_off + lf.rank_baca);
      lf.tape_cols.assign(h_cols.begin() + ld[s].tape_off, h_cols.begin() + ld[s].tape_off + lf.rank_baca);
      lf.it_dk.assign(h_dk.begin() + ld[s].it_off, h_dk.begin() + ld[s].it_off + lf.iters);
      lf.it_nu.assign(h_nu.begin() + ld[s].it_off, h_nu.begin() + ld[s].it_off + lf.iters);
      lf.it_mu.assign(h_mu.begin() + ld[s].it_off, h_mu.begin() + ld[s].it_off + lf.iters);
    }
    if (frozen)
      lf.fz.assign(h_fz.begin() + (size_t)ld[s].it_off * A.fz_stride,
                   h_fz.begin() + (size_t)(ld[s].it_off + lf.iters) * A.fz_stride);
    S.leaf_rank_baca_max = std::max(S.leaf_rank_baca_max, lf.rank_baca);
    S.iters_max = std::max(S.iters_max, lf.iters);
    S.iters_total += lf.iters;
    S.select_swaps += bo[s].swaps;
  }
  // algorithmic counters of the residual passes (iteration k streams r_{k-1}
  // columns of U and V once and evaluates d (m0 + n0) entries)
  {
    const double phi = scalar ? 4.0 : 1.0;
    for (size_t s = 0; s < nleaves; ++s) {
      const LeafHost& lf = R->leaves[order[s]];
      int r = 0;
      for (int k = 0; k < lf.iters; ++k) {
        const double mn = (double)lf.m0 + lf.n0;
        S.resid_bytes += (double)bbytes * r * mn;
        S.resid_cr_bytes += (double)bbytes *
                            ((double)std::min(c.d, lf.n0) * lf.m0 + (double)std::min(c.d, lf.m0) * lf.n0);
        S.resid_flops += 2.0 * phi * std::min(c.d, lf.n0) * r * mn;
        S.entries_evaluated += (double)std::min(c.d, lf.n0) * mn;
        r += h_dk[ld[s].it_off + k];
      }
    }
  }
  // the leaf BACA factors as blocks (stop_after == 1)
  std::vector<Block> leafblk(nleaves);
  for (size_t s = 0; s < nleaves; ++s) {
    const int li = order[s];
    Block& b = leafblk[li];
    b.m = ld[s].m0;
    b.n = ld[s].n0;
    b.r = bo[s].rank;
    b.U = (char*)A.U + (size_t)ld[s].u_off * bbytes;
    b.Vh = (char*)A.V + (size_t)ld[s].v_off * bbytes;
  }
  DevMem cvt_mem;
  cvt_mem.st = st;
  if (mixed) {
    // widen the used factor columns to FP64
    size_t tot = 0;
    for (auto& b : leafblk) tot += (size_t)(b.m + b.n) * b.r;
    double* wide = cvt_mem.get<double>(std::max<size_t>(tot, 1));
    std::vector<CvtDev> cj;
    size_t off = 0;
    for (auto& b : leafblk) {
      if (b.r == 0) {
        b.U = wide;
        b.Vh = wide;
        continue;
      }
      cj.push_back(CvtDev{(const float*)b.U, wide + off, (int64_t)b.m * b.r});
      b.U = wide + off;
      off += (size_t)b.m * b.r;
      cj.push_back(CvtDev{(const float*)b.Vh, wide + off, (int64_t)b.n * b.r});
      b.Vh = wide + off;
      off += (size_t)b.n * b.r;
    }
    if (!cj.empty()) {
      CvtDev* dj = upload(tmp, cj, st);
      for (size_t j0 = 0; j0 < cj.size(); j0 += 65535) {
        const unsigned ny = (unsigned)std::min<size_t>(65535, cj.size() - j0);
        hipLaunchKernelGGL(cvt_f2d_kernel, dim3(8, ny), dim3(256), 0, st, dj + j0);
        HB_HIP(hipGetLastError());
      }
    }
  }
  Engine Eng(st, scalar, c.tol, tmp);
  Eng.panel = P.diag_panel;
  Eng.svd_storage = P.diag_svd_storage;
  if (P.stop_after == 1) {
    // keep the BACA arena in the result; blocks are leaves with sigma = 1
    for (void* p : baca_mem.ptrs) R->keep.ptrs.push_back(p);
    baca_mem.ptrs.clear();
    for (void* p : cvt_mem.ptrs) R->keep.ptrs.push_back(p);
    cvt_mem.ptrs.clear();
    int maxr = 1;
    for (auto& b : leafblk) maxr = std::max(maxr, b.r);
    std::vector<double> ones(maxr, 1.0);
    double* dones = upload(R->keep, ones, st);
    for (auto& b : leafblk) b.S = dones;
    R->out_blocks = leafblk;
    S.n_blocks = (int32_t)nleaves;
    HB_HIP(hipEventRecord(ev[3], st));
    HB_HIP(hipEventRecord(ev[4], st));
  } else {
    // ---- leaf SVD re-compression
    DevMem lvl_mem;
    lvl_mem.st = st;
    std::vector<Block> cur(nleaves);
    std::vector<RecJob> rj;
    for (size_t i = 0; i < nleaves; ++i)
      rj.push_back(RecJob{leafblk[i].U, leafblk[i].Vh, leafblk[i].m, leafblk[i].n, leafblk[i].r, &cur[i]});
    run_recompress(Eng, rj, lvl_mem);
    {
      const double phi = scalar ? 4.0 : 1.0;
      for (size_t i = 0; i < nleaves; ++i) {
        const double rb = leafblk[i].r, rho = cur[i].r;
        const double mn = (double)leafblk[i].m + (double)leafblk[i].n;
        S.recompress_flops += 2.0 * phi * mn * rb * rb + 2.0 * phi * mn * rb * rho;
      }
    }
    baca_mem.release();
    cvt_mem.release();
    HB_HIP(hipEventRecord(ev[3], st));
    for (size_t i = 0; i < nleaves; ++i) {
      R->leaves[i].rank_leaf = cur[i].r;
      S.leaf_rank_max = std::max(S.leaf_rank_max, cur[i].r);
    }
    S.step_rank_max[0] = S.leaf_rank_max;
    if (P.stop_after == 2) {
      for (void* p : lvl_mem.ptrs) R->keep.ptrs.push_back(p);
      lvl_mem.ptrs.clear();
      R->out_blocks = cur;
      S.n_blocks = (int32_t)nleaves;
    } else {
      // ---- merges: per problem a map (t, v) -> block at the current depth
      std::vector<std::vector<Block>> blk(np);
      std::vector<int> depth(np);
      {
        size_t i = 0;
        for (size_t p = 0; p < np; ++p) {
          const int nb = 1 << R->problems[p].L;
          blk[p].assign(cur.begin() + i, cur.begin() + i + (size_t)nb * nb);
          depth[p] = R->problems[p].L;
          i += (size_t)nb * nb;
        }
      }
      DevMem* prev_mem = &lvl_mem;
      std::vector<std::unique_ptr<DevMem>> mems;
      int step = 0;
      for (int l = 1; l <= Lmax; ++l) {
        // horizontal: (tau_i, nu) from (tau_i, nu_1) and (tau_i, nu_2)
        std::unique_ptr<DevMem> hm(new DevMem());
        hm->st = st;
        std::vector<std::vector<Block>> hb(np);
        std::vector<MergeJob> jobs;
        for (size_t p = 0; p < np; ++p) {
          if (depth[p] < 1) continue;
          const int nbc = 1 << depth[p];
          const int nbp = nbc / 2;
          hb[p].assign((size_t)nbc * nbp, Block{});
          for (int ti = 0; ti < nbc; ++ti)
            for (int v = 0; v < nbp; ++v) {
              const Block& b1 = blk[p][(size_t)ti * nbc + 2 * v];
              const Block& b2 = blk[p][(size_t)ti * nbc + 2 * v + 1];
              MergeJob J{};
              J.rows = b1.m;
              J.P1 = b1.U; J.r1 = b1.r; J.S1 = b1.S;
              J.P2 = b2.U; J.r2 = b2.r; J.S2 = b2.S;
              J.O1 = b1.Vh; J.n1 = b1.n;
              J.O2 = b2.Vh; J.n2 = b2.n;
              J.p_is_u = true;
              J.outP_owner = &hb[p][(size_t)ti * nbp + v];
              jobs.push_back(J);
            }
        }
        run_merges(Eng, jobs, *hm);
        S.merge_flops += merge_job_flops(jobs, scalar);
        int mx = 0;
        for (auto& J : jobs) mx = std::max(mx, J.outP_owner->r);
        if (frozen && np == 1) {
          std::vector<int> rk;
          for (auto& J : jobs) rk.push_back(J.outP_owner->r);
          R->fz_hrank.push_back(rk);
        }
        S.step_rank_max[std::min(++step, 63)] = mx;
        if (P.stop_after == 2 + step) {  // diagnostics: blocks after this step
          for (size_t p = 0; p < np; ++p)
            for (auto& b : hb[p]) R->out_blocks.push_back(b);
          for (void* q : hm->ptrs) R->keep.ptrs.push_back(q);
          hm->ptrs.clear();
          for (auto& m : mems)
            for (void* q : m->ptrs) R->keep.ptrs.push_back(q);
          for (auto& m : mems) m->ptrs.clear();
          for (void* q : prev_mem->ptrs) R->keep.ptrs.push_back(q);
          prev_mem->ptrs.clear();
          break;
        }
        // The previous level's memory holds the finished roots of every
        // problem whose tree ended there (L = l - 1); those move to the
        // result, the rest of that memory is free for reuse.
        {
          bool holds_root = false;
          for (size_t p = 0; p < np; ++p)
            if (R->problems[p].L == l - 1) holds_root = true;
          if (holds_root) {
            for (void* q : prev_mem->ptrs) R->keep.ptrs.push_back(q);
            prev_mem->ptrs.clear();
          }
        }
        prev_mem->release();
        // vertical: (tau, nu) from (tau_1, nu) and (tau_2, nu)
        std::unique_ptr<DevMem> vm(new DevMem());
        vm->st = st;
        jobs.clear();
        std::vector<std::vector<Block>> vb(np);
        for (size_t p = 0; p < np; ++p) {
          if (depth[p] < 1) continue;
          const int nbc = 1 << depth[p];
          const int nbp = nbc / 2;
          vb[p].assign((size_t)nbp * nbp, Block{});
          for (int t = 0; t < nbp; ++t)
            for (int v = 0; v < nbp; ++v) {
              const Block& b1 = hb[p][(size_t)(2 * t) * nbp + v];
              const Block& b2 = hb[p][(size_t)(2 * t + 1) * nbp + v];
              MergeJob J{};
              J.rows = b1.n;
              J.P1 = b1.Vh; J.r1 = b1.r; J.S1 = b1.S;
              J.P2 = b2.Vh; J.r2 = b2.r; J.S2 = b2.S;
              J.O1 = b1.U; J.n1 = b1.m;
              J.O2 = b2.U; J.n2 = b2.m;
              J.p_is_u = false;
              J.outP_owner = &vb[p][(size_t)t * nbp + v];
              jobs.push_back(J);
            }
        }
        run_merges(Eng, jobs, *vm);
        S.merge_flops += merge_job_flops(jobs, scalar);
        mx = 0;
        for (auto& J : jobs) mx = std::max(mx, J.outP_owner->r);
        if (frozen && np == 1) {
          std::vector<int> rk;
          for (auto& J : jobs) rk.push_back(J.outP_owner->r);
          R->fz_vrank.push_back(rk);
        }
        S.step_rank_max[std::min(++step, 63)] = mx;
        if (P.stop_after == 2 + step) {  // diagnostics: blocks after this step
          for (size_t p = 0; p < np; ++p)
            for (auto& b : vb[p]) R->out_blocks.push_back(b);
          for (void* q : vm->ptrs) R->keep.ptrs.push_back(q);
          vm->ptrs.clear();
          for (void* q : hm->ptrs) R->keep.ptrs.push_back(q);
          hm->ptrs.clear();
          for (auto& m : mems)
            for (void* q : m->ptrs) R->keep.ptrs.push_back(q);
          for (auto& m : mems) m->ptrs.clear();
          break;
        }
        hm->release();
        for (size_t p = 0; p < np; ++p)
          if (depth[p] >= 1) {
            blk[p] = vb[p];
            depth[p] -= 1;
          }
        mems.push_back(std::move(vm));
        prev_mem = mems.back().get();
        tmp.release();
      }
      S.n_steps = step + 1;
      if (P.stop_after > 2) {
        S.n_blocks = (int32_t)R->out_blocks.size();
        HB_HIP(hipEventRecord(ev[4], st));
        goto finish;
      }
      // roots: keep their memory
      for (auto& m : mems)
        for (void* p : m->ptrs) R->keep.ptrs.push_back(p);
      for (auto& m : mems) m->ptrs.clear();
      if (mems.empty()) {
        for (void* p : lvl_mem.ptrs) R->keep.ptrs.push_back(p);
        lvl_mem.ptrs.clear();
      }
      for (size_t p = 0; p < np; ++p) {
        R->problems[p].root = blk[p][0];
        R->out_blocks.push_back(blk[p][0]);
      }
      R->fz_complete = frozen && np == 1;
    }
    HB_HIP(hipEventRecord(ev[4], st));
  }
finish:
  S.svd_sweeps_max = Eng.svd_sweeps_max;
  HB_HIP(hipEventRecord(ev[5], st));
  HB_HIP(hipStreamSynchronize(st));
  {
    double ms[KC_N] = {0.0, 0.0, 0.0};
    int nl[KC_N] = {0, 0, 0};
    Eng.clock.totals(ms, nl);
    S.ms_svd = ms[KC_SVD];
    S.ms_qr = ms[KC_QR];
    S.ms_gemm = ms[KC_GEMM];
    S.svd_launches = nl[KC_SVD];
    S.qr_launches = nl[KC_QR];
    S.svd_flops = Eng.svd_flops;
  }
  S.ms_setup = elapsed(ev[0], ev[1]);
  S.ms_baca = elapsed(ev[1], ev[2]);
  S.ms_recompress = elapsed(ev[2], ev[3]);
  S.ms_merge = elapsed(ev[3], ev[4]);
  S.ms_total = elapsed(ev[0], ev[5]);
  tmp.release();
  *out = R.release();
  return HB_OK;
}

static hb_status guarded(const CallSpec& c, hb_result** out) {
  try {
    return run(c, out);
  } catch (const HbError& e) {
    if (out) *out = nullptr;
    return e.st;
  } catch (const std::bad_alloc&) {
    if (out) *out = nullptr;
    return HB_ENOMEM;
  } catch (...) {
    if (out) *out = nullptr;
    return HB_EDEVICE;
  }
}

}  // namespace

// ------------------------------------------------------------ HODLR matrix ---
// A hierarchical (HODLR) matrix of the kernel matrix of one KD-ordered point
// set with itself: the cluster tree of [0, N) splits a node into ceil(s/2)
// and floor(s/2) down to the depth whose nodes hold at most nmin points;
// both off-diagonal blocks A(c1, c2), A(c2, c1) of every internal node are
// compressed by H-BACA in one batched call, the leaves' diagonal blocks are
// kept dense (the construction of hierarchical matrices the paper names as
// the method's use; Introduction and Section "Numerical Results").
struct HodlrJob {
  const double* U;   // rows x r
  const double* Vh;  // cols x r
  const double* S;   // r
  int64_t row0, rows, col0, cols;
  int r;
  int pad;
  int64_t t_off;     // offset of this block's r products in t
};

// t[t_off + j] = S_j sum_i Vh(i, j) x[col0 + i]: one workgroup per (column
// j, block), a fixed-order tree sum.
__global__ __launch_bounds__(AP_NT) void hodlr_reduce_kernel(const HodlrJob* __restrict__ jobs,
                                                             const double* __restrict__ x,
                                                             double* __restrict__ t) {
  const HodlrJob J = jobs[blockIdx.y];
  const int j = blockIdx.x;
  if (j >= J.r) return;
  const double* v = J.Vh + (int64_t)j * J.cols;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < J.cols; i += AP_NT) acc = fma(v[i], x[J.col0 + i], acc);
  acc = group_sum<64>(acc);
  __shared__ double part[AP_NT / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = part[0];
    for (int w = 1; w < AP_NT / 64; ++w) sum += part[w];
    t[J.t_off + j] = sum * J.S[j];
  }
}

// y[row0 + i] += sum_j U(i, j) t[t_off + j]: one thread per row; the blocks
// of one launch have disjoint rows (one tree level), so no atomics.
__global__ __launch_bounds__(AP_NT) void hodlr_expand_kernel(const HodlrJob* __restrict__ jobs,
                                                             const double* __restrict__ t,
                                                             double* __restrict__ y) {
  const HodlrJob J = jobs[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * AP_NT + threadIdx.x;
  if (i >= J.rows) return;
  double acc = 0.0;
  for (int j = 0; j < J.r; ++j) acc = fma(J.U[(int64_t)j * J.rows + i], t[J.t_off + j], acc);
  y[J.row0 + i] += acc;
}

struct HodlrLeafDev {
  int64_t off, size, d_off;  // rows/columns [off, off + size); dense block at D + d_off
};

// D_l(i, j) = A(off + i, off + j), column-major: one thread per entry.
__global__ void hodlr_dense_kernel(EntryDev E, const HodlrLeafDev* __restrict__ leaves,
                                   double* __restrict__ D) {
  const HodlrLeafDev L = leaves[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= L.size * L.size) return;
  const int64_t i = e % L.size, j = e / L.size;
  double xi[HB_MAXDIM], yj[HB_MAXDIM];
  for (int q = 0; q < HB_MAXDIM; ++q) {
    xi[q] = q < E.dim ? E.X[(int64_t)q * E.ldx + L.off + i] : 0.0;
    yj[q] = q < E.dim ? E.Y[(int64_t)q * E.ldy + L.off + j] : 0.0;
  }
  D[L.d_off + e] = eval_entry<double>(E, L.off + i, L.off + j, xi, yj);
}

// y[off + i] = sum_j D_l(i, j) x[off + j]: one thread per row of a leaf.
__global__ __launch_bounds__(AP_NT) void hodlr_diag_kernel(const HodlrLeafDev* __restrict__ leaves,
                                                           const double* __restrict__ D,
                                                           const double* __restrict__ x,
                                                           double* __restrict__ y) {
  const HodlrLeafDev L = leaves[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * AP_NT + threadIdx.x;
  if (i >= L.size) return;
  const double* Dl = D + L.d_off;
  double acc = 0.0;
  for (int64_t j = 0; j < L.size; ++j) acc = fma(Dl[j * L.size + i], x[L.off + j], acc);
  y[L.off + i] = acc;
}

hb_hodlr::~hb_hodlr() {
  if (blocks) hb_result_free(blocks);
}

// ============================================================== C ABI =======
namespace {

// The per-column products t = diag(S) X^H v of hbaca_apply live in this
// buffer for hbaca_apply_noalloc (callers that cannot allocate).  Each
// device holds its own copy until the process ends.
constexpr size_t kApplyScratchBytes = 64 * 1024;
static __device__ __align__(256) unsigned char scratch[kApplyScratchBytes];

// Device address of `scratch` on the current device, looked up once per
// device with that device current (the array's name in host code is only a
// host-side stand-in, never a device address).
static void* apply_scratch_ptr() {
  static std::mutex mu;
  static std::vector<void*> ptrs;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  if ((size_t)dev >= ptrs.size()) ptrs.resize((size_t)dev + 1, nullptr);
  if (!ptrs[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptrs[dev] = p;
  }
  return ptrs[dev];
}

// y = U diag(S) Vh^H v (adjoint 0) or Vh diag(S) U^H v (adjoint 1) with the
// r products t held in `t` (any device buffer of r scalars).
static hb_status apply_blocks(const Block& B, int scalar, const void* in, void* out, int adjoint,
                              void* t, hipStream_t st) {
  const int64_t nin = adjoint ? B.m : B.n, nout = adjoint ? B.n : B.m;
  const size_t sb = scalar_bytes(scalar);
  if (B.r == 0) {
    if (nout > 0 && hbk::zero_fill_launch(out, (size_t)nout * sb, st) != 0) return HB_EDEVICE;
    return HB_OK;
  }
  const void* X = adjoint ? B.U : B.Vh;  // reduced against the input
  const void* Z = adjoint ? B.Vh : B.U;  // expanded into the output
  const unsigned ng = (unsigned)((nout + AP_NT - 1) / AP_NT);
  const size_t sh = (size_t)B.r * sb;
  if (scalar == 0) {
    hipLaunchKernelGGL(apply_reduce_kernel<double>, dim3(B.r), dim3(AP_NT), 0, st,
                       (const double*)X, nin, B.r, B.S, (const double*)in, (double*)t);
    hipLaunchKernelGGL(apply_expand_kernel<double>, dim3(ng), dim3(AP_NT), sh, st,
                       (const double*)Z, nout, B.r, (const double*)t, (double*)out);
  } else {
    hipLaunchKernelGGL(apply_reduce_kernel<hb_cplx>, dim3(B.r), dim3(AP_NT), 0, st,
                       (const hb_cplx*)X, nin, B.r, B.S, (const hb_cplx*)in, (hb_cplx*)t);
    hipLaunchKernelGGL(apply_expand_kernel<hb_cplx>, dim3(ng), dim3(AP_NT), sh, st,
                       (const hb_cplx*)Z, nout, B.r, (const hb_cplx*)t, (hb_cplx*)out);
  }
  return hipGetLastError() == hipSuccess ? HB_OK : HB_EDEVICE;
}

struct GpuAdjExec {
  const AdjArgs& a;
  hipStream_t st;
  int err;
  void launch(int kind, int base, int count) {
    if (err == 0) err = hbk::adj_launch(kind, base, count, a, st);
  }
};

// The plan of the frozen pipeline recorded in a result (record_tape = 2).
static hb_status frozen_plan(const hb_result* r, AdjPlan& P) {
  const Problem& pr = r->problems[0];
  AdjPlanIn in;
  in.m = pr.m;
  in.n = pr.n;
  in.L = pr.L;
  in.dim = r->E.dim;
  in.fz_stride = r->fz_stride;
  in.dmax = (r->fz_stride - 3) / 3;
  for (const LeafHost& lf : r->leaves) {
    AdjLeafIn li;
    li.row0 = lf.row0 - pr.row_base;
    li.col0 = lf.col0 - pr.col_base;
    li.m0 = lf.m0;
    li.n0 = lf.n0;
    li.nrec = lf.iters;
    li.rank_leaf = lf.rank_leaf;
    li.rec = lf.fz.empty() ? nullptr : lf.fz.data();
    if ((int64_t)lf.fz.size() != (int64_t)lf.iters * r->fz_stride) return HB_EINVAL;
    in.leaves.push_back(li);
  }
  in.hrank = r->fz_hrank;
  in.vrank = r->fz_vrank;
  const int ps = adj_plan(in, P);
  if (ps == -6) return HB_EUNSUPPORTED;
  return ps == 0 ? HB_OK : HB_EINVAL;
}

// Arena and descriptors on the device; the points and width of `r`.
static AdjArgs frozen_args(const hb_result* r, const AdjPlan& P, DevMem& mem, hipStream_t st) {
  double* D = mem.get<double>((size_t)P.arena);
  AdjArgs a{};
  a.D = D;
  a.ws = D + P.ws_off;
  a.fz = upload(mem, P.fz, st);
  a.leaves = upload(mem, P.leaves, st);
  a.blocks = upload(mem, P.blocks, st);
  a.merges = upload(mem, P.merges, st);
  a.chunks = upload(mem, P.chunks, st);
  a.tasks = upload(mem, P.tasks, st);
  a.X = r->E.X;
  a.Y = r->E.Y;
  a.ldx = r->E.ldx;
  a.ldy = r->E.ldy;
  a.dim = r->E.dim;
  a.dmax = (r->fz_stride - 3) / 3;
  a.fz_stride = 3 + 3 * a.dmax;
  a.root = P.root;
  a.nb = P.nb;
  a.nleaves = (int32_t)P.leaves.size();
  a.h = r->fz_h;
  a.nic = r->E.neg_inv_ch2;
  return a;
}

static hb_status vjp_run(const hb_result* r, const double* w, const double* ybar, double* gw,
                         double* gh, double* gX, double* gY, hipStream_t st) {
  AdjPlan P;
  const hb_status ps = frozen_plan(r, P);
  if (ps != HB_OK) return ps;
  DevMem mem;
  mem.st = st;
  AdjArgs a = frozen_args(r, P, mem, st);
  a.w = w;
  a.ybar = ybar;
  a.gw = gw;
  a.gh = gh;
  a.gX = gX;
  a.gY = gY;
  GpuAdjExec ex{a, st, 0};
  adj_execute(ex, P, gX != nullptr, gY != nullptr, gh != nullptr);
  if (ex.err != 0) {
    hb_report("adjoint launch", ex.err, hipGetErrorString((hipError_t)ex.err), __LINE__);
    return HB_EDEVICE;
  }
  HB_HIP(hipStreamSynchronize(st));
  return HB_OK;
}

// The frozen operator of `t` at new points and width: a result of its own
// that carries the same frozen structure.
static hb_status recompute_run(const hb_result* t, const hb_params* p, const double* X,
                               const double* Y, hipStream_t st, hb_result** out) {
  const Problem& pr = t->problems[0];
  AdjPlan P;
  const hb_status ps = frozen_plan(t, P);
  if (ps != HB_OK) return ps;
  std::unique_ptr<hb_result> R(new (std::nothrow) hb_result());
  if (!R) return HB_ENOMEM;
  R->keep.st = st;
  R->keep.sync_free = true;
  R->scalar = 0;
  R->entry = HB_K_GAUSS;
  EntryDev E = t->E;
  double* Xs = R->keep.get<double>((size_t)pr.m * p->dim);
  double* Ys = R->keep.get<double>((size_t)pr.n * p->dim);
  hipLaunchKernelGGL(aos_to_soa_kernel, dim3((unsigned)((pr.m + 255) / 256)), dim3(256), 0, st, X,
                     Xs, pr.m, p->dim);
  hipLaunchKernelGGL(aos_to_soa_kernel, dim3((unsigned)((pr.n + 255) / 256)), dim3(256), 0, st, Y,
                     Ys, pr.n, p->dim);
  HB_HIP(hipGetLastError());
  E.X = Xs;
  E.Y = Ys;
  E.ldx = pr.m;
  E.ldy = pr.n;
  E.neg_inv_ch2 = -1.0 / (p->gauss_c * p->h * p->h);
  R->E = E;
  R->problems.push_back(pr);
  R->problems[0].root = Block{};
  R->problems[0].row_base = 0;
  R->problems[0].col_base = 0;
  R->leaves = t->leaves;
  for (LeafHost& lf : R->leaves) {
    lf.row0 -= pr.row_base;
    lf.col0 -= pr.col_base;
  }
  R->fz_stride = t->fz_stride;
  R->fz_complete = true;
  R->fz_hrank = t->fz_hrank;
  R->fz_vrank = t->fz_vrank;
  R->fz_h = p->h;
  R->fz_c = p->gauss_c;
  DevMem mem;
  mem.st = st;
  const AdjArgs a = frozen_args(R.get(), P, mem, st);
  GpuAdjExec ex{a, st, 0};
  adj_execute_forward(ex, P);
  if (ex.err != 0) {
    hb_report("frozen replay launch", ex.err, hipGetErrorString((hipError_t)ex.err), __LINE__);
    return HB_EDEVICE;
  }
  const AdjBlock& B = P.blocks[P.root];
  Block root;
  root.m = pr.m;
  root.n = pr.n;
  root.r = B.r;
  root.U = R->keep.alloc((size_t)pr.m * std::max(B.r, 1) * 8);
  root.Vh = R->keep.alloc((size_t)pr.n * std::max(B.r, 1) * 8);
  root.S = R->keep.get<double>((size_t)std::max(B.r, 1));
  if (B.r > 0) {
    HB_HIP(hipMemcpy2DAsync(root.U, (size_t)pr.m * 8, a.D + B.U, (size_t)B.ldU * 8,
                            (size_t)pr.m * 8, (size_t)B.r, hipMemcpyDeviceToDevice, st));
    HB_HIP(hipMemcpy2DAsync(root.Vh, (size_t)pr.n * 8, a.D + B.Vt, (size_t)B.ldVt * 8,
                            (size_t)pr.n * 8, (size_t)B.r, hipMemcpyDeviceToDevice, st));
    HB_HIP(hipMemcpyAsync(root.S, a.D + B.S, (size_t)B.r * 8, hipMemcpyDeviceToDevice, st));
  }
  R->problems[0].root = root;
  R->out_blocks.push_back(root);
  R->stats.n_blocks = 1;
  R->stats.n_leaves = (int32_t)R->leaves.size();
  R->stats.levels_max = pr.L;
  HB_HIP(hipStreamSynchronize(st));
  *out = R.release();
  return HB_OK;
}

}  // namespace

extern "C" {

hb_status hbaca_compress(int entry_fn_id, const hb_params* params, const double* points_row,
                         const double* points_col, int64_t m, int64_t n, double tol, int32_t d,
                         int32_t leaf, void* stream, hb_result** out) {
  if (out) *out = nullptr;
  if (!out || m < 1 || n < 1) return HB_EINVAL;
  CallSpec c;
  c.entry = entry_fn_id;
  c.prm = params;
  c.X = points_row;
  c.Y = points_col;
  c.nx = m;
  c.ny = n;
  c.roff = {0};
  c.rcnt = {m};
  c.coff = {0};
  c.ccnt = {n};
  c.tol = tol;
  c.d = d;
  c.leaf = leaf;
  c.st = (hipStream_t)stream;
  c.batched = false;
  return guarded(c, out);
}

hb_status hbaca_compress_batched(int entry_fn_id, const hb_params* params, int64_t nblocks,
                                 const double* points_row, const int64_t* row_off,
                                 const int64_t* row_cnt, const double* points_col,
                                 const int64_t* col_off, const int64_t* col_cnt, double tol,
                                 int32_t d, int32_t leaf, void* stream, hb_result** out) {
  if (out) *out = nullptr;
  if (!out || nblocks < 1 || !row_off || !row_cnt || !col_off || !col_cnt) return HB_EINVAL;
  CallSpec c;
  c.entry = entry_fn_id;
  c.prm = params;
  c.X = points_row;
  c.Y = points_col;
  c.nx = 0;
  c.ny = 0;
  try {
    c.roff.assign(row_off, row_off + nblocks);
    c.rcnt.assign(row_cnt, row_cnt + nblocks);
    c.coff.assign(col_off, col_off + nblocks);
    c.ccnt.assign(col_cnt, col_cnt + nblocks);
  } catch (...) {
    return HB_ENOMEM;
  }
  for (int64_t b = 0; b < nblocks; ++b) {
    c.nx = std::max(c.nx, row_off[b] + row_cnt[b]);
    c.ny = std::max(c.ny, col_off[b] + col_cnt[b]);
  }
  c.tol = tol;
  c.d = d;
  c.leaf = leaf;
  c.st = (hipStream_t)stream;
  c.batched = true;
  return guarded(c, out);
}

int64_t hb_result_nblocks(const hb_result* r) { return r ? (int64_t)r->out_blocks.size() : -1; }
int64_t hb_result_rank(const hb_result* r, int64_t b) {
  if (!r || b < 0 || b >= (int64_t)r->out_blocks.size()) return -1;
  return r->out_blocks[b].r;
}
int64_t hb_result_rows(const hb_result* r, int64_t b) {
  if (!r || b < 0 || b >= (int64_t)r->out_blocks.size()) return -1;
  return r->out_blocks[b].m;
}
int64_t hb_result_cols(const hb_result* r, int64_t b) {
  if (!r || b < 0 || b >= (int64_t)r->out_blocks.size()) return -1;
  return r->out_blocks[b].n;
}
int32_t hb_result_is_complex(const hb_result* r) { return r ? r->scalar : -1; }

hb_status hb_result_copy(const hb_result* r, int64_t b, void* U, double* sigma, void* Vh,
                         void* stream) {
  if (!r || b < 0 || b >= (int64_t)r->out_blocks.size()) return HB_EINVAL;
  const Block& B = r->out_blocks[b];
  if (B.r == 0) return HB_OK;
  const size_t sb = scalar_bytes(r->scalar);
  hipStream_t st = (hipStream_t)stream;
  if (U && hipMemcpyAsync(U, B.U, (size_t)B.m * B.r * sb, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return HB_EDEVICE;
  if (Vh && hipMemcpyAsync(Vh, B.Vh, (size_t)B.n * B.r * sb, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return HB_EDEVICE;
  if (sigma && hipMemcpyAsync(sigma, B.S, (size_t)B.r * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return HB_EDEVICE;
  return HB_OK;
}

hb_status hbaca_apply(const hb_result* r, int64_t b, const void* in, void* out, int32_t adjoint,
                      void* stream) {
  if (!r || b < 0 || b >= (int64_t)r->out_blocks.size() || !in || !out) return HB_EINVAL;
  if (adjoint != 0 && adjoint != 1) return HB_EINVAL;
  const Block& B = r->out_blocks[b];
  hipStream_t st = (hipStream_t)stream;
  const size_t sb = scalar_bytes(r->scalar);
  if (B.r == 0) return apply_blocks(B, r->scalar, in, out, adjoint, nullptr, st);
  if ((size_t)B.r * sb > kApplyScratchBytes) return HB_EUNSUPPORTED;
  void* t = BlockCache::get().alloc((size_t)B.r * sb, st);
  if (!t) return HB_ENOMEM;
  const hb_status s = apply_blocks(B, r->scalar, in, out, adjoint, t, st);
  BlockCache::get().release(t, st, false);
  return s;
}

hb_status hbaca_apply_noalloc(const hb_result* r, int64_t b, const void* in, void* out,
                              int32_t adjoint, void* stream) {
  if (!r || b < 0 || b >= (int64_t)r->out_blocks.size() || !in || !out) return HB_EINVAL;
  if (adjoint != 0 && adjoint != 1) return HB_EINVAL;
  const Block& B = r->out_blocks[b];
  hipStream_t st = (hipStream_t)stream;
  if ((size_t)B.r * scalar_bytes(r->scalar) > kApplyScratchBytes) return HB_EUNSUPPORTED;
  void* t = nullptr;
  if (B.r > 0) {
    t = apply_scratch_ptr();
    if (!t) return HB_EDEVICE;
  }
  return apply_blocks(B, r->scalar, in, out, adjoint, t, st);
}


hb_status hb_partition(int64_t m, int64_t n, int32_t leaf, int32_t d, uint64_t seed,
                       int32_t* L_out, int64_t* leaves, int32_t* j1) {
  if (m < 1 || n < 1 || leaf < 1 || d < 1 || !L_out) return HB_EINVAL;
  const int L = tree_levels(m, n, leaf);
  *L_out = L;
  if (!leaves && !j1) return HB_OK;
  try {
    const auto rt = cluster_tree(m, L);
    const auto ct = cluster_tree(n, L);
    const int64_t nb = (int64_t)1 << L;
    for (int64_t t = 0; t < nb; ++t)
      for (int64_t v = 0; v < nb; ++v) {
        const int64_t b = t * nb + v;
        const Node& rn = rt[L][t];
        const Node& cn = ct[L][v];
        if (leaves) {
          leaves[4 * b] = rn.off;
          leaves[4 * b + 1] = rn.size;
          leaves[4 * b + 2] = cn.off;
          leaves[4 * b + 3] = cn.size;
        }
        if (j1) {
          const int n0 = (int)cn.size;
          const int q = std::min<int>(d, n0);
          first_column_block(seed, (uint64_t)b, n0, d, j1 + b * d);
          for (int k = q; k < d; ++k) j1[b * d + k] = -1;
        }
      }
  } catch (const std::bad_alloc&) {
    return HB_ENOMEM;
  }
  return HB_OK;
}

hb_status hbaca_recompute_frozen(const hb_result* tape, const hb_params* params,
                                 const double* points_row, const double* points_col, void* stream,
                                 hb_result** out) {
  if (!out) return HB_EINVAL;
  *out = nullptr;
  if (!tape || !params || !points_row || !points_col) return HB_EINVAL;
  if (tape->entry != HB_K_GAUSS || tape->scalar != 0) return HB_EUNSUPPORTED;
  if (!tape->fz_complete || tape->fz_stride < 6 || tape->problems.size() != 1) return HB_EINVAL;
  if (!std::isfinite(params->h) || !std::isfinite(params->gauss_c)) return HB_ENONFINITE;
  if (!(params->h > 0.0) || !(params->gauss_c > 0.0) || params->dim != tape->E.dim)
    return HB_EINVAL;
  try {
    return recompute_run(tape, params, points_row, points_col, (hipStream_t)stream, out);
  } catch (const HbError& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    return HB_ENOMEM;
  }
}

// A result the adjoint can replay: a single real Gaussian problem compressed
// with its frozen structure recorded.
static hb_status vjp_check(const hb_result* r) {
  if (r->entry != HB_K_GAUSS || r->scalar != 0) return HB_EUNSUPPORTED;
  if (!r->fz_complete || r->fz_stride < 6 || r->problems.size() != 1) return HB_EINVAL;
  return HB_OK;
}

hb_status hbaca_vjp(const hb_result* r, const double* w, const double* ybar, double* grad_w,
                    double* grad_h, double* grad_points_row, double* grad_points_col,
                    void* stream) {
  if (!r || !w || !ybar) return HB_EINVAL;
  const hb_status ok = vjp_check(r);
  if (ok != HB_OK) return ok;
  try {
    return vjp_run(r, w, ybar, grad_w, grad_h, grad_points_row, grad_points_col,
                   (hipStream_t)stream);
  } catch (const HbError& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    return HB_ENOMEM;
  }
}

hb_status hbaca_adjoint(const hb_result* r, const float* w, const float* ybar, float* wbar,
                        double* hbar, double* points_row_bar, double* points_col_bar,
                        void* stream) {
  if (!r || !w || !ybar) return HB_EINVAL;
  const hb_status ok = vjp_check(r);
  if (ok != HB_OK) return ok;
  try {
    const hipStream_t st = (hipStream_t)stream;
    const int64_t m = r->problems[0].m, n = r->problems[0].n;
    DevMem mem;
    mem.st = st;
    double* wd = mem.get<double>((size_t)n);
    double* yd = mem.get<double>((size_t)m);
    double* gw = wbar ? mem.get<double>((size_t)n) : nullptr;
    hipLaunchKernelGGL(widen_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, wd,
                       n);
    hipLaunchKernelGGL(widen_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, ybar,
                       yd, m);
    HB_HIP(hipGetLastError());
    const hb_status vs = vjp_run(r, wd, yd, gw, hbar, points_row_bar, points_col_bar, st);
    if (vs != HB_OK) return vs;
    if (wbar) {
      hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gw,
                         wbar, n);
      HB_HIP(hipGetLastError());
      HB_HIP(hipStreamSynchronize(st));
    }
    return HB_OK;
  } catch (const HbError& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    return HB_ENOMEM;
  }
}

hb_status hb_result_stats(const hb_result* r, hb_stats* out) {
  if (!r || !out) return HB_EINVAL;
  *out = r->stats;
  return HB_OK;
}

int64_t hb_result_nleaves(const hb_result* r) { return r ? (int64_t)r->leaves.size() : -1; }

hb_status hb_result_leaf_info(const hb_result* r, int64_t leaf, int64_t* info) {
  if (!r || !info || leaf < 0 || leaf >= (int64_t)r->leaves.size()) return HB_EINVAL;
  const LeafHost& L = r->leaves[leaf];
  const Problem& P = r->problems[L.problem];
  info[0] = L.problem;
  info[1] = L.t;
  info[2] = L.v;
  info[3] = L.row0 - P.row_base;
  info[4] = L.col0 - P.col_base;
  info[5] = L.m0;
  info[6] = L.n0;
  info[7] = L.rank_baca;
  info[8] = L.rank_leaf;
  info[9] = L.iters;
  info[10] = L.status;
  info[11] = (int64_t)L.tape_rows.size();
  return HB_OK;
}

hb_status hb_result_leaf_tape(const hb_result* r, int64_t leaf, int32_t* rows, int32_t* cols,
                              int32_t* dk, double* nu, double* mu) {
  if (!r || leaf < 0 || leaf >= (int64_t)r->leaves.size()) return HB_EINVAL;
  const LeafHost& L = r->leaves[leaf];
  if (L.tape_rows.size() != (size_t)L.rank_baca) return HB_EINVAL;  // no tape recorded
  if (rows) std::memcpy(rows, L.tape_rows.data(), L.tape_rows.size() * 4);
  if (cols) std::memcpy(cols, L.tape_cols.data(), L.tape_cols.size() * 4);
  if (dk) std::memcpy(dk, L.it_dk.data(), L.it_dk.size() * 4);
  if (nu) std::memcpy(nu, L.it_nu.data(), L.it_nu.size() * 8);
  if (mu) std::memcpy(mu, L.it_mu.data(), L.it_mu.size() * 8);
  return HB_OK;
}

hb_status hb_result_leaf_frozen(const hb_result* r, int64_t leaf, int32_t* stride,
                                int32_t* records) {
  if (!r || !stride || leaf < 0 || leaf >= (int64_t)r->leaves.size()) return HB_EINVAL;
  const LeafHost& L = r->leaves[leaf];
  if (r->fz_stride == 0 || L.fz.size() != (size_t)L.iters * (size_t)r->fz_stride)
    return HB_EINVAL;
  *stride = r->fz_stride;
  if (records && !L.fz.empty()) std::memcpy(records, L.fz.data(), L.fz.size() * 4);
  return HB_OK;
}

hb_status hb_result_merge_ranks(const hb_result* r, int32_t* ranks, int64_t* count) {
  if (!r || !count || !r->fz_complete) return HB_EINVAL;
  int64_t n = 0;
  for (size_t l = 0; l < r->fz_hrank.size(); ++l) {
    for (int v : r->fz_hrank[l]) {
      if (ranks) ranks[n] = v;
      ++n;
    }
    for (int v : r->fz_vrank[l]) {
      if (ranks) ranks[n] = v;
      ++n;
    }
  }
  *count = n;
  return HB_OK;
}

hb_status hb_result_error(const hb_result* r, int64_t b, int64_t stride, double* err2, double* ref2,
                          void* stream) {
  if (!r || !err2 || !ref2 || stride < 1 || b < 0 || b >= (int64_t)r->out_blocks.size())
    return HB_EINVAL;
  try {
    const Block& B = r->out_blocks[b];
    int64_t rb = 0, cb = 0;
    if (r->out_blocks.size() == r->problems.size()) {
      rb = r->problems[b].row_base;
      cb = r->problems[b].col_base;
    } else {
      rb = r->leaves[b].row0;
      cb = r->leaves[b].col0;
    }
    hipStream_t st = (hipStream_t)stream;
    DevMem mem;
    mem.st = st;
    const int64_t nrows_s = (B.m + stride - 1) / stride;
    dim3 grid((unsigned)((B.n + 255) / 256), (unsigned)std::min<int64_t>(nrows_s, 64));
    double* part = mem.get<double>((size_t)2 * grid.x * grid.y);
    const double* S = B.S;
    if (r->scalar == 0)
      hipLaunchKernelGGL((error_kernel<double>), grid, dim3(256), 0, st, r->E, rb, cb, B.m, B.n,
                         (const double*)B.U, S, (const double*)B.Vh, B.r, stride, nrows_s, part);
    else
      hipLaunchKernelGGL((error_kernel<hb_cplx>), grid, dim3(256), 0, st, r->E, rb, cb, B.m, B.n,
                         (const hb_cplx*)B.U, S, (const hb_cplx*)B.Vh, B.r, stride, nrows_s, part);
    HB_HIP(hipGetLastError());
    std::vector<double> h((size_t)2 * grid.x * grid.y);
    HB_HIP(hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, st));
    HB_HIP(hipStreamSynchronize(st));
    double e = 0, a = 0;
    for (size_t i = 0; i < h.size(); i += 2) {
      e += h[i];
      a += h[i + 1];
    }
    *err2 = e;
    *ref2 = a;
    return HB_OK;
  } catch (const HbError& e) {
    return e.st;
  }
}

void hb_result_free(hb_result* r) {
  if (!r) return;
  (void)hipDeviceSynchronize();
  delete r;
}

hb_status hb_hodlr_build(int entry_fn_id, const hb_params* params, const double* points, int64_t N,
                         int32_t nmin, double tol, int32_t d, int32_t leaf, void* stream,
                         hb_hodlr** out) {
  if (out) *out = nullptr;
  if (!out || !params || !points || N < 1 || nmin < 1) return HB_EINVAL;
  if (entry_fn_id != HB_K_GAUSS && entry_fn_id != HB_K_POLYNOMIAL) return HB_EUNSUPPORTED;
  const hb_params& P = *params;
  if (P.dim < 1 || P.dim > (entry_fn_id == HB_K_POLYNOMIAL ? HB_POLY_MAXDIM : HB_MAXDIM))
    return HB_EINVAL;
  if (!std::isfinite(P.h)) return HB_ENONFINITE;
  if (entry_fn_id == HB_K_GAUSS && (!(P.h > 0.0) || !(P.gauss_c > 0.0))) return HB_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  try {
    std::unique_ptr<hb_hodlr> H(new hb_hodlr());
    H->N = N;
    H->keep.st = st;
    H->keep.sync_free = true;
    int Lh = 0;
    while ((N + ((int64_t)1 << Lh) - 1) / ((int64_t)1 << Lh) > nmin) ++Lh;
    H->levels = Lh;
    const auto tree = cluster_tree(N, Lh);
    H->by_level.assign(Lh, {});
    for (int lev = 0; lev < Lh; ++lev)
      for (size_t i = 0; i < tree[lev].size(); ++i) {
        const Node c1 = tree[lev + 1][2 * i], c2 = tree[lev + 1][2 * i + 1];
        for (int side = 0; side < 2; ++side) {
          const Node a = side ? c2 : c1, b = side ? c1 : c2;
          H->by_level[lev].push_back((int)H->level.size());
          H->level.push_back(lev);
          H->roff.push_back(a.off);
          H->rcnt.push_back(a.size);
          H->coff.push_back(b.off);
          H->ccnt.push_back(b.size);
        }
      }
    const size_t nb = H->level.size();
    if (nb > 0) {
      CallSpec c;
      c.entry = entry_fn_id;
      c.prm = params;
      c.X = points;
      c.Y = points;
      c.nx = N;
      c.ny = N;
      c.roff = H->roff;
      c.rcnt = H->rcnt;
      c.coff = H->coff;
      c.ccnt = H->ccnt;
      c.tol = tol;
      c.d = d;
      c.leaf = leaf;
      c.st = st;
      c.batched = true;
      const hb_status bs = guarded(c, &H->blocks);
      if (bs != HB_OK) return bs;
    }
    // points as one array per coordinate for the dense leaves
    EntryDev E{};
    E.kind = entry_fn_id;
    E.dim = entry_fn_id == HB_K_POLYNOMIAL ? 0 : P.dim;
    E.pdim = entry_fn_id == HB_K_POLYNOMIAL ? P.dim : 0;
    E.poly_h = P.h;
    E.neg_inv_ch2 = entry_fn_id == HB_K_GAUSS ? -1.0 / (P.gauss_c * P.h * P.h) : 0.0;
    double* Xs = H->keep.get<double>((size_t)N * P.dim);
    hipLaunchKernelGGL(aos_to_soa_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                       points, Xs, N, P.dim);
    HB_HIP(hipGetLastError());
    E.X = Xs;
    E.Y = Xs;
    E.ldx = N;
    E.ldy = N;
    // dense diagonal leaves
    std::vector<HodlrLeafDev> lv;
    for (const Node& nd : tree[Lh]) {
      lv.push_back(HodlrLeafDev{nd.off, nd.size, H->dense_elems});
      H->dense_elems += nd.size * nd.size;
      H->leaf_off.push_back(nd.off);
      H->leaf_size.push_back(nd.size);
      H->leaf_max = std::max(H->leaf_max, nd.size);
    }
    H->nleaves = (int64_t)lv.size();
    H->dense = H->keep.get<double>((size_t)std::max<int64_t>(H->dense_elems, 1));
    HodlrLeafDev* dl = upload(H->keep, lv, st);
    H->leaves_dev = dl;
    if (H->nleaves > 65535) throw HbError{HB_EUNSUPPORTED};
    hipLaunchKernelGGL(hodlr_dense_kernel,
                       dim3((unsigned)((H->leaf_max * H->leaf_max + 255) / 256), (unsigned)H->nleaves),
                       dim3(256), 0, st, E, dl, H->dense);
    HB_HIP(hipGetLastError());
    // the low-rank blocks of each level as apply jobs
    H->jobs_dev.assign(Lh, nullptr);
    H->level_rmax.assign(Lh, 0);
    H->level_rowmax.assign(Lh, 0);
    for (int lev = 0; lev < Lh; ++lev) {
      std::vector<HodlrJob> jobs;
      for (int b : H->by_level[lev]) {
        const Block& B = H->blocks->out_blocks[b];
        HodlrJob J{};
        J.U = (const double*)B.U;
        J.Vh = (const double*)B.Vh;
        J.S = B.S;
        J.row0 = H->roff[b];
        J.rows = H->rcnt[b];
        J.col0 = H->coff[b];
        J.cols = H->ccnt[b];
        J.r = B.r;
        J.t_off = H->t_elems;
        H->t_elems += B.r;
        H->level_rmax[lev] = std::max(H->level_rmax[lev], B.r);
        H->level_rowmax[lev] = std::max<int64_t>(H->level_rowmax[lev], J.rows);
        jobs.push_back(J);
      }
      if (jobs.size() > 65535) throw HbError{HB_EUNSUPPORTED};
      H->jobs_dev[lev] = upload(H->keep, jobs, st);
    }
    HB_HIP(hipStreamSynchronize(st));
    *out = H.release();
    return HB_OK;
  } catch (const HbError& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    return HB_ENOMEM;
  } catch (...) {
    return HB_EDEVICE;
  }
}

hb_status hb_autotune(void* stream, int32_t* table, double* us) {
  try {
    const int e = hbk::tsqr_autotune((hipStream_t)stream, table, us);
    return e == 0 ? HB_OK : HB_EDEVICE;
  } catch (...) {
    return HB_EDEVICE;
  }
}

const hb_result* hb_hodlr_blocks(const hb_hodlr* h) { return h ? h->blocks : nullptr; }

int64_t hb_hodlr_nblocks(const hb_hodlr* h) { return h ? (int64_t)h->level.size() : -1; }

int64_t hb_hodlr_nleaves(const hb_hodlr* h) { return h ? h->nleaves : -1; }

hb_status hb_hodlr_block_info(const hb_hodlr* h, int64_t b, int64_t* info5) {
  if (!h || !info5 || b < 0 || b >= (int64_t)h->level.size()) return HB_EINVAL;
  info5[0] = h->level[b];
  info5[1] = h->roff[b];
  info5[2] = h->rcnt[b];
  info5[3] = h->coff[b];
  info5[4] = h->ccnt[b];
  return HB_OK;
}

hb_status hb_hodlr_matvec(const hb_hodlr* h, const double* x, double* y, void* stream) {
  if (!h || !x || !y) return HB_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  double* t = nullptr;
  if (h->t_elems > 0) {
    t = (double*)BlockCache::get().alloc((size_t)h->t_elems * 8, st);
    if (!t) return HB_ENOMEM;
  }
  hipLaunchKernelGGL(hodlr_diag_kernel,
                     dim3((unsigned)((h->leaf_max + AP_NT - 1) / AP_NT), (unsigned)h->nleaves),
                     dim3(AP_NT), 0, st, (const HodlrLeafDev*)h->leaves_dev, h->dense, x, y);
  for (int lev = 0; lev < h->levels; ++lev) {
    const unsigned nj = (unsigned)h->by_level[lev].size();
    if (nj == 0 || h->level_rmax[lev] == 0) continue;
    const HodlrJob* J = (const HodlrJob*)h->jobs_dev[lev];
    hipLaunchKernelGGL(hodlr_reduce_kernel, dim3((unsigned)h->level_rmax[lev], nj), dim3(AP_NT), 0,
                       st, J, x, t);
    hipLaunchKernelGGL(hodlr_expand_kernel,
                       dim3((unsigned)((h->level_rowmax[lev] + AP_NT - 1) / AP_NT), nj),
                       dim3(AP_NT), 0, st, J, t, y);
  }
  const hipError_t e = hipGetLastError();
  if (t) BlockCache::get().release(t, st, false);
  return e == hipSuccess ? HB_OK : HB_EDEVICE;
}

void hb_hodlr_free(hb_hodlr* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  delete h;
}

const char* hb_status_string(hb_status s) {
  switch (s) {
    case HB_OK: return "ok";
    case HB_EINVAL: return "invalid argument";
    case HB_ENOMEM: return "device allocation failed";
    case HB_EDEVICE: return "HIP call or kernel launch failed";
    case HB_ERANKCAP: return "a leaf needed more columns than rank_cap";
    case HB_ENONFINITE: return "non-finite scalar parameter";
    case HB_EUNSUPPORTED: return "size or option outside the built kernels";
  }
  return "unknown status";
}

}  // extern "C"

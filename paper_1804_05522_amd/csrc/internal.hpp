// Internal definitions shared by the HIP sources of the HODLR fractional
// diffusion library (gfx950).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hodlr_fde.h"

namespace hfde {

constexpr int kWG = 512;          // threads per work-group of the per-problem kernels
constexpr int kCoreWG = 256;      // threads of the recompression-core kernels: one wave per SIMD, so a
                                  // wave may hold 512 registers (a pivoted-Cholesky column of 64 doubles
                                  // stays in registers)
constexpr int kRS = 32;           // column stride of every off-diagonal factor array (max rank)
constexpr int kMaxLeaf = 64;      // largest leaf size b
constexpr int kLdsLeaf = kMaxLeaf + 1;   // padded leading dimension of leaf tiles in LDS
constexpr int kMaxCat = 2 * kRS;  // widest concatenation [U, P] entering a recompression
constexpr int kLdG = kMaxCat + 1; // padded leading dimension of small dense matrices in LDS
constexpr int kMaxLevels = 20;

// One HODLR problem of a batch, as the device sees it.  Rows of problem p are
// rows row0 .. row0+n-1 of every concatenated vector.
struct Item {
  int64_t n;
  int64_t row0;          // first row in concatenated vectors
  int L;                 // number of split levels; leaves live at depth L
  int kind;              // discretization: 0 Grunwald-Letnikov differences, 1 P1 finite elements
  int64_t leaf0;         // first leaf in the global leaf arrays (2^L leaves)
  int64_t node0;         // first node in the global node table (2^(L+1)-1 nodes, all depths)
  int64_t lvl0;          // offset (doubles) of this problem's per-level factor block
                         //   level d starts at lvl0 + d*n*kRS, column-major, ld = n
  int64_t g0;            // offset of g_0 in the weights array (n+3 weights)
  int64_t w0;            // offset of the Hankel factor W (nh x kRS, ld = nh)
  int64_t nh;            // Hankel size ceil(n/2)
  int64_t z0;            // offset (doubles) of this problem's hmatvec scratch
  int64_t tw0;           // offset (complex) of the twiddles e^{-2 pi i j/M}, j < M
  int64_t mu0;           // offset (complex) of the far-field multipliers, M entries
  int64_t ws0;           // offset (complex) of the FFT scratch, 2*M per column
  int64_t wsc0;          // offset (complex) of the FFT scratch of column 0 when the problems' scratch
                         //   is packed (2*M each, one column a launch)
  double alpha, nu, shift;
  double mass;           // diagonal of the matrix that the shift multiplies: 1 (identity) or 2/3 (P1 mass / h)
  double mc;             // its off-diagonals relative to the diagonal: 0 or 1/4
  double fig, fig_lo;    // finite elements: 1/Gamma(4 - alpha) as a double-double
  double tolH;           // absolute trace tolerance of the Hankel compression
  double tau;            // absolute truncation tolerance eps * (lower bound of ||M||_2)
  int k;                 // Hankel rank (set on device by the compression)
  int r;                 // off-diagonal rank of M's blocks: k + 1 (corner)
  int fftlog;            // log2 of the circulant length M used by the exact matvec
  int band;              // near-field band width w of the exact matvec
};

// Node table entry: start row (relative to the problem) and size, all depths.
// Node (d, j) of problem p lives at index node0 + (2^d - 1) + j.
struct Node {
  int32_t start;
  int32_t size;
};

// Device pointers of one built operator batch (everything lives in one
// allocation owned by the hodlr_mat handle).
struct DevPtrs {
  Item* items;
  Node* nodes;
  int32_t* rowleaf;      // per concatenated row: leaf index within its problem
  double* g;             // weights
  double* W;             // Hankel factors
  double* dplus;         // concatenated d+ samples
  double* dminus;        // concatenated d- samples
  double* Aleaf;         // input leaves, b x b column-major (identity padded)
  double* LU;            // packed leaf LU factors
  double* LUinv;         // strict lower: L^{-1} (unit), upper: U^{-1}
  int32_t* perm;         // leaf row permutation: (P^T S)[i] = S[perm[i]]
  int32_t* perminv;
  double* XL;            // M's off-diagonal left factors per level (U12 on c1 rows, U21 on c2 rows)
  double* XR;            // right factors (V21 on c1 rows, V12 on c2 rows)
  double* FL;            // L-factor blocks: U21' on c2 rows, V~21 on c1 rows
  double* FU;            // U-factor blocks: U~12 on c1 rows, V12' on c2 rows
  double* IL;            // inverse of L: Phi on c2 rows, Psi on c1 rows
  double* IU;            // inverse of U: Phi' on c1 rows, Psi' on c2 rows
  double* T1;            // factorisation temporaries (per level)
  double* T2;
  double* PP;            // pending Schur update left factors (per depth)
  double* PQ;            // pending right factors (per depth)
  double* Z;             // hmatvec scratch
  int32_t* rankL;        // per node: rank of the L-factor block (and of IL)
  int32_t* rankU;        // per node: rank of the U-factor block (and of IU)
  int32_t* rankP;        // per node: rank of the pending Schur update it was factored with
  double2* tw;           // FFT twiddles
  double2* mu;           // far-field circulant multipliers
  double2* fws;          // FFT scratch
  int32_t* status;       // per problem: hodlr_status bits
  int32_t* diag;         // per problem: [singular leaf, max rank, erank flag, k]
  int32_t fws_compact;   // 1: fws holds one column per problem at Item.wsc0 (see fws_off)
  int32_t pad_;
};

// Work lists of the multi-work-group kernels.
struct WorkUnit {          // one leaf of one problem, with the geometry the solve kernels read
  int32_t item;
  int32_t leaf;            // leaf index within the problem
  int32_t start;           // first row of the leaf within the problem
  int32_t size;            // rows of the leaf
  int64_t row0;            // the problem's first row in concatenated vectors
  int64_t lvl0;            // the problem's per-level factor offset (Item.lvl0)
  int64_t n;               // rows of the problem
  int64_t gl;              // global leaf index (Item.leaf0 + leaf)
  int64_t node0;           // the problem's first node (Item.node0)
  int32_t L;               // split levels of the problem
  int32_t pad;
};
struct NodeUnit {          // one internal node of one problem
  int32_t item;
  int32_t level;
  int32_t j;
  int32_t pad;
};
struct FftUnit {           // one (problem, column, tile) of an FFT pass
  int32_t item;
  int32_t col;
  int32_t tile;
  int32_t pad;
};
struct bf16 {              // bfloat16 storage (round to nearest even on store)
  uint16_t v;
};
// Factor arrays used by one solve: off-diagonal factors in TF, leaf inverses in TL.
template <typename TF, typename TL>
struct SolveFactors {
  const TF* IL;
  const TF* IU;
  const TL* LUinv;
};

__host__ __device__ inline int64_t node_index(const Item& it, int d, int64_t j) {
  return it.node0 + ((int64_t(1) << d) - 1) + j;
}

// First complex value of the transform scratch of (problem, column): 2*M
// values per column at ws0 + col*2M in the handle's own scratch, or, when the
// scratch is a packed buffer for single-column launches, at wsc0.
__device__ inline int64_t fws_off(const DevPtrs& P, const Item& it, int col) {
  return P.fws_compact ? it.wsc0 : it.ws0 + int64_t(col) * 2 * (int64_t(1) << it.fftlog);
}

__device__ inline double* lvl_ptr(double* base, const Item& it, int d) {
  return base + it.lvl0 + int64_t(d) * it.n * kRS;
}

// Buffer loads whose range check returns zero without a memory access: a
// wave can issue every load of a block at once and fetch only the entries a
// product uses.
constexpr int kOob = 0x7ffffff0;               // byte offset past every buffer: loads return 0

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                           int(min<int64_t>(bytes, int64_t(0x7fffffff))), 0x00020000);
}
__device__ inline float bload(__amdgpu_buffer_rsrc_t r, int off, const float*) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline double bload(__amdgpu_buffer_rsrc_t r, int off, const double*) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ inline bf16 bload(__amdgpu_buffer_rsrc_t r, int off, const bf16*) {
  return bf16{__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0)};
}

typedef double hfde_d4 __attribute__((ext_vector_type(4)));

// FP64 16x16x4 matrix-core product: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; element v of the result of lane l is D[4v + l/16][l%16].
__device__ inline hfde_d4 mfma64(double a, double b, hfde_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace hfde

// Device plan: the tables the kernels read, their layout inside the caller's
// work buffer, and the work-item vocabulary of the traversal.
//
// Work items (one workgroup each):
//   ITEM_G  (K, a, b), a >= b: block (a, b) of X_{C,C}, gathered from the
//           ancestors' X panels through the ancestor maps and written with its
//           mirror into the node's dense c x c buffer (nodes with a dense
//           buffer only).
//   ITEM_Y  (K, a, b | part << 16): rows 64a.. and columns 64b.. of GEMM-1
//           X_{C,K} = -X_{C,C} Lhat_{C,K} (Alg. 1 step 3), contraction indices
//           [part * kchunk, (part + 1) * kchunk) of the node's split.  X_{C,C}
//           comes from the dense buffer or is gathered on the fly.  Nodes
//           without an R phase store the tile into X and its share of
//           GEMM-2 directly; the others store a partial tile.
//   ITEM_R  (K, a, b | r << 16 | rq << 24): sum of a node's partial tiles
//           into X, and the row tile's share of GEMM-2 (split nodes, and
//           unsplit nodes of sparsely filled depths whose share spans several
//           64-row blocks); with rq > 1 the share is cut into rq items by
//           64-row blocks of the s x s product and item r = 0 stores the tile.
//   ITEM_D  (K, a, b), a >= b: blocks (a, b) and (b, a) of X_KK = Dt_K^{-1} -
//           Lhat_{C,K}^T X_{C,K} (step 4), symmetrized (Section 2.3).  Nodes
//           with at least kDSlabRows row tiles split each block pair into
//           64 / kDSlabW column slabs: b = block | (slab + 1) << 16.
//   ITEM_S  (K): a node with c <= 64 and s <= 64 done by one workgroup.
//   ITEM_P  (K, a, b | r << 16 | rq << 24): the row tile's share of GEMM-2
//           (step 4) for a node whose GEMM-1 tiles stored X_{C,K} directly and
//           left GEMM-2 out (level schedule, nodes with a dense X_{C,C}
//           buffer and an unsplit contraction: their GEMM-1 tiles then run in
//           a kernel of their own with fewer registers, two workgroups per
//           CU); the tile is read back from X.  rq as for ITEM_R.
//   ITEM_YU  (LU plans) the GEMM-1 tile of the upper part: rows 64a.. of
//           X_{K,C}^T = -(X_{C,C})^T Uhat_{K,C}^T into the U half of X.
// Phases of a node: 0 = ITEM_G, 1 = ITEM_Y / ITEM_YU, 2 = ITEM_R / ITEM_P, 3 = ITEM_D / ITEM_S
// (never empty).  A node's first non-empty phase becomes ready when its
// parent's phase 3 is done (C(K) lies in the ancestors, Eq. (newset)); every
// later phase becomes ready when the previous non-empty phase is done.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace selinv {

enum ItemType : int32_t { ITEM_Y = 0, ITEM_D = 1, ITEM_S = 2, ITEM_G = 3, ITEM_R = 4, ITEM_P = 5, ITEM_YU = 6 };
constexpr int kPhases = 4;
__host__ __device__ constexpr int item_phase(int type) {
  return type == ITEM_G ? 0 : (type == ITEM_Y || type == ITEM_YU) ? 1 : (type == ITEM_R || type == ITEM_P) ? 2 : 3;
}

// Work items of the adjoint (reverse) sweep; see adjoint.hip.  R1 runs
// leaves -> root, R3 root -> leaves; each is listed by etree depth and phase.
enum BackItemType : int32_t {
  BI_T = 0,   // R1 phase 0: Tbar = sym(Xbar_KK) from the stored lower triangle
  BI_G = 1,   // R1 phase 0: dense X_{C,C} gather block (nodes with a dense buffer)
  BI_Z = 2,   // R1 phase 1: Zbar = Xbar_{C,K} - Lhat Tbar
  BI_L = 3,   // R1 phase 2: Lhatbar = -(X_{C,C} Zbar + X_{C,K} Tbar)
  BI_SC = 4,  // R1 phase 2: scatter-add of -(Zbar Lhat^T + Lhat Zbar^T) into the ancestors
  BI_F = 5,   // R1 phase 2: F = Tbar E   (E = Dt^{-1})
  BI_D0 = 6,  // R1 phase 3: Dtbar0 = -E F
  BI_SG = 7,  // R3 phase 0: dense Sbar_{C,C} gather block
  BI_M = 8,   // R3 phase 1: M = Sbar_{C,C} Lhat
  BI_LB = 9,  // R3 phase 2: Lb = Lhatbar - 2 M Dt
  BI_N = 10,  // R3 phase 3: N = Lb E; Sbar_{C,K} = N / 2; GEMM-2 share of Lhat^T (M + N)
  BI_DF = 11, // R3 phase 4: Sbar_KK = sym(Dtbar0 - Lhat^T (M + N))
  BI_TINY_R1 = 12,  // (selinv_items only) all of R1 for a small node, one wavefront
  BI_TINY_R3 = 13   // (selinv_items only) all of R3 for a small node, one wavefront
};
constexpr int kBackR1Phases = 4;
constexpr int kBackR3Phases = 5;

constexpr int kTileM = 64;   // GEMM-1 rows per item
constexpr int kTileN = 64;   // columns per item (of s)
constexpr int kSmallC = 64;  // fused single-item node bounds
constexpr int kSmallNormS = 16;  // widest node normalized by the single-wavefront kernel
constexpr int kDSlabW = 16;     // column slab of a split ITEM_D
constexpr int kDSlabRows = 4;   // row tiles from which ITEM_D splits
constexpr int kSmallS = 64;

struct alignas(16) Item {
  int32_t K, type, a, b;
};

// What a traversal item reads about its node.  The level launches carry it in
// each item's record, so an item's first dependent load is its record alone.
struct alignas(16) NodeInfo {
  int32_t K, s, c, ldg;      // node, width, |C(K)|, leading dimension of its dense X_{C,C} buffer
  int32_t split, kchunk, defer2, glow;  // GEMM-1 contraction parts and their length; GEMM-2 in ITEM_P items;
                                        // glow: the dense buffer holds the lower triangle and the diagonal
                                        // 64 x 64 blocks only (its GEMM-1 reads the rest mirrored)
  int64_t off, rp, goff;     // panel offset, first row of C(K) in the row tables, dense buffer (-1: none)
  int64_t poff, yoff, pad2;  // GEMM-2 partial products, partial tiles of a split contraction
};
struct alignas(16) LRec {
  Item it;
  NodeInfo nd;
};

// Nodes small enough for one wavefront (c <= kTinyC, s <= kTinyS) skip the
// 64 x 64 tile machinery in the level schedule: one record each, in launch
// order, and a host-built table of the byte offsets of X_{C,C} in the panel
// array (c x c row-major, entry i c + k, followed by kTinyCF zeros).  The
// forward sweep of an FP64 plan takes nodes up to c <= kTinyCF that way
// (one row of X_{C,C} per lane); each depth lists its c <= kTinyC nodes
// first, and the adjoint's small-node launches cover that prefix only.
// Table entries are 32-bit byte offsets (plans whose panel array of one
// matrix spans 4 GiB or more have no single-wavefront nodes).
constexpr int kTinyC = 32;
constexpr int kTinyCF = 64;
constexpr int kTinyS = 8;
// leading dimension of the forward sweep's LDS blocks
template <typename T> __host__ __device__ constexpr int tiny_ldc() { return sizeof(T) == 8 ? kTinyCF : kTinyC; }
struct alignas(16) TinyRec {
  int32_t K, it, s, c;  // node, its item id, width, off-diagonal rows
  int64_t off, tbl;     // panel offset of the node; first table entry
};

// Control words of the persistent scheduler: an error flag and the ticket
// counter, on cache lines of their own.  Workgroups draw tickets in order;
// ticket t names the item order[t] (a topological order of the dependency
// graph, so the smallest unfinished ticket can always run).
enum Ctrl : int32_t { CTRL_ERR = 0, CTRL_TICKET = 32, CTRL_WORDS = 64 };

// Raw device pointers, valid for one (context, work buffer) pair.
struct DevPlan {
  int64_t n, ns, nitems, batch, panel_elems, sq_elems, nnzA, total_rows, part_elems;
  int32_t *node_s, *node_c;
  int64_t *node_off, *node_rowptr, *node_sq, *node_first, *node_poff;
  int64_t *kcol, *kpos;
  int32_t *posarr;
  Item *items;
  int32_t *item_ptr;   // [ns+1]
  int32_t *nph;        // [kPhases][ns] items of each phase
  int32_t *node_split; // [ns] contraction split of the GEMM-1 tiles (1 = unsplit)
  int32_t *node_kchunk;// [ns] contraction indices per split part
  int64_t *node_yoff;  // [ns] element offset of the partial tiles (split nodes)
  int64_t *node_goff;  // [ns] element offset of the dense X_{C,C} buffer (-1: gathered on the fly)
  int32_t *node_ldg;   // [ns] its leading dimension (c rounded up to 16)
  int64_t g_elems;     // dense buffers of one matrix, in scalars
  int32_t *node_parent; // [ns] supernodal etree parent (-1 at a root)
  int32_t *order;      // [batch * nitems] ticket -> l * nitems + item
  int32_t *lvl_items;  // item ids grouped by (level, phase)
  uint32_t *toff;      // X_{C,C} offset tables of the single-wavefront nodes (bit 0 set on the
                       // upper-triangle entries of a Hermitian plan: read conjugated)
  int64_t *apos;       // [nnzA] A entry -> panel element
  uint8_t *adiag;      // [nnzA]
  uint8_t *aflip;      // [nnzA] the entry lands in B's upper triangle (conjugated if Hermitian)
  double csign;        // -1: Hermitian plan (conjugate transposes), +1 otherwise
  int64_t half;        // LU plans: elements of one panel set; a matrix's panels (and X) are the L
                       // set, then the U^T set (panel_elems = 2 half); 0 otherwise
  // scratch
  void *linv;          // [batch][sq_elems] scalars
  void *dinv;          // [batch][n] scalars
  void *part;          // [batch][part_elems] GEMM-2 partial products
  void *gbuf;          // [batch][g_elems] dense X_{C,C} buffers
  void *ypart;         // [batch][y_elems] partial GEMM-1 tiles of split nodes
  int64_t y_elems;
  int32_t *cnt;        // [kPhases][batch][ns] outstanding items of each phase
  // adjoint scratch, [batch][panel_elems] each (panel layout) and
  // [batch][sq_elems] each (s x s per node, column-major); null when the work area
  // was sized without them
  void *adj_z, *adj_l, *adj_s;  // Zbar then M; Lhatbar then Lb; Sbar
  void *adj_t, *adj_f, *adj_d;  // Tbar; F; Dtbar0
  Item *bitems;        // adjoint work items
  int64_t *dpos;       // [n] panel element of each pivot D_jj (one matrix)
  unsigned long long *ferr;  // [batch] device factorization: first column with a bad pivot (~0: none)
  double *fldet;       // [batch][2] device factorization: log det (re, im)
  int32_t *ctrl;       // CTRL_WORDS
  int64_t *trace;      // optional: per ticket {item id, workgroup, t_ticket, t_start, t_end, 0, 0, 0}
};

// Kernels of the level launches.
enum LevelKind : int32_t {
  LVL_ITEMS = 0, LVL_TINY = 1, LVL_YDENSE = 2, LVL_PUSH = 3, LVL_Y128 = 4, LVL_GATHER = 5, LVL_GEMM2 = 6
};

// A tile of the left-looking (push) form, Alg. 2: supernode K pushes into the
// X panel of a descendant I (K owns rows C(I)[st, en) of I's row set).  The
// tile covers rows i0 .. i0 + 63 (C(I)-local, i0 >= st) and columns
// x0 .. x0 + 63 of X_{C(I), I}, and subtracts
//   sum over k in [st, kend) with min(i, k) < en of X_{C(I),C(I)}(i, k) Lhat_I(k, x),
// the O (i >= en), I and ID (i < en) updates of Eqs. (outerprod) and
// (innerprod); every X_{C(I),C(I)}(i, k) it reads lies in K's X panel.
// kend = en when the tile lies below R_K, else c(I).
struct alignas(16) PushRec {
  int32_t I, i0, x0, st;
  int32_t en, kend, pad0, pad1;
};

// Host-side launch lists (device pointers into the work buffer, except lvl_ptr).
struct LaunchAux {
  const int32_t *small_nodes;  // nodes with s <= kSmallNormS, normalized by one wavefront each
  int32_t nsmall;
  const int2 *chunks;       // normalization column blocks (K, 16-column block) of L_KK^{-1}, s > 64
  int32_t nchunks;
  const int2 *chunks_narrow;  // the same for 16 < s <= 64
  int32_t nchunks_narrow;
  const int2 *rblocks;      // normalization GEMM row blocks (K, 64-row block of C(K))
  int32_t nrblocks;
  const int4 *sq_tiles;     // normalization 32 x 32 tiles (K, ti, tj, 0)
  int32_t nsq_tiles;
  const int32_t *lvl_items; // item ids grouped by (level, phase)
  const LRec *lvl_recs;     // the same items' records with their nodes, in that order
  const int32_t *lvl_ptr;   // host array [nlvl + 1]
  const int32_t *lvl_tiny;  // host array [nlvl]: -1 (work items), else the first TinyRec of the range
  const int32_t *lvl_kind;  // host array [nlvl]: a LevelKind
  const int32_t *lvl_tsplit; // host array [nlvl]: a single-wavefront launch's first forward-only position, else -1
  const PushRec *push;      // push-form tiles (LVL_PUSH launches start at lvl_tiny[q])
  const Item *y128;         // 128 x 128 GEMM-1 tiles of FP64 dense-buffer nodes (LVL_Y128 launches
                            // start at lvl_tiny[q]): {K, ITEM_Y, row tile, column tile | part << 16}
  const TinyRec *tiny;      // single-wavefront node records, in launch order
  int32_t nlvl;
  const int4 *blaunch;        // host array: adjoint launches {kind, first, count, 0} in order; kind 0 =
                              // bitems [first, first + count), 1 / 2 = R1 / R3 of small-node records
  int32_t nblaunch;
  // Top of the tree: the level launches of the depths whose tiles fill at
  // most a quarter of the GPU (0: none).
  int32_t lvl_top;
  // Normalization chunks (the lists run root first): chunk q covers the level
  // launches [lvl_cut[q], lvl_cut[q + 1]) and, of list j (small, narrow,
  // chunks, rblocks, sq), the entries [norm_cut[5 q + j], norm_cut[5 (q + 1) + j]);
  // chunk 0 is the top depths.  Host arrays.
  int32_t nnorm_chunks;
  const int32_t *lvl_cut, *norm_cut;
};

// Launches of the device factorization, one entry per etree depth (deepest
// first): ranges of the lists in FactorAux.
struct FacLevel {
  int32_t nodes_b, nodes_n;    // nodes of the depth (diagonal-block factorization)
  int32_t narrow_b, narrow_n;  // 16-column blocks of L_KK^{-1}, s <= 64
  int32_t wide_b, wide_n;      // the same, s > 64
  int32_t rb_b, rb_n;          // 64-row blocks of C(K) (L_{C,K})
  int32_t tiles_b, tiles_n;    // lower 64 x 64 block pairs of C(K) x C(K) (Schur update)
};
struct FactorAux {
  const int32_t *nodes;        // device lists
  const int2 *chunks_narrow, *chunks_wide, *rblocks;
  const int4 *tiles;
  const FacLevel *lev;         // host array
  int32_t nlev;
};

// Normalization steps, for launching them separately.
enum NormSteps : int { NORM_INV = 1, NORM_GEMM = 2, NORM_SQ = 4, NORM_ALL = 7 };

}  // namespace selinv

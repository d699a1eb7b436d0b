// Internal declarations shared by the HIP translation units of libadelia.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <array>
#include <vector>

#define ADELIA_CHECK_HIP(expr)                                  \
  do {                                                          \
    hipError_t e_ = (expr);                                     \
    if (e_ != hipSuccess) return ADELIA_E_HIP;                  \
  } while (0)

typedef double v4d __attribute__((ext_vector_type(4)));

namespace adelia {

constexpr int kMaxFields = 4;
constexpr int kMaxTheta = 4 * kMaxFields + kMaxFields * (kMaxFields - 1) / 2;
constexpr int kPanel = 64;  // POTRF panel width == GEMM tile edge
// The GEMM reads each quadrant of an operand view through a buffer descriptor whose record
// count and per-lane byte offsets are 32-bit (at most kMaxOperandBytes): every operand a sweep
// forms, up to a b x (b + 65) block, must stay inside that range.  kMaxBlock is the largest
// block size for which it does (8 b (b + 65) <= kMaxOperandBytes); larger shapes are rejected
// at the entry points instead of reading zeros past the range.
constexpr long long kMaxOperandBytes = 0x7ffffff0LL;
constexpr int kMaxBlock = 16320;
static_assert(8LL * kMaxBlock * (kMaxBlock + 65) <= kMaxOperandBytes, "block limit");

// A strided view of a logical matrix split into up to four quadrants at (rs, cs):
// q = (r >= rs) + 2 * (c >= cs).  Element (r, c) of quadrant q lives at
//   p[q] + z * zs[q] + y * ys[q] + (r - rs*[r>=rs]) * sr[q] + (c - cs*[c>=cs]) * sc[q],
// where z = blockIdx.z (independent chain) and y = blockIdx.y (sub-problem).
// Transposition is expressed through the strides.
struct View {
  double* p[4];
  long long sr[4];
  long long sc[4];
  long long zs[4];
  long long ys[4];
  int rs, cs;
};

enum KRange {
  KR_FULL = 0,
  KR_GE_N0 = 1,   // op(B)(k, n) == 0 for k < n  (B lower triangular)
  KR_LT_N1 = 2,   // op(B)(k, n) == 0 for k > n  (B upper triangular)
  KR_LT_M1 = 3,   // op(A)(m, k) == 0 for k > m  (A lower triangular)
  KR_GE_MAX = 4,  // op(A) upper and op(B) lower
};

enum Tri { TRI_NONE = 0, TRI_LOWER = 1, TRI_UPPER = 2 };  // zero where col > row / row > col

enum OutMode { OUT_ALL = 0, OUT_LOWER = 1, OUT_LOWER_MIRROR = 2 };

struct GemmPhase {
  View A, B;
  int K, Klast;   // Klast: K for the last grid.y sub-problem
  int kmode;
  int triA, triB;
  double alpha;
};

// K split of the last, partial round of a launch's output tiles (launch_gemm): when the tiles
// of a one-phase launch (ny == 1) take r >= 2 rounds of the device's resident workgroups and the
// last round is at most half full, the first r - 1 rounds run as usual and the tiles of the
// last are split along K over otherwise idle workgroups, their partial tiles summed in a fixed
// order by a second launch (deterministic).  p: room for `tiles` 64 x 64 partial tiles; slots:
// resident workgroups of the GEMM kernel on the device.  p == nullptr: no split.  A workspace
// serves one stream at a time, and C must not overlap A or B.
struct TailWs {
  double* p;
  int tiles;
  int slots;
};
constexpr int kTailTiles = 512;  // partial tiles of the INLA workspaces

struct GemmArgs {
  GemmPhase ph[2];
  int nph;
  View C;
  int M, N, Mlast, Nlast;
  double beta;
  int omode;
  int tag;  // role of the launch, for the opt-in profiler (GemmTag) and the tile table
  int blk;  // block size of the sweep it belongs to (0: none): with tag, the tile table's key
  // Uneven batches: chain z takes part only while step < zn[z] (zn == nullptr: always).
  const int32_t* zn;
  int step;
  // zdiv > 0: grid.z runs over (chain, block) pairs, z = chain * zdiv + block (the views' z
  // strides are then block strides), and the pair takes part only while block < zn[chain]
  int zdiv;
  // 0: one workgroup per output tile; otherwise at most maxwg workgroups (a multiple of 8, at
  // least 8), each walking several tiles, which leaves CUs free for work on other streams
  int maxwg;
  TailWs tail;  // the last round's K split (uncapped launches only)
};

enum GemmTag { GT_OTHER = 0, GT_TRAIL, GT_TRTRI, GT_PROWS, GT_SYRK, GT_SI_W, GT_SI_Z, GT_SI_D, GT_COUNT };

// Whether grid.z index z of a launch with per-chain block counts zn (null: none) has no work:
// its chain's block count is reached at `step`, or (zdiv > 0) z names a block past it.
__host__ __device__ inline bool z_idle(const int32_t* zn, int step, int zdiv, int z) {
  if (!zn) return false;
  return zdiv > 0 ? (z % zdiv) >= zn[z / zdiv] : step >= zn[z];
}

// ---- host helpers (gemm.hip) --------------------------------------------------------------
View view_plain(double* p, long long ld, long long zstride, bool trans = false);
View view_rowsplit(double* p0, long long ld0, long long zs0, double* p1, long long ld1,
                   long long zs1, int rsplit, bool trans = false);
void view_set_y(View& v, long long ystride);
int launch_gemm(const GemmArgs& a, int ny, int nz, hipStream_t s);
// Workgroups of the one-tile-per-workgroup GEMM kernel that one CU holds at once (the runtime's
// occupancy query, made once per process; 0 if it fails).
int gemm_resident_per_cu();
// Tile edge (64 or 32) of the launches of role `tag` in sweeps of block size blk: the table the
// autotuner fills (process-wide, read when a launch is enqueued; 64 without an entry).
int tuned_tile(int blk, int tag);
void set_tuned_tile(int blk, int tag, int tile);
std::vector<std::array<int, 3>> tuned_tiles();  // entries (blk, tag, tile) other than 64
void clear_tuned_tiles();
double gemm_flops(const GemmArgs& a, int ny);  // algorithmic flops of one chain
double gemm_bytes(const GemmArgs& a, int ny);  // compulsory HBM bytes of one chain

// ---- small kernels (util.hip) -------------------------------------------------------------
int launch_fill(double* p, long long n, double v, hipStream_t s);
int launch_fill_i32(int32_t* p, long long n, int32_t v, hipStream_t s);
int launch_copy2d(const double* src, long long lds, long long zs_src, double* dst, long long ldd,
                  long long zs_dst, int rows, int cols, int nz, hipStream_t s);
int launch_zero_upper(double* p, int b, long long ld, long long blockstride, int nblk,
                      long long zs, int nz, hipStream_t s);

// ---- BTA sweeps (bta.hip) -----------------------------------------------------------------
// Uniform batch of `nz` BTA chains with identical (n, b, a).  Chain z's arrays start at
// base + z * stride.  Arrow buffers have `ap` rows (a arrow rows, plus one right-hand-side row
// when ap == a + 1).  Block t of an array with `slots` slots lives at slot t % slots.
struct BtaChains {
  int n, b, a, ap, nz;
  double* D; long long zD; int slotsD;      // in: D_t (lower) ; out: L_Dt
  long long sD;                             // slot stride of D (0: b*b)
  const double* Bin; long long zB; int slotsB;  // B_t, ld b
  double* C; long long zC;                  // n blocks ap x b (ld ap): in C_t|r_t, updated in place
  // (b+ap) x b blocks, ld b+ap: out [L_Bt; L_Ct | z_t] (the rows solved with the panels of
  // L_Dt); for the last block only rows b.. are used
  double* LBC; long long zLBC; int slotsLBC;
  double* T; long long zT;                  // ap x ap (ld ap): in T|r_T, out L_T | z_T
  double* G; long long zG; int slotsG;      // out: the 64 x 64 diagonal tiles of L_Dt^-1, and
  bool invert;                              //   all of L_Dt^-1 when invert is set
  double* ldpart; long long zLd;            // logdet partials, n*npanel + 1 per chain
  int32_t* info;                            // per chain (stride 1)
  int32_t* cnt;                             // per chain (stride 1), zero: panel write-back counters
  const int32_t* zn;                        // per chain block count (uneven batch) or nullptr
  double* scratch; long long zS;            // b*b per chain (TRTRI temporaries)
  double* zsq;                              // per chain: |z|^2 (if ap == a+1), may be null
  double* ZT; long long zZT;                // a x a per chain: [Q^-1]_{T,T} (may be null)
  double* xT; long long zXT;                // a per chain: L_T^-T z_T (may be null)
  int inv_maxwg;                            // workgroup cap of bta_invert_block's launches
  bool b_in_place;                          // B_t already assembled into the rows of [L_B; L_C]
  double* Vp; long long zVp;                // 64 x 64 per chain (split panels with look-ahead)
  // rebuild a block's factor from its stored Schur-updated diagonal block: B_i already in the
  // rows of [L_B; L_C], the arrow rows stored elsewhere (not solved again), no Schur update
  bool refactor;
  TailWs tail;  // K split of the Schur update's last round (its stream's own workspace)
};
int bta_forward(const BtaChains& c, hipStream_t s);
// Look-ahead for the block Cholesky: each panel launch first applies the previous panel's
// rank-64 update to its own columns, and the update of the columns after them runs beside the
// next panel.  Batches whose panel workgroups fit on the CUs get it in the same launch
// (launch_panel_step, consecutive steps in stream order); larger batches run it on stream ts,
// ordered by events (panel k waits for the update issued after panel k-2).
struct Lookahead {
  int maxwg;  // workgroup cap of the update part of a fused step (0: one per tile)
  int cus;    // CUs of the device: fused steps while the panel workgroups <= cus
  int slots;  // resident workgroups of the GEMM kernel on the device (cus x its occupancy)
  hipEvent_t mark;  // if not null: recorded on the sweep's stream after step (panel) mark_step
  int mark_step;
  hipStream_t ts;
  hipEvent_t pdone[3], tdone[3];
};
int bta_forward_block(const BtaChains& c, int i, hipStream_t s,
                      const Lookahead* la = nullptr);  // one block step
int bta_invert_block(const BtaChains& c, int i, hipStream_t s);   // G_i = L_Di^-1 after step i
// G = L_D^-1 for many blocks at once: nzb problems in grid.z, z = chain * zdiv + block; problem
// z's L_D, G and scratch are the b x b blocks at D + z*sD, G + z*b*b, S + z*b*b; blocks at or
// past zn[chain] are skipped (zn may be null).
int bta_invert_blocks(double* D, long long sD, double* G, double* S, int b, int nzb, int zdiv,
                      const int32_t* zn, hipStream_t s);
int bta_tip(const BtaChains& c, hipStream_t s);
int bta_logdet_reduce(const double* ldpart, long long zLd, int nparts, double* out, long long zout,
                      int nz, hipStream_t s);

struct SelinvChains {
  int n, b, a, nz;
  const double* G; long long zG; int slotsG;
  const double* LB; long long zLB; int slotsLB; int ldLB; long long sLB;  // block t at slot t % slotsLB, slot stride sLB
  const double* LC; long long zLC; int ldLC; long long sLC;  // block t at LC + t*sLC, ld ldLC, first a rows
  const double* ZT; long long zZT;               // a x a (ld a)
  double* ZD; long long zZD; int slotsZD;        // b x b blocks (full symmetric)
  double* ZB; long long zZB; int slotsZB;
  double* ZC; long long zZC; int slotsZC;        // a x b (ld a)
  double* W; long long zW; int slotsW;           // [W; V] of block t in slot t % slotsW, b*b + a*b each
  int prep_maxwg;                                // workgroup cap of selinv_prepare's launches
  int fin_maxwg;                                 // workgroup cap of selinv_finish's launches
  // W_j (the b rows of [W_j; V_j]) is formed by the caller after selinv_prepare, from
  // G_j^T G_j (W_j = L_Bj G_j = B_j D~_j^-1 = B_j G_j^T G_j, for a sparse B_j); selinv_prepare
  // then forms V_j and G_j^T G_j only
  bool w_external;
  // per chain block count of an uneven batch (nullptr: n for every chain): chain z takes part
  // in step j only while j < zn[z]; its block zn[z] - 1 has a zero coupling block (W = 0), and
  // the Z_D and Z_C slots of block zn[z] must hold zeros (finite) when step zn[z] - 1 runs
  const int32_t* zn;
  TailWs tail;  // K split of the Z_D update's last round (selinv_finish's stream's workspace)
};
// The parts of backward step j that do not depend on Z (they can run as soon as G_j exists):
// [W_j; V_j] = [L_Bj; L_Cj] G_j, and Z_Dj's lower triangle set to G_j^T G_j.
int selinv_prepare(const SelinvChains& c, int j, hipStream_t s);
// The rest of backward step j (from n-1 down to 0), after selinv_prepare(j) and with Z_D/Z_C of
// block j+1 present: [Z_Bj; Z_Cj] = -Zhat_{j+1} [W_j; V_j], Z_Dj -= [Z_Bj; Z_Cj]^T [W_j; V_j]
// (mirrored to a full symmetric block).
int selinv_finish(const SelinvChains& c, int j, hipStream_t s);
inline int selinv_block(const SelinvChains& c, int j, hipStream_t s) {
  const int r = selinv_prepare(c, j, s);
  return r ? r : selinv_finish(c, j, s);
}

// Upper triangular solve x = L^-T z (Sec. III-A-2, Eqs. 3-5), all chains.
struct SolveChains {
  int n, b, a, nz;
  const double* G; long long zG; int slotsG;
  const double* LB; long long zLB; int slotsLB; int ldLB; long long sLB;
  const double* LC; long long zLC; int ldLC; long long sLC;
  const double* z; long long zz; long long sz_blk; long long sz_elem;  // z_t element at z + t*sz_blk + r*sz_elem
  const double* xT; long long zxT;               // a
  double* x; long long zx;                        // length n*b + a (contiguous)
  double* y; long long zy;                        // scratch b
  const int32_t* zn;  // per chain block count (uneven batch; its x must start as zeros) or nullptr
  int zn_stride = 1;  // chain z of the solve reads zn[z * zn_stride]
};
int bta_upper_solve(const SolveChains& c, hipStream_t s);
// One block of it (x_i from x_{i+1} and x_T), and the tip part of x (after block 0).
int bta_upper_solve_block(const SolveChains& c, int i, hipStream_t s);
int bta_upper_solve_tip(const SolveChains& c, hipStream_t s);

// y(m) = beta*y0(m) + alpha * sum_k A(k, m) x(k) over k in [klo(m), K), A column-major (ld),
// plus optional alpha2 * sum_c A2(c, m) x2(c) (A2 is r2 x M, ld2).  klo(m) = m if lowerA.
struct GemvT {
  const double* A; long long ld; long long zA;
  const double* x; long long zx; long long incx;
  const double* A2; long long ld2; long long zA2; int r2;
  const double* x2; long long zx2;
  const double* y0; long long zy0; long long incy0;
  double* y; long long zy; long long incy;
  int M, K; int lowerA; double alpha, alpha2, beta;
  // chain z takes part only while step < zn[z * zn_stride] (zn may be null)
  const int32_t* zn; int step; int zn_stride = 1;
};
int launch_gemv_t(const GemvT& g, int nz, hipStream_t s);

}  // namespace adelia

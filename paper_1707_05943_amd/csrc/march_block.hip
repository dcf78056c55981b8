// The blocked march of Eq. (1).
//
// Update of one square (Eq. 3 for the line-1 terms, Eq. 4 bars for the
// source terms, the drive at the square's centre):
//
//   psi(j, r) = alpha psi(j-1, r) + beta(j, r)
//   beta      = cA psi(j-1, r-1) + cB psi(j, r-1) + cinv S
//             = psi(j-1, r-1) + [(cA - 1) psi(j-1, r-1) + cB psi(j, r-1) + cinv S]
// (the second form is the one evaluated: cA is close to 1, and its rounding
// would otherwise enter once per row along every characteristic)
//   S         = (G/8)[psi(j-1-D, r-1-D) + psi(j-D, r-1-D) + psi(j-1-D, r-D) + psi(j-D, r-D)]   (r-1 >= D)
//               - (G/2)[bar(-j, r-j) - bar(D-j, r-j)]                                        (r-j >= 0)
//               - (G/2)[bar(2D-j, r-j+D) - bar(D-j, r-j+D)]                                  (j > D, r-j+D >= 0)
//               + c_drive phi(x_j - t_r)[phi(-a - t_c) - phi(a - t_c)]
//
// with bar(i, rho) = [psi(i, rho) + psi(i+1, rho)]/2 and psi at columns <= 0
// the exact solution Phi[rho - i] Et[rho].  In the exact parts this gives
//   bar(-j, r-j)       = Et[r-j] (Phi[r] + Phi[r-1]) / 2
//   bar(D-j, r-j)      = Et[r-j] (Phi[r-D] + Phi[r-D-1]) / 2           (j > D)
//   bar(D-j, r-j+D)    = Et[r-j+D] (Phi[r] + Phi[r-1]) / 2            (j > D)
//   bar(2D-j, r-j+D)   = Et[r-j+D] (Phi[r-D] + Phi[r-D-1]) / 2        (j > 2D)
// while the strip (j <= D) and the near outgoing region (D < j <= 2D) read
// marched values along the anti-diagonal rho - i = r - D ("mirror" reads).
//
// Decomposition.  One launch marches a block of T rows of the outgoing
// region (columns D+1..Nx) and, one block ahead, a block of the strip
// (columns 1..D), which depends on nothing to its right.  Each workgroup
// owns a column range and marches it through the block using only values
// written by earlier launches:
//  * the outgoing region's first workgroup takes psi(D, r) from the strip
//    (already marched), so its within-row recurrence is exact;
//  * the strip's first workgroup starts from the exact column 0;
//  * every other workgroup recomputes a trapezoidal halo: at block row tau it
//    evaluates columns from c0 - (H+1)(T - tau) + 1.  Each row the halo loses
//    H+1 columns -- one to the square's left corner, H to the recurrence
//    psi = alpha psi_left + beta, whose terms beyond H columns are below
//    |alpha|^H < 2^-60 relative -- so the owned columns are exact to that
//    bound at every row;
//  * mirror reads of the strip at lags below T (only columns j < T do this)
//    come from a window in LDS that the strip's first workgroup fills from a
//    cone of columns at the strip's right end, computed the same way by its
//    second half of threads in the same row pass;
//  * all other mirror reads come from a copy of the strip stored along
//    anti-diagonals, so that the reads of one row are contiguous.
// Each workgroup runs the row loop of its region -- the strip (its delay
// corners are exact), the near outgoing region D < j <= 2D + halo (delay
// from the ring, second source mirrored), or the far region (every source
// exact) -- with the region's terms and no per-cell branching on the region.
// The kernel boundary between launches makes every write of a launch
// visible to the next one; no flags or fences are needed.

#include <string.h>

#include "fdtd_common.h"

namespace {

constexpr int NT = BM_THREADS;
constexpr int K = BM_K;
constexpr int NW = NT / 64;
constexpr int DSTAGE = 64 * K * NW + 8;        // row stage entries for a whole workgroup (64 K NW + K, padded)
constexpr int NSTAGE = BM_NEAR_CAP + 136;      // near stage: K + BM_NEAR_CAP + 1 entries, a pad of 64, 64 carry copies
constexpr int NCARRY = NSTAGE - 64;
constexpr int TBL = 1608;                  // LDS table entries (>= BM_CAP + BM_TMAX + 2, and 2 x (NT/2 K + BM_TMAX + 2))
constexpr int TBLN = BM_NEAR_CAP + BM_TMAX + 8;  // near workgroups' table entries

__device__ inline cd zero() { return mk(0.0, 0.0); }
__device__ inline int64_t dec_slot(int64_t s, int64_t R) { return s == 0 ? R - 1 : s - 1; }
__device__ inline int64_t inc_slot(int64_t s, int64_t R) { return s + 1 == R ? 0 : s + 1; }
__device__ inline int64_t slot_or_neg(int64_t rho, int64_t R) { return rho < 0 ? -1 : rho % R; }

// c ? a : b on values (a conditional between two complex lvalues would
// select their addresses and keep both in scratch memory)
__device__ __forceinline__ cd csel(bool c, const cd a, const cd b) { return mk(c ? a.re : b.re, c ? a.im : b.im); }
__device__ inline cd phi_at(const Bufs& b, int64_t q) { return q >= 0 ? b.Phi[q] : zero(); }
__device__ inline cd et_at(const Bufs& b, int64_t q) { return q >= 0 ? b.Et[q] : zero(); }

// cross-lane moves with DPP (GFX9 encodings); lanes without a source get 0
// (bound_ctrl), every row is written: the row-broadcast stages' multipliers
// are zero on the rows a broadcast must not change
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long bits = __double_as_longlong(v);
    int lo = (int)(unsigned)(bits & 0xffffffffLL), hi = (int)(bits >> 32);
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL, int RM>
__device__ __forceinline__ cd dpp_cd(cd v) { return mk(dpp_f64<CTRL, RM>(v.re), dpp_f64<CTRL, RM>(v.im)); }

constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118;
constexpr int DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143, DPP_WAVE_SHR1 = 0x138;

// Powers of alpha for the scan of psi = alpha psi_left + beta (kept in LDS):
// a[i] = alpha^i (i <= K), s[k] = alpha^(K 2^k) (k < 4), m64 = alpha^(64 K),
// and per lane l: m15 = alpha^(K((l mod 32) - 15)), m31 = alpha^(K(l - 31)),
// lp = alpha^(K l).
struct Pow {
    cd a[K + 1];
    cd s[4];
    cd m64;
    cd m15[64], m31[64], lp[64];
};

__device__ inline cd cpow_u(cd x, int e)
{
    cd r = mk(1.0, 0.0);
    while (e > 0) {
        if (e & 1) r = r * x;
        x = x * x;
        e >>= 1;
    }
    return r;
}

// by the second wave (and one thread of the third): the first forms the
// block's per-row values meanwhile
__device__ void fill_pow(cd al, Pow& p)
{
    const int t = (int)threadIdx.x - 64;
    if (t >= 0 && t < 64) {
        const cd aK = cpow_u(al, K);
        const int l32 = t & 31;
        p.m15[t] = (l32 >= 16) ? cpow_u(aK, l32 - 15) : mk(0.0, 0.0);
        p.m31[t] = (t >= 32) ? cpow_u(aK, t - 31) : mk(0.0, 0.0);
        p.lp[t] = cpow_u(aK, t);
    } else if (t == 64) {
        p.a[0] = mk(1.0, 0.0);
        for (int i = 1; i <= K; ++i) p.a[i] = p.a[i - 1] * al;
        cd m = p.a[K];
        for (int k = 0; k < 4; ++k) { p.s[k] = m; m = m * m; }
        p.m64 = cpow_u(p.a[K], 64);
    }
}

// inclusive scan over a wave of x_l = v_l + alpha^K x_{l-1}.  Inside each
// row of 16 lanes only the first `nst` doubling stages run: lane l then sums
// lanes l - 2^nst + 1 .. l of its row, the older terms carrying
// alpha^(K 2^nst) or less, below 2^-60 relative when 2^nst K exceeds the
// recurrence's horizon H.  The two row-crossing stages always run, so the
// first lanes of a row take the previous row's last lane (nst is uniform:
// the branches do not diverge).
__device__ __forceinline__ cd wave_scan(cd x, const Pow& P, int lane, int nst)
{
    if (nst > 0) x += P.s[0] * dpp_cd<DPP_ROW_SHR1, 0xF>(x);
    if (nst > 1) x += P.s[1] * dpp_cd<DPP_ROW_SHR2, 0xF>(x);
    if (nst > 2) x += P.s[2] * dpp_cd<DPP_ROW_SHR4, 0xF>(x);
    if (nst > 3) x += P.s[3] * dpp_cd<DPP_ROW_SHR8, 0xF>(x);
    x += P.m15[lane] * dpp_cd<DPP_ROW_BCAST15, 0xA>(x);
    x += P.m31[lane] * dpp_cd<DPP_ROW_BCAST31, 0xC>(x);
    return x;
}

// sum over a wave, complete in lane 63
__device__ __forceinline__ double wave_sum63(double v)
{
    v += dpp_f64<DPP_ROW_SHR1, 0xF>(v);
    v += dpp_f64<DPP_ROW_SHR2, 0xF>(v);
    v += dpp_f64<DPP_ROW_SHR4, 0xF>(v);
    v += dpp_f64<DPP_ROW_SHR8, 0xF>(v);
    v += dpp_f64<DPP_ROW_BCAST15, 0xA>(v);
    v += dpp_f64<DPP_ROW_BCAST31, 0xC>(v);
    return v;
}

struct Win {                     // the strip's right end for the rows of the current strip block
    cd (*w)[BM_TMAX];
    int64_t lo;                  // first column held
    int64_t row0;                // first row held (the block's first row)
};

// Per-row values shared by the whole workgroup (computed once per block)
struct RowInfo {
    int64_t slot;                // ring slot of row r; also the row of diagonal r - D in Md
    int64_t slot_m1;             // ring slot of row r-1; also the row of diagonal r - D - 1 in Md
    int64_t slot_pf;             // ring slot of row r+1-D (-1 if that row is before t = 0)
    cd half_pr;                  // (Phi[r] + Phi[r-1]) / 2
    cd half_qr;                  // (Phi[r-D] + Phi[r-D-1]) / 2
    cd drv;                      // drive factor of row r
    int delay_on;                // r - 1 >= D
    // far columns: S / d = g8r dsum + krc (Et[q] - Et[q+D]) + drc Phi[q]
    cd g8r;                      // cinv Gamma/8 (0 before the delay starts)
    cd krc;                      // cinv (-Gamma/2) (half_pr - half_qr)
    cd drc;                      // cinv drv
    // strip columns: their delay corners lie at x <= -a, psi = Phi Et there
    cd ga, gb;                   // g8r Et[r-1-D], g8r Et[r-D]
    cd hp;                       // cinv (-Gamma/2) half_pr
    cd psi0;                     // psi(0, r) = Phi[r] Et[r]
    cd z0, z1;                   // psi(0, r-D), psi(0, r-1-D) (zero before t = 0)
};

// A thread's column range and role.  Threads t0 .. t0+nt-1 of the workgroup
// march columns lo .. hi-1 (thread t0+i from lo + iK); the range's first
// thread takes the value left of lo as the carry (exact, or zero for a halo).
struct Seg {
    int64_t lo, hi, own_lo;      // own_lo: first column written to the ring
    int t0, w0;                  // first thread and first wave of the segment
    int exact;                   // the value left of lo is exact in every row
    int trap;                    // trapezoid: the first evaluated column moves H+1 right per row
    int write_ring, write_md, write_win, use_win;
    int64_t qa;                  // q = r - j of table entry 0
    const cd* tE;                // far: Et[q] - Et[q+D]; otherwise Et[q]
    const cd* tP;                // Phi[q]
    const cd* tE2;               // Et[q+D] (near columns)
};

// acc += a b with four fused multiply-adds
__device__ __forceinline__ void cmac(cd& acc, const cd a, const cd b)
{
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Rows staged through LDS.  Row values a workgroup needs at K columns'
// stride per lane are fetched with coalesced loads instead: the nw waves of
// a segment load entries 0 .. 64 K nw - 1 of the row (the planner keeps a
// segment's entries below that), wave v entries 64 (K v + i) + lane, and
// write them to a stage; each thread reads its K+1 entries back after a
// barrier.  Entry e reads src[clamp(e, elo, ehi)], so every load is from a
// valid address and no value is selected before it is used; entries outside
// [elo, ehi] are never used.  Stage rho holds what row rho reads.  Row r
// takes stage r before its barrier, writes stage r+2 (fetched by row r-1)
// into the same buffer after it, then its outputs, and last issues the loads
// of stage r+3.  Every fetched value is written to the stage on every path,
// unpredicated, so that when a row's stores and the next loads issue no load
// is still outstanding: the loads a row waits for are the only ones in
// flight, and they have a whole row to arrive.
__device__ __forceinline__ void stage_fetch(cd (&Rn)[K], const cd* src, int64_t elo, int64_t ehi, int v, int lane)
{
    #pragma unroll
    for (int i = 0; i < K; ++i) {
        int64_t e = 64 * (K * v + i) + lane;
        e = e < elo ? elo : (e > ehi ? ehi : e);
        const double2 x = *reinterpret_cast<const double2*>(src + e);
        Rn[i] = mk(x.x, x.y);
    }
}
template <int N>
__device__ __forceinline__ void stage_zero(cd (&Rn)[N])
{
    #pragma unroll
    for (int i = 0; i < N; ++i) Rn[i] = zero();
}
// a stage that holds every entry of the segment's waves
__device__ __forceinline__ void stage_put(cd* st, const cd (&Rn)[K], int v, int lane)
{
    #pragma unroll
    for (int i = 0; i < K; ++i)
        *reinterpret_cast<double2*>(st + 64 * (K * v + i) + lane) = make_double2(Rn[i].re, Rn[i].im);
}
// a stage that holds entries 0..n and a pad of 64 after them: entries beyond
// n land in the pad, one slot per lane
__device__ __forceinline__ void stage_put_pad(cd* st, const cd (&Rn)[K], int64_t n, int v, int lane)
{
    #pragma unroll
    for (int i = 0; i < K; ++i) {
        const int64_t e = 64 * (K * v + i) + lane;
        *reinterpret_cast<double2*>(st + (e <= n ? e : n + 1 + lane)) = make_double2(Rn[i].re, Rn[i].im);
    }
}
__device__ __forceinline__ void stage_take(cd (&dst)[K + 1], const cd* st)
{
    #pragma unroll
    for (int i = 0; i <= K; ++i) dst[i] = st[i];
}
__device__ __forceinline__ cd ld2(const cd* p)
{
    const double2 x = *reinterpret_cast<const double2*>(p);
    return mk(x.x, x.y);
}

// A wave's values of a row written with coalesced stores: lane l holds
// columns cw + K l .. cw + K l + K-1 (cw: the wave's first column); through
// the wave's own LDS slot (no barrier: one wave writes and reads it, in
// order) the wave stores columns cw + 64 i + l, those in [c_lo, c_hi].  The
// stores go through a buffer resource over the row (row_bytes long): a
// column outside the range gets an offset past the end, which the hardware
// drops, so no store sits in a branch.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int RAW_BUFFER_WORD3 = 0x00020000;     // raw (unswizzled, stride 0) buffer, 32-bit data
constexpr int OUT_OF_RANGE = 0x7ffffff0;

// Ring rows are read again D rows later.  When the grid writes more than the
// last-level cache holds in between (Plan::stream), they leave as streaming
// stores (the NT cache policy), which keeps them from filling L2 and from the
// write-back at the kernel's end; otherwise ordinary stores keep them cached
// for that read.  Stores of the diagonal copy, which the mirror reads a block
// later, stay ordinary.
constexpr int CPOL_NT = 2;
constexpr double LLC_BYTES = 256.0 * 1024 * 1024;    // MI355X last-level (Infinity) cache
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_stream(void* p, cd v)
{
    d2v x;
    x.x = v.re;
    x.y = v.im;
    __builtin_nontemporal_store(x, reinterpret_cast<d2v*>(p));
}

template <bool STREAM>
__device__ __forceinline__ void wave_store(cd* slot, const cd (&v)[K], cd* row, int row_bytes, int64_t cw,
                                           int64_t c_lo, int64_t c_hi, int lane)
{
    #pragma unroll
    for (int i = 0; i < K; ++i)
        *reinterpret_cast<double2*>(slot + K * lane + i) = make_double2(v[i].re, v[i].im);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(row, 0, row_bytes, RAW_BUFFER_WORD3);
    u32x4 x[K];
    #pragma unroll
    for (int i = 0; i < K; ++i) x[i] = *reinterpret_cast<const u32x4*>(slot + 64 * i + lane);
    #pragma unroll
    for (int i = 0; i < K; ++i) {
        const int64_t c = cw + 64 * i + lane;
        const int off = (c >= c_lo && c <= c_hi) ? (int)(c * 16) : OUT_OF_RANGE;
        __builtin_amdgcn_raw_buffer_store_b128(x[i], rs, off, 0, STREAM ? CPOL_NT : 0);
    }
    __builtin_amdgcn_wave_barrier();              // the slot is rewritten by the next row
}

// The rows of a workgroup whose every column lies beyond 2D: all source
// terms are exact (tables Et[q] - Et[q+D] and Phi[q] in LDS), the delay rows
// are the only reads of the ring.  The workgroup's range starts a halo left
// of its own columns (the trapezoid moves H+1 columns right per row), so the
// carry into its first column is zero.
template <bool STREAM>
__device__ __forceinline__ void far_rows(const Geom& g, const Bufs& b, const Pow& pw, cd (*wave_tot)[NW],
                                         const RowInfo* rinfo, double (*pe_lds)[NW], const Seg& S, int64_t ra,
                                         int64_t rb, int H1, int nst, cd (*dstage)[DSTAGE], cd* wslot)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t D = g.D, C = g.C;
    const int64_t j0 = S.lo + (int64_t)K * tid;
    const int64_t jmax = (S.hi - 1 < g.Nx) ? S.hi - 1 : g.Nx;
    const bool live = j0 <= jmax;
    const unsigned own = (unsigned)(j0 * 16);                 // byte offset of column j0 in a row
    const cd al = g.alpha, cAm1 = g.cAm1, cB = g.cB;
    cd ap[K], lp;                                             // alpha^(i+1), alpha^(K lane): read after the
                                                              // prologue's barrier (the set-up writes them)
    const cd* tE = S.tE;
    const cd* tP = S.tP;

    // ring slot sl (< 0: a row before t = 0) as a base pointer in scalar registers
    auto ring_row = [&](int64_t sl) -> const char* {
        return reinterpret_cast<const char*>(b.ring + (int64_t)uni((int)sl) * C);
    };
    // stage rho: delay row rho - D, entry s is column d0 + s (d0 = lo-1-D > D);
    // thread t reads entries Kt .. Kt+K
    const int64_t d0 = S.lo - 1 - D;
    const int64_t nd = jmax - D - d0;                         // last entry any thread uses
    const int ed = live ? K * tid : 0;
    auto fetch = [&](cd (&R)[K], int64_t sl) __attribute__((always_inline)) {
        if (uni((int)sl) < 0) stage_zero(R);
        else stage_fetch(R, reinterpret_cast<const cd*>(ring_row(sl)) + d0, 0, nd, wv, lane);
    };

    // a wave with no column in the range (and no stage entry another wave
    // reads: entry jmax-lo+1 is the last) only keeps the barrier count (and
    // zero P_e parts), leaving its SIMD to the waves that march
    if (uni((int)(j0 - K * lane > jmax + 1))) {
        __syncthreads();                                      // the prologue's
        for (int64_t r = ra; r <= rb; ++r) {
            if (lane == 63) pe_lds[r - ra][wv] = 0.0;
            __syncthreads();
        }
        return;
    }

    // the base row ra-1 (own columns and the one to the left) and delay row
    // ra-1-D, read directly; stages ra and ra+1 filled, stage ra+2 in flight
    cd up[K + 1], X[K + 1], Y[K + 1], Rn[K];
    {
        const char* rp = ring_row((ra - 1) % g.R) + own;
        const int64_t sx = slot_or_neg(ra - 1 - D, g.R);
        const cd* xp = reinterpret_cast<const cd*>(ring_row(sx < 0 ? 0 : sx)) + d0;
        #pragma unroll
        for (int i = 0; i <= K; ++i) {
            const int64_t j = j0 - 1 + i;
            up[i] = (live && j <= jmax) ? *reinterpret_cast<const cd*>(rp + 16 * (i - 1)) : zero();
            const int64_t e = ed + i;
            X[i] = ld2(xp + (e < nd ? e : nd));
        }
        if (uni((int)sx) < 0) stage_zero(X);
        cd R0[K], R1[K];
        fetch(R0, slot_or_neg(ra - D, g.R));
        if (ra + 1 <= rb) fetch(R1, slot_or_neg(ra + 1 - D, g.R));
        stage_put(dstage[0], R0, wv, lane);
        if (ra + 1 <= rb) stage_put(dstage[1], R1, wv, lane);
        if (ra + 2 <= rb) fetch(Rn, slot_or_neg(ra + 2 - D, g.R));
    }
    __syncthreads();                                          // also publishes the set-up (tables, rows, powers)
    #pragma unroll
    for (int i = 0; i < K; ++i) ap[i] = pw.a[i + 1];
    lp = pw.lp[lane];

    // row r: A holds delay row r-1-D, Bv receives row r-D from stage r
    auto step = [&](int64_t r, const cd (&A)[K + 1], cd (&Bv)[K + 1]) __attribute__((always_inline)) {
        const int tau = (int)(r - ra);
        const int par = tau & 1;
        const RowInfo& ri = rinfo[tau];
        const int64_t act_lo = S.trap ? S.lo + (int64_t)H1 * tau : S.lo;
        stage_take(Bv, dstage[par] + ed);
        // beta of the three columns
        cd p[K + 1];
        #pragma unroll
        for (int i = 0; i <= K; ++i) p[i] = A[i] + Bv[i];
        const int64_t t0 = r - j0 - S.qa;
        const cd g8r = ri.g8r, krc = ri.krc, drc = ri.drc;
        cd u[K];
        #pragma unroll
        for (int i = 0; i < K; ++i) {
            const int64_t j = j0 + i;
            cd v = up[i];                                     // cA psi(j-1, r-1) = psi(j-1, r-1) + cAm1 psi(j-1, r-1)
            cmac(v, cAm1, up[i]);
            cmac(v, cB, up[i + 1]);
            cmac(v, g8r, p[i] + p[i + 1]);
            const int64_t t = live ? t0 - i : 0;
            cmac(v, krc, tE[t]);
            cmac(v, drc, tP[t]);
            u[i] = (j >= act_lo && j <= jmax) ? v : zero();
        }
        #pragma unroll
        for (int i = 1; i < K; ++i) cmac(u[i], al, u[i - 1]);
        // carries across threads and waves
        cd x = wave_scan(u[K - 1], pw, lane, nst);
        if (lane == 63) wave_tot[par][wv] = x;
        const cd prevx = dpp_cd<DPP_WAVE_SHR1, 0xF>(x);
        __syncthreads();
        stage_put(dstage[par], Rn, wv, lane);           // stage r+2 (not read if r+2 > rb)
        cd cin = prevx;
        if (wv > 0) cmac(cin, lp, wave_tot[par][wv - 1]);
        // the row's values, the ring, P_e
        double pe = 0.0;
        up[0] = cin;
        #pragma unroll
        for (int i = 0; i < K; ++i) {
            const int64_t j = j0 + i;
            const bool act = (j >= act_lo && j <= jmax);
            cd v = u[i];
            cmac(v, ap[i], cin);
            v = act ? v : zero();
            up[i + 1] = v;
            const double m2 = norm2(v);
            pe += (j < S.own_lo || j > jmax) ? 0.0 : ((j == g.Nx) ? 0.5 * m2 : m2);
        }
        wave_store<STREAM>(wslot, *reinterpret_cast<const cd(*)[K]>(up + 1), b.ring + (int64_t)uni((int)ri.slot) * C,
                   (int)(C * 16), j0 - K * lane, S.own_lo, jmax, lane);
        pe = wave_sum63(pe);
        if (lane == 63) pe_lds[tau][wv] = pe;
        if (r + 3 <= rb) fetch(Rn, rinfo[tau + 2].slot_pf);
    };

    for (int64_t r = ra; r <= rb; r += 2) {
        step(r, X, Y);
        if (r + 1 <= rb) step(r + 1, Y, X);
    }
}

// The rows of a near workgroup (columns D+1 .. 2D + hmax, spanning at most
// BM_NEAR_CAP columns).  The delay corners are ring values (column 0, which
// only the region's first column reads, is the exact solution); the first
// source term is exact, the second reads the mirror pair psi(2D-j, q+D),
// psi(2D-j+1, q+D) from the diagonal copy for j < 2D, with psi(0, q+D)
// exact at j = 2D and both exact beyond.  The delay rows, the diagonal-copy
// rows and (first workgroup) the carry psi(D, r) pass through LDS stages.
template <bool STREAM>
__device__ __forceinline__ void near_rows(const Geom& g, const Bufs& b, const Pow& pw, cd (*wave_tot)[NW],
                                          const RowInfo* rinfo, double (*pe_lds)[NW], const Seg& S, int64_t ra,
                                          int64_t rb, int H1, int nst, cd (*dstage)[NSTAGE], cd (*mstage)[NSTAGE])
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t D = g.D, C = g.C, Mc = g.Mc;
    const int64_t j0 = S.lo + (int64_t)K * tid;
    const int64_t jmax = (S.hi - 1 < g.Nx) ? S.hi - 1 : g.Nx;
    const bool live = j0 <= jmax;
    const unsigned own = (unsigned)(j0 * 16);
    const cd al = g.alpha, cAm1 = g.cAm1, cB = g.cB;
    const cd c4 = (0.25 * g.Gamma) * g.cinv;
    cd ap[K], lp;                                             // alpha^(i+1), alpha^(K lane): read after the
                                                              // prologue's barrier (the set-up writes them)
    const cd* tE = S.tE;
    const cd* tP = S.tP;
    const cd* tE2 = S.tE2;
    const bool first = (tid == 0);
    const bool col0 = first && S.lo == D + 1;                 // reads the delay corners at column 0
    const bool carry = first && S.exact;                      // takes psi(lo-1, r) from the strip

    auto ring_row = [&](int64_t sl) -> const char* {
        return reinterpret_cast<const char*>(b.ring + (int64_t)uni((int)sl) * C);
    };
    // stage rho, delay part: delay row rho - D, entry s is column d0 + s
    // (d0 = lo-1-D >= 0); thread t reads entries Kt .. Kt+K.  Entries
    // NCARRY.. hold psi(lo-1, rho), one copy per lane (the first workgroup's
    // carry; the others load and store it too, so that no access is predicated).
    const int64_t d0 = S.lo - 1 - D;
    const int64_t nd = jmax - D - d0;
    const int ed = live ? K * tid : 0;
    // stage rho, mirror part: the Md row of diagonal rho - D, entry s is its
    // column cm + s (cm = 2D - jmax), stored K entries in; cell j0 + i reads
    // entry jmax - j0 - i (mirror psi(2D-j, .)) of stage r and entry
    // jmax - j0 - i + 1 (psi(2D-j+1, .)) of stage r-1.  Columns outside 1..D
    // are never used.
    const int64_t cm = 2 * D - jmax;
    const int64_t nm = jmax - S.lo + 1;
    const int64_t mlo = cm < 1 ? 1 - cm : 0;
    const int64_t mhi = D - cm < nm ? D - cm : nm;
    const int em = K + (live ? (int)(jmax - j0) - (K - 1) : 0);
    const unsigned cofs = (unsigned)((S.lo - 1) * 16);
    cd Rd[K], Rm[K], Rc;
    // the loads of stage rho (ring slot of delay row rho - D, row rho's slot)
    auto fetch = [&](cd (&Pd)[K], cd (&Pm)[K], cd& Pc, int64_t sd, int64_t sr) __attribute__((always_inline)) {
        if (uni((int)sd) < 0) stage_zero(Pd);
        else stage_fetch(Pd, reinterpret_cast<const cd*>(ring_row(sd)) + d0, 0, nd, wv, lane);
        stage_fetch(Pm, b.Md + (int64_t)uni((int)sr) * Mc + cm, mlo, mhi, wv, lane);
        Pc = ld2(reinterpret_cast<const cd*>(ring_row(sr) + cofs));
    };
    auto put = [&](int par, const cd (&Pd)[K], const cd (&Pm)[K], const cd& Pc) __attribute__((always_inline)) {
        stage_put_pad(dstage[par], Pd, nd, wv, lane);
        stage_put_pad(mstage[par] + K, Pm, nm, wv, lane);
        dstage[par][NCARRY + lane] = Pc;
    };

    // a wave with no column in the range (and no stage entry another wave
    // reads: entry jmax-lo+1 is the last) only keeps the barrier count (and
    // zero P_e parts), leaving its SIMD to the waves that march
    if (uni((int)(j0 - K * lane > jmax + 1))) {
        __syncthreads();                                      // the prologue's
        for (int64_t r = ra; r <= rb; ++r) {
            if (lane == 63) pe_lds[r - ra][wv] = 0.0;
            __syncthreads();
        }
        return;
    }

    // base row ra-1, delay row ra-1-D and the second mirror values of row ra
    // (Md row of diagonal ra-1-D) read directly; stages ra, ra+1 filled,
    // stage ra+2 in flight
    cd up[K + 1], X[K + 1], Y[K + 1];
    cd MB0[K], MB1[K];
    {
        const char* rp = ring_row((ra - 1) % g.R) + own;
        const int64_t sx = slot_or_neg(ra - 1 - D, g.R);
        const cd* xp = reinterpret_cast<const cd*>(ring_row(sx < 0 ? 0 : sx)) + d0;
        const cd* mp = b.Md + (int64_t)uni((int)((ra - 1) % g.R)) * Mc + cm;
        #pragma unroll
        for (int i = 0; i <= K; ++i) {
            const int64_t j = j0 - 1 + i;
            up[i] = (live && j <= jmax) ? *reinterpret_cast<const cd*>(rp + 16 * (i - 1)) : zero();
            const int64_t e = ed + i;
            X[i] = ld2(xp + (e < nd ? e : nd));
        }
        if (uni((int)sx) < 0) stage_zero(X);
        #pragma unroll
        for (int i = 0; i < K; ++i) {
            int64_t e = em - K + (K - i);                     // entry jmax - j0 - i + 1
            e = e < mlo ? mlo : (e > mhi ? mhi : e);
            MB0[i] = ld2(mp + e);
        }
        cd P0[K], P1[K], M0[K], M1[K], c0, c1;
        fetch(P0, M0, c0, slot_or_neg(ra - D, g.R), ra % g.R);
        if (ra + 1 <= rb) fetch(P1, M1, c1, slot_or_neg(ra + 1 - D, g.R), (ra + 1) % g.R);
        put(0, P0, M0, c0);
        if (ra + 1 <= rb) put(1, P1, M1, c1);
        if (ra + 2 <= rb) fetch(Rd, Rm, Rc, slot_or_neg(ra + 2 - D, g.R), (ra + 2) % g.R);
    }
    __syncthreads();                                          // also publishes the set-up (tables, rows, powers)
    #pragma unroll
    for (int i = 0; i < K; ++i) ap[i] = pw.a[i + 1];
    lp = pw.lp[lane];

    // row r: A holds delay row r-1-D, Bv receives row r-D; mB holds the
    // second mirror values of row r, mBn receives those of row r+1
    auto step = [&](int64_t r, const cd (&A)[K + 1], cd (&Bv)[K + 1], const cd (&mB)[K], cd (&mBn)[K])
                    __attribute__((always_inline)) {
        const int tau = (int)(r - ra);
        const int par = tau & 1;
        const RowInfo& ri = rinfo[tau];
        const int64_t act_lo = S.trap ? S.lo + (int64_t)H1 * tau : S.lo;
        stage_take(Bv, dstage[par] + ed);
        const cd carry0 = dstage[par][NCARRY];
        cd mA[K];
        {
            cd V[K + 1];
            stage_take(V, mstage[par] + em);
            #pragma unroll
            for (int i = 0; i < K; ++i) {
                mA[i] = V[K - 1 - i];
                mBn[i] = V[K - i];
            }
        }
        cd p[K + 1];
        #pragma unroll
        for (int i = 0; i <= K; ++i) p[i] = A[i] + Bv[i];
        if (col0) p[0] = ri.z1 + ri.z0;                      // column 0 of rows r-1-D, r-D, exact
        const int64_t t0 = r - j0 - S.qa;
        const cd g8r = ri.g8r, krc = ri.krc, drc = ri.drc, hp = ri.hp, z0 = ri.z0;
        cd u[K];
        #pragma unroll
        for (int i = 0; i < K; ++i) {
            const int64_t j = j0 + i;
            const int64_t q = r - j;
            const bool cell = (j >= act_lo && j <= jmax);
            const int64_t t = live ? t0 - i : 0;
            const cd et = tE[t], ph = tP[t], et2 = tE2[t];
            cd v = up[i];                                     // cA psi(j-1, r-1) = psi(j-1, r-1) + cAm1 psi(j-1, r-1)
            cmac(v, cAm1, up[i]);
            cmac(v, cB, up[i + 1]);
            cmac(v, g8r, p[i] + p[i + 1]);
            cmac(v, krc, et);                           // first source, exact
            cmac(v, drc, ph);
            if (j <= 2 * D) {
                // second source: -(G/2)[ (m0 + m1)/2 - Et[q+D] half_pr ], with
                // m0 = psi(0, r-D) exact at j = 2D
                const cd m0 = csel(j == 2 * D, z0, mA[i]);
                cmac(v, -c4, (q + D >= 0) ? m0 + mB[i] : zero());
                cmac(v, -hp, et2);
            } else {
                cmac(v, -krc, et2);                     // both parts exact
            }
            u[i] = cell ? v : zero();
        }
        #pragma unroll
        for (int i = 1; i < K; ++i) cmac(u[i], al, u[i - 1]);
        cd x = u[K - 1];
        if (carry) cmac(x, ap[K - 1], carry0);
        x = wave_scan(x, pw, lane, nst);
        if (lane == 63) wave_tot[par][wv] = x;
        const cd prevx = dpp_cd<DPP_WAVE_SHR1, 0xF>(x);
        __syncthreads();
        put(par, Rd, Rm, Rc);                                 // stage r+2 (not read if r+2 > rb)
        cd cin = prevx;
        if (wv > 0) cmac(cin, lp, wave_tot[par][wv - 1]);
        if (first) cin = S.exact ? carry0 : zero();
        char* wp = const_cast<char*>(ring_row(ri.slot)) + own;
        double pe = 0.0;
        up[0] = cin;
        #pragma unroll
        for (int i = 0; i < K; ++i) {
            const int64_t j = j0 + i;
            const bool act = (j >= act_lo && j <= jmax);
            cd v = u[i];
            cmac(v, ap[i], cin);
            v = act ? v : zero();
            up[i + 1] = v;
            if (act && j >= S.own_lo) {
                if constexpr (STREAM) store_stream(wp + 16 * i, v);
                else *reinterpret_cast<cd*>(wp + 16 * i) = v;
                const double m2 = norm2(v);
                pe += (j == g.Nx) ? 0.5 * m2 : m2;
            }
        }
        pe = wave_sum63(pe);
        if (lane == 63) pe_lds[tau][wv] = pe;
        if (r + 3 <= rb) fetch(Rd, Rm, Rc, rinfo[tau + 2].slot_pf, rinfo[tau + 3].slot);
    };

    for (int64_t r = ra; r <= rb; r += 2) {
        step(r, X, Y, MB0, MB1);
        if (r + 1 <= rb) step(r + 1, Y, X, MB1, MB0);
    }
}

// What a segment of strip columns does with the LDS window of the current
// block (the strip's right end, which the strip's first columns mirror at
// lags below T):
enum StripMode {
    SM_PLAIN = 0,   // no window: every mirror read is older than the block
    SM_LATE = 1,    // reads the window; column 1's pair psi(D-1, r-1), psi(D, r-1) is written by another wave
                    // after row r-1's barrier, so its term enters after row r's barrier, as alpha^(j-1)
                    // times itself in column j (the recurrence is linear)
    SM_WIN = 2,     // reads the window, every entry of it written before the row's barrier: by a one-wave cone
                    // (SM_CONE1), or by the same wave (a strip of one wave writes its own window)
    SM_CONE1 = 3    // a cone of one wave: completes each row, its window entries included, before the row's
                    // barrier (no carry from another wave is needed)
};

// The rows of a segment of strip columns (1 <= j <= D): the strip's own
// workgroups and the cone.  A strip cell's four delay corners lie at
// x <= -a, so with q = r - j they are Et[r-1-D] (Phi[q] + Phi[q-1]) and
// Et[r-D] (Phi[q+1] + Phi[q]) from the LDS table; the mirror reads
// psi(D-j, q), psi(D-j+1, q) come from the diagonal copy (its rows staged
// through LDS) or, for the strip's first columns, from the LDS window of the
// current block.  The table here starts one entry before q = S.qa + 1.
template <int MODE, bool STREAM>
__device__ __forceinline__ void strip_rows(const Geom& g, const Bufs& b, const Win& W, const Pow& pw,
                                           cd (*wave_tot)[NW], const RowInfo* rinfo, double (*pe_lds)[NW],
                                           const Seg& S, int64_t ra, int64_t rb, int H1, int T, int cone,
                                           int nst, cd (*mstage)[DSTAGE])
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t D = g.D, C = g.C, Mc = g.Mc;
    const int64_t j0 = S.lo + (int64_t)K * (tid - S.t0);
    const int64_t jmax = (S.hi - 1 < D) ? S.hi - 1 : D;
    const bool live = j0 <= jmax;
    const cd al = g.alpha, cAm1 = g.cAm1, cB = g.cB;
    const cd c4 = (0.25 * g.Gamma) * g.cinv;
    cd ap[K], lp;                                             // alpha^(i+1), alpha^(K lane): read after the
                                                              // prologue's barrier (the set-up writes them)
    const cd* tE = S.tE;
    const cd* tP = S.tP;
    const bool first = (tid == S.t0);
    // the window's column offset, and alpha^(K lane - 1) (lanes >= 1): the
    // weight of the late column-1 term in the carried value of column j0-1
    const int dwl = (int)(D - W.lo);
    cd lpm = zero();

    // stage rho: the Md row of diagonal rho - D, entry s is its column
    // cm + s (cm = D - jmax), stored K entries in, each segment in its own
    // half of the stage when the workgroup has two; cell j0 + i reads entry
    // jmax - j0 - i (psi(D-j, .)) of stage r and entry jmax - j0 - i + 1
    // (psi(D-j+1, .)) of stage r-1.  Column 0 (j = D) is exact and never read.
    const int sv = wv - S.w0;                                 // the segment's waves
    const int soff = (S.t0 ? DSTAGE / 2 : 0) + K;
    const int64_t cm = D - jmax;
    const int64_t nm = jmax - S.lo + 1;
    const int64_t mlo = cm < 1 ? 1 - cm : 0;
    const int em = soff + (live ? (int)(jmax - j0) - (K - 1) : 0);
    cd RmA[K], RmB[K];                                        // stages of even / odd rows, two rows ahead
    auto fetch = [&](cd (&R)[K], int64_t sl) __attribute__((always_inline)) {
        stage_fetch(R, b.Md + (int64_t)uni((int)sl) * Mc + cm, mlo, nm, sv, lane);
    };

    // a wave with no column in the range (and no stage entry another wave
    // reads: entry jmax-lo+1 is the last) only keeps the barrier count (and
    // zero P_e parts), leaving its SIMD to the waves that march
    if (uni((int)(j0 - K * lane > jmax + 1))) {
        __syncthreads();                                      // the prologue's
        for (int64_t r = ra; r <= rb; ++r) {
            if (lane == 63) pe_lds[r - ra][wv] = 0.0;
            __syncthreads();
        }
        return;
    }

    // base row ra-1 and the second mirror values of row ra (Md row of
    // diagonal ra-1-D) read directly; stages ra, ra+1 filled, ra+2 in flight
    cd up[K + 1];
    cd MB0[K], MB1[K];
    {
        const cd* rp = b.ring + (int64_t)uni((int)((ra - 1) % g.R)) * C;
        #pragma unroll
        for (int i = 0; i <= K; ++i) {
            const int64_t j = j0 - 1 + i;
            up[i] = (live && j <= jmax) ? (j >= 1 ? rp[j] : phi_at(b, ra - 1) * et_at(b, ra - 1)) : zero();
        }
        const cd* mp = b.Md + (int64_t)uni((int)((ra - 1) % g.R)) * Mc + cm;
        #pragma unroll
        for (int i = 0; i < K; ++i) {
            int64_t e = em - soff + (K - i);                  // entry jmax - j0 - i + 1
            e = e < mlo ? mlo : (e > nm ? nm : e);
            MB0[i] = ld2(mp + e);
        }
        cd P0[K], P1[K];
        fetch(P0, ra % g.R);
        if (ra + 1 <= rb) fetch(P1, (ra + 1) % g.R);
        stage_put(mstage[0] + soff, P0, sv, lane);
        if (ra + 1 <= rb) stage_put(mstage[1] + soff, P1, sv, lane);
        if (ra + 2 <= rb) fetch(RmA, (ra + 2) % g.R);
        if (ra + 3 <= rb) fetch(RmB, (ra + 3) % g.R);
    }
    __syncthreads();                                          // also publishes the set-up (tables, rows, powers)
    #pragma unroll
    for (int i = 0; i < K; ++i) ap[i] = pw.a[i + 1];
    lp = pw.lp[lane];
    if constexpr (MODE == SM_LATE) lpm = csel(lane > 0, pw.lp[lane > 0 ? lane - 1 : 0] * pw.a[K - 1], zero());
    // only cells j <= T - 1 read the window (row r - j inside the block): the
    // waves past them skip it (a wave-uniform branch)
    const bool wwave = (MODE == SM_LATE || MODE == SM_WIN) && uni((int)(j0 - K * lane <= T - 1));
    const int64_t R = g.R;
    int64_t sdr = ((ra - j0 + D) % R + R) % R;                  // Md row of diagonal r - j0, row by row

    auto step = [&](int64_t r, const cd (&mB)[K], cd (&mBn)[K], cd (&Rm)[K]) __attribute__((always_inline)) {
        const int tau = (int)(r - ra);
        const int par = tau & 1;
        const RowInfo& ri = rinfo[tau];
        int64_t act_lo = S.trap ? S.lo + (int64_t)H1 * tau : S.lo;
        if (cone && S.t0 != 0 && tau > T - 2) act_lo = S.hi;            // the cone stops a row early
        cd mA[K];
        {
            cd V[K + 1];
            stage_take(V, mstage[par] + em);
            #pragma unroll
            for (int i = 0; i < K; ++i) {
                mA[i] = V[K - 1 - i];
                mBn[i] = V[K - i];
            }
        }
        const cd ga = ri.ga, gb = ri.gb, hp = ri.hp, drc = ri.drc;
        const int64_t q0 = r - j0;
        const int64_t t0 = q0 - S.qa;                 // table index of q0 (entry 0 is q = S.qa)
        cd u[K];
        #pragma unroll
        for (int i = 0; i < K; ++i) {
            const int64_t j = j0 + i;
            const int64_t q = q0 - i;
            const bool cell = (j >= act_lo && j <= jmax);
            int64_t t = live ? t0 - i : 1;
            t = t < 1 ? 1 : t;                        // cells past the range read a valid entry, then drop out
            const cd pq = tP[t], pm = tP[t - 1], pp = tP[t + 1];
            const cd et = tE[t];
            cd v = up[i];                                     // cA psi(j-1, r-1) = psi(j-1, r-1) + cAm1 psi(j-1, r-1)
            cmac(v, cAm1, up[i]);
            cmac(v, cB, up[i + 1]);
            cmac(v, ga, pq + pm);
            cmac(v, gb, pp + pq);
            cmac(v, hp, et);
            cmac(v, drc, pq);
            // bar(D-j, q): the mirror pair, from the window inside the block
            // (the strip's first workgroup reads the window at a valid entry
            // for every cell, so that only values are selected).  The pair of
            // column 1, psi(D-1, r-1) and psi(D, r-1), is written after the
            // previous row's barrier: its term is added after this row's
            // barrier instead (see below).
            cd m0 = mA[i], m1 = mB[i];
            if constexpr (MODE == SM_LATE || MODE == SM_WIN) {
                if (wwave) {
                    // window row q - ra = tau - j, column D - j - W.lo (32-bit: j < NT K).
                    // Column 1 is the first cell of lane 0 only (the segment starts
                    // at column 1); column D takes the exact value below.
                    const int jj = (int)j;
                    const int wr = tau - jj;
                    const bool inwin = cell && wr >= 0;
                    const cd* wp = &W.w[0][0] + (inwin ? wr * BM_TMAX + (dwl - jj) : 0);
                    const cd w0 = wp[0], w1 = wp[1];
                    if (MODE == SM_LATE && i == 0) {
                        const bool late = (jj == 1);
                        m0 = csel(inwin, csel(!late, w0, zero()), m0);
                        m1 = csel(inwin, csel(!late, w1, zero()), m1);
                    } else {
                        m0 = csel(inwin, w0, m0);
                        m1 = csel(inwin, w1, m1);
                    }
                }
            }
            if (j == D) m0 = pq * et;                 // psi(0, q)
            cmac(v, c4, (q >= 0) ? m0 + m1 : zero());
            u[i] = cell ? v : zero();
        }
        #pragma unroll
        for (int i = 1; i < K; ++i) cmac(u[i], al, u[i - 1]);
        // carries: the first thread of an exact segment takes psi(0, r)
        cd x = u[K - 1];
        if (first && S.exact) cmac(x, ap[K - 1], ri.psi0);
        x = wave_scan(x, pw, lane, nst);
        if (lane == 63) wave_tot[par][wv] = x;
        const cd prevx = dpp_cd<DPP_WAVE_SHR1, 0xF>(x);
        if constexpr (MODE != SM_CONE1) __syncthreads();
        stage_put(mstage[par] + soff, Rm, sv, lane);          // stage r+2 (not read if r+2 > rb)
        cd cin = prevx;
        if (MODE != SM_CONE1 && wv > S.w0) cmac(cin, lp, wave_tot[par][wv - 1]);
        if (first) cin = S.exact ? ri.psi0 : zero();
        // the late term of column 1: c4 (psi(D-1, r-1) + psi(D, r-1)) enters
        // column j as alpha^(j-1) times itself (the recurrence is linear), the
        // carry cin (column j0-1) included; past the first wave of the
        // segment its weight is below alpha^(64K)
        cd late = zero(), latep = zero();
        if constexpr (MODE == SM_LATE) {
            if (S.use_win && wv == S.w0 && tau >= 1) {
                const cd* wl = W.w[tau - 1] + dwl;
                const cd pd = wl[0];
                const cd dl = c4 * (D > 1 ? wl[-1] + pd : pd);
                late = lp * dl;
                latep = lpm * dl;
            }
        }
        // outputs
        cd* rowp = b.ring + (int64_t)uni((int)ri.slot) * C;
        double pe = 0.0;
        int64_t sd = sdr;
        sdr = inc_slot(sdr, R);
        up[0] = cin + latep;
        #pragma unroll
        for (int i = 0; i < K; ++i) {
            const int64_t j = j0 + i;
            const bool act = (j >= act_lo && j <= jmax);
            cd v = u[i];
            cmac(v, ap[i], cin);
            if constexpr (MODE == SM_LATE) {
                v = v + late;
                late = late * al;
            }
            v = act ? v : zero();
            up[i + 1] = v;
            if (act && j >= S.own_lo) {
                if (S.write_ring) {
                    if constexpr (STREAM) store_stream(&rowp[j], v);
                    else rowp[j] = v;
                }
                if (S.write_md) b.Md[sd * Mc + j] = v;
                pe += norm2(v);
            }
            if (S.write_win && act && j >= W.lo) W.w[r - W.row0][j - W.lo] = v;
            sd = dec_slot(sd, R);
        }
        pe = wave_sum63(pe);
        if (lane == 63) pe_lds[tau][wv] = pe;
        if (r + 4 <= rb) fetch(Rm, rinfo[tau + 4].slot);
        // a one-wave cone's row, window entries included, is complete here:
        // the strip's next row reads it after this barrier
        if constexpr (MODE == SM_CONE1) __syncthreads();
    };

    for (int64_t r = ra; r <= rb; r += 2) {
        step(r, MB0, MB1, RmA);
        if (r + 1 <= rb) step(r + 1, MB1, MB0, RmB);
    }
}

// tables of q = r - j over a block for the columns lo..hi-1 and rows ra..rb,
// by the threads t_begin .. t_begin + t_count - 1.  A thread issues the loads
// of its first FT_UNROLL entries before it stores any of them, so the set-up
// waits for one memory round trip, not one per entry (FT_UNROLL t_count
// covers every table the planner makes: n < TBL with t_count = NT, n < TBL/2
// with t_count = NT/2, n < TBLN for the near tables); a plain loop takes any
// entries beyond.
constexpr int FT_UNROLL = 4;
static_assert(FT_UNROLL * NT >= TBL && FT_UNROLL * (NT / 2) >= TBL / 2 && FT_UNROLL * NT >= TBLN,
              "set-up tables in one round of loads");

struct TabEntry {
    cd e, p, e2;
};

// Et[q + D] is read only where a table holds it (far: Et[q] - Et[q+D]; near: tE2)
__device__ __forceinline__ TabEntry table_entry(const Bufs& b, int64_t D, int far, bool e2, int64_t q)
{
    TabEntry x;
    const cd eq = et_at(b, q), eqd = (far || e2) ? et_at(b, q + D) : zero();
    x.e = far ? eq - eqd : eq;
    x.e2 = eqd;
    x.p = phi_at(b, q);
    return x;
}

// one thread's share of a table: entries u, u + t_count, ... of qa .. qa + n,
// u = threadIdx.x - t_begin (every thread of the workgroup has one job)
struct TabJob {
    int64_t qa, n;
    cd *tE, *tP, *tE2;
    int t_begin, t_count, far;
};

__device__ __forceinline__ void tab_load(const Bufs& b, int64_t D, const TabJob& J, TabEntry (&x)[FT_UNROLL])
{
    const int u = (int)threadIdx.x - J.t_begin;
    #pragma unroll
    for (int i = 0; i < FT_UNROLL; ++i) {
        const int64_t t = u + (int64_t)i * J.t_count;
        x[i] = table_entry(b, D, J.far, J.tE2 != nullptr, J.qa + (t <= J.n ? t : 0));
    }
}

__device__ __forceinline__ void tab_store(const Bufs& b, int64_t D, const TabJob& J, const TabEntry (&x)[FT_UNROLL])
{
    const int u = (int)threadIdx.x - J.t_begin;
    #pragma unroll
    for (int i = 0; i < FT_UNROLL; ++i) {
        const int64_t t = u + (int64_t)i * J.t_count;
        if (t <= J.n) {
            J.tE[t] = x[i].e;
            J.tP[t] = x[i].p;
            if (J.tE2) J.tE2[t] = x[i].e2;
        }
    }
    for (int64_t t = u + (int64_t)FT_UNROLL * J.t_count; t <= J.n; t += J.t_count) {
        const TabEntry y = table_entry(b, D, J.far, J.tE2 != nullptr, J.qa + t);
        J.tE[t] = y.e;
        J.tP[t] = y.p;
        if (J.tE2) J.tE2[t] = y.e2;
    }
}

// LDS of a workgroup: the part its region's row loop uses, and the rest
struct FarLds {
    cd tab[2][TBL];              // Et[q] - Et[q+D], Phi[q]
    cd dstage[2][DSTAGE];        // delay rows
    cd wslot[NW][64 * K];        // each wave's row values on their way to coalesced stores
};
struct NearLds {
    cd tab[3][TBLN];             // Et[q], Phi[q], Et[q+D]
    cd dstage[2][NSTAGE];        // delay rows
    cd mstage[2][NSTAGE];        // diagonal-copy rows
};
struct StripLds {
    cd tab[2][TBL];              // Et[q], Phi[q] (the cone's in the second halves)
    cd win[BM_TMAX][BM_TMAX];    // the strip's right end over the block
    cd mstage[2][DSTAGE];        // diagonal-copy rows
};
struct Shared {
    union {
        FarLds f;
        NearLds n;
        StripLds s;
    } u;
    cd wave_tot[2][NW];
    double pe_lds[BM_TMAX][NW];
    RowInfo rinfo[BM_TMAX];
    Pow pw;
};

// Workgroup w of an instance's launch: the outgoing region over rows m0..m1
// and the strip over rows s0..s1 (either range may be empty).
template <bool STREAM>
__device__ __forceinline__ void block_body(const Geom& g, const Bufs& b, const Plan& P, int64_t m0, int64_t m1,
                                           int64_t s0, int64_t s1, int w, Shared& sh)
{
    cd(*wave_tot)[NW] = sh.wave_tot;
    double(*pe_lds)[NW] = sh.pe_lds;
    RowInfo* rinfo = sh.rinfo;
    Pow& pw = sh.pw;

    if (w >= P.nwg) return;
    const int is_strip = w < P.Gs;
    const int64_t ra = is_strip ? s0 : m0;
    const int64_t rb = is_strip ? s1 : m1;
    if (rb < ra) return;

    const int64_t D = g.D;
    int64_t c0, c1;
    int exact;
    if (is_strip) {
        c0 = 1 + (int64_t)w * P.strip_w;
        c1 = (w == P.Gs - 1) ? D + 1 : c0 + P.strip_w;
        exact = (w == 0);
    } else {
        const int m = w - P.Gs;
        if (m < P.Gn) {
            c0 = D + 1 + (int64_t)m * P.near_w;
            c1 = (m == P.Gn - 1) ? P.near_end + 1 : c0 + P.near_w;
        } else {
            const int f = m - P.Gn;
            c0 = P.near_end + 1 + (int64_t)f * P.far_w;
            c1 = (m == P.Gm - 1) ? g.Nx + 1 : c0 + P.far_w;
        }
        exact = (m == 0);
    }
    const int H1 = P.H + 1;
    const int64_t lo = exact ? c0 : c0 - P.hmax;
    const int far = (!is_strip) && (lo > 2 * D);
    const int nrows = (int)(rb - ra + 1);
    const int cone = is_strip && w == 0 && P.cone_mode == 1;
    const int use_win = is_strip && w == 0;
    cd* tab0 = far ? sh.u.f.tab[0] : (is_strip ? sh.u.s.tab[0] : sh.u.n.tab[0]);
    cd* tab1 = far ? sh.u.f.tab[1] : (is_strip ? sh.u.s.tab[1] : sh.u.n.tab[1]);
    cd* tab2 = sh.u.n.tab[2];

    // this thread's segment: the whole workgroup, or (strip workgroup 0 in
    // cone mode) the first half for its columns and the second half for the cone
    Seg S;
    S.t0 = 0;
    S.w0 = 0;
    S.lo = lo;
    S.hi = c1;
    S.own_lo = c0;
    S.exact = exact;
    S.trap = !exact;
    S.write_ring = 1;
    S.write_md = is_strip;
    S.write_win = use_win && (P.cone_mode == 0);
    S.use_win = use_win;
    S.qa = ra - (c1 - 1);
    S.tE = tab0;
    S.tP = tab1;
    S.tE2 = tab2;
    // The cone's waves follow the strip half's marching waves on the SIMDs
    // (wave w runs on SIMD w mod 4) when both fit in four: waves of the
    // second half before the cone are idle members of the strip half.
    int cone_w0 = NW / 2;
    if (cone) {
        const int a = (int)(((P.strip_w + K - 1) / K + 63) / 64);
        const int bw = (int)(((P.cone_L0 + K - 1) / K + 63) / 64);
        cone_w0 = NW / 2 + a < NW - bw ? NW / 2 + a : NW - bw;
    }
    if (cone && (int)threadIdx.x >= 64 * cone_w0) {
        S.t0 = 64 * cone_w0;
        S.w0 = cone_w0;
        S.lo = D + 1 - P.cone_L0;
        S.hi = D + 1;
        S.own_lo = D + 1;                        // nothing owned: the cone only fills the window
        S.exact = 0;
        S.trap = 1;
        S.write_ring = 0;
        S.write_md = 0;
        S.write_win = 1;
        S.use_win = 0;                           // the cone's mirror reads are older than the block
        S.qa = ra - D;
        S.tE = tab0 + TBL / 2;
        S.tP = tab1 + TBL / 2;
    }

    // tables of the block (in cone mode the two halves of the workgroup fill
    // the strip's and the cone's; strip tables reach one entry beyond each
    // end, Phi[q-1] and Phi[q+1]).  Their loads go out first; the per-row
    // values and the scan constants are formed while they are in flight.
    TabJob J;
    if (is_strip) {
        S.qa -= 1;
        const bool second = cone && (int)threadIdx.x >= NT / 2;
        J.far = 0;
        J.tE2 = nullptr;
        J.t_begin = second ? NT / 2 : 0;
        J.t_count = cone ? NT / 2 : NT;
        J.qa = second ? ra - D - 1 : ra - (c1 - 1) - 1;
        J.n = second ? P.cone_L0 + (rb - ra) + 2 : (c1 - lo) + (rb - ra) + 2;
        J.tE = second ? tab0 + TBL / 2 : tab0;
        J.tP = second ? tab1 + TBL / 2 : tab1;
    } else {
        J.far = far;
        J.tE2 = far ? nullptr : tab2;
        J.t_begin = 0;
        J.t_count = NT;
        J.qa = ra - (c1 - 1);
        J.n = (c1 - lo) + (rb - ra);
        J.tE = tab0;
        J.tP = tab1;
    }
    TabEntry tx[FT_UNROLL];
    tab_load(b, D, J, tx);
    const int64_t slot_a = ra % g.R;                 // one (scalar) division; R > D + 1 and nrows <= R
    if (threadIdx.x < nrows) {
        const int64_t r = ra + threadIdx.x;
        RowInfo ri;
        ri.slot = slot_a + threadIdx.x < g.R ? slot_a + threadIdx.x : slot_a + threadIdx.x - g.R;
        ri.slot_m1 = dec_slot(ri.slot, g.R);
        const int64_t spf = ri.slot + 1 - D;          // (r + 1 - D) mod R, from r mod R
        ri.slot_pf = (r + 1 - D < 0) ? -1 : (spf < 0 ? spf + g.R : spf);
        ri.half_pr = 0.5 * (phi_at(b, r) + phi_at(b, r - 1));
        ri.half_qr = 0.5 * (phi_at(b, r - D) + phi_at(b, r - D - 1));
        ri.drv = b.Drv[r];
        ri.delay_on = (r - 1 >= D);
        ri.g8r = ri.delay_on ? (0.125 * g.Gamma) * g.cinv : zero();
        ri.krc = g.cinv * ((-0.5 * g.Gamma) * (ri.half_pr - ri.half_qr));
        ri.drc = g.cinv * ri.drv;
        ri.ga = ri.g8r * et_at(b, r - 1 - D);
        ri.gb = ri.g8r * et_at(b, r - D);
        ri.hp = g.cinv * ((-0.5 * g.Gamma) * ri.half_pr);
        ri.psi0 = phi_at(b, r) * et_at(b, r);
        ri.z0 = phi_at(b, r - D) * et_at(b, r - D);
        ri.z1 = phi_at(b, r - 1 - D) * et_at(b, r - 1 - D);
        rinfo[threadIdx.x] = ri;
    }
    fill_pow(g.alpha, pw);
    tab_store(b, D, J, tx);
    // no barrier here: the row loops' prologues issue their loads first and
    // their barrier publishes these tables, rows and powers as well

    Win W;
    W.w = sh.u.s.win;
    W.lo = P.win_lo;
    W.row0 = ra;

    cd* wslot = sh.u.f.wslot[threadIdx.x >> 6];
    // the window's writer completes its rows before their barriers when it is
    // one wave: a cone of at most 64 K columns, or a strip of one workgroup
    // whose D columns fit one wave (it writes its own window)
    const int one_wave_cone = cone && (P.cone_L0 + K - 1) / K <= 64;
    const int one_wave_strip = is_strip && P.cone_mode == 0 && (D + K - 1) / K <= 64;
    if (far) far_rows<STREAM>(g, b, pw, wave_tot, rinfo, pe_lds, S, ra, rb, H1, P.nst, sh.u.f.dstage, wslot);
    else if (is_strip) {
        if (use_win && S.t0 == 0) {
            if (one_wave_cone || one_wave_strip)
                strip_rows<SM_WIN, STREAM>(g, b, W, pw, wave_tot, rinfo, pe_lds, S, ra, rb, H1, P.T, cone, P.nst, sh.u.s.mstage);
            else
                strip_rows<SM_LATE, STREAM>(g, b, W, pw, wave_tot, rinfo, pe_lds, S, ra, rb, H1, P.T, cone, P.nst, sh.u.s.mstage);
        } else if (one_wave_cone && S.t0 != 0) {
            strip_rows<SM_CONE1, STREAM>(g, b, W, pw, wave_tot, rinfo, pe_lds, S, ra, rb, H1, P.T, cone, P.nst, sh.u.s.mstage);
        } else {
            strip_rows<SM_PLAIN, STREAM>(g, b, W, pw, wave_tot, rinfo, pe_lds, S, ra, rb, H1, P.T, cone, P.nst, sh.u.s.mstage);
        }
    } else near_rows<STREAM>(g, b, pw, wave_tot, rinfo, pe_lds, S, ra, rb, H1, P.nst, sh.u.n.dstage, sh.u.n.mstage);
    __syncthreads();
    if (threadIdx.x < nrows) {
        const int tau = threadIdx.x;
        const int64_t r = ra + tau;
        double tot = 0.0;
        for (int w2 = 0; w2 < (cone ? NW / 2 : NW); ++w2) tot += pe_lds[tau][w2];
        if (is_strip && w == 0) {
            const cd v0 = b.Phi[r] * b.Et[r];
            tot += 0.5 * norm2(v0);
        }
        b.Ppart[r * P.nwg + w] = tot;
    }
}

template <bool STREAM>
__device__ __forceinline__ void block_entry(const Geom& g, const Bufs& b, const Plan& P, int64_t m0, int64_t m1,
                                            int64_t s0, int64_t s1)
{
    __shared__ Shared sh;
    const int bid = blockIdx.x;
    // neighbouring column ranges share an XCD; the strip's first workgroup,
    // which ends every launch, takes the last slot of the last XCD, away from
    // the other strip workgroups' diagonal-copy traffic on the first
    // (measured: 66.8-67.1 -> 65.9 us per launch on the D=10000 grid)
    int w = (bid % 8) * (P.nb / 8) + bid / 8;
    if (w == 0) w = P.nb - 1;
    else if (w == P.nb - 1) w = 0;
    block_body<STREAM>(g, b, P, m0, m1, s0, s1, w, sh);
}

// one instance, ring rows as streaming stores (Plan::stream: grids whose
// rows leave the last-level cache before they are read again)
__global__ __launch_bounds__(BM_THREADS) void k_block(Geom g, Bufs b, Plan P, int64_t m0, int64_t m1,
                                                       int64_t s0, int64_t s1)
{
    block_entry<true>(g, b, P, m0, m1, s0, s1);
}

// one instance, ordinary ring stores (rows still cached when read again)
__global__ __launch_bounds__(BM_THREADS) void k_block_cached(Geom g, Bufs b, Plan P, int64_t m0, int64_t m1,
                                                              int64_t s0, int64_t s1)
{
    block_entry<false>(g, b, P, m0, m1, s0, s1);
}

// Many instances in one launch: launch k advances every instance whose march
// needs more than k launches (a prefix of the table, which is sorted by that
// count) by one block.  Workgroup ids are laid out instance after instance
// (tab[i].wg_begin) and dealt to the XCDs in contiguous runs, as above.
__global__ __launch_bounds__(BM_THREADS) void k_block_batch(const BInst* __restrict__ tab, int n_active, int64_t k,
                                                             int nb)
{
    __shared__ Shared sh;
    const int bid = blockIdx.x;
    const int64_t wgl = (int64_t)(bid % 8) * (nb / 8) + bid / 8;
    int lo = 0, hi = n_active - 1;
    while (lo < hi) {                                    // last instance with wg_begin <= wgl
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].wg_begin <= wgl) lo = mid; else hi = mid - 1;
    }
    const BInst& e = tab[lo];
    const int w = (int)(wgl - e.wg_begin);
    if (w >= e.P.nwg || k >= e.launches) return;
    int64_t m0, m1, s0, s1;
    block_rows(e.P.T, e.g.Nt, k, &m0, &m1, &s0, &s1);
    block_body<false>(e.g, e.b, e.P, m0, m1, s0, s1, w, sh);
}

}  // namespace

int launch_block(fdtd_ctx* c, int64_t m0, int64_t m1, int64_t s0, int64_t s1)
{
    if (c->plan.stream)
        hipLaunchKernelGGL(k_block, dim3(c->plan.nb), dim3(BM_THREADS), 0, c->stream, c->g, c->b, c->plan, m0, m1, s0,
                           s1);
    else
        hipLaunchKernelGGL(k_block_cached, dim3(c->plan.nb), dim3(BM_THREADS), 0, c->stream, c->g, c->b, c->plan, m0,
                           m1, s0, s1);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_block_batch(const BInst* d_tab, int n_active, int64_t k, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_block_batch, dim3(nb), dim3(BM_THREADS), 0, s, d_tab, n_active, k, nb);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

// Planner: rows per block T, halo, and the split of the columns into
// workgroups of about equal cost (columns with mirror reads -- the strip and
// the near part of the outgoing region -- count MIRROR_COST times a far
// column), about kn.ncu workgroups (one per compute unit for an instance that
// runs alone; an instance of a batch asks for the widest workgroups).
static const double MIRROR_COST = 3.5;
// the widest column range of a workgroup (one segment) and of each half of
// the strip's first workgroup: the row stages hold one entry less than the
// threads' columns
static const int64_t SPAN_CAP = BM_CAP - 1;
static const int64_t HALF_CAP = (int64_t)(BM_THREADS / 2) * BM_K - 1;

int make_plan(const fdtd_params* p, int H, const PlanKnobs& kn, Plan* out, char* why, size_t n)
{
    const int64_t D = p->D, Nx = p->Nx;
    const int NCU = kn.ncu < 1 ? 1 : kn.ncu;
    const int targets[] = {32, 24, 16, 12, 8, 6, 4, 3, 2, 1};
    for (int T : targets) {
        if (T > BM_TMAX || T > kn.tmax || T > D) continue;
        Plan P;
        memset(&P, 0, sizeof P);
        P.T = T;
        P.H = H;
        P.hmax = (H + 1) * T - 1;
        int64_t room = SPAN_CAP - P.hmax;               // owned columns a halo workgroup can hold
        if (room < 64) continue;
        // a narrower cap, but never below twice the halo
        const int64_t cap = kn.wmax > 2 * (int64_t)P.hmax ? kn.wmax : 2 * (int64_t)P.hmax;
        if (cap < room) room = cap;
        // the near part ends where far workgroups' halos hold no mirror reads
        P.near_end = 2 * D + P.hmax;
        if (P.near_end > Nx) P.near_end = Nx;
        const int64_t near_cols = P.near_end - D;
        const int64_t far_cols = Nx - P.near_end;
        // widths: at least twice the halo, at most what a workgroup holds
        int64_t minw = 2 * (int64_t)P.hmax;
        if (minw < 64) minw = 64;
        if (minw > room) minw = room;
        if (BM_NEAR_CAP - (int64_t)P.hmax < minw) continue;
        double budget = (MIRROR_COST * (double)(D + near_cols) + (double)far_cols) / NCU;
        int ok = 0;
        for (int it = 0; it < 2000; ++it, budget *= 1.02) {
            int64_t wm = (int64_t)(budget / MIRROR_COST), wf = (int64_t)budget;
            if (wm < minw) wm = minw;
            if (wf < minw) wf = minw;
            if (wm > room) wm = room;
            if (wf > room) wf = room;
            // strip
            P.cone_L0 = T + (int64_t)H * (T - 1);
            const int can_cone = (D + 1 - P.cone_L0 >= T) && (P.cone_L0 <= HALF_CAP);
            if (D <= SPAN_CAP && (D <= wm + wm / 2 || !can_cone)) {
                P.cone_mode = 0;
                P.Gs = 1;
                P.strip_w = D;
            } else if (can_cone) {
                P.cone_mode = 1;
                // the strip's first workgroup holds its columns in half its threads
                const int64_t ws = wm < HALF_CAP ? wm : HALF_CAP;
                int64_t Gs = (D + ws - 1) / ws;
                if (Gs < 2) Gs = 2;
                P.strip_w = (D + Gs - 1) / Gs;
                P.Gs = (int)((D + P.strip_w - 1) / P.strip_w);
                if (P.strip_w + 1 - P.hmax < T) break;            // halo mirror reads must be older than the block
                // the strip's first workgroup holds its columns and the cone in one half each
                if (P.strip_w > HALF_CAP || P.cone_L0 > HALF_CAP) break;
                if (D - (int64_t)(P.Gs - 1) * P.strip_w + P.hmax > SPAN_CAP) break;
            } else {
                break;
            }
            // near part (the first near workgroup needs no halo); a near
            // workgroup spans at most BM_NEAR_CAP columns with its halo
            int64_t wn = wm;
            if (wn > BM_NEAR_CAP - (int64_t)P.hmax) wn = BM_NEAR_CAP - (int64_t)P.hmax;
            int64_t Gn = (near_cols + wn - 1) / wn;
            if (Gn < 1) Gn = 1;
            P.near_w = (near_cols + Gn - 1) / Gn;
            P.Gn = (int)((near_cols + P.near_w - 1) / P.near_w);
            // far part
            int64_t Gf = (far_cols > 0) ? (far_cols + wf - 1) / wf : 0;
            P.far_w = Gf ? (far_cols + Gf - 1) / Gf : 1;
            Gf = Gf ? (far_cols + P.far_w - 1) / P.far_w : 0;
            P.Gm = P.Gn + (int)Gf;
            P.nwg = P.Gs + P.Gm;
            if (P.near_w > room && P.Gn > 1) continue;
            if (P.far_w > room) continue;
            if (P.nwg <= NCU || (wm >= room && wf >= room)) { ok = 1; break; }
        }
        if (!ok) continue;
        // halos start right of column 0
        if (P.Gn > 1 && D + 1 + P.near_w - P.hmax < 1) continue;
        P.win_lo = D - T + 1 < 1 ? 1 : D - T + 1;
        // scan stages inside a row of 16 lanes: a lane needs the carries of
        // ceil(H / K) lanes to its left
        const int look = (H + BM_K - 1) / BM_K;
        P.nst = 0;
        while (P.nst < 4 && (1 << P.nst) < look + 1) ++P.nst;
        P.nb = ((P.nwg + 7) / 8) * 8;
        // streaming ring stores when the rows written between a row's store
        // and its re-read D rows later exceed the last-level cache
        P.stream = kn.stream_ok && (double)D * (double)(Nx + 1) * 16.0 > LLC_BYTES;
        *out = P;
        return FDTD_OK;
    }
    snprintf(why, n, "no block decomposition fits (D=%lld, Nx=%lld, halo %d per row)", (long long)D,
             (long long)Nx, H + 1);
    return FDTD_EINVAL;
}

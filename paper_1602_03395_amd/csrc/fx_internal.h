// Internal declarations shared by the host runtime (fx.cpp, tables.cpp) and the
// HIP kernels (kernels.hip). Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/fx.h"

namespace fx {

constexpr int kMaxStages = 24;     // radix stages of one in-LDS transform
constexpr int kThreads = 256;      // threads per workgroup of every pass kernel
constexpr int kMaxTilePoints = 4096;  // TS * M of one tile (accumulator registers cap)

// Mixed-radix factorisation of one transform length (Stockham, natural order out).
struct RadixPlan {
    int n = 1;
    int nst = 0;
    int rad[kMaxStages] = {0};
};

RadixPlan make_radix_plan(int n);

// Per-axis device view of the method's tables, for data type T (float or double).
// Table layout: [lam][M] complex, row q.
//   TA[q][n]  = exp(-i alpha_q (x_n - a))                         (presA premultiply)
//   TB[q][m]  = exp(i k_m (abar - a - (k_m + 2 alpha_q) hbar t/2m))  (presB chirp, umklapp applied)
//   Tf[q][nb] = (1/lam) exp(i alpha_q (xbar_nb - a - alpha_q hbar t/2m))  (presf twiddle)
//   tw[k]     = exp(-2 pi i k / M), k < M                         (FFT roots)
struct AxisDev {
    const void* TA = nullptr;
    const void* TB = nullptr;
    const void* Tf = nullptr;
    const void* tw = nullptr;
    const void* HT = nullptr;  // [lam][P][g] chirp-folded table of the register E kernel (or null)
    const void* HTx = nullptr; // HT arranged for the select-free first reduction step (or null)
    const void* HTl = nullptr; // [lam][g][P] (each lane's P values contiguous): for power-of-two
                               // P <= min(g, 8) row n2 turned by bitrev(n2 mod P), else HTx reordered
    int M = 1;        // axis length
    int P = 1;        // M / g: number of distinct n'' values (output-pruned length)
    int g = 1;        // gcd(lam, M)
    int lam = 1;
    int lg = 1;       // (lam / g) mod P: n'' = g * ((nb * lg) mod P)
    int lg_inv = 0;   // inverse of lg modulo P: nb0(r) = (r * lg_inv) mod P
    double scale = 1; // 1 / M
    RadixPlan fm;     // radix plan of length M
    RadixPlan fp;     // radix plan of length P
    RadixPlan fg;     // radix plan of length g (structured accumulate)
};

// Geometry of one pass along an axis of a tensor laid out as [Qin][A][L][S].
struct PassGeom {
    int64_t Qin = 1;   // leading slice count of the input
    int64_t A = 1;     // product of the lengths before the axis
    int64_t S = 1;     // product of the lengths after the axis (stride of the line)
    int qb = 0;        // first magnification index handled along this axis
    int qn = 1;        // number of magnification indices handled
    int TS = 1;        // lines per workgroup tile
    int64_t ntiles = 1;  // tiles per (slice, q)
    int max_blocks = 0;  // persistent grid: cap on workgroups (0 = one per tile)
    int qc = 0;        // > 0: register E kernel, magnification indices per workgroup
    bool reg_a = false;  // A pass: register structured accumulate
    bool eas = false;    // EA pass: waves share the terms of 64 / g lines, structured accumulate
    bool eaw = false;    // EA pass (g = 8): one wave per tile of 8 lines, every term, structured accumulate
    bool erw = false;    // E pass (g = 8, P = 16..64, contiguous lines): register form, a line per 8 P / V lanes
    bool erg = false;    // E, EA or EH pass (g = 2, 4, 8; P = 16..64): register form, a line per g P / 8 lanes
    bool eh2 = false;    // EH pass: compile-time power-of-two kernel, one output line per workgroup
};

enum class Kind { E, A, EA, EH, AH, EAH, AA, AAH };

// Groups per tile of the structured accumulate (A via a g-point transform over q mod g).
int as_tile_groups(int g);
size_t as_lds_bytes(bool dbl, int g, int M);

struct KernelCfg {
    int ts_target = 2048;  // preferred TS*L points per tile
};

// Kernel launchers (kernels.hip). All return hipSuccess or the launch error.
hipError_t launch_pass(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax,
                       const PassGeom& g, int accumulate, void* rho, hipStream_t st);
hipError_t launch_density(bool dbl, const void* psi, void* rho, int64_t n, hipStream_t st);
hipError_t launch_column(bool dbl, const void* rho, void* img, int64_t A, int64_t L, int64_t S,
                         double w, hipStream_t st);
hipError_t launch_gather(bool dbl, const void* const* srcs, void* dst, int64_t n_each, int count,
                         hipStream_t st);
hipError_t launch_scatter(bool dbl, const void* src, void* const* dsts, int64_t n_each, int count,
                          int want_rho, void* const* rhos, hipStream_t st);
size_t pass_lds_bytes(Kind kind, bool dbl, int TS, int M);
// Compile-time specialised E / EA kernels for power-of-two axes of 8..2048 points (kernels_p2.hip):
// they always take tiles of p2_tile_lines(M) lines.
bool p2_applicable(Kind kind, int M);
int p2_tile_lines(int M);
size_t p2_lds_bytes(Kind kind, bool dbl, int M);
hipError_t launch_pass_p2(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                          int accumulate, void* rho, hipStream_t st);
// Compile-time EH (adjoint of E) for power-of-two axes of 256..2048 points (kernels_p2.hip): one
// output line per workgroup, 2048 / M terms transformed together.
bool eh2_applicable(int M, int P);
size_t eh2_lds_bytes(bool dbl, int M);
hipError_t launch_pass_eh2(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                           int accumulate, hipStream_t st);
// Compile-time E / EA kernels for axis lengths 3 * 2^k, 12..1536 (kernels_ct.hip), tiles of
// ct_tile_lines(M) lines.
bool ct_applicable(Kind kind, int M);
int ct_tile_lines(int M);
size_t ct_lds_bytes(Kind kind, bool dbl, int M);
hipError_t launch_pass_ct(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                          int accumulate, void* rho, hipStream_t st);
int lds_limit_bytes();

// Host-built FP64 tables (tables.cpp).
struct AxisTables {
    std::vector<double> TA, TB, Tf, tw;  // interleaved re,im; [lam][M] for TA/TB/Tf, [M] for tw
    std::vector<double> HT;              // [lam][P][g] when requested, else empty
    std::vector<double> HTx;             // HT for odd n2 lanes swapped or sign-modulated (see build_ht)
    std::vector<double> HTl;             // [lam][g][P], rows turned for the rotated reduction (see build_ht)
};
struct AxisParams {
    int64_t M = 1;
    int lam = 1;
    double dx = 1, a = 0, abar = 0;
    double t = 0, m_over_hbar = 1;
    // Optional spectrum: phase[i] = t * omega(kappa_l) in radians for the fine wave
    // number l = i - floor(lam M / 2); NULL keeps hbar t kappa^2 / 2m.
    const double* phase = nullptr;
    bool want_ht = false;  // also build the chirp-folded table HT
};
AxisTables build_axis_tables(const AxisParams& p);

// Register E kernel (output-pruned transform with the chirp folded into HT, kernels_cfp.hip).
bool cfp_applicable(Kind kind, bool dbl, int M, int g);
int cfp_tile_lines(int g);
size_t cfp_lds_bytes(bool dbl, int M, int g);
hipError_t launch_pass_cfp(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                           int accumulate, void* rho, hipStream_t st);
// The last two accumulate passes of the paper schedule fused (axes u < v): input
// [O][qn_v][qn_u][X][P_u][Y][P_v][Z] -> output [O][X][M_u][Y][M_v][Z].
struct AAGeom {
    int64_t O = 1, X = 1, Y = 1, Z = 1;
    int qn_u = 1, qb_u = 0, qn_v = 1, qb_v = 0;
    int tsg = 1;  // groups per workgroup
};
bool aa_applicable(bool dbl, int gu, int gv);
// Register form of the fused pass (k_AAR): g_u = g_v = 16 or 32, axes u, v the last two (Y = Z = 1).
bool aar_applicable(int gu, int gv, int Pu, int Pv, const AAGeom& g);
// Its adjoint (k_AAHR): the first two AH passes of the adjoint schedule fused, same conditions.
hipError_t launch_pass_aah(bool dbl, const void* in, void* out, const AxisDev& au, const AxisDev& av,
                           const AAGeom& g, int accumulate, hipStream_t st);
int aa_tile_groups(int gu, int gv);
size_t aa_lds_bytes(bool dbl, int gu, int gv);
hipError_t launch_pass_aa(bool dbl, const void* in, void* out, const AxisDev& au, const AxisDev& av, const AAGeom& g,
                          int accumulate, void* rho, hipStream_t st);
// EA in register form with the structured accumulate (power-of-two P <= g, 8 <= g <= 64, P <= 16):
// 64 / g lines per workgroup, its waves share the terms.
bool eas_applicable(bool dbl, int M, int g, int qn);
int eas_tile_lines(int g);
hipError_t launch_pass_eas(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                           void* rho, hipStream_t st);
// Register E and EA with a line over g P / 8 lanes (g = 2, 4, 8; P = 16, 32, 64; any line stride).
bool erg_applicable(bool dbl, int M, int g);
int erg_tile_lines(int M, int g);
size_t erg_lds_bytes(bool dbl, Kind kind, int M, int g, int qc, int qn, bool strided);
hipError_t launch_pass_erg(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                           int accumulate, void* rho, hipStream_t st);
// Its adjoint (EH) in the same lane layout.
size_t ehg_lds_bytes(bool dbl, int M, int g, int qn, bool strided);
hipError_t launch_pass_ehg(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                           hipStream_t st);

// Register E with 8 P / V lanes per line (g = 8, P = 16, 32, 48, 64, contiguous lines; kernels_cfp.hip).
bool erw_applicable(bool dbl, int M, int g);
int erw_tile_lines(int P);
size_t erw_lds_bytes(bool dbl, int P, int qc);
hipError_t launch_pass_erw(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g, hipStream_t st);

// EA in register form with the structured accumulate for g = 8 and P in {2, 3, 4, 6, 8}: one wave
// per tile of 8 lines running every term, the partial sums over q mod 8 in registers.
bool eaw_applicable(bool dbl, int M, int g, int qn);
int eaw_tile_lines();
hipError_t launch_pass_eaw(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                           void* rho, hipStream_t st);
// Adjoint of E in register form (power-of-two P <= g <= 64, P <= 16): 64 / g lines per workgroup.
bool ehr_applicable(int M, int g);
int ehr_tile_lines(int g);
hipError_t launch_pass_ehr(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                           hipStream_t st);
// Structured accumulate (A) and its adjoint (AH) in registers: one thread per output group for
// g <= 8, g / 8 lanes per group for g = 16, 32, 64.
bool asr_applicable(int g, int max_g);
hipError_t launch_pass_asr(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                           int accumulate, void* rho, hipStream_t st);

void set_error(const std::string& msg);

}  // namespace fx

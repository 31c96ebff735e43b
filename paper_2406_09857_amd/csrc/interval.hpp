// Device interval core for gfx950: outward-rounded FP64 interval arithmetic
// with one hardware rounding mode per kernel.
//
// Representation.  An interval [lo, hi] is held as the pair (nlo, hi) with
// nlo = -lo.  Every kernel switches the wave's FP64 rounding mode to "toward
// +infinity" once, at entry; from then on every FP64 add and multiply the
// compiler emits rounds up.  The lower endpoint is obtained through
// RD(x) = -RU(-x): with nlo stored, a rounded-down lower bound is simply a
// rounded-up operation on negated operands, and the negations live in the data
// (negated coefficients, negated box endpoints), never in the instruction
// stream.
//
// Why inline asm for the mode switch.  The AMDGPU backend assumes round-to-
// nearest for every FP64 instruction and re-inserts a mode reset in front of
// them after a visible s_setreg; it also folds -((-x)*y) into x*y, which is
// only valid under round-to-nearest.  Writing the MODE register from inline
// asm hides the switch from that bookkeeping, and keeping negations out of the
// arithmetic (or behind `opaque`) leaves no fold that depends on the mode.
// Kernels must therefore (1) call `round_up_mode()` before any FP64 arithmetic,
// (2) never feed a negated value into a multiply or add without `opaque`,
// (3) be compiled with -ffp-contract=off (fused multiply-adds only where they
// are written out, as in the Horner steps below).
//
// Interval rules (Sec. 3.2 of Moroz, arXiv 2406.09857, names interval
// arithmetic and gives the sum; the product is the textbook min/max rule):
//   [a,b] + [c,d] = [RD(a+c), RU(b+d)]
//   [a,b] * [c,d] = [RD(min P), RU(max P)],  P = {ac, ad, bc, bd}.
// The Horner step J*I + C of polynomial evaluation is one operation: the
// exact range [min P + lo(C), max P + hi(C)] of the set J*I + C, each endpoint
// rounded outward once (an FMA in round-up mode: RU(p + c) exactly).
// RD/RU are monotone, so RD(min P + c) = min RD(p + c) over P: every formula
// below that picks a subset of P known to contain the extremum gives the same
// bits (up to the sign of a zero).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vx {

// Switch this wave's FP64 rounding mode to round-toward-+infinity
// (MODE.FP_ROUND bits [3:2] = 1).  The "memory" clobber keeps loads after it.
__device__ __forceinline__ void round_up_mode() {
  asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 1" ::: "memory");
}

// Hide a value's provenance from the optimizer (no instruction emitted).
__device__ __forceinline__ double opaque(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Sign class of a box interval on one axis.
enum : int { CLS_POS = 0, CLS_NEG = 1, CLS_STRADDLE = 2 };

// Grid cell enclosure on one axis (round-up mode must be active).
// Cell `label` of the 2^level grid on [dlo, dhi] is
//   [RD(dlo + RD(label * RD(dhi-dlo)) 2^-level), RU(dlo + RU((label+1) * RU(dhi-dlo)) 2^-level)].
// Returned as nlo = -lo and hi.  On dyadic domains such as [-1,1] both are exact.
// With centre = 1 the "cell" is the degenerate box of the cell's centre, the
// common endpoint of cells 2*label and 2*label+1 at level+1: its lower bound is
// the lower end of cell 2*label+1, its upper bound the upper end of cell
// 2*label (the centre enclosures of the Taylor forms).  With centre = 2 it is
// grid vertex `label` (0 .. 2^level), the common endpoint of cells label-1 and
// label: the lower end of cell label and the upper end of cell label-1 (the
// vertex enclosures of the inclusion criterion).
struct AxisGrid {
  double dlo, ndlo, dhi, ndhi;  // domain endpoints and their negations (host-negated)
  int level;
  int centre;                   // 0: cells, 1: cell centres, 2: grid vertices
};

__device__ __forceinline__ void cell(const AxisGrid& g, int32_t label, double& nlo, double& hi) {
  const double wu = g.dhi + g.ndlo;   // RU(dhi - dlo)
  const double nw = g.dlo + g.ndhi;   // RU(dlo - dhi) = -RD(dhi - dlo)
  const int sh = g.centre == 1 ? 1 : 0;  // centres are vertices of level + 1
  const int64_t base = (int64_t)label << sh;
  const int64_t a = base + (g.centre == 1 ? 1 : 0);  // lower end: of cell a
  const int64_t b = base + (g.centre == 2 ? 0 : 1);  // upper end: of cell b - 1
  nlo = g.ndlo + ldexp((double)a * nw, -(g.level + sh));
  hi = g.dlo + ldexp((double)b * wu, -(g.level + sh));
}

__device__ __forceinline__ int cell_class(double nlo, double hi) {
  // lo >= 0  <=>  nlo <= 0 ;  hi <= 0
  return nlo <= 0.0 ? CLS_POS : (hi <= 0.0 ? CLS_NEG : CLS_STRADDLE);
}

// Multiplier operands of a cell for its class.
//   POS (0 <= a <= b):  u = a,  v = b
//   NEG (a <= b <= 0):  u = -a, v = -b      (both >= 0)
//   STRADDLE:           a, b, na = -a, nb = -b
struct CellOps { double u, v, nu, nv; };

__device__ __forceinline__ CellOps cell_ops(double nlo, double hi, int cls) {
  CellOps o;
  if (cls == CLS_NEG) { o.u = nlo; o.v = opaque(-hi); o.nu = 0; o.nv = 0; }
  else { o.u = opaque(-nlo); o.v = hi; o.nu = nlo; o.nv = opaque(-hi); }
  return o;
}

// One Horner step J <- J*I + C for a cell of class POS: I = [u, v], u >= 0.
//   lo' = min(lo*u, lo*v) + lo(C)  ->  nlo' = max(RU(nlo*u + cn), RU(nlo*v + cn))
//   hi' = max(hi*u, hi*v) + hi(C)  ->  hi'  = max(RU(hi*u + ch), RU(hi*v + ch))
// (cn = -lo(C), ch = hi(C)); 4 FMAs and 2 maxima.
__device__ __forceinline__ void step_pos(double& nlo, double& hi, double u, double v, double cn, double ch) {
  const double a = fmax(__builtin_fma(nlo, u, cn), __builtin_fma(nlo, v, cn));
  const double b = fmax(__builtin_fma(hi, u, ch), __builtin_fma(hi, v, ch));
  nlo = a;
  hi = b;
}

// Class NEG: I = [a, b] <= 0 with u = -a, v = -b:
//   lo' = min(hi*a, hi*b) + lo(C)  ->  nlo' = max(RU(hi*u + cn), RU(hi*v + cn))
//   hi' = max(lo*a, lo*b) + hi(C)  ->  hi'  = max(RU(nlo*u + ch), RU(nlo*v + ch))
__device__ __forceinline__ void step_neg(double& nlo, double& hi, double u, double v, double cn, double ch) {
  const double a = fmax(__builtin_fma(hi, u, cn), __builtin_fma(hi, v, cn));
  const double b = fmax(__builtin_fma(nlo, u, ch), __builtin_fma(nlo, v, ch));
  nlo = a;
  hi = b;
}

// General product (any signs): I = [a, b], na = -a, nb = -b.
//   nlo' = max RU(-p - lo(C)) over p in P = max over {nlo*a, nlo*b, hi*na, hi*nb} of RU(. + cn)
//   hi'  = max RU(p + hi(C))              = max over {nlo*na, nlo*nb, hi*a, hi*b} of RU(. + ch)
__device__ __forceinline__ void step_gen(double& nlo, double& hi, const CellOps& o, double cn, double ch) {
  const double a = fmax(fmax(__builtin_fma(nlo, o.u, cn), __builtin_fma(nlo, o.v, cn)),
                        fmax(__builtin_fma(hi, o.nu, cn), __builtin_fma(hi, o.nv, cn)));
  const double b = fmax(fmax(__builtin_fma(nlo, o.nu, ch), __builtin_fma(nlo, o.nv, ch)),
                        fmax(__builtin_fma(hi, o.u, ch), __builtin_fma(hi, o.v, ch)));
  nlo = a;
  hi = b;
}

// Product, then sum, each rounded outward (not a Horner step): J <- J*X + A
// for the combination formulas of the exclusion and inclusion tests, whose
// definitions sum separately rounded products.  Same operands as step_gen.
__device__ __forceinline__ void mul_add_sep(double& nlo, double& hi, const CellOps& o, double cn, double ch) {
  const double a = fmax(fmax(nlo * o.u, nlo * o.v), fmax(hi * o.nu, hi * o.nv));
  const double b = fmax(fmax(nlo * o.nu, nlo * o.nv), fmax(hi * o.u, hi * o.v));
  nlo = a + cn;
  hi = b + ch;
}

}  // namespace vx

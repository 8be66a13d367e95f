// Geometric multigrid for the 3-D model (multigrid.hip): the level
// hierarchy in the workspace, the kernels' arguments and launchers.
#pragma once

#include "common.h"

namespace ens {

constexpr int kMgMaxLevels = 12;   // n + 1 = 2^k cells, k <= 12
constexpr double kMgRatio = 30.0;  // default lambda_max / lambda_min of the smoother
constexpr int kMgDegree = 2;       // smoother degree

// One level of the V-cycle: its operator (27 slots) and vectors, and the
// per-member smoother coefficients (Members::cheb, Members::lmax; every
// other member field of a coarse level is unused; ctl is the solve's).
struct MgLevel {
  int m;          // interior nodes per direction
  Geometry g;     // 3-D geometry of m^3 rows (full 27-value reads on coarse levels)
  const double* V;
  const double* b;  // right-hand side of the level's correction equation
  double* x;        // the level's V-cycle output
  double* res;      // residual b - A x
  double* za;       // smoother iterate (started by the caller)
  double* Vt;       // levels of at most kMgTailNodes nodes per direction: the 27
                    // slots member-major, [S][27][m^3], for the fused coarse tail
  Members mem;
};

struct MgHierarchy {
  int L;   // levels, fine first; level L - 1 has one node and is solved exactly
  int levelwise;   // 1: no fused coarse tail (every level with its own launches)
  MgLevel lv[kMgMaxLevels];
};

// nodes per direction of each level (n, (n - 1) / 2, ..., 1); 0 if n + 1 is
// not a power of two >= 2 or there would be more than kMgMaxLevels levels
int mg_levels(int n, int* ms);
// bytes of the coarse levels (1 .. L - 1) for an ensemble of S members,
// with the member-major operator copies of the levels of at most
// kMgTailNodes nodes per direction
size_t mg_bytes(int n, int S);
// carve the coarse levels from `base` (mg_bytes(n, S) bytes); level 0's
// fields are left for the caller
void mg_carve(void* base, int n, int S, const int* ctl, MgHierarchy& H);

struct MgRapArgs {
  const double* Vf;  // fine operator, 27 slots of stride vstride_f
  double* Vc;        // coarse operator, 27 slots of stride vstride_c
  int mc, S, Sp;     // coarse nodes per direction, members, member slots
  size_t nrc, vstride_f, vstride_c;
};

struct MgGershArgs {
  const double* V;   // 27 slots
  double* partial;   // [groups][Sp] per-workgroup maxima of sum_j |a_ij| / a_ii
  int S, Sp;
  size_t nr, vstride;
};

struct MgCoefArgs {
  const double* partial;  // MgGershArgs::partial
  int G, S, Sp;
  double ratio;
  double* lmax;   // [Sp]
  double* cheb;   // [Sp][kChebCoef]: theta, then c1, c2 of the one step of degree 2
};

enum MgTransfer { MG_RESTRICT = 0, MG_RESTRICT_START = 1, MG_RESTRICT_SOLVE = 2, MG_PROLONG = 3 };

struct MgTransferArgs {
  const double* fine_in;   // restriction: the fine residual
  double* coarse_out;      // restriction: the coarse right-hand side
  const double* coarse_in; // prolongation: the coarse correction
  double* fine_x;          // prolongation: the fine iterate, corrected in place
  const double* Vc;        // restriction with start or solve: the coarse operator (diagonal slot)
  const double* cheb;      // restriction with start: the coarse smoother's theta per member
  double* z;               // restriction with start: z = D^-1 b / theta
  double* x;               // restriction with solve: x = b / a (one node)
  const int* done;
  int op;                  // MgTransfer
  int mc, S, Sp;
  size_t vstride_c;
};

// The coarse end of the V-cycle in one launch: levels of at most
// kMgTailNodes nodes per direction (7, 3, 1 or 3, 1), one workgroup per
// member holding the levels' operators and vectors in LDS.  Input: the
// first tail level's right-hand side; output: its V-cycle result x (the
// post-smoother's correction already added).  The operations and their
// order are those of the per-level kernels.
constexpr int kMgTailNodes = 7;
constexpr int kMgTailLevels = 3;
struct MgTailLevel {
  const double* Vt;    // 27 slots member-major: [S][27][m^3]
  const double* cheb;  // [Sp][kChebCoef]: theta, c1, c2
  int m;
};
struct MgTailArgs {
  MgTailLevel lv[kMgTailLevels];
  int nlev;            // tail levels (the last has one node)
  const double* b;     // [m0^3][S]
  double* x;           // [m0^3][S]
  const int* done;
  int S;
};

void launch_mg_rap(const MgRapArgs& a, hipStream_t s);
void launch_mg_tail(const MgTailArgs& a, hipStream_t s);
// Vt[s][slot][r] = V[slot * vstride + r * S + s] for the m^3 rows of a level
void launch_mg_pack(const double* V, size_t vstride, double* Vt, int m, int S, hipStream_t s);
void launch_mg_gersh(const MgGershArgs& a, int groups, hipStream_t s);
void launch_mg_coef(const MgCoefArgs& a, hipStream_t s);
void launch_mg_transfer(const MgTransferArgs& a, hipStream_t s);
int mg_groups(size_t nr, int Sp);

}  // namespace ens

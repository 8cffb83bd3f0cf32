// LDS of one TJM workgroup.
//
// Every workgroup routine finds its LDS in the one file-scope object
// tjm_lds rather than through pointer arguments: the heavy routines are
// separate (non-inlined) device functions, and an LDS address that reaches
// them only through a generic pointer would be accessed with flat
// instructions instead of ds_read/ds_write.
#pragma once
#include <dev_gemm.hpp>
#include "tjm_params.h"

#define TJM_KMAX 32                 // largest Krylov dimension supported

// Householder QR: the reflector of the current step and the diagonal of R.
constexpr int QR_MROWS = 128;
constexpr int QR_TPC = TJM_NT >= 16 ? 16 : 1;                   // threads per column
constexpr int QR_RPT = (QR_MROWS + QR_TPC - 1) / QR_TPC;        // rows per thread

struct QrLds {
  double vnorm2[QR_MROWS];
  double bre[QR_MROWS], bim[QR_MROWS];  // diagonal of R before the gauge fix
  zd v[QR_MROWS];                       // reflector of the current step
  double a2next;                        // ||column j+1, rows j+1..||^2
};

// Register-resident QR (m <= 128, n <= 64): the reflector of the current
// step (two buffers) and per column beta and ||v||^2.
constexpr int QRF_ROWS = 128, QRF_COLS = 64, QRF_RPT = QRF_ROWS / 4;
struct QrfLds {
  zd v[2][QRF_ROWS];
  zd v0[QRF_COLS];
  double bre[QRF_COLS], bim[QRF_COLS], vn[QRF_COLS];
};

// Jacobi SVD: singular values, their order, convergence flags.
constexpr int SVD_LDS_BYTES = 64 * 64 * 16;   // a working matrix of up to 4096 complex doubles
static_assert(sizeof(QrLds) <= SVD_LDS_BYTES, "the preconditioning QR keeps its reflector in the SVD's LDS");

struct SvdLds {
  double s[128];
  int order[128];
  int rotated;
  int k;
  unsigned long long offmax;   // bits of the largest |w_a^H w_b| / (|w_a| |w_b|) of a sweep
};

// Lanczos: the tridiagonal matrix, the small exponential and the
// Gram-Schmidt projections.
struct LanczosLds {
  double alpha[TJM_KMAX], beta[TJM_KMAX];
  double cre[TJM_KMAX], cim[TJM_KMAX];
  double hre[TJM_KMAX], him[TJM_KMAX];
  double hsre[TJM_KMAX], hsim[TJM_KMAX];   // h_i s_i, then b0 c_i s_i
  double scale[TJM_KMAX];                  // s_i: q_i = s_i B_i
  double red[TJM_NWAVE][2 * TJM_KMAX];
  double ur[TJM_KMAX], ui[TJM_KMAX], tr[TJM_KMAX], ti[TJM_KMAX];
  int done;
};

constexpr int LDS_WORK_BYTES = GEMM_LDS_BYTES > SVD_LDS_BYTES ? GEMM_LDS_BYTES : SVD_LDS_BYTES;

struct Lds {
  alignas(16) char gemm[LDS_WORK_BYTES];   // GEMM staging, or the SVD working matrix
  BlkScratch S;
  union { QrLds qr; QrfLds qrf; };
  SvdLds sv;
  LanczosLds lz;
  unsigned long long st[TJM_NSTAT];
  int item;
  int pick;
  double rho[4];
};

static __shared__ Lds tjm_lds;

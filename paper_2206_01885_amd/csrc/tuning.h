// Launch parameters set by measurement.  paper_2206_01885_amd/autotune.py
// times one-at-a-time variants of them on the n = 2^20 cube (Coulomb,
// tol 1e-6, 32 RHS: build + apply) and records the fastest in tuning.json,
// which the build passes as -D flags; the values below are the defaults.
// None of them changes a result, only launch shapes.
#pragma once

// Transposed coupling sweep: 16-column blocks loaded ahead.
#ifndef H2_TUNE_SWEEP_T_P
#define H2_TUNE_SWEEP_T_P 3
#endif
// Narrow IDs: a bin of fewer tasks than this joins the next smaller bin.
#ifndef H2_TUNE_BIN_MIN
#define H2_TUNE_BIN_MIN 256
#endif
// Top-down DataReduct: boxes with more candidates are searched child by child.
#ifndef H2_TUNE_SPLIT_MIN
#define H2_TUNE_SPLIT_MIN 64
#endif
// Top-down DataReduct: levels with fewer nodes take 1024 lanes per node.
#ifndef H2_TUNE_DOWN_WIDE
#define H2_TUNE_DOWN_WIDE 2048
#endif

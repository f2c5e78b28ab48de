// kernel_list.h -- every instantiation of the template kernels the host code
// launches, in lists that the kernel units expand as explicit instantiations
// (DECL = template) and the host unit as declarations (DECL = extern template),
// so that the kernel units compile in parallel.
#pragma once
#include "ssfm_kernels.h"

// Column and row passes, propagator tables and the adaptive-step kernels of
// real type R (row range 2, rows of 4096 points, exists in FP32 only).
#define OPO_PASS_KERNELS_COMMON(DECL, R)                                                           \
    DECL __global__ void column_pass<R, kColRanges[0][0], kColRanges[0][1], 2>(StepArgs<R>);       \
    DECL __global__ void column_pass<R, kColRanges[0][0], kColRanges[0][1], 3>(StepArgs<R>);       \
    DECL __global__ void column_pass<R, kColRanges[1][0], kColRanges[1][1], 2>(StepArgs<R>);       \
    DECL __global__ void column_pass<R, kColRanges[1][0], kColRanges[1][1], 3>(StepArgs<R>);       \
    DECL __global__ void column_pass<R, kColRanges[2][0], kColRanges[2][1], 2>(StepArgs<R>);       \
    DECL __global__ void column_pass<R, kColRanges[2][0], kColRanges[2][1], 3>(StepArgs<R>);       \
    DECL __global__ void row_pass<R, kRowRanges[0][0], kRowRanges[0][1]>(StepArgs<R>);             \
    DECL __global__ void row_pass<R, kRowRanges[1][0], kRowRanges[1][1]>(StepArgs<R>);             \
    DECL __global__ void disp_table<R>(const InstDesc *, int, Phasor<R> *, double, int);           \
    DECL __global__ void adapt_begin<R>(const InstDesc *, const AdaptState *, int, cplx<R> *,      \
                                        const cplx<R> *, const cplx<R> *, Phasor<R> *);            \
    DECL __global__ void adapt_error<R>(const InstDesc *, const AdaptState *, int, const cplx<R> *, \
                                        const cplx<R> *, double *);                                \
    DECL __global__ void spectrum_order<R>(const InstDesc *, const cplx<R> *, cplx<R> *);

#define OPO_PASS_KERNELS_F32(DECL)                                                                 \
    OPO_PASS_KERNELS_COMMON(DECL, float)                                                           \
    DECL __global__ void row_pass<float, kRowRanges[2][0], kRowRanges[2][1]>(StepArgs<float>);

#define OPO_PASS_KERNELS_F64(DECL) OPO_PASS_KERNELS_COMMON(DECL, double)

// Mixed column/row launches for the (column range, row range) pairs the
// four-step split produces, per field count.
#define OPO_MIXED_KERNELS_F32_CR0(DECL, NF)                                                       \
    DECL __global__ void mixed_pass<float, 0, 0, NF>(StepArgs<float>, StepArgs<float>);          \
    DECL __global__ void mixed_pass<float, 0, 1, NF>(StepArgs<float>, StepArgs<float>);          \
    DECL __global__ void mixed_pass<float, 0, 2, NF>(StepArgs<float>, StepArgs<float>);

#define OPO_MIXED_KERNELS_F32_CR12(DECL, NF)                                                      \
    DECL __global__ void mixed_pass<float, 1, 1, NF>(StepArgs<float>, StepArgs<float>);          \
    DECL __global__ void mixed_pass<float, 1, 2, NF>(StepArgs<float>, StepArgs<float>);          \
    DECL __global__ void mixed_pass<float, 2, 1, NF>(StepArgs<float>, StepArgs<float>);          \
    DECL __global__ void mixed_pass<float, 2, 2, NF>(StepArgs<float>, StepArgs<float>);

#define OPO_MIXED_KERNELS_F64(DECL, NF)                                                           \
    DECL __global__ void mixed_pass<double, 0, 0, NF>(StepArgs<double>, StepArgs<double>);       \
    DECL __global__ void mixed_pass<double, 0, 1, NF>(StepArgs<double>, StepArgs<double>);       \
    DECL __global__ void mixed_pass<double, 1, 1, NF>(StepArgs<double>, StepArgs<double>);       \
    DECL __global__ void mixed_pass<double, 2, 1, NF>(StepArgs<double>, StepArgs<double>);

// Resident passes: FP32 nt 2^10..2^12, FP64 2^10..2^11, two or three waves.
#define OPO_RESIDENT_KERNELS_NF(DECL, NF)                                                         \
    DECL __global__ void resident_pass<float, 10, NF>(StepArgs<float>);                           \
    DECL __global__ void resident_pass<float, 11, NF>(StepArgs<float>);                           \
    DECL __global__ void resident_pass<float, 12, NF>(StepArgs<float>);                           \
    DECL __global__ void resident_pass<double, 10, NF>(StepArgs<double>);                         \
    DECL __global__ void resident_pass<double, 11, NF>(StepArgs<double>);

#define OPO_RESIDENT_KERNELS(DECL)                                                                 \
    OPO_RESIDENT_KERNELS_NF(DECL, 2)                                                               \
    OPO_RESIDENT_KERNELS_NF(DECL, 3)

#define OPO_ALL_KERNELS(DECL)                                                                      \
    OPO_PASS_KERNELS_F32(DECL)                                                                     \
    OPO_PASS_KERNELS_F64(DECL)                                                                     \
    OPO_MIXED_KERNELS_F32_CR0(DECL, 2)                                                             \
    OPO_MIXED_KERNELS_F32_CR0(DECL, 3)                                                             \
    OPO_MIXED_KERNELS_F32_CR12(DECL, 2)                                                            \
    OPO_MIXED_KERNELS_F32_CR12(DECL, 3)                                                            \
    OPO_MIXED_KERNELS_F64(DECL, 2)                                                                 \
    OPO_MIXED_KERNELS_F64(DECL, 3)                                                                 \
    OPO_RESIDENT_KERNELS(DECL)

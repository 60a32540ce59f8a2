// Launchers of the penalty-step operator kernels (apply_kernel.h, PEN = true):
// instantiated in their own translation unit so the two builds run in parallel.

#include "apply_kernel.h"

namespace sipg {

template <int N, typename T, bool CURVED>
static hipError_t launch_pen_n(const OpData<T>& op, const ApplyIO<T>& io, int mode, hipStream_t s) {
    using Sh = Shape<N, 3, sizeof(T) == 8>;
    const int blocks = (op.ncell + Sh::CPB - 1) / Sh::CPB;
    if (mode == MODE_APPLY)
        hipLaunchKernelGGL((k_apply<N, 3, T, CURVED, MODE_APPLY, true>), dim3(blocks), dim3(Sh::THREADS), 0, s, op,
                           io);
    else if (mode == MODE_RESID)
        hipLaunchKernelGGL((k_apply<N, 3, T, CURVED, MODE_RESID, true>), dim3(blocks), dim3(Sh::THREADS), 0, s, op,
                           io);
    else if (mode == MODE_CONT)
        hipLaunchKernelGGL((k_apply<N, 3, T, CURVED, MODE_CONT, true>), dim3(blocks), dim3(Sh::THREADS), 0, s, op,
                           io);
    else
        hipLaunchKernelGGL((k_apply<N, 3, T, CURVED, MODE_CHEB, true>), dim3(blocks), dim3(Sh::THREADS), 0, s, op,
                           io);
    return hipGetLastError();
}

template <typename T, bool CURVED>
static hipError_t launch_pen_c(int n, const OpData<T>& op, const ApplyIO<T>& io, int mode, hipStream_t s) {
    switch (n) {
        case 2: return launch_pen_n<2, T, CURVED>(op, io, mode, s);
        case 3: return launch_pen_n<3, T, CURVED>(op, io, mode, s);
        case 4: return launch_pen_n<4, T, CURVED>(op, io, mode, s);
        case 5: return launch_pen_n<5, T, CURVED>(op, io, mode, s);
        case 6: return launch_pen_n<6, T, CURVED>(op, io, mode, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_apply_pen(int n, bool curved, const OpData<T>& op, const ApplyIO<T>& io, int mode, hipStream_t s) {
    return curved ? launch_pen_c<T, true>(n, op, io, mode, s) : launch_pen_c<T, false>(n, op, io, mode, s);
}

template hipError_t launch_apply_pen<double>(int, bool, const OpData<double>&, const ApplyIO<double>&, int,
                                             hipStream_t);
template hipError_t launch_apply_pen<float>(int, bool, const OpData<float>&, const ApplyIO<float>&, int,
                                            hipStream_t);

}  // namespace sipg

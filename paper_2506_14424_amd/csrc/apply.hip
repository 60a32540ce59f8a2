// Launchers of the SIPG viscous and Poisson operator kernels (apply_kernel.h).

#include "apply_kernel.h"

namespace sipg {

template <int N, int C, typename T, bool CURVED>
static hipError_t launch_nc(const OpData<T>& op, const ApplyIO<T>& io, int mode, hipStream_t s) {
    using Sh = Shape<N, C, sizeof(T) == 8>;
    const int blocks = (op.ncell + Sh::CPB - 1) / Sh::CPB;
    if (mode == MODE_APPLY)
        hipLaunchKernelGGL((k_apply<N, C, T, CURVED, MODE_APPLY, false>), dim3(blocks), dim3(Sh::THREADS), 0, s, op,
                           io);
    else if (mode == MODE_RESID)
        hipLaunchKernelGGL((k_apply<N, C, T, CURVED, MODE_RESID, false>), dim3(blocks), dim3(Sh::THREADS), 0, s, op,
                           io);
    else if (mode == MODE_CONT)
        hipLaunchKernelGGL((k_apply<N, C, T, CURVED, MODE_CONT, false>), dim3(blocks), dim3(Sh::THREADS), 0, s, op,
                           io);
    else
        hipLaunchKernelGGL((k_apply<N, C, T, CURVED, MODE_CHEB, false>), dim3(blocks), dim3(Sh::THREADS), 0, s, op,
                           io);
    return hipGetLastError();
}

template <int C, typename T, bool CURVED>
static hipError_t launch_c(int n, const OpData<T>& op, const ApplyIO<T>& io, int mode, hipStream_t s) {
    switch (n) {
        case 2: return launch_nc<2, C, T, CURVED>(op, io, mode, s);
        case 3: return launch_nc<3, C, T, CURVED>(op, io, mode, s);
        case 4: return launch_nc<4, C, T, CURVED>(op, io, mode, s);
        case 5: return launch_nc<5, C, T, CURVED>(op, io, mode, s);
        case 6: return launch_nc<6, C, T, CURVED>(op, io, mode, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_apply(int n, int C, bool curved, const OpData<T>& op, const ApplyIO<T>& io, int mode,
                        hipStream_t s) {
    if (op.ncell <= 0) return hipSuccess;
    if (op.pen) return launch_apply_pen<T>(n, curved, op, io, mode, s);
    if (C == 3) return curved ? launch_c<3, T, true>(n, op, io, mode, s) : launch_c<3, T, false>(n, op, io, mode, s);
    return curved ? launch_c<1, T, true>(n, op, io, mode, s) : launch_c<1, T, false>(n, op, io, mode, s);
}

template hipError_t launch_apply<double>(int, int, bool, const OpData<double>&, const ApplyIO<double>&, int,
                                         hipStream_t);
template hipError_t launch_apply<float>(int, int, bool, const OpData<float>&, const ApplyIO<float>&, int,
                                        hipStream_t);

}  // namespace sipg

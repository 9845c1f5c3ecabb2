// pic_k64.hip -- FP64 form of the same kernels (reference-precision path on the GPU).
#include "pic_kernels.inc"

template struct pic::Launchers<double>;

// pic_k32.hip -- FP32 form: int32 cell + float offset positions, float fields, push and deposit.
#include "pic_kernels.inc"

template struct pic::Launchers<float>;

"""MI355X-native batched 2D physics step of VMAS (Bettini et al., 2022).

The physics runs in hand-written HIP kernels (libvmas.so, C boundary in
include/vmas.h); `binding` marshals torch tensors to it, `workloads` draws
seeded synthetic inputs.
"""
__all__ = ["binding", "workloads"]

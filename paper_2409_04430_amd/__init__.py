"""MI355X-native NEP path-integral MD hot path.

The compute path lives in the HIP C-ABI library `libneppimd.so` (sources in
`csrc/`, declarations in `include/neppimd.h`); `lib` is its thin Python
binding.  `inputs` and `configs` produce the seeded synthetic workloads.
"""
__all__ = ["inputs", "configs", "lib"]

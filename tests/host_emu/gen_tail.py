"""Host build of the spatial-cycle tail kernel (k_spatial_tail) for bounds
checking on the CPU: the kernel text and the device helpers it calls are
taken from the sources, barriers become no-ops, and every simulated thread of
a workgroup runs the whole body in turn.  The kernel's addresses do not
depend on the data, so this visits exactly the LDS, private and global
locations the GPU visits; AddressSanitizer (LDS and the vectors are heap
buffers of exactly the launch's sizes, the private arrays live on the stack)
reports any access outside them."""
import os
import re

ROOT = os.path.join(os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))),
                    "paper_1411_0519_amd", "csrc")

PRELUDE = """#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cmath>
#include <vector>
struct Dim3 { unsigned x = 0, y = 0, z = 0; };
static Dim3 threadIdx, blockIdx, blockDim, gridDim;
static unsigned char* g_lds = nullptr;
#define __global__
#define __device__
#define __host__
#define __launch_bounds__(x)
#define __restrict__
#define __syncthreads() ((void)0)
#define __align__(x) alignas(x)
"""


def grab(text, start_pat, end_pat):
    i = text.index(start_pat)
    return text[i:text.index(end_pat, i)]


def generate(outdir):
    """Write tail_kernel.inc (the host form of the kernel) into outdir."""
    sp = open(os.path.join(ROOT, "stmg_spatial.hip")).read()
    dv = open(os.path.join(ROOT, "stmg_device.h")).read()
    it = open(os.path.join(ROOT, "stmg_internal.h")).read()
    kernel = grab(sp, "template <typename T, int D, int NT>\n__global__ __launch_bounds__(256) void k_spatial_tail",
                  "}  // namespace\n")
    taps = grab(sp, "__device__ inline int coarse_taps",
                "template <typename T, int D, int NT>\n__global__ __launch_bounds__(256) void k_prolong_space")
    stencil = grab(dv, "template <typename T, int D, int NT>\n__device__ inline void stencil_mk", "}  // namespace dev")
    node = grab(dv, "template <int D>\n__device__ inline void node_coords", "}  // namespace dev")
    lds_fn = grab(sp, "size_t spatial_tail_lds(", "#define SPATIAL_DISPATCH")
    tailargs = grab(it, "template <typename T>\nstruct TailArgs", "// LDS bytes of the tail")
    consts = re.findall(r"constexpr int (?:TAIL_MAX|NT_MAX)[^;]*;", it)
    upd = re.search(r"enum\s*\{[^}]*UPD_ADD[^}]*\};", it).group(0)
    marker = "extern __shared__ __align__(16) unsigned char lds_raw[];"
    assert marker in kernel
    kernel = kernel.replace(marker, "unsigned char* lds_raw = g_lds;")
    if node in stencil:
        node = ""
    out = (PRELUDE + "namespace stmg {\n" + "\n".join(consts) + "\n" + upd + "\n" + tailargs
           + "namespace dev {\n"
           + "inline long long slab_index() { return (long long)blockIdx.y + (long long)gridDim.y * blockIdx.z; }\n"
           + stencil + node + "}  // namespace dev\nusing namespace dev;\n"
           + taps + kernel + lds_fn + "}  // namespace stmg\n")
    path = os.path.join(outdir, "tail_kernel.inc")
    with open(path, "w") as fh:
        fh.write(out)
    return path

"""Build the CPU emulation of the amqft kernels (test infrastructure).

The kernel sources are compiled for the host with the HIP shim of
tests/emu/shim under AddressSanitizer and UndefinedBehaviorSanitizer.  Two
textual changes are made to copies of the sources: the dynamic-LDS
declaration becomes a pointer to the emulated workgroup's LDS block, and the
whole-value LDS accessors ldc / stc of amqft_device.h report every access to
the shim's barrier-interval race checker, and the in-place path's signal
accessors xld / xst report to its cross-workgroup checker.  Objects are cached under
_build/emu by a hash of their inputs."""
from __future__ import annotations

import hashlib
import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1404_1810_amd", "csrc")
OUT_DIR = os.path.join(ROOT, "_build", "emu")
KERNELS = ["amqft_kA.hip", "amqft_lds.hip", "amqft_fast.hip", "amqft_kB.hip", "amqft_kLT.hip", "amqft_multipass.hip"]
HEADERS = ["amqft_device.h", "amqft_internal.h", "amqft_levels.h", "amqft_leaf.h", "amqft_kA_passes.h", "amqft_kB_passes.h",
           "amqft_iplayout.h"]
CXX = os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++")
SMEM = re.compile(r"extern\s+__shared__\s+__align__\(\d+\)\s+unsigned\s+char\s+smem\[\];")
FLAGS = ["-std=c++20", "-O0", "-gline-tables-only", "-ffp-contract=off", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-Wno-unused-value", "-Wno-ignored-attributes", "-pthread"]


def _transform_header(name: str, text: str) -> str:
    if name == "amqft_device.h":
        a = "    const typename vec2<R>::T v = *reinterpret_cast<const typename vec2<R>::T*>(p);"
        b = "    *reinterpret_cast<typename vec2<R>::T*>(p) = v;"
        assert a in text and b in text, "ldc / stc bodies changed: update the emulation transform"
        text = text.replace(a, "    ::emu::lds_touch(p, sizeof(cx<R>), false);\n" + a)
        text = text.replace(b, "    ::emu::lds_touch(p, sizeof(cx<R>), true);\n" + b)
        # the fixed-point overloads
        a = "    const vec2<fx32>::T v = *reinterpret_cast<const vec2<fx32>::T*>(p);"
        b = "    *reinterpret_cast<vec2<fx32>::T*>(p) = v;"
        assert a in text and b in text, "fixed-point ldc / stc bodies changed: update the emulation transform"
        text = text.replace(a, "    ::emu::lds_touch(p, sizeof(cx<fx32>), false);\n" + a)
        text = text.replace(b, "    ::emu::lds_touch(p, sizeof(cx<fx32>), true);\n" + b)
        # the in-place path's signal accesses
        a = "    const cx<R> v = *p;  // in-place signal read"
        b = "    *p = v;  // in-place signal write"
        assert a in text and b in text, "xld / xst bodies changed: update the emulation transform"
        text = text.replace(a, "    ::emu::global_touch(p, sizeof(cx<R>), false);\n" + a)
        text = text.replace(b, "    ::emu::global_touch(p, sizeof(cx<R>), true);\n" + b)
    return text


def _digest(*parts) -> str:
    h = hashlib.sha256()
    for p in parts:
        h.update(p if isinstance(p, bytes) else p.encode())
    return h.hexdigest()[:16]


def build() -> str:
    shim = [os.path.join(HERE, "shim", "hip", f) for f in ("hip_runtime.h", "hip_fp16.h")]
    common = b"".join(open(f, "rb").read() for f in shim + [os.path.abspath(__file__)]) + " ".join(FLAGS).encode()
    hdr_dir_tag = _digest(common, *[open(os.path.join(CSRC, h), "rb").read() for h in HEADERS])
    inc = os.path.join(OUT_DIR, "inc_" + hdr_dir_tag)
    if not os.path.isdir(inc):
        os.makedirs(inc + ".tmp", exist_ok=True)
        for h in HEADERS:
            with open(os.path.join(inc + ".tmp", h), "w") as f:
                f.write(_transform_header(h, open(os.path.join(CSRC, h)).read()))
        os.replace(inc + ".tmp", inc)
    incs = ["-isystem", os.path.join(HERE, "shim"), "-I", inc, "-I", os.path.join(ROOT, "include")]
    units = []
    for k in KERNELS + ["emu_main.cpp"]:
        p = os.path.join(CSRC, k) if k != "emu_main.cpp" else os.path.join(HERE, k)
        if not os.path.exists(p):
            continue
        text = SMEM.sub("unsigned char* smem = ::emu::lds_base();", open(p).read())
        tag = _digest(hdr_dir_tag, text)
        units.append((k, text, os.path.join(OUT_DIR, "%s_%s.o" % (os.path.splitext(k)[0], tag))))
    todo = [u for u in units if not os.path.exists(u[2])]

    def compile_one(u):
        k, text, obj = u
        src = obj[:-2] + ".cpp"
        with open(src, "w") as f:
            f.write(text)
        r = subprocess.run([CXX] + FLAGS + incs + ["-c", src, "-o", obj + ".tmp"], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("emulation build failed on %s:\n%s" % (k, r.stderr[-6000:]))
        os.replace(obj + ".tmp", obj)

    os.makedirs(OUT_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(compile_one, todo))
    objs = [u[2] for u in units]
    exe = os.path.join(OUT_DIR, "amqft_emu_" + _digest(*[o.encode() for o in objs]))
    if not os.path.exists(exe):
        subprocess.check_call([CXX] + FLAGS + objs + ["-o", exe + ".tmp"])
        os.replace(exe + ".tmp", exe)
    return exe


if __name__ == "__main__":
    print(build())

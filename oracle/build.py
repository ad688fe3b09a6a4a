"""Build the oracle shared library with gcc (test infrastructure only).

The oracle is compiled without FMA contraction or fast-math so that each
floating-point operation is one correctly rounded binary64 operation, in the
order the source writes it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chx_oracle.c")
LIB = os.path.join(HERE, "libchx_oracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wextra", "-Werror"]


# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source (a
# checking build: load it with the sanitizer runtime preloaded, e.g.
# LD_PRELOAD=$(gcc -print-file-name=libasan.so), and run the oracle's tests)
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer", "-g"]


def build(force=True, extra=()):
    """Compile oracle/chx_oracle.c into oracle/libchx_oracle.so."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra, SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(extra=SANITIZE if "--sanitize" in sys.argv else ()))

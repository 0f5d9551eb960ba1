"""Compile the CPU oracle (test infrastructure) into oracle/liboracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dses_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


# AddressSanitizer + UndefinedBehaviorSanitizer build (tests only): any report aborts
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all"]


def build_oracle(force: bool = True, out: str = None, sanitize: bool = False) -> str:
    lib = out or LIB
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(SRC):
        return lib
    tmp = lib + ".tmp"
    opt = SANITIZE_FLAGS if sanitize else ["-O2"]
    subprocess.check_call(["gcc", *opt, "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-pthread", SRC, "-o", tmp, "-lm"])
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build_oracle())

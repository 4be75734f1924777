"""Compile a host-side C/C++ test library.

With BODEX_SANITIZE=1 in the environment the library is built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc, -O1 -g, every UB report
fatal); the process that loads it must then have libasan first in its library
list (LD_PRELOAD), which the sanitizer test sets up for the pytest child it
starts."""
import os
import subprocess

SANITIZE = os.environ.get("BODEX_SANITIZE") == "1"
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-O1", "-g"]


def build(src, out, cxx=True, extra=()):
    cmd = ["g++" if cxx else "gcc", "-std=c++17" if cxx else "-std=c11", "-O2", "-fPIC", "-shared",
           "-ffp-contract=off", *extra]
    if SANITIZE:
        cmd += SAN_FLAGS
    cmd += [src, "-o", out]
    subprocess.check_call(cmd)
    return out

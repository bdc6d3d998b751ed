"""Translate a .hip source (kernels.hip, krr_kernels.hip) into C++ for the CPU emulation (emu_hip.h).

Four mechanical rewrites, nothing else: triple-chevron launches become
emu::launch calls, __shared__ arrays become static arrays filled with garbage
once per block, the dynamic LDS array becomes the block's emulated LDS, and
file-scope device arrays become host arrays registered as device memory.
"""
import re
import sys

_HOOK = '''
namespace emu {
template <> struct StructCheck<hdf::MfArgs> {
  static void run(const char* k, int i, const hdf::MfArgs& a) {
    check_ptr(k, "a.x_soa", i, a.x_soa); check_ptr(k, "a.geo", i, a.geo); check_ptr(k, "a.jobs", i, a.jobs);
    check_ptr(k, "a.job_off", i, a.job_off); check_ptr(k, "a.btab", i, a.btab); check_ptr(k, "a.chain", i, a.chain);
    check_ptr(k, "a.qmat", i, a.qmat);
  }
};
template <> struct StructCheck<hdf::BuildTables> {
  static void run(const char* k, int i, const hdf::BuildTables& t) {
    check_ptr(k, "tb.col_of", i, t.col_of); check_ptr(k, "tb.chain", i, t.chain);
    check_ptr(k, "tb.q_len", i, t.q_len); check_ptr(k, "tb.q_off", i, t.q_off);
    check_ptr(k, "tb.q_coef", i, t.q_coef);
  }
};
}
'''


def translate(src, header="kernels.hpp"):
    n0 = src.count("<<<")
    hook = header == "kernels.hpp" and n0 > 0
    src, n = re.subn(r'(k_\w+(?:<[^<>;]*?>)?)<<<(.*?)>>>\(',
                     lambda m: f'emu::launch("{m.group(1)}", {m.group(2)}, {m.group(1)}, ', src)
    if n != n0:
        raise ValueError(f"translated {n} of {n0} launches")
    src = re.sub(r'extern __shared__ unsigned char (\w+)\[\];', r'unsigned char* \1 = emu::dyn_smem();', src)

    def shared(m):
        typ, rest = re.match(r'(\w+)\s+(.*)', m.group(1)).groups()
        arrays = re.findall(r'(\w+)\s*(?:\[[^\]]*\])+\s*(?:,|$)', rest)
        scalar = re.fullmatch(r'\s*(\w+)\s*', rest)
        if arrays:
            return f'static {typ} {rest};' + ''.join(f' emu::garbage_once({x}, sizeof({x}));' for x in arrays)
        if scalar:
            x = scalar.group(1)
            return f'static {typ} {x}; emu::garbage_once(&{x}, sizeof({x}));'
        raise ValueError(m.group(0))
    src = re.sub(r'__shared__ ([^;]*);', shared, src)
    # file-scope device arrays: registered with the emulator as device memory of their size
    src = re.sub(r'static __device__ (__align__\(\d+\) )?(\w[\w ]*?) (\w+)\[([^\]]+)\];',
                 lambda m: (f'static {m.group(1) or ""}{m.group(2)} {m.group(3)}[{m.group(4)}]; '
                            f'static emu::SymbolReg {m.group(3)}_emu_reg({m.group(3)}, sizeof({m.group(3)}));'), src)
    inc = f'#include "{header}"\n'
    if inc not in src:
        raise ValueError(f"{header} include not found")
    if hook:
        src = src.replace(inc, inc + _HOOK, 1)
    return '#define EMU_DEVICE_CODE\n' + src


if __name__ == "__main__":
    open(sys.argv[2], "w").write(translate(open(sys.argv[1]).read()))
